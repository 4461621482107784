"""GPU parity: libphi (through the C ABI) against the FP64 oracle.

Tolerances: relative L2 <= 1e-5 for FP32 arithmetic with complex64 G, and
for FP16/BF16 G against the oracle run on the same rounded G; the error
against the unrounded FP64 G is reported and bounded (<= 2e-3 for FP16).
"""
import sys

import numpy as np
import pytest

from _cases import Case, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

_CACHE = {}


def case(name, oracle_prec=None):
    key = (name, oracle_prec)
    if key not in _CACHE:
        _CACHE[key] = Case(name, oracle_prec=oracle_prec)
    return _CACHE[key]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_forward(c, plan):
    x = torch.from_numpy(c.cube(c.X)).cuda()
    y = plan.from_plan(plan.forward(x))
    torch.cuda.synchronize()
    return c.split(y.cpu().numpy().astype(np.complex128))


def gpu_adjoint(c, plan, V):
    v = torch.from_numpy(c.flat(V).astype(np.complex64)).cuda()
    x = plan.adjoint(plan.to_plan(v))
    torch.cuda.synchronize()
    return x.cpu().numpy().astype(np.float64)


def gpu_dual(c, plan, V, eps, sigma):
    xt = torch.from_numpy(c.cube(c.Xt)).cuda()
    v = plan.to_plan(torch.from_numpy(c.flat(V).astype(np.complex64)).cuda())
    y = plan.to_plan(torch.from_numpy(c.flat(c.Y).astype(np.complex64)).cuda())
    e = torch.from_numpy(np.asarray(eps, np.float64)).cuda()
    s = None if sigma is None else torch.from_numpy(np.asarray(sigma, np.float64)).cuda()
    grad, rho, res = plan.dual_step(xt, v, y, e, s)
    vp = plan.from_plan(v)
    torch.cuda.synchronize()
    plan.check()
    return (c.split(vp.cpu().numpy().astype(np.complex128)), grad.cpu().numpy().astype(np.float64),
            rho.cpu().numpy(), res.cpu().numpy())


NAMES = ["tiny", "tiny_w", "tiny_dde", "C1", "C2s", "C3s", "C4s"]


@pytest.mark.parametrize("name", NAMES)
def test_forward_adjoint(name):
    _say("[parity] forward/adjoint", name)
    c = case(name)
    plan = c.plan()
    Xo = {l: x.astype(np.float64) for l, x in c.X.items()}
    want = c.op.forward(Xo)
    got = gpu_forward(c, plan)
    err = rel_l2(np.concatenate(got), np.concatenate(want))
    _say("  forward rel L2", err)
    assert err <= 1e-5
    for g, w in zip(got, want):
        if len(w):
            assert rel_l2(g, w) <= 1e-5
    want_a = c.op.adjoint(c.Y)
    got_a = gpu_adjoint(c, plan, c.Y)
    for l in range(c.prob.L):
        e = rel_l2(got_a[l], want_a[l])
        _say("  adjoint ch", l, "rel L2", e)
        assert e <= 1e-5


@pytest.mark.parametrize("name", NAMES)
def test_dual_step(name):
    _say("[parity] dual step", name)
    c = case(name)
    plan = c.plan()
    nb = len(c.blocks)
    sigma = np.linspace(0.7, 1.4, nb)
    Vp_o, grad_o, rho_o, res_o = __import__("oracle").dual_step(
        c.op, {l: x.astype(np.float64) for l, x in c.Xt.items()}, c.V, c.Y, c.eps, sigma)
    Vp, grad, rho, res = gpu_dual(c, plan, c.V, c.eps, sigma)
    assert np.all(rho_o > c.eps)     # the state sits outside every ball
    assert rel_l2(rho, rho_o) <= 1e-5 and rel_l2(res, res_o) <= 1e-5
    e = rel_l2(np.concatenate(Vp), np.concatenate(Vp_o))
    _say("  v+ rel L2", e)
    assert e <= 1e-5
    for l in range(c.prob.L):
        assert rel_l2(grad[l], grad_o[l]) <= 1e-5


def test_dual_step_both_branches_and_exact_zero():
    c = case("C3s")
    plan = c.plan()
    nb = len(c.blocks)
    op = c.op
    Xt = {l: x.astype(np.float64) for l, x in c.Xt.items()}
    phix = op.forward(Xt)
    rho0 = np.array([np.linalg.norm(c.V[k] + phix[k] - c.Y[k]) for k in range(nb)])
    eps = rho0 * np.where(np.arange(nb) % 2 == 0, 0.7, 1.3)     # alternate inside/outside
    Vp_o, grad_o, rho_o, res_o = __import__("oracle").dual_step(op, Xt, c.V, c.Y, eps, None)
    Vp, grad, rho, res = gpu_dual(c, plan, c.V, eps, None)
    for k in range(nb):
        if eps[k] >= rho0[k]:
            assert np.all(Vp[k] == 0)             # closed-form shrink gives exact zeros
        else:
            assert rel_l2(Vp[k], Vp_o[k]) <= 1e-5
    for l in range(c.prob.L):
        assert rel_l2(grad[l], grad_o[l]) <= 1e-5


@pytest.mark.parametrize("prec,bound_exact", [("f16", 2e-3), ("bf16", 1e-2)])
def test_reduced_precision_g(prec, bound_exact):
    _say("[parity] G storage", prec)
    c = case("C4s", oracle_prec=prec)
    plan = c.plan(g_prec=prec)
    Xo = {l: x.astype(np.float64) for l, x in c.X.items()}
    got = np.concatenate(gpu_forward(c, plan))
    e_q = rel_l2(got, np.concatenate(c.op.forward(Xo)))
    e_x = rel_l2(got, np.concatenate(c.op_exact.forward(Xo)))
    _say("  forward vs rounded-G oracle", e_q, "vs FP64-G oracle", e_x)
    assert e_q <= 1e-5
    assert e_x <= bound_exact
    nb = len(c.blocks)
    Vp_o, grad_o, rho_o, res_o = __import__("oracle").dual_step(
        c.op, {l: x.astype(np.float64) for l, x in c.Xt.items()}, c.V, c.Y, c.eps, None)
    Vp, grad, rho, res = gpu_dual(c, plan, c.V, c.eps, None)
    assert rel_l2(np.concatenate(Vp), np.concatenate(Vp_o)) <= 1e-5
    assert rel_l2(rho, rho_o) <= 1e-5
    for l in range(c.prob.L):
        assert rel_l2(grad[l], grad_o[l]) <= 1e-5


@pytest.mark.parametrize("mode", ["per_channel", "persistent", "graph", "tile16", "tile64"])
def test_launch_forms_bitwise_equal(mode):
    """Every launch form computes the same sums in the same order."""
    from paper_2209_07604_amd import PER_CHANNEL, GRAPH, PERSISTENT
    _say("[forms]", mode)
    c = case("C2s")
    base = c.plan()
    kw = dict(per_channel=dict(flags=PER_CHANNEL), persistent=dict(flags=PERSISTENT, persist_blocks=97),
              graph=dict(flags=GRAPH), tile16=dict(tile=16), tile64=dict(tile=64))[mode]
    other = c.plan(**kw)
    a = gpu_dual(c, base, c.V, c.eps, None)
    b = gpu_dual(c, other, c.V, c.eps, None)
    if mode.startswith("tile"):       # different tiling changes the G^H summation order
        assert rel_l2(np.concatenate(b[0]), np.concatenate(a[0])) <= 1e-6
        assert rel_l2(b[1], a[1]) <= 1e-5
    else:
        assert all(np.array_equal(x, y) for x, y in zip(a[0], b[0]))
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    if mode == "graph":
        # replays with eager work in between must keep matching the eager result
        xt = torch.from_numpy(c.cube(c.Xt)).cuda()
        y = other.to_plan(torch.from_numpy(c.flat(c.Y).astype(np.complex64)).cuda())
        e = torch.from_numpy(c.eps).cuda()
        v0 = other.to_plan(torch.from_numpy(c.flat(c.V).astype(np.complex64)).cuda())
        grad = torch.empty((c.prob.L, c.prob.Ny, c.prob.Nx), dtype=torch.float32, device="cuda")
        rho = torch.empty(len(c.blocks), dtype=torch.float64, device="cuda")
        res = torch.empty_like(rho)
        v = v0.clone()
        for rep in range(4):
            v.copy_(v0)
            other.dual_step(xt, v, y, e, None, grad, rho, res)
            torch.cuda.synchronize()
            _ = (torch.randn(1000, device="cuda") * 2).sum().item()   # eager work between replays
            vp = c.split(other.from_plan(v).cpu().numpy().astype(np.complex128))
            assert all(np.array_equal(x, y_) for x, y_ in zip(vp, a[0])), rep
            assert np.array_equal(grad.cpu().numpy().astype(np.float64), a[1])


@pytest.mark.parametrize("tile,persist", [(16, 0), (32, 301), (64, 0)])
def test_tuning_choices_match_oracle(tile, persist):
    """Every tile edge and launch shape the autotuner may pick is exact."""
    _say("[tuning]", tile, persist)
    c = case("C3s")
    plan = c.plan()
    plan.set_tuning(tile, persist)
    Vp_o, grad_o, rho_o, res_o = __import__("oracle").dual_step(
        c.op, {l: x.astype(np.float64) for l, x in c.Xt.items()}, c.V, c.Y, c.eps, None)
    got = gpu_dual(c, plan, c.V, c.eps, None)
    assert rel_l2(np.concatenate(got[0]), np.concatenate(Vp_o)) <= 1e-5
    assert rel_l2(got[2], rho_o) <= 1e-5
    for l in range(c.prob.L):
        assert rel_l2(got[1][l], grad_o[l]) <= 1e-5
    Xo = {l: x.astype(np.float64) for l, x in c.X.items()}
    assert rel_l2(np.concatenate(gpu_forward(c, plan)), np.concatenate(c.op.forward(Xo))) <= 1e-5


def test_autotune_keeps_results():
    c = case("C2s")
    plan = c.plan()
    ref = gpu_dual(c, plan, c.V, c.eps, None)
    assert plan.autotune(2) == 0
    info = plan.info()
    _say("[autotune] tile", info["tile"], "persist", info["persist_blocks"])
    got = gpu_dual(c, plan, c.V, c.eps, None)
    Vp_o, grad_o, rho_o, res_o = __import__("oracle").dual_step(
        c.op, {l: x.astype(np.float64) for l, x in c.Xt.items()}, c.V, c.Y, c.eps, None)
    assert rel_l2(np.concatenate(got[0]), np.concatenate(Vp_o)) <= 1e-5
    for l in range(c.prob.L):
        assert rel_l2(got[1][l], grad_o[l]) <= 1e-5
    # a different tiling regroups the FP32 window sums: equal up to rounding
    assert rel_l2(got[2], ref[2]) <= 1e-6


def test_determinism_and_permutation_roundtrip():
    c = case("C3s")
    plan = c.plan()
    runs = [gpu_dual(c, plan, c.V, c.eps, None) for _ in range(3)]
    for r in runs[1:]:
        assert all(np.array_equal(x, y) for x, y in zip(r[0], runs[0][0]))
        assert np.array_equal(r[1], runs[0][1]) and np.array_equal(r[2], runs[0][2])
    v = torch.from_numpy(c.flat(c.V).astype(np.complex64)).cuda()
    back = plan.from_plan(plan.to_plan(v))
    assert torch.equal(back, v)


def test_edge_cases():
    """Empty block, one-visibility block, S = 1 and S = 21 windows on the grid
    edge (wrap-around), zero image."""
    import oracle
    from synth.kb import deapodisation
    from paper_2209_07604_amd import Plan
    rng = np.random.default_rng(5)
    Ny = Nx = 32
    Ky = Kx = 64
    n_vis = [0, 1, 40]
    S = np.array([21] + list(rng.choice([1, 3, 21, 7], 40)), dtype=np.uint8)
    base = np.stack([rng.integers(0, Ky, 41), rng.integers(0, Kx, 41)], 1).astype(np.int32)
    base[0] = [Ky - 3, Kx - 1]
    base[1] = [Ky - 1, 0]
    off = np.concatenate([[0], np.cumsum(S.astype(np.int64) ** 2)])
    w = rng.standard_normal(off[-1]) + 1j * rng.standard_normal(off[-1])
    sy, sx = deapodisation(Ny, Ky), deapodisation(Nx, Kx)
    theta = np.array([1.0, 0.5, 2.0])
    plan = Plan(Ny, Nx, [3], n_vis, base, S, sy, sx, theta)
    plan.load_g(0, np.zeros(0, complex))
    plan.load_g(1, w[:off[1]])
    plan.load_g(2, w[off[1]:])
    blocks = [oracle.BlockG(0, theta[0], oracle.g_matrix(np.zeros((0, 2), int), np.zeros(0, int), np.zeros(0),
                                                           np.zeros(1, int), Ky, Kx, theta[0])),
              oracle.BlockG(0, theta[1], oracle.g_matrix(base[:1], S[:1], w[:off[1]], off[:2], Ky, Kx, theta[1])),
              oracle.BlockG(0, theta[2], oracle.g_matrix(base[1:], S[1:], w[off[1]:], off[1:] - off[1], Ky, Kx,
                                                         theta[2]))]
    op = oracle.Operator(Ny, Nx, sy, sx, blocks)
    x = rng.random((Ny, Nx)).astype(np.float32)
    want = np.concatenate(op.forward({0: x.astype(np.float64)}))
    got = plan.from_plan(plan.forward(torch.from_numpy(x[None]).cuda())).cpu().numpy()
    assert rel_l2(got, want) <= 1e-5
    v = (rng.standard_normal(41) + 1j * rng.standard_normal(41))
    got_a = plan.adjoint(plan.to_plan(torch.from_numpy(v.astype(np.complex64)).cuda())).cpu().numpy()[0]
    want_a = op.adjoint([v[:0], v[:1], v[1:]])[0]
    assert rel_l2(got_a, want_a) <= 1e-5
    zero = plan.forward(torch.zeros((1, Ny, Nx), dtype=torch.float32, device="cuda"))
    assert torch.count_nonzero(zero).item() == 0
    # dual step: empty block has rho = 0 <= eps, so its scale is 0
    eps = torch.tensor([1.0, 0.0, 1e-3], dtype=torch.float64, device="cuda")
    vv = torch.zeros(41, dtype=torch.complex64, device="cuda")
    yy = plan.to_plan(torch.from_numpy(v.astype(np.complex64)).cuda())
    grad, rho, res = plan.dual_step(torch.from_numpy(x[None]).cuda(), vv, yy, eps)
    torch.cuda.synchronize()
    assert rho[0].item() == 0.0 and res[0].item() == 0.0
