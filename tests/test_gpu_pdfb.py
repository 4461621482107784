"""GPU parity of the regularizer-free PDFB calls (phi_pdfb_primal,
phi_eps_update, phi_pdfb_run) against the FP64 oracle, through the C ABI.

Tolerances.  One dual step of the FP32 path is within ~1e-6 (relative L2) of
FP64; the iteration map is non-expansive, so after K iterations the
trajectories differ by at most about K such errors: 2e-4 for the runs of up
to 60 iterations here.  Decisions of the adaptive rule are taken in FP64 on
both sides from norms that differ in the 6th digit; the cases below keep
every decision far from its threshold, so the rule states must match
exactly."""
import sys

import numpy as np
import pytest

import synth
from _cases import Case, rel_l2
from oracle import analysis, pdfb

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

_CACHE = {}


def case(name):
    if name not in _CACHE:
        if name == "nnls16":
            _CACHE[name] = Case(name, problem=synth.make_problem("tiny", Ny=16, Nx=16, n_vis=[[800]]))
        else:
            _CACHE[name] = Case(name)
    return _CACHE[name]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _steps(c, op):
    """sigma_b = 0.9 / nu_l (nu_l: oracle power estimate of ||Phi_l||^2),
    tau_l = 0.9, so tau sigma ||Phi_l||^2 < 1."""
    rng = np.random.default_rng(21)
    nu = {}
    for l in range(c.prob.L):
        nu[l], _ = analysis.power_iteration(op, l, rng.standard_normal((c.prob.Ny, c.prob.Nx)), 20)
    sigma = np.array([0.9 / nu[blk.l] for blk in op.blocks])
    tau = {l: 0.9 for l in range(c.prob.L)}
    return sigma, tau


def _dev(c, plan, X, V, Y, eps, sigma, tau):
    x = torch.from_numpy(c.cube(X)).cuda()
    v = plan.to_plan(torch.from_numpy(c.flat(V).astype(np.complex64)).cuda())
    y = plan.to_plan(torch.from_numpy(c.flat(Y).astype(np.complex64)).cuda())
    e = torch.from_numpy(np.asarray(eps, np.float64)).cuda()
    s = torch.from_numpy(np.asarray(sigma, np.float64)).cuda()
    t = torch.from_numpy(np.array([tau[l] for l in range(c.prob.L)], np.float64)).cuda()
    return x, v, y, e, s, t


def _inputs32(c, X, V, Y):
    """The oracle takes exactly the FP32 / complex64 values the GPU gets."""
    X32 = {l: np.asarray(x, np.float32).astype(np.float64) for l, x in X.items()}
    V32 = [np.asarray(v, np.complex64).astype(np.complex128) for v in V]
    Y32 = [np.asarray(y, np.complex64).astype(np.complex128) for y in Y]
    return X32, V32, Y32


def test_primal_step():
    c = case("tiny_w")
    _say("[pdfb] primal step")
    plan = c.plan()
    rng = np.random.default_rng(5)
    X = {l: rng.standard_normal((c.prob.Ny, c.prob.Nx)).astype(np.float32) for l in range(c.prob.L)}
    G = {l: rng.standard_normal((c.prob.Ny, c.prob.Nx)).astype(np.float32) for l in range(c.prob.L)}
    tau = {0: 0.37, 1: 1.9}
    x = torch.from_numpy(c.cube(X)).cuda()
    xt = torch.empty_like(x)
    g = torch.from_numpy(c.cube(G)).cuda()
    t = torch.tensor([tau[0], tau[1]], dtype=torch.float64, device="cuda")
    var = plan.pdfb_primal(x, xt, g, t)
    torch.cuda.synchronize()
    Xp, Xt, var_o = pdfb.primal_step({l: X[l].astype(np.float64) for l in X},
                                     {l: G[l].astype(np.float64) for l in G},
                                     {l: float(np.float32(tau[l])) for l in tau})
    for l in range(c.prob.L):
        assert rel_l2(x[l].cpu().numpy(), Xp[l]) <= 1e-6
        assert rel_l2(xt[l].cpu().numpy(), Xt[l]) <= 1e-6
        assert (x[l] >= 0).all()
        vv = var[l].cpu().numpy()
        # the FP64 sums are of the FP32 results: check against those exactly-rounded values
        xn = x[l].cpu().numpy().astype(np.float64)
        want = (np.sum((xn - X[l].astype(np.float64)) ** 2), np.sum(xn ** 2))
        assert abs(vv[0] - want[0]) <= 1e-12 * want[0] and abs(vv[1] - want[1]) <= 1e-12 * want[1]
        assert abs(vv[0] - var_o[l][0]) <= 1e-5 * var_o[l][0]


def test_eps_update_branches():
    """Every branch of the rule on one call: fixed blocks untouched, the
    freeze test, settled/outside/gap combinations, a zero image."""
    c = case("tiny_w")                       # blocks 0, 1 -> channel 0; block 2 -> channel 1
    _say("[pdfb] eps update branches")
    plan = c.plan()
    op = c.op
    rule = dict(lambda_lo=0.99, lambda_hi=1.01, lambda_mix=0.618, var_tol=1e-3, min_gap=3, freeze=True)
    r_c = plan.eps_rule(**rule)
    scen = [
        # (res, eps, state, var_ch0, var_ch1)
        ([2.0, 5.0, 1.0], [1.0, 5.0, 3.0], [[4, 0, 1], [0, 0, 0], [9, 1, 2]], (1e-9, 1.0), (0.0, 0.0)),
        ([2.0, 0.5, 7.0], [1.0, 1.0, 3.0], [[4, 0, 1], [2, 0, 0], [9, 0, 2]], (1e-9, 1.0), (1e-9, 1.0)),
        ([2.0, 0.5, 7.0], [1.0, 1.0, 3.0], [[1, 0, 1], [8, 0, 0], [9, 0, 2]], (1e-5, 1.0), (0.0, 0.0)),
    ]
    for freeze in (1, 0):
        r_c.freeze = freeze
        ro = dict(rule, freeze=bool(freeze))
        for res, eps, st, v0, v1 in scen:
            res_d = torch.tensor(res, dtype=torch.float64, device="cuda")
            eps_d = torch.tensor(eps, dtype=torch.float64, device="cuda")
            st_d = torch.tensor(st, dtype=torch.int32, device="cuda")
            var_d = torch.tensor([v0, v1], dtype=torch.float64, device="cuda")
            plan.eps_update(res_d, var_d, eps_d, st_d, r_c)
            torch.cuda.synchronize()
            so = {"since": np.array([s[0] for s in st]), "fixed": np.array([bool(s[1]) for s in st]),
                  "count": np.array([s[2] for s in st])}
            eo = pdfb.eps_update(op, np.array(eps), np.array(res), {0: v0, 1: v1}, so, ro)
            got = st_d.cpu().numpy()
            assert np.array_equal(got[:, 0], so["since"]) and np.array_equal(got[:, 1], so["fixed"].astype(int))
            assert np.array_equal(got[:, 2], so["count"])
            assert np.allclose(eps_d.cpu().numpy(), eo, rtol=1e-15, atol=0)


RUNS = [("tiny", None, 60), ("tiny_w", None, 40), ("tiny_w", "f16", 40), ("C2s", None, 12)]


@pytest.mark.parametrize("name,prec,n_iter", RUNS)
def test_pdfb_run_fixed_bounds(name, prec, n_iter):
    """n_iter iterations from x = 0, v = 0 with the chi-square bounds."""
    c = case(name)
    _say("[pdfb] run", name, prec or "c64", n_iter)
    op = c.op if prec is None else c.operator(c.theta, prec=prec)
    plan = c.plan(g_prec=prec or "c64")
    sigma, tau = _steps(c, op)
    X0 = {l: np.zeros((c.prob.Ny, c.prob.Nx), np.float32) for l in range(c.prob.L)}
    V0 = [np.zeros(len(y), complex) for y in c.Y]
    X32, V32, Y32 = _inputs32(c, X0, V0, c.Y)
    want = pdfb.pdfb(op, X32, V32, Y32, c.eps, sigma, tau, n_iter)
    x, v, y, e, s, t = _dev(c, plan, X0, V0, c.Y, c.eps, sigma, tau)
    xt = x.clone()
    grad, rho, res, var, _ = plan.pdfb_run(x, xt, v, y, e, t, n_iter, sigma=s)
    plan.check()
    vp = c.split(plan.from_plan(v).cpu().numpy())
    for l in range(c.prob.L):
        ex = rel_l2(x[l].cpu().numpy(), want["X"][l])
        et = rel_l2(xt[l].cpu().numpy(), want["Xt"][l])
        _say("  channel", l, "x rel L2", ex, "x~ rel L2", et)
        assert ex <= 2e-4 and et <= 2e-4
        assert (x[l] >= 0).all()
    ev = rel_l2(np.concatenate(vp), np.concatenate(want["V"]))
    er = rel_l2(res.cpu().numpy(), want["res"])
    _say("  v rel L2", ev, "res rel L2", er)
    assert ev <= 2e-4 and er <= 2e-4
    assert rel_l2(rho.cpu().numpy(), want["rho"]) <= 2e-4
    vo = np.array([want["var"][l] for l in range(c.prob.L)])
    assert rel_l2(var.cpu().numpy()[:, 1], vo[:, 1]) <= 2e-4


def test_pdfb_run_adaptive_bounds():
    """Noise twice the assumed level (the chi-square bound is infeasible):
    both sides raise eps the same number of times, fix it at the same
    iteration count, and end at the same bounds and image."""
    c = case("nnls16")
    _say("[pdfb] adaptive run")
    op = c.op
    rng = np.random.default_rng(31)
    X64 = {0: c.X[0].astype(np.float64)}
    y0 = op.forward(X64)
    Y = [y + 2.0 * (rng.standard_normal(len(y)) + 1j * rng.standard_normal(len(y))) / np.sqrt(2) for y in y0]
    sigma, tau = _steps(c, op)
    n_iter = 300
    rule = dict(pdfb.DEFAULT_RULE)
    X0 = {0: np.zeros((c.prob.Ny, c.prob.Nx), np.float32)}
    V0 = [np.zeros(len(y), complex) for y in Y]
    X32, V32, Y32 = _inputs32(c, X0, V0, Y)
    want = pdfb.pdfb(op, X32, V32, Y32, c.eps, sigma, tau, n_iter, rule=rule)
    assert want["state"]["count"][0] >= 2 and want["state"]["fixed"][0]
    plan = c.plan()
    x, v, y, e, s, t = _dev(c, plan, X0, V0, Y, c.eps, sigma, tau)
    xt = x.clone()
    grad, rho, res, var, state = plan.pdfb_run(x, xt, v, y, e, t, n_iter, sigma=s, rule=plan.eps_rule(**rule))
    plan.check()
    st = state.cpu().numpy()
    _say("  state", st.tolist(), "oracle", want["state"], "eps", e.cpu().numpy(), want["eps"])
    assert st[0, 1] == 1 and st[0, 2] == want["state"]["count"][0]
    assert st[0, 0] == want["state"]["since"][0]
    assert abs(e.item() - want["eps"][0]) <= 1e-5 * want["eps"][0]
    assert rel_l2(x[0].cpu().numpy(), want["X"][0]) <= 1e-3


def test_pdfb_run_launch_forms_agree():
    """Batched, per-channel, persistent and graph-replayed dual steps inside
    the loop give bitwise the same iterates."""
    from paper_2209_07604_amd import PER_CHANNEL, GRAPH, PERSISTENT
    c = case("C2s")
    _say("[pdfb] launch forms")
    plan = c.plan()
    sigma = np.full(len(c.blocks), 1e-3)
    tau = {l: 0.5 for l in range(c.prob.L)}
    X0 = {l: np.zeros((c.prob.Ny, c.prob.Nx), np.float32) for l in range(c.prob.L)}
    V0 = [np.zeros(len(y), complex) for y in c.Y]
    outs = []
    for flags in (0, PER_CHANNEL, PERSISTENT, GRAPH):
        plan.set_flags(flags)
        x, v, y, e, s, t = _dev(c, plan, X0, V0, c.Y, c.eps, sigma, tau)
        xt = x.clone()
        plan.pdfb_run(x, xt, v, y, e, t, 5, sigma=s, rule=plan.eps_rule(var_tol=0.5, min_gap=1, freeze=False))
        torch.cuda.synchronize()
        outs.append((x.clone(), v.clone(), e.clone()))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert torch.equal(a, b)
