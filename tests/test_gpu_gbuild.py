"""GPU parity of the device G builder (phi_plan_build_g) against the FP64
oracle's rows (Kaiser-Bessel taps, w-chirp, DDE pair kernel; Sections
3.1-3.2), through the C ABI.

The builder computes in FP64 and rounds each tap once to the stored
precision, as the host loader does from FP64 windows, so both sides take the
rounding decision in the same precision.  Their FP64 sums differ in the last
bits (operation order, fused multiply-adds), by at most ~1e-16 of the summed
terms, which exceeds a tap's own magnitude where its real or imaginary part
cancels; every stored code must therefore be a correct rounding of the
oracle's value moved by at most 1e-12 of the window's largest tap, and
differing codes must stay rare.  The
operator built on the device is then checked against the oracle at the FP32
bound and against the same plan loaded from the oracle's windows."""
import sys

import numpy as np
import pytest

from _cases import quantise, rel_l2
from oracle import gbuild

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

J = 7
NY = NX = 64
K = (2 * NY, 2 * NX)
N_VIS = [700, 500]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _inputs(seed, with_dde):
    rng = np.random.default_rng(seed)
    out = []
    n_ant, sa = 6, 3
    dde = 0.2 * (rng.standard_normal((n_ant, sa, sa)) + 1j * rng.standard_normal((n_ant, sa, sa)))
    dde[:, 1, 1] += np.exp(1j * rng.uniform(-np.pi, np.pi, n_ant))
    for n in N_VIS:
        kappa = np.stack([rng.uniform(-K[0], 2 * K[0], n), rng.uniform(-K[1], 2 * K[1], n)], axis=1)
        h = rng.integers(0, 5, n).astype(np.int32)
        a = rng.uniform(0.2, 5.0, n)
        ant = None
        if with_dde:
            i = rng.integers(0, n_ant, n)
            j = (i + 1 + rng.integers(0, n_ant - 1, n)) % n_ant
            ant = np.stack([i, j], axis=1).astype(np.int32)
            ant[rng.random(n) < 0.25] = -1            # rows without DDE
        base, S, w, off = gbuild.block_windows(kappa, J, h, a, ant, dde if with_dde else None, K=K)
        out.append(dict(kappa=kappa, h=h, a=a, ant=ant, base=base, S=S, w=w, off=off))
    return out, (dde if with_dde else None)


def _plan(blocks, prec):
    from paper_2209_07604_amd import Plan
    base = np.concatenate([b["base"] for b in blocks]).astype(np.int32)
    S = np.concatenate([b["S"] for b in blocks]).astype(np.uint8)
    return Plan(NY, NX, [len(blocks)], [len(b["S"]) for b in blocks], base, S, np.ones(NY), np.ones(NX), None,
                g_prec=prec)


def _build(plan, k, b, dde):
    dev = "cuda"
    ant = None if b["ant"] is None else torch.from_numpy(b["ant"]).to(dev)
    dd = None if dde is None else torch.from_numpy(dde).to(dev)
    plan.build_g(k, torch.from_numpy(b["kappa"]).to(dev), torch.from_numpy(b["h"]).to(dev),
                 torch.from_numpy(b["a"]).to(dev), ant, dd, J=J)


@pytest.mark.parametrize("prec", ["c64", "f16", "bf16"])
@pytest.mark.parametrize("with_dde", [False, True])
def test_stored_codes_match_oracle_rows(prec, with_dde):
    _say("[gbuild] codes", prec, "dde" if with_dde else "die")
    blocks, dde = _inputs(1 if with_dde else 2, with_dde)
    plan = _plan(blocks, prec)
    for k, b in enumerate(blocks):
        _build(plan, k, b, dde)
    torch.cuda.synchronize()
    for k, b in enumerate(blocks):
        got = plan.read_g(k, b["off"][-1])
        want = quantise(b["w"], prec)
        nd = int(np.count_nonzero(got != want))
        # a code may differ from the oracle's only where the two FP64 values
        # straddle a rounding boundary: it must be a correct rounding of the
        # oracle's value moved by at most the FP64 slack of the window's sums
        scale = np.repeat([np.abs(b["w"][o0:o1]).max() for o0, o1 in zip(b["off"][:-1], b["off"][1:])],
                          np.diff(b["off"]))
        slack = 1e-12 * scale
        lo = quantise(b["w"].real - slack, prec).real, quantise(b["w"].imag - slack, prec).real
        hi = quantise(b["w"].real + slack, prec).real, quantise(b["w"].imag + slack, prec).real
        ok = (lo[0] <= got.real) & (got.real <= hi[0]) & (lo[1] <= got.imag) & (got.imag <= hi[1])
        _say("  block", k, "taps", len(got), "codes differing", nd, "outside the FP64 slack",
             int(np.count_nonzero(~ok)))
        assert ok.all()
        assert nd <= len(got) // 100


def test_device_built_operator():
    import oracle
    _say("[gbuild] operator")
    blocks, dde = _inputs(3, True)
    p_dev = _plan(blocks, "c64")
    p_host = _plan(blocks, "c64")
    for k, b in enumerate(blocks):
        _build(p_dev, k, b, dde)
        p_host.load_g(k, b["w"])
    rng = np.random.default_rng(9)
    x = rng.random((1, NY, NX)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    y_dev = p_dev.from_plan(p_dev.forward(xd)).cpu().numpy()
    y_host = p_host.from_plan(p_host.forward(xd)).cpu().numpy()
    e = rel_l2(y_dev, y_host)
    _say("  device-built vs host-loaded G, forward rel L2", e)
    assert e <= 1e-6                                  # rare last-bit codes only
    ops = [oracle.BlockG(0, 1.0, oracle.g_matrix(b["base"], b["S"], b["w"], b["off"], K[0], K[1])) for b in blocks]
    op = oracle.Operator(NY, NX, np.ones(NY), np.ones(NX), ops)
    want = np.concatenate(op.forward({0: x[0].astype(np.float64)}))
    e = rel_l2(y_dev, want)
    _say("  forward rel L2", e)
    assert e <= 1e-5


def test_rows_that_do_not_match_their_window_are_rejected():
    from paper_2209_07604_amd import PhiError
    blocks, dde = _inputs(4, True)
    plan = _plan(blocks, "f16")
    b = dict(blocks[0])
    b["h"] = b["h"].copy()
    b["h"][5] += 1                                    # S no longer the declared one
    with pytest.raises(PhiError):
        _build(plan, 0, b, dde)
    b = dict(blocks[0])
    b["kappa"] = b["kappa"].copy()
    b["kappa"][7, 1] += 1.0                           # first cell moved
    with pytest.raises(PhiError):
        _build(plan, 0, b, dde)
    b = dict(blocks[0])
    b["ant"] = b["ant"].copy()
    b["ant"][3] = (0, 6)                              # antenna outside the table
    with pytest.raises(PhiError):
        _build(plan, 0, b, dde)
    _build(plan, 0, blocks[0], dde)                  # consistent tables load
    _build(plan, 1, blocks[1], dde)
    x = torch.ones((1, NY, NX), dtype=torch.float32, device="cuda")
    plan.forward(x)
    torch.cuda.synchronize()
