"""The fused dual step (each G tap read once: c and G^H theta c in one pass,
the per-block factor sigma_b * scale_b applied to v+ and in the merge,
G^H(s c) = s G^H c; PHI_FUSED_GH) against the separate passes and the
FP64 oracle, through the C ABI.  The fused pass keeps the item's grid tile
and one accumulator per wave in LDS, so it runs where that fits a work-group
(16-cell tiles here); elsewhere the plan keeps the separate passes."""
import sys

import numpy as np
import pytest

from _cases import Case, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

_CACHE = {}


def case(name):
    if name not in _CACHE:
        _CACHE[name] = Case(name)
    return _CACHE[name]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("name,prec", [("tiny_w", "c64"), ("tiny_dde", "c64"), ("C2s", "c64"), ("C2s", "f16"),
                                       ("C3s", "bf16"), ("C4s", "c64")])
def test_fused_matches_separate_and_oracle(name, prec):
    from test_gpu_parity import gpu_dual
    from paper_2209_07604_amd import FUSED_GH, GRAPH
    import oracle
    _say("[fused]", name, prec)
    c = case(name)
    plan = c.plan(g_prec=prec)
    plan.set_tuning(16, 0)          # 16-cell tiles: the fused pass's LDS fits (the bench's autotuned tile)
    info_s = plan.info()
    plan.set_flags(FUSED_GH)
    info_f = plan.info()
    # the fused pass is in use: one G read per dual step instead of two
    assert info_f["alg_bytes_dual_step"] < info_s["alg_bytes_dual_step"]
    nb = len(c.blocks)
    sigma = np.linspace(0.8, 1.2, nb)
    fus = gpu_dual(c, plan, c.V, c.eps, sigma)
    plan.set_flags(FUSED_GH | GRAPH)
    fus_g = gpu_dual(c, plan, c.V, c.eps, sigma)
    plan.set_flags(0)
    sep = gpu_dual(c, plan, c.V, c.eps, sigma)
    for a_, b_ in zip(fus, fus_g):                    # graph replay equals the eager step
        assert all(np.array_equal(x, y) for x, y in zip(a_, b_)) if isinstance(a_, list) else np.array_equal(a_, b_)
    op = c.op if prec == "c64" else c.operator(c.theta, prec=prec)
    Vp_o, grad_o, rho_o, res_o = oracle.dual_step(op, {l: x.astype(np.float64) for l, x in c.Xt.items()},
                                                  c.V, c.Y, c.eps, sigma)
    Vp_f, grad_f, rho_f, res_f = fus
    Vp_s, grad_s, rho_s, res_s = sep
    ev = rel_l2(np.concatenate(Vp_f), np.concatenate(Vp_o))
    _say("  v+ vs oracle", ev, "vs separate", rel_l2(np.concatenate(Vp_f), np.concatenate(Vp_s)))
    assert ev <= 1e-5
    assert rel_l2(rho_f, rho_o) <= 1e-5 and rel_l2(res_f, res_o) <= 1e-5
    assert np.array_equal(rho_f, rho_s) and np.array_equal(res_f, res_s)   # same gather, same norms
    for l in range(c.prob.L):
        e = rel_l2(grad_f[l], grad_o[l])
        _say("  grad ch", l, "vs oracle", e, "vs separate", rel_l2(grad_f[l], grad_s[l]))
        assert e <= 1e-5


@pytest.mark.parametrize("prec", ["f16", "c64"])
def test_fused_over_pitch_classes(prec, monkeypatch):
    """The one-pass step over all channels runs once per pitch class on the
    items regrouped by pitch, largest first.  Forced to one class per pitch,
    it must still give v+ bitwise equal to the two passes, equal norms, and
    grad within the bound of the oracle."""
    from test_gpu_parity import gpu_dual
    from paper_2209_07604_amd import FUSED_GH
    import oracle
    monkeypatch.setenv("PHI_PITCH_CLASS_ITEMS", "1")
    c = case("C2s")
    plan = c.plan(g_prec=prec)           # the variable is read when the plan is created
    plan.set_tuning(16, 0)
    plan.set_flags(FUSED_GH)
    info = plan.info()
    _say("[fused classes]", prec, "pitch classes", info["pitch_classes"])
    assert info["fused"] == 1 and info["pitch_classes"] > 1
    nb = len(c.blocks)
    sigma = np.linspace(0.9, 1.1, nb)
    Vp_f, grad_f, rho_f, res_f = gpu_dual(c, plan, c.V, c.eps, sigma)
    plan.set_flags(0)
    Vp_s, grad_s, rho_s, res_s = gpu_dual(c, plan, c.V, c.eps, sigma)
    assert all(np.array_equal(x, y) for x, y in zip(Vp_f, Vp_s))
    assert np.array_equal(rho_f, rho_s) and np.array_equal(res_f, res_s)
    op = c.op if prec == "c64" else c.operator(c.theta, prec=prec)
    _, grad_o, rho_o, _ = oracle.dual_step(op, {l: x.astype(np.float64) for l, x in c.Xt.items()},
                                           c.V, c.Y, c.eps, sigma)
    assert rel_l2(rho_f, rho_o) <= 1e-5
    for l in range(c.prob.L):
        e = rel_l2(grad_f[l], grad_o[l])
        _say("  grad ch", l, "vs oracle", e)
        assert e <= 1e-5



@pytest.mark.parametrize("prec", ["f16", "c64"])
def test_fused_persistent_grid(prec):
    """A persistent grid smaller than the item count makes each work-group run
    many items, so the one pass prefetches the next item's descriptor and grid
    region while the current one runs.  v+ and the norms must equal the run
    with one work-group per item bitwise, and grad to the last bit as well
    (the merge order does not depend on the launch shape)."""
    from test_gpu_parity import gpu_dual
    from paper_2209_07604_amd import FUSED_GH, PERSISTENT, GRAPH
    c = case("C2s")
    plan = c.plan(g_prec=prec)
    plan.set_tuning(16, 0)
    plan.set_flags(FUSED_GH)
    n_items = plan.info()["n_items"]
    sigma = np.linspace(0.9, 1.1, len(c.blocks))
    ref = gpu_dual(c, plan, c.V, c.eps, sigma)
    for pb in (97, 1024):
        plan.set_tuning(16, pb)
        plan.set_flags(FUSED_GH | PERSISTENT | GRAPH)
        info = plan.info()
        _say("[fused persistent]", prec, "items", n_items, "grid", info["persist_blocks"])
        assert info["fused"] == 1 and info["persist_blocks"] == pb and pb < n_items
        got = gpu_dual(c, plan, c.V, c.eps, sigma)
        assert all(np.array_equal(x, y) for x, y in zip(got[0], ref[0]))
        assert np.array_equal(got[1], ref[1])
        assert np.array_equal(got[2], ref[2]) and np.array_equal(got[3], ref[3])


@pytest.mark.parametrize("fused", [False, True])
def test_nonfinite_norm_reported_once(fused):
    """A NaN in one block's data makes that block's FP64 norm non-finite: the
    dual step records it on the device, phi_plan_check reports
    PHI_ERR_NONFINITE once and clears the flag, and a clean step afterwards
    checks OK.  (Only the data is non-finite; every kernel runs normally.)"""
    from paper_2209_07604_amd import FUSED_GH, PhiError
    from paper_2209_07604_amd._lib import STATUS
    c = case("C2s")
    plan = c.plan(g_prec="f16")
    plan.set_tuning(16, 0)
    plan.set_flags(FUSED_GH if fused else 0)
    assert plan.info()["fused"] == (1 if fused else 0)
    xt = torch.from_numpy(c.cube(c.Xt)).cuda()
    Y = [y.copy() for y in c.Y]
    Y[2][5] = np.nan
    y_bad = plan.to_plan(torch.from_numpy(c.flat(Y).astype(np.complex64)).cuda())
    y_ok = plan.to_plan(torch.from_numpy(c.flat(c.Y).astype(np.complex64)).cuda())
    v0 = plan.to_plan(torch.from_numpy(c.flat(c.V).astype(np.complex64)).cuda())
    eps = torch.from_numpy(np.asarray(c.eps, np.float64)).cuda()
    v = v0.clone()
    _, rho, _ = plan.dual_step(xt, v, y_bad, eps)
    with pytest.raises(PhiError) as ei:
        plan.check()
    assert STATUS[ei.value.code] == "PHI_ERR_NONFINITE"
    r = rho.cpu().numpy()
    assert not np.isfinite(r[2]) and np.all(np.isfinite(np.delete(r, 2)))
    plan.check()                                   # the flag was cleared
    v = v0.clone()
    _, rho, _ = plan.dual_step(xt, v, y_ok, eps)
    plan.check()
    assert np.all(np.isfinite(rho.cpu().numpy()))
