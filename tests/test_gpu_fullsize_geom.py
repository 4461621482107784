"""Full-geometry parity on the largest images: one whole channel checked
against the FP64 oracle on every output (v+, grad, rho, r).

* 4096^2 images (8192^2 grid, 8192-point rows and columns), 16 channels of
  8M visibilities with 7 x 7 rows, G built on the device: the workload and
  launch form bench.py times (autotuned, hipGraph replay), and the one pass
  over G forced on a persistent grid.  Channel 0 carries the oracle's data;
  the other 15 carry seeded random data, so a channel mix-up would show in
  channel 0.  FP16 G: 2e-3 against the FP64 G, 1e-5 against the oracle run
  on the same rounded G.
* 1536 x 2560 images (3072 x 5120 grid: radix-3 columns, radix-5 rows), one
  channel of 3M visibilities in two blocks with w-stencils 7..17, host
  windows: complex64 G at 1e-5, FP16 G at 2e-3 against the FP64 G.
* 2048^2 images (4096^2 grid) with w + DDE windows 7..21 in 8 uneven blocks
  (one channel of the 64-channel workload), at the same bounds.
"""
import sys

import numpy as np
import pytest

from _cases import rel_l2, quantise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_channel(prob, l, windows, theta, gprec=None):
    """theta_b G_b of channel l's blocks as the oracle's operator."""
    import oracle
    s_y, s_x = prob.deapodisation()
    blks = []
    for b, (blk, w, off) in enumerate(windows):
        wq = w if gprec is None else quantise(w, gprec)
        blks.append(oracle.BlockG(l, theta, oracle.g_matrix(blk.base, blk.S, wq, off, prob.Ky, prob.Kx, theta)))
    return oracle.Operator(prob.Ny, prob.Nx, s_y, s_x, blks)


def _channel_inputs(prob, l, windows):
    """Oracle data of channel l: theta at 30 dB, y = theta Phi0 x + n,
    v ~ 0.1 CN, eps per block (all FP64, from the generator and the oracle)."""
    from oracle.dual import block_radii
    op1 = _oracle_channel(prob, l, windows, 1.0)
    x = prob.image(l).astype(np.float64)
    y0 = op1.forward({l: x})
    del op1
    m = float(sum(len(y) for y in y0))
    theta = 1.0 / np.sqrt(sum(float(np.vdot(y, y).real) for y in y0) / m * 1e-3)
    rng = np.random.default_rng(np.random.SeedSequence((220907604, 99, l)))
    Y = [theta * y + (rng.standard_normal(len(y)) + 1j * rng.standard_normal(len(y))) / np.sqrt(2) for y in y0]
    V = [0.1 * (rng.standard_normal(len(y)) + 1j * rng.standard_normal(len(y))) for y in Y]
    return dict(theta=theta, Y=Y, V=V, eps=block_radii(prob.n_vis[l]), Xt={l: 0.5 * x})


def _check(tag, got, want, eps, bound):
    vp, grad, rho, res = got
    Vp_o, grad_o, rho_o, res_o = want
    e = dict(v=rel_l2(vp, np.concatenate(Vp_o)), grad=rel_l2(grad, grad_o), rho=rel_l2(rho, rho_o),
             res=rel_l2(res, res_o))
    _say("[geom] %s: rel L2 v+ %.2e grad %.2e rho %.2e res %.2e (rho/eps %s)" % (
        tag, e["v"], e["grad"], e["rho"], e["res"], np.round(rho_o / eps, 3)))
    assert np.all(rho_o > eps)
    assert max(e.values()) <= bound


@pytest.mark.timeout(1200)
def test_c5_full_channel_headline():
    import oracle
    import synth
    from paper_2209_07604_amd import Plan, GRAPH, FUSED_GH, PERSISTENT
    prob = synth.make_problem("C5")
    L = prob.L
    tabs = []
    for l in range(L):
        blk = prob.block(l, 0)
        K = np.array([prob.Ky, prob.Kx], dtype=np.float64)
        tabs.append((blk, blk.omega * K / (2 * np.pi)))
    _say("[geom] C5 tables ready")
    blk0 = tabs[0][0]
    win0 = [(blk0,) + tuple(blk0.windows(np.complex128))]
    D = _channel_inputs(prob, 0, win0)
    _say("[geom] C5 channel-0 oracle inputs ready, theta %.4g" % D["theta"])
    n_vis = [t[0].M for t in tabs]
    base = np.concatenate([t[0].base for t in tabs])
    S = np.concatenate([t[0].S for t in tabs])
    s_y, s_x = prob.deapodisation()
    theta = np.ones(L)
    theta[0] = D["theta"]
    plan = Plan(prob.Ny, prob.Nx, prob.n_blocks, n_vis, base, S, s_y, s_x, theta, g_prec="f16")
    for k, (blk, kap) in enumerate(tabs):
        plan.build_g(k, torch.from_numpy(np.ascontiguousarray(kap)).cuda(), torch.from_numpy(blk.w_h).cuda(),
                     torch.from_numpy(np.ascontiguousarray(blk.w_a)).cuda(), J=7)
    _say("[geom] C5 plan with device G", plan.info())
    # channel 0: the oracle's data; channels 1..15: seeded random data
    rng = np.random.default_rng(np.random.SeedSequence((220907604, 98)))
    M0, M = n_vis[0], sum(n_vis)
    vh = np.empty(M, np.complex64)
    yh = np.empty(M, np.complex64)
    vh[:M0] = D["V"][0]
    yh[:M0] = D["Y"][0]
    vh[M0:] = 0.1 * (rng.standard_normal(M - M0) + 1j * rng.standard_normal(M - M0))
    yh[M0:] = 40.0 * (rng.standard_normal(M - M0) + 1j * rng.standard_normal(M - M0))
    xt = torch.from_numpy(np.stack([0.5 * prob.image(l) for l in range(L)]).astype(np.float32)).cuda()
    v0 = plan.to_plan(torch.from_numpy(vh).cuda())
    y = plan.to_plan(torch.from_numpy(yh).cuda())
    eps_h = np.concatenate([[D["eps"][0]], [float(np.sqrt(m + 2 * np.sqrt(m))) for m in n_vis[1:]]])
    eps = torch.from_numpy(eps_h).cuda()
    outs = {}
    for form in ("headline", "fused_persistent"):
        if form == "headline":
            plan.autotune(3)
            i = plan.info()
            plan.set_flags(GRAPH | (PERSISTENT if i["persist_blocks"] else 0) | (FUSED_GH if i["fused"] else 0))
        else:
            plan.set_tuning(16, 1024)
            plan.set_flags(GRAPH | PERSISTENT | FUSED_GH)
        _say("[geom] C5", form, plan.info())
        v = v0.clone()
        grad, rho, res = plan.dual_step(xt, v, y, eps)
        vp = plan.from_plan(v)[:M0].cpu().numpy()
        torch.cuda.synchronize()
        plan.check()
        outs[form] = (vp, grad[0].cpu().numpy().astype(np.float64), rho[:1].cpu().numpy(), res[:1].cpu().numpy())
    del plan, v0, y, xt
    torch.cuda.empty_cache()
    for gprec, bound in ((None, 2e-3), ("f16", 1e-5)):
        op = _oracle_channel(prob, 0, win0, D["theta"], gprec)
        want = oracle.dual_step(op, D["Xt"], D["V"], D["Y"], D["eps"])
        del op
        for form, got in outs.items():
            _check("C5 channel 0, %s vs oracle with %s G" % (form, gprec or "FP64"), got,
                   (want[0], want[1][0], want[2], want[3]), D["eps"], bound)


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("prec,bound", [("c64", 1e-5), ("f16", 2e-3)])
def test_c4_geometry_channel(prec, bound):
    import oracle
    import synth
    from paper_2209_07604_amd import Plan, GRAPH, FUSED_GH, PERSISTENT
    full = synth.make_problem("C4")
    prob = synth.make_problem("C4", L=1, n_blocks=[full.n_blocks[0]], n_vis=[full.n_vis[0]], nu=full.nu[:1])
    key = "c4"
    if key not in _C4:
        wins = []
        for b in range(prob.n_blocks[0]):
            blk = prob.block(0, b)
            wins.append((blk,) + tuple(blk.windows(np.complex128)))
        D = _channel_inputs(prob, 0, wins)
        op = _oracle_channel(prob, 0, wins, D["theta"])
        want = oracle.dual_step(op, D["Xt"], D["V"], D["Y"], D["eps"])
        del op
        _C4[key] = (wins, D, want)
        _say("[geom] C4 channel oracle ready")
    wins, D, want = _C4[key]
    s_y, s_x = prob.deapodisation()
    n_vis = [w[0].M for w in wins]
    plan = Plan(prob.Ny, prob.Nx, prob.n_blocks, n_vis, np.concatenate([w[0].base for w in wins]),
                np.concatenate([w[0].S for w in wins]), s_y, s_x, np.full(len(wins), D["theta"]), g_prec=prec)
    for k, w in enumerate(wins):
        plan.load_g(k, w[1])
    plan.autotune(3)
    i = plan.info()
    plan.set_flags(GRAPH | (PERSISTENT if i["persist_blocks"] else 0) | (FUSED_GH if i["fused"] else 0))
    _say("[geom] C4", prec, plan.info())
    xt = torch.from_numpy((0.5 * prob.image(0))[None].astype(np.float32)).cuda()
    v = plan.to_plan(torch.from_numpy(np.concatenate(D["V"]).astype(np.complex64)).cuda())
    y = plan.to_plan(torch.from_numpy(np.concatenate(D["Y"]).astype(np.complex64)).cuda())
    eps = torch.from_numpy(np.asarray(D["eps"], np.float64)).cuda()
    grad, rho, res = plan.dual_step(xt, v, y, eps)
    vp = plan.from_plan(v).cpu().numpy()
    torch.cuda.synchronize()
    plan.check()
    _check("C4 geometry channel 0, %s headline vs oracle with FP64 G" % prec,
           (vp, grad[0].cpu().numpy().astype(np.float64), rho.cpu().numpy(), res.cpu().numpy()),
           (want[0], want[1][0], want[2], want[3]), D["eps"], bound)


_C4 = {}


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("prec,bound", [("c64", 1e-5), ("f16", 2e-3)])
def test_c3_geometry_channel(prec, bound):
    """Channel 9 of the 64-channel w + DDE workload at its full geometry:
    2048^2 image (4096^2 grid, image-first transform), 8 uneven blocks
    (1.0e4 ... 9.8e4 visibilities, 3.4e5 in all), windows 7 ... 21 (the
    largest step class), host windows; autotuned launch form and hipGraph."""
    import oracle
    import synth
    from paper_2209_07604_amd import Plan, GRAPH, FUSED_GH, PERSISTENT
    full = synth.make_problem("C3")
    c = 9
    prob = synth.make_problem("C3", L=1, n_blocks=[full.n_blocks[c]], n_vis=[full.n_vis[c]], nu=full.nu[c:c + 1])
    if "c3" not in _C3:
        wins = []
        for b in range(prob.n_blocks[0]):
            blk = prob.block(0, b)
            wins.append((blk,) + tuple(blk.windows(np.complex128)))
        D = _channel_inputs(prob, 0, wins)
        op = _oracle_channel(prob, 0, wins, D["theta"])
        want = oracle.dual_step(op, D["Xt"], D["V"], D["Y"], D["eps"])
        del op
        _C3["c3"] = (wins, D, want)
        _say("[geom] C3 channel oracle ready")
    wins, D, want = _C3["c3"]
    s_y, s_x = prob.deapodisation()
    n_vis = [w[0].M for w in wins]
    S = np.concatenate([w[0].S for w in wins])
    assert S.min() == 7 and S.max() == 21 and len(wins) == 8
    plan = Plan(prob.Ny, prob.Nx, prob.n_blocks, n_vis, np.concatenate([w[0].base for w in wins]), S, s_y, s_x,
                np.full(len(wins), D["theta"]), g_prec=prec)
    for k, w in enumerate(wins):
        plan.load_g(k, w[1])
    plan.autotune(3)
    i = plan.info()
    assert i["fft_image_first"] == 1
    plan.set_flags(GRAPH | (PERSISTENT if i["persist_blocks"] else 0) | (FUSED_GH if i["fused"] else 0))
    _say("[geom] C3", prec, plan.info())
    xt = torch.from_numpy((0.5 * prob.image(0))[None].astype(np.float32)).cuda()
    v = plan.to_plan(torch.from_numpy(np.concatenate(D["V"]).astype(np.complex64)).cuda())
    y = plan.to_plan(torch.from_numpy(np.concatenate(D["Y"]).astype(np.complex64)).cuda())
    eps = torch.from_numpy(np.asarray(D["eps"], np.float64)).cuda()
    grad, rho, res = plan.dual_step(xt, v, y, eps)
    vp = plan.from_plan(v).cpu().numpy()
    torch.cuda.synchronize()
    plan.check()
    _check("C3 geometry channel 9, %s headline vs oracle with FP64 G" % prec,
           (vp, grad[0].cpu().numpy().astype(np.float64), rho.cpu().numpy(), res.cpu().numpy()),
           (want[0], want[1][0], want[2], want[3]), D["eps"], bound)


_C3 = {}
