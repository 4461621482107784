"""Throughput of the Phi -> l2-ball -> Phi^dagger data-fidelity step on MI355X.

One step = one l2ball_dual_step over every (channel, block) of the workload:
Z + 2-D FFT, G gather with the residual, FP64 block norms and projection
scale, G^H scatter of the new dual variable, merge, inverse FFT and Z^T.

Workload (default): 16 channels x 4 blocks, 1024 x 1024 image (2048 x 2048
grid), 1.5M visibilities per channel, w-projection stencils 7x7 .. 17x17,
30 dB input SNR, synthetic (seeded) data shaped like the paper's wideband VLA
data.  Forms timed on the same data: plain FP32 (complex64 G, every stage
launched per channel), batched FP32, batched FP16-G (the headline), batched
BF16-G; batched forms replay a hipGraph.  On direction-independent workloads
(one window size) the form batched_kb evaluates the Kaiser-Bessel taps in the
kernels instead of reading stored G; fused_<prec> runs the dual step in one
pass over G (PHI_FUSED_GH).  The autotuner picks one pass or two for the
batched forms; twopass_<prec> times the same tuning with gather and scatter as
separate passes, reported as roofline_two_pass.

Prints ONE JSON line.  Inputs are resident in HBM before timing starts.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Φ+Φ† visibilities/s and HBM GB/s, batched FP16-G vs plain FP32 at ≤2e-3 err"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("paper_2209_07604_amd/csrc/phi_kernels.hip", "paper_2209_07604_amd/csrc/phi_host.cpp"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel, launch_alg_bytes):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def generate(name, log_every=8, channels=0, windows=True):
    """Problem, per-block (base, S, windows or None) and per-block continuous
    grid coordinates [M, 2] (for the Kaiser-Bessel form)."""
    import synth
    prob = synth.make_problem(name)
    if channels and channels < prob.L:
        sel = np.linspace(0, prob.L - 1, channels).round().astype(int)
        prob = synth.make_problem(name, L=channels, n_blocks=[prob.n_blocks[l] for l in sel],
                                  n_vis=[prob.n_vis[l] for l in sel],
                                  nu=None if prob.nu is None else prob.nu[sel])
    t0 = time.time()
    blocks, kappas, wtab = [], [], []
    K = np.array([prob.Ky, prob.Kx], dtype=np.float64)
    for k, (l, b) in enumerate(prob.block_list()):
        blk = prob.block(l, b)
        w = blk.windows(np.complex64)[0] if windows else None
        blocks.append((blk.base, blk.S, w))
        kappas.append(blk.omega * K / (2 * np.pi))
        # the generator's w-kernel tables (half-width h, chirp parameter a)
        # for rows without DDE, as the device G builder takes them
        if not prob.dde:
            h = ((blk._skw - 7) // 2).astype(np.int32)
            a = prob.w_max_cells * blk.w
            wtab.append((h, np.where(np.round(a) > h, h.astype(np.float64), a)))
        if k % log_every == 0:
            log("[bench] generated block %d/%d (%.0f s)" % (k + 1, len(prob.block_list()), time.time() - t0))
    generate.seconds = time.time() - t0
    return prob, blocks, kappas, wtab


def cpu_baseline(prob, plan, theta, budget_s=30.0):
    """The FP64 oracle's dual step on channel 0 of the same workload, timed on
    the host cores (numpy/scipy as they stand).  The same inputs then go
    through the headline GPU plan, and its channel-0 outputs are compared with
    the oracle's (error of the timed form against FP64)."""
    import torch
    import oracle
    from oracle.dual import block_radii
    t_setup = time.time()
    nb0 = prob.n_blocks[0]
    sel = [(0, b) for b in range(nb0)]
    rng = np.random.default_rng(5)
    op = oracle.Operator.from_problem(prob, {k: theta[i] for i, k in enumerate(sel)}, blocks=sel)
    x = prob.image(0).astype(np.float64)
    Y = op.forward({0: x})
    V = [0.1 * (rng.standard_normal(len(y)) + 1j * rng.standard_normal(len(y))) for y in Y]
    Y = [y + (rng.standard_normal(len(y)) + 1j * rng.standard_normal(len(y))) / np.sqrt(2) for y in Y]
    eps = block_radii(prob.n_vis[0])
    log("[bench] cpu baseline set-up %.1f s" % (time.time() - t_setup))
    n, t_tot = 0, 0.0
    while n == 0 or (t_tot < budget_s / 3 and n < 3):
        t0 = time.perf_counter()
        Vp_o, grad_o, rho_o, res_o = oracle.dual_step(op, {0: 0.5 * x}, V, Y, eps)
        t_tot += time.perf_counter() - t0
        n += 1
    m = int(sum(prob.n_vis[0]))
    base = {"value": m * n / t_tot, "unit": "visibilities/s", "cores": 1, "kind": "oracle",
            "sample": "channel 0 (%d blocks, %d visibilities, %dx%d grid) of the same workload, FP64 "
                      "numpy/scipy dual step, %d run(s), %.2f s each; numpy.fft and scipy.sparse run "
                      "single-threaded" % (nb0, m, prob.Ky, prob.Kx, n, t_tot / n)}
    # the same channel-0 inputs through the GPU plan (other channels: zero data)
    M = plan.M
    vh = np.zeros(M, np.complex64)
    yh = np.zeros(M, np.complex64)
    vh[:m] = np.concatenate(V)
    yh[:m] = np.concatenate(Y)
    dev = plan.device
    xt = torch.zeros((plan.L, prob.Ny, prob.Nx), dtype=torch.float32, device=dev)
    xt[0] = torch.from_numpy((0.5 * x).astype(np.float32))
    v = plan.to_plan(torch.from_numpy(vh).to(dev))
    y = plan.to_plan(torch.from_numpy(yh).to(dev))
    e_all = np.ones(plan.nblk)
    e_all[:nb0] = eps
    grad, rho, res = plan.dual_step(xt, v, y, torch.from_numpy(e_all).to(dev))
    vp = plan.from_plan(v).cpu().numpy()[:m].astype(np.complex128)
    g0 = grad[0].cpu().numpy().astype(np.float64)
    r0 = rho.cpu().numpy()[:nb0]

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    err = {"v_plus": rel(vp, np.concatenate(Vp_o)), "grad": rel(g0, grad_o[0]), "rho": rel(r0, rho_o),
           "sample": "channel 0, all %d blocks, same inputs as the cpu baseline" % nb0}
    return base, err


def _event_ms(fn, n):
    """Average milliseconds of fn() over n calls (HIP events on the current stream)."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(n):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def stream_copy_gbs(dev, mib=2048):
    """Device-to-device copy rate (read + write bytes / time) of a plain
    library copy of a 2 GiB buffer: a practical streaming bound on this GPU."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ms = _event_ms(lambda: dst.copy_(src), 10)
    del src, dst
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def time_extras(p, x, xt, v0, y, eps, steps, warmup, dev):
    """phi_forward and phi_adjoint alone, and the regularizer-free PDFB
    iteration (dual step + primal step + adaptive bounds) on the same plan."""
    import torch
    L, nblk = p.L, p.nblk
    yv = torch.empty(p.M, dtype=torch.complex64, device=dev)
    img = torch.empty_like(x)
    for _ in range(warmup):
        p.forward(x, out=yv)
        p.adjoint(yv, out=img)
    torch.cuda.synchronize()
    out = {"forward_ms": _event_ms(lambda: p.forward(x, out=yv), steps),
           "adjoint_ms": _event_ms(lambda: p.adjoint(yv, out=img), steps)}
    # step sizes: sigma_b = 1 / ||Phi_l||^2 (10 power steps), tau_l = 0.9
    w = x.clone()
    nu = p.power_iteration(w, 10, tmp=img)
    ch = torch.repeat_interleave(torch.arange(L, device=dev), torch.tensor(p._n_blocks.astype(np.int64), device=dev))
    sigma = (1.0 / nu)[ch].contiguous()
    tau = torch.full((L,), 0.9, dtype=torch.float64, device=dev)
    rule = p.eps_rule()
    xi, xti, v, e = x.clone(), x.clone(), v0.clone(), eps.clone()
    grad = torch.empty_like(x)
    rho = torch.empty(nblk, dtype=torch.float64, device=dev)
    res = torch.empty_like(rho)
    var = torch.empty((L, 2), dtype=torch.float64, device=dev)
    state = torch.zeros((nblk, 3), dtype=torch.int32, device=dev)

    def run(n):
        p.pdfb_run(xi, xti, v, y, e, tau, n, sigma=sigma, rule=rule, state=state, grad=grad, rho=rho, res=res,
                   var=var)
    run(warmup)
    torch.cuda.synchronize()
    ms = _event_ms(lambda: run(steps), 1) / steps
    p.set_timing(True)
    run(steps)
    torch.cuda.synchronize()
    p.set_timing(False)
    stages, calls = p.get_timing()
    px = L * p.ny * p.nx
    prim_ms = stages["pdfb_primal"] / max(calls, 1)
    out["pdfb"] = {"ms_per_iter": ms, "primal_ms": prim_ms, "eps_update_ms": stages["eps_update"] / max(calls, 1),
                   "primal_alg_bytes": 16.0 * px,
                   "primal_GBs": 16.0 * px / (prim_ms * 1e-3) / 1e9,
                   "rule": "adaptive l2 bounds (lambda 0.99/1.01/0.618, var_tol 1e-3, min_gap 10)",
                   "steps": "sigma_b = 1/||Phi_l||^2 (10 power steps), tau_l = 0.9"}
    return out


def time_gbuild(p, kappas, wtab, xt, v0, y, eps, dev):
    """Rebuild every block's G on the device (phi_plan_build_g) from the
    generator's tables, timed on the wall clock (each call is synchronous),
    then one dual step on the rebuilt G against the step on the host-loaded
    G (same inputs)."""
    import torch
    v = v0.clone()
    grad0, _, _ = p.dual_step(xt, v, y, eps)
    vp0, grad0 = v.clone(), grad0.clone()
    tabs = [(torch.from_numpy(np.ascontiguousarray(k)).to(dev), torch.from_numpy(h).to(dev),
             torch.from_numpy(np.ascontiguousarray(a)).to(dev)) for k, (h, a) in zip(kappas, wtab)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, (k, h, a) in enumerate(tabs):
        p.build_g(b, k, h, a, J=7)
    ms = (time.perf_counter() - t0) * 1e3
    v = v0.clone()
    grad1, _, _ = p.dual_step(xt, v, y, eps)
    torch.cuda.synchronize()
    rel = lambda a_, b_: float(torch.linalg.vector_norm((a_ - b_).to(torch.complex128)) /
                               torch.linalg.vector_norm(b_.to(torch.complex128)))
    info = p.info()
    return {"ms": ms, "taps": int(info["n_taps"]), "G_bytes": int(info["g_bytes"]),
            "G_GB_per_s_written": info["g_bytes"] / (ms * 1e-3) / 1e9,
            "host_generation_s": generate.seconds,
            "dual_step_rel_diff_vs_host_G": {"v_plus": rel(v, vp0), "grad": rel(grad1, grad0)},
            "note": "FP64 rows (Kaiser-Bessel taps (*) w-chirp) rounded once to the stored precision; wall "
                    "clock of one synchronous call per block; host_generation_s is the seeded generator "
                    "building the same windows on the host; the host-loaded G came from complex64 windows "
                    "(rounded twice), hence the small step difference"}


def run_dr(args, prob, blocks, theta, y_user, starts, s_y, s_x, results, dev):
    """Reduce every block (host, FP64) and time the reduced dual step with the
    same precision and launch form as the headline; returns a summary."""
    import torch
    from paper_2209_07604_amd import Plan, dr_reduce, GRAPH, PERSISTENT
    t0 = time.time()
    outs = []
    for k, (b_, S_, w_) in enumerate(blocks):
        outs.append(dr_reduce(prob.Ky, prob.Kx, b_, S_, w_, theta[k],
                              y_user[starts[k]:starts[k + 1]].astype(np.complex128)))
    t_red = time.time() - t0
    n_red = [len(o["S"]) for o in outs]
    log("[bench] reduction %.1f s, M' per block %s" % (t_red, n_red))
    prec = "f16"
    p = Plan(prob.Ny, prob.Nx, prob.n_blocks, n_red, np.concatenate([o["base"] for o in outs]),
             np.concatenate([o["S"] for o in outs]), s_y, s_x, None, g_prec=prec, device=dev)
    for k, o in enumerate(outs):
        p.load_g(k, o["windows"].astype(np.complex64))
    yr = p.to_plan(torch.from_numpy(np.concatenate([o["y"] for o in outs]).astype(np.complex64)).to(dev))
    del outs
    p.autotune(3)
    p.set_flags(GRAPH | (PERSISTENT if p.info()["persist_blocks"] else 0))
    mr = int(sum(n_red))
    eps = torch.tensor([np.sqrt(m + 2.0 * np.sqrt(m)) for m in n_red], dtype=torch.float64, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    v = (0.1 * torch.complex(torch.randn(mr, generator=gen, device=dev),
                             torch.randn(mr, generator=gen, device=dev))).contiguous()
    xt = torch.from_numpy(np.stack([0.5 * prob.image(l) for l in range(prob.L)])).to(dev)
    grad = torch.empty_like(xt)
    rho = torch.empty(len(n_red), dtype=torch.float64, device=dev)
    res = torch.empty_like(rho)
    for _ in range(args.warmup):
        p.dual_step(xt, v, yr, eps, None, grad, rho, res)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        p.dual_step(xt, v, yr, eps, None, grad, rho, res)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    info = p.info()
    M = int(sum(len(s) for (_, s, _) in blocks))
    ref = results.get("batched_f16")
    out = {"M": M, "M_reduced": mr, "M_over_M_reduced": M / mr, "taps_G": ref["info"]["n_taps"] if ref else None,
           "taps_H": info["n_taps"], "g_bytes_f16": ref["info"]["g_bytes"] if ref else None,
           "h_bytes_f16": info["g_bytes"], "reduce_host_s": t_red, "ms_per_step_reduced": ms,
           "ms_per_step_unreduced": ref["ms_per_step"] if ref else None,
           "visibilities_per_s_reduced": M / (ms * 1e-3), "tile": info["tile"]}
    if ref:
        out["speedup"] = ref["ms_per_step"] / ms
    log("[bench] reduced step: %s" % out)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--forms", default="plain_c64,batched_c64,batched_f16,twopass_f16,batched_bf16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="fix the tile edge (skips the autotuner)")
    ap.add_argument("--persist", type=int, default=0, help="persistent G-stage grid with --tile")
    ap.add_argument("--channels", type=int, default=0, help="use this many channels of the configuration")
    ap.add_argument("--dr", action="store_true",
                    help="also time the visibility-gridding reduced step (Section 3.4) on the same data")
    ap.add_argument("--no-gbuild", action="store_true", help="skip timing the device G builder")
    ap.add_argument("--device-g", action="store_true",
                    help="build G on the device from the generator's tables (no host windows)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, run one plain device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the data-fidelity step shards by channel with no exchange, "
              "and this build runs on a single MI355X; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2209_07604_amd import Plan, PER_CHANNEL, GRAPH, PERSISTENT, FUSED_GH

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    forms = [f for f in args.forms.split(",") if f]
    if args.device_g and args.dr:
        print("--device-g and --dr are exclusive (the reduction needs host windows)", file=sys.stderr)
        sys.exit(2)
    prob, blocks, kappas, wtab = generate(args.config, channels=args.channels,
                                          windows=not args.device_g and
                                          (args.dr or any(not f.endswith("_kb") for f in forms)))
    if args.device_g and not wtab:
        print("--device-g needs a workload without DDE", file=sys.stderr)
        sys.exit(2)
    L = prob.L
    n_vis = [len(s) for (_, s, _) in blocks]
    base = np.concatenate([b for (b, _, _) in blocks])
    S = np.concatenate([s for (_, s, _) in blocks])
    s_y, s_x = prob.deapodisation()
    M = int(len(S))
    precs = sorted({f.split("_")[1] for f in forms}, key=["c64", "f16", "bf16", "kb"].index)
    plans = {}
    t0 = time.time()
    for prec in precs:
        p = Plan(prob.Ny, prob.Nx, prob.n_blocks, n_vis, base, S, s_y, s_x, None, g_prec=prec, device=dev)
        for k, (_, _, w) in enumerate(blocks):
            if prec == "kb":
                p.load_kb(k, kappas[k])   # taps evaluated in the kernels
            elif args.device_g:           # rows computed on the device from the generator's tables
                p.build_g(k, torch.from_numpy(np.ascontiguousarray(kappas[k])).to(dev),
                          torch.from_numpy(wtab[k][0]).to(dev),
                          torch.from_numpy(np.ascontiguousarray(wtab[k][1])).to(dev), J=7)
            else:
                p.load_g(k, w)
        plans[prec] = p
        log("[bench] plan %s ready (%.0f s), info %s" % (prec, time.time() - t0, p.info()))
    if not args.dr:
        del blocks

    # inputs: x~ = x/2, y = theta Phi0 x + n at 30 dB (theta from the c64 form), v ~ 0.1 CN
    gen = torch.Generator(device=dev)
    gen.manual_seed(220907604)
    x = torch.from_numpy(np.stack([prob.image(l) for l in range(L)])).to(dev)
    log("[bench] images ready (%.0f s)" % (time.time() - t0))
    pref = plans[precs[0]]
    y0 = pref.forward(x)
    ch_of_blk = np.repeat(np.arange(L), prob.n_blocks)
    starts = np.concatenate([[0], np.cumsum(n_vis)])
    pw = np.zeros(L)
    y0h = y0.abs().square().double()
    for k in range(len(n_vis)):
        pw[ch_of_blk[k]] += y0h[starts[k]:starts[k + 1]].sum().item()
    m_ch = np.array([sum(m) for m in prob.n_vis], dtype=np.float64)
    theta_ch = 1.0 / np.sqrt(pw / m_ch * 1e-3)
    log("[bench] noiseless data and channel powers ready (%.0f s)" % (time.time() - t0))
    theta = theta_ch[ch_of_blk]
    noise = torch.complex(torch.randn(M, generator=gen, device=dev), torch.randn(M, generator=gen, device=dev))
    noise = noise * (0.5 ** 0.5)
    th_vis = torch.from_numpy(np.repeat(theta, n_vis).astype(np.float32)).to(dev)
    y_plan = {}
    for prec, p in plans.items():
        p.set_theta(theta)
        y_plan[prec] = p.to_plan((th_vis * pref.from_plan(y0) + noise).contiguous())
    v_init = (0.1 * torch.complex(torch.randn(M, generator=gen, device=dev),
                                  torch.randn(M, generator=gen, device=dev))).contiguous()
    xt = (0.5 * x).contiguous()
    # chi-square radii (eq. 2): eps_l^2 = M_l + 2 sqrt(M_l), eps_lb^2 = eps_l^2 M_lb / M_l
    eps_h = []
    for nv in prob.n_vis:
        ml = float(sum(nv))
        eps_h += [np.sqrt((ml + 2.0 * np.sqrt(ml)) * m / ml) for m in nv]
    eps = torch.tensor(eps_h, dtype=torch.float64, device=dev)
    nblk = len(n_vis)
    torch.cuda.synchronize()
    log("[bench] inputs resident (%.0f s)" % (time.time() - t0))

    results = {}
    for form in forms:
        kind, prec = form.split("_")
        p = plans[prec]
        v = p.to_plan(v_init)
        v0 = v.clone()
        grad = torch.empty((L, prob.Ny, prob.Nx), dtype=torch.float32, device=dev)
        rho = torch.empty(nblk, dtype=torch.float64, device=dev)
        res = torch.empty(nblk, dtype=torch.float64, device=dev)
        if kind in ("batched", "fused", "twopass") and args.tile:
            p.set_tuning(args.tile, args.persist)
        elif kind in ("batched", "fused") and not args.no_autotune:
            rc = p.autotune(3)
            log("[bench] autotune %s -> rc %d, tile %d, persist %d" % (
                prec, rc, p.info()["tile"], p.info()["persist_blocks"]))
        # the autotuner may have chosen the one-pass dual step (info "fused");
        # fused_<prec> forces it; plain_<prec> and twopass_<prec> (the batched
        # form on the same tuning, gather and scatter as separate passes) never
        # use it
        fused = kind == "fused" or (kind == "batched" and bool(p.info()["fused"]))
        flags_now = (p.info()["persist_blocks"] and PERSISTENT) | (FUSED_GH if fused else 0)
        p.set_flags((PER_CHANNEL if kind == "plain" else GRAPH) | flags_now)
        log("[bench] %s: warm-up" % form)
        for _ in range(args.warmup):
            v.copy_(v0)
            p.dual_step(xt, v, y_plan[prec], eps, None, grad, rho, res)
        v.copy_(v0)
        torch.cuda.synchronize()
        log("[bench] %s: timing %d steps" % (form, args.steps))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t_wall = time.perf_counter()
        e0.record()
        for _ in range(args.steps):
            p.dual_step(xt, v, y_plan[prec], eps, None, grad, rho, res)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_wall
        ms = e0.elapsed_time(e1) / args.steps
        p.check()
        # per-stage HIP-event timing over a second run of the same steps
        # (stage-by-stage launches of the same kernels on the same stream)
        p.set_flags((PER_CHANNEL if kind == "plain" else 0) | flags_now)
        v.copy_(v0)
        torch.cuda.synchronize()
        p.set_timing(True)
        for _ in range(args.steps):
            p.dual_step(xt, v, y_plan[prec], eps, None, grad, rho, res)
        torch.cuda.synchronize()
        p.set_timing(False)
        stages, calls = p.get_timing()
        info = info_t = p.info()
        results[form] = dict(ms_per_step=ms, tile=info_t["tile"], persist_blocks=info_t["persist_blocks"],
                             one_pass=bool(fused), wall_ms_per_step=1e3 * wall / args.steps,
                             vis_per_s=M / (ms * 1e-3),
                             alg_GBs=info["alg_bytes_dual_step"] / (ms * 1e-3) / 1e9,
                             stage_ms={k_: v_ / max(calls, 1) for k_, v_ in stages.items()},
                             info=info, rho0=float(rho[0].item()))
        log("[bench] %s: %.3f ms/step, %.3g vis/s, stages %s" % (
            form, ms, M / (ms * 1e-3), {k_: round(v_ / max(calls, 1), 3) for k_, v_ in stages.items()}))

    line_gb = None
    if wtab and not args.no_gbuild and "batched_f16" in results:
        log("[bench] device G builder")
        line_gb = time_gbuild(plans["f16"], kappas, wtab, xt, plans["f16"].to_plan(v_init), y_plan["f16"], eps, dev)
        log("[bench] G builder: %s" % line_gb)
    del kappas
    if args.dr:
        line_dr = run_dr(args, prob, blocks, theta, (th_vis * pref.from_plan(y0) + noise).cpu().numpy(),
                         starts, s_y, s_x, results, dev)
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy of %d MiB done" % args.calib_copy_mib)
        del src, dst
    head = "batched_f16" if "batched_f16" in results else forms[-1]
    hp = plans[head.split("_")[1]]
    # the headline form's launch settings (a later form may have changed the plan's flags)
    hp.set_flags(GRAPH | (PERSISTENT if hp.info()["persist_blocks"] else 0) |
                 (FUSED_GH if results[head]["one_pass"] else 0))
    log("[bench] %s: forward, adjoint and PDFB iterations" % head)
    extras = time_extras(hp, x, xt, hp.to_plan(v_init), y_plan[head.split("_")[1]], eps, args.steps, args.warmup,
                         dev)
    # (not in counter runs: their only large copy must be the calibration copy)
    copy_gbs = None if args.calib_copy_mib else stream_copy_gbs(dev)
    log("[bench] extras %s, stream copy %s GB/s" % (extras, copy_gbs))
    if "batched_kb" in results and "batched_f16" in results:
        results["batched_kb"]["speedup_vs_batched_f16"] = (results["batched_f16"]["ms_per_step"] /
                                                           results["batched_kb"]["ms_per_step"])
    r = results[head]
    info = r["info"]
    # dominant G kernel: gather, scatter, or the fused pass (which moves the
    # gather's algorithmic bytes: G once, metadata, v and y in, c out)
    cand = {k_: r["stage_ms"].get(k_, 0.0) for k_ in ("gather", "scatter", "dual_gs")}
    dom = max(cand, key=cand.get)
    alg = info["alg_bytes_scatter"] if dom == "scatter" else info["alg_bytes_gather"]
    dur = cand[dom] * 1e-3
    achieved = alg / dur / 1e9
    line = {
        "metric": METRIC,
        "value": r["vis_per_s"],
        "unit": "visibilities/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %d channels x %s blocks, %dx%d image (%dx%d grid), %d visibilities, "
                               "w-stencils %d..%d, 30 dB" % (args.config, L, sorted(set(prob.n_blocks)),
                                                              prob.Ny, prob.Nx, prob.Ky, prob.Kx, M,
                                                              int(S.min()), int(S.max())),
                   "g_source": "device builder" if args.device_g else "host windows",
                   "form": head.replace("_", " ") + " (hipGraph)", "g_storage": head.split("_")[1],
                   "taps": int(info["n_taps"])},
        "hbm_alg_GBs": r["alg_GBs"],
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_for(dom, alg), "alg_bytes_per_launch": alg,
                     "avg_launch_ms": dur * 1e3,
                     # the one-pass stage is one launch per pitch class; its bytes
                     # and time are per step (the sum over those launches)
                     "launches_per_step": info["pitch_classes"] if dom == "dual_gs" else 1,
                     "stream_copy_GBs": copy_gbs,
                     "frac_of_stream_copy": achieved / copy_gbs if copy_gbs else None},
        "forward_ms": extras["forward_ms"], "adjoint_ms": extras["adjoint_ms"],
        "pdfb": dict(extras["pdfb"], primal_frac=extras["pdfb"]["primal_GBs"] / HBM_PEAK_GBS),
        "forms": {k: {kk: vv for kk, vv in v.items() if kk != "info"} for k, v in results.items()},
    }
    two = "twopass_" + head.split("_")[1]
    if two in results and two != head:
        # the same step with gather and scatter as separate passes (G read
        # twice): its dominant kernel against the same peak
        r2 = results[two]
        c2 = {k_: r2["stage_ms"].get(k_, 0.0) for k_ in ("gather", "scatter")}
        d2 = max(c2, key=c2.get)
        a2 = info["alg_bytes_scatter"] if d2 == "scatter" else info["alg_bytes_gather"]
        ach2 = a2 / (c2[d2] * 1e-3) / 1e9
        line["roofline_two_pass"] = {"bound": "hbm", "kernel": d2, "achieved": ach2, "peak": HBM_PEAK_GBS,
                                     "unit": "GB/s", "frac": ach2 / HBM_PEAK_GBS, "traffic": traffic_for(d2, a2),
                                     "alg_bytes_per_launch": a2, "avg_launch_ms": c2[d2],
                                     "ms_per_step": r2["ms_per_step"],
                                     "frac_of_stream_copy": ach2 / copy_gbs if copy_gbs else None}
    if "plain_c64" in results:
        line["speedup_vs_plain_fp32"] = results["plain_c64"]["ms_per_step"] / r["ms_per_step"]
    if args.dr:
        line["dimensionality_reduction"] = line_dr
    if line_gb:
        line["g_builder"] = line_gb
    if not args.no_cpu_baseline:
        line["cpu_baseline"], line["err_vs_fp64_" + head] = cpu_baseline(prob, hp, theta)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
