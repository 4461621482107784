"""Throughput of the Phi -> l2-ball -> Phi^dagger data-fidelity step on MI355X.

One step = one l2ball_dual_step over every (channel, block) of the workload:
Z + 2-D FFT, G gather with the residual, FP64 block norms and projection
scale, G^H of the new dual variable, merge, inverse FFT and Z^T.

Workload (default C5): 16 channels x 1 block, 4096 x 4096 image (8192 x 8192
grid), 8M visibilities per channel (1.28e8 in all), 7 x 7 Kaiser-Bessel rows
(direction-independent data, the dimensionality-reduction experiment's
shape), 30 dB input SNR, synthetic (seeded) data shaped like the paper's
wideband VLA data.  G is computed on the device by the library's builder from
the per-visibility grid coordinates (host windows with --host-g).

Forms timed on the same resident data: plain FP32 (complex64 G, every stage
launched per channel, two passes over G), batched FP32, batched FP16-G (the
headline), the same FP16 plan with two passes over G, batched BF16-G.  The
batched forms are autotuned (tile edge, launch shape, one pass or two over G)
and replay a hipGraph.  Plans are built one precision at a time and freed
after their forms, so the largest workloads fit the GPU.

Roofline accounting: every stage is charged the algorithmic bytes of the
minimal-pass design (per visibility 2 S^2 b_G + 48 B over the step, with G
read by the gather and again by G^H; per channel 48 K + 8 N B), split over
the stages that do that work; the one-pass stage, which replaces the gather
and the G^H pass, is charged both G reads.  `roofline` is the dominant stage;
`traffic` is the HBM byte count from a committed rocprofv3 counter run of the
same kernels (null when the sources changed since).

The CPU baseline is the FP64 oracle's dual step on whole channels of the same
workload, one channel per process (the oracle as written: numpy.fft and
scipy.sparse, single-threaded in each process), timed together on the host.
Its channel-0 inputs also run through every GPU form, which gives each form's
error against FP64.

Prints ONE JSON line.  Inputs are resident in HBM before timing starts.
"""
import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Φ+Φ† visibilities/s and HBM GB/s, batched FP16-G vs plain FP32 at ≤2e-3 err"
HBM_PEAK_GBS = 8000.0
STAGES_G = ("gather", "scatter", "dual_gs")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("paper_2209_07604_amd/csrc/phi_kernels.hip", "paper_2209_07604_amd/csrc/phi_host.cpp"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(workload, kernel):
    """HBM bytes per step of one stage from the committed rocprofv3 counter
    summary of this workload, if it was taken on the current kernel sources;
    else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
    except ValueError:
        return None
    w = t.get("workloads", {}).get(workload)
    if not w or w.get("source_hash") != kernel_source_hash():
        return None
    k = w.get("stages", {}).get(kernel)
    return None if k is None else k.get("bytes_per_step")


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    mem_gb = avail_gb = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal:"):
                mem_gb = int(line.split()[1]) / 1e6
            elif line.startswith("MemAvailable:"):
                avail_gb = int(line.split()[1]) / 1e6
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model, "ram_GB": mem_gb,
            "ram_available_GB": avail_gb}


# ------------------------------------------------------------ CPU baseline
def _oracle_worker(config, l, sample, barrier, q_early, q_out, omp):
    """One channel of the workload through the FP64 oracle (own process)."""
    os.environ["OMP_NUM_THREADS"] = str(omp)
    try:
        import synth
        import oracle
        from oracle.dual import block_radii
        prob = synth.make_problem(config)
        sel = [(l, b) for b in range(prob.n_blocks[l])]
        t0 = time.time()
        op = oracle.Operator.from_problem(prob, None, blocks=sel)
        x = prob.image(l).astype(np.float64)
        Y0 = op.forward({l: x})
        ml = float(sum(prob.n_vis[l]))
        # 30 dB input SNR, then whitened: theta = 1 / sigma (in place on the CSR data)
        theta = 1.0 / np.sqrt(sum(float(np.vdot(y, y).real) for y in Y0) / ml * 1e-3)
        for blk in op.blocks:
            blk.G.data *= theta
            blk.theta = theta
        rng = np.random.default_rng(np.random.SeedSequence((220907604, 777, l)))
        Y = [theta * y + (rng.standard_normal(len(y)) + 1j * rng.standard_normal(len(y))) / np.sqrt(2.0)
             for y in Y0]
        V = [0.1 * (rng.standard_normal(len(y)) + 1j * rng.standard_normal(len(y))) for y in Y]
        eps = block_radii(prob.n_vis[l])
        del Y0
        if sample:
            q_early.put({"l": l, "theta": theta, "Y": Y, "V": V, "eps": eps, "setup_s": time.time() - t0})
        barrier.wait(timeout=1800)
        t1 = time.perf_counter()
        Vp, grad, rho, res = oracle.dual_step(op, {l: 0.5 * x}, V, Y, eps)
        dt = time.perf_counter() - t1
        out = {"l": l, "M": int(ml), "s": dt}
        if sample:
            out.update(Vp=np.concatenate(Vp), grad=grad[l], rho=rho, res=res)
        q_out.put(out)
    except BaseException as e:  # report, never hang the parent
        q_out.put({"l": l, "error": repr(e)})
        if sample:
            q_early.put({"l": l, "error": repr(e)})
        try:
            barrier.abort()
        except Exception:
            pass


class CpuBaseline:
    """The oracle on `workers` whole channels, one per spawned process
    (started before the GPU is touched).  Channel 0 is the error sample."""

    def __init__(self, config, L, workers):
        ctx = mp.get_context("spawn")
        self.chans = sorted(set(np.linspace(0, L - 1, workers).round().astype(int).tolist()))
        n = len(self.chans)
        hi = host_info()
        omp = max(1, (hi["usable_cpus"] or 1) // n)
        self.barrier = ctx.Barrier(n)
        self.q_early, self.q_out = ctx.Queue(), ctx.Queue()
        self.procs = [ctx.Process(target=_oracle_worker,
                                  args=(config, l, l == self.chans[0], self.barrier, self.q_early, self.q_out, omp),
                                  daemon=True) for l in self.chans]
        for p in self.procs:
            p.start()
        self._sample = None
        self.host = hi

    def sample(self):
        """Channel-0 inputs of the oracle (blocks until they are ready)."""
        if self._sample is None:
            s = self.q_early.get(timeout=1800)
            if "error" in s:
                raise RuntimeError("oracle worker failed: " + s["error"])
            self._sample = s
        return self._sample

    def results(self):
        outs = [self.q_out.get(timeout=1800) for _ in self.procs]
        for p in self.procs:
            p.join(timeout=60)
        bad = [o for o in outs if "error" in o]
        if bad:
            raise RuntimeError("oracle worker failed: %s" % bad[0]["error"])
        return outs


# --------------------------------------------------------------- workload
def generate(name, channels=0, host_windows=False):
    """Problem and per-block (base, S, windows or None, kappa [M, 2], w-table)."""
    import synth
    prob = synth.make_problem(name)
    if channels and channels < prob.L:
        sel = np.linspace(0, prob.L - 1, channels).round().astype(int)
        prob = synth.make_problem(name, L=channels, n_blocks=[prob.n_blocks[l] for l in sel],
                                  n_vis=[prob.n_vis[l] for l in sel],
                                  nu=None if prob.nu is None else prob.nu[sel])
    t0 = time.time()
    blocks = []
    K = np.array([prob.Ky, prob.Kx], dtype=np.float64)
    nb = len(prob.block_list())
    for k, (l, b) in enumerate(prob.block_list()):
        blk = prob.block(l, b)
        w = blk.windows(np.complex64)[0] if host_windows else None
        blocks.append(dict(base=blk.base, S=blk.S, windows=w, kappa=blk.omega * K / (2 * np.pi),
                           h=blk.w_h, a=blk.w_a))
        if k % 8 == 0 or k == nb - 1:
            log("[bench] generated block %d/%d (%.0f s)" % (k + 1, nb, time.time() - t0))
    generate.seconds = time.time() - t0
    return prob, blocks


def stage_alg_bytes(info, L, N, K):
    """Algorithmic HBM bytes per step of every stage (minimal-pass design:
    G read by the gather and again by G^H; v and y read, c written and read,
    v+ written; x read, half grid written and read, grid written and read per
    direction).  The one-pass stage is charged the gather's and the G^H
    pass's bytes except the c read and v+ write, which the v+ scale does."""
    T, M = float(info["n_taps"]), float(info["n_vis_total"])
    G = float(info["g_bytes"])
    out = {"rowfft_fwd": L * (4.0 * N + 4.0 * K), "colfft_fwd": L * 12.0 * K,
           "gather": G + 28.0 * M + L * 8.0 * K, "scatter": G + 20.0 * M,
           "dual_gs": 2.0 * G + 32.0 * M + L * 8.0 * K, "vscale": 16.0 * M, "finalize": 0.0,
           "merge": L * 8.0 * K, "colfft_inv": L * 12.0 * K, "rowfft_inv": L * (4.0 * K + 4.0 * N)}
    if info.get("fft_image_first"):
        # columns of the image first (x in, the Ky x Nx intermediate out: 4 K),
        # then the rows (intermediate in, grid out); the adjoint mirrors it
        out.update(colfft_fwd=L * (4.0 * N + 4.0 * K), rowfft_fwd=L * 12.0 * K,
                   rowfft_inv=L * 12.0 * K, colfft_inv=L * (4.0 * K + 4.0 * N))
    return out


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


def stream_rates(dev, mib=2048):
    """A plain library device copy (read + write bytes / time) and a plain
    library reduction (read bytes / time) of 2 GiB: practical streaming
    rates of this GPU beside the 8 TB/s specification."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
        src.sum()
    torch.cuda.synchronize()
    copy_ms = _event_ms(lambda: dst.copy_(src), 10)
    sum_ms = _event_ms(lambda: src.sum(), 10)
    del src, dst
    return {"copy_GBs": 2.0 * n * 4 / (copy_ms * 1e-3) / 1e9, "read_GBs": n * 4 / (sum_ms * 1e-3) / 1e9}


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
    del xi, xti, v, e, grad, var, state, w, img, yv
    out["pdfb"] = {"ms_per_iter": ms, "primal_ms": prim_ms, "eps_update_ms": stages["eps_update"] / max(calls, 1),
                   "primal_alg_bytes": 16.0 * px,
                   "primal_GBs": 16.0 * px / (prim_ms * 1e-3) / 1e9,
                   "rule": "adaptive l2 bounds (lambda 0.99/1.01/0.618, var_tol 1e-3, min_gap 10)",
                   "steps": "sigma_b = 1/||Phi_l||^2 (10 power steps), tau_l = 0.9"}
    return out


def time_dr(make_plan, blocks, device_g, xt, y_user, head, args, dev):
    """The visibility-gridding reduction (Section 3.4) on a plan created with
    PHI_DR from the same blocks (its own G kept in complex64, the reduced rows
    in the headline precision): device set-up time, then the reduced dual
    step (autotuned, hipGraph) against the unreduced headline step on the same
    data; both forms' row and byte counts, and the form the bytes rule keeps."""
    import torch
    from paper_2209_07604_amd import GRAPH, PERSISTENT, FUSED_GH
    p = make_plan()
    for k, b in enumerate(blocks):
        if device_g:
            p.build_g(k, torch.from_numpy(np.ascontiguousarray(b["kappa"])).to(dev),
                      torch.from_numpy(np.ascontiguousarray(b["h"])).to(dev),
                      torch.from_numpy(np.ascontiguousarray(b["a"])).to(dev), J=7)
        else:
            p.load_g(k, b["windows"])
    y = p.to_plan(y_user)
    info = p.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    yred, m_red = p.dr_setup(y)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    rp = p.reduced()
    rp.autotune(3)
    ri = rp.info()
    rp.set_flags(GRAPH | (PERSISTENT if ri["persist_blocks"] else 0) | (FUSED_GH if ri["fused"] else 0))
    eps = torch.tensor([np.sqrt(m + 2.0 * np.sqrt(m)) for m in m_red], dtype=torch.float64, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    mr = int(m_red.sum())
    v0 = (0.1 * torch.complex(torch.randn(mr, generator=gen, device=dev),
                              torch.randn(mr, generator=gen, device=dev))).contiguous()
    v = v0.clone()
    grad = torch.empty_like(xt)
    rho = torch.empty(p.nblk, dtype=torch.float64, device=dev)
    res = torch.empty_like(rho)
    for _ in range(args.warmup):
        p.dual_step_dr(xt, v, yred, eps, None, grad, rho, res)
    v.copy_(v0)
    torch.cuda.synchronize()
    ms = _event_ms(lambda: p.dual_step_dr(xt, v, yred, eps, None, grad, rho, res), args.steps)
    rp.check()
    rp.set_flags(0 | (PERSISTENT if ri["persist_blocks"] else 0) | (FUSED_GH if ri["fused"] else 0))
    v.copy_(v0)
    torch.cuda.synchronize()
    rp.set_timing(True)
    for _ in range(args.steps):
        p.dual_step_dr(xt, v, yred, eps, None, grad, rho, res)
    torch.cuda.synchronize()
    rp.set_timing(False)
    stages, calls = rp.get_timing()
    M = int(info["n_vis_total"])
    g_bytes_head = int(head["g_bytes"])
    out = {"M": M, "M_reduced": mr, "M_over_M_reduced": M / mr, "taps_G": int(info["n_taps"]),
           "taps_H": int(info["dr_taps"]), "bytes_G": g_bytes_head, "bytes_H": int(info["dr_bytes"]),
           "largest_row_window": int(info["dr_max_window"]), "setup_ms": setup_ms,
           "ms_per_step_reduced": ms, "ms_per_step_unreduced": head["ms_per_step"],
           "visibilities_per_s_reduced": M / (ms * 1e-3), "tile": ri["tile"], "one_pass": bool(ri["fused"]),
           "stage_ms": {k_: v_ / max(calls, 1) for k_, v_ in stages.items() if v_ > 0},
           "kept": "reduced" if info["dr_bytes"] < g_bytes_head else "unreduced",
           "rule": "keep the reduced form only if the rows of Lam H hold fewer bytes than G"}
    out["speedup"] = head["ms_per_step"] / ms
    log("[bench] reduced step: %s" % out)
    del v, v0, grad, yred, y, rp
    p.close()
    torch.cuda.empty_cache()
    return out


def run_sample(p, prob, smp, theta, flags, dev):
    """The oracle's channel-0 inputs through plan p (other channels zero):
    (v+ channel 0 user order, grad channel 0, rho, res of channel 0's blocks)."""
    import torch
    nb0 = prob.n_blocks[0]
    m0 = int(sum(prob.n_vis[0]))
    th = np.array(theta, dtype=np.float64)
    th[:nb0] = smp["theta"]
    p.set_theta(th)
    vh = np.zeros(p.M, np.complex64)
    yh = np.zeros(p.M, np.complex64)
    vh[:m0] = np.concatenate(smp["V"])
    yh[:m0] = np.concatenate(smp["Y"])
    xt = torch.zeros((p.L, prob.Ny, prob.Nx), dtype=torch.float32, device=dev)
    xt[0] = torch.from_numpy((0.5 * prob.image(0)).astype(np.float32))
    v = p.to_plan(torch.from_numpy(vh).to(dev))
    y = p.to_plan(torch.from_numpy(yh).to(dev))
    e_all = np.ones(p.nblk)
    e_all[:nb0] = smp["eps"]
    p.set_flags(flags)
    grad, rho, res = p.dual_step(xt, v, y, torch.from_numpy(e_all).to(dev))
    p.check()
    out = (p.from_plan(v)[:m0].cpu().numpy(), grad[0].cpu().numpy(), rho[:nb0].cpu().numpy(),
           res[:nb0].cpu().numpy())
    p.set_theta(theta)
    del v, y, xt, grad, rho, res
    return out


def rel_err(gpu, ref):
    def rel(a, b):
        a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) else np.float64)
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    vp, g, rho, res = gpu
    return {"v_plus": rel(vp, ref["Vp"]), "grad": rel(g, ref["grad"]), "rho": rel(rho, ref["rho"]),
            "res": rel(res, ref["res"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C5")
    ap.add_argument("--forms", default="plain_c64,batched_c64,batched_bf16,batched_kb,twopass_f16,batched_f16",
                    help="forms to time: <plain|batched|fused|twopass>_<c64|bf16|f16|kb>; kb: taps evaluated "
                         "in the kernels (Kaiser-Bessel windows without w-term only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="channels of the CPU baseline, one process each; 0: every usable core (capped by host "
                         "memory and the channel count)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="fix the tile edge (skips the autotuner)")
    ap.add_argument("--persist", type=int, default=0, help="persistent G-stage grid with --tile")
    ap.add_argument("--channels", type=int, default=0, help="use this many channels of the configuration")
    ap.add_argument("--host-g", action="store_true",
                    help="load G from host windows built by the generator instead of the device builder")
    ap.add_argument("--no-extras", action="store_true", help="skip forward/adjoint/PDFB timings")
    ap.add_argument("--dr", action="store_true",
                    help="also time the visibility-gridding reduced step (Section 3.4) on the headline plan, "
                         "e.g. --config C5t (VLA-like tracks)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, run one plain device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the data-fidelity step shards by channel with no exchange, "
              "and this build runs on a single MI355X; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import synth
    forms = [f for f in args.forms.split(",") if f]
    cfg_prob = synth.make_problem(args.config)
    device_g = not args.host_g and not cfg_prob.dde
    if not device_g and not args.host_g:
        log("[bench] %s has DDE rows: G from host windows" % args.config)
    # the CPU baseline's processes start before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        hi = host_info()
        per_chan_gb = 2.5 * 16.0 * cfg_prob.M_total / cfg_prob.L * 49 / 1e9 + 4.0
        cap_mem = int(max(1.0, ((hi["ram_available_GB"] or 64.0) * 0.6) // per_chan_gb))
        want = args.cpu_workers if args.cpu_workers > 0 else (hi["usable_cpus"] or 1)
        nw = max(1, min(want, cfg_prob.L, hi["usable_cpus"] or 1, cap_mem))
        cpu = CpuBaseline(args.config, cfg_prob.L, nw)
        cpu.limits = {"requested": want, "channels": cfg_prob.L, "usable_cpus": hi["usable_cpus"],
                      "memory": cap_mem, "GB_per_process_estimate": round(per_chan_gb, 1)}
        log("[bench] cpu baseline: %d oracle process(es) on channels %s, host %s" % (nw, cpu.chans, cpu.host))

    import torch
    from paper_2209_07604_amd import Plan, PER_CHANNEL, GRAPH, PERSISTENT, FUSED_GH, DR

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    prob, blocks = generate(args.config, channels=args.channels, host_windows=not device_g)
    L = prob.L
    t0 = time.time()
    n_vis = [len(b["S"]) for b in blocks]
    base = np.concatenate([b["base"] for b in blocks])
    S = np.concatenate([b["S"] for b in blocks])
    s_y, s_x = prob.deapodisation()
    M = int(len(S))
    Kc, Nc = prob.Ky * prob.Kx, prob.Ny * prob.Nx
    if any(f.endswith("_kb") for f in forms) and not (np.all(S == 7) and all(np.all(b["h"] == 0) for b in blocks)):
        log("[bench] %s has w-terms or other than 7 x 7 windows: no Kaiser-Bessel forms" % args.config)
        forms = [f for f in forms if not f.endswith("_kb")]
    precs = []
    for f in forms:
        pr = f.split("_")[1]
        if pr not in precs:
            precs.append(pr)
    head = "batched_f16" if "batched_f16" in forms else forms[-1]
    hprec = head.split("_")[1]
    precs = [q for q in precs if q != hprec] + [hprec]   # the headline plan is built last and kept

    x = torch.from_numpy(np.stack([prob.image(l) for l in range(L)])).to(dev)
    xt = (0.5 * x).contiguous()
    log("[bench] images resident (%.0f s)" % (time.time() - t0))
    gen = torch.Generator(device=dev)
    gen.manual_seed(220907604)
    noise = None
    y_user = theta = None
    v_init = (0.1 * torch.complex(torch.randn(M, generator=gen, device=dev),
                                  torch.randn(M, generator=gen, device=dev))).contiguous()
    # chi-square radii (eq. 2): eps_l^2 = M_l + 2 sqrt(M_l), eps_lb^2 = eps_l^2 M_lb / M_l
    eps_h = []
    for nv in prob.n_vis:
        ml = float(sum(nv))
        eps_h += [np.sqrt((ml + 2.0 * np.sqrt(ml)) * m / ml) for m in nv]
    eps = torch.tensor(eps_h, dtype=torch.float64, device=dev)
    nblk = len(n_vis)
    ch_of_blk = np.repeat(np.arange(L), prob.n_blocks)
    starts = np.concatenate([[0], np.cumsum(n_vis)])

    results, samples, gb_build = {}, {}, {}
    hp = None
    for prec in precs:
        tp = time.time()
        p = Plan(prob.Ny, prob.Nx, prob.n_blocks, n_vis, base, S, s_y, s_x, None, g_prec=prec, device=dev)
        tile0 = p.info()["tile"]
        log("[bench] plan %s created (%.1f s), workspace %.1f GB" % (prec, time.time() - tp, p.workspace_size() / 1e9))
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for k, b in enumerate(blocks):
            if prec == "kb":   # no stored G: the kernels evaluate the taps from kappa
                p.load_kb(k, b["kappa"])
            elif device_g:   # rows computed on the device from the generator's tables
                p.build_g(k, torch.from_numpy(np.ascontiguousarray(b["kappa"])).to(dev),
                          torch.from_numpy(np.ascontiguousarray(b["h"])).to(dev),
                          torch.from_numpy(np.ascontiguousarray(b["a"])).to(dev), J=7)
            else:
                p.load_g(k, b["windows"])
        torch.cuda.synchronize()
        gb_build[prec] = time.perf_counter() - tb
        info0 = p.info()
        log("[bench] plan %s G ready (%.1f s), info %s" % (prec, gb_build[prec], info0))
        if y_user is None:
            # y = theta Phi0 x + n at 30 dB per channel (theta from this plan's noiseless forward)
            y0 = p.from_plan(p.forward(x))
            pw = np.zeros(L)
            y0h = y0.abs().square().double()
            for k in range(nblk):
                pw[ch_of_blk[k]] += y0h[starts[k]:starts[k + 1]].sum().item()
            del y0h
            m_ch = np.array([sum(m) for m in prob.n_vis], dtype=np.float64)
            theta = (1.0 / np.sqrt(pw / m_ch * 1e-3))[ch_of_blk]
            noise = torch.complex(torch.randn(M, generator=gen, device=dev), torch.randn(M, generator=gen, device=dev))
            th_vis = torch.from_numpy(np.repeat(theta, n_vis).astype(np.float32)).to(dev)
            y_user = (th_vis * y0 + noise * (0.5 ** 0.5)).contiguous()
            del y0, noise, th_vis
        p.set_theta(theta)
        y = p.to_plan(y_user)
        order = ["plain", "batched", "fused", "twopass"]
        for form in sorted([f for f in forms if f.split("_")[1] == prec], key=lambda f: order.index(f.split("_")[0])):
            kind = form.split("_")[0]
            v = p.to_plan(v_init)
            v0 = v.clone()
            grad = torch.empty((L, prob.Ny, prob.Nx), dtype=torch.float32, device=dev)
            rho = torch.empty(nblk, dtype=torch.float64, device=dev)
            res = torch.empty(nblk, dtype=torch.float64, device=dev)
            if kind in ("batched", "fused", "twopass") and args.tile:
                p.set_tuning(args.tile, args.persist)
            elif kind in ("batched", "fused") and not args.no_autotune:
                ta = time.time()
                p.autotune(3)
                log("[bench] autotune %s (%.1f s) -> tile %d, persist %d, one pass %d" % (
                    prec, time.time() - ta, p.info()["tile"], p.info()["persist_blocks"], p.info()["fused"]))
            # batched_<prec> keeps the autotuner's choice of one pass or two;
            # fused_<prec> forces one pass; plain_ and twopass_ use two passes
            # (twopass_ on the batched form's tuning)
            fused = kind == "fused" or (kind == "batched" and bool(p.info()["fused"]))
            flags_now = (PERSISTENT if (kind != "plain" and p.info()["persist_blocks"]) else 0) | \
                (FUSED_GH if fused else 0)
            if kind == "plain":
                p.set_tuning(tile0, 0)
            graph_flags = (PER_CHANNEL if kind == "plain" else GRAPH) | flags_now
            p.set_flags(graph_flags)
            log("[bench] %s: warm-up" % form)
            for _ in range(args.warmup):
                v.copy_(v0)
                p.dual_step(xt, v, y, eps, None, grad, rho, res)
            v.copy_(v0)
            torch.cuda.synchronize()
            log("[bench] %s: timing %d steps" % (form, args.steps))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t_wall = time.perf_counter()
            e0.record()
            for _ in range(args.steps):
                p.dual_step(xt, v, y, eps, None, grad, rho, res)
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
                p.dual_step(xt, v, y, eps, None, grad, rho, res)
            torch.cuda.synchronize()
            p.set_timing(False)
            stages, calls = p.get_timing()
            info = p.info()
            st_ms = {k_: v_ / max(calls, 1) for k_, v_ in stages.items() if v_ > 0}
            alg = stage_alg_bytes(info, L, Nc, Kc)
            b_step = sum(alg[k_] for k_ in st_ms if k_ in alg and not (fused and k_ in ("gather", "scatter")))
            results[form] = dict(ms_per_step=ms, tile=info["tile"], persist_blocks=info["persist_blocks"],
                                 one_pass=bool(fused), wall_ms_per_step=1e3 * wall / args.steps,
                                 vis_per_s=M / (ms * 1e-3), stage_ms=st_ms,
                                 alg_bytes_step=b_step, alg_GBs=b_step / (ms * 1e-3) / 1e9,
                                 hbm_frac=b_step / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 g_bytes=int(info["g_bytes"]), partial_bytes=int(info["partial_bytes"]),
                                 pitch_classes=int(info["pitch_classes"]), info=info, graph_flags=graph_flags)
            log("[bench] %s: %.3f ms/step, %.3g vis/s, stages %s" % (
                form, ms, M / (ms * 1e-3), {k_: round(v_, 3) for k_, v_ in st_ms.items()}))
            del v, v0, grad, rho, res
            if cpu is not None:
                smp = cpu.sample()
                samples[form] = run_sample(p, prob, smp, theta, graph_flags, dev)
                log("[bench] %s: channel-0 oracle sample run" % form)
        if prec == hprec:
            hp = p
            hp_y = y
        else:
            del y, p
            torch.cuda.empty_cache()

    r = results[head]
    info = r["info"]
    hflags = r["graph_flags"]
    hp.set_flags(hflags)
    line_dr = None
    if args.dr:
        mk = lambda: Plan(prob.Ny, prob.Nx, prob.n_blocks, n_vis, base, S, s_y, s_x, theta, g_prec=hprec,
                          device=dev, flags=DR)
        line_dr = time_dr(mk, blocks, device_g, xt, y_user, r, args, dev)
    line_extra = {}
    if not args.no_extras:
        log("[bench] %s: forward, adjoint and PDFB iterations" % head)
        extras = time_extras(hp, x, xt, hp.to_plan(v_init), hp_y, eps, args.steps, args.warmup, dev)
        line_extra = {"forward_ms": extras["forward_ms"], "adjoint_ms": extras["adjoint_ms"],
                      "pdfb": dict(extras["pdfb"], primal_frac=extras["pdfb"]["primal_GBs"] / HBM_PEAK_GBS)}
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy of %d MiB done" % args.calib_copy_mib)
        del src, dst
    # (not in counter runs: their only large copy must be the calibration copy)
    rates = None if args.calib_copy_mib else stream_rates(dev)
    log("[bench] streaming rates %s" % rates)

    alg = stage_alg_bytes(info, L, Nc, Kc)
    workload = args.config if not args.channels else "%s_%dch" % (args.config, L)
    stages_tab = {}
    for k_, t_ in r["stage_ms"].items():
        if k_ not in alg or t_ <= 0:
            continue
        a_ = alg[k_]
        tr = traffic_for(workload, k_)
        stages_tab[k_] = {"ms": t_, "alg_bytes": a_, "alg_GBs": a_ / (t_ * 1e-3) / 1e9,
                          "frac": a_ / (t_ * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "traffic": tr, "frac_physical": None if tr is None else tr / (t_ * 1e-3) / 1e9 / HBM_PEAK_GBS}
    dom = max(stages_tab, key=lambda k_: stages_tab[k_]["ms"])
    d = stages_tab[dom]
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
                               "windows %d..%d, 30 dB" % (workload, L, sorted(set(prob.n_blocks)),
                                                          prob.Ny, prob.Nx, prob.Ky, prob.Kx, M,
                                                          int(S.min()), int(S.max())),
                   "g_source": "device builder" if device_g else "host windows",
                   "form": head.replace("_", " ") + " (hipGraph)" + (", one pass over G" if r["one_pass"] else ""),
                   "g_storage": hprec, "taps": int(info["n_taps"])},
        "hbm_alg_GBs": r["alg_GBs"],
        "step_alg_bytes": r["alg_bytes_step"],
        "step_frac": r["hbm_frac"],
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": d["alg_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": d["frac"], "traffic": d["traffic"],
                     "frac_physical": d["frac_physical"], "alg_bytes_per_launch": d["alg_bytes"],
                     "avg_launch_ms": d["ms"],
                     # the one-pass stage is one launch per pitch class; its bytes and
                     # time are per step (the sum over those launches)
                     "launches_per_step": info["pitch_classes"] if dom == "dual_gs" else 1,
                     "stream_copy_GBs": rates and rates["copy_GBs"], "stream_read_GBs": rates and rates["read_GBs"]},
        "stages": stages_tab,
        "forms": {k: {kk: vv for kk, vv in v.items() if kk not in ("info", "graph_flags")}
                  for k, v in results.items()},
        "g_builder_s": gb_build if device_g else None,
    }
    line.update(line_extra)
    if line_dr:
        line["dimensionality_reduction"] = line_dr
    if "plain_c64" in results:
        line["speedup_vs_plain_fp32"] = results["plain_c64"]["ms_per_step"] / r["ms_per_step"]
    if cpu is not None:
        outs = cpu.results()
        ref = [o for o in outs if o["l"] == cpu.chans[0]][0]
        mtot = sum(o["M"] for o in outs)
        tmax = max(o["s"] for o in outs)
        line["cpu_baseline"] = {
            "value": mtot / tmax, "unit": "visibilities/s", "cores": len(outs), "kind": "oracle",
            "sample": "%d whole channel(s) %s of the same workload (%d visibilities each, %dx%d grid), one FP64 "
                      "oracle dual step per channel, each in its own process (numpy.fft and scipy.sparse, "
                      "single-threaded per process), started together; slowest %.1f s" % (
                          len(outs), cpu.chans, outs[0]["M"], prob.Ky, prob.Kx, tmax),
            "host": cpu.host,
            # processes = min of these (each holds one channel's FP64 operator;
            # "memory": how many fit in 60% of the available RAM)
            "worker_limits": cpu.limits}
        line["err_vs_fp64"] = {f: rel_err(g, ref) for f, g in samples.items()}
        line["err_vs_fp64"]["sample"] = "channel 0 (all its blocks): the oracle's inputs (x~ = x/2, v ~ 0.1 CN, " \
                                        "y at 30 dB) through each form's plan and launch flags"
        line["vs_cpu_baseline"] = r["vis_per_s"] / line["cpu_baseline"]["value"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
