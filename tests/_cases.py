"""Shared set-up for the GPU parity tests: one synthetic problem, its FP64
oracle data (y at 30 dB input SNR, radii, a dual-step state) and a libphi
plan loaded with the same G windows.  The oracle side never sees a value the
HIP path produced.
"""
import numpy as np

import oracle
import synth


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def quantise(w, prec):
    """The G storage rounding, written with NumPy (RNE per real part)."""
    if prec == "c64":
        return (w.real.astype(np.float32).astype(np.float64)
                + 1j * w.imag.astype(np.float32).astype(np.float64))
    if prec == "f16":
        return w.real.astype(np.float16).astype(np.float64) + 1j * w.imag.astype(np.float16).astype(np.float64)
    if prec == "bf16":
        def bf(x):
            m, e = np.frexp(x)                   # x = m 2^e, |m| in [0.5, 1)
            q = np.maximum(e - 8, -133)
            return np.rint(np.ldexp(x, -q)) * np.ldexp(1.0, q)   # ties to even
        return bf(w.real) + 1j * bf(w.imag)
    raise ValueError(prec)


class Case:
    """Problem + oracle state.  `quant` quantises the oracle's G like the plan."""

    def __init__(self, name, seed=0, oracle_prec=None, problem=None):
        self.prob = prob = problem if problem is not None else synth.make_problem(name)
        self.blocks = prob.block_list()
        self.data = [prob.block(l, b) for (l, b) in self.blocks]
        self.wins = [blk.windows(np.complex128) for blk in self.data]
        self.s_y, self.s_x = prob.deapodisation()
        self.X = {l: prob.image(l) for l in range(prob.L)}
        rng = np.random.default_rng(np.random.SeedSequence((220907604, 77, seed)))
        X64 = {l: x.astype(np.float64) for l, x in self.X.items()}
        # 30 dB input SNR per channel: sigma_l^2 = ||Phi0_l x_l||^2 / M_l * 1e-3
        op1 = self.operator(None, prec=None)
        y0 = op1.forward(X64)
        pw = {}
        for (l, b), y in zip(self.blocks, y0):
            s = pw.setdefault(l, [0.0, 0])
            s[0] += float(np.vdot(y, y).real)
            s[1] += len(y)
        theta_l = {l: 1.0 / np.sqrt(max(p / max(n, 1), 1e-300) * 1e-3) for l, (p, n) in pw.items()}
        self.theta = np.array([theta_l[l] for (l, b) in self.blocks])
        self.op = self.operator(self.theta, prec=oracle_prec)
        self.op_exact = self.operator(self.theta, prec=None) if oracle_prec else self.op
        self.Y = []
        for k, y in enumerate(y0):
            n = (rng.standard_normal(len(y)) + 1j * rng.standard_normal(len(y))) / np.sqrt(2)
            self.Y.append(self.theta[k] * y + n)
        self.eps = np.concatenate([oracle.block_radii(nv) for nv in prob.n_vis])
        # dual-step state: x~ = x/2, v ~ 0.1 CN(0, 1)  (rho > eps with cancellation)
        self.Xt = {l: (0.5 * x).astype(np.float32) for l, x in self.X.items()}
        self.V = [0.1 * (rng.standard_normal(len(y)) + 1j * rng.standard_normal(len(y))) for y in self.Y]
        self.rng = rng

    def operator(self, theta, prec):
        ops = []
        for k, ((l, b), blk, (w, off)) in enumerate(zip(self.blocks, self.data, self.wins)):
            wq = w if prec is None else quantise(w, prec)
            th = 1.0 if theta is None else float(theta[k])
            ops.append(oracle.BlockG(l, th, oracle.g_matrix(blk.base, blk.S, wq, off,
                                                            self.prob.Ky, self.prob.Kx, th)))
        return oracle.Operator(self.prob.Ny, self.prob.Nx, self.s_y, self.s_x, ops)

    # ---- flat (user order) views
    def flat(self, parts):
        return np.concatenate(parts) if parts else np.zeros(0, complex)

    def split(self, flat):
        out, o = [], 0
        for blk in self.data:
            out.append(flat[o:o + blk.M])
            o += blk.M
        return out

    def cube(self, X):
        return np.stack([X[l] for l in range(self.prob.L)]).astype(np.float32)

    def plan(self, g_prec="c64", flags=0, tile=0, persist_blocks=0, device="cuda:0"):
        from paper_2209_07604_amd import Plan
        prob = self.prob
        base = np.concatenate([blk.base for blk in self.data]) if self.data else np.zeros((0, 2), np.int32)
        S = np.concatenate([blk.S for blk in self.data]) if self.data else np.zeros(0, np.uint8)
        n_vis = [blk.M for blk in self.data]
        p = Plan(prob.Ny, prob.Nx, prob.n_blocks, n_vis, base, S, self.s_y, self.s_x, self.theta,
                 g_prec=g_prec, flags=flags, tile=tile, persist_blocks=persist_blocks, device=device)
        if g_prec == "kb":
            # direction-independent rows: the kernels evaluate the Kaiser-Bessel
            # taps from the continuous grid coordinates
            for k, blk in enumerate(self.data):
                p.load_kb(k, self.kappa(blk))
        else:
            for k, (w, off) in enumerate(self.wins):
                p.load_g(k, w)
        return p

    def kappa(self, blk):
        """Continuous grid coordinates omega K / (2 pi) of a block, [M, 2]."""
        K = np.array([self.prob.Ky, self.prob.Kx], dtype=np.float64)
        return blk.omega * K / (2 * np.pi)
