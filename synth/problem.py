"""Synthetic wideband RI problems shaped like the paper's VLA workloads.

A ``Problem`` describes sizes; ``Problem.block(l, b)`` regenerates one data
block (uv points, w, window sizes, window bases and the windows of G) and
``Problem.image(l)`` one channel of the sky cube, each from its own
``SeedSequence((220907604, cfg_id, l, b))``.  Nothing here applies Phi.

Recipes (stand-ins for the VLA Cyg A data of Section 5, which is not used):
  * sky: 20 point sources (uniform in the central 80 %, fluxes log-uniform in
    [1e-3, 1]) plus one extended blob (white noise smoothed by a Gaussian of
    sigma = 8 px, clipped at 0, inside an ellipse); channel l is
    x_ref * (nu_l / nu_0)^(-alpha(p)) with a smooth spectral-index map
    alpha in [0.5, 1] (power-law spectra, as in the spectral analysis of Section 6.2).
  * uv: omega ~ N(0, (pi/4)^2 I) rejection-sampled into [-pi, pi)^2 (radially
    concentrated); for wideband configurations one reference draw is scaled by
    nu_l / nu_max per channel.  Blocks split a channel by |omega| quantiles
    (inner/outer, as the A/C configuration blocks of Section 6.1).
  * w-projection: w ~ U[0, w_max]; the per-axis w-kernel half-width is
    a = 5 w / w_max cells, S_w = 1 + 2 round(a); the window is the
    7-tap Kaiser-Bessel vector convolved with the S_w-tap kernel per axis
    (paraxial chirp, separable), S = 6 + S_w.
  * DDE: 27 antennas with 1x1 or 3x3 Fourier kernels (random smooth phase
    screens), the pair kernel d_i * conj(flip(d_j)) is convolved in 2-D,
    widening S by 0, 2 or 4; S is capped at 21.
"""
from dataclasses import dataclass, field

import numpy as np
from scipy.ndimage import fourier_gaussian, gaussian_filter

from .kb import KB_J, kb_beta, kb_psi, deapodisation, window_base
from .windows import windows_c, windows_numpy, SD_MAX

ROOT_SEED = 220907604


def _smooth(a, sigma):
    """Periodic Gaussian smoothing (standard deviation sigma pixels) through
    the FFT: seconds at 4096^2, where a direct 8-sigma-wide filter is not."""
    Ny, Nx = a.shape
    return np.fft.irfft2(fourier_gaussian(np.fft.rfft2(a), sigma, n=Nx), s=(Ny, Nx))


@dataclass
class Block:
    l: int
    b: int
    Ky: int
    Kx: int
    omega: np.ndarray          # [M, 2] float64 (omega_y, omega_x) rad/pixel
    w: np.ndarray              # [M] float64 w (units of w_max)
    S: np.ndarray              # [M] int32 window size (odd)
    base: np.ndarray           # [M, 2] int32 first window row/column, in [0, K)
    _skw: np.ndarray = field(repr=False, default=None)
    _uy: np.ndarray = field(repr=False, default=None)
    _ux: np.ndarray = field(repr=False, default=None)
    _taps: object = field(repr=False, default=None)   # builds (_uy, _ux) on first use
    w_h: np.ndarray = field(repr=False, default=None)    # [M] w-kernel half-width h (cells)
    w_a: np.ndarray = field(repr=False, default=None)    # [M] w-chirp parameter (cells)
    _pair_id: np.ndarray = field(repr=False, default=None)
    _pairs: np.ndarray = field(repr=False, default=None)
    _pair_sd: np.ndarray = field(repr=False, default=None)

    @property
    def M(self):
        return len(self.S)

    def windows(self, dtype=np.complex128, engine="c"):
        """(flat windows, offsets[M+1]); window m is S[m] x S[m] row-major,
        entry (i, j) multiplies grid cell ((base_y+i) mod Ky, (base_x+j) mod Kx)."""
        if self._uy is None and self._taps is not None:
            self._uy, self._ux = self._taps()
        if engine == "numpy":
            w, off, S = windows_numpy(self._skw, self._uy, self._ux, self._pair_id,
                                      self._pairs, self._pair_sd)
            w = w.astype(dtype)
        else:
            w, off, S = windows_c(self._skw, self._uy, self._ux, self._pair_id,
                                  self._pairs, self._pair_sd, dtype=dtype)
        assert np.array_equal(S, self.S)
        return w, off


@dataclass
class Problem:
    name: str
    cfg_id: int
    Ny: int
    Nx: int
    L: int
    n_blocks: list
    n_vis: list                # list (per channel) of lists (per block)
    w_max_cells: float = 0.0   # max w-kernel half-width a (0 = no w-term)
    dde: bool = False
    s_cap: int = 21
    nu: np.ndarray = None      # channel frequencies (GHz)
    coverage: str = "gauss"
    n_sources: int = 20
    blob: bool = True
    blocks_by: str = "radius"  # "radius" quantiles or "uneven" random splits
    shared_uv: bool = True     # wideband: one uv draw scaled by nu_l / nu_max

    @property
    def Ky(self):
        return 2 * self.Ny

    @property
    def Kx(self):
        return 2 * self.Nx

    @property
    def M_total(self):
        return int(sum(sum(m) for m in self.n_vis))

    def block_list(self):
        return [(l, b) for l in range(self.L) for b in range(self.n_blocks[l])]

    def deapodisation(self):
        """(s_y[Ny], s_x[Nx]) FP64 scale vectors of Z."""
        return deapodisation(self.Ny, self.Ky), deapodisation(self.Nx, self.Kx)

    def rng(self, *key):
        return np.random.default_rng(np.random.SeedSequence((ROOT_SEED, self.cfg_id) + tuple(key)))

    # ------------------------------------------------------------------ sky
    def _ref_image(self):
        cache = self.__dict__.setdefault("_sky_cache", {})
        if "ref" not in cache:
            cache["ref"] = self._ref_image_draw()
        return cache["ref"]

    def _alpha(self):
        """Spectral-index map in [0.5, 1] (smooth, seeded)."""
        cache = self.__dict__.setdefault("_sky_cache", {})
        if "alpha" not in cache:
            rng = self.rng(10_001)
            a = _smooth(rng.standard_normal((self.Ny, self.Nx)), max(2.0, self.Ny / 16))
            a = (a - a.min()) / max(a.max() - a.min(), 1e-30)
            cache["alpha"] = 0.5 + 0.5 * a
        return cache["alpha"]

    def _ref_image_draw(self):
        rng = self.rng(10_000)
        Ny, Nx = self.Ny, self.Nx
        x = np.zeros((Ny, Nx))
        py = rng.integers(int(0.1 * Ny), int(0.9 * Ny), self.n_sources)
        px = rng.integers(int(0.1 * Nx), int(0.9 * Nx), self.n_sources)
        flux = 10.0 ** rng.uniform(-3.0, 0.0, self.n_sources)
        np.add.at(x, (py, px), flux)
        if self.blob:
            sig = max(1.0, 8.0 * min(Ny, Nx) / 256.0)
            noise = _smooth(rng.standard_normal((Ny, Nx)), sig)
            noise = np.clip(noise, 0.0, None)
            yy, xx = np.meshgrid(np.arange(Ny) - Ny / 2, np.arange(Nx) - Nx / 2, indexing="ij")
            ay, ax = 0.3 * Ny, 0.2 * Nx
            th = 0.5
            u = (yy * np.cos(th) + xx * np.sin(th)) / ay
            v = (-yy * np.sin(th) + xx * np.cos(th)) / ax
            mask = (u * u + v * v) <= 1.0
            if noise.max() > 0:
                noise = noise / noise.max() * 0.05
            x += noise * mask
        return x

    def image(self, l):
        """Channel l of the sky cube, float32 [Ny, Nx], nonnegative."""
        x = self._ref_image()
        if self.L > 1:
            x = x * (self.nu[l] / self.nu[0]) ** (-self._alpha())
        return x.astype(np.float32)

    # ------------------------------------------------------------------ uv
    def _gauss_omega(self, rng, M):
        out = np.empty((0, 2))
        sd = np.pi / 4
        while len(out) < M:
            d = rng.normal(0.0, sd, size=(int((M - len(out)) * 1.05) + 16, 2))
            ok = np.all((d >= -np.pi) & (d < np.pi), axis=1)
            out = np.concatenate([out, d[ok]])
        return out[:M]

    def _track_omega(self, M):
        """Earth-rotation tracks of a 27-antenna Y array (VLA-like): 351
        baselines sampled over hour angles [-4 h, 4 h] at declination
        +40.7 deg (the Cyg A phase centre of Section 5.1), scaled so the
        longest projected baseline reaches |omega| = 0.9 pi."""
        rng = self.rng(20_003)
        lat, dec = np.deg2rad(34.08), np.deg2rad(40.73)
        arms = np.deg2rad([5.0, 125.0, 245.0]) + rng.uniform(-0.02, 0.02, 3)
        d = (np.arange(1, 10) / 9.0) ** 1.716
        ant_e = np.concatenate([d * np.sin(a) for a in arms])
        ant_n = np.concatenate([d * np.cos(a) for a in arms])
        i, j = np.triu_indices(27, 1)
        E, N = ant_e[j] - ant_e[i], ant_n[j] - ant_n[i]
        Lx, Ly, Lz = -np.sin(lat) * N, E, np.cos(lat) * N
        nt = -(-M // len(E))
        H = np.linspace(-np.pi / 3, np.pi / 3, nt)
        sH, cH = np.sin(H)[None, :], np.cos(H)[None, :]
        u = sH * Lx[:, None] + cH * Ly[:, None]
        v = -np.sin(dec) * cH * Lx[:, None] + np.sin(dec) * sH * Ly[:, None] + np.cos(dec) * Lz[:, None]
        r = np.hypot(u, v).max()
        om = np.stack([v.ravel(), u.ravel()], axis=1) * (0.9 * np.pi / r)
        return om[:M]

    def _channel_uv(self, l):
        """All uv points and w of channel l, grouped into blocks (list of index arrays)."""
        cache = self.__dict__.setdefault("_uv_cache", {})
        if l not in cache:
            cache.clear()
            cache[l] = self._channel_uv_draw(l)
        return cache[l]

    def _ref_uv(self):
        """The reference (omega, w) draw that wideband channels scale."""
        cache = self.__dict__.setdefault("_ref_uv_cache", {})
        if "ref" not in cache:
            rng = self.rng(20_000)
            Mref = max(int(sum(m)) for m in self.n_vis)
            if self.coverage == "tracks":
                om = self._track_omega(Mref)
            else:
                om = self._gauss_omega(rng, Mref)
            cache["ref"] = (om, rng.uniform(0.0, 1.0, Mref))
        return cache["ref"]

    def _channel_uv_draw(self, l):
        Ml = int(sum(self.n_vis[l]))
        if self.coverage == "tracks" or self.shared_uv:
            om_ref, w_ref = self._ref_uv()
            scale = self.nu[l] / self.nu.max() if self.nu is not None else 1.0
            om = om_ref[:Ml] * scale
            w = w_ref[:Ml] * scale
            # blocks split by |omega| quantiles of the reference draw (the
            # channel's draw is that draw scaled by one positive factor)
            cache = self.__dict__.setdefault("_ref_uv_cache", {})
            if ("order", Ml) not in cache:
                cache[("order", Ml)] = np.argsort(np.hypot(om_ref[:Ml, 0], om_ref[:Ml, 1]), kind="stable")
            order = cache[("order", Ml)]
        else:
            rng = self.rng(20_001, l)
            om = self._gauss_omega(rng, Ml)
            w = rng.uniform(0.0, 1.0, Ml)
            order = np.argsort(np.hypot(om[:, 0], om[:, 1]), kind="stable")
        bounds = np.concatenate([[0], np.cumsum(self.n_vis[l])])
        groups = []
        rng2 = self.rng(20_002, l)
        for b in range(self.n_blocks[l]):
            idx = order[bounds[b]:bounds[b + 1]]
            groups.append(rng2.permutation(idx))   # user order is arbitrary
        return om, w, groups

    # ------------------------------------------------------------------ G
    def _wkernel(self, a):
        """Separable w-kernel taps (per axis) for half-width a (cells)."""
        h = int(np.round(a))
        if h == 0:
            return np.ones(1, dtype=np.complex128)
        k = np.arange(-h, h + 1, dtype=np.float64)
        taper = np.cos(np.pi * k / (2.0 * (h + 1))) ** 2
        c = taper * np.exp(-1j * np.pi * k * k / (4.0 * max(a, 0.5)))
        return c / c.sum()

    def _wkernel_batch(self, a, h):
        """Vectorised _wkernel for many half-widths a sharing round(a) == h."""
        k = np.arange(-h, h + 1, dtype=np.float64)
        taper = np.cos(np.pi * k / (2.0 * (h + 1))) ** 2
        c = taper[None, :] * np.exp(-1j * np.pi * k[None, :] ** 2
                                    / (4.0 * np.maximum(a, 0.5))[:, None])
        return c / c.sum(axis=1, keepdims=True)

    def _dde_tables(self, l):
        rng = self.rng(30_000, l)
        n_ant = 27
        size = rng.choice([1, 3], n_ant)
        ants = []
        for s in size:
            if s == 1:
                ants.append(np.exp(1j * rng.uniform(-np.pi, np.pi)) * np.ones((1, 1)))
            else:
                d = 0.12 * (rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3)))
                d = gaussian_filter(d.real, 0.7) + 1j * gaussian_filter(d.imag, 0.7)
                d[1, 1] += np.exp(1j * rng.uniform(-np.pi, np.pi))
                ants.append(d)
        from scipy.signal import convolve2d
        pairs = []
        for i in range(n_ant):
            for j in range(i + 1, n_ant):
                pairs.append(convolve2d(ants[i], np.conj(ants[j][::-1, ::-1]), mode="full"))
        pair_sd = np.array([p.shape[0] for p in pairs], dtype=np.int32)
        tab = np.zeros((len(pairs), SD_MAX, SD_MAX), dtype=np.complex128)
        for k, p in enumerate(pairs):
            tab[k, :p.shape[0], :p.shape[1]] = p
        return tab, pair_sd

    def block(self, l, b):
        om_all, w_all, groups = self._channel_uv(l)
        idx = groups[b]
        om = om_all[idx]
        w = w_all[idx]
        Ky, Kx = self.Ky, self.Kx
        beta = kb_beta(KB_J)
        kap_y = om[:, 0] * Ky / (2 * np.pi)
        kap_x = om[:, 1] * Kx / (2 * np.pi)
        M = len(idx)
        a = self.w_max_cells * w
        h = np.round(a).astype(np.int64)
        if self.dde:
            tab, pair_sd = self._dde_tables(l)
            rng = self.rng(30_001, l, b)
            pair_id = rng.integers(0, len(pair_sd), M).astype(np.int32)
            sd = pair_sd[pair_id]
        else:
            tab = pair_sd = pair_id = None
            sd = np.ones(M, dtype=np.int32)
        # cap S: shrink the w half-width where needed
        hmax = np.maximum((self.s_cap - (KB_J - 1) - sd) // 2, 0)
        h = np.minimum(h, hmax)
        skw = (KB_J + 2 * h).astype(np.int32)
        S = (skw + sd - 1).astype(np.int32)
        by_kb = window_base(kap_y, KB_J)
        bx_kb = window_base(kap_x, KB_J)
        a_eff = np.where(np.round(a) > h, h.astype(np.float64), a)

        def taps():
            # per-axis tap vectors: the Kaiser-Bessel taps convolved with the
            # w-kernel (built only when the windows themselves are asked for)
            ldu = int(skw.max()) if M else 1
            uy = np.zeros((M, ldu), dtype=np.complex128)
            ux = np.zeros((M, ldu), dtype=np.complex128)
            t = np.arange(KB_J)
            psi_y = kb_psi(kap_y[:, None] - (by_kb[:, None] + t), KB_J, beta)
            psi_x = kb_psi(kap_x[:, None] - (bx_kb[:, None] + t), KB_J, beta)
            for hv in np.unique(h):
                sel = np.nonzero(h == hv)[0]
                if hv == 0:
                    uy[sel, :KB_J] = psi_y[sel]
                    ux[sel, :KB_J] = psi_x[sel]
                    continue
                wk = self._wkernel_batch(a_eff[sel], int(hv))      # [Mg, 2hv+1]
                for k in range(2 * int(hv) + 1):
                    uy[sel, k:k + KB_J] += psi_y[sel] * wk[:, k:k + 1]
                    ux[sel, k:k + KB_J] += psi_x[sel] * wk[:, k:k + 1]
            return uy, ux

        # window bases: w-kernel widens by h, DDE kernel by (sd-1)/2 on each side
        ext = h + (sd - 1) // 2
        by = by_kb - ext
        bx = bx_kb - ext
        base = np.stack([np.mod(by, Ky), np.mod(bx, Kx)], axis=1).astype(np.int32)
        blk = Block(l=l, b=b, Ky=Ky, Kx=Kx, omega=om, w=w, S=S, base=base,
                    _skw=skw, _taps=taps, w_h=h.astype(np.int32), w_a=a_eff, _pair_id=pair_id, _pairs=tab, _pair_sd=pair_sd)
        return blk


def _problem(name, **kw):
    return Problem(name=name, **kw)


def _wide(L, lo, hi):
    return np.linspace(lo, hi, L)


def make_problem(name, **over):
    """Build a named configuration (see CONFIGS), optionally overriding fields."""
    if name not in CONFIGS:
        raise KeyError(name)
    kw = dict(CONFIGS[name]())
    kw.update(over)
    return Problem(name=name, **kw)


def _c3_layout(L, scale=1.0, seed_id=3):
    rng = np.random.default_rng(np.random.SeedSequence((ROOT_SEED, seed_id, 99_999)))
    Ml = np.exp(rng.uniform(np.log(2e5 * scale), np.log(4e6 * scale), L)).astype(np.int64)
    B = rng.integers(1, 9, L)
    n_vis = []
    for l in range(L):
        p = rng.dirichlet(np.full(B[l], 2.0))
        sizes = np.maximum(1, np.floor(p * Ml[l]).astype(np.int64))
        sizes[-1] += Ml[l] - sizes.sum()
        if sizes[-1] < 1:
            sizes[-1] = 1
        n_vis.append([int(s) for s in sizes])
    return [int(b) for b in B], n_vis


def _cfg_c3():
    B, n_vis = _c3_layout(64)
    return dict(cfg_id=3, Ny=2048, Nx=2048, L=64, n_blocks=B, n_vis=n_vis,
                w_max_cells=5.0, dde=True, s_cap=21, nu=_wide(64, 1.0, 2.0),
                shared_uv=False)


def _cfg_c3s():
    B, n_vis = _c3_layout(6, scale=0.01, seed_id=103)
    return dict(cfg_id=103, Ny=256, Nx=256, L=6, n_blocks=B, n_vis=n_vis,
                w_max_cells=5.0, dde=True, s_cap=21, nu=_wide(6, 1.0, 2.0),
                shared_uv=False)


CONFIGS = {
    # one channel, one block, 7x7 KB, no w (the paper's plain NUFFT)
    "C1": lambda: dict(cfg_id=1, Ny=256, Nx=256, L=1, n_blocks=[1], n_vis=[[100_000]]),
    # 16 channels x 4 blocks, 1024^2, 1.5M vis/channel, w-stencils 7..17
    "C2": lambda: dict(cfg_id=2, Ny=1024, Nx=1024, L=16, n_blocks=[4] * 16,
                       n_vis=[[375_000] * 4] * 16, w_max_cells=5.0, s_cap=17,
                       nu=_wide(16, 1.0, 2.0)),
    # 64 channels, 1-8 uneven blocks, 0.2-4M vis/channel, w + DDE, S <= 21
    "C3": _cfg_c3,
    # Exp 1 image size, 32 channels x 2 blocks, 3M vis/channel, S <= 17
    "C4": lambda: dict(cfg_id=4, Ny=1536, Nx=2560, L=32, n_blocks=[2] * 32,
                       n_vis=[[1_500_000] * 2] * 32, w_max_cells=5.0, s_cap=17,
                       nu=_wide(32, 3.979, 8.019)),
    # DR configuration: 4096^2 x 16 channels, 8M vis/channel, 7x7 only
    "C5": lambda: dict(cfg_id=5, Ny=4096, Nx=4096, L=16, n_blocks=[1] * 16,
                       n_vis=[[8_000_000]] * 16, nu=_wide(16, 3.979, 8.019)),
    # ---- reduced-size cases for tests (same recipes, seconds on the oracle)
    "tiny": lambda: dict(cfg_id=100, Ny=32, Nx=32, L=1, n_blocks=[1], n_vis=[[500]],
                         n_sources=5),
    "tiny_w": lambda: dict(cfg_id=101, Ny=32, Nx=32, L=2, n_blocks=[2, 1],
                           n_vis=[[200, 150], [300]], w_max_cells=5.0, s_cap=17,
                           nu=_wide(2, 1.0, 2.0), n_sources=5),
    "tiny_dde": lambda: dict(cfg_id=102, Ny=32, Nx=48, L=2, n_blocks=[1, 3],
                             n_vis=[[400], [100, 57, 1]], w_max_cells=5.0, dde=True,
                             s_cap=21, nu=_wide(2, 1.0, 2.0), n_sources=5,
                             shared_uv=False),
    "C2s": lambda: dict(cfg_id=102_2, Ny=256, Nx=256, L=4, n_blocks=[4] * 4,
                        n_vis=[[12_000, 12_001, 11_999, 7_777]] * 4, w_max_cells=5.0,
                        s_cap=17, nu=_wide(4, 1.0, 2.0)),
    "C3s": _cfg_c3s,
    "C4s": lambda: dict(cfg_id=104, Ny=192, Nx=320, L=3, n_blocks=[2] * 3,
                        n_vis=[[20_000, 13_333]] * 3, w_max_cells=5.0, s_cap=17,
                        nu=_wide(3, 3.979, 8.019)),
    "C5s": lambda: dict(cfg_id=105, Ny=256, Nx=256, L=2, n_blocks=[1] * 2,
                        n_vis=[[200_000]] * 2, nu=_wide(2, 3.979, 8.019)),
    # C5 with VLA-like Earth-rotation tracks (the regime where gridding pays)
    "C5t": lambda: dict(cfg_id=5, Ny=4096, Nx=4096, L=16, n_blocks=[1] * 16,
                        n_vis=[[8_000_000]] * 16, nu=_wide(16, 3.979, 8.019), coverage="tracks"),
    "C5ts": lambda: dict(cfg_id=106, Ny=128, Nx=128, L=2, n_blocks=[1] * 2,
                         n_vis=[[60_000]] * 2, nu=_wide(2, 3.979, 8.019), coverage="tracks"),
    "dr_tiny": lambda: dict(cfg_id=107, Ny=32, Nx=32, L=2, n_blocks=[2, 1],
                            n_vis=[[300, 211], [400]], nu=_wide(2, 1.0, 2.0), coverage="tracks",
                            w_max_cells=2.0, s_cap=11, n_sources=5),
}


def config_names():
    return list(CONFIGS)
