"""Rows of G from per-visibility tables, in FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

A row of G is the compact-support interpolation kernel centred on the
visibility's uv point, convolved with the Fourier kernels of the w-term
(w-projection, Section 3.2) and of the antenna pair's DDEs (Section 3.1).
The paper gives no formula for either kernel; the readings taken are:

* interpolation kernel: separable Kaiser-Bessel of width J,
  psi(d) = I0(beta sqrt(1 - (2d/J)^2)) / I0(beta) (0 outside |d| <= J/2),
  sampled at kappa - (b + i), i = 0..J-1, with b = floor(kappa - J/2) + 1
  the first grid cell of the support;
* w-kernel (per axis, separable): half-width h cells, taps
  t_k = cos^2(pi k / (2 (h + 1))) exp(-i pi k^2 / (4 max(a, 1/2))),
  k = -h..h, divided by their sum (h = 0 gives the single tap 1);
* DDE kernel of the pair (i, j): d_i convolved with conj(flip(d_j)), the
  antennas' Fourier kernels (square, odd edge).

The row's per-axis factor is u = psi (*) t (length J + 2h), the window is
outer(u_y, u_x) (*) (d_i (*) conj(flip(d_j))) of edge S = J + 2h + sd - 1
(sd = edge of the pair kernel), and its first grid cell is
b - h - (sd - 1) / 2 on each axis (mod K).
"""
import numpy as np
from scipy.signal import convolve2d
from scipy.special import i0


def kb_beta(J):
    """Kaiser-Bessel shape for 2x oversampling (Beatty et al. 2005)."""
    return np.pi * np.sqrt((J / 2.0) ** 2 * 1.5 ** 2 - 0.8)


def kb_taps(kappa, J):
    """(b, [psi(kappa - b - i)]_i) for one axis."""
    b = int(np.floor(kappa - J / 2.0)) + 1
    d = kappa - (b + np.arange(J))
    t = 1.0 - (2.0 * d / J) ** 2
    beta = kb_beta(J)
    psi = np.where(t >= 0.0, i0(beta * np.sqrt(np.maximum(t, 0.0))) / i0(beta), 0.0)
    return b, psi


def w_taps(h, a):
    """Normalised w-kernel taps of half-width h (per axis)."""
    if h == 0:
        return np.ones(1, dtype=np.complex128)
    k = np.arange(-h, h + 1, dtype=np.float64)
    c = np.cos(np.pi * k / (2.0 * (h + 1))) ** 2 * np.exp(-1j * np.pi * k * k / (4.0 * max(a, 0.5)))
    return c / c.sum()


def pair_kernel(d_i, d_j):
    """DDE kernel of an antenna pair: d_i (*) conj(flip(d_j))."""
    return convolve2d(d_i, np.conj(d_j[::-1, ::-1]), mode="full")


def window(kappa_y, kappa_x, J, h, a, dde_pair=None):
    """(first cell (b_y, b_x), S, S x S complex128 window) of one row."""
    by, py = kb_taps(kappa_y, J)
    bx, px = kb_taps(kappa_x, J)
    t = w_taps(h, a)
    uy = np.convolve(py, t)
    ux = np.convolve(px, t)
    win = np.outer(uy, ux)
    sd = 1
    if dde_pair is not None:
        win = convolve2d(win, dde_pair, mode="full")
        sd = dde_pair.shape[0]
    ext = h + (sd - 1) // 2
    return (by - ext, bx - ext), win.shape[0], win


def block_windows(kappa, J, h, a, ant=None, dde=None, K=None):
    """Windows of many rows: kappa [n, 2], h [n] int, a [n], ant [n, 2] or
    None, dde [n_ant, sa, sa] or None.  Returns (base [n, 2] (mod K if given),
    S [n], flat windows, offsets)."""
    n = len(h)
    base = np.zeros((n, 2), dtype=np.int64)
    S = np.zeros(n, dtype=np.int64)
    wins = []
    for m in range(n):
        pk = None
        if ant is not None and ant[m, 0] >= 0:
            pk = pair_kernel(dde[ant[m, 0]], dde[ant[m, 1]])
        (b_y, b_x), s, w = window(kappa[m, 0], kappa[m, 1], J, int(h[m]), float(a[m]), pk)
        base[m] = (b_y, b_x)
        S[m] = s
        wins.append(w.ravel())
    if K is not None:
        base = np.mod(base, np.asarray(K, dtype=np.int64))
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(S * S, out=off[1:])
    return base, S, (np.concatenate(wins) if wins else np.zeros(0, complex)), off
