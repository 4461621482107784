"""Kaiser-Bessel interpolation kernel used to build the rows of G.

The paper builds G from a compact-support non-uniform Fourier interpolation
kernel following the NUFFT of Fessler & Sutton (Section 2.1, eq. 1) and leaves the
kernel type and width to a parameter file.  The generator uses the
Kaiser-Bessel kernel of width J = 7 on a 2x oversampled grid, with the shape
parameter of Beatty, Nishimura & Pauly (2005):

    psi(d)     = I0(beta sqrt(1 - (2d/J)^2)) / I0(beta),   |d| <= J/2
    psi_hat(f) = J sinh(sqrt(beta^2 - (pi J f)^2)) / (I0(beta) sqrt(beta^2 - (pi J f)^2))
    beta       = pi sqrt((J/alpha)^2 (alpha - 1/2)^2 - 0.8)

psi_hat is the continuous Fourier transform of psi.  Z scales pixel
(p, q) by s_y[p] s_x[q] with s = 1/psi_hat(pbar / K) (deapodisation), where
pbar = p - N/2 is the pixel offset from the phase centre.

I0 is scipy.special.i0 (called, not reimplemented).
"""
import numpy as np
from scipy.special import i0

KB_J = 7
KB_ALPHA = 2.0


def kb_beta(J=KB_J, alpha=KB_ALPHA):
    """Beatty et al. (2005) shape parameter for width J, oversampling alpha."""
    return np.pi * np.sqrt((J / alpha) ** 2 * (alpha - 0.5) ** 2 - 0.8)


def kb_psi(d, J=KB_J, beta=None):
    """Kernel value at signed distance d (grid cells); 0 outside |d| <= J/2."""
    if beta is None:
        beta = kb_beta(J)
    d = np.asarray(d, dtype=np.float64)
    t = 1.0 - (2.0 * d / J) ** 2
    inside = t >= 0.0
    out = np.zeros_like(d)
    out[inside] = i0(beta * np.sqrt(t[inside])) / i0(beta)
    return out


def kb_psi_hat(f, J=KB_J, beta=None):
    """Closed-form Fourier transform of kb_psi at frequency f (cycles/cell).

    Valid while (pi J f) < beta, which holds for |f| <= 1/4 at alpha = 2.
    """
    if beta is None:
        beta = kb_beta(J)
    f = np.asarray(f, dtype=np.float64)
    z2 = beta ** 2 - (np.pi * J * f) ** 2
    if np.any(z2 <= 0):
        raise ValueError("frequency outside the closed-form range")
    z = np.sqrt(z2)
    return J * np.sinh(z) / (i0(beta) * z)


def deapodisation(N, K, J=KB_J, beta=None):
    """Per-axis scale s[p] = 1 / psi_hat((p - N/2) / K), p = 0..N-1 (FP64)."""
    pbar = np.arange(N, dtype=np.float64) - N // 2
    return 1.0 / kb_psi_hat(pbar / K, J, beta)


def window_base(kappa, S):
    """First grid index of an S-tap window centred on continuous index kappa.

    b = floor(kappa - S/2) + 1, so the taps b .. b+S-1 are the S integers
    closest to kappa (their distances lie in (-S/2, S/2]).  Computed in FP64.
    """
    return np.floor(np.asarray(kappa, dtype=np.float64) - S / 2.0).astype(np.int64) + 1


def kb_taps_1d(kappa, J=KB_J, beta=None):
    """J kernel taps along one axis for each kappa: returns (base, taps[M, J])."""
    kappa = np.asarray(kappa, dtype=np.float64)
    b = window_base(kappa, J)
    d = kappa[:, None] - (b[:, None] + np.arange(J)[None, :])
    return b, kb_psi(d, J, beta)
