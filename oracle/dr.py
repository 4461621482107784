"""Visibility-gridding dimensionality reduction (Section 3.4, eqs. 4-5), FP64.

For one data block with whitened data y, whitening Theta (here theta * I) and
de-gridding matrix G (M x K):

    H     = G^H Theta^H Theta G          (K x K, Hermitian, the holographic matrix)
    S     = {p : H_pp != 0}              (its nonzero rows, M' of them)
    Lam   = H_pp^(-1/2) on S, 0 elsewhere
    Gamma = Lam G^H Theta^H              (the gridding operator)
    y'    = Gamma y                      (restricted to S)
    Phi'  = Lam H F Z                    (eq. 5, rows restricted to S)

Phi'^H v' = Z^T F^H H Lam v' (H Hermitian, Lam real).  The l2 bound on the
reduced data follows the chi-square rule with M' points (an approximation:
the reduced noise Gamma n has covariance Lam H Lam, unit diagonal but not
white).  Everything here is plain sparse linear algebra on the oracle's G.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .operator import fft2_adj, fft2_fwd, zpad, zpad_adj


@dataclass
class Reduced:
    support: np.ndarray      # [M'] flat grid indices p (row-major, Ky x Kx), increasing
    lam: np.ndarray          # [M'] Lam_p = H_pp^(-1/2)
    H: sp.csr_matrix         # K x K holographic matrix
    Gamma: sp.csr_matrix     # M' x M gridding operator (rows on the support)
    A: sp.csr_matrix         # M' x K: rows of Lam H on the support (Phi' = A F Z)


def reduce_block(G_theta):
    """Reduction of one block from Theta G (CSR, M x K, theta already folded)."""
    Gt = sp.csr_matrix(G_theta)
    H = (Gt.conj().T @ Gt).tocsr()
    d = H.diagonal().real
    support = np.nonzero(d > 0)[0]
    lam = 1.0 / np.sqrt(d[support])
    L = sp.diags(lam)
    Gamma = (L @ Gt.conj().T[support, :]).tocsr()
    A = (L @ H[support, :]).tocsr()
    return Reduced(support, lam, H, Gamma, A)


def reduced_data(red, y):
    """y' = Gamma y."""
    return red.Gamma @ np.asarray(y, dtype=np.complex128)


def phi_reduced(red, x, s_y, s_x, Ky, Kx):
    """Phi' x = Lam H F Z x on the support."""
    return red.A @ fft2_fwd(zpad(x, s_y, s_x, Ky, Kx)).ravel()


def phi_reduced_adj(red, v, s_y, s_x, Ny, Nx, Ky, Kx):
    """Re Phi'^H v = Re Z^T F^H A^H v."""
    g = (red.A.conj().T @ np.asarray(v, dtype=np.complex128)).reshape(Ky, Kx)
    return zpad_adj(fft2_adj(g), s_y, s_x, Ny, Nx).real
