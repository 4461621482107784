"""Per-channel analysis quantities around Phi, in FP64.

* PSF and its normalisation (the paper's residual-image definition, in its
  section on data and evaluation metrics): with delta the image that is 1 at
  the phase centre (pixel (Ny/2, Nx/2)) and 0 elsewhere, the per-channel PSF
  is Phi_l^dagger Phi_l delta and eta_l is the factor that makes its peak 1.
  The peak is read at the phase centre, where Phi^dagger Phi delta equals
  ||Phi delta||^2 (a Rayleigh quotient of a positive operator).
* Residual image r_l = eta_l Phi_l^dagger (y_l - Phi_l x_l) (same passage).
* Operator norm ||Phi_l||^2 = largest eigenvalue of Phi_l^dagger Phi_l, the
  bound primal-dual step sizes must respect (the PDFB iteration of Section
  2.2).  ``op_norm2_dense`` is that definition written out (the explicit
  N x N matrix, for small images); ``power_iteration`` is the iterative
  method the GPU runs, step by step.

Phi^dagger is the adjoint for real images (``Operator.adjoint``).
"""
import numpy as np


def delta_image(Ny, Nx):
    """1 at the phase centre (Ny/2, Nx/2), 0 elsewhere."""
    d = np.zeros((Ny, Nx))
    d[Ny // 2, Nx // 2] = 1.0
    return d


def channel_operator(op, l):
    """Phi_l: the blocks of channel l only."""
    from .operator import Operator
    return Operator(op.Ny, op.Nx, op.s_y, op.s_x, [blk for blk in op.blocks if blk.l == l])


def normal(op, l, x):
    """Phi_l^dagger Phi_l x for one channel (sum over its blocks)."""
    sub = channel_operator(op, l)
    return sub.adjoint(sub.forward({l: x}))[l]


def psf(op, l):
    """Phi_l^dagger Phi_l delta."""
    return normal(op, l, delta_image(op.Ny, op.Nx))


def psf_peak(op, l):
    """Value of the PSF at the phase centre; eta_l = 1 / psf_peak."""
    return psf(op, l)[op.Ny // 2, op.Nx // 2]


def residual_image(op, X, Y, eta=None):
    """{l: eta_l Phi_l^dagger (y_l - Phi_l x_l)}; Y is the per-block list."""
    R = [np.asarray(y, complex) - p for y, p in zip(Y, op.forward(X))]
    out = op.adjoint(R)
    if eta is not None:
        out = {l: eta[l] * r for l, r in out.items()}
    return out


def op_norm2_dense(op, l):
    """Largest eigenvalue of the explicit N x N matrix Phi_l^dagger Phi_l
    (columns are the operator applied to the unit images)."""
    N = op.Ny * op.Nx
    A = np.empty((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        A[:, k] = normal(op, l, e.reshape(op.Ny, op.Nx)).ravel()
    A = 0.5 * (A + A.T)  # symmetric up to rounding
    return float(np.linalg.eigvalsh(A)[-1])


def power_iteration(op, l, x0, n_iter):
    """Power method on Phi_l^dagger Phi_l from x0: normalise, then n_iter
    times x <- A x / ||A x|| with nu = ||A x|| (x of unit norm).  Returns
    (nu, x) after the last step."""
    x = np.asarray(x0, dtype=np.float64)
    x = x / np.linalg.norm(x)
    nu = 0.0
    for _ in range(n_iter):
        ax = normal(op, l, x)
        nu = float(np.linalg.norm(ax))
        x = ax / nu
    return nu, x
