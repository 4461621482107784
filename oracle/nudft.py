"""Direct non-uniform DFT: the map the NUFFT Phi of eq. (1) approximates.

y_m = theta * sum_{p,q} x[p, q] exp(-i (omega_y,m pbar + omega_x,m qbar)),
pbar = p - Ny/2, qbar = q - Nx/2 (phase centre at pixel (Ny/2, Nx/2)).
O(M N): tiny inputs only.
"""
import numpy as np


def nudft(x, omega, theta=1.0):
    x = np.asarray(x, dtype=np.float64)
    Ny, Nx = x.shape
    pbar = np.arange(Ny) - Ny // 2
    qbar = np.arange(Nx) - Nx // 2
    ey = np.exp(-1j * np.outer(omega[:, 0], pbar))      # [M, Ny]
    ex = np.exp(-1j * np.outer(omega[:, 1], qbar))      # [M, Nx]
    return theta * np.einsum("mp,pq,mq->m", ey, x, ex)
