"""Phi_{l,b} = Theta_{l,b} G_{l,b} F Z and its adjoint, in FP64 (Section 2.1, eq. 1).

Definitions used here (the paper fixes the factorisation, not the
conventions; the readings are the ones listed in the design notes):

* Z (K x N, real): zero-padding and scaling.  Pixel (p, q) of the Ny x Nx
  image, with offsets pbar = p - Ny/2, qbar = q - Nx/2 from the phase centre,
  is multiplied by s_y[p] s_x[q] and placed at grid cell
  (pbar mod Ky, qbar mod Kx) of the Ky x Kx oversampled grid.
* F (K x K): the unnormalised 2-D DFT, X[k] = sum_n x[n] exp(-2 pi i k.n / K).
  Its adjoint is the unnormalised inverse DFT, i.e. K * numpy.fft.ifft2.
* G (M x K, sparse): row m is a dense S_m x S_m window placed at grid rows
  (b_y + i) mod Ky and columns (b_x + j) mod Kx.
* Theta: diagonal whitening, one real scalar theta_b per data block.

Phi^dagger used for a real image is the adjoint for the real inner product
<x, x'> = sum x x' on images and Re <z, z'> on visibilities:
Phi^dagger v = Re(Z^T F^H G^H Theta v).  ``adjoint_complex`` omits the Re.
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


def _centred_rows(N, K):
    """Grid index (n - N/2) mod K of every image index n."""
    return (np.arange(N) - N // 2) % K


def zpad(x, s_y, s_x, Ky, Kx):
    """Z x: scale by s_y[p] s_x[q] and place at the centred wrapped cell."""
    x = np.asarray(x, dtype=np.float64)
    Ny, Nx = x.shape
    grid = np.zeros((Ky, Kx), dtype=np.complex128)
    grid[np.ix_(_centred_rows(Ny, Ky), _centred_rows(Nx, Kx))] = np.outer(s_y, s_x) * x
    return grid


def zpad_adj(grid, s_y, s_x, Ny, Nx):
    """Z^T g: read back the centred cells and scale (complex in, complex out)."""
    Ky, Kx = grid.shape
    return grid[np.ix_(_centred_rows(Ny, Ky), _centred_rows(Nx, Kx))] * np.outer(s_y, s_x)


def fft2_fwd(grid):
    """F g: unnormalised forward 2-D DFT with exp(-2 pi i k n / K)."""
    return np.fft.fft2(grid)


def fft2_adj(grid):
    """F^H g = K * ifft2(g): numpy's ifft2 carries 1/K, which the adjoint does not."""
    return np.fft.ifft2(grid) * grid.size


def g_matrix(base, S, windows, offsets, Ky, Kx, theta=1.0):
    """theta * G as a CSR matrix (M x Ky*Kx) built from dense windows."""
    base = np.asarray(base, dtype=np.int64)
    S = np.asarray(S, dtype=np.int64)
    M = len(S)
    nnz = S * S
    indptr = np.zeros(M + 1, dtype=np.int64)
    np.cumsum(nnz, out=indptr[1:])
    assert indptr[-1] == offsets[-1]
    cols = np.empty(indptr[-1], dtype=np.int64)
    for s in np.unique(S):
        sel = np.nonzero(S == s)[0]
        i = np.repeat(np.arange(s), s)
        j = np.tile(np.arange(s), s)
        r = (base[sel, 0][:, None] + i[None, :]) % Ky
        c = (base[sel, 1][:, None] + j[None, :]) % Kx
        pos = indptr[sel][:, None] + np.arange(s * s)[None, :]
        cols[pos] = r * Kx + c
    vals = np.asarray(windows, dtype=np.complex128) * theta
    return sp.csr_matrix((vals, cols, indptr), shape=(M, Ky * Kx))


@dataclass
class BlockG:
    """One data block (l, b): theta_b * G_{l,b} as CSR plus its channel."""
    l: int
    theta: float
    G: sp.csr_matrix


def grid_fwd(x, s_y, s_x, Ky, Kx):
    """F Z x flattened row-major (length Ky*Kx)."""
    return fft2_fwd(zpad(x, s_y, s_x, Ky, Kx)).ravel()


class Operator:
    """Phi for a list of blocks over L channels sharing one grid geometry."""

    def __init__(self, Ny, Nx, s_y, s_x, blocks):
        self.Ny, self.Nx = Ny, Nx
        self.Ky, self.Kx = 2 * Ny, 2 * Nx
        self.s_y = np.asarray(s_y, dtype=np.float64)
        self.s_x = np.asarray(s_x, dtype=np.float64)
        self.blocks = blocks

    @classmethod
    def from_problem(cls, prob, theta=None, blocks=None):
        """Build from a synth.Problem; theta maps (l, b) -> whitening scalar."""
        s_y, s_x = prob.deapodisation()
        out = []
        for (l, b) in (blocks if blocks is not None else prob.block_list()):
            blk = prob.block(l, b)
            w, off = blk.windows(np.complex128)
            th = 1.0 if theta is None else float(theta[(l, b)])
            out.append(BlockG(l, th, g_matrix(blk.base, blk.S, w, off, prob.Ky, prob.Kx, th)))
        return cls(prob.Ny, prob.Nx, s_y, s_x, out)

    def forward(self, X):
        """[Phi_{l,b} x_l for every block]; X maps channel -> image."""
        grids = {}
        out = []
        for blk in self.blocks:
            if blk.l not in grids:
                grids[blk.l] = grid_fwd(X[blk.l], self.s_y, self.s_x, self.Ky, self.Kx)
            out.append(blk.G @ grids[blk.l])
        return out

    def adjoint_complex(self, V):
        """{l: sum_b Phi_{l,b}^H v_b} as complex images (no real part taken)."""
        acc = {}
        for blk, v in zip(self.blocks, V):
            g = blk.G.conj().T @ np.asarray(v, dtype=np.complex128)
            acc[blk.l] = acc.get(blk.l, 0) + g
        out = {}
        for l, g in acc.items():
            grid = fft2_adj(g.reshape(self.Ky, self.Kx))
            out[l] = zpad_adj(grid, self.s_y, self.s_x, self.Ny, self.Nx)
        return out

    def adjoint(self, V):
        """{l: Re sum_b Phi_{l,b}^H v_b}: the adjoint for real images."""
        return {l: g.real for l, g in self.adjoint_complex(V).items()}
