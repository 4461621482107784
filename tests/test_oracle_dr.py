"""Pins for the FP64 oracle of the visibility-gridding reduction (Section 3.4,
eqs. 4-5): H = G^H Theta^H Theta G, Lam = H_pp^(-1/2) on the nonzero rows,
Gamma = Lam G^H Theta^H, Phi' = Lam H F Z."""
import numpy as np
import pytest

import oracle
import synth
from oracle import dr


@pytest.fixture(scope="module")
def case():
    prob = synth.make_problem("dr_tiny")
    blk = prob.block(0, 0)
    w, off = blk.windows(np.complex128)
    theta = 0.7
    G = oracle.g_matrix(blk.base, blk.S, w, off, prob.Ky, prob.Kx, theta)
    s_y, s_x = prob.deapodisation()
    return prob, blk, w, off, theta, G, dr.reduce_block(G), s_y, s_x


def test_support_and_diagonal_from_windows(case):
    prob, blk, w, off, theta, G, red, s_y, s_x = case
    diag = np.zeros(prob.Ky * prob.Kx)
    for m in range(blk.M):
        S = blk.S[m]
        i, j = np.divmod(np.arange(S * S), S)
        cells = ((blk.base[m, 0] + i) % prob.Ky) * prob.Kx + (blk.base[m, 1] + j) % prob.Kx
        np.add.at(diag, cells, theta ** 2 * np.abs(w[off[m]:off[m + 1]]) ** 2)
    assert np.array_equal(red.support, np.nonzero(diag > 0)[0])
    assert np.allclose(red.lam, 1 / np.sqrt(diag[red.support]), rtol=1e-13, atol=0)


def test_holographic_matrix_is_hermitian_psd(case):
    prob, blk, w, off, theta, G, red, *_ = case
    H = red.H
    assert abs(H - H.conj().T).max() <= 1e-13 * abs(H).max()
    rng = np.random.default_rng(1)
    for _ in range(5):
        v = rng.standard_normal(H.shape[0]) + 1j * rng.standard_normal(H.shape[0])
        q = np.vdot(v, H @ v)
        g = G @ v
        assert abs(q.imag) <= 1e-12 * abs(q) and abs(q.real - np.vdot(g, g).real) <= 1e-12 * q.real
    # unit diagonal after whitening on the support
    LHL = red.A[:, red.support] @ np.diag(red.lam)
    assert np.allclose(np.diag(LHL), 1.0, rtol=0, atol=1e-13)


def test_gridding_of_model_data_is_reduced_operator(case):
    """Gamma (Phi x) = Phi' x: the reduced operator is the gridded plain one."""
    prob, blk, w, off, theta, G, red, s_y, s_x = case
    x = prob.image(0).astype(np.float64)
    op = oracle.Operator(prob.Ny, prob.Nx, s_y, s_x, [oracle.BlockG(0, theta, G)])
    y = op.forward({0: x})[0]
    lhs = dr.reduced_data(red, y)
    rhs = dr.phi_reduced(red, x, s_y, s_x, prob.Ky, prob.Kx)
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-13 * np.abs(rhs).max())


def test_reduced_adjoint_identity(case):
    prob, blk, w, off, theta, G, red, s_y, s_x = case
    rng = np.random.default_rng(2)
    x = rng.standard_normal((prob.Ny, prob.Nx))
    v = rng.standard_normal(len(red.support)) + 1j * rng.standard_normal(len(red.support))
    y = dr.phi_reduced(red, x, s_y, s_x, prob.Ky, prob.Kx)
    a = dr.phi_reduced_adj(red, v, s_y, s_x, prob.Ny, prob.Nx, prob.Ky, prob.Kx)
    lhs, rhs = np.vdot(v, y).real, np.sum(x * a)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(y) * np.linalg.norm(v)


def test_gridded_noise_has_unit_variance(case):
    """Gamma n has covariance Lam H Lam (unit diagonal) for standard complex n."""
    prob, blk, w, off, theta, G, red, *_ = case
    rng = np.random.default_rng(3)
    n = (rng.standard_normal((blk.M, 4000)) + 1j * rng.standard_normal((blk.M, 4000))) / np.sqrt(2)
    gn = red.Gamma @ n
    var = np.mean(np.abs(gn) ** 2, axis=1)
    assert abs(var.mean() - 1.0) < 0.02
    assert np.all(np.abs(var - 1.0) < 0.2)
