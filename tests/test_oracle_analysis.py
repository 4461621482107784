"""Pins for the FP64 oracle of the per-channel analysis quantities: PSF and
its peak normalisation, residual image (the paper's residual-image
definition, r_l = eta_l Phi_l^dagger (y_l - Phi_l x_l) with eta_l making the
PSF peak 1), and ||Phi_l||^2 by power iteration."""
import numpy as np
import pytest

import oracle
import synth
from oracle import analysis


@pytest.fixture(scope="module")
def case():
    prob = synth.make_problem("tiny_w")
    theta = {(l, b): 0.5 + 0.25 * k for k, (l, b) in enumerate(prob.block_list())}
    op = oracle.Operator.from_problem(prob, theta=theta)
    return prob, theta, op


def test_psf_peak_is_closed_form_from_window_sums(case):
    """delta at the phase centre lands on grid cell (0, 0) with value
    s_y[Ny/2] s_x[Nx/2]; its DFT is that constant everywhere, so
    (Phi delta)_m = theta s_c sum_t g_m[t] and the PSF peak is
    ||Phi delta||^2, computed here from the window tap sums alone."""
    prob, theta, op = case
    s_y, s_x = prob.deapodisation()
    s_c = s_y[prob.Ny // 2] * s_x[prob.Nx // 2]
    for l in range(prob.L):
        want = 0.0
        for (ll, b) in prob.block_list():
            if ll != l:
                continue
            blk = prob.block(ll, b)
            w, off = blk.windows(np.complex128)
            sums = np.add.reduceat(w, off[:-1]) if len(off) > 1 else np.zeros(0)
            want += float(np.sum(np.abs(theta[(ll, b)] * s_c * sums) ** 2))
        got = analysis.psf_peak(op, l)
        assert abs(got - want) <= 1e-12 * want


def test_power_iteration_converges_to_largest_eigenvalue(case):
    prob, theta, op = case
    l = 1
    lam = analysis.op_norm2_dense(op, l)
    rng = np.random.default_rng(5)
    x0 = rng.standard_normal((prob.Ny, prob.Nx))
    prev = 0.0
    for n in (1, 2, 5, 20, 60):
        nu, _ = analysis.power_iteration(op, l, x0, n)
        # ||A x|| over unit x never exceeds lambda_max, and for a symmetric PSD
        # operator it does not decrease along the power sequence
        assert nu <= lam * (1 + 1e-12)
        assert nu >= prev * (1 - 1e-12)
        prev = nu
    nu, x = analysis.power_iteration(op, l, x0, 400)
    assert abs(nu - lam) <= 1e-6 * lam
    # the iterate is (close to) an eigenvector
    ax = analysis.normal(op, l, x)
    assert np.linalg.norm(ax - lam * x) <= 1e-2 * lam


def test_psf_peak_is_a_rayleigh_quotient(case):
    """delta has unit norm, so the peak (<delta, A delta>) is at most lambda_max."""
    prob, theta, op = case
    for l in range(prob.L):
        assert 0 < analysis.psf_peak(op, l) <= analysis.op_norm2_dense(op, l) * (1 + 1e-12)


def test_residual_image(case):
    prob, theta, op = case
    rng = np.random.default_rng(6)
    X = {l: rng.standard_normal((prob.Ny, prob.Nx)) for l in range(prob.L)}
    Y0 = op.forward(X)
    # exact data: zero residual
    R0 = analysis.residual_image(op, X, Y0)
    for l in range(prob.L):
        assert np.abs(R0[l]).max() <= 1e-12 * max(np.abs(Y0[0]).max(), 1.0)
    # noisy data: <r, x'> = eta Re <y - Phi x, Phi x'> for any real x'
    Y = [y + rng.standard_normal(y.shape) + 1j * rng.standard_normal(y.shape) for y in Y0]
    eta = {l: 1.0 / analysis.psf_peak(op, l) for l in range(prob.L)}
    R = analysis.residual_image(op, X, Y, eta)
    Xp = {l: rng.standard_normal((prob.Ny, prob.Nx)) for l in range(prob.L)}
    P = op.forward(Xp)
    for l in range(prob.L):
        lhs = float(np.sum(R[l] * Xp[l]))
        rhs = eta[l] * sum(float(np.vdot(P[k], Y[k] - Y0[k]).real)
                           for k, blk in enumerate(op.blocks) if blk.l == l)
        assert abs(lhs - rhs) <= 1e-10 * (abs(rhs) + 1e-30)
    # the normalised PSF peaks at 1
    for l in range(prob.L):
        p = eta[l] * analysis.psf(op, l)
        assert abs(p[prob.Ny // 2, prob.Nx // 2] - 1.0) <= 1e-13
