"""Pins for the FP64 oracle of the regularizer-free PDFB loop and its adaptive
l2 bounds (Section 2.2: eq. 2 with the non-negativity constraint only;
Section 3.3: effective noise estimation).

The loop solves: find x >= 0 with ||Phi x - y|| <= eps.  What fixes its
result independently of the iteration:
* the non-negative least-squares optimum x*, r* = min_{x>=0} ||Phi x - y||
  (scipy.optimize.nnls on the dense real system).  Any x >= 0 satisfies
  ||Phi x - y||^2 >= r*^2 + ||Phi (x - x*)||^2 (the variational inequality of
  x*), so a feasible limit obeys ||Phi (x - x*)||^2 <= eps^2 - r*^2;
* on noiseless data, any feasible x is within 2 eps of the truth in data
  space (triangle inequality);
* with noise above the assumed level the chi-square bound is infeasible
  (eps < r*); the adaptive rule raises eps until the residual is within
  lambda_hi of it, which brackets the final bound in [r*/lambda_hi, r*].
"""
import numpy as np
import pytest
import scipy.optimize

import oracle
import synth
from oracle import pdfb

NY = NX = 16
M = 800


@pytest.fixture(scope="module")
def small():
    prob = synth.make_problem("tiny", Ny=NY, Nx=NX, n_vis=[[M]])
    op = oracle.Operator.from_problem(prob)
    N = NY * NX
    A = np.empty((2 * M, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        y = op.forward({0: e.reshape(NY, NX)})[0]
        A[:M, k], A[M:, k] = y.real, y.imag
    lam = float(np.linalg.norm(A, 2) ** 2)
    return prob, op, A, lam


def _data(prob, op, kappa, seed=3):
    x_true = prob.image(0).astype(np.float64)
    rng = np.random.default_rng(seed)
    n = (rng.standard_normal(M) + 1j * rng.standard_normal(M)) / np.sqrt(2.0)
    return x_true, op.forward({0: x_true})[0] + kappa * n


def _nnls(A, y):
    b = np.concatenate([y.real, y.imag])
    xs, rs = scipy.optimize.nnls(A, b, maxiter=20 * A.shape[1])
    return xs, rs, b


def _run(op, y, eps, lam, n_iter, rule=None):
    return pdfb.pdfb(op, {0: np.zeros((NY, NX))}, [np.zeros(M, complex)], [y], eps, [1.0 / lam], {0: 0.99},
                     n_iter, rule=rule)


def test_limit_is_feasible_and_obeys_the_nnls_inequality(small):
    prob, op, A, lam = small
    _, y = _data(prob, op, 1.0)
    xs, rs, b = _nnls(A, y)
    eps = oracle.block_radii([M])
    assert rs < eps[0]                               # the chi-square bound is feasible here
    out = _run(op, y, eps, lam, 400)
    x = out["X"][0].ravel()
    assert x.min() >= 0.0
    r = np.linalg.norm(A @ x - b)
    assert r <= eps[0] * (1 + 1e-9)
    d2 = np.linalg.norm(A @ (x - xs)) ** 2
    assert d2 <= eps[0] ** 2 - rs ** 2 + 1e-6 * eps[0] ** 2
    # the iteration has settled: the primal step no longer moves x
    d, n = out["var"][0]
    assert d <= 1e-20 * n


def test_noiseless_data_is_fitted_within_twice_eps(small):
    prob, op, A, lam = small
    x_true, y = _data(prob, op, 0.0)
    eps = np.array([1e-3 * np.linalg.norm(y)])
    out = _run(op, y, eps, lam, 1500)
    x = out["X"][0].ravel()
    assert x.min() >= 0.0
    b = np.concatenate([y.real, y.imag])
    assert np.linalg.norm(A @ x - b) <= eps[0] * (1 + 1e-6)
    assert np.linalg.norm(A @ (x - x_true.ravel())) <= 2 * eps[0] * (1 + 1e-6)


def test_adaptive_bounds_settle_at_the_nnls_residual(small):
    prob, op, A, lam = small
    _, y = _data(prob, op, 2.0)                      # effective noise twice the assumed level
    xs, rs, b = _nnls(A, y)
    eps0 = oracle.block_radii([M])
    assert eps0[0] < rs                              # infeasible as given
    rule = dict(pdfb.DEFAULT_RULE)
    out = _run(op, y, eps0, lam, 1000, rule=rule)
    st = out["state"]
    assert st["fixed"][0] and st["count"][0] >= 1
    eps = out["eps"][0]
    assert rs / rule["lambda_hi"] * (1 - 1e-9) <= eps <= rs * (1 + 1e-9)
    # the bound ends (slightly) below r*, so the iterate is drawn to x* itself
    x = out["X"][0].ravel()
    assert np.linalg.norm(A @ (x - xs)) <= 1e-3 * rs


def test_rule_that_never_fires_keeps_the_bounds(small):
    prob, op, A, lam = small
    _, y = _data(prob, op, 2.0)
    eps0 = oracle.block_radii([M])
    for over in (dict(var_tol=0.0), dict(min_gap=10 ** 9)):
        rule = dict(pdfb.DEFAULT_RULE, **over)
        out = _run(op, y, eps0, lam, 200, rule=rule)
        assert out["eps"][0] == eps0[0] and out["state"]["count"][0] == 0
        assert out["state"]["since"][0] == 200 and not out["state"]["fixed"][0]


def test_degenerate_steps(small):
    prob, op, A, lam = small
    _, y = _data(prob, op, 1.0)
    rng = np.random.default_rng(9)
    x0 = rng.standard_normal((NY, NX))
    v0 = [rng.standard_normal(M) + 1j * rng.standard_normal(M)]
    # tau = 0: the primal iterate is the projection of x0 after one step and
    # never moves again; x~ = 2 P(x0) - x0 then x~ = x
    out = pdfb.pdfb(op, {0: x0}, v0, [y], oracle.block_radii([M]), [1.0 / lam], {0: 0.0}, 3)
    assert np.array_equal(out["X"][0], np.maximum(x0, 0.0))
    assert np.array_equal(out["Xt"][0], np.maximum(x0, 0.0))
    # an unbounded ball with v = 0: the dual stays 0 (up to the rounding of
    # the literal Moreau form, z - sigma (z / sigma)), so x = P_+(x0)
    out = pdfb.pdfb(op, {0: x0}, [np.zeros(M, complex)], [y], [1e300], [1.0 / lam], {0: 0.99}, 2)
    phix = op.forward(out["Xt"])[0]
    assert np.abs(out["V"][0]).max() <= 1e-15 * np.abs(phix).max() / lam
    assert np.abs(out["X"][0] - np.maximum(x0, 0.0)).max() <= 1e-14 * np.abs(x0).max()


def test_channels_and_blocks_run_independently():
    """Channels are separate problems: the loop over an operator with two
    channels equals the loops over each channel's operator alone."""
    from oracle.analysis import channel_operator
    prob = synth.make_problem("tiny_w")
    op = oracle.Operator.from_problem(prob)
    rng = np.random.default_rng(4)
    X0 = {l: np.abs(rng.standard_normal((prob.Ny, prob.Nx))) for l in range(prob.L)}
    Y = [rng.standard_normal(blk.G.shape[0]) + 1j * rng.standard_normal(blk.G.shape[0]) for blk in op.blocks]
    V0 = [0.1 * y for y in Y]
    eps = np.array([0.5 * np.linalg.norm(y) for y in Y])
    sigma = np.linspace(0.5, 1.5, len(Y)) * 1e-3
    tau = {0: 0.3, 1: 0.7}
    rule = dict(pdfb.DEFAULT_RULE, var_tol=0.9, min_gap=2, freeze=False)
    both = pdfb.pdfb(op, X0, V0, Y, eps, sigma, tau, 6, rule=rule)
    for l in range(prob.L):
        ks = [k for k, blk in enumerate(op.blocks) if blk.l == l]
        one = pdfb.pdfb(channel_operator(op, l), {l: X0[l]}, [V0[k] for k in ks], [Y[k] for k in ks],
                        eps[ks], sigma[ks], tau, 6, rule=rule)
        assert np.array_equal(one["X"][l], both["X"][l])
        assert np.array_equal(one["eps"], both["eps"][ks])
        for i, k in enumerate(ks):
            assert np.array_equal(one["V"][i], both["V"][k])
