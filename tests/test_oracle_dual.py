"""Pins for the l2-ball projection and the PDFB dual step (Section 2.2, eq. 2)."""
import os

import numpy as np
import pytest
from scipy import optimize, stats

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_c(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def test_projection_properties():
    rng = np.random.default_rng(0)
    for _ in range(50):
        n = rng.integers(1, 40)
        y, z = _rand_c(rng, n), 3 * _rand_c(rng, n)
        eps = rng.uniform(0.1, 5.0)
        p = oracle.l2ball_project(z, y, eps)
        assert np.linalg.norm(p - y) <= eps * (1 + 1e-15)
        assert np.allclose(oracle.l2ball_project(p, y, eps), p, rtol=0, atol=1e-15 * np.abs(p).max())
        if np.linalg.norm(z - y) <= eps:
            assert np.array_equal(p, z)
        else:
            assert abs(np.linalg.norm(p - y) - eps) <= 1e-14 * eps
        # variational inequality: Re <z - p, u - p> <= 0 for any u in the ball
        for _ in range(20):
            u = y + eps * rng.uniform() ** (1 / (2 * n)) * (lambda d: d / np.linalg.norm(d))(_rand_c(rng, n))
            assert np.vdot(z - p, u - p).real <= 1e-12 * (1 + np.abs(z).max() ** 2)


def test_dual_step_is_prox_of_the_conjugate():
    """v+ minimises sigma f*(u) + 1/2 ||u - z||^2 with f* the support function
    of the ball: f*(u) = Re <u, y> + eps ||u||  (brute force on 3 complex entries)."""
    rng = np.random.default_rng(5)
    for trial in range(6):
        n = 3
        y, v, phix = _rand_c(rng, n), _rand_c(rng, n), _rand_c(rng, n)
        sigma = rng.uniform(0.3, 2.0)
        eps = [0.2, 1.0, 3.0, 30.0, 0.0, 1.5][trial]
        z = v + sigma * phix
        vp = z - sigma * oracle.l2ball_project(z / sigma, y, eps)

        def obj(u):
            uc = u[:n] + 1j * u[n:]
            return sigma * (np.vdot(uc, y).real + eps * np.linalg.norm(uc)) + 0.5 * np.linalg.norm(uc - z) ** 2
        best = None
        for start in [np.zeros(2 * n), np.concatenate([z.real, z.imag]), rng.standard_normal(2 * n)]:
            res = optimize.minimize(obj, start, method="Nelder-Mead",
                                    options=dict(xatol=1e-11, fatol=1e-14, maxiter=40000, maxfev=40000))
            if best is None or res.fun < best.fun:
                best = res
        u = best.x[:n] + 1j * best.x[n:]
        assert np.linalg.norm(u - vp) <= 1e-5 * max(1.0, np.linalg.norm(vp))
        assert obj(np.concatenate([vp.real, vp.imag])) <= best.fun + 1e-10


def _problem_state(name="tiny_w", seed=3):
    prob = synth.make_problem(name)
    rng = np.random.default_rng(seed)
    op = oracle.Operator.from_problem(prob, {k: rng.uniform(0.5, 2) for k in prob.block_list()})
    X = {l: prob.image(l).astype(np.float64) for l in range(prob.L)}
    Y = [y + 0.05 * _rand_c(rng, len(y)) for y in op.forward(X)]
    Xt = {l: 0.5 * X[l] for l in X}
    V = [0.1 * _rand_c(rng, len(y)) for y in Y]
    return prob, op, Xt, V, Y


def test_dual_step_limits():
    prob, op, Xt, V, Y = _problem_state()
    nb = len(Y)
    phix = op.forward(Xt)
    sig = np.linspace(0.5, 2.0, nb)
    # eps -> infinity: the ball contains everything, v+ = 0, grad = 0
    # (the Moreau form z - sigma (z / sigma) leaves only rounding residue)
    Vp, grad, rho, r = oracle.dual_step(op, Xt, V, Y, np.full(nb, 1e30), sig)
    for k in range(nb):
        z = V[k] + sig[k] * phix[k]
        assert np.max(np.abs(Vp[k])) <= 4e-16 * np.max(np.abs(z))
    # eps = 0: projection onto {y}, v+ = v + sigma (Phi x - y)
    Vp, grad, rho, r = oracle.dual_step(op, Xt, V, Y, np.zeros(nb), sig)
    for k in range(nb):
        want = V[k] + sig[k] * (phix[k] - Y[k])
        assert np.allclose(Vp[k], want, rtol=0, atol=1e-13 * np.abs(want).max())
        assert abs(rho[k] - np.linalg.norm(V[k] / sig[k] + phix[k] - Y[k])) <= 1e-13 * rho[k]
        assert abs(r[k] - np.linalg.norm(phix[k] - Y[k])) <= 1e-13 * r[k]
    # v = 0: rho == r
    Vz = [np.zeros_like(v) for v in V]
    _, _, rho, r = oracle.dual_step(op, Xt, Vz, Y, np.ones(nb), sig)
    assert np.allclose(rho, r, rtol=1e-15, atol=0)


def test_dual_step_shrink_form_and_branches():
    """Outside the ball v+ = sigma (1 - eps/rho) c with c = v/sigma + Phi x - y;
    inside it v+ = 0 exactly."""
    prob, op, Xt, V, Y = _problem_state("tiny_dde", 9)
    nb = len(Y)
    phix = op.forward(Xt)
    c = [V[k] + phix[k] - Y[k] for k in range(nb)]
    nrm = np.array([np.linalg.norm(ck) for ck in c])
    eps = nrm * np.where(np.arange(nb) % 2 == 0, 0.5, 1.5)
    Vp, grad, rho, r = oracle.dual_step(op, Xt, V, Y, eps, np.ones(nb))
    for k in range(nb):
        if eps[k] < nrm[k]:
            want = (1 - eps[k] / nrm[k]) * c[k]
            assert np.allclose(Vp[k], want, rtol=0, atol=1e-13 * np.abs(want).max())
        else:
            assert np.max(np.abs(Vp[k])) <= 4e-16 * np.max(np.abs(V[k] + phix[k]))
    G = op.adjoint(Vp)
    for l in grad:
        assert np.array_equal(grad[l], G[l])


def test_chi2_radius_coverage():
    """P(||n||^2 <= eps^2) for standard complex noise: the exact Gamma(M, 1)
    law of ||n||^2 and a Monte-Carlo draw both give ~0.977 (mean + 2 sd)."""
    M = 1000
    eps = oracle.chi2_radius(M)
    exact = stats.gamma.cdf(eps ** 2, a=M)
    assert abs(exact - stats.norm.cdf(2.0)) < 0.01
    rng = np.random.default_rng(2022)
    n = (rng.standard_normal((10_000, M)) + 1j * rng.standard_normal((10_000, M))) / np.sqrt(2)
    frac = np.mean(np.sum(np.abs(n) ** 2, axis=1) <= eps ** 2)
    assert abs(frac - exact) < 0.005


def test_block_radii_golden():
    tab = np.loadtxt(os.path.join(GOLDEN, "chi2_exp1_blocks.txt"))
    for M_l, M_b, e2 in tab:
        other = M_l - M_b
        eps = oracle.block_radii([M_b, other])
        assert abs(eps[0] ** 2 - e2) <= 1e-9 * e2
    eps = oracle.block_radii([800_000, 200_000])
    assert abs(np.sum(eps ** 2) - oracle.chi2_radius(1e6) ** 2) <= 1e-9 * 1e6
