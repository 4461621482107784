"""Regularizer-free PDFB iteration with adaptive l2 bounds, in FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

Problem: eq. (2) with the regularization r reduced to the non-negativity
constraint the paper imposes on the image cube (Section 2.2.1):

    find x_l >= 0 with ||Phi_{l,b} x_l - y_{l,b}||_2 <= eps_{l,b} for every b.

Channels are independent here (no regularizer couples them).  It is solved by
the primal-dual forward-backward iteration Section 2.2.3 builds on (Condat
2013, Vu 2013), taken with the data-fidelity dual update first:

    v^{k+1}  = dual step at x~^k           (``dual.dual_step``: Moreau form)
    x^{k+1}  = P_+(x^k - tau_l sum_b Re Phi_{l,b}^H v_b^{k+1})
    x~^{k+1} = 2 x^{k+1} - x^k

which is the primal-first Condat-Vu sequence with its indices shifted by one
half step.  It converges for tau_l ||sum_b sigma_b Phi_{l,b}^H Phi_{l,b}|| < 1
(tau_l sigma_l ||Phi_l||^2 < 1 when every block of channel l has sigma_l).

Adaptive l2 bounds (Section 3.3, effective noise level estimation): the paper
describes the strategy -- start without active priors, update the noise-level
estimates and the l2 bounds as the iteration proceeds, fix them once the
bounds are satisfied -- and cites Dabbech et al. (2018) for it.  The update
taken is that work's adaptive-bound rule.  After the primal update of
iteration k, every block b of channel l whose bound is not yet fixed:

  1. counts one more iteration since its last update (``since``);
  2. if ``freeze`` and r_b <= lambda_hi eps_b: its bound is satisfied and
     fixed from now on;
  3. else, if the channel's relative image variation
     ||x^{k+1} - x^k|| / ||x^{k+1}|| is below ``var_tol`` (an image that is
     zero counts as not settled), ``since >= min_gap`` and r_b lies outside
     [lambda_lo eps_b, lambda_hi eps_b]:
         eps_b <- lambda_mix r_b + (1 - lambda_mix) eps_b,  since <- 0.

r_b is the residual ||Phi_b x~^k - y_b|| that the dual step of the same
iteration reports.  The variation test is taken on squared norms,
d2 < var_tol^2 n2, so no square root enters the decision.
"""
import numpy as np

from .dual import dual_step

DEFAULT_RULE = dict(lambda_lo=0.99, lambda_hi=1.01, lambda_mix=0.618, var_tol=1e-3, min_gap=10,
                    freeze=True)


def primal_step(X, grad, tau):
    """x+ = max(x - tau_l grad_l, 0), x~ = 2 x+ - x, per channel.
    Returns (X+, Xt+, var) with var[l] = (||x+ - x||^2, ||x+||^2)."""
    Xp, Xt, var = {}, {}, {}
    for l, x in X.items():
        x = np.asarray(x, dtype=np.float64)
        xp = np.maximum(x - tau[l] * np.asarray(grad[l], dtype=np.float64), 0.0)
        Xp[l] = xp
        Xt[l] = 2.0 * xp - x
        var[l] = (float(np.sum((xp - x) ** 2)), float(np.sum(xp ** 2)))
    return Xp, Xt, var


def new_state(nb):
    """Per-block rule state: iterations since the last update, fixed flag,
    number of updates."""
    return {"since": np.zeros(nb, dtype=np.int64), "fixed": np.zeros(nb, dtype=bool),
            "count": np.zeros(nb, dtype=np.int64)}


def eps_update(op, eps, res, var, state, rule):
    """One application of the adaptive-bound rule (module header) to every
    block; returns the new eps (state is updated in place)."""
    eps = np.array(eps, dtype=np.float64)
    for k, blk in enumerate(op.blocks):
        if state["fixed"][k]:
            continue
        state["since"][k] += 1
        if rule["freeze"] and res[k] <= rule["lambda_hi"] * eps[k]:
            state["fixed"][k] = True
            continue
        d2, n2 = var[blk.l]
        settled = n2 > 0.0 and d2 < rule["var_tol"] ** 2 * n2
        outside = res[k] < rule["lambda_lo"] * eps[k] or res[k] > rule["lambda_hi"] * eps[k]
        if settled and outside and state["since"][k] >= rule["min_gap"]:
            eps[k] = rule["lambda_mix"] * res[k] + (1.0 - rule["lambda_mix"]) * eps[k]
            state["since"][k] = 0
            state["count"][k] += 1
    return eps


def pdfb(op, X0, V0, Y, eps0, sigma, tau, n_iter, rule=None, Xt0=None, state=None):
    """n_iter iterations from (x^0, x~^0 = Xt0 or X0, v^0).

    X0: {l: image}; V0, Y: per-block lists; eps0, sigma: per block; tau: per
    channel (dict or sequence).  rule: None (fixed bounds) or a dict with the
    keys of DEFAULT_RULE.  Returns a dict with the final X, Xt, V, eps,
    state, and the last iteration's grad, rho, res and var."""
    X = {l: np.asarray(x, dtype=np.float64) for l, x in X0.items()}
    Xt = {l: np.asarray(x, dtype=np.float64) for l, x in (Xt0 if Xt0 is not None else X0).items()}
    V = [np.asarray(v, dtype=np.complex128) for v in V0]
    eps = np.array(eps0, dtype=np.float64)
    if state is None:
        state = new_state(len(op.blocks))
    grad = rho = res = var = None
    for _ in range(n_iter):
        V, grad, rho, res = dual_step(op, Xt, V, Y, eps, sigma)
        X, Xt, var = primal_step(X, grad, tau)
        if rule is not None:
            eps = eps_update(op, eps, res, var, state, rule)
    return {"X": X, "Xt": Xt, "V": V, "eps": eps, "state": state, "grad": grad, "rho": rho, "res": res,
            "var": var}
