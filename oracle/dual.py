"""The l2-ball data-fidelity term and its PDFB dual update (Section 2.2, eq. 2).

Each block (l, b) carries the constraint Phi_{l,b} x_l in
B(y_{l,b}, eps_{l,b}) = {z : ||z - y_{l,b}||_2 <= eps_{l,b}}, whose indicator is
the data-fidelity term of eq. (2).  The radius follows the chi-square rule
stated under eq. (2): eps_l^2 = M_l + 2 sqrt(M_l) and
eps_{l,b}^2 = eps_l^2 M_{l,b} / M_l.

The dual step is the data-fidelity half of a primal-dual forward-backward
iteration (Condat 2013 / Vu 2013, cited in Section 2.2.3); the paper defers
its listing to the companion paper, so the step is taken in its standard
form via the Moreau identity for the conjugate of an indicator:

    z      = v + sigma * Phi x~
    v+     = z - sigma * P_B(y, eps)(z / sigma)
    grad_l = sum_b Re Phi_{l,b}^H v+_b

together with the two monitored norms rho = ||v/sigma + Phi x~ - y||
(the distance the projection acts on) and r = ||Phi x~ - y|| (residual).
"""
import numpy as np


def chi2_radius(M_l):
    """eps_l for a channel with M_l whitened visibilities: sqrt(M + 2 sqrt(M))."""
    M_l = np.asarray(M_l, dtype=np.float64)
    return np.sqrt(M_l + 2.0 * np.sqrt(M_l))


def block_radii(n_vis_l):
    """[eps_{l,b}] for one channel: eps_{l,b}^2 = eps_l^2 M_{l,b} / M_l."""
    n = np.asarray(n_vis_l, dtype=np.float64)
    M_l = n.sum()
    return np.sqrt(chi2_radius(M_l) ** 2 * n / M_l)


def l2ball_project(z, y, eps):
    """Euclidean projection of z onto {u : ||u - y|| <= eps}."""
    z = np.asarray(z, dtype=np.complex128)
    y = np.asarray(y, dtype=np.complex128)
    d = z - y
    n = np.linalg.norm(d)
    if n <= eps:
        return z.copy()
    return y + (eps / n) * d


def dual_step(op, Xt, V, Y, eps, sigma=None):
    """One data-fidelity dual step over every block of ``op`` (an Operator).

    Returns (V_plus, grad, rho, r): V_plus is the list of updated duals,
    grad maps channel -> sum_b Re Phi_{l,b}^H v+_b, rho/r are per-block norms.
    """
    nb = len(op.blocks)
    if sigma is None:
        sigma = np.ones(nb)
    phix = op.forward(Xt)
    Vp, rho, r = [], np.zeros(nb), np.zeros(nb)
    for k in range(nb):
        v = np.asarray(V[k], dtype=np.complex128)
        y = np.asarray(Y[k], dtype=np.complex128)
        s = float(sigma[k])
        z = v + s * phix[k]
        Vp.append(z - s * l2ball_project(z / s, y, float(eps[k])))
        rho[k] = np.linalg.norm(v / s + phix[k] - y)
        r[k] = np.linalg.norm(phix[k] - y)
    return Vp, op.adjoint(Vp), rho, r
