"""GPU parity of the visibility-gridding reduction (Section 3.4, eqs. 4-5)
computed on the device: phi_dr_setup's rows of Lam H and gridded data
y' = Gamma y, then Phi', its adjoint and the reduced dual step
(l2ball_dual_step_dr), against the FP64 oracle of the reduction.

Complex64 rows: 1e-5.  FP16 rows: 2e-3 against the FP64 G (a plan that
reduces keeps G itself in complex64, so the FP16 error is the rows' own
rounding).  Cases: VLA-like tracks with 7 x 7 windows
(4096^2-grid shape at small size), w-stencils up to 11 x 11, and 13 x 13 /
15 x 15 windows whose reduced rows grow up to 21 x 21.
"""
import sys

import numpy as np
import pytest

from _cases import rel_l2, quantise
from test_dr_geometry import wide_windows_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _blocks(name):
    import synth
    if name == "wide":
        return wide_windows_problem()
    prob = synth.make_problem(name)
    return prob, [prob.block(l, b) for (l, b) in prob.block_list()]


CASES = [("dr_tiny", "c64", 1e-5), ("C5ts", "c64", 1e-5), ("C5ts", "f16", 2e-3), ("wide", "c64", 1e-5),
         ("wide", "f16", 2e-3)]


@pytest.mark.parametrize("name,prec,tol", CASES)
def test_device_reduction(name, prec, tol):
    import oracle
    from oracle import dr
    from paper_2209_07604_amd import Plan, DR, GRAPH
    _say("[dr]", name, prec)
    prob, blocks = _blocks(name)
    s_y, s_x = prob.deapodisation()
    rng = np.random.default_rng(np.random.SeedSequence((220907604, 66)))
    ch = [l for (l, b) in prob.block_list()]
    theta = 0.5 + rng.random(len(blocks))
    X = {l: prob.image(l).astype(np.float64) for l in range(prob.L)}
    wins = [blk.windows(np.complex128) for blk in blocks]
    # the oracle's data: y = theta Phi x + n per block
    Y = []
    for k, blk in enumerate(blocks):
        G = oracle.g_matrix(blk.base, blk.S, wins[k][0], wins[k][1], prob.Ky, prob.Kx, theta[k])
        y = oracle.Operator(prob.Ny, prob.Nx, s_y, s_x, [oracle.BlockG(ch[k], theta[k], G)]).forward(X)[0]
        Y.append(y + (rng.standard_normal(blk.M) + 1j * rng.standard_normal(blk.M)) / np.sqrt(2))
    plan = Plan(prob.Ny, prob.Nx, prob.n_blocks, [b.M for b in blocks], np.concatenate([b.base for b in blocks]),
                np.concatenate([b.S for b in blocks]), s_y, s_x, theta, g_prec=prec, flags=DR)
    for k, (w, off) in enumerate(wins):
        plan.load_g(k, w)
    info = plan.info()
    _say("  M %d -> M' %d, taps G %d H %d, largest row %d" % (
        info["n_vis_total"], info["dr_rows"], info["n_taps"], info["dr_taps"], info["dr_max_window"]))
    y = plan.to_plan(torch.from_numpy(np.concatenate(Y).astype(np.complex64)).cuda())
    yred_p, m_red = plan.dr_setup(y)
    red_plan = plan.reduced()
    yred = red_plan.from_plan(yred_p).cpu().numpy().astype(np.complex128)   # cell order per block
    torch.cuda.synchronize()
    cells, rbase, rS = plan.dr_rows()
    assert info["g_bytes"] == 8 * info["n_taps"]          # G kept in complex64
    for gq, bound in [(None, tol)]:
        reds, yo, ops = [], [], []
        for k, blk in enumerate(blocks):
            w = wins[k][0] if gq is None else quantise(wins[k][0], gq)
            red = dr.reduce_block(oracle.g_matrix(blk.base, blk.S, w, wins[k][1], prob.Ky, prob.Kx, theta[k]))
            reds.append(red)
            yo.append(dr.reduced_data(red, Y[k]))
            ops.append(oracle.BlockG(ch[k], 1.0, red.A))
        assert list(m_red) == [len(r.support) for r in reds]
        # y' and the rows of Lam H (read back from the reduced plan, times theta)
        e_y = rel_l2(yred, np.concatenate(yo))
        o = 0
        e_h = 0.0
        for k, red in enumerate(reds):
            m = len(red.support)
            # the reduced plan's user order is cell order per block
            order = np.argsort(cells[o:o + m], kind="stable")
            assert np.array_equal(cells[o:o + m][order], red.support)
            su = rS[o:o + m][order].astype(np.int64)
            offs = np.concatenate([[0], np.cumsum(su ** 2)])
            got = red_plan.read_g(k, int(offs[-1]))
            A = oracle.g_matrix(rbase[o:o + m][order], su, got, offs, prob.Ky, prob.Kx, theta[k])
            e_h = max(e_h, abs(A - red.A).max() / abs(red.A).max())
            o += m
        op = oracle.Operator(prob.Ny, prob.Nx, s_y, s_x, ops)
        # Phi', Re Phi'^dagger and the reduced dual step
        x = torch.from_numpy(np.stack([X[l] for l in range(prob.L)]).astype(np.float32)).cuda()
        yf = red_plan.from_plan(red_plan.forward(x)).cpu().numpy().astype(np.complex128)
        e_f = rel_l2(yf, np.concatenate(op.forward({l: X[l].astype(np.float32).astype(np.float64) for l in X})))
        ag = red_plan.adjoint(yred_p).cpu().numpy().astype(np.float64)
        ao = op.adjoint(yo)
        e_a = max(rel_l2(ag[l], ao[l]) for l in range(prob.L))
        eps = np.array([oracle.chi2_radius(m) for m in m_red])
        Xt = {l: 0.5 * X[l].astype(np.float32).astype(np.float64) for l in X}
        rng2 = np.random.default_rng(5)
        V = [0.1 * (rng2.standard_normal(m) + 1j * rng2.standard_normal(m)) for m in m_red]
        Vp_o, grad_o, rho_o, res_o = oracle.dual_step(op, Xt, V, yo, eps)
        xt = torch.from_numpy(np.stack([Xt[l] for l in range(prob.L)]).astype(np.float32)).cuda()
        vr = red_plan.to_plan(torch.from_numpy(np.concatenate(V).astype(np.complex64)).cuda())
        red_plan.set_flags(GRAPH)
        grad, rho, res = plan.dual_step_dr(xt, vr, yred_p, torch.from_numpy(eps).cuda())
        vp = red_plan.from_plan(vr).cpu().numpy().astype(np.complex128)
        torch.cuda.synchronize()
        red_plan.check()
        e_v = rel_l2(vp, np.concatenate(Vp_o))
        e_g = max(rel_l2(grad.cpu().numpy()[l], grad_o[l]) for l in range(prob.L))
        e_r = rel_l2(rho.cpu().numpy(), rho_o)
        e_s = rel_l2(res.cpu().numpy(), res_o)
        _say("  vs oracle with %s G: y' %.2e rows %.2e forward %.2e adjoint %.2e v+ %.2e grad %.2e rho %.2e "
             "res %.2e (rho/eps %s)" % (gq or "FP64", e_y, e_h, e_f, e_a, e_v, e_g, e_r, e_s,
                                        np.round(rho_o / eps, 2)))
        assert max(e_y, e_h, e_f, e_a, e_v, e_g, e_r, e_s) <= bound
        if name == "C5ts":
            assert np.all(rho_o > eps)     # the projection is active on every block
