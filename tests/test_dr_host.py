"""The library's host-side gridding reduction (phi_dr_*) against the FP64
oracle of Section 3.4 (no GPU needed): support, Lam, the rows of Lam H and
the gridded data y' = Gamma y."""
import numpy as np
import pytest

import oracle
import synth
from oracle import dr


@pytest.mark.parametrize("name,l,b", [("dr_tiny", 0, 0), ("dr_tiny", 0, 1), ("dr_tiny", 1, 0), ("C5ts", 0, 0)])
def test_reduction_matches_oracle(name, l, b):
    from paper_2209_07604_amd import dr_reduce
    prob = synth.make_problem(name)
    blk = prob.block(l, b)
    w, off = blk.windows(np.complex128)
    rng = np.random.default_rng(l * 10 + b)
    theta = 0.5 + rng.random()
    y = rng.standard_normal(blk.M) + 1j * rng.standard_normal(blk.M)
    red = dr.reduce_block(oracle.g_matrix(blk.base, blk.S, w, off, prob.Ky, prob.Kx, theta))
    out = dr_reduce(prob.Ky, prob.Kx, blk.base, blk.S, w, theta, y)
    assert np.array_equal(out["cell"], red.support)
    assert np.allclose(out["lam"], red.lam, rtol=1e-12, atol=0)
    W = out["W"]
    assert W == 2 * int(blk.S.max()) - 1 and np.all(out["S"] == W)
    offs = np.arange(len(out["S"]) + 1, dtype=np.int64) * W * W
    A = oracle.g_matrix(out["base"], out["S"].astype(np.int64), out["windows"], offs, prob.Ky, prob.Kx, 1.0)
    diff = abs(A - red.A).max()
    assert diff <= 1e-12 * abs(red.A).max()
    yr = dr.reduced_data(red, y)
    assert np.allclose(out["y"], yr, rtol=0, atol=1e-12 * np.abs(yr).max())
    if name == "C5ts":
        assert blk.M / len(red.support) > 4      # tracks: the gridded data are several times smaller


def test_reduction_rejects():
    from paper_2209_07604_amd import dr_reduce, PhiError
    base = np.zeros((2, 2), np.int32)
    w = np.ones(2 * 169, complex)
    with pytest.raises(PhiError):          # S = 13 > 11: reduced windows would exceed 21
        dr_reduce(64, 64, base, [13, 13], w)
    with pytest.raises(PhiError):          # grid too small for the tiles
        dr_reduce(24, 64, base, [7, 7], np.ones(98, complex))
    with pytest.raises(PhiError):
        dr_reduce(64, 64, base, [7, 7], np.ones(98, complex), theta=0.0)
