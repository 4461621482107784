"""Geometry of the visibility-gridding reduction (Section 3.4, eqs. 4-5) that
a plan created with PHI_DR computes on the host, against the FP64 oracle's
holographic matrix (no GPU needed): the reduced rows are exactly the
oracle's support {p : H_pp > 0}, every nonzero of row p of Lam H lies inside
the row's window, and that window is the smallest odd square doing so.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from oracle import dr


def _plan(prob, blocks, prec="c64", flags=None):
    from paper_2209_07604_amd import Plan, DR
    s_y, s_x = prob.deapodisation()
    base = np.concatenate([b.base for b in blocks])
    S = np.concatenate([b.S for b in blocks])
    return Plan(prob.Ny, prob.Nx, prob.n_blocks, [b.M for b in blocks], base, S, s_y, s_x, None, g_prec=prec,
                flags=DR if flags is None else flags, bind=False)


class _Blk:
    """A block given by its window origins, sizes and windows."""

    def __init__(self, base, S, rng):
        self.base = np.ascontiguousarray(base, np.int32)
        self.S = np.ascontiguousarray(S, np.int32)
        self.M = len(self.S)
        n = (self.S.astype(np.int64) ** 2)
        self._off = np.concatenate([[0], np.cumsum(n)])
        self._w = rng.standard_normal(self._off[-1]) + 1j * rng.standard_normal(self._off[-1])

    def windows(self, dtype):
        return self._w.astype(dtype), self._off


def wide_windows_problem():
    """13 x 13 and 15 x 15 windows (S > 11) in overlapping pairs (offsets of up
    to 5 cells) on a sparse lattice that wraps across the grid's edge: the
    reduced rows grow past S but stay within 21 x 21.  Two blocks of one
    64 x 64 image."""
    rng = np.random.default_rng(np.random.SeedSequence((220907604, 555)))
    prob = synth.make_problem("dr_tiny", Ny=64, Nx=64, L=1, n_blocks=[2], n_vis=[[24, 16]],
                              nu=np.array([1.0]))
    blocks = []
    for n in (24, 16):
        k = np.arange(n)
        pair, mem = k // 2, k % 2
        by = (pair // 4) * 30 + mem * rng.integers(2, 5, n) + (3 if n == 16 else 0)
        bx = (pair % 4) * 32 + mem * rng.integers(0, 3, n) + 120
        S = rng.choice([13, 15], n)
        blocks.append(_Blk(np.stack([by % 128, bx % 128], axis=1), S, rng))
    return prob, blocks


@pytest.mark.parametrize("name", ["dr_tiny", "wide", "C5ts"])
def test_rows_are_the_support_with_tight_windows(name):
    if name == "wide":
        prob, blocks = wide_windows_problem()
    else:
        prob = synth.make_problem(name)
        blocks = [prob.block(l, b) for (l, b) in prob.block_list()]
    plan = _plan(prob, blocks)
    cells, base, sten = plan.dr_rows()
    info = plan.info()
    assert info["dr_rows"] == len(cells) and info["dr_taps"] == int((sten.astype(np.int64) ** 2).sum())
    assert info["dr_max_window"] == int(sten.max())
    Ky, Kx = prob.Ky, prob.Kx
    o = 0
    for k, blk in enumerate(blocks):
        w, off = blk.windows(np.complex128)
        red = dr.reduce_block(oracle.g_matrix(blk.base, blk.S, w, off, Ky, Kx, 1.0))
        m = len(red.support)
        c, bb, ss = cells[o:o + m], base[o:o + m], sten[o:o + m].astype(np.int64)
        o += m
        # the reduced rows of block k are its support, once each
        assert np.array_equal(np.sort(c), red.support)
        assert np.all(ss % 2 == 1) and np.all(ss >= blk.S.min()) and np.all(ss <= 2 * blk.S.max() - 1)
        A = red.A.tocsr()
        row_of = {p: i for i, p in enumerate(red.support)}
        for j in range(m):
            a = A.getrow(row_of[c[j]])
            qy, qx = a.indices // Kx, a.indices % Kx
            dy = (qy - bb[j, 0]) % Ky
            dx = (qx - bb[j, 1]) % Kx
            # every nonzero of the row inside its window ...
            assert np.all(dy < ss[j]) and np.all(dx < ss[j])
            # ... which starts at the nonzeros' first row and column and is
            # the smallest odd square holding them
            assert dy.min() == 0 and dx.min() == 0
            ext = max(dy.max(), dx.max()) + 1
            assert ss[j] == ext + (1 - ext % 2)
        if name == "C5ts":
            assert blk.M / m > 2      # tracks: fewer gridded cells than visibilities
        if name == "wide":
            assert ss.max() > blk.S.max()   # overlapping windows widen the rows


def test_reduction_rejects():
    from paper_2209_07604_amd import PhiError, DR, GRAPH
    prob = synth.make_problem("dr_tiny")
    blocks = [prob.block(l, b) for (l, b) in prob.block_list()]
    with pytest.raises(PhiError) as e:       # no stored G to reduce
        _plan(prob, blocks, prec="kb", flags=DR)
    assert e.value.code == -1
    # 13 x 13 windows piled on one cell: the rows would need 25 x 25 windows
    from paper_2209_07604_amd import Plan
    base = np.array([[10, 10], [22, 22], [16, 16]], np.int32)
    with pytest.raises(PhiError) as e:
        Plan(32, 32, [1], [3], base, [13, 13, 13], np.ones(32), np.ones(32), None, flags=DR, bind=False)
    assert e.value.code == -7
    # the reduced plan's workspace comes on top of the plan's own
    p0 = _plan(prob, blocks, flags=GRAPH)
    p1 = _plan(prob, blocks, flags=GRAPH | DR)
    assert p1.workspace_size() > p0.workspace_size()
    assert p0.info()["dr_rows"] == 0
    with pytest.raises(PhiError) as e:        # no reduced plan without PHI_DR
        p0.reduced()
    assert e.value.code == -8
    r = p1.reduced()
    assert r.info()["reduced"] == 1 and r.info()["n_vis_total"] == p1.info()["dr_rows"]
    lib = p1._lib
    assert lib.phi_plan_destroy(r._h) == -8                       # owned by p1
    assert lib.phi_plan_workspace_size(r._h, ctypes.byref(ctypes.c_size_t())) == -8
    n = p1.info()["dr_rows"]
    assert lib.phi_plan_load_g(r._h, 0, np.zeros(1, np.complex128).ctypes.data, 0, None) == -8
