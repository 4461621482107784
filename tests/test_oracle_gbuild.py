"""Pins for the FP64 oracle of the rows of G (interpolation kernel convolved
with the w-kernel and the antenna pair's DDE kernel, Sections 3.1-3.2).

Identities that hold for the row definition and fail under the plausible
mistakes (a lost normalisation, a missing conjugate or flip, an index shift,
a wrong first cell):
* the tap sum factorises: sum(window) = sum(psi_y) sum(psi_x) sum(d_i)
  conj(sum(d_j)), because the w-kernel taps sum to 1;
* first moments add under convolution: the window's (complex-weighted) row
  centroid is centroid(psi_y) + h + centroid of the pair kernel's rows;
* a row without DDE is an outer product (rank one);
* at an integer kappa the Kaiser-Bessel taps are palindromic with centre
  tap exactly 1, and the support's cells are centred on kappa;
* the pair kernel of an antenna with itself is its autocorrelation:
  Hermitian about the centre, with centre value sum |d|^2;
* the w-kernel is even with unit sum, and tends to the normalised taper as
  the chirp flattens (a -> infinity).
"""
import numpy as np
import pytest

from oracle import gbuild

J = 7


def _dde(rng, n_ant=5, sa=3):
    d = 0.2 * (rng.standard_normal((n_ant, sa, sa)) + 1j * rng.standard_normal((n_ant, sa, sa)))
    d[:, sa // 2, sa // 2] += np.exp(1j * rng.uniform(-np.pi, np.pi, n_ant))
    return d


def _centroid_rows(w):
    r = np.arange(w.shape[0])[:, None]
    return np.sum(r * w) / np.sum(w)


@pytest.mark.parametrize("h", [0, 1, 3, 5])
@pytest.mark.parametrize("with_dde", [False, True])
def test_tap_sum_factorises(h, with_dde):
    rng = np.random.default_rng(10 + h)
    dde = _dde(rng)
    for _ in range(20):
        ky, kx = rng.uniform(-50, 50, 2)
        a = rng.uniform(0.2, 6.0)
        pk = gbuild.pair_kernel(dde[1], dde[3]) if with_dde else None
        _, S, w = gbuild.window(ky, kx, J, h, a, pk)
        _, py = gbuild.kb_taps(ky, J)
        _, px = gbuild.kb_taps(kx, J)
        want = py.sum() * px.sum()
        if with_dde:
            want *= dde[1].sum() * np.conj(dde[3].sum())
        # rounding scale: the sums of magnitudes (the chirp taps cancel)
        t = gbuild.w_taps(h, a)
        scale = np.abs(py).sum() * np.abs(px).sum() * np.abs(t).sum() ** 2 / abs(t.sum()) ** 2
        if with_dde:
            scale *= np.abs(pk).sum()
        assert abs(w.sum() - want) <= 1e-13 * scale
        assert S == J + 2 * h + (3 + 3 - 1 - 1 if with_dde else 0)


def test_first_moments_add():
    rng = np.random.default_rng(3)
    dde = _dde(rng)
    for h in (0, 2, 4):
        for _ in range(10):
            ky, kx = rng.uniform(-20, 20, 2)
            pk = gbuild.pair_kernel(dde[0], dde[2])
            _, _, w = gbuild.window(ky, kx, J, h, rng.uniform(0.5, 4.0), pk)
            _, py = gbuild.kb_taps(ky, J)
            want = _centroid_rows(py[:, None]) + h + _centroid_rows(pk)
            assert abs(_centroid_rows(w) - want) <= 1e-11


def test_die_rows_are_rank_one():
    rng = np.random.default_rng(4)
    for h in (0, 1, 4):
        _, _, w = gbuild.window(rng.uniform(0, 99), rng.uniform(0, 99), J, h, 2.5, None)
        sv = np.linalg.svd(w, compute_uv=False)
        assert sv[1] <= 1e-13 * sv[0]


def test_kb_taps_at_integer_kappa():
    for kappa in (0.0, 17.0, -5.0):
        b, psi = gbuild.kb_taps(kappa, J)
        assert np.array_equal(psi, psi[::-1])
        assert psi[J // 2] == 1.0
        assert b + J // 2 == kappa          # support centred on kappa
        assert np.all(psi > 0)              # psi(+-3) > 0 inside the support


def test_first_cell_follows_support():
    """The row's first cell is the Kaiser-Bessel support's first cell moved
    out by the w half-width and the DDE half-width."""
    rng = np.random.default_rng(6)
    dde = _dde(rng)
    for _ in range(20):
        ky, kx = rng.uniform(-30, 30, 2)
        h = int(rng.integers(0, 5))
        (b_y, b_x), S, _ = gbuild.window(ky, kx, J, h, 1.5, gbuild.pair_kernel(dde[0], dde[1]))
        assert b_y == int(np.floor(ky - J / 2)) + 1 - h - 2
        assert b_x == int(np.floor(kx - J / 2)) + 1 - h - 2
        # the window's centre cell is within half a cell of kappa
        assert abs(b_y + (S - 1) / 2 - ky) <= 0.5 + 1e-12


def test_self_pair_is_autocorrelation():
    rng = np.random.default_rng(7)
    d = _dde(rng)[2]
    p = gbuild.pair_kernel(d, d)
    assert np.allclose(p, np.conj(p[::-1, ::-1]), rtol=0, atol=1e-15)
    c = p.shape[0] // 2
    assert abs(p[c, c] - np.sum(np.abs(d) ** 2)) <= 1e-14


def test_w_kernel():
    for h in (1, 2, 5):
        for a in (0.3, 1.0, 4.0):
            t = gbuild.w_taps(h, a)
            assert abs(t.sum() - 1.0) <= 1e-15
            assert np.allclose(t, t[::-1], rtol=0, atol=1e-16)
        k = np.arange(-h, h + 1)
        taper = np.cos(np.pi * k / (2 * (h + 1))) ** 2
        assert np.allclose(gbuild.w_taps(h, 1e12), taper / taper.sum(), rtol=0, atol=1e-9)
    assert np.array_equal(gbuild.w_taps(0, 3.0), np.ones(1))


@pytest.mark.parametrize("name", ["tiny_w", "tiny_dde"])
def test_generator_rows_follow_the_definition(name):
    """The seeded generator's windows (the G the plans load) are the rows
    defined here: same first cells, sizes and taps."""
    import synth
    prob = synth.make_problem(name)
    K = np.array([prob.Ky, prob.Kx])
    for (l, b) in prob.block_list():
        blk = prob.block(l, b)
        kappa = blk.omega * K / (2 * np.pi)
        h = (blk._skw - J) // 2
        a = prob.w_max_cells * blk.w
        a = np.where(np.round(a) > h, h.astype(np.float64), a)   # the generator's cap of the half-width
        w, off = blk.windows(np.complex128)
        for m in range(len(h)):
            pk = None
            if blk._pair_id is not None and blk._pair_id[m] >= 0:
                sd = int(blk._pair_sd[blk._pair_id[m]])
                pk = blk._pairs[blk._pair_id[m], :sd, :sd]
            (b_y, b_x), S, win = gbuild.window(kappa[m, 0], kappa[m, 1], J, int(h[m]), float(a[m]), pk)
            assert S == blk.S[m]
            assert (b_y % prob.Ky, b_x % prob.Kx) == tuple(blk.base[m])
            got = w[off[m]:off[m + 1]]
            assert np.abs(got - win.ravel()).max() <= 1e-13 * np.abs(win).max()
