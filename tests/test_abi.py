"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad descriptors before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2209_07604_amd import _lib as L
    return L, L.load()


def test_exports_match_header():
    L, lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "phi.h")).read()
    declared = set(re.findall(r"^(?:phi_status|const char\*)\s+(\w+)\(", hdr, re.M))
    assert declared == set(L.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def _desc(L, ny=32, nx=32, n_blocks=(1,), n_vis=(3,), base=None, S=None, theta=None, keep=None, **kw):
    keep = [] if keep is None else keep
    nb = np.array(n_blocks, np.int32)
    nv = np.array(n_vis, np.int64)
    M = int(nv.sum())
    base = np.zeros((max(M, 0), 2), np.int32) if base is None else np.ascontiguousarray(base, np.int32)
    S = np.full(max(M, 0), 7, np.uint8) if S is None else np.ascontiguousarray(S, np.uint8)
    sy, sx = np.ones(ny), np.ones(nx)
    keep += [nb, nv, base, S, sy, sx]
    d = L.Desc()
    d.n_channels, d.ny, d.nx = len(nb), ny, nx
    d.h_n_blocks, d.h_n_vis = nb.ctypes.data, nv.ctypes.data
    d.h_base, d.h_stencil = base.ctypes.data, S.ctypes.data
    if theta is not None:
        th = np.asarray(theta, np.float64)
        keep.append(th)
        d.h_theta = th.ctypes.data
    d.h_scale_y, d.h_scale_x = sy.ctypes.data, sx.ctypes.data
    for k, v in kw.items():
        setattr(d, k, v)
    return d, keep


def _create(L, lib, d):
    h = ctypes.c_void_p()
    rc = lib.phi_plan_create(ctypes.byref(d), ctypes.byref(h))
    if rc == 0:
        lib.phi_plan_destroy(h)
    return rc


@pytest.mark.parametrize("kw,code", [
    (dict(ny=31), -2), (dict(ny=4), -2), (dict(nx=8192), -7), (dict(ny=36), -7),
    (dict(n_blocks=(0,), n_vis=()), -2), (dict(n_vis=(-1,)), -2),
    (dict(S=[7, 8, 7]), -3), (dict(S=[0, 7, 7]), -3), (dict(S=[23, 7, 7]), -3),
    (dict(base=[[0, 0], [64, 0], [0, 0]]), -3), (dict(base=[[0, 0], [0, -1], [0, 0]]), -3),
    (dict(theta=[0.0]), -3), (dict(theta=[np.nan]), -3),
    (dict(g_prec=4), -1), (dict(flags=64), -1), (dict(tile=8), -1), (dict(tile=48), -1),
    (dict(persist_blocks=-1), -1),
])
def test_create_rejects(kw, code):
    L, lib = _lib()
    d, keep = _desc(L, **kw)
    assert _create(L, lib, d) == code


def test_create_null_and_ok():
    L, lib = _lib()
    h = ctypes.c_void_p()
    assert lib.phi_plan_create(None, ctypes.byref(h)) == -1
    d, keep = _desc(L)
    assert lib.phi_plan_create(ctypes.byref(d), None) == -1
    d, keep = _desc(L, n_blocks=(2, 1), n_vis=(2, 0, 1), S=[1, 21, 7], base=[[0, 0], [63, 63], [5, 9]],
                    theta=[1.0, 2.0, 0.5])
    assert lib.phi_plan_create(ctypes.byref(d), ctypes.byref(h)) == 0
    info = L.Info()
    assert lib.phi_plan_get_info(h, ctypes.byref(info)) == 0
    assert info.n_vis_total == 3 and info.n_taps == 1 + 441 + 49 and info.n_blocks_total == 3
    assert info.ky == 64 and info.kx == 64 and info.tile == 32
    assert info.g_bytes == 8 * info.n_taps
    n = ctypes.c_size_t()
    assert lib.phi_plan_workspace_size(h, ctypes.byref(n)) == 0 and n.value >= info.g_bytes
    # calls in the wrong order or with bad buffers fail before touching HIP
    assert lib.phi_forward(h, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == -8
    assert lib.l2ball_dual_step(h, *([ctypes.c_void_p(16)] * 8), None) == -8
    assert lib.phi_psf(h, ctypes.c_void_p(16), None, None) == -8
    assert lib.phi_residual_image(h, *([ctypes.c_void_p(16)] * 4), None) == -8
    assert lib.phi_power_iteration(h, ctypes.c_void_p(16), ctypes.c_void_p(32), 3, ctypes.c_void_p(64), None) == -8
    assert lib.phi_plan_load_kb(h, 0, ctypes.c_void_p(16), None) == -8   # not a Kaiser-Bessel plan
    assert lib.phi_psf(None, ctypes.c_void_p(16), None, None) == -1
    # PDFB calls: rule and iteration count are checked first, then the plan state
    buf = [ctypes.c_void_p(16 * (k + 1)) for k in range(16)]
    good = L.EpsRule(0.99, 1.01, 0.618, 1e-3, 10, 1)
    assert lib.phi_pdfb_primal(h, buf[0], buf[1], buf[2], buf[3], None, None) == -8
    assert lib.phi_eps_update(h, buf[0], buf[1], ctypes.byref(good), buf[2], buf[3], None) == -8
    run = lambda n_iter, rule: lib.phi_pdfb_run(h, *buf[:7], n_iter, rule, *buf[7:13], None)
    assert run(3, None) == -8 and run(3, ctypes.byref(good)) == -8
    assert run(0, None) == -3
    for bad in (dict(lambda_lo=0.0), dict(lambda_lo=1.2), dict(lambda_hi=0.9), dict(lambda_mix=0.0),
                dict(lambda_mix=1.5), dict(var_tol=-1.0), dict(var_tol=np.inf), dict(min_gap=-1),
                dict(lambda_hi=np.nan)):
        r = L.EpsRule(0.99, 1.01, 0.618, 1e-3, 10, 1)
        for k, v in bad.items():
            setattr(r, k, v)
        assert run(3, ctypes.byref(r)) == -3, bad
        assert lib.phi_eps_update(h, buf[0], buf[1], ctypes.byref(r), buf[2], buf[3], None) == -3, bad
    assert lib.phi_eps_update(h, buf[0], buf[1], None, buf[2], buf[3], None) == -1
    # G builder: descriptor checks first, then the plan state
    gb = L.GBuild(7, 0, 1, 0)
    assert lib.phi_plan_build_g(h, 0, ctypes.byref(gb), buf[0], buf[1], buf[2], None, None, None) == -8
    assert lib.phi_plan_build_g(h, 7, ctypes.byref(gb), buf[0], buf[1], buf[2], None, None, None) == -3
    assert lib.phi_plan_build_g(h, 0, None, buf[0], buf[1], buf[2], None, None, None) == -1
    assert lib.phi_plan_build_g(None, 0, ctypes.byref(gb), buf[0], buf[1], buf[2], None, None, None) == -1
    for J in (2, 4, 13):
        assert lib.phi_plan_build_g(h, 0, ctypes.byref(L.GBuild(J, 0, 1, 0)), buf[0], buf[1], buf[2],
                                    None, None, None) == -3
    assert lib.phi_plan_build_g(h, 0, ctypes.byref(gb), buf[0], buf[1], buf[2], buf[3], None, None) == -1
    for n_ant, sa in ((0, 3), (4, 2), (4, 9)):
        assert lib.phi_plan_build_g(h, 0, ctypes.byref(L.GBuild(7, n_ant, sa, 0)), buf[0], buf[1], buf[2],
                                    buf[3], buf[4], None) == -3
    assert lib.phi_plan_read_g(h, 0, buf[0], 0, None) == -8
    assert lib.phi_plan_read_g(h, 0, buf[0], 5, None) == -1
    assert lib.phi_plan_read_g(h, 9, buf[0], 0, None) == -3
    assert lib.phi_pdfb_primal(None, buf[0], buf[1], buf[2], buf[3], None, None) == -1
    assert lib.phi_power_iteration(None, None, None, 3, None, None) == -1
    assert lib.phi_plan_bind(h, None, n.value, None) == -1
    assert lib.phi_plan_bind(h, ctypes.c_void_p(256), n.value - 1, None) == -4
    assert lib.phi_plan_bind(h, ctypes.c_void_p(255), n.value, None) == -4
    assert lib.phi_plan_load_g(h, 5, ctypes.c_void_p(16), 0, None) == -3
    assert lib.phi_plan_load_g(h, 0, ctypes.c_void_p(16), 0, None) == -8
    bad = np.array([1.0, -2.0, 1.0])
    assert lib.phi_plan_set_theta(h, ctypes.c_void_p(bad.ctypes.data), None) == -3
    assert lib.phi_plan_destroy(h) == 0
    assert lib.phi_status_string(-5) == b"non-finite norm"


def test_info_counts_follow_synthetic_problem():
    import synth
    L, lib = _lib()
    prob = synth.make_problem("C3s")
    blocks = [prob.block(l, b) for (l, b) in prob.block_list()]
    base = np.concatenate([b.base for b in blocks])
    S = np.concatenate([b.S for b in blocks])
    d, keep = _desc(L, ny=prob.Ny, nx=prob.Nx, n_blocks=prob.n_blocks,
                    n_vis=[b.M for b in blocks], base=base, S=S)
    h = ctypes.c_void_p()
    assert lib.phi_plan_create(ctypes.byref(d), ctypes.byref(h)) == 0
    info = L.Info()
    lib.phi_plan_get_info(h, ctypes.byref(info))
    assert info.n_taps == int(np.sum(S.astype(np.int64) ** 2))
    assert info.n_vis_total == len(S)
    lib.phi_plan_destroy(h)


def test_kaiser_bessel_mode_checks():
    """PHI_G_KB: one width J in {3, 5, 7, 9, 11}; G loading calls are mode-specific."""
    L, lib = _lib()
    h = ctypes.c_void_p()
    d, keep = _desc(L, n_vis=(3,), S=[7, 7, 9], g_prec=3)
    assert lib.phi_plan_create(ctypes.byref(d), ctypes.byref(h)) == -3
    d, keep = _desc(L, n_vis=(2,), S=[13, 13], g_prec=3)
    assert lib.phi_plan_create(ctypes.byref(d), ctypes.byref(h)) == -7
    d, keep = _desc(L, n_vis=(2,), S=[7, 7], g_prec=3)
    assert lib.phi_plan_create(ctypes.byref(d), ctypes.byref(h)) == 0
    info = L.Info()
    assert lib.phi_plan_get_info(h, ctypes.byref(info)) == 0
    assert info.g_bytes == 0
    assert lib.phi_plan_load_g(h, 0, ctypes.c_void_p(16), 0, None) == -8
    assert lib.phi_plan_load_kb(h, 0, ctypes.c_void_p(16), None) == -8   # not bound yet
    assert lib.phi_plan_load_kb(h, 3, ctypes.c_void_p(16), None) == -3
    assert lib.phi_plan_destroy(h) == 0


def test_pitch_classes(monkeypatch):
    """The one-pass dual step launches once per group of item pitches (host
    logic, no GPU): pitches are grouped from the smallest up until a group
    holds PHI_PITCH_CLASS_ITEMS items (default 8192).  Three items in three
    tiles with windows 1, 7 and 21 have pitches 32, 38 and 52 at T = 32."""
    L, lib = _lib()
    kw = dict(n_blocks=(1,), n_vis=(3,), S=[1, 7, 21], base=[[0, 0], [40, 40], [5, 50]], theta=[1.0])

    def classes():
        d, keep = _desc(L, **kw)
        h = ctypes.c_void_p()
        assert lib.phi_plan_create(ctypes.byref(d), ctypes.byref(h)) == 0
        info = L.Info()
        assert lib.phi_plan_get_info(h, ctypes.byref(info)) == 0
        assert info.n_items == 3
        lib.phi_plan_destroy(h)
        return info.pitch_classes

    monkeypatch.delenv("PHI_PITCH_CLASS_ITEMS", raising=False)
    assert classes() == 1
    monkeypatch.setenv("PHI_PITCH_CLASS_ITEMS", "1")
    assert classes() == 3
    monkeypatch.setenv("PHI_PITCH_CLASS_ITEMS", "2")   # 32 + 38 close a group; 52 alone joins it
    assert classes() == 1
