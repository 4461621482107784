"""Long grid columns (Ky = 3072 ... 8192): the column transforms of these
lengths run in two passes (N = N1 N2); long rows (Kx = 3072 ... 8192) run as
half-length complex transforms with radix-3 and radix-5 passes where the
length has those factors (3072 = 3 2^10, 5120 = 5 2^10, 6144 = 3 2^11) and
192 ... 512 threads per row.  Tall, narrow images keep the FP64 oracle
cheap while the column length is that of the 4096^2-image workloads.
Forward, adjoint and the dual step against the oracle at the FP32 bound."""
import sys

import numpy as np
import pytest

import synth
from _cases import Case, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


# (Ny, Nx): Ky = 2 Ny (image edges are multiples of 16, so Kx is a multiple
# of 32 and every such plan takes the two-pass transform)
SHAPES = [(1536, 16), (2048, 16), (2560, 16), (3072, 16), (4096, 16), (4096, 32),
          # long rows: Kx = 3072 (radix 3), 4096, 5120 (radix 5, the 1536 x 2560
          # image's rows), 6144 (radix 3), 8192
          (16, 1536), (16, 2048), (16, 2560), (16, 3072), (16, 4096),
          # long columns and long rows together (the image-first order with
          # the persistent row passes): Kx = 3072, 5120, 6144, 8192
          (1536, 1536), (1536, 2560), (2048, 3072), (2048, 4096)]


@pytest.mark.parametrize("ny,nx", SHAPES)
def test_long_transforms(ny, nx):
    from test_gpu_parity import gpu_forward, gpu_adjoint, gpu_dual
    import oracle
    _say("[fft-long] Ny", ny, "Nx", nx)
    prob = synth.make_problem("tiny", Ny=ny, Nx=nx, n_vis=[[3000]])
    c = Case("long%d_%d" % (ny, nx), problem=prob)
    plan = c.plan()
    want = c.op.forward({l: x.astype(np.float64) for l, x in c.X.items()})
    got = gpu_forward(c, plan)
    e = rel_l2(np.concatenate(got), np.concatenate(want))
    _say("  forward rel L2", e)
    assert e <= 1e-5
    want_a = c.op.adjoint(c.Y)
    got_a = gpu_adjoint(c, plan, c.Y)
    e = rel_l2(got_a[0], want_a[0])
    _say("  adjoint rel L2", e)
    assert e <= 1e-5
    Vp_o, grad_o, rho_o, res_o = oracle.dual_step(c.op, {l: x.astype(np.float64) for l, x in c.Xt.items()},
                                                  c.V, c.Y, c.eps)
    Vp, grad, rho, res = gpu_dual(c, plan, c.V, c.eps, None)
    assert rel_l2(rho, rho_o) <= 1e-5 and rel_l2(res, res_o) <= 1e-5
    assert rel_l2(np.concatenate(Vp), np.concatenate(Vp_o)) <= 1e-5
    e = rel_l2(grad[0], grad_o[0])
    _say("  grad rel L2", e)
    assert e <= 1e-5


@pytest.mark.parametrize("tile", [16, 32, 64])
def test_sparse_adjoint_over_tilings(tile):
    """With few visibilities on an image-first grid most merge regions are
    dead: the merge writes only the live ones into a zeroed adjoint grid and
    the inverse row pass loads only the 128-cell slabs with a live region
    (regions of 32 cells at 16- and 32-cell tiles, 64 at 64-cell tiles).
    The adjoint and the dual step's gradient must match the oracle at every
    tiling, twice in a row (the grid's dead cells stay zero)."""
    from test_gpu_parity import gpu_adjoint, gpu_dual
    import oracle
    prob = synth.make_problem("tiny", Ny=1536, Nx=2560, n_vis=[[1500]])
    c = Case("sparse1536_2560", problem=prob)
    plan = c.plan()
    plan.set_tuning(tile, 0)
    _say("[fft-long sparse] tile", tile, "info tile", plan.info()["tile"])
    assert plan.info()["tile"] == tile
    want_a = c.op.adjoint(c.Y)
    _, grad_o, _, _ = oracle.dual_step(c.op, {l: x.astype(np.float64) for l, x in c.Xt.items()},
                                       c.V, c.Y, c.eps)
    for _ in range(2):
        got_a = gpu_adjoint(c, plan, c.Y)
        e = rel_l2(got_a[0], want_a[0])
        _say("  adjoint rel L2", e)
        assert e <= 1e-5
        _, grad, _, _ = gpu_dual(c, plan, c.V, c.eps, None)
        e = rel_l2(grad[0], grad_o[0])
        _say("  grad rel L2", e)
        assert e <= 1e-5
