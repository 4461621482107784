"""Grid columns of 1024 and 2048 points (512^2 and 1024^2 images, the
default workload's length): one-pass column transforms with 8 and 4 columns
per work-group.  Tall images keep the FP64 oracle cheap while the column
length is the workload's; the wider ones span several panels and the
XCD-aware panel order.  Forward, adjoint and the dual step against the
oracle at the FP32 bound."""
import sys

import numpy as np
import pytest

import synth
from _cases import Case, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


# (Ny, Nx): Ky = 2 Ny = 1024 (8 columns per work-group) or 2048 (4 columns)
SHAPES = [(512, 16), (512, 128), (1024, 16), (1024, 128)]


@pytest.mark.parametrize("ny,nx", SHAPES)
def test_mid_column_transforms(ny, nx):
    from test_gpu_parity import gpu_forward, gpu_adjoint, gpu_dual
    import oracle
    _say("[fft-mid] Ny", ny, "Nx", nx)
    prob = synth.make_problem("tiny", Ny=ny, Nx=nx, n_vis=[[3000]])
    c = Case("mid%d_%d" % (ny, nx), problem=prob)
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
