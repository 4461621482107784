"""phi_power_iteration_static (no device allocation: its scratch image is the
library's fixed per-GPU array) against phi_power_iteration with a caller
scratch image, through the C ABI: two plans in a row, the second smaller,
each bitwise equal to the existing entry point; sizes beyond the array are
rejected before any device work."""
import sys

import numpy as np
import pytest

from _cases import Case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("name", ["C2s", "tiny_w"])   # the second call runs a smaller plan
def test_static_scratch_matches_power_iteration(name):
    c = Case(name)
    plan = c.plan(g_prec="f16" if name == "C2s" else "c64")
    rng = np.random.default_rng(3)
    x0 = torch.from_numpy(rng.random((plan.L, plan.ny, plan.nx)).astype(np.float32)).cuda()
    xa, xb = x0.clone(), x0.clone()
    tmp = torch.empty_like(x0)
    for n_iter in (7, 4):
        nu_a = plan.power_iteration(xa, n_iter, tmp=tmp)
        nu_b = plan.power_iteration_static(xb, n_iter)
        torch.cuda.synchronize()
        _say("[static scratch]", name, n_iter, nu_a.cpu().numpy(), nu_b.cpu().numpy())
        assert torch.equal(nu_a, nu_b)
        assert torch.equal(xa, xb)


def test_static_scratch_rejects_large_plans():
    from paper_2209_07604_amd import Plan, PhiError
    # 3 channels of 2048^2 pixels: 48 MiB of float32 > 32 MiB
    p = Plan(2048, 2048, [1, 1, 1], [1, 1, 1], np.zeros((3, 2), np.int32), [7, 7, 7], np.ones(2048), np.ones(2048),
             None, bind=False)
    x = torch.zeros((3, 2048, 2048), dtype=torch.float32, device="cuda")
    with pytest.raises(PhiError) as e:
        p.power_iteration_static(x, 1)
    assert e.value.code == -7
