"""The allocation-free operator apply (igaf_apply_static) against igaf_apply.

igaf_apply_static runs the kernels of igaf_apply with the library's static
device scratch in place of the caller's workspace.  Both sum every DOF in
the same fixed order, so the outputs must be equal bit for bit.  Two calls in
a row, the second on a smaller patch (the array keeps the first call's
contents), each for the mass-only and the full operator; a patch whose
slots exceed the static array is refused on the host before any launch,
leaving y untouched.
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import nonuniform_knots, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ig():
    import torch

    assert torch.cuda.is_available()
    from paper_2207_00280_amd import igafem

    return igafem


def test_apply_static_matches_apply(ig):
    import torch

    L = ig.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for call, (p, K) in enumerate(((3, (40, 7, 6)), (2, (9, 4, 3)))):   # the second smaller
        knots = [nonuniform_knots(k, p, 90 + 3 * call + d) for d, k in enumerate(K)]
        plan = ig.Plan(p, K, knots)
        kd = to_dev(W.kappa_lognormal(plan.nelem, plan.nqp, seed=70 + call))
        ud = to_dev(W.normal_vector(plan.ndof, 80 + call))
        for aM, aK in ((1.0, 0.0), (0.7, -1.3)):
            ref = plan.apply(kd, ud, aM, aK)
            y = torch.full_like(ud, float("nan"))
            st = L.igaf_apply_static(plan.handle, kd.data_ptr(), ud.data_ptr(), aM, aK, y.data_ptr(), stream)
            assert st == ig.OK, L.igaf_last_error().decode()
            torch.cuda.synchronize()
            assert torch.equal(y, ref), (call, aM, aK)
        # the Python wrapper of the same entry point
        y2 = plan.apply_static(kd, ud, torch.empty_like(ud), 0.7, -1.3)
        torch.cuda.synchronize()
        assert torch.equal(y2, ref)


def test_apply_static_refuses_oversized_patch(ig):
    import torch

    L = ig.lib()
    p, K = 3, (32, 128, 128)   # 16 384 runs of 16 x 35 slot values: 9.2 M doubles > 8 M
    plan = ig.Plan(p, K, [W.open_uniform_knots(k, p) for k in K])
    assert plan.apply_workspace() > 8 << 20
    tiny = torch.full((8,), 3.0, dtype=torch.float64, device="cuda")
    st = L.igaf_apply_static(plan.handle, tiny.data_ptr(), tiny.data_ptr(), 1.0, 1.0,
                             tiny[4:].data_ptr(), None)
    assert st == ig.EUNSUPPORTED
    assert "static array" in L.igaf_last_error().decode()
    torch.cuda.synchronize()
    assert bool((tiny == 3.0).all())
    assert L.igaf_apply_static(None, None, None, 1.0, 1.0, None, None) == ig.EINVAL
