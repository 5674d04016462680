"""The allocation-free mass entry point (GPU): tlb_mass_noalloc, whose partial
sums live in the library's static device array, gives bitwise the sums and
the non-finite count of tlb_mass, on two calls in a row (the second on a
smaller lattice, so stale partials from the first call would show), in every
storage precision."""
import ctypes as C

import numpy as np
import pytest

from paper_1710_09534_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_09534_amd import tlb as t
    return t


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
def test_mass_noalloc_equals_tlb_mass(tlb, precision):
    import torch
    cases = [(W.random_fields(130, 70, geometry="cylinder", rho=(3.0, 2.0, 1.0)), 37),
             (W.reduction_case(nx=40, ny=24, R=8.0), 11)]
    for p, steps in cases:
        print("case no-alloc mass %s %s %dx%d steps=%d" % (precision, p["name"], p["nx"], p["ny"],
                                                           steps), flush=True)
        s = tlb.from_problem(p, precision)
        s.set_check_interval(0)
        s.step(steps)
        out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda:0")
        st = tlb.lib.tlb_mass_noalloc(s.ctx, C.c_void_p(out.data_ptr()))
        assert st == tlb.TLB_OK, tlb.tlb_last_error(s.ctx)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = s.mass()
        assert np.array_equal(got[:3], ref), (got, ref)
        assert got[3] == 0.0


def test_mass_noalloc_rejects_null_and_uninitialised(tlb):
    import torch
    p = W.reduction_case(nx=40, ny=24, R=8.0)
    s = tlb.Solver(40, 24, p["fluid"])
    out = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    assert tlb.lib.tlb_mass_noalloc(s.ctx, C.c_void_p(out.data_ptr())) == tlb.TLB_ESTATE
    assert tlb.lib.tlb_mass_noalloc(s.ctx, None) == tlb.TLB_EINVAL
