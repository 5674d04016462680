"""Edge cases of the 2-D step on the GPU, through the C ABI, against the FP64
oracle:

* the largest lattice each storage precision accepts (a ragged width, the
  last row that keeps every 9-plane family below 2 GiB), stepped in the
  default launch configuration and compared on sampled windows -- around
  walls, drops and triple junctions placed across the periodic corner, on
  the ragged right edge, on the top edge and in the centre -- with cut-out
  oracle runs (tests/sampling.py; the technique is checked on the oracle in
  tests/test_oracle_window.py);
* tiny lattices: 3 x 3, single fluid rows and columns, a second strip column
  holding one node column, a single row of lattice height 3;
* a single phase filling the domain, a fixed point of the method that every
  storage precision must keep exactly;
* zero steps.
Bars: FP64 max-abs <= 1e-12 on every field; FP32 and FP16-dev within 1e-4 on
the order parameters (FP32 also within 1e-6 on the velocity, a few hundred
FP32 roundings of O(1e-2) values over four steps).
"""
import numpy as np
import pytest

import oracle
from paper_1710_09534_amd import workloads as W
from sampling import window_fields

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def tlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_09534_amd import tlb as t
    return t


def _max_rows(nx, elem, hist_elem):
    pitch = -(-nx // 64) * 64
    lim = (1 << 31) - 1
    return min(lim // (9 * pitch * elem), lim // (4 * pitch * hist_elem))


@pytest.mark.parametrize("precision,nx,elem,hist", [
    ("fp64", 5430, 8, 8), ("fp32", 7710, 4, 4), ("fp16dev", 7650, 4, 4)],
    ids=["fp64_5430", "fp32_7710", "fp16dev_7650"])
def test_largest_lattice_sampled(tlb, precision, nx, elem, hist):
    ny = _max_rows(nx, elem, hist)
    steps = 4
    print("case largest %s %dx%d (%.1f M nodes) steps=%d" % (precision, nx, ny, nx * ny / 1e6,
                                                          steps), flush=True)
    assert tlb.tlb_workspace_bytes(nx, ny + 1, tlb.PRECISIONS[precision]) == 0
    p = W.large_lattice(nx, ny)
    g = tlb.from_problem(p, precision)
    g.step(steps)
    names = ("c1", "c2", "ux", "uy") if precision != "fp64" else tlb.FIELDS
    mask = sum(1 << tlb.FIELDS.index(k) for k in names)
    f = g.read_fields(mask)
    g.destroy()
    worst = {}
    for (x0, y0, w, h) in p["features"]:
        wf, ys, xs = window_fields(oracle, p, x0, y0, w, h, 4 * steps + 8, steps)
        for k in names:
            d = float(np.abs(f[k][np.ix_(ys, xs)] - wf[k]).max())
            worst[k] = max(worst.get(k, 0.0), d)
    print("max-abs over the windows:", worst, flush=True)
    if precision == "fp64":
        assert all(v <= TOL64 for v in worst.values()), worst
    else:
        assert worst["c1"] <= 1e-4 and worst["c2"] <= 1e-4, worst
        if precision == "fp32":
            assert worst["ux"] <= 1e-6 and worst["uy"] <= 1e-6, worst


@pytest.mark.parametrize("geometry,nx,ny", [
    ("periodic", 3, 3), ("periodic", 4, 5), ("periodic", 130, 3), ("channel", 5, 3),
    ("channel", 65, 6), ("box", 3, 7), ("box", 7, 4)])
def test_tiny_lattices(tlb, geometry, nx, ny):
    p = W.random_fields(nx, ny, geometry=geometry, U=0.01 if geometry == "channel" else 0.0,
                        rho=(3.0, 2.0, 1.0))
    print("case tiny %s %dx%d steps=200" % (geometry, nx, ny), flush=True)
    g = tlb.from_problem(p)
    o = oracle.Oracle(p)
    o.init(p["c1"], p["c2"], p["ux"], p["uy"])
    g.step(200)
    o.step(200)
    fg, fo = g.read_fields(), o.fields()
    d = {k: float(np.abs(fg[k] - fo[k]).max()) for k in fo}
    assert all(v <= TOL64 for v in d.values()), d
    pg, po = g.read_populations(), o.populations()
    po[:, o.material != 0] = 0.0
    assert np.abs(pg - po).max() <= TOL64


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16dev"])
@pytest.mark.parametrize("phase", [1, 2, 3])
@pytest.mark.parametrize("geometry", ["cylinder", "box"])
def test_single_phase_is_kept_exactly(tlb, precision, phase, geometry):
    """With one phase everywhere at rest, every chemical potential, force,
    velocity and pressure vanishes and the populations are the rest state;
    the wetting ghosts of a pure phase equal the fluid value, so walls of any
    wettability change nothing."""
    p = W.random_fields(130, 70, geometry=geometry)
    fluid = p["material"] == 0
    one = np.where(fluid, 1.0, 0.0)
    zero = np.zeros_like(one)
    p["c1"] = one if phase == 1 else zero
    p["c2"] = one if phase == 2 else zero
    p["ux"] = zero
    p["uy"] = zero
    print("case single phase %d %s %s steps=300" % (phase, geometry, precision), flush=True)
    g = tlb.from_problem(p, precision)
    g.step(300)
    f = g.read_fields()
    for k, i in (("c1", 1), ("c2", 2), ("c3", 3)):
        assert np.array_equal(f[k], one if phase == i else zero), k
    for k in ("ux", "uy", "p", "mu1", "mu2", "mu3"):
        assert not f[k].any(), k


def test_zero_steps_is_a_no_op(tlb):
    p = W.random_fields(100, 37, geometry="channel", U=0.01)
    g = tlb.from_problem(p)
    g.step(5)
    a = g.read_populations()
    n0 = g.step_count
    g.step(0)
    assert g.step_count == n0
    assert np.array_equal(g.read_populations(), a)
    with pytest.raises(tlb.TlbError) as e:
        g.step(-1)
    assert e.value.status == tlb.TLB_EINVAL
