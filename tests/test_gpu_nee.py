"""GPU parity of the velocity boundary (non-equilibrium extrapolation,
Sec. III.D, Eqs. 51-53) against the FP64 oracle, through the C ABI.

Bar: FP64 max-abs <= 1e-12 on every field and population; FP32 and FP16-dev
order parameters within 1e-4 of the oracle.  Cases: the compound-drop shear
of Sec. III.D (reduced and at its 400 x 150 size), random three-phase fields
with a velocity boundary on top, on the bottom and on both sides (density
contrast, gravity, tangential and normal boundary velocity), ragged sizes
that span several 64-column strips, and the exact Couette profile.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1710_09534_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def tlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_09534_amd import tlb as t
    return t


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(tlb, p, steps, precision="fp64", rows=None):
    _say("case %s %dx%d steps=%d %s" % (p["name"], p["nx"], p["ny"], steps, precision))
    g = tlb.from_problem(p, precision)
    if rows:
        g.set_tile_rows(rows)
    o = oracle.Oracle(p)
    o.init(p["c1"], p["c2"], p["ux"], p["uy"])
    if steps:
        g.step(steps)
        o.step(steps)
    return g, o


def _check(g, o, tol=TOL64, pops=True):
    fg, fo = g.read_fields(), o.fields()
    d = {k: float(np.abs(fg[k] - fo[k]).max()) for k in fo}
    assert all(v <= tol for v in d.values()), d
    if pops:
        pg, po = g.read_populations(), o.populations()
        po[:, o.material != 0] = 0.0
        assert np.abs(pg - po).max() <= tol


def _random_with_velocity(nx, ny, top=True, bottom=False, u_top=(0.02, 0.0),
                          u_bot=(-0.01, 0.0), seed=7):
    p = W.random_fields(nx, ny, geometry="channel", U=0.01, rho=(3.0, 2.0, 1.0),
                        gravity=(0.0, -1e-6), seed=seed)
    mats = list(p["mats"])
    if bottom:
        mats[0] = W.velocity_boundary(u_bot)
    if top:
        mats[1] = W.velocity_boundary(u_top)
    p = dict(p, mats=mats, name=p["name"] + ("_vtop" if top else "") + ("_vbot" if bottom else ""))
    return p


def test_shear_small_fp64(tlb):
    p = W.nee_shear(nx=128, ny=64, U0=0.05, R_core=8.0, R_shell=18.0, offset=3.0)
    g, o = _pair(tlb, p, 600)
    _check(g, o)


def test_shear_full_size_fp64(tlb):
    """The 400 x 150 shear setup of Sec. III.D (U0 = 0.1), 1000 steps, every
    field and population."""
    p = W.nee_shear()
    g, o = _pair(tlb, p, 1000)
    _check(g, o)


@pytest.mark.parametrize("nx,ny,top,bottom,u_top", [
    (100, 37, True, False, (0.02, 0.0)),
    (130, 20, False, True, (0.0, 0.0)),
    (70, 9, True, True, (0.02, 0.005)),
    (64, 4, True, True, (0.01, 0.0)),
])
def test_random_fields_with_velocity_boundaries(tlb, nx, ny, top, bottom, u_top):
    p = _random_with_velocity(nx, ny, top=top, bottom=bottom, u_top=u_top)
    g, o = _pair(tlb, p, 300)
    _check(g, o)


@pytest.mark.parametrize("rows", [8, 20])
def test_strip_height_invariance_with_velocity_boundary(tlb, rows):
    p = _random_with_velocity(100, 37, top=True, bottom=True)
    a, _ = _pair(tlb, p, 60)
    b = tlb.from_problem(p)
    b.set_tile_rows(rows)
    b.step(60)
    assert np.array_equal(a.read_populations(), b.read_populations())


@pytest.mark.parametrize("precision", ["fp32", "fp16dev"])
def test_shear_reduced_precision(tlb, precision):
    p = W.nee_shear(nx=128, ny=64, U0=0.05, R_core=8.0, R_shell=18.0, offset=3.0)
    g, o = _pair(tlb, p, 1000, precision=precision)
    fg, fo = g.read_fields(), o.fields()
    err = {k: float(np.abs(fg[k] - fo[k]).max()) for k in ("c1", "c2", "c3", "ux", "uy")}
    _say("%s errors after 1000 steps: %s" % (precision, {k: "%.2e" % v for k, v in err.items()}))
    assert max(err["c1"], err["c2"], err["c3"]) <= 1e-4


def test_couette_exact_on_gpu(tlb):
    nx, ny, U = 64, 12, 0.01
    mask = np.zeros((ny, nx), np.uint8)
    mask[0, :] = 1
    mask[ny - 1, :] = 2
    fl = W.fluid(tau=(0.8, 0.8), nu=(0.1, 0.1, 0.1))
    z = np.zeros((ny, nx))
    p = W._problem("couette_nee", nx, ny, fl, (1, 0), mask,
                   [W.material(90, 90), W.velocity_boundary((U, 0.0))], z, z)
    g = tlb.from_problem(p)
    g.step(8000)
    f = g.read_fields()
    y = np.arange(1, ny - 1)
    exact = U * (y - 0.5) / (ny - 1.5)
    assert np.abs(f["ux"][1:-1, :] - exact[:, None]).max() < 1e-12 * U


def test_velocity_boundary_rejections(tlb):
    p = W.nee_shear(nx=64, ny=32, U0=0.02, R_core=4.0, R_shell=9.0, offset=2.0)
    s = tlb.Solver(64, 32, p["fluid"])
    with pytest.raises(tlb.TlbError) as e:        # periodic in y
        s.set_geometry(p["material"], p["mats"], (1, 1))
    assert e.value.status == tlb.TLB_EINVAL
    m = p["material"].copy()
    m[10, 10] = 2                                 # velocity node off the edge rows
    with pytest.raises(tlb.TlbError) as e:
        s.set_geometry(m, p["mats"], (1, 0))
    assert e.value.status == tlb.TLB_EINVAL
    m = p["material"].copy()
    m[30, 5] = 1                                  # solid node inside a velocity node
    with pytest.raises(tlb.TlbError) as e:
        s.set_geometry(m, p["mats"], (1, 0))
    assert e.value.status == tlb.TLB_EINVAL
    bad = [dict(p["mats"][0]), dict(p["mats"][1], kind=7)]
    with pytest.raises(tlb.TlbError) as e:
        s.set_geometry(p["material"], bad, (1, 0))
    assert e.value.status == tlb.TLB_EINVAL
    th = s.set_geometry(p["material"], p["mats"], (1, 0))
    assert abs(th[0] - 30.0) < 0.01 and np.isnan(th[1])
