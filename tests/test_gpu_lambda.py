"""GPU parity of the bulk energy with lambda > 0 (Eqs. 5-6) against the FP64
oracle, through the C ABI: max-abs <= 1e-12 on every field and population
(FP64), on random three-phase fields in every geometry kind, including
surface tensions with lambda_i <= lambda_T / 2 that only the lambda > 0
energy admits, and the bitwise absence of an absent phase."""
import sys

import numpy as np
import pytest

import oracle
from paper_1710_09534_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_09534_amd import tlb as t
    return t


def _pair(tlb, p, steps, precision="fp64"):
    print("case %s %dx%d steps=%d %s lambda=%g" % (p["name"], p["nx"], p["ny"], steps, precision,
                                                   p["fluid"].get("lambda", 0.0)), flush=True)
    g = tlb.from_problem(p, precision)
    o = oracle.Oracle(p)
    o.init(p["c1"], p["c2"], p["ux"], p["uy"])
    g.step(steps)
    o.step(steps)
    return g, o


def _check(g, o, tol=1e-12):
    fg, fo = g.read_fields(), o.fields()
    d = {k: float(np.abs(fg[k] - fo[k]).max()) for k in fo}
    assert all(v <= tol for v in d.values()), d
    pg, po = g.read_populations(), o.populations()
    po[:, o.material != 0] = 0.0
    assert np.abs(pg - po).max() <= tol


@pytest.mark.parametrize("geometry,nx,ny,lam", [
    ("channel", 100, 37, 2e-3), ("cylinder", 130, 70, 5e-2), ("periodic", 64, 24, 1e-2)])
def test_random_fields_with_lambda(tlb, geometry, nx, ny, lam):
    p = W.random_fields(nx, ny, geometry=geometry, U=0.01 if geometry == "channel" else 0.0,
                        rho=(3.0, 2.0, 1.0))
    p["fluid"] = dict(p["fluid"], **{"lambda": lam})
    g, o = _pair(tlb, p, 300)
    _check(g, o)


def test_lambda_admits_small_lambda_i(tlb):
    """sigma = (1.6, 1.0, 1.0) e-3 gives lambda_3 = lambda_T / 2: rejected
    for lambda = 0, accepted and in parity for lambda > 0."""
    p = W.random_fields(70, 50, geometry="box", sigma=(1.6e-3, 1e-3, 1e-3))
    with pytest.raises(tlb.TlbError) as e:
        tlb.Solver(70, 50, p["fluid"])
    assert e.value.status == tlb.TLB_EPARAM
    p["fluid"] = dict(p["fluid"], **{"lambda": 1e-3})
    g, o = _pair(tlb, p, 300)
    _check(g, o)


def test_absent_phase_bitwise_with_lambda(tlb):
    p = W.reduction_case(nx=64, ny=48, R=12)
    p["fluid"] = dict(p["fluid"], **{"lambda": 0.05})
    g, o = _pair(tlb, p, 500)
    _check(g, o)
    assert np.all(g.read_populations()[9:18] == 0.0)


@pytest.mark.parametrize("precision", ["fp32", "fp16dev"])
def test_lambda_reduced_precision(tlb, precision):
    p = W.random_fields(130, 70, geometry="cylinder", rho=(3.0, 2.0, 1.0))
    p["fluid"] = dict(p["fluid"], **{"lambda": 5e-2})
    g, o = _pair(tlb, p, 1000, precision)
    fg, fo = g.read_fields(), o.fields()
    err = max(float(np.abs(fg[k] - fo[k]).max()) for k in ("c1", "c2", "c3"))
    print("%s lambda: max order-parameter error %.2e" % (precision, err), flush=True)
    assert err <= 1e-4
