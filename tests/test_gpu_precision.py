"""FP32 and FP16-deviation storage against the FP64 oracle (GPU).

Bars: order parameters within 1e-4 of the oracle after 1000 steps of the
64x64 reduction workload and of a three-phase drop workload; the equilibrium
contact angle of a sessile drop within 0.5 deg of the FP64 result.  The
measured errors per result (c_i, u, p, theta) are printed for the record.
"""
import math

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


def errors(g, ref):
    f = g.read_fields()
    return {k: float(np.abs(f[k] - ref[k]).max()) for k in ref}


@pytest.mark.parametrize("precision", ["fp32", "fp16dev"])
@pytest.mark.parametrize("case", ["reduction", "binary"])
def test_order_parameters_within_1e4(tlb, precision, case):
    if case == "reduction":
        p = W.reduction_case()
    else:
        p = W.binary_drops(seed=2, nx=128, ny=64, R=16)
    o = oracle.Oracle(p)
    o.init(p["c1"], p["c2"], p["ux"], p["uy"])
    o.step(1000)
    ref = o.fields()
    g = tlb.from_problem(p, precision)
    g.step(1000)
    e = errors(g, ref)
    print("%s %s errors after 1000 steps: %s" % (case, precision,
          {k: "%.2e" % v for k, v in e.items()}), flush=True)
    assert e["c1"] <= 1e-4 and e["c2"] <= 1e-4 and e["c3"] <= 1e-4, e
    m0 = o.mass()
    m = g.mass()
    assert np.all(np.abs(m - m0) <= 1e-5 * np.abs(m0) + 1e-9)


def _cap_angle(c, y_wall=0.5):
    ny, nx = c.shape

    def crossings(row):
        xs = []
        for x in range(nx - 1):
            a, b = row[x], row[x + 1]
            if (a - 0.5) * (b - 0.5) < 0:
                xs.append(x + (0.5 - a) / (b - a))
        return xs

    widths = []
    for yy in (1, 2):
        xs = crossings(c[yy])
        widths.append(max(xs) - min(xs))
    Ls = widths[0] + (widths[0] - widths[1]) * (1 - y_wall)
    col = c[:, nx // 2]
    top = None
    for yy in range(1, ny - 1):
        if (col[yy] - 0.5) * (col[yy + 1] - 0.5) < 0:
            top = yy + (0.5 - col[yy]) / (col[yy + 1] - col[yy])
    return math.degrees(2 * math.atan(2 * (top - y_wall) / Ls))


@pytest.mark.parametrize("theta", [60.0, 120.0])
def test_contact_angle_within_half_degree(tlb, theta):
    p = W.reduction_case(nx=96, ny=48, R=14.0, theta13=theta, sigma=(1e-2, 1e-2, 1e-2), noise=0)
    ang = {}
    for prec in ("fp64", "fp32", "fp16dev"):
        g = tlb.from_problem(p, prec)
        g.step(6000)
        ang[prec] = _cap_angle(g.read_fields()["c1"])
    print("contact angle %g: %s" % (theta, {k: "%.3f" % v for k, v in ang.items()}), flush=True)
    assert abs(ang["fp64"] - theta) < 3.0
    assert abs(ang["fp32"] - ang["fp64"]) <= 0.5
    assert abs(ang["fp16dev"] - ang["fp64"]) <= 0.5
