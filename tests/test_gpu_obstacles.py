"""GPU parity on scattered obstacles of six wetting materials, half of them
moving (single nodes, blocks, one-node-thick bars, L shapes and diagonal
staircases, touching each other, wrapping across the periodic seams and
crossing strip boundaries): every wall path of the step (wetting ghosts of
Eq. 42 across each link kind, the symmetric ghosts of Eq. 43, bounce-back of
Eq. 44 with the moving-wall term into neighbours of every direction) against
the FP64 oracle.  FP64: every field and population within 1e-12 after 300
steps, at the default strip height and at 8-row strips; FP32 and FP16-dev:
order parameters within 1e-4.
"""
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


@pytest.fixture(scope="module")
def case():
    p = W.random_obstacles(150, 90, seed=3, n_obstacles=40)
    o = oracle.Oracle(p)
    o.init(p["c1"], p["c2"], p["ux"], p["uy"])
    o.step(300)
    po = o.populations()
    po[:, o.material != 0] = 0.0
    return p, o.fields(), po


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("rows", [None, 8])
def test_obstacles_fp64(tlb, case, rows):
    p, fo, po = case
    _say("case %s fp64 300 steps rows=%s" % (p["name"], rows))
    g = tlb.from_problem(p, "fp64")
    if rows:
        g.set_tile_rows(rows)
    g.step(300)
    fg = g.read_fields()
    e = {k: float(np.abs(fg[k] - fo[k]).max()) for k in fo}
    _say("obstacles fp64 rows=%s: %s" % (rows, {k: "%.1e" % v for k, v in e.items()}))
    assert max(e.values()) <= 1e-12, e
    assert np.abs(g.read_populations() - po).max() <= 1e-12


@pytest.mark.parametrize("precision", ["fp32", "fp16dev"])
def test_obstacles_reduced_precision(tlb, case, precision):
    p, fo, _ = case
    _say("case %s %s 300 steps" % (p["name"], precision))
    g = tlb.from_problem(p, precision)
    g.step(300)
    fg = g.read_fields()
    e = {k: float(np.abs(fg[k] - fo[k]).max()) for k in fo}
    _say("obstacles %s: %s" % (precision, {k: "%.1e" % v for k, v in e.items()}))
    assert e["c1"] <= 1e-4 and e["c2"] <= 1e-4 and e["c3"] <= 1e-4, e
