"""The cut-out technique of tests/sampling.py, checked on the oracle: after s
steps a cut-out with margin 4 s + 8 reproduces the whole-lattice oracle
bitwise on its box (every field), and a margin below the step's reach does
not, so the check can fail.  This is what licenses comparing the GPU on the
largest lattices against cut-out oracle runs."""
import numpy as np
import pytest

import oracle
from paper_1710_09534_amd import workloads as W
from sampling import window_fields


def margin_for(steps):
    return 4 * steps + 8


@pytest.fixture(scope="module")
def case():
    p = W.large_lattice(230, 196, seed=3)
    runs = {}
    for s in (0, 4):
        o = oracle.Oracle(p)
        o.init(p["c1"], p["c2"], p["ux"], p["uy"])
        if s:
            o.step(s)
        runs[s] = o.fields()
    return p, runs


@pytest.mark.parametrize("steps", [0, 4])
def test_cutout_reproduces_whole_lattice(case, steps):
    p, runs = case
    full = runs[steps]
    for (x0, y0, w, h) in p["features"]:
        wf, ys, xs = window_fields(oracle, p, x0, y0, min(w, 64), min(h, 64),
                                   margin_for(steps), steps)
        for k in full:
            assert np.array_equal(wf[k], full[k][np.ix_(ys, xs)]), (k, x0, y0)


def test_too_small_margin_is_detected(case):
    p, runs = case
    x0, y0, w, h = p["features"][3]
    wf, ys, xs = window_fields(oracle, p, x0, y0, 48, 48, 1, 4)
    diff = max(float(np.abs(wf[k] - runs[4][k][np.ix_(ys, xs)]).max()) for k in wf)
    assert diff > 1e-9


def test_features_cover_walls_and_both_drops(case):
    p, _ = case
    for (x0, y0, w, h) in p["features"]:
        ys = np.arange(y0, y0 + h) % p["ny"]
        xs = np.arange(x0, x0 + w) % p["nx"]
        m = p["material"][np.ix_(ys, xs)]
        assert (m != 0).any() and (m == 0).any()
        assert p["c1"][np.ix_(ys, xs)].max() > 0.9 and p["c2"][np.ix_(ys, xs)].max() > 0.9


def test_cutout_reproduces_whole_lattice_3d():
    """The same technique on the D3Q19 oracle: after 2 steps, cut-outs with
    margin 4 s + 8 match the whole lattice bitwise on every field; a 1-node
    margin does not."""
    from sampling import window_fields3
    p = W.large_lattice3(70, 60, 64, seed=2)
    o = oracle.Oracle3D(p)
    o.init(p["c1"], p["c2"], p["ux"], p["uy"], p["uz"])
    o.step(2)
    full = o.fields()
    for b in p["features"]:
        b = b[:3] + tuple(min(v, 24) for v in b[3:])
        wf, zs, ys, xs = window_fields3(oracle, p, b, margin_for(2), 2)
        for k in full:
            assert np.array_equal(wf[k], full[k][np.ix_(zs, ys, xs)]), (k, b)
    wf, zs, ys, xs = window_fields3(oracle, p, b, 1, 2)
    assert max(float(np.abs(wf[k] - full[k][np.ix_(zs, ys, xs)]).max()) for k in wf) > 1e-9
