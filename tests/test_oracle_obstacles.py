"""Oracle pin on scattered obstacles (CPU): with static walls of six wetting
materials in every shape the obstacle generator makes (single nodes, blocks,
one-node-thick bars, L shapes, diagonal staircases touching each other and the
periodic seams), half-way bounce-back (Eq. 44) returns every population that
leaves a fluid node towards a wall to that node, and the collision (Eq. 45)
conserves sum_k f^i_k, so the total of each order parameter over the fluid
stays fixed.  A wrong opposite direction, a missed link or a store into the
wrong slot at any corner changes it.  The pin also requires the wetting ghosts
(Eq. 42) to keep the run finite.
"""
import numpy as np

import oracle
from paper_1710_09534_amd import workloads as W


def test_mass_is_conserved_between_static_obstacles():
    p = W.random_obstacles(96, 64, seed=5, n_obstacles=30, moving=False)
    assert len(set(p["material"].ravel().tolist())) == 7   # fluid and six materials
    o = oracle.Oracle(p)
    o.init(p["c1"], p["c2"], p["ux"], p["uy"])
    m0 = o.mass()
    o.step(300)
    m1 = o.mass()
    f = o.fields()
    assert np.isfinite(f["c1"]).all() and np.isfinite(f["ux"]).all()
    # the total of c1 and c2 (about 2e3 each) kept to rounding over 300 steps
    assert abs(m1[0] - m0[0]) <= 1e-9 * abs(m0[0]), (m0, m1)
    assert abs(m1[1] - m0[1]) <= 1e-9 * abs(m0[1]), (m0, m1)
    # the fields moved: the pin is not a run that did nothing
    assert np.abs(f["c1"] - np.where(p["material"] != 0, 0.0, p["c1"])).max() > 1e-4


def test_moving_obstacles_change_the_flow_only_through_the_wall_term():
    """The same geometry with every other material moving: the run stays
    finite, and it differs from the static one (the moving-wall term of the
    bounce-back acts)."""
    ps = W.random_obstacles(64, 48, seed=6, n_obstacles=20, moving=False)
    pm = W.random_obstacles(64, 48, seed=6, n_obstacles=20, moving=True)
    assert np.array_equal(ps["material"], pm["material"])
    out = []
    for p in (ps, pm):
        o = oracle.Oracle(p)
        o.init(p["c1"], p["c2"], p["ux"], p["uy"])
        o.step(100)
        out.append(o.fields())
    assert all(np.isfinite(f["ux"]).all() for f in out)
    assert np.abs(out[0]["ux"] - out[1]["ux"]).max() > 1e-5
