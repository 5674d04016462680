"""Sampled parity on lattices too large for the whole-lattice oracle.

A node's state after s steps depends only on the initial state within a
finite distance of it (every stencil of the step has a bounded reach), so the
oracle run on a periodic cut-out of the lattice reproduces the whole-lattice
result exactly in the cut-out's interior, once the cut-out's margin exceeds
s times the per-step reach plus the reach of the initialisation.
`tests/test_oracle_window.py` checks that claim on the oracle itself,
whole lattice against cut-outs.
"""
import numpy as np


def window(p, x0, y0, w, h, margin):
    """Cut-out of the fully periodic problem ``p``: the box of w x h nodes at
    (x0, y0) plus ``margin`` nodes on every side, taken with periodic wrap and
    made periodic itself.  Returns (sub-problem, row indices, column indices)
    of the box's nodes in ``p``."""
    assert tuple(p["periodic"]) == (1, 1), "cut-outs need a fully periodic lattice"
    nx, ny = p["nx"], p["ny"]
    xs = np.arange(x0 - margin, x0 + w + margin) % nx
    ys = np.arange(y0 - margin, y0 + h + margin) % ny
    box = np.ix_(ys, xs)

    def cut(a):
        return None if a is None else np.ascontiguousarray(a[box])

    sub = {"name": "%s_win_%d_%d" % (p["name"], x0, y0), "nx": w + 2 * margin,
           "ny": h + 2 * margin, "fluid": p["fluid"], "periodic": (1, 1),
           "material": cut(p["material"]), "mats": p["mats"],
           "c1": cut(p["c1"]), "c2": cut(p["c2"]), "ux": cut(p.get("ux")), "uy": cut(p.get("uy"))}
    return sub, ys[margin:margin + h], xs[margin:margin + w]


def window_fields(oracle_mod, p, x0, y0, w, h, margin, steps):
    """Oracle fields of the box after ``steps`` steps, from a cut-out run.
    Returns (fields of the box, row indices, column indices)."""
    sub, ys, xs = window(p, x0, y0, w, h, margin)
    o = oracle_mod.Oracle(sub)
    o.init(sub["c1"], sub["c2"], sub["ux"], sub["uy"])
    if steps:
        o.step(steps)
    f = o.fields()
    core = (slice(margin, margin + h), slice(margin, margin + w))
    return {k: v[core] for k, v in f.items()}, ys, xs


def window3(p, x0, y0, z0, w, h, d, margin):
    """The 3-D cut-out of the fully periodic problem ``p`` (as `window`).
    Returns (sub-problem, z, y, x indices of the box's nodes in ``p``)."""
    assert tuple(p["periodic"]) == (1, 1, 1), "cut-outs need a fully periodic lattice"
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    xs = np.arange(x0 - margin, x0 + w + margin) % nx
    ys = np.arange(y0 - margin, y0 + h + margin) % ny
    zs = np.arange(z0 - margin, z0 + d + margin) % nz
    box = np.ix_(zs, ys, xs)

    def cut(a):
        return None if a is None else np.ascontiguousarray(a[box])

    sub = {"name": "%s_win" % p["name"], "nx": w + 2 * margin, "ny": h + 2 * margin,
           "nz": d + 2 * margin, "fluid": p["fluid"], "periodic": (1, 1, 1),
           "material": cut(p["material"]), "mats": p["mats"], "c1": cut(p["c1"]),
           "c2": cut(p["c2"]), "ux": cut(p.get("ux")), "uy": cut(p.get("uy")),
           "uz": cut(p.get("uz"))}
    m = margin
    return sub, zs[m:m + d], ys[m:m + h], xs[m:m + w]


def window_fields3(oracle_mod, p, box, margin, steps):
    """3-D oracle fields of box = (x0, y0, z0, w, h, d) after ``steps`` steps
    from a cut-out run: (fields of the box, z, y, x indices)."""
    x0, y0, z0, w, h, d = box
    sub, zs, ys, xs = window3(p, x0, y0, z0, w, h, d, margin)
    o = oracle_mod.Oracle3D(sub)
    o.init(sub["c1"], sub["c2"], sub["ux"], sub["uy"], sub["uz"])
    if steps:
        o.step(steps)
    f = o.fields()
    core = (slice(margin, margin + d), slice(margin, margin + h), slice(margin, margin + w))
    return {k: v[core] for k, v in f.items()}, zs, ys, xs
