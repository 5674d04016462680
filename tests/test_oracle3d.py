"""Pins of the three-dimensional (D3Q19) oracle to what mathematics and the
paper fix (CPU only).

* D3Q19 weights and links: lattice moments up to fourth order of an
  isotropic lattice with c_s^2 = 1/3 (the property Eq. 20's stencils need).
* For fields that do not vary along z, the D3Q19 gradient and Laplacian
  stencils equal the D2Q9 ones of the independent 2-D oracle (the z-links
  project onto the in-plane weights 4/9, 1/9, 1/36), with and without walls.
* Exactness of the stencils on linear and quadratic fields.
* Per-component mass conservation, an absent phase stays absent, reduction
  consistency, plane Couette flow, and the 3-D Laplace law dp = 2 sigma / R.
"""
import numpy as np
import pytest

import oracle
from paper_1710_09534_amd import workloads as W


def test_d3q19_isotropy():
    ex, ey, ez, w, opp = oracle.lattice3()
    e = np.stack([ex, ey, ez], 1).astype(float)
    cs2 = 1.0 / 3.0
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w @ e, 0.0, atol=1e-16)
    assert np.allclose(np.einsum("k,ka,kb->ab", w, e, e), cs2 * np.eye(3), atol=1e-16)
    assert np.allclose(np.einsum("k,ka,kb,kc->abc", w, e, e, e), 0.0, atol=1e-16)
    d = np.eye(3)
    iso4 = cs2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                       + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(np.einsum("k,ka,kb,kc,kd->abcd", w, e, e, e, e), iso4, atol=1e-16)
    assert np.all(e[opp] == -e)
    assert len(set(map(tuple, e.astype(int)))) == 19


def _plain(nx, ny, nz, mask3, periodic3):
    fl = W.fluid()
    z = np.zeros((nz, ny, nx))
    return W._problem3("st", nx, ny, nz, fl, periodic3, mask3,
                       [W.material(90, 90)] * int(mask3.max()), z, z)


@pytest.mark.parametrize("walls", [False, True])
def test_stencils_reduce_to_d2q9_for_z_invariant_fields(walls):
    nx, ny, nz = 20, 14, 4
    rng = np.random.default_rng(3)
    chi2 = rng.standard_normal((ny, nx))
    mask2 = np.zeros((ny, nx), np.uint8)
    if walls:
        mask2[0, :] = 1
        mask2[ny - 1, :] = 1
        mask2[5:7, 8:11] = 1          # an obstacle with corners
    mask3 = np.repeat(mask2[None], nz, axis=0)
    p3 = _plain(nx, ny, nz, mask3, (1, 0 if walls else 1, 1))
    o3 = oracle.Oracle3D(p3)
    z2 = np.zeros((ny, nx))
    p2 = W._problem("st2", nx, ny, W.fluid(), (1, 0 if walls else 1), mask2,
                    [W.material(90, 90)] if walls else [], z2, z2)
    o2 = oracle.Oracle(p2)
    chi3 = np.repeat(chi2[None], nz, axis=0)
    g3 = o3.grad(chi3)
    l3 = o3.lap(chi3)
    g2x, g2y = o2.grad(chi2)
    l2 = o2.lap(chi2)
    for zz in range(nz):
        assert np.abs(g3[0][zz] - g2x).max() < 1e-13
        assert np.abs(g3[1][zz] - g2y).max() < 1e-13
        assert np.abs(g3[2][zz]).max() < 1e-13
        assert np.abs(l3[zz] - l2).max() < 1e-13


def test_stencils_exact_on_polynomials():
    n = 12
    p3 = _plain(n, n, n, np.zeros((n, n, n), np.uint8), (1, 1, 1))
    o3 = oracle.Oracle3D(p3)
    x, y, z = W.coords3(n, n, n)
    lin = 0.3 * x - 0.7 * y + 1.1 * z
    gx, gy, gz = o3.grad(lin)
    inner = (slice(2, n - 2),) * 3
    assert np.allclose(gx[inner], 0.3) and np.allclose(gy[inner], -0.7) and np.allclose(gz[inner], 1.1)
    quad = x ** 2 + 2 * y ** 2 - 0.5 * z ** 2 + x * y
    assert np.allclose(o3.lap(quad)[inner], 2 + 4 - 1, atol=1e-11)


def _run(p, steps):
    s = oracle.Oracle3D(p)
    s.init(p["c1"], p["c2"], p["ux"], p["uy"], p["uz"])
    if steps:
        s.step(steps)
    return s


@pytest.mark.parametrize("geometry", ["channel", "sphere", "box"])
def test_mass_conserved_3d(geometry):
    p = W.random_fields3(20, 16, 14, geometry=geometry, U=0.01, rho=(3.0, 2.0, 1.0))
    s = _run(p, 0)
    m0 = s.mass()
    s.step(150)
    m1 = s.mass()
    assert np.all(np.abs(m1 - m0) <= 1e-12 * np.abs(m0))


def test_absent_phase_stays_zero_3d():
    p = W.sessile3d(nx=24, ny=24, nz=14, R_core=5.0, R_shell=9.0)
    p["c1"] = p["c1"] + p["c2"]
    p["c2"] = np.zeros_like(p["c2"])
    s = _run(p, 150)
    assert np.all(s.populations()[19:38] == 0.0)


def test_reduction_consistency_3d():
    a = W.sessile3d(nx=24, ny=24, nz=14, R_core=5.0, R_shell=9.0)
    a["c1"] = a["c1"] + a["c2"]
    a["c2"] = np.zeros_like(a["c2"])
    b = dict(a)
    b["fluid"] = dict(a["fluid"], sigma12=1.5e-3, sigma23=1.2e-3)
    b["mats"] = [W.material(60.0, 70.0), a["mats"][1]]
    fa, fb = _run(a, 150).fields(), _run(b, 150).fields()
    assert np.abs(fa["c1"] - fb["c1"]).max() < 1e-12


def test_couette_3d():
    """Walls in z = 0 and nz-1 moving at -U and +U along x: exact linear
    profile through -U at z = 1/2 and +U at z = nz - 3/2."""
    nx, ny, nz, U = 4, 4, 12, 0.01
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[0], mask[nz - 1] = 1, 2
    z0 = np.zeros((nz, ny, nx))
    fl = W.fluid(nu=(1 / 6,) * 3, tau=(1.0, 1.0))
    p = W._problem3("couette3", nx, ny, nz, fl, (1, 1, 0), mask,
                    [W.material(90, 90, (-U, 0)), W.material(90, 90, (U, 0))], z0, z0)
    f = _run(p, 4000).fields()
    z = np.arange(1, nz - 1)
    exact = -U + 2 * U * (z - 0.5) / (nz - 2)
    assert np.abs(f["ux"][1:-1] - exact[:, None, None]).max() < 1e-10 * U / U
    assert np.abs(f["uy"]).max() < 1e-15 and np.abs(f["uz"]).max() < 1e-15


def test_laplace_law_3d():
    """A spherical drop of phase 1 in phase 3: p_in - p_out = 2 sigma / R
    within 4 % (R = 8, D = 4)."""
    n, R, sigma = 32, 8.0, 1e-3
    c1 = W.tanh_ball(n, n, n, n / 2, n / 2, n / 2, R, 4.0)
    fl = W.fluid(sigma=(sigma,) * 3, M0=1e-4)
    p = W._problem3("laplace3", n, n, n, fl, (1, 1, 1), np.zeros((n, n, n), np.uint8), [], c1,
                    np.zeros_like(c1))
    f = _run(p, 1500).fields()
    x, y, z = W.coords3(n, n, n)
    r = np.sqrt((x - n / 2) ** 2 + (y - n / 2) ** 2 + (z - n / 2) ** 2)
    dp = f["p"][r < R - 4].mean() - f["p"][r > R + 6].mean()
    assert abs(dp - 2 * sigma / R) <= 0.04 * 2 * sigma / R, dp


def test_validation_3d():
    p = W.random_fields3(12, 10, 8, geometry="channel")
    with pytest.raises(ValueError):                     # open z edge with fluid
        oracle.Oracle3D(dict(p, periodic=(1, 1, 1), material=np.zeros((8, 10, 12), np.uint8),
                             mats=[]) | {"periodic": (1, 1, 0)})
    with pytest.raises(ValueError):                     # velocity boundaries are 2-D only
        oracle.Oracle3D(dict(p, mats=[W.velocity_boundary((0.01, 0.0)), p["mats"][1]]))


def test_mass_conserved_between_static_obstacles_3d():
    """Scattered static obstacles of five materials (voxels, cubes, bars along
    every axis, plates, diagonal staircases, touching and wrapping): both
    order-parameter totals kept to rounding over 100 steps (half-way
    bounce-back returns every population sent towards a wall, Eq. 44)."""
    p = W.random_obstacles3(30, 24, 20, seed=21, n_obstacles=25, moving=False)
    assert len(set(p["material"].ravel().tolist())) == 6
    s = _run(p, 0)
    m0 = s.mass()
    s.step(100)
    m1 = s.mass()
    assert np.isfinite(s.fields()["ux"]).all()
    assert np.all(np.abs(m1[:2] - m0[:2]) <= 1e-9 * np.abs(m0[:2])), (m0, m1)
