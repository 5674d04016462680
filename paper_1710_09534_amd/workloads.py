"""Seeded synthetic inputs for the ternary wetting lattice Boltzmann solver.

This module builds the *inputs* of a solve -- grid, solid geometry, contact
angles, fluid properties and initial order-parameter / velocity fields -- for
the paper's workload shapes.  It contains none of the method's arithmetic and
is the only module shared by the GPU path and the FP64 oracle.

Initial profiles follow the smooth tanh drop of the paper's set-ups (Sec. III,
Eqs. 46, 50, 56), read as c = 1/2 + 1/2 tanh(2 (R - r) / D) with r the
Euclidean distance to the drop centre; a compound drop takes
c_core = profile(R_core) and c_shell = profile(R_shell) - c_core (Eq. 56).
Flat walls are the solid rows 0 and ny-1; a wall surface lies half a link
from the first fluid row (Sec. II.B), so a drop "centred on the bottom wall"
has y_c = 0.5.

Random numbers come from SplitMix64 (Steele, Lea & Flood 2014), implemented
here so that both solvers receive identical arrays.
"""
from __future__ import annotations

import math

import numpy as np

_MASK = (1 << 64) - 1


def splitmix64(seed: int, n: int) -> np.ndarray:
    """First n outputs of SplitMix64 started from ``seed`` (uint64 array)."""
    out = np.empty(n, dtype=np.uint64)
    s = seed & _MASK
    for i in range(n):
        s = (s + 0x9E3779B97F4A7C15) & _MASK
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        out[i] = z ^ (z >> 31)
    return out


def uniform(seed: int, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """n doubles in [lo, hi) from the top 53 bits of SplitMix64 outputs."""
    u = (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    return lo + (hi - lo) * u


class Rng:
    """Sequential scalar draws from one SplitMix64 stream."""

    def __init__(self, seed: int):
        self.s = seed & _MASK

    def next_u64(self) -> int:
        self.s = (self.s + 0x9E3779B97F4A7C15) & _MASK
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))

    def choice(self, n: int) -> int:
        return int(self.uniform() * n) % n


# ----------------------------------------------------------------- geometry
def coords(nx: int, ny: int):
    y, x = np.mgrid[0:ny, 0:nx]
    return x.astype(np.float64), y.astype(np.float64)


def tanh_drop(nx, ny, xc, yc, R, D):
    """Smooth disc indicator 1/2 + 1/2 tanh(2 (R - r) / D)."""
    x, y = coords(nx, ny)
    r = np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
    return 0.5 + 0.5 * np.tanh(2.0 * (R - r) / D)


def channel_mask(nx, ny, bottom=1, top=2):
    """Solid rows 0 (material ``bottom``) and ny-1 (material ``top``)."""
    m = np.zeros((ny, nx), dtype=np.uint8)
    m[0, :] = bottom
    m[ny - 1, :] = top
    return m


def cylinder_mask(nx, ny, xc, yc, R, material=1):
    x, y = coords(nx, ny)
    m = np.zeros((ny, nx), dtype=np.uint8)
    m[(x - xc) ** 2 + (y - yc) ** 2 <= R * R] = material
    return m


def fluid(sigma=(1e-3, 1e-3, 1e-3), D=4.0, M0=1e-4, tau=(0.8, 0.8), rho=(1.0, 1.0, 1.0),
          nu=(0.1, 0.1, 0.1), gravity=(0.0, 0.0), lam=0.0) -> dict:
    return {"sigma12": float(sigma[0]), "sigma13": float(sigma[1]), "sigma23": float(sigma[2]),
            "D": float(D), "M0": float(M0), "tau1": float(tau[0]), "tau2": float(tau[1]),
            "rho": [float(r) for r in rho], "nu": [float(v) for v in nu],
            "gravity": [float(g) for g in gravity], "lambda": float(lam)}


WALL, VELOCITY = 0, 1     # material kinds


def material(theta13, theta23, wall_u=(0.0, 0.0)) -> dict:
    """A solid wall with contact angles theta13, theta23 (degrees) moving
    tangentially at wall_u."""
    return {"theta13": float(theta13), "theta23": float(theta23),
            "wall_u": [float(wall_u[0]), float(wall_u[1])], "kind": WALL}


def velocity_boundary(u) -> dict:
    """A row of velocity boundary nodes with prescribed velocity u (the
    non-equilibrium extrapolation boundary of Sec. III.D)."""
    return {"theta13": 90.0, "theta23": 90.0, "wall_u": [float(u[0]), float(u[1])],
            "kind": VELOCITY}


def admissible(sigma12, sigma13, sigma23, theta13=None, theta23=None) -> bool:
    """Acceptance rule of the sampled inputs: the surface tensions must give
    lambda_i > 0 and lambda_i > lambda_T / 2 (the admissible range stated with
    Eq. 7), and the prescribed angles must give |cos theta12| <= 1 (Eq. 39)."""
    lam = (sigma12 + sigma13 - sigma23, sigma12 + sigma23 - sigma13,
           sigma13 + sigma23 - sigma12)
    if min(lam) <= 0:
        return False
    lam_t = 3.0 / sum(1.0 / v for v in lam)
    if min(lam) <= 0.5 * lam_t:
        return False
    if theta13 is not None:
        c = (sigma13 * math.cos(math.radians(theta13))
             - sigma23 * math.cos(math.radians(theta23))) / sigma12
        if abs(c) > 1.0:
            return False
    return True


def sample_sigma(rng: Rng, lo=5e-4, hi=2e-3, theta13=None, theta23=None, max_draws=100000):
    draws = 0
    while True:
        draws += 1
        s = (rng.uniform(lo, hi), rng.uniform(lo, hi), rng.uniform(lo, hi))
        if admissible(*s, theta13=theta13, theta23=theta23):
            return s, draws
        if draws > max_draws:
            raise RuntimeError("no admissible surface tensions")


def _problem(name, nx, ny, fl, periodic, mask, mats, c1, c2, ux=None, uy=None, steps=0,
             **extra):
    solid = mask != 0
    c1 = np.where(solid, 0.0, c1)
    c2 = np.where(solid, 0.0, c2)
    p = {"name": name, "nx": nx, "ny": ny, "fluid": fl, "periodic": periodic,
         "material": np.ascontiguousarray(mask, dtype=np.uint8), "mats": mats,
         "c1": np.ascontiguousarray(c1), "c2": np.ascontiguousarray(c2),
         "ux": None if ux is None else np.ascontiguousarray(np.where(solid, 0.0, ux)),
         "uy": None if uy is None else np.ascontiguousarray(np.where(solid, 0.0, uy)),
         "steps": steps}
    p.update(extra)
    return p


# ------------------------------------------------------------------ configs
def reduction_case(nx=64, ny=64, R=16.0, theta13=60.0, sigma=(1e-3, 1e-3, 1e-3), seed=1,
                   noise=1e-6, steps=2000, theta23=90.0):
    """Semicircular phase-1 drop on the bottom wall of a channel, phase 2
    absent (64x64, R = 16, 60 deg, sigma = 1e-3, noise 1e-6 on c1)."""
    D = 4.0
    mask = channel_mask(nx, ny)
    mats = [material(theta13, theta23), material(90.0, 90.0)]
    c1 = tanh_drop(nx, ny, nx / 2.0, 0.5, R, D)
    if noise:
        c1 = c1 + uniform(seed, nx * ny, -noise, noise).reshape(ny, nx)
    c2 = np.zeros((ny, nx))
    fl = fluid(sigma=sigma, D=D, M0=0.1 * sigma[1], tau=(0.8, 0.8), rho=(1, 1, 1),
               nu=(0.1, 0.1, 0.1))
    return _problem("reduction_%dx%d" % (nx, ny), nx, ny, fl, (1, 0), mask, mats, c1, c2,
                    steps=steps, R=R, theta=theta13)


def binary_drops(seed=0, nx=256, ny=128, R=24.0, steps=20000):
    """Adjacent phase-1 and phase-2 semicircles (R = 24) touching at x = nx/2
    on the bottom wall; sigma_ij ~ U[5e-4, 2e-3] (admissible draws);
    theta13 = 60, theta23 = 120; densities 10/5/1."""
    D = 4.0
    rng = Rng(seed)
    th13, th23 = 60.0, 120.0
    sig, draws = sample_sigma(rng, theta13=th13, theta23=th23)
    mask = channel_mask(nx, ny)
    mats = [material(th13, th23), material(90.0, 90.0)]
    c1 = tanh_drop(nx, ny, nx / 2.0 - R, 0.5, R, D)
    c2 = tanh_drop(nx, ny, nx / 2.0 + R, 0.5, R, D)
    s = np.minimum(c1 + c2, 1.0)
    over = (c1 + c2) > 1.0
    c2 = np.where(over, s - c1, c2)
    fl = fluid(sigma=sig, D=D, M0=0.1 * (sum(sig) / 3.0), tau=(0.8, 0.8), rho=(10, 5, 1),
               nu=(0.1, 0.1, 0.1))
    return _problem("binary_drops_%dx%d_s%d" % (nx, ny, seed), nx, ny, fl, (1, 0), mask, mats,
                    c1, c2, steps=steps, sigma_draws=draws, R=R)


def compound_shear(seed=0, nx=512, ny=256, U=0.01, R_core=20.0, R_shell=40.0, steps=50000):
    """Phase-2 core inside a phase-1 shell resting on the bottom wall; walls
    move at -U (bottom) and +U (top); theta13 ~ U[45, 135], theta23 = 90;
    equal sigma from Ca = rho nu (2U/(ny-2)) R_shell / sigma, Ca ~ U[0.1, 0.3]."""
    D = 4.0
    rng = Rng(seed)
    while True:
        th13 = rng.uniform(45.0, 135.0)
        ca = rng.uniform(0.1, 0.3)
        rho, nu = 1.0, 0.1
        gdot = 2.0 * U / (ny - 2)
        sig = rho * nu * gdot * R_shell / ca
        if admissible(sig, sig, sig, theta13=th13, theta23=90.0):
            break
    mask = channel_mask(nx, ny)
    mats = [material(th13, 90.0, wall_u=(-U, 0.0)), material(90.0, 90.0, wall_u=(U, 0.0))]
    yc = 0.5 + R_shell
    core = tanh_drop(nx, ny, nx / 2.0, yc, R_core, D)
    shell = tanh_drop(nx, ny, nx / 2.0, yc, R_shell, D) - core
    fl = fluid(sigma=(sig, sig, sig), D=D, M0=0.1 * sig, tau=(0.8, 0.8), rho=(1, 1, 1),
               nu=(nu, nu, nu))
    return _problem("compound_shear_%dx%d_s%d" % (nx, ny, seed), nx, ny, fl, (1, 0), mask,
                    mats, shell, core, steps=steps, theta13=th13, Ca=ca, U=U)


def nee_shear(nx=400, ny=150, U0=0.1, R_core=25.5, R_shell=60.0, offset=7.5,
              sigma=0.01, M0=1e-3, steps=30000):
    """Compound drop sheared by a velocity boundary (Sec. III.D): periodic in x,
    a wetting wall in row 0 (theta12 = 30, theta13 = 68.53, theta23 = 120),
    velocity boundary nodes moving at (U0, 0) in the top row.  Phase-2 drop
    of radius R_shell with a phase-1 core of radius R_core, both centred on
    the wall surface y = 1/2, the core shifted by `offset` along x.
    sigma = 0.01 for every pair, tau = 0.8, M0 = 1e-3, unit densities."""
    D = 4.0
    xs = 0.5 * nx - 0.5 * offset
    core = tanh_drop(nx, ny, xs + offset, 0.5, R_core, D)
    shell = tanh_drop(nx, ny, xs, 0.5, R_shell, D) - core
    mask = np.zeros((ny, nx), dtype=np.uint8)
    mask[0, :] = 1
    mask[ny - 1, :] = 2
    core[mask != 0] = 0.0
    shell[mask != 0] = 0.0
    mats = [material(68.53, 120.0), velocity_boundary((U0, 0.0))]
    fl = fluid(sigma=(sigma, sigma, sigma), D=D, M0=M0, tau=(0.8, 0.8), rho=(1, 1, 1),
               nu=(0.1, 0.1, 0.1))
    return _problem("nee_shear_%dx%d_U%g" % (nx, ny, U0), nx, ny, fl, (1, 0), mask, mats,
                    core, np.clip(shell, 0.0, None), steps=steps, U0=U0)


def gravity_puddles(g=4e-5, nx=600, ny=150, R=60.0, theta=90.0, sigma=0.1, M0=0.01,
                    steps=200000):
    """Two drops (densities 10 and 5 in an ambient fluid of density 1) on a
    wall under gravity G = (0, -rho g) (Sec. III.A): drops of radius
    R = nx/10 centred on the wall surface at x = nx/4 and 3nx/4, L = 4W,
    sigma = 0.1 for every pair, theta13 = theta23 = theta, tau = 0.8,
    M0 = 0.01; walls in rows 0 (wetting) and ny-1 (neutral)."""
    D = 4.0
    c1 = tanh_drop(nx, ny, 0.25 * nx, 0.5, R, D)
    c2 = tanh_drop(nx, ny, 0.75 * nx, 0.5, R, D)
    mask = channel_mask(nx, ny)
    mats = [material(theta, theta), material(90.0, 90.0)]
    fl = fluid(sigma=(sigma, sigma, sigma), D=D, M0=M0, tau=(0.8, 0.8), rho=(10, 5, 1),
               nu=(0.1, 0.1, 0.1), gravity=(0.0, -g))
    return _problem("gravity_puddles_%dx%d_g%g" % (nx, ny, g), nx, ny, fl, (1, 0), mask, mats,
                    c1, c2, steps=steps, g=g, R=R)


def cylinder_impact(We=10.0, theta=90.0, nx=1024, ny=2048, R_cyl=128.0, R_shell=96.0,
                    R_core=48.0, sigma=5e-3, steps=100000):
    """Compound drop (phase-1 core, phase-2 shell) falling onto a staircase
    cylinder in a fully periodic box; theta13 = theta23 = theta, theta12 = 90;
    densities 10/10/1; U = sqrt(We sigma_bar / (rho_bar xi)), xi = 2 R_shell
    (the Weber number of Eq. 55)."""
    D = 4.0
    xi = 2.0 * R_shell
    rho_bar = 10.0
    U = math.sqrt(We * sigma / (rho_bar * xi))
    xc, yc = nx / 2.0, ny / 2.0
    mask = cylinder_mask(nx, ny, xc, yc, R_cyl)
    mats = [material(theta, theta)]
    ydrop = yc + R_cyl + R_shell
    core = tanh_drop(nx, ny, xc, ydrop, R_core, D)
    shell = tanh_drop(nx, ny, xc, ydrop, R_shell, D) - core
    uy = -U * (core + shell)
    ux = np.zeros_like(uy)
    fl = fluid(sigma=(sigma, sigma, sigma), D=D, M0=0.1 * sigma, tau=(0.8, 0.8),
               rho=(10, 10, 1), nu=(0.1, 0.1, 0.1))
    return _problem("cylinder_impact_%dx%d_We%g_th%g" % (nx, ny, We, theta), nx, ny, fl,
                    (1, 1), mask, mats, core, shell, ux, uy, steps=steps, U=U, We=We)


def free_drop(nx=64, ny=64, R=16.0, sigma=1e-3, D=4.0, steps=2000, rho=(1, 1, 1),
              phase=1):
    """Drop of phase ``phase`` in phase 3 in a fully periodic box (no solid)."""
    mask = np.zeros((ny, nx), dtype=np.uint8)
    c = tanh_drop(nx, ny, nx / 2.0, ny / 2.0, R, D)
    z = np.zeros((ny, nx))
    c1, c2 = (c, z) if phase == 1 else (z, c)
    fl = fluid(sigma=(sigma, sigma, sigma), D=D, M0=0.1 * sigma, rho=rho)
    return _problem("free_drop_%dx%d_R%g" % (nx, ny, R), nx, ny, fl, (1, 1), mask, [], c1, c2,
                    steps=steps, R=R)


def random_fields(nx, ny, seed=7, amp=0.2, geometry="channel", U=0.0, rho=(1.0, 1.0, 1.0),
                  sigma=(1e-3, 1.3e-3, 1.1e-3), thetas=((60.0, 100.0), (120.0, 75.0)),
                  gravity=(0.0, 0.0)):
    """Smooth random three-phase mixture (sums of low-order Fourier modes) for
    parity tests: exercises every term with all three phases present."""
    x, y = coords(nx, ny)
    rng = Rng(seed)

    def smooth():
        f = np.zeros((ny, nx))
        for _ in range(4):
            kx, ky = rng.choice(3) + 1, rng.choice(3) + 1
            ph1, ph2 = rng.uniform(0, 2 * math.pi), rng.uniform(0, 2 * math.pi)
            f += np.sin(2 * math.pi * kx * x / nx + ph1) * np.cos(2 * math.pi * ky * y / ny + ph2)
        return f / 4.0

    a, b = smooth(), smooth()
    c1 = 1.0 / 3.0 + amp * a
    c2 = 1.0 / 3.0 + amp * b
    ux = 0.01 * smooth()
    uy = 0.01 * smooth()
    if geometry == "channel":
        mask = channel_mask(nx, ny)
        periodic = (1, 0)
        mats = [material(*thetas[0], wall_u=(-U, 0.0)), material(*thetas[1], wall_u=(U, 0.0))]
    elif geometry == "cylinder":
        mask = cylinder_mask(nx, ny, nx / 2.0, ny / 2.0, min(nx, ny) / 5.0)
        periodic = (1, 1)
        mats = [material(*thetas[0])]
    elif geometry == "box":
        mask = np.zeros((ny, nx), dtype=np.uint8)
        mask[0, :] = 1
        mask[-1, :] = 2
        mask[:, 0] = 1
        mask[:, -1] = 2
        periodic = (0, 0)
        mats = [material(*thetas[0]), material(*thetas[1])]
    else:
        mask = np.zeros((ny, nx), dtype=np.uint8)
        periodic = (1, 1)
        mats = []
    fl = fluid(sigma=sigma, D=4.0, M0=1e-4, tau=(0.8, 0.9), rho=rho, nu=(0.1, 0.05, 0.15),
               gravity=gravity)
    return _problem("random_%s_%dx%d_s%d" % (geometry, nx, ny, seed), nx, ny, fl, periodic, mask,
                    mats, c1, c2, ux, uy, steps=0)


def random_obstacles(nx, ny, seed=3, n_obstacles=40, n_materials=6, amp=0.2, U=0.01,
                     moving=True):
    """The smooth random three-phase mixture of ``random_fields`` in a fully
    periodic box scattered with small solid obstacles of ``n_materials``
    wetting materials: single nodes, 2x2 blocks, one-node-thick bars, L shapes
    and diagonal staircases, placed anywhere (so they touch each other, wrap
    across the periodic seams and cross strip boundaries).  Each material's
    contact angles are drawn until they are admissible; with ``moving`` every
    other material moves at speed U along x or y.  For parity tests of the
    wall paths: ghosts across every kind of link, corners, and bounce-back
    into neighbours of every direction."""
    rng = Rng(seed)
    sigma = (1e-3, 1.3e-3, 1.1e-3)
    mats = []
    for m in range(n_materials):
        while True:
            t13, t23 = rng.uniform(45.0, 135.0), rng.uniform(45.0, 135.0)
            if admissible(*sigma, theta13=t13, theta23=t23):
                break
        if moving and m % 2 == 1:
            u = (U, 0.0) if (m // 2) % 2 == 0 else (0.0, -U)
        else:
            u = (0.0, 0.0)
        mats.append(material(t13, t23, wall_u=u))
    mask = np.zeros((ny, nx), dtype=np.uint8)
    shapes = [[(0, 0)], [(0, 0), (1, 0), (0, 1), (1, 1)],
              [(i, 0) for i in range(5)], [(0, j) for j in range(4)],
              [(i, 0) for i in range(4)] + [(0, j) for j in range(1, 4)],
              [(i, i) for i in range(4)]]
    for _ in range(n_obstacles):
        x0, y0 = rng.choice(nx), rng.choice(ny)
        shape = shapes[rng.choice(len(shapes))]
        mid = 1 + rng.choice(n_materials)
        for dx, dy in shape:
            mask[(y0 + dy) % ny, (x0 + dx) % nx] = mid
    base = random_fields(nx, ny, seed=seed + 1000, amp=amp, geometry="periodic")
    fl = dict(base["fluid"])
    fl["sigma12"], fl["sigma13"], fl["sigma23"] = sigma
    return _problem("obstacles_%dx%d_s%d" % (nx, ny, seed), nx, ny, fl, (1, 1), mask, mats,
                    base["c1"], base["c2"], base["ux"], base["uy"], steps=0)


def bandwidth_case(nx, ny):
    """Cylinder geometry without a drop (pure phase 3 at rest): the memory
    sweep workload."""
    mask = cylinder_mask(nx, ny, nx / 2.0, ny / 2.0, min(nx, ny) / 8.0)
    z = np.zeros((ny, nx))
    fl = fluid(sigma=(5e-3,) * 3, M0=5e-4, rho=(10, 10, 1))
    return _problem("sweep_%dx%d" % (nx, ny), nx, ny, fl, (1, 1), mask, [material(90, 90)],
                    z, z, steps=500)


def floating_lens(nx=128, ny=128, R=20.0, sigma=(1e-2, 1e-2, 1e-2), D=4.0, M0=None, tau=0.8):
    """Liquid lens (Sec. III.B, Eq. 49): a disc of phase 2 of radius R centred
    on the flat interface y = ny/2 between a band of phase 1 (ny/8 <= y <
    ny/2) and phase 3, in a fully periodic box.  Unit densities; sigma =
    (sigma12, sigma13, sigma23)."""
    x, y = coords(nx, ny)
    yc = ny / 2.0
    c2 = tanh_drop(nx, ny, nx / 2.0, yc, R, D)
    band = (0.5 + 0.5 * np.tanh(2.0 * (yc - y) / D)) * (0.5 + 0.5 * np.tanh(2.0 * (y - ny / 8.0) / D))
    c1 = (1.0 - c2) * band
    mean_sigma = sum(sigma) / 3.0
    fl = fluid(sigma=sigma, D=D, M0=(0.1 * mean_sigma if M0 is None else M0), tau=(tau, tau))
    mask = np.zeros((ny, nx), dtype=np.uint8)
    return _problem("lens_%dx%d_R%g" % (nx, ny, R), nx, ny, fl, (1, 1), mask, [], c1, c2,
                    steps=0)


def large_lattice(nx, ny, seed=5):
    """Fully periodic three-phase lattice for size-limit tests: a smooth
    background mixture of all three phases (integer Fourier modes of about
    100-node wavelength, so it is periodic), a slow shear-like velocity, and
    five features, each a staircase cylinder of one of two wetting materials
    with a phase-1 and a phase-2 drop resting on it and on each other.  The
    features sit across the periodic corner, on the right edge (the ragged
    last strip column when nx is not a multiple of 64), on the top edge, in
    the centre, and near the bottom-right corner.  ``features`` lists their
    bounding boxes (x0, y0, w, h) for sampling."""
    rng = Rng(seed)
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)

    def mode(n, coord):
        k = max(1, n // 100) + rng.choice(3)
        return np.sin(2.0 * math.pi * k * coord / n + rng.uniform(0.0, 2.0 * math.pi))

    c1 = np.multiply.outer(mode(ny, y), mode(nx, x))
    c1 *= 0.15
    c1 += 1.0 / 3.0
    c2 = np.multiply.outer(mode(ny, y), mode(nx, x))
    c2 *= 0.15
    c2 += 1.0 / 3.0
    ux = np.multiply.outer(mode(ny, y), np.full(nx, 0.004))
    uy = np.multiply.outer(np.full(ny, 0.003), mode(nx, x))
    mask = np.zeros((ny, nx), dtype=np.uint8)
    centres = [(0, 0), (nx - 1, ny // 2), (nx // 2, ny - 1), (nx // 2, ny // 2),
               (nx - 40, 40)]
    D = 4.0
    features = []
    for i, (xc, yc) in enumerate(centres):
        Rc, Rd = 10.0 + 2 * i, 14.0
        phase = 1 + (i % 2)
        drops = [(xc + Rc + Rd - 3.0, yc + 4.0, phase),
                 (xc + Rc + Rd - 3.0, yc + 4.0 + 2 * Rd - 4.0, 3 - phase)]
        bx0, by0 = int(xc - Rc - 8), int(yc - Rc - 8)
        w = int(Rc + 2 * Rd + Rc + 24)
        h = int(Rc + 4 * Rd + 24)
        features.append((bx0 % nx, by0 % ny, w, h))
        xs = np.arange(bx0, bx0 + w)
        ys = np.arange(by0, by0 + h)
        box = np.ix_(ys % ny, xs % nx)
        X, Y = np.meshgrid(xs.astype(np.float64), ys.astype(np.float64))
        b1, b2 = c1[box], c2[box]
        for (dx, dy, ph) in drops:
            d = 0.5 + 0.5 * np.tanh(2.0 * (Rd - np.hypot(X - dx, Y - dy)) / D)
            b1 = (1.0 - d) * b1 + (d if ph == 1 else 0.0)
            b2 = (1.0 - d) * b2 + (d if ph == 2 else 0.0)
        c1[box], c2[box] = b1, b2
        cyl = np.hypot(X - xc, Y - yc) <= Rc
        mb = mask[box]
        mb[cyl] = 1 + (i % 2)
        mask[box] = mb
    fl = fluid(sigma=(1e-3, 1.3e-3, 1.1e-3), D=D, M0=1e-4, tau=(0.8, 0.9), rho=(3.0, 2.0, 1.0),
               nu=(0.1, 0.05, 0.15))
    mats = [material(60.0, 100.0), material(120.0, 75.0)]
    return _problem("large_%dx%d_s%d" % (nx, ny, seed), nx, ny, fl, (1, 1), mask, mats, c1, c2,
                    ux, uy, steps=0, features=features)


def serving_request(rng: Rng, n: int, kind: int, precision_steps=(1000, 20000)):
    """One serving request: a single (kind 0), binary (1) or compound (2)
    drop on the bottom wall of an n x n channel; contact angles ~ U[30, 150]
    deg, surface tensions ~ U[5e-4, 2e-3] (admissible draws), steps ~
    U{lo..hi}."""
    D = 4.0
    while True:
        th13, th23 = rng.uniform(30.0, 150.0), rng.uniform(30.0, 150.0)
        sig = (rng.uniform(5e-4, 2e-3), rng.uniform(5e-4, 2e-3), rng.uniform(5e-4, 2e-3))
        if admissible(*sig, theta13=th13, theta23=th23):
            break
    mask = channel_mask(n, n)
    mats = [material(th13, th23), material(90.0, 90.0)]
    R = n / 8.0
    if kind == 0:
        c1 = tanh_drop(n, n, n / 2.0, 0.5, R, D)
        c2 = np.zeros((n, n))
    elif kind == 1:
        c1 = tanh_drop(n, n, n / 2.0 - R, 0.5, R, D)
        c2 = tanh_drop(n, n, n / 2.0 + R, 0.5, R, D)
        c2 = np.where(c1 + c2 > 1.0, 1.0 - c1, c2)
    else:
        c2 = tanh_drop(n, n, n / 2.0, 0.5 + R, R / 2.0, D)
        c1 = tanh_drop(n, n, n / 2.0, 0.5 + R, R, D) - c2
    fl = fluid(sigma=sig, D=D, M0=0.1 * (sum(sig) / 3.0), rho=(1.0, 1.0, 1.0))
    lo, hi = precision_steps
    steps = lo + rng.choice(hi - lo + 1)
    return _problem("serve_%d_k%d" % (n, kind), n, n, fl, (1, 0), mask, mats, c1, c2,
                    steps=steps)


def serving_stream(n_requests=1000, seed=2026, sizes=(64, 128, 256, 512, 1024),
                   weights=(0.40, 0.30, 0.15, 0.10, 0.05), steps=(1000, 20000)):
    """A stream of independent requests: sizes drawn with the given weights,
    drop kind single / binary / compound with probability 1/3 each.  Returns
    (size, kind, steps, problem-factory) tuples; arrival times are drawn by
    the caller (Poisson at a chosen rate)."""
    rng = Rng(seed)
    cum = np.cumsum(weights) / np.sum(weights)
    out = []
    for _ in range(n_requests):
        u = rng.uniform()
        n = sizes[int(np.searchsorted(cum, u, side="right"))] if u < cum[-1] else sizes[-1]
        kind = rng.choice(3)
        sub = Rng(rng.next_u64())
        out.append((n, kind, sub))
    return [(n, kind, (lambda n=n, kind=kind, sub=sub: serving_request(Rng(sub.s), n, kind, steps)))
            for n, kind, sub in out]


def poisson_arrivals(n, rate, seed=7):
    """n arrival times (seconds) of a Poisson process with the given rate."""
    rng = Rng(seed)
    t, out = 0.0, []
    for _ in range(n):
        t += -math.log(1.0 - rng.uniform()) / rate
        out.append(t)
    return out


# ----------------------------------------------------------------- 3-D inputs
def coords3(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def tanh_ball(nx, ny, nz, xc, yc, zc, R, D):
    """Smooth ball indicator 1/2 + 1/2 tanh(2 (R - r) / D)."""
    x, y, z = coords3(nx, ny, nz)
    r = np.sqrt((x - xc) ** 2 + (y - yc) ** 2 + (z - zc) ** 2)
    return 0.5 + 0.5 * np.tanh(2.0 * (R - r) / D)


def _problem3(name, nx, ny, nz, fl, periodic, mask, mats, c1, c2, u=None, gravity_z=0.0,
              steps=0, **extra):
    solid = mask != 0
    fl = dict(fl, gravity_z=float(gravity_z))
    p = {"name": name, "nx": nx, "ny": ny, "nz": nz, "fluid": fl, "periodic": periodic,
         "material": np.ascontiguousarray(mask, dtype=np.uint8), "mats": mats,
         "c1": np.ascontiguousarray(np.where(solid, 0.0, c1)),
         "c2": np.ascontiguousarray(np.where(solid, 0.0, c2)),
         "ux": None, "uy": None, "uz": None, "steps": steps}
    if u is not None:
        for k, a in zip(("ux", "uy", "uz"), u):
            p[k] = np.ascontiguousarray(np.where(solid, 0.0, a))
    p.update(extra)
    return p


def random_fields3(nx, ny, nz, seed=11, amp=0.2, geometry="channel", U=0.0,
                   rho=(1.0, 1.0, 1.0), sigma=(1e-3, 1.3e-3, 1.1e-3),
                   thetas=((60.0, 100.0), (120.0, 75.0)), gravity=(0.0, 0.0, 0.0), lam=0.0):
    """Smooth random three-phase mixture in 3-D (low-order Fourier modes) for
    parity tests.  Geometries: 'channel' (walls in z = 0 and nz-1 moving at
    -U and +U along x), 'sphere' (a staircase ball in a periodic box), 'box'
    (walls on every face), 'periodic'."""
    x, y, z = coords3(nx, ny, nz)
    rng = Rng(seed)

    def field():
        acc = np.zeros((nz, ny, nx))
        for _ in range(4):
            kx, ky, kz = (int(rng.uniform(1, 3)) for _ in range(3))
            ph = rng.uniform(0.0, 2.0 * math.pi)
            acc += np.sin(2 * math.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + ph)
        return acc / 4.0

    c1 = 0.33 + amp * field()
    c2 = 0.33 + amp * field()
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    if geometry == "channel":
        mask[0], mask[nz - 1] = 1, 2
        mats = [material(*thetas[0], wall_u=(-U, 0.0)), material(*thetas[1], wall_u=(U, 0.0))]
        periodic = (1, 1, 0)
    elif geometry == "sphere":
        r = np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2)
        mask[r <= min(nx, ny, nz) / 5.0] = 1
        mats = [material(*thetas[0])]
        periodic = (1, 1, 1)
    elif geometry == "box":
        mask[0], mask[nz - 1] = 1, 1
        mask[:, 0], mask[:, ny - 1] = 2, 2
        mask[:, :, 0], mask[:, :, nx - 1] = 2, 2
        mats = [material(*thetas[0]), material(*thetas[1])]
        periodic = (0, 0, 0)
    else:
        mats = []
        periodic = (1, 1, 1)
    ux = 0.01 * np.sin(2 * math.pi * y / ny)
    uy = 0.01 * np.cos(2 * math.pi * z / nz)
    uz = 0.01 * np.sin(2 * math.pi * x / nx)
    fl = fluid(sigma=sigma, D=4.0, M0=1e-4, tau=(0.8, 0.9), rho=rho, nu=(0.1, 0.05, 0.15),
               gravity=gravity[:2], lam=lam)
    return _problem3("random3_%s_%dx%dx%d_s%d" % (geometry, nx, ny, nz, seed), nx, ny, nz, fl,
                     periodic, mask, mats, c1, c2, u=(ux, uy, uz), gravity_z=gravity[2])


def random_obstacles3(nx, ny, nz, seed=13, n_obstacles=30, n_materials=5, amp=0.2, U=0.01,
                      moving=True):
    """The 3-D counterpart of ``random_obstacles``: the smooth random mixture of
    ``random_fields3`` in a fully periodic box scattered with small solids of
    ``n_materials`` wetting materials (single voxels, 2x2x2 cubes, bars along
    x, y and z, 3x3 plates, staircases along an x-z diagonal), anywhere, so
    that they touch, wrap across the seams and cross tile and z-chunk
    boundaries; with ``moving`` every other material moves at U along x or y
    (walls move in the x-y plane)."""
    rng = Rng(seed)
    sigma = (1e-3, 1.3e-3, 1.1e-3)
    mats = []
    for m in range(n_materials):
        while True:
            t13, t23 = rng.uniform(45.0, 135.0), rng.uniform(45.0, 135.0)
            if admissible(*sigma, theta13=t13, theta23=t23):
                break
        if moving and m % 2 == 1:
            u = (U, 0.0) if (m // 2) % 2 == 0 else (0.0, -U)
        else:
            u = (0.0, 0.0)
        mats.append(material(t13, t23, wall_u=u))
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    shapes = [[(0, 0, 0)],
              [(i, j, k) for i in range(2) for j in range(2) for k in range(2)],
              [(i, 0, 0) for i in range(4)], [(0, j, 0) for j in range(4)],
              [(0, 0, k) for k in range(4)],
              [(i, j, 0) for i in range(3) for j in range(3)],
              [(i, 0, i) for i in range(4)]]
    for _ in range(n_obstacles):
        x0, y0, z0 = rng.choice(nx), rng.choice(ny), rng.choice(nz)
        shape = shapes[rng.choice(len(shapes))]
        mid = 1 + rng.choice(n_materials)
        for dx, dy, dz in shape:
            mask[(z0 + dz) % nz, (y0 + dy) % ny, (x0 + dx) % nx] = mid
    base = random_fields3(nx, ny, nz, seed=seed + 1000, amp=amp, geometry="periodic")
    fl = dict(base["fluid"])
    fl["sigma12"], fl["sigma13"], fl["sigma23"] = sigma
    return _problem3("obstacles3_%dx%dx%d_s%d" % (nx, ny, nz, seed), nx, ny, nz, fl, (1, 1, 1),
                     mask, mats, base["c1"], base["c2"], u=(base["ux"], base["uy"], base["uz"]))


def large_lattice3(nx, ny, nz, seed=5):
    """Fully periodic three-phase D3Q19 lattice for size-limit tests: a
    smooth background mixture of all three phases (products of integer
    Fourier modes of about 60-node wavelength), a slow velocity field, and
    four features, each a staircase ball of one of two wetting materials with
    a phase-1 and a phase-2 drop resting on it and on each other, placed
    across the periodic corner, on the ragged x edge, on the top edges and in
    the centre.  ``features`` lists their boxes (x0, y0, z0, w, h, d)."""
    rng = Rng(seed)

    def mode(n):
        k = max(1, n // 60) + rng.choice(2)
        return np.sin(2.0 * math.pi * k * np.arange(n) / n + rng.uniform(0.0, 2.0 * math.pi))

    def background(amp, off):
        a = np.multiply.outer(np.multiply.outer(mode(nz), mode(ny)), mode(nx))
        a *= amp
        a += off
        return a

    c1 = background(0.15, 1.0 / 3.0)
    c2 = background(0.15, 1.0 / 3.0)
    ux = background(0.004, 0.0)
    uy = background(0.003, 0.0)
    uz = background(0.003, 0.0)
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    centres = [(0, 0, 0), (nx - 1, ny // 2, nz // 2), (nx // 2, ny - 1, nz - 1),
               (nx // 2, ny // 2, nz // 2)]
    D = 4.0
    features = []
    for i, (xc, yc, zc) in enumerate(centres):
        Rb, Rd = 7.0 + i, 9.0
        phase = 1 + (i % 2)
        drops = [(xc + Rb + Rd - 2.0, yc, zc + 2.0, phase),
                 (xc + Rb + Rd - 2.0, yc, zc + 2.0 + 2 * Rd - 3.0, 3 - phase)]
        x0, y0, z0 = int(xc - Rb - 6), int(yc - Rb - 6), int(zc - Rb - 6)
        w, h, d = int(2 * Rb + 2 * Rd + 12), int(2 * Rb + 12), int(Rb + 4 * Rd + 12)
        features.append((x0 % nx, y0 % ny, z0 % nz, w, h, d))
        xs, ys, zs = np.arange(x0, x0 + w), np.arange(y0, y0 + h), np.arange(z0, z0 + d)
        box = np.ix_(zs % nz, ys % ny, xs % nx)
        Z, Y, X = np.meshgrid(zs.astype(float), ys.astype(float), xs.astype(float), indexing="ij")
        b1, b2 = c1[box], c2[box]
        for (dx, dy, dz, ph) in drops:
            dd = 0.5 + 0.5 * np.tanh(2.0 * (Rd - np.sqrt((X - dx) ** 2 + (Y - dy) ** 2 + (Z - dz) ** 2)) / D)
            b1 = (1.0 - dd) * b1 + (dd if ph == 1 else 0.0)
            b2 = (1.0 - dd) * b2 + (dd if ph == 2 else 0.0)
        c1[box], c2[box] = b1, b2
        mb = mask[box]
        mb[np.sqrt((X - xc) ** 2 + (Y - yc) ** 2 + (Z - zc) ** 2) <= Rb] = 1 + (i % 2)
        mask[box] = mb
    fl = fluid(sigma=(1e-3, 1.3e-3, 1.1e-3), D=D, M0=1e-4, tau=(0.8, 0.9), rho=(3.0, 2.0, 1.0),
               nu=(0.1, 0.05, 0.15))
    mats = [material(60.0, 100.0), material(120.0, 75.0)]
    return _problem3("large3_%dx%dx%d_s%d" % (nx, ny, nz, seed), nx, ny, nz, fl, (1, 1, 1), mask,
                     mats, c1, c2, u=(ux, uy, uz), features=features)


def sessile3d(nx=128, ny=128, nz=64, R_core=16.0, R_shell=32.0, theta13=60.0, theta23=90.0,
              sigma=1e-3, steps=2000):
    """Compound drop (phase-1 core, phase-2 shell) resting on a wetting wall
    in the plane z = 0 of a box periodic in x and y, neutral wall on top; the
    3-D analogue of the sessile drops of Sec. III.A-B."""
    D = 4.0
    core = tanh_ball(nx, ny, nz, nx / 2, ny / 2, 0.5, R_core, D)
    shell = tanh_ball(nx, ny, nz, nx / 2, ny / 2, 0.5, R_shell, D) - core
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    mask[0], mask[nz - 1] = 1, 2
    mats = [material(theta13, theta23), material(90.0, 90.0)]
    fl = fluid(sigma=(sigma, sigma, sigma), D=D, M0=0.1 * sigma, tau=(0.8, 0.8),
               rho=(1, 1, 1), nu=(0.1, 0.1, 0.1))
    return _problem3("sessile3d_%dx%dx%d" % (nx, ny, nz), nx, ny, nz, fl, (1, 1, 0), mask, mats,
                     core, np.clip(shell, 0.0, None), steps=steps)


def sphere_impact3d(nx=192, ny=192, nz=256, R_sphere=40.0, R_shell=32.0, R_core=16.0,
                    We=10.0, theta=90.0, sigma=5e-3):
    """3-D analogue of the cylinder impact of Sec. III.E: a compound drop
    (phase-1 core, phase-2 shell, densities 10/10/1) moving down onto a
    staircase sphere in a periodic box, touching it at t = 0."""
    D = 4.0
    xs, ys, zs = nx / 2.0, ny / 2.0, nz * 0.4
    zd = zs + R_sphere + R_shell
    core = tanh_ball(nx, ny, nz, xs, ys, zd, R_core, D)
    shell = tanh_ball(nx, ny, nz, xs, ys, zd, R_shell, D) - core
    x, y, z = coords3(nx, ny, nz)
    mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    mask[(x - xs) ** 2 + (y - ys) ** 2 + (z - zs) ** 2 <= R_sphere ** 2] = 1
    rho_bar, xi = 10.0, 2.0 * R_shell
    U = math.sqrt(We * sigma / (rho_bar * xi))
    cs = np.clip(shell, 0.0, None)
    uz = -U * (core + cs)
    fl = fluid(sigma=(sigma, sigma, sigma), D=D, M0=0.1 * sigma, tau=(0.8, 0.8),
               rho=(10, 10, 1), nu=(0.1, 0.1, 0.1))
    z0 = np.zeros_like(uz)
    return _problem3("sphere_impact3d_%dx%dx%d_We%g" % (nx, ny, nz, We), nx, ny, nz, fl,
                     (1, 1, 1), mask, [material(theta, theta)], core, cs, u=(z0, z0, uz),
                     U=U, We=We)
