"""Measurement of a floating liquid lens and its analytic shape (Sec. III.B,
Eq. 49): helpers shared by the oracle pin and the GPU physics test.

At equilibrium the lens of phase 2 on the flat 1|3 interface is bounded by
two circular arcs (Laplace: the pressure jump across each arc is sigma/R,
and phases 1 and 3 are at one pressure, so sigma12/R12 = sigma23/R23).  The
three tensions balance at the triple points (Neumann's triangle, Eq. 49):
the lower (1|2) arc leaves the interface at beta1 below the horizontal and
the upper (2|3) arc at beta3 above it, with
    cos beta1 = (s13^2 + s12^2 - s23^2) / (2 s13 s12)
    cos beta3 = (s13^2 + s23^2 - s12^2) / (2 s13 s23)
and the angles inside the phases phi1 = 180 - beta1, phi2 = beta1 + beta3,
phi3 = 180 - beta3 (sin phi1 / s23 = sin phi2 / s13 = sin phi3 / s12).  The
lens area A fixes the chord L: A = L^2/4 sum_a (beta_a - sin beta_a cos
beta_a) / sin^2 beta_a, and the thickness is H = sum_a R_a (1 - cos beta_a)
with R_a = L / (2 sin beta_a).
"""
import math

import numpy as np


def analytic(s12, s13, s23, area):
    b1 = math.acos((s13 ** 2 + s12 ** 2 - s23 ** 2) / (2 * s13 * s12))
    b3 = math.acos((s13 ** 2 + s23 ** 2 - s12 ** 2) / (2 * s13 * s23))
    k = sum((b - math.sin(b) * math.cos(b)) / math.sin(b) ** 2 for b in (b1, b3))
    L = 2.0 * math.sqrt(area / k)
    R12, R23 = L / (2 * math.sin(b1)), L / (2 * math.sin(b3))
    H = R12 * (1 - math.cos(b1)) + R23 * (1 - math.cos(b3))
    deg = math.degrees
    return {"phi1": 180 - deg(b1), "phi2": deg(b1 + b3), "phi3": 180 - deg(b3),
            "L": L, "H": H, "R12": R12, "R23": R23}


def _fit_circle(xs, ys):
    A = np.column_stack([xs, ys, np.ones_like(xs)])
    (d, e, f), *_ = np.linalg.lstsq(A, -(xs ** 2 + ys ** 2), rcond=None)
    xc, yc = -d / 2, -e / 2
    return xc, yc, math.sqrt(xc * xc + yc * yc - f)


def _run_length(v):
    """Length of the c > 0.5 run through the maximum of the periodic profile
    v, with linear interpolation at both ends."""
    n = len(v)
    i = int(np.argmax(v))
    a = b = i
    while v[(a - 1) % n] > 0.5:
        a -= 1
    while v[(b + 1) % n] > 0.5:
        b += 1
    lo = (a - 1) + (0.5 - v[(a - 1) % n]) / (v[a % n] - v[(a - 1) % n])
    hi = b + (v[b % n] - 0.5) / (v[b % n] - v[(b + 1) % n])
    return hi - lo


def measure(c1, c2):
    """Angles phi_i from circle fits of the c2 = 0.5 contour above and below
    the 1|3 interface (columns through the lens, more than 3 nodes from the
    interface), the arcs' radii, the lens length along the interface and its
    thickness through its centre column (the lens must not straddle the
    x wrap), and the interface height far away."""
    ny, nx = c1.shape
    col = c1[:, 0]
    j = ny // 2 - 10
    while col[j + 1] > 0.5:
        j += 1
    yi = j + (col[j] - 0.5) / (col[j] - col[j + 1])
    up, dn = [], []
    for x in range(nx):
        v = c2[:, x]
        if v.max() < 0.9:
            continue
        t = b = int(np.argmax(v))
        while v[t + 1] > 0.5:
            t += 1
        while v[b - 1] > 0.5:
            b -= 1
        yt = t + (v[t] - 0.5) / (v[t] - v[t + 1])
        yb = b - (v[b] - 0.5) / (v[b] - v[b - 1])
        if yt - yi > 3:
            up.append((x, yt))
        if yi - yb > 3:
            dn.append((x, yb))
    up, dn = np.array(up, float), np.array(dn, float)
    _, yu, R23 = _fit_circle(up[:, 0], up[:, 1])
    _, yd, R12 = _fit_circle(dn[:, 0], dn[:, 1])
    b3 = math.degrees(math.acos(max(-1.0, min(1.0, (yi - yu) / R23))))
    b1 = math.degrees(math.acos(max(-1.0, min(1.0, (yd - yi) / R12))))
    xc = int(round(float((c2.sum(axis=0) * np.arange(nx)).sum() / c2.sum())))  # lens centre column
    r = int(math.floor(yi))
    row = 0.5 * (c2[r, :] + c2[r + 1, :])
    return {"phi1": 180 - b1, "phi2": b1 + b3, "phi3": 180 - b3, "R12": R12, "R23": R23,
            "L": _run_length(row), "H": _run_length(c2[:, xc]), "y_interface": yi}
