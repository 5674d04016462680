"""Geometry of a sessile drop: the contact angle measured on the c = 0.5
contour (Sec. III.A: theta_n = 2 arctan(2 H_d / L_s)) and the circular cap of
the same area that Eq. 47 predicts for a prescribed angle."""
import math


def measure(c, y_wall=0.5):
    """(theta_n in degrees, L_s, H_d) of the drop in field c (rows y, columns
    x): L_s from the c = 0.5 crossings on the first two fluid rows,
    extrapolated to the wall surface y_wall; H_d the apex height above the
    wall on the centre column (linear interpolation along lattice lines)."""
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
    Hd = top - y_wall
    return math.degrees(2 * math.atan(2 * Hd / Ls)), Ls, Hd


def de_gennes(R, theta_deg):
    """(L_s, H_d) of the circular cap with contact angle theta whose area
    equals that of a half disc of radius R (Eq. 47)."""
    te = math.radians(theta_deg)
    k = math.sqrt((math.pi / 2) / (te - math.sin(te) * math.cos(te)))
    return 2 * R * k * math.sin(te), R * k * (1 - math.cos(te))


def contour_points(c, level=0.5):
    """Points of the c = level contour: crossings along every row and every
    column of the lattice, by linear interpolation between neighbours."""
    import numpy as np
    ny, nx = c.shape
    pts = []
    for y in range(ny):
        row = c[y]
        for x in range(nx - 1):
            a, b = row[x], row[x + 1]
            if (a - level) * (b - level) < 0:
                pts.append((x + (level - a) / (b - a), float(y)))
    for x in range(nx):
        col = c[:, x]
        for y in range(ny - 1):
            a, b = col[y], col[y + 1]
            if (a - level) * (b - level) < 0:
                pts.append((float(x), y + (level - a) / (b - a)))
    return np.array(pts)


def circle_fit(c, y_wall=0.5, exclude=4.0):
    """Second estimate of the contact angle: a circle fitted to the c = 0.5
    contour points higher than `exclude` above the wall surface (the cap away
    from the wall's diffuse layer), least squares in the algebraic form
    x^2 + y^2 + a x + b y + d = 0 refined by Gauss-Newton on the geometric
    distances; the angle inside the drop where that circle meets the wall
    line, arccos(-(y_c - y_wall) / r).  Returns (theta in degrees, x_c, y_c, r)."""
    import numpy as np
    pts = contour_points(c)
    pts = pts[pts[:, 1] >= y_wall + exclude]
    x, y = pts[:, 0], pts[:, 1]
    A = np.c_[x, y, np.ones_like(x)]
    a, b, d = np.linalg.lstsq(A, -(x * x + y * y), rcond=None)[0]
    xc, yc = -a / 2, -b / 2
    r = math.sqrt(xc * xc + yc * yc - d)
    for _ in range(20):
        dx, dy = x - xc, y - yc
        rho = np.hypot(dx, dy)
        J = np.c_[-dx / rho, -dy / rho, -np.ones_like(rho)]
        step = np.linalg.lstsq(J, -(rho - r), rcond=None)[0]
        xc, yc, r = xc + step[0], yc + step[1], r + step[2]
        if np.abs(step).max() < 1e-12:
            break
    return math.degrees(math.acos(-(yc - y_wall) / r)), xc, yc, r
