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
