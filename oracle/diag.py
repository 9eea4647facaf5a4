"""Definitions of the integral diagnostics, written plainly in numpy on FP64 fields.

Test infrastructure: these are what the GPU library's reductions are checked against.
Input is the dict of [ny][nx] fields returned by ``OracleSim.moments``.

mask = (xc, yc, r_in, r_out, y_row):
  p_in   mean of p over nodes whose periodic distance to (xc, yc) is < r_in
  p_out  mean of p over nodes whose periodic distance to (xc, yc) is > r_out
         (the Laplace-law pressure jump of a static drop is p_in - p_out)
  spread_radius  on row y_row, the largest |x* - xc| over points x* where phi crosses
         0.5 between horizontally adjacent nodes, x* found by linear interpolation in
         cell-centred coordinates (node i sits at x = i + 0.5)
Node coordinates are cell-centred (i + 0.5, j + 0.5).
"""
import numpy as np

KEYS = ("sum_phi", "sum_rho", "kinetic", "max_u", "min_rho", "min_phi", "max_phi",
        "p_in", "p_out", "interface_crossings", "spread_radius")


def periodic_distance(nx, ny, xc, yc, periodic_y=True):
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    dx = np.abs(x - xc)
    dx = np.minimum(dx, nx - dx)
    dy = np.abs(y - yc)
    if periodic_y:
        dy = np.minimum(dy, ny - dy)
    return np.sqrt(dx[None, :] ** 2 + dy[:, None] ** 2)


def crossings(phi, periodic_y):
    """Number of x- and y-neighbour pairs whose phi lie on different sides of 0.5
    (a node with phi >= 0.5 counts as liquid).  x is periodic; y wraps only if periodic."""
    liq = phi >= 0.5
    n = int(np.count_nonzero(liq != np.roll(liq, -1, axis=1)))
    if periodic_y:
        n += int(np.count_nonzero(liq != np.roll(liq, -1, axis=0)))
    else:
        n += int(np.count_nonzero(liq[:-1, :] != liq[1:, :]))
    return n


def spread_radius(phi, xc, y_row):
    row = phi[int(y_row)]
    best = 0.0
    for i in range(row.size - 1):
        a, b = row[i] - 0.5, row[i + 1] - 0.5
        if (a >= 0) != (b >= 0):
            xs = i + 0.5 + a / (a - b)
            best = max(best, abs(xs - xc))
    return best


def diagnostics(m, rho_l, rho_g, mask=(0.0, 0.0, 0.0, 0.0, 0.0), periodic_y=True):
    phi, rho, p, ux, uy = m["phi"], m["rho"], m["p"], m["ux"], m["uy"]
    ny, nx = phi.shape
    xc, yc, r_in, r_out, y_row = mask
    u2 = ux * ux + uy * uy
    d = {
        "sum_phi": float(np.sum(phi)),
        "sum_rho": float(np.sum(rho)),
        "kinetic": float(np.sum(0.5 * rho * u2)),
        "max_u": float(np.sqrt(np.max(u2))),
        "min_rho": float(np.min(rho)),
        "min_phi": float(np.min(phi)),
        "max_phi": float(np.max(phi)),
    }
    r = periodic_distance(nx, ny, xc, yc, periodic_y)
    inside, outside = r < r_in, r > r_out
    d["p_in"] = float(p[inside].mean()) if inside.any() else 0.0
    d["p_out"] = float(p[outside].mean()) if outside.any() else 0.0
    d["interface_crossings"] = float(crossings(phi, periodic_y))
    d["spread_radius"] = float(spread_radius(phi, xc, y_row)) if 0 <= y_row < ny else 0.0
    finite = np.isfinite(phi) & np.isfinite(rho) & np.isfinite(p) & np.isfinite(ux) & np.isfinite(uy)
    d["nonfinite"] = int(np.count_nonzero(~finite))
    return d
