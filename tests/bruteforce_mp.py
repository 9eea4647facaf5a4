"""Brute-force, hand-expanded update of the phase-field LB step in 40-digit mpmath.

An independent second reading of Secs. 2.2-2.3 for tiny grids, used to pin the FP64
oracle: no loops over lattice directions, every population written out on its own line,
no code shared with the oracle.  Boundaries: x periodic; y periodic, half-way bounce-back
wall, or open side held at the ambient pressure p = 0 (an incoming population is what the
edge node at x - c_ix sent out in that direction, its g with the pressure part of the
equilibrium moved from the node's p to 0); the stencil's ghost rows mirror the first
interior row at walls and open sides.
"""
import mpmath as mp

mp.mp.dps = 40

W0, WA, WD = mp.mpf(4) / 9, mp.mpf(1) / 9, mp.mpf(1) / 36
V0, VA = mp.mpf(1) / 3, mp.mpf(1) / 6          # D2Q5 phase-field weights
HALF = mp.mpf(1) / 2
PERIODIC, WALL, OPEN = 0, 1, 2


class Grid:
    def __init__(self, nx, ny, bc_ylo, bc_yhi):
        self.nx, self.ny, self.lo, self.hi = nx, ny, bc_ylo, bc_yhi

    def gx(self, x):
        return x % self.nx

    def gy(self, y):
        if y < 0:
            return y + self.ny if self.lo == PERIODIC else 0
        if y >= self.ny:
            return y - self.ny if self.hi == PERIODIC else self.ny - 1
        return y


def viscosity(prm, phi, rho):
    law = prm["visc_law"]
    if law == 0:
        return phi * (prm["nu_l"] - prm["nu_g"]) + prm["nu_g"]
    if law == 1:
        return 1 / (phi * (1 / prm["nu_l"] - 1 / prm["nu_g"]) + 1 / prm["nu_g"])
    mu = prm["rho_l"] * prm["nu_l"] if phi >= HALF else prm["rho_g"] * prm["nu_g"]
    return mu / rho


def node_update(prm, P, x, y, grid, f, g, q):
    """Returns post-collision (f*, g*) at node (x, y) and the new q; P(x, y) gives phi."""
    X, Xp, Xm = x, grid.gx(x + 1), grid.gx(x - 1)
    Y, Yp, Ym = y, grid.gy(y + 1), grid.gy(y - 1)
    pc = P[Y][X]
    pE, pN, pWe, pS = P[Y][Xp], P[Yp][X], P[Y][Xm], P[Ym][X]
    pNE, pNW, pSW, pSE = P[Yp][Xp], P[Yp][Xm], P[Ym][Xm], P[Ym][Xp]
    # Eq. 27 (weights over c_s^2 = 1/3), Eq. 28
    dpx = 3 * (WA * (pE - pWe) + WD * (pNE - pNW - pSW + pSE))
    dpy = 3 * (WA * (pN - pS) + WD * (pNE + pNW - pSW - pSE))
    lap = 6 * (WA * (pE + pN + pWe + pS - 4 * pc) + WD * (pNE + pNW + pSW + pSE - 4 * pc))

    rl, rg = prm["rho_l"], prm["rho_g"]
    sigma, Wd, M = prm["sigma"], prm["W"], prm["M"]
    kap = mp.mpf(3) / 2 * sigma * Wd
    bet = 12 * sigma / Wd
    tau_f = 3 * M + HALF
    q5 = prm.get("f_lattice", 9) == 5
    if q5:
        phi = f[0] + f[1] + f[2] + f[3] + f[4]
    else:
        phi = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8]
    assert abs(phi - pc) < mp.mpf(10) ** -35
    rho = phi * (rl - rg) + rg
    mu_phi = 4 * bet * phi * (phi - 1) * (phi - HALF) - kap * lap
    lam = 4 * phi * (1 - phi) / Wd
    mag = mp.sqrt(dpx * dpx + dpy * dpy)
    if mag > mp.mpf("1e-12"):
        nx_, ny_ = dpx / mag, dpy / mag
    else:
        nx_, ny_ = mp.mpf(0), mp.mpf(0)
    tau_g = 3 * viscosity(prm, phi, rho) + HALF
    Fx = mu_phi * dpx + prm["Gx"]
    Fy = mu_phi * dpy + prm["Gy"]
    jx = g[1] - g[3] + g[5] - g[6] - g[7] + g[8]
    jy = g[2] - g[4] + g[5] + g[6] - g[7] - g[8]
    ux = (jx + HALF * Fx) / rho
    uy = (jy + HALF * Fy) / rho
    uu = ux * ux + uy * uy
    s0 = -mp.mpf(2) / 3 * uu
    sum_nz = g[1] + g[2] + g[3] + g[4] + g[5] + g[6] + g[7] + g[8]
    p = (mp.mpf(1) / 3) / (1 - W0) * (sum_nz + HALF * (rl - rg) * (ux * dpx + uy * dpy) + rho * s0)

    # backward difference of phi u
    Dx, Dy = phi * ux - q[0], phi * uy - q[1]
    qn = (phi * ux, phi * uy)

    # f equilibrium (Eq. 9) and source (Eq. 11), written per direction
    if q5:
        fe = [V0 * phi,
              VA * phi * (1 + 3 * ux), VA * phi * (1 + 3 * uy),
              VA * phi * (1 - 3 * ux), VA * phi * (1 - 3 * uy)]
    else:
        fe = [W0 * phi,
              WA * phi * (1 + 3 * ux), WA * phi * (1 + 3 * uy),
              WA * phi * (1 - 3 * ux), WA * phi * (1 - 3 * uy),
              WD * phi * (1 + 3 * (ux + uy)), WD * phi * (1 + 3 * (-ux + uy)),
              WD * phi * (1 + 3 * (-ux - uy)), WD * phi * (1 + 3 * (ux - uy))]
    if prm.get("grad_scheme", 0) == 1:
        # Eq. 29 in its printed two-step form: |grad phi| from Eq. 29a, then grad phi from
        # Eq. 29b, then n = grad phi / |grad phi|; C is the first moment of f - f^eq plus
        # half the time derivative of phi u.  Where C vanishes the direction is undefined
        # and n is zero.
        if q5:
            Cx = (f[1] - fe[1]) - (f[3] - fe[3]) + HALF * Dx
            Cy = (f[2] - fe[2]) - (f[4] - fe[4]) + HALF * Dy
        else:
            Cx = ((f[1] - fe[1]) - (f[3] - fe[3]) + (f[5] - fe[5]) - (f[6] - fe[6])
                  - (f[7] - fe[7]) + (f[8] - fe[8]) + HALF * Dx)
            Cy = ((f[2] - fe[2]) - (f[4] - fe[4]) + (f[5] - fe[5]) + (f[6] - fe[6])
                  - (f[7] - fe[7]) - (f[8] - fe[8]) + HALF * Dy)
        Cm = mp.sqrt(Cx * Cx + Cy * Cy)
        if Cm > mp.mpf("1e-12"):
            A = -tau_f / 3
            B = M * lam
            gm = (-Cm - B) / A
            den = A + B / gm
            nx_, ny_ = (Cx / den) / gm, (Cy / den) / gm
        else:
            nx_, ny_ = mp.mpf(0), mp.mpf(0)
    ax = 3 * Dx + lam * nx_
    ay = 3 * Dy + lam * ny_
    cf = 1 - 1 / (2 * tau_f)
    if q5:
        fs = [mp.mpf(0), cf * VA * ax, cf * VA * ay, -cf * VA * ax, -cf * VA * ay]
    else:
        fs = [mp.mpf(0),
              cf * WA * ax, cf * WA * ay, -cf * WA * ax, -cf * WA * ay,
              cf * WD * (ax + ay), cf * WD * (-ax + ay), cf * WD * (-ax - ay), cf * WD * (ax - ay)]
    fp = [f[i] - (f[i] - fe[i]) / tau_f + fs[i] for i in range(len(fe))]

    # g equilibrium (Eqs. 16-17) and forcing (Eq. 20), per direction
    def s_ax(cu):
        return WA * (3 * cu + mp.mpf(9) / 2 * cu * cu - mp.mpf(3) / 2 * uu)

    def s_dg(cu):
        return WD * (3 * cu + mp.mpf(9) / 2 * cu * cu - mp.mpf(3) / 2 * uu)

    ge = [3 * p * (W0 - 1) + rho * s0,
          3 * p * WA + rho * s_ax(ux), 3 * p * WA + rho * s_ax(uy),
          3 * p * WA + rho * s_ax(-ux), 3 * p * WA + rho * s_ax(-uy),
          3 * p * WD + rho * s_dg(ux + uy), 3 * p * WD + rho * s_dg(-ux + uy),
          3 * p * WD + rho * s_dg(-ux - uy), 3 * p * WD + rho * s_dg(ux - uy)]
    cg = 1 - 1 / (2 * tau_g)
    dr = rl - rg
    gf = [mp.mpf(0),
          cg * WA * (3 * Fx + 3 * dr * ux * dpx),
          cg * WA * (3 * Fy + 3 * dr * uy * dpy),
          cg * WA * (-3 * Fx + 3 * dr * ux * dpx),
          cg * WA * (-3 * Fy + 3 * dr * uy * dpy),
          cg * WD * (3 * (Fx + Fy) + 3 * dr * (ux + uy) * (dpx + dpy)),
          cg * WD * (3 * (-Fx + Fy) + 3 * dr * (-ux + uy) * (-dpx + dpy)),
          cg * WD * (3 * (-Fx - Fy) + 3 * dr * (ux + uy) * (dpx + dpy)),
          cg * WD * (3 * (Fx - Fy) + 3 * dr * (ux - uy) * (dpx - dpy))]
    gp = [g[i] - (g[i] - ge[i]) / tau_g + gf[i] for i in range(9)]
    return fp, gp, qn, dict(phi=phi, rho=rho, p=p, ux=ux, uy=uy)


# direction table used only for streaming destinations: (dx, dy, opposite)
_DIRS = {0: (0, 0, 0), 1: (1, 0, 3), 2: (0, 1, 4), 3: (-1, 0, 1), 4: (0, -1, 2),
         5: (1, 1, 7), 6: (-1, 1, 8), 7: (-1, -1, 5), 8: (1, -1, 6)}


def step(prm, grid, F, G, Q):
    """F, G: [ny][nx] lists of 9-lists (post-streaming); Q: [ny][nx] of 2-tuples."""
    nx, ny = grid.nx, grid.ny
    P = [[sum(F[y][x]) for x in range(nx)] for y in range(ny)]
    qf = len(F[0][0])
    Fn = [[[None] * qf for _ in range(nx)] for _ in range(ny)]
    Gn = [[[None] * 9 for _ in range(nx)] for _ in range(ny)]
    Qn = [[None] * nx for _ in range(ny)]
    Pr = [[None] * nx for _ in range(ny)]
    for y in range(ny):
        for x in range(nx):
            fp, gp, qn, mom = node_update(prm, P, x, y, grid, F[y][x], G[y][x], Q[y][x])
            Qn[y][x] = qn
            Pr[y][x] = mom["p"]
            for i in range(9):
                dx, dy, o = _DIRS[i]
                xd, yd = (x + dx) % nx, y + dy
                side = grid.lo if yd < 0 else (grid.hi if yd >= ny else None)
                if side is None or side == PERIODIC:
                    if i < qf:
                        Fn[yd % ny][xd][i] = fp[i]
                    Gn[yd % ny][xd][i] = gp[i]
                elif side == WALL:
                    if i < qf:
                        Fn[y][x][o] = fp[i]
                    Gn[y][x][o] = gp[i]
    if grid.hi == OPEN:
        t = ny - 1
        for x in range(nx):
            xl, xr = (x - 1) % nx, (x + 1) % nx
            # down (0,-1) from x; down-left (-1,-1) from x + 1; down-right (1,-1) from x - 1
            if qf > 4:
                Fn[t][x][4] = Fn[t - 1][x][4]
            if qf > 8:
                Fn[t][x][7] = Fn[t - 1][x][7]
                Fn[t][x][8] = Fn[t - 1][x][8]
            Gn[t][x][4] = Gn[t - 1][x][4] + 3 * WA * (0 - Pr[t][x])
            Gn[t][x][7] = Gn[t - 1][x][7] + 3 * WD * (0 - Pr[t][xr])
            Gn[t][x][8] = Gn[t - 1][x][8] + 3 * WD * (0 - Pr[t][xl])
    if grid.lo == OPEN:
        for x in range(nx):
            xl, xr = (x - 1) % nx, (x + 1) % nx
            # up (0,1) from x; up-right (1,1) from x - 1; up-left (-1,1) from x + 1
            Fn[0][x][2] = Fn[1][x][2]
            if qf > 8:
                Fn[0][x][5] = Fn[1][x][5]
                Fn[0][x][6] = Fn[1][x][6]
            Gn[0][x][2] = Gn[1][x][2] + 3 * WA * (0 - Pr[0][x])
            Gn[0][x][5] = Gn[1][x][5] + 3 * WD * (0 - Pr[0][xl])
            Gn[0][x][6] = Gn[1][x][6] + 3 * WD * (0 - Pr[0][xr])
    return Fn, Gn, Qn


def moments(prm, grid, F, G, Q):
    nx, ny = grid.nx, grid.ny
    P = [[sum(F[y][x]) for x in range(nx)] for y in range(ny)]
    out = [[None] * nx for _ in range(ny)]
    for y in range(ny):
        for x in range(nx):
            out[y][x] = node_update(prm, P, x, y, grid, F[y][x], G[y][x], Q[y][x])[3]
    return out


def to_mp(prm):
    return {k: (mp.mpf(v) if isinstance(v, float) else v) for k, v in prm.items()}
