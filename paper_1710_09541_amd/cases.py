"""Seeded synthetic workloads shaped like the paper's four experiments (Sec. 3).

This module only builds inputs: parameter dicts and the initial fields phi0, u0.  It holds
none of the lattice Boltzmann arithmetic, and it is the one module both the GPU library's
callers and the CPU oracle's callers take their inputs from.

Every case is a dict with
  nx, ny, bc_ylo, bc_yhi           grid (x always periodic) and y boundaries
  visc_law                         0 linear nu (Eq. 24), 1 inverse-linear (Eq. 25), 2 step mu (Eq. 26)
  rho_l, rho_g, nu_l, nu_g, sigma, W, M, Gx, Gy
  phi0, ux0, uy0                   float64 [ny][nx], row-major, x fastest
  u_scale, p_scale                 magnitudes used to normalise max-norm errors
  mask                             (xc, yc, r_in, r_out, y_row) for the diagnostics
Node (i, j) sits at the cell centre (i + 0.5, j + 0.5); a half-way wall lies on the
domain edge y = 0 or y = ny.  Absolute densities use rho_g = 1 (only the ratio matters).
"""
import numpy as np

PERIODIC, WALL, OPEN = 0, 1, 2
NU_LINEAR, NU_INVERSE, MU_STEP = 0, 1, 2

PARAM_KEYS = ("rho_l", "rho_g", "nu_l", "nu_g", "sigma", "W", "M", "Gx", "Gy")
GRAD_ISOTROPIC, GRAD_LOCAL_NEQ = 0, 1   # normal in the phase-field source: Eq. 27 or Eq. 29
D2Q9, D2Q5 = 9, 5                        # velocity sets of the phase-field lattice


def _grid(nx, ny):
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    return np.meshgrid(x, y)  # X[j, i], Y[j, i]


def _base(name, nx, ny, bc_ylo, bc_yhi, visc_law, rho_l, rho_g, nu_l, nu_g, sigma, W, M,
          Gx=0.0, Gy=0.0):
    return dict(name=name, nx=int(nx), ny=int(ny), bc_ylo=bc_ylo, bc_yhi=bc_yhi,
                visc_law=visc_law, rho_l=float(rho_l), rho_g=float(rho_g), nu_l=float(nu_l),
                nu_g=float(nu_g), sigma=float(sigma), W=float(W), M=float(M), Gx=float(Gx),
                Gy=float(Gy), grad_scheme=GRAD_ISOTROPIC, f_lattice=9,
                mask=(0.0, 0.0, 0.0, 0.0, -1.0))


def tanh_profile(d, W):
    """phi = 0.5 + 0.5 tanh(2 d / W), d the signed distance into the liquid (Eqs. 30, 33)."""
    return 0.5 + 0.5 * np.tanh(2.0 * d / W)


def static_drop(nx=64, ny=64, R=16.0, W=4.0, ratio=1000.0, sigma=0.01, nu=0.1, M=0.1,
                visc_law=NU_LINEAR):
    """Sec. 3.1: a drop of radius R at the domain centre, periodic in x and y, u = 0.
    Eq. 30 with the distance under a square root (the printed formula drops it)."""
    c = _base("static_drop", nx, ny, PERIODIC, PERIODIC, visc_law, ratio, 1.0, nu, nu, sigma,
              W, M)
    X, Y = _grid(nx, ny)
    xc, yc = nx / 2.0, ny / 2.0
    r = np.sqrt((X - xc) ** 2 + (Y - yc) ** 2)
    c["phi0"] = tanh_profile(R - r, W)
    c["ux0"] = np.zeros((ny, nx))
    c["uy0"] = np.zeros((ny, nx))
    c["R"] = float(R)
    c["u_scale"] = sigma / (ratio * nu)
    c["p_scale"] = sigma / R
    c["mask"] = (xc, yc, max(R - W, 1.0), R + 2.0 * W, -1.0)
    return c


def spinodal(n=1024, seed=0, ratio=3.0, sigma=0.001, W=4.0, M=0.1, nu_l=0.1, nu_g=1.0,
             phi_mean=0.5, amp=0.01):
    """Sec. 3.3: a near-uniform mixture phi = phi_mean + uniform noise of amplitude amp,
    periodic in x and y, u = 0.  The noise is drawn once here from a seeded generator."""
    c = _base("spinodal", n, n, PERIODIC, PERIODIC, NU_LINEAR, ratio, 1.0, nu_l, nu_g, sigma,
              W, M)
    rng = np.random.default_rng(seed)
    c["phi0"] = phi_mean + rng.uniform(-amp, amp, size=(n, n))
    c["ux0"] = np.zeros((n, n))
    c["uy0"] = np.zeros((n, n))
    c["u_scale"] = float(np.sqrt(sigma / (ratio * W)))
    c["p_scale"] = sigma / W
    return c


def poiseuille_profile(y_a, h, mu_l, mu_g, Gx):
    """Eq. 31: steady two-layer channel profile, gas on 0 < y <= h, liquid on -h <= y <= 0."""
    s = y_a / h
    a = (mu_g - mu_l) / (mu_g + mu_l)
    gas = Gx * h * h / (2.0 * mu_g) * (-s * s - s * a + 2.0 * mu_g / (mu_g + mu_l))
    liq = Gx * h * h / (2.0 * mu_l) * (-s * s - s * a + 2.0 * mu_l / (mu_g + mu_l))
    return np.where(y_a > 0, gas, liq)


def layered_poiseuille(nx=16, ny=512, ratio=1000.0, nu_l=0.1, nu_g=1.0, W=5.0, sigma=0.001,
                       M=0.1, u_max=1e-3, u_c=None, init="analytic", visc_law=MU_STEP):
    """Sec. 3.2: liquid in the lower half, gas in the upper half, half-way bounce-back walls
    at y = 0 and y = ny, driven by a uniform body-force density G_x.

    Either u_c (the paper's centre-line speed: G_x = u_c (mu_l + mu_g) / h^2) or u_max (the
    largest speed of the analytic profile) fixes G_x.  init = "analytic" starts from the
    Eq. 31 profile, "rest" from u = 0.  Eq. 33 gives phi (cell-centred y)."""
    mu_l, mu_g = ratio * nu_l, 1.0 * nu_g
    h = ny / 2.0
    X, Y = _grid(nx, ny)
    y_a = Y - h
    if u_c is not None:
        Gx = u_c * (mu_l + mu_g) / (h * h)
    else:
        fine = np.linspace(-h, h, 200001)
        Gx = u_max / np.max(np.abs(poiseuille_profile(fine, h, mu_l, mu_g, 1.0)))
    c = _base("layered_poiseuille", nx, ny, WALL, WALL, visc_law, ratio, 1.0, nu_l, nu_g,
              sigma, W, M, Gx=Gx)
    c["phi0"] = tanh_profile(h - Y, W)
    ua = poiseuille_profile(y_a, h, mu_l, mu_g, Gx)
    c["ux_analytic"] = ua
    c["ux0"] = ua.copy() if init == "analytic" else np.zeros((ny, nx))
    c["uy0"] = np.zeros((ny, nx))
    c["u_scale"] = float(np.max(np.abs(ua)))
    # the dynamic pressure of the flow, rho_l u_max^2 (the pressure itself varies only by
    # about G_x ny, two orders less, so that is no scale for its rounding)
    c["p_scale"] = ratio * c["u_scale"] ** 2
    return c


def relative_error_eu(ux, ux_analytic):
    """Eq. 32 on the x-averaged numerical profile."""
    un = ux.mean(axis=1)
    ua = ux_analytic.mean(axis=1)
    return float(np.sum(np.abs(un - ua)) / np.sum(np.abs(ua)))


def droplet_impact(nx=2048, ny=512, D=256.0, Re=100.0, We=8000.0, U=0.05, ratio=1000.0, W=5.0,
                   M=0.1, film=0.1, nu_ratio_at_re500=10.0):
    """Sec. 3.4: a drop of diameter D moving down at U onto a liquid film of height film * D
    on a bounce-back floor; an open top (held at the ambient pressure); periodic in x.
    Re = D U / nu_l (Eq. 38) sets nu_l; We = rho_l D U^2 / sigma (Eq. 39) sets sigma; the gas
    viscosity is held at nu_ratio_at_re500 times the Re = 500 liquid value.  phi is the
    larger of the film profile (Eq. 35) and the drop profile (Eq. 36, drop only above the
    film), and the drop carries (0, -U phi_drop) (Eq. 37)."""
    R = D / 2.0
    Hw = film * D
    nu_l = D * U / Re
    nu_g = nu_ratio_at_re500 * D * U / 500.0
    sigma = ratio * D * U * U / We
    c = _base("droplet_impact", nx, ny, WALL, OPEN, NU_LINEAR, ratio, 1.0, nu_l, nu_g, sigma,
              W, M)
    X, Y = _grid(nx, ny)
    xc, yc = nx / 2.0, Hw + R
    r = np.sqrt((X - xc) ** 2 + (Y - yc) ** 2)
    above = Y > Hw
    phi_film = tanh_profile(Hw - Y, W)
    phi_drop = np.where(above, tanh_profile(R - r, W), 0.0)
    c["phi0"] = np.maximum(phi_film, phi_drop)
    c["ux0"] = np.zeros((ny, nx))
    c["uy0"] = np.where(above, -U * phi_drop, 0.0)
    c.update(D=float(D), U=float(U), Re=float(Re), We=float(We), Hw=float(Hw))
    c["u_scale"] = U
    c["p_scale"] = ratio * U * U
    y_row = int(np.floor(Hw + W))
    c["mask"] = (xc, yc, 0.0, 0.0, float(y_row))
    return c


def batch_ensemble(n=256, seed=1, lo=32, hi=512):
    """Many independent instances of uneven size: each is a static drop or a layered
    Poiseuille channel with density ratio drawn from {10, 100, 1000}; grids uniform in
    [lo, hi] on each axis.  Drops: R = r min(nx, ny), r ~ U[0.15, 0.35], W = 4,
    sigma = 0.01, nu = 0.1, M = 0.1.  Channels: W = 5, sigma = 0.001, nu_l = 0.1,
    nu_g / nu_l = 10 at ratio 1000 else 1, u_max = 1e-3, analytic start, step mu, and
    an even row count (ny rounded up)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nx, ny = (int(v) for v in rng.integers(lo, hi + 1, size=2))
        is_drop = bool(rng.random() < 0.5)
        ratio = float(rng.choice([10.0, 100.0, 1000.0]))
        r = float(rng.uniform(0.15, 0.35))
        if is_drop:
            out.append(static_drop(nx, ny, R=r * min(nx, ny), W=4.0, ratio=ratio, sigma=0.01,
                                   nu=0.1, M=0.1))
        else:
            # an even number of rows puts the interface between two nodes; with an odd
            # number a node would sit exactly on phi = 0.5, where the step viscosity law
            # switches and rounding alone decides the branch
            ny += ny % 2
            nu_g = 1.0 if ratio == 1000.0 else 0.1
            out.append(layered_poiseuille(nx, ny, ratio=ratio, nu_l=0.1, nu_g=nu_g, W=5.0,
                                          sigma=0.001, M=0.1, u_max=1e-3))
    return out


def taylor_green(n=32, nu=0.05, u0=1e-3, m=1):
    """Single-phase check: rho_l = rho_g, sigma = 0, phi = 1, the decaying vortex
    u = u0 (-cos kx sin ky, sin kx cos ky) with k = 2 pi m / n."""
    c = _base("taylor_green", n, n, PERIODIC, PERIODIC, NU_LINEAR, 1.0, 1.0, nu, nu, 0.0, 4.0,
              0.1)
    X, Y = _grid(n, n)
    k = 2.0 * np.pi * m / n
    c["phi0"] = np.ones((n, n))
    c["ux0"] = -u0 * np.cos(k * X) * np.sin(k * Y)
    c["uy0"] = u0 * np.sin(k * X) * np.cos(k * Y)
    c["k"] = k
    c["u_scale"] = u0
    c["p_scale"] = u0 * u0
    return c


def planar_interface(nx=8, ny=64, W=4.0, ratio=1000.0, sigma=0.01, nu=0.1, M=0.1, ux=0.0,
                     uy=0.0, bc=PERIODIC):
    """A flat liquid layer between y = ny/4 and 3ny/4 (two tanh interfaces, Eq. 33 form),
    optionally translating with a uniform velocity."""
    c = _base("planar", nx, ny, bc, bc, NU_LINEAR, ratio, 1.0, nu, nu, sigma, W, M)
    X, Y = _grid(nx, ny)
    d = np.minimum(Y - ny / 4.0, 3.0 * ny / 4.0 - Y)
    c["phi0"] = tanh_profile(d, W)
    c["ux0"] = np.full((ny, nx), float(ux))
    c["uy0"] = np.full((ny, nx), float(uy))
    c["u_scale"] = max(abs(ux), abs(uy), 1e-6)
    c["p_scale"] = sigma / W
    return c


def random_state_case(nx=4, ny=4, bc=PERIODIC, seed=0, visc_law=NU_LINEAR):
    """Tiny grid with random phi in [0.2, 0.8] and random u of size 1e-2, for brute-force
    comparisons of a few steps."""
    rng = np.random.default_rng(seed)
    c = _base("random", nx, ny, bc, bc, visc_law, 10.0, 1.0, 0.1, 0.3, 0.01, 3.0, 0.05,
              Gx=1e-5, Gy=-2e-5)
    c["phi0"] = rng.uniform(0.2, 0.8, size=(ny, nx))
    c["ux0"] = rng.uniform(-1e-2, 1e-2, size=(ny, nx))
    c["uy0"] = rng.uniform(-1e-2, 1e-2, size=(ny, nx))
    c["u_scale"] = 1e-2
    c["p_scale"] = 1e-2
    return c
