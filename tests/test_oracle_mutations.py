"""Planted mistakes in the oracle (CPU only).

Each mutant is a copy of oracle/lbm_oracle.c with one plausible slip: a dropped term, a
flipped sign, a transposed index, a wrong constant or a missed boundary rule.  It is
built with the oracle's own flags and loaded in a separate process (ORACLE_LIB), where the
oracle's pins run against it; every mutant must make at least one pin fail.  An unaltered
copy, built and loaded the same way, must pass, so a failure is the mutant's doing.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, what the slip breaks, text in lbm_oracle.c, replacement)
MUTANTS = [
    ("fsource_drops_dt_phi_u", "Eq. 11: the d_t(phi u) term of F_i",
     "double vx = dtx * INV_CS2 + lambda * nx_;\n    double vy = dty * INV_CS2 + lambda * ny_;",
     "double vx = lambda * nx_;\n    double vy = lambda * ny_;"),
    ("fsource_prefactor", "Eq. 11: (1 - 1/(2 tau_phi)) taken as (1 - 1/tau_phi)",
     "(1.0 - 1.0 / (2.0 * tau_f))", "(1.0 - 1.0 / tau_f)"),
    ("mu_laplacian_sign", "Eq. 6: sign of the k lap(phi) term",
     "- s->kappa * lap;  /* Eq. 6 */", "+ s->kappa * lap;  /* Eq. 6 */"),
    ("lambda_factor", "Eq. 3: the factor 4 of lambda",
     "4.0 * phi * (1.0 - phi) / p->W;", "phi * (1.0 - phi) / p->W;"),
    ("velocity_drops_half_force", "Eq. 22a: the F/2 of rho u",
     "o->ux = (mx + 0.5 * o->Fx) / o->rho;", "o->ux = mx / o->rho;"),
    ("pressure_prefactor", "Eq. 22b: c_s^2 / (1 - w_0) = 0.6",
     "o->p = 0.6 * (", "o->p = 0.5 * ("),
    ("gradient_transposed", "Eq. 27: c_y used for the x component",
     "sx += WGT[i] * CX[i] * v;", "sx += WGT[i] * CY[i] * v;"),
    ("laplacian_factor", "Eq. 28: the factor 2 of the Laplacian",
     "sl += 2.0 * WGT[i] * (v - c);", "sl += WGT[i] * (v - c);"),
    ("geq_rest_sign", "Eq. 16: sign of (w_0 - 1) in g_0^eq",
     "out[0] = p * INV_CS2 * (WGT[0] - 1.0)", "out[0] = p * INV_CS2 * (1.0 - WGT[0])"),
    ("s_quadratic_coefficient", "Eq. 17: (c.u)^2 / (2 c_s^4) = 4.5 (c.u)^2",
     "cu * cu * 4.5", "cu * cu * 3.0"),
    ("gforce_drops_density_jump", "Eq. 20: the (rho_l - rho_g) u.grad(phi) term of G_i",
     "(cF * INV_CS2 + drho * cu * cgp * INV_CS2)", "(cF * INV_CS2)"),
    ("tau_g_offset", "Eq. 23: tau = nu / c_s^2 + 1/2",
     "o->tau_g = nu * INV_CS2 + 0.5;", "o->tau_g = nu * INV_CS2 + 1.0;"),
    ("inverse_viscosity_swapped", "Eq. 25: the phases swapped",
     "return 1.0 / (phi * (1.0 / p->nu_l - 1.0 / p->nu_g) + 1.0 / p->nu_g);",
     "return 1.0 / (phi * (1.0 / p->nu_g - 1.0 / p->nu_l) + 1.0 / p->nu_l);"),
    ("bounce_back_same_slot", "half-way bounce-back: g returns in its own slot",
     "s->gn[AT(OPP[i], y, x, nx, ny)] = gpost[i];", "s->gn[AT(i, y, x, nx, ny)] = gpost[i];"),
    ("open_side_not_filled", "open side: incoming g not filled from the edge row",
     "s->gn[AT(i, ny - 1, x, nx, ny)] =\n                    s->gn[AT(i, ny - 2, x, nx, ny)]",
     "s->gn[AT(i, ny - 1, x, nx, ny)] =\n                    0.0 * s->gn[AT(i, ny - 2, x, nx, ny)]"),
    ("open_side_pressure_free", "open side: g copied with the source's own pressure (zero gradient)",
     "s->gn[AT(i, ny - 2, x, nx, ny)] + (P_AMBIENT - s->p_edge[nx + xs]) * INV_CS2 * WGT[i];",
     "s->gn[AT(i, ny - 2, x, nx, ny)];"),
    ("open_side_pressure_of_receiver", "open side: the receiving node's pressure, not the source's",
     "(P_AMBIENT - s->p_edge[nx + xs])", "(P_AMBIENT - s->p_edge[nx + x])"),
    ("eq29_normal_sign", "Eq. 29: n = -C / |C| taken as +C / |C|",
     "*nx_ = -cx / cmag;\n        *ny_ = -cy / cmag;",
     "*nx_ = cx / cmag;\n        *ny_ = cy / cmag;"),
    ("d2q5_weight", "D2Q5 phase field: the moving weights 1/6",
     "{1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0}",
     "{1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 5.0}"),
]

# the pins, less the three slow long runs
PIN_SELECTION = ("not spurious_velocity and not spreading_power_law and not test_laplace_law "
                 "and not runs_to_t5")


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    with open(obuild.SRC) as fh:
        src = fh.read()
    d = tmp_path_factory.mktemp("mutants")
    jobs = {"unaltered": src}
    for name, _, old, new in MUTANTS:
        assert src.count(old) == 1, "mutation site of %s not found once" % name
        jobs[name] = src.replace(old, new)

    def one(item):
        name, text = item
        c = d / (name + ".c")
        c.write_text(text)
        return name, obuild.build(src=str(c), out=str(d / ("lib_" + name + ".so")))

    with ThreadPoolExecutor(max_workers=4) as ex:
        return dict(ex.map(one, jobs.items()))


def _run_pins(lib, stop_at_first):
    env = dict(os.environ, ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    cmd = [sys.executable, "-m", "pytest", "tests/test_oracle_pins.py", "-q", "-p",
           "no:cacheprovider", "-k", PIN_SELECTION] + (["-x"] if stop_at_first else [])
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_unaltered_copy_passes_the_pins(builds):
    r = _run_pins(builds["unaltered"], stop_at_first=True)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-2000:]


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_mutant_fails_a_pin(name, builds):
    r = _run_pins(builds[name], stop_at_first=True)
    # exit status 1: tests ran and at least one failed (not a collection or usage error)
    assert r.returncode == 1, (name, r.returncode, r.stdout[-2000:] + r.stderr[-2000:])
    failed = [l for l in r.stdout.splitlines() if l.startswith("FAILED")]
    print("[mutant] %-28s caught by %s" % (name, failed[0].split()[1] if failed else "?"))
