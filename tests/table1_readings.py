"""E_u of the layered Poiseuille flow (Sec. 3.2, Eqs. 31-33, Table 1) under the readings of
the set-up the paper leaves open, computed with the FP64 oracle.

Not a test: a script (python -m tests.table1_readings) that prints the table quoted in the
design notes.  Every number comes from oracle/ on inputs built by the case generators.

The paper's set-up: N_y x N_x = 100 x 10, walls at the bottom and top (half-way
bounce-back), liquid in the lower half, u_c = 1e-4, W = 5, sigma = 1e-3, nu_l = 0.1,
M = 0.1, nu_g / nu_l = 1 at density ratios 10, 100, 150 and 10 at ratio 1000, dynamic
viscosity by Eq. 26.  The flow is x-invariant, so 4 columns stand for the 10.
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RATIOS = (10.0, 100.0, 150.0, 1000.0)
PAPER = {10.0: 8.9e-3, 100.0: 6.9e-3, 150.0: 5.4e-3, 1000.0: 3.2e-2}
STEADY = 200000

# reading -> (description, steps, start, node-centred, viscosity law, normal scheme)
READINGS = [
    ("steady", "cell-centred nodes (interface between nodes 49 and 50), steady state, "
     "started from the profile of Eq. 31", STEADY, "analytic", False, "step", 0),
    ("rest", "as steady, started from rest", STEADY, "rest", False, "step", 0),
    ("rest_2e4", "started from rest, E_u after 20,000 steps", 20000, "rest", False, "step", 0),
    ("rest_5e4", "started from rest, E_u after 50,000 steps", 50000, "rest", False, "step", 0),
    ("node", "node-centred y_j = j (Eq. 33 with integer y puts a node on phi = 0.5, which "
     "Eq. 26 gives mu_l), walls half a node outside, steady", STEADY, "analytic", True,
     "step", 0),
    ("eq29", "as steady, with the normal of Eq. 29 in the phase-field source", STEADY,
     "analytic", False, "step", 1),
    ("linear_nu", "as steady, linear nu (Eq. 24) instead of Eq. 26", STEADY, "analytic", False,
     "linear", 0),
    ("inverse_nu", "as steady, 1/nu linear (Eq. 25) instead of Eq. 26", STEADY, "analytic",
     False, "inverse", 0),
]


def case_for(ratio, start, node_centred, law, scheme):
    from paper_1710_09541_amd import cases
    nu_g = 1.0 if ratio == 1000.0 else 0.1
    vl = {"step": cases.MU_STEP, "linear": cases.NU_LINEAR, "inverse": cases.NU_INVERSE}[law]
    c = cases.layered_poiseuille(nx=4, ny=100, ratio=ratio, nu_l=0.1, nu_g=nu_g, W=5.0,
                                 sigma=1e-3, M=0.1, u_c=1e-4, init=start, visc_law=vl)
    c["grad_scheme"] = scheme
    if node_centred:
        # node j at y = j; the interface of Eq. 33 at y = N_y / 2 = 50 sits on node 50; the
        # profile of Eq. 31 is taken about that interface with h = N_y / 2
        y = np.arange(100, dtype=float)[:, None] * np.ones((1, 4))
        c["phi0"] = cases.tanh_profile(50.0 - y, 5.0)
        mu_l, mu_g = ratio * 0.1, nu_g
        ua = cases.poiseuille_profile(y - 50.0, 50.0, mu_l, mu_g, c["Gx"])
        c["ux_analytic"] = ua
        c["ux0"] = ua.copy() if start == "analytic" else np.zeros_like(ua)
    return c


def one(job):
    key, ratio = job
    os.environ["OMP_NUM_THREADS"] = "1"
    sys.path.insert(0, ROOT)
    from oracle.oracle import OracleSim
    from paper_1710_09541_amd import cases
    _, _, steps, start, node, law, scheme = next(r for r in READINGS if r[0] == key)
    c = case_for(ratio, start, node, law, scheme)
    s = OracleSim(c, c["phi0"], c["ux0"], c["uy0"])
    s.step(steps)
    return key, ratio, cases.relative_error_eu(s.moments()["ux"], c["ux_analytic"])


def main():
    jobs = [(r[0], ratio) for r in READINGS for ratio in RATIOS]
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        res = {(k, ratio): eu for k, ratio, eu in pool.map(one, jobs)}
    print("| reading | " + " | ".join("ratio %g" % r for r in RATIOS) + " |")
    print("|---|" + "---|" * len(RATIOS))
    print("| Table 1, present model | " + " | ".join("%.1e" % PAPER[r] for r in RATIOS) + " |")
    for key, desc, *_ in READINGS:
        print("| %s: %s | " % (key, desc) + " | ".join("%.2e" % res[(key, r)] for r in RATIOS)
              + " |")


if __name__ == "__main__":
    main()
