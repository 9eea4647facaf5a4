"""Helpers shared by the GPU parity tests: run a case on the oracle and on the HIP library
and measure the max-norm error of each field, normalised as
    E_q = max |q - q_oracle| / max(max |q_oracle|, q_scale)
with q_scale = 1 for phi, u_scale for u and p_scale for p (set per case)."""
import os

import numpy as np

from oracle.oracle import OracleSim
from paper_1710_09541_amd import lbm

TOL = {"f64": 1e-12, "f32": 1e-5, "f16": 1e-3}


def paper_value(key):
    """A number the paper prints, from tests/golden/paper_values.txt (with its citation)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if parts and not parts[0].startswith("#") and parts[0] == key:
                return float(parts[1])
    raise KeyError(key)


def run_oracle(case, steps):
    s = OracleSim(case, case["phi0"], case["ux0"], case["uy0"])
    s.step(steps)
    return s.moments()


def run_hip(case, steps, storage, **kw):
    with lbm.Simulation(case, storage=storage, **kw) as sim:
        sim.step(steps)
        return sim.moments()


def errors(case, got, ref):
    u_ref = np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2)
    scale_u = max(float(u_ref.max()), case["u_scale"])
    e = {
        "phi": float(np.max(np.abs(got["phi"] - ref["phi"]))) / max(float(np.abs(ref["phi"]).max()), 1.0),
        "u": max(float(np.max(np.abs(got["ux"] - ref["ux"]))),
                 float(np.max(np.abs(got["uy"] - ref["uy"])))) / scale_u,
        "p": float(np.max(np.abs(got["p"] - ref["p"]))) / max(float(np.abs(ref["p"]).max()), case["p_scale"]),
        "rho": float(np.max(np.abs(got["rho"] - ref["rho"]) / ref["rho"])),
    }
    return e


def perturbed(case, steps, eps=1e-7, seed=5):
    """The oracle's moments after `steps` from phi0 perturbed by relative noise of size eps."""
    rng = np.random.default_rng(seed)
    phi = case["phi0"] * (1.0 + eps * rng.standard_normal(case["phi0"].shape))
    s = OracleSim(case, phi, case["ux0"], case["uy0"])
    s.step(steps)
    return s.moments()


def sensitivity(case, steps, eps=1e-7, seed=5):
    """Errors of the oracle against itself when phi0 is perturbed by relative noise of size
    eps (about the rounding of a 32-bit store).  Where the interface normal is taken at a
    point of vanishing gradient (the centre of a symmetric drop, the midpoint between
    periodic images) the direction of n = grad phi / |grad phi| is set by rounding, so a
    result can be no closer to the oracle than this spread."""
    rng = np.random.default_rng(seed)
    phi = case["phi0"] * (1.0 + eps * rng.standard_normal(case["phi0"].shape))
    s = OracleSim(case, phi, case["ux0"], case["uy0"])
    s.step(steps)
    return errors(case, s.moments(), run_oracle(case, steps))


def report(name, storage, e):
    print("[parity] %-28s %-4s phi %.2e  u %.2e  p %.2e  rho %.2e  (tol %.0e)"
          % (name, storage, e["phi"], e["u"], e["p"], e["rho"], TOL[storage]), flush=True)
