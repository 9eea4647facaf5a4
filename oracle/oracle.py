"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Loaded by the tests, the smoke check and the CPU-baseline leg of the benchmark; never by
the product path.  Arrays are numpy float64, row-major [ny][nx] (x fastest).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

PERIODIC, WALL, OPEN = 0, 1, 2
NU_LINEAR, NU_INVERSE, MU_STEP = 0, 1, 2
GRAD_ISOTROPIC, GRAD_LOCAL_NEQ = 0, 1


class OrcParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("bc_ylo", C.c_int32), ("bc_yhi", C.c_int32),
                ("visc_law", C.c_int32), ("grad_scheme", C.c_int32),
                ("rho_l", C.c_double), ("rho_g", C.c_double),
                ("nu_l", C.c_double), ("nu_g", C.c_double),
                ("sigma", C.c_double), ("W", C.c_double), ("M", C.c_double),
                ("Gx", C.c_double), ("Gy", C.c_double),
                ("f_lattice", C.c_int32), ("reserved", C.c_int32)]


_lib = None
_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    """The oracle library: oracle/liblbm_oracle.so (built on first use), or the build that
    the environment variable ORACLE_LIB names (the mutation test loads altered copies)."""
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB")
        if not path:
            path = _build.LIB
            if not os.path.exists(path):
                _build.build()
        L = C.CDLL(path)
        P = C.POINTER(OrcParams)
        L.orc_check.argtypes = [P]
        L.orc_create.argtypes = [P, _D, _D, _D]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_steps_done.argtypes = [C.c_void_p]
        L.orc_steps_done.restype = C.c_int64
        L.orc_moments.argtypes = [C.c_void_p, _D, _D, _D, _D, _D]
        L.orc_get_state.argtypes = [C.c_void_p, _D, _D, _D]
        L.orc_set_state.argtypes = [C.c_void_p, _D, _D, _D]
        L.orc_lattice.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_int32), _D,
                                  C.POINTER(C.c_int32)]
        L.orc_feq.argtypes = [C.c_int32] + [C.c_double] * 3 + [_D]
        L.orc_geq.argtypes = [C.c_double] * 4 + [_D]
        L.orc_fsource.argtypes = [C.c_int32] + [C.c_double] * 6 + [_D]
        L.orc_fweights.argtypes = [C.c_int32, _D]
        L.orc_gforce.argtypes = [C.c_double] * 8 + [_D]
        L.orc_stencil.argtypes = [P, _D, _D, _D, _D]
        L.orc_closure.argtypes = [P] + [C.c_double] * 4 + [_D, _D]
        L.orc_normal_local_neq.argtypes = [C.c_int32, _D] + [C.c_double] * 5 + [_D]
        _lib = L
    return _lib


def make_params(case) -> OrcParams:
    """Builds the oracle's parameter block from a case dict (see the case generators)."""
    p = OrcParams()
    p.nx, p.ny = int(case["nx"]), int(case["ny"])
    p.bc_ylo, p.bc_yhi = int(case["bc_ylo"]), int(case["bc_yhi"])
    p.visc_law = int(case["visc_law"])
    p.grad_scheme = int(case.get("grad_scheme", GRAD_ISOTROPIC))
    p.f_lattice = int(case.get("f_lattice", 9))
    for k in ("rho_l", "rho_g", "nu_l", "nu_g", "sigma", "W", "M", "Gx", "Gy"):
        setattr(p, k, float(case[k]))
    return p


def check(case) -> int:
    return lib().orc_check(C.byref(make_params(case)))


class OracleSim:
    """One simulation on the CPU oracle."""

    def __init__(self, case, phi0, ux0, uy0):
        self.case = case
        self.params = make_params(case)
        self.nx, self.ny = self.params.nx, self.params.ny
        shape = (self.ny, self.nx)
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))
                for a in (phi0, ux0, uy0)]
        h = lib().orc_create(C.byref(self.params), *arrs)
        if not h:
            raise ValueError("oracle rejected the parameters (code %d)" % check(case))
        self._h = C.c_void_p(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and lib is not None and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    def step(self, n: int):
        lib().orc_step(self._h, int(n))

    @property
    def steps(self) -> int:
        return lib().orc_steps_done(self._h)

    def moments(self):
        """dict of phi, rho, p, ux, uy, each [ny][nx] float64 (S1-S5 on the current state)."""
        out = {k: np.empty((self.ny, self.nx)) for k in ("phi", "rho", "p", "ux", "uy")}
        lib().orc_moments(self._h, out["phi"], out["rho"], out["p"], out["ux"], out["uy"])
        return out

    def get_state(self):
        n = self.nx * self.ny
        f = np.empty(9 * n)
        g = np.empty(9 * n)
        q = np.empty(2 * n)
        lib().orc_get_state(self._h, f, g, q)
        shp = (self.ny, self.nx)
        return f.reshape((9,) + shp), g.reshape((9,) + shp), q.reshape((2,) + shp)

    def set_state(self, f, g, q):
        lib().orc_set_state(self._h, *[np.ascontiguousarray(a, dtype=np.float64).ravel()
                                       for a in (f, g, q)])


def lattice():
    cx = (C.c_int32 * 9)()
    cy = (C.c_int32 * 9)()
    opp = (C.c_int32 * 9)()
    w = np.empty(9)
    lib().orc_lattice(cx, cy, w, opp)
    return np.array(cx[:]), np.array(cy[:]), w, np.array(opp[:])


def feq(phi, ux, uy, qf=9):
    out = np.empty(9)
    lib().orc_feq(qf, phi, ux, uy, out)
    return out[:qf]


def geq(p, rho, ux, uy):
    out = np.empty(9)
    lib().orc_geq(p, rho, ux, uy, out)
    return out


def fsource(tau_f, dtx, dty, lam, nx, ny, qf=9):
    out = np.empty(9)
    lib().orc_fsource(qf, tau_f, dtx, dty, lam, nx, ny, out)
    return out[:qf]


def fweights(qf):
    """Weights of the phase-field lattice with qf velocities (c_0 .. c_{qf-1} of D2Q9)."""
    out = np.empty(9)
    lib().orc_fweights(qf, out)
    return out[:qf]


def gforce(tau_g, Fx, Fy, drho, ux, uy, dpx, dpy):
    out = np.empty(9)
    lib().orc_gforce(tau_g, Fx, Fy, drho, ux, uy, dpx, dpy, out)
    return out


def stencil(case, phi):
    p = make_params(case)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    gx, gy, lap = np.empty_like(phi), np.empty_like(phi), np.empty_like(phi)
    rc = lib().orc_stencil(C.byref(p), phi, gx, gy, lap)
    if rc != 0:
        raise ValueError("bad parameters")
    return gx, gy, lap


CLOSURE_KEYS = ("rho", "mu_phi", "lambda", "n_x", "n_y", "tau_g", "F_x", "F_y", "u_x", "u_y", "p")


def closure(case, phi, dpx, dpy, lap, g):
    out = np.empty(11)
    lib().orc_closure(C.byref(make_params(case)), phi, dpx, dpy, lap,
                      np.ascontiguousarray(g, dtype=np.float64), out)
    return dict(zip(CLOSURE_KEYS, out))


def normal_local_neq(f, phi, ux, uy, dtx, dty, qf=9):
    """Eq. 29 normal at one node from its qf phase-field populations; returns (n_x, n_y)."""
    out = np.empty(2)
    fa = np.zeros(9)
    fa[:qf] = np.asarray(f, dtype=np.float64)[:qf]
    lib().orc_normal_local_neq(qf, fa, phi, ux, uy, dtx, dty, out)
    return out
