"""ctypes binding of liblbm_hip.so (the C-ABI in include/lbm.h).

Argument marshalling only: every step of the computation runs in the HIP library.  The
functions keep the C names (lbm_init, lbm_step, ...); ``Simulation`` wraps one context.
Loading fails loudly if the library has not been built.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_hip.so")

LBM_OK, LBM_ERR_PARAM, LBM_ERR_ALLOC, LBM_ERR_DEVICE, LBM_ERR_NONFINITE, LBM_ERR_RANGE = (
    0, -1, -2, -3, -4, -5)
LBM_BC_PERIODIC, LBM_BC_WALL, LBM_BC_OPEN = 0, 1, 2
LBM_VISC_LINEAR, LBM_VISC_INVERSE, LBM_VISC_STEP_MU = 0, 1, 2
LBM_STORE_F64, LBM_STORE_F32, LBM_STORE_F16 = 0, 1, 2
LBM_KERNEL_AUTO, LBM_KERNEL_FUSED, LBM_KERNEL_SPLIT = 0, 1, 2
LBM_GRAD_ISOTROPIC, LBM_GRAD_LOCAL_NEQ = 0, 1
LBM_LATTICE_D2Q9, LBM_LATTICE_D2Q5 = 9, 5
LBM_EXP_AUTO = -1000

STORAGE = {"f64": LBM_STORE_F64, "f32": LBM_STORE_F32, "f16": LBM_STORE_F16}
KERNEL = {"auto": LBM_KERNEL_AUTO, "fused": LBM_KERNEL_FUSED, "split": LBM_KERNEL_SPLIT}

EXPORTS = ("lbm_init", "lbm_step", "lbm_moments", "lbm_moments_device", "lbm_reduce",
           "lbm_reduce_noalloc", "lbm_get_state", "lbm_set_state", "lbm_info", "lbm_build_id",
           "lbm_last_error", "lbm_destroy")


class lbm_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32),
                ("bc_ylo", C.c_int32), ("bc_yhi", C.c_int32),
                ("visc_law", C.c_int32), ("grad_scheme", C.c_int32),
                ("rho_l", C.c_double), ("rho_g", C.c_double),
                ("nu_l", C.c_double), ("nu_g", C.c_double),
                ("sigma", C.c_double), ("W", C.c_double), ("M", C.c_double),
                ("Gx", C.c_double), ("Gy", C.c_double),
                ("exp_f", C.c_int32), ("exp_g", C.c_int32),
                ("f_lattice", C.c_int32), ("reserved1", C.c_int32)]


class lbm_options(C.Structure):
    _fields_ = [("storage", C.c_int32), ("kernel", C.c_int32), ("tile_rows", C.c_int32),
                ("use_graph", C.c_int32), ("check_every", C.c_int32),
                ("stores", C.c_int32), ("grid", C.c_int32), ("strip", C.c_int32),
                ("narrow_tiles", C.c_int32), ("deal", C.c_int32)]


class lbm_diag(C.Structure):
    _fields_ = [("sum_phi", C.c_double), ("sum_rho", C.c_double), ("kinetic", C.c_double),
                ("max_u", C.c_double), ("min_rho", C.c_double), ("min_phi", C.c_double),
                ("max_phi", C.c_double), ("p_in", C.c_double), ("p_out", C.c_double),
                ("interface_crossings", C.c_double), ("spread_radius", C.c_double),
                ("nonfinite", C.c_int64), ("step", C.c_int64)]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("lbm error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load():
    """Loads liblbm_hip.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblbm_hip.so is not built; run `python -m paper_1710_09541_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname; loading it first makes the
    # library and torch share one runtime, so torch streams and device pointers are valid
    # arguments.  (Loaded the other way round, the process would hold two runtimes.)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P, D = C.POINTER, C.POINTER(C.c_double)
    L.lbm_init.argtypes = [P(lbm_params), C.c_int32, P(lbm_options), P(D), P(D), P(D),
                           C.c_void_p, P(C.c_void_p)]
    L.lbm_step.argtypes = [C.c_void_p, C.c_int64]
    L.lbm_moments.argtypes = [C.c_void_p, C.c_int32, D, D, D, D, D]
    L.lbm_moments_device.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
    L.lbm_reduce.argtypes = [C.c_void_p, C.c_int32, D, P(lbm_diag)]
    L.lbm_reduce_noalloc.argtypes = [C.c_void_p, C.c_int32, D, P(lbm_diag)]
    L.lbm_get_state.argtypes = [C.c_void_p, C.c_void_p, P(C.c_size_t)]
    L.lbm_set_state.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
    L.lbm_info.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int32), P(C.c_int32), P(C.c_int32),
                           P(C.c_int32), P(C.c_int32), P(C.c_int32), P(C.c_int32)]
    L.lbm_last_error.argtypes = [C.c_void_p]
    L.lbm_last_error.restype = C.c_char_p
    L.lbm_destroy.argtypes = [C.c_void_p]
    L.lbm_destroy.restype = None
    L.lbm_build_id.argtypes = []
    L.lbm_build_id.restype = C.c_char_p
    from . import build as _build
    built, here = L.lbm_build_id().decode(), _build.source_hash()
    if built != here:
        raise RuntimeError("liblbm_hip.so was built from other sources (build id %s, sources "
                           "%s); rebuild with `python -m paper_1710_09541_amd.build`"
                           % (built[:16], here[:16]))
    _lib = L
    return L


def build_id() -> str:
    """sha256 of the sources the loaded library was built from (equal to the sources'
    own, which load() checks)."""
    return load().lbm_build_id().decode()


def _check(rc, ctx=None):
    if rc != LBM_OK:
        msg = load().lbm_last_error(ctx)
        raise LbmError(rc, msg.decode() if msg else "")


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(case, exp_f=LBM_EXP_AUTO, exp_g=LBM_EXP_AUTO) -> lbm_params:
    p = lbm_params()
    p.nx, p.ny = int(case["nx"]), int(case["ny"])
    p.bc_ylo, p.bc_yhi = int(case["bc_ylo"]), int(case["bc_yhi"])
    p.visc_law = int(case["visc_law"])
    p.grad_scheme = int(case.get("grad_scheme", 0))
    for k in ("rho_l", "rho_g", "nu_l", "nu_g", "sigma", "W", "M", "Gx", "Gy"):
        setattr(p, k, float(case[k]))
    p.exp_f, p.exp_g = int(exp_f), int(exp_g)
    p.f_lattice = int(case.get("f_lattice", 9))
    return p


STORES = {"auto": 0, "cached": 1, "streaming": 2}
GRID = {"auto": 0, "tiles": 1, "persistent": 2}
STRIP = {"auto": 0, "rows": -1}
NARROW = {"auto": 0, "off": -1, "on": 1}
DEAL = {"auto": 0, "bands": -1}   # or a chunk of 1 to 4096 tiles


def make_options(storage="f32", kernel="auto", tile_rows=0, use_graph=True, check_every=0,
                 stores="auto", grid="auto", strip="auto", narrow="auto", deal="auto"):
    o = lbm_options()
    o.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    o.kernel = KERNEL[kernel] if isinstance(kernel, str) else int(kernel)
    o.tile_rows = int(tile_rows)
    o.use_graph = 1 if use_graph else 0
    o.check_every = int(check_every)
    o.stores = STORES[stores] if isinstance(stores, str) else int(stores)
    o.grid = GRID[grid] if isinstance(grid, str) else int(grid)
    o.strip = STRIP[strip] if isinstance(strip, str) else int(strip)
    o.narrow_tiles = NARROW[narrow] if isinstance(narrow, str) else int(narrow)
    o.deal = DEAL[deal] if isinstance(deal, str) else int(deal)
    return o


def lbm_init(params, options, phi0, ux0, uy0, stream=None):
    """params: list of lbm_params; phi0/ux0/uy0: lists of float64 [ny][nx] arrays.
    Returns the context handle (c_void_p)."""
    L = load()
    n = len(params)
    arr = (lbm_params * n)(*params)
    fields = list(phi0) + list(ux0) + list(uy0)
    if len(fields) != 3 * n:
        raise ValueError("need one phi0, ux0 and uy0 per instance")
    keep = [np.ascontiguousarray(a, dtype=np.float64) for a in fields]
    for j, a in enumerate(keep):
        p = params[j % n]
        # the library reads exactly ny * nx values of each field
        if a.shape != (p.ny, p.nx):
            raise ValueError("instance %d: initial field has shape %s, expected (ny, nx) = (%d, %d)"
                             % (j % n, a.shape, p.ny, p.nx))
    ptrs = [_dptr(a) for a in keep]
    DP = C.POINTER(C.c_double) * n
    h = C.c_void_p()
    rc = L.lbm_init(arr, n, C.byref(options) if options is not None else None,
                    DP(*ptrs[:n]), DP(*ptrs[n:2 * n]), DP(*ptrs[2 * n:]),
                    C.c_void_p(stream) if stream else None, C.byref(h))
    _check(rc)
    return h


def lbm_step(ctx, n):
    _check(load().lbm_step(ctx, int(n)), ctx)


def lbm_moments(ctx, inst, nx, ny):
    out = [np.empty((ny, nx)) for _ in range(5)]
    _check(load().lbm_moments(ctx, int(inst), *[_dptr(a) for a in out]), ctx)
    return dict(zip(("phi", "rho", "p", "ux", "uy"), out))


def lbm_moments_device(ctx, inst, d_ptr):
    _check(load().lbm_moments_device(ctx, int(inst), C.c_void_p(d_ptr)), ctx)


def _reduce(fn, ctx, inst, mask):
    d = lbm_diag()
    m = None
    if mask is not None:
        m_arr = np.ascontiguousarray(mask, dtype=np.float64).ravel()
        if m_arr.size != 5:
            raise ValueError("mask is (xc, yc, r_in, r_out, y_row): 5 values")
        m = _dptr(m_arr)
    _check(fn(ctx, int(inst), m, C.byref(d)), ctx)
    return {k: getattr(d, k) for k, _ in lbm_diag._fields_}


def lbm_reduce(ctx, inst, mask=None):
    return _reduce(load().lbm_reduce, ctx, inst, mask)


def lbm_reduce_noalloc(ctx, inst, mask=None):
    """lbm_reduce through the library's fixed device scratch (no allocation in the call)."""
    return _reduce(load().lbm_reduce_noalloc, ctx, inst, mask)


def lbm_get_state(ctx) -> bytes:
    L = load()
    n = C.c_size_t(0)
    _check(L.lbm_get_state(ctx, None, C.byref(n)), ctx)
    buf = C.create_string_buffer(n.value)
    _check(L.lbm_get_state(ctx, buf, C.byref(n)), ctx)
    return buf.raw[:n.value]


def lbm_set_state(ctx, blob: bytes):
    buf = C.create_string_buffer(blob, len(blob))
    _check(load().lbm_set_state(ctx, buf, len(blob)), ctx)


def lbm_info(ctx):
    s, k, r, st, g, o, nw, d = (C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(),
                                C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32())
    _check(load().lbm_info(ctx, C.byref(s), C.byref(k), C.byref(r), C.byref(st), C.byref(g),
                           C.byref(o), C.byref(nw), C.byref(d)), ctx)
    return {"step": s.value, "kernel": k.value, "tile_rows": r.value,
            "stores": {1: "cached", 2: "streaming"}.get(st.value, st.value),
            "grid": {1: "tiles", 2: "persistent"}.get(g.value, g.value),
            "strip": "rows" if o.value == -1 else o.value,
            "narrow": {1: "on", -1: "off"}.get(nw.value, nw.value),
            "deal": "bands" if d.value == -1 else d.value}


def lbm_last_error(ctx=None) -> str:
    m = load().lbm_last_error(ctx)
    return m.decode() if m else ""


def lbm_destroy(ctx):
    load().lbm_destroy(ctx)


class Simulation:
    """One library context over one or more cases (dicts from ``cases``)."""

    def __init__(self, case_or_cases, storage="f32", kernel="auto", tile_rows=0,
                 use_graph=True, check_every=0, stream=None, stores="auto", grid="auto",
                 strip="auto", narrow="auto", deal="auto"):
        cs = case_or_cases if isinstance(case_or_cases, (list, tuple)) else [case_or_cases]
        self.cases = list(cs)
        params = [make_params(c) for c in self.cases]
        opts = make_options(storage, kernel, tile_rows, use_graph, check_every, stores, grid,
                            strip, narrow, deal)
        self.ctx = lbm_init(params, opts, [c["phi0"] for c in self.cases],
                            [c["ux0"] for c in self.cases], [c["uy0"] for c in self.cases],
                            stream=stream)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, n):
        lbm_step(self.ctx, n)

    def moments(self, inst=0):
        c = self.cases[inst]
        return lbm_moments(self.ctx, inst, c["nx"], c["ny"])

    def reduce(self, inst=0, mask=None):
        return lbm_reduce(self.ctx, inst, self.cases[inst]["mask"] if mask is None else mask)

    def get_state(self):
        return lbm_get_state(self.ctx)

    def set_state(self, blob):
        lbm_set_state(self.ctx, blob)

    def info(self):
        return lbm_info(self.ctx)
