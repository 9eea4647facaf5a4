"""Host-only checks of the C-ABI library: it loads, exports every entry point the header
declares, its ctypes structures match the C layout, and parameter validation reports
errors before touching a device (so these run without a GPU)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1710_09541_amd import cases, lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(lbm_\w+)\s*\(", text, re.M)))


def test_header_declares_the_binding_names():
    assert declared_functions() == sorted(lbm.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = lbm.load()
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (lbm_\w+)", out))
    assert set(declared_functions()) <= exported


def _c_layout(struct, fields, tmp_path):
    src = tmp_path / "layout.c"
    body = "".join('printf("%s %%zu\\n", offsetof(%s, %s));\n' % (f, struct, f) for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lbm.h"\nint main(void){\n'
                   + body + 'printf("sizeof %%zu\\n", sizeof(%s));\nreturn 0;}\n' % struct)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return dict((k, int(v)) for k, v in (line.split() for line in out.strip().splitlines()))


@pytest.mark.parametrize("cls", [lbm.lbm_params, lbm.lbm_options, lbm.lbm_diag])
def test_ctypes_layout_matches_header(cls, tmp_path):
    fields = [f for f, _ in cls._fields_ if not f.startswith("reserved")]
    lay = _c_layout(cls.__name__, fields, tmp_path)
    for f in fields:
        assert getattr(cls, f).offset == lay[f], f
    assert C.sizeof(cls) == lay["sizeof"]


def _init(case, **kw):
    return lbm.lbm_init([lbm.make_params(case)], lbm.make_options(**kw), [case["phi0"]],
                        [case["ux0"]], [case["uy0"]])


@pytest.mark.parametrize("key,value", [("nx", 2), ("ny", 1), ("rho_g", 0.0), ("W", 0.0),
                                       ("M", -1.0), ("nu_l", 0.0), ("visc_law", 9), ("grad_scheme", 2), ("f_lattice", 7),
                                       ("sigma", -1.0), ("Gx", float("nan"))])
def test_invalid_parameters_rejected_before_device(key, value):
    c = cases.static_drop(16, 16, R=4)
    c[key] = value
    if key in ("nx", "ny"):   # fields of the shape the parameters name reach the library
        for k in ("phi0", "ux0", "uy0"):
            c[k] = np.zeros((c["ny"], c["nx"]))
    with pytest.raises(lbm.LbmError) as e:
        _init(c)
    assert e.value.code == lbm.LBM_ERR_PARAM
    assert lbm.lbm_last_error()


def test_invalid_boundary_and_options_rejected():
    c = cases.static_drop(16, 16, R=4)
    c["bc_ylo"] = lbm.LBM_BC_WALL           # periodic on one side only
    with pytest.raises(lbm.LbmError) as e:
        _init(c)
    assert e.value.code == lbm.LBM_ERR_PARAM and "periodic" in lbm.lbm_last_error()
    c = cases.static_drop(16, 16, R=4)
    for kw in ({"storage": 7}, {"tile_rows": 5}, {"kernel": 9}, {"check_every": -1},
               {"stores": 3}, {"grid": 3}, {"grid": -1}, {"strip": 4}, {"strip": -2},
               {"deal": -2}, {"deal": 4097}):
        with pytest.raises(lbm.LbmError) as e:
            _init(c, **kw)
        assert e.value.code == lbm.LBM_ERR_PARAM


@pytest.mark.parametrize("storage,n", [("f64", 7744), ("f32", 10944), ("f16", 15488)])
def test_instance_beyond_4gib_rejected_before_device(storage, n):
    """One instance's 9 population planes must stay below 4 GiB (the buffer addressing
    uses 32-bit byte offsets); the next multiple of 64 above the largest admitted grid is
    refused before any device call."""
    c = cases.static_drop(16, 16, R=4)
    c["nx"] = c["ny"] = n
    for k in ("phi0", "ux0", "uy0"):
        c[k] = np.zeros((n, n))
    with pytest.raises(lbm.LbmError) as e:
        _init(c, storage=storage)
    assert e.value.code == lbm.LBM_ERR_PARAM
    assert "too large" in lbm.lbm_last_error()


def test_null_context_calls():
    L = lbm.load()
    assert L.lbm_step(None, 1) == lbm.LBM_ERR_PARAM
    assert L.lbm_info(None, None, None, None, None, None, None, None, None) == lbm.LBM_ERR_PARAM
    assert L.lbm_reduce(None, 0, None, None) == lbm.LBM_ERR_PARAM
    assert L.lbm_reduce_noalloc(None, 0, None, None) == lbm.LBM_ERR_PARAM
    L.lbm_destroy(None)
    assert lbm.lbm_last_error()


def test_no_device_reported_as_device_error():
    """On a machine without a GPU a valid parameter set fails with LBM_ERR_DEVICE."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    c = cases.static_drop(16, 16, R=4)
    with pytest.raises(lbm.LbmError) as e:
        _init(c)
    assert e.value.code == lbm.LBM_ERR_DEVICE


def test_mixed_phase_field_lattices_rejected():
    a = cases.static_drop(16, 16, R=4)
    b = cases.static_drop(16, 16, R=4)
    b["f_lattice"] = cases.D2Q5
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_init([lbm.make_params(a), lbm.make_params(b)], lbm.make_options(),
                     [a["phi0"], b["phi0"]], [a["ux0"], b["ux0"]], [a["uy0"], b["uy0"]])
    assert e.value.code == lbm.LBM_ERR_PARAM
    assert "lattice" in lbm.lbm_last_error()


@pytest.mark.parametrize("field", ["phi0", "ux0", "uy0"])
def test_initial_field_of_wrong_shape_refused(field):
    """The library reads ny * nx values of each initial field; the binding refuses any other
    shape (the transpose included) before calling it."""
    c = cases.static_drop(16, 24, R=4)
    assert c[field].shape == (24, 16)
    for bad in (c[field][:-1], c[field].T, c[field].ravel()):
        d = dict(c)
        d[field] = bad
        with pytest.raises(ValueError, match="expected"):
            lbm.lbm_init([lbm.make_params(d)], lbm.make_options(), [d["phi0"]], [d["ux0"]],
                         [d["uy0"]])


def test_reduce_mask_length_checked():
    with pytest.raises(ValueError, match="5 values"):
        lbm.lbm_reduce(None, 0, mask=(0.0, 0.0, 1.0))


def test_missing_library_fails_loudly(monkeypatch):
    """Without the built HIP library the binding raises; nothing falls back to another
    implementation."""
    monkeypatch.setattr(lbm, "_lib", None)
    monkeypatch.setattr(lbm, "LIB_PATH", "/nonexistent/liblbm_hip.so")
    with pytest.raises(RuntimeError, match="not built"):
        lbm.load()
    c = cases.static_drop(8, 8, R=2)
    with pytest.raises(RuntimeError):
        lbm.Simulation(c, storage="f64")


def test_build_id_matches_the_sources():
    """The library carries the sha256 of the sources it was built from (lbm_build_id), and
    the binding loads it only if that equals the hash of the sources beside it."""
    from paper_1710_09541_amd import build
    lbm.load()
    bid = lbm.build_id()
    assert re.fullmatch(r"[0-9a-f]{64}", bid)
    assert bid == build.source_hash()


def test_stale_build_refused(monkeypatch):
    """A library whose build id differs from the sources' hash is refused at load."""
    from paper_1710_09541_amd import build
    monkeypatch.setattr(build, "source_hash", lambda: "0" * 64)
    monkeypatch.setattr(lbm, "_lib", None)
    with pytest.raises(RuntimeError, match="other sources"):
        lbm.load()
