"""Builds liblbm_hip.so (gfx950) in-tree from csrc/.

Usage: python -m paper_1710_09541_amd.build   (or build() from Python)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm_hip.so")
SOURCES = ["lbm_kernels.hip", "lbm_reduce.hip", "lbm_api.hip"]
HEADERS = [os.path.join(CSRC, "lbm_device.h"),
           os.path.join(os.path.dirname(HERE), "include", "lbm.h")]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")


def source_hash() -> str:
    """sha256 over the bytes of every file the library is built from (the three sources,
    then the two headers, in that order, each preceded by its name).  The build compiles it
    into the library, where lbm_build_id() returns it, so a loaded library can be checked
    against the sources beside it."""
    import hashlib
    h = hashlib.sha256()
    for path in [os.path.join(CSRC, s) for s in SOURCES] + HEADERS:
        h.update(os.path.basename(path).encode() + b"\0")
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, extra=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ([hipcc] + HIPCC_FLAGS + ['-DLBM_SOURCE_SHA256="%s"' % source_hash()] + list(extra)
           + srcs + ["-o", tmp])
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
