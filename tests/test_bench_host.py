"""Host-only checks of the benchmark's contract and bookkeeping (no GPU needed)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_refused_with_a_message():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_lattice_update():
    # 18 population values read and 18 written, plus the per-node state (FP64: phi u read and
    # written, 2 x 2 x 8 B; FP32: one float3 read and one written, 2 x 12 B; 16-bit: one
    # float4 read and one written, 2 x 16 B)
    assert bench.alg_bytes("f64", 9) == 36 * 8 + 32
    assert bench.alg_bytes("f32", 9) == 36 * 4 + 24
    assert bench.alg_bytes("f16", 9) == 36 * 2 + 32
    # D2Q5 phase field: 14 populations per node instead of 18
    assert bench.alg_bytes("f32", 5) == 28 * 4 + 24


def test_code_hash_ignores_comments_and_blank_space():
    a = "int f(int x) {\n    return x + 1;  // one more\n}\n"
    b = "/* a comment */\nint f(int x) {\n\n  return x + 1;\n}\n"
    c = "int f(int x) {\n    return x + 2;\n}\n"
    assert bench.code_hash(a) == bench.code_hash(b)
    assert bench.code_hash(a) != bench.code_hash(c)


def test_traffic_taken_only_from_profiles_of_the_current_kernels(tmp_path, monkeypatch):
    """roofline.traffic comes from a committed counter summary only while that summary was
    taken on the kernels as they are; otherwise it is null."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profile("spinodal1024", "f32") is None
    rec = {"kernel_source_sha256": bench.kernel_source_hash(), "hbm_bytes_per_launch": 1.5e8}
    (prof / "pmc_spinodal1024_f32.json").write_text(json.dumps(rec))
    assert bench.traffic_from_profile("spinodal1024", "f32") == 1.5e8
    rec["kernel_source_sha256"] = "0" * 16
    (prof / "pmc_spinodal1024_f32.json").write_text(json.dumps(rec))
    assert bench.traffic_from_profile("spinodal1024", "f32") is None


def test_committed_profiles_name_their_commands_and_kernel():
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        path = os.path.join(ROOT, "profiles", name)
        if name.startswith("step_"):
            text = open(path).read()
            assert "rocprofv3" in text and "Kernel code hash" in text, name
            # the device's streaming rate beside the copy that calibrates the counters
            assert "Streaming rate:" in text and "Copy calibration:" in text, name
            # the summary averages the step kernel's last `steps` dispatches, which are the
            # timed ones only when the traced bench command skips the host round trip
            traced = [l for l in text.splitlines() if "--kernel-trace" in l and "bench.py" in l
                      and "--calibrate-copy" not in l]
            assert traced and all("--no-round-trip" in l for l in traced), name
        if name.startswith("pmc_"):
            d = json.load(open(path))
            assert {"kernel", "kernel_source_sha256", "avg_duration_ns",
                    "hbm_bytes_per_launch"} <= set(d), name


def test_method_bytes_per_lattice_update():
    """The algorithmic bytes of the roofline: 18 population values read and 18 written, phi
    written and read once and phi u of the previous step (two values) read and written once;
    phi and phi u in FP64 for the FP64 format and in FP32 otherwise."""
    assert bench.method_bytes("f64", 9) == 36 * 8 + 6 * 8 == 336
    assert bench.method_bytes("f32", 9) == 36 * 4 + 6 * 4 == 168
    assert bench.method_bytes("f16", 9) == 36 * 2 + 6 * 4 == 96
    assert bench.method_bytes("f32", 5) == 28 * 4 + 6 * 4
