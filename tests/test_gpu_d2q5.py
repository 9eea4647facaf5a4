"""GPU parity of the D2Q5 phase-field lattice (f_lattice = 5) against the FP64 CPU oracle:
the FP64 format bit for bit on every workload and boundary type, FP32 and FP16-deviation
storage within the tolerances of the D2Q9 path, every launch variant bitwise equal."""
import numpy as np
import pytest

from oracle import diag
from paper_1710_09541_amd import cases, lbm
from tests.parity import TOL, errors, report, run_hip, run_oracle

pytestmark = pytest.mark.gpu


def _q5(c):
    c["f_lattice"] = cases.D2Q5
    return c


def _bitwise(name, c, steps, **kw):
    ref = run_oracle(c, steps)
    got = run_hip(c, steps, "f64", **kw)
    ndiff = sum(int(np.count_nonzero(got[k] != ref[k])) for k in ref)
    print("[bitwise] d2q5 %s f64 %d steps: %d differing values" % (name, steps, ndiff),
          flush=True)
    assert ndiff == 0


@pytest.mark.parametrize("name,make,steps", [
    ("static drop 64^2", lambda: cases.static_drop(), 2000),
    ("poiseuille 16x512", lambda: cases.layered_poiseuille(), 1000),
    ("impact 512x128 Re100", lambda: cases.droplet_impact(512, 128, D=64, Re=100), 500),
    ("spinodal 256^2", lambda: cases.spinodal(256, seed=0), 300)])
def test_d2q5_f64_bitwise_equal_to_oracle(name, make, steps):
    _bitwise(name, _q5(make()), steps)


@pytest.mark.parametrize("nx,ny,bc,seed", [(100, 37, cases.PERIODIC, 0), (70, 45, cases.WALL, 1),
                                           (3, 5, cases.WALL, 2), (130, 6, cases.OPEN, 3)])
def test_d2q5_f64_ragged_and_boundaries(nx, ny, bc, seed):
    _bitwise("random %dx%d bc%d" % (nx, ny, bc), _q5(cases.random_state_case(nx, ny, bc=bc,
                                                                              seed=seed)), 30)


def test_d2q5_eq29_f64_bitwise():
    c = _q5(cases.droplet_impact(256, 96, D=40, Re=20))
    c["grad_scheme"] = cases.GRAD_LOCAL_NEQ
    _bitwise("eq29 impact 256x96", c, 200)


def test_d2q5_variants_bitwise():
    """Fused tile heights, the split kernel and graph replay give the same bits (FP32)."""
    c = _q5(cases.droplet_impact(256, 96, D=40, Re=20))
    ref = run_hip(c, 40, "f32", kernel="fused", tile_rows=4)
    for kw in (dict(kernel="fused", tile_rows=8), dict(kernel="fused", tile_rows=16),
               dict(kernel="split", tile_rows=4), dict(kernel="fused", tile_rows=4,
                                                       use_graph=False)):
        got = run_hip(c, 40, "f32", **kw)
        for k in ref:
            assert np.array_equal(ref[k], got[k]), kw


@pytest.mark.parametrize("storage,fields", [("f32", ("phi", "u")), ("f16", ("u",))])
@pytest.mark.parametrize("name,make,steps", [
    ("static drop 64^2", lambda: cases.static_drop(), 1000),
    ("poiseuille 16x512", lambda: cases.layered_poiseuille(), 1000),
    ("impact 512x128 Re100", lambda: cases.droplet_impact(512, 128, D=64, Re=100), 10)])
def test_d2q5_reduced_storage(storage, fields, name, make, steps):
    c = _q5(make())
    e = errors(c, run_hip(c, steps, storage), run_oracle(c, steps))
    report("d2q5 " + name, storage, e)
    for f in fields:
        assert e[f] <= TOL[storage]


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_d2q5_spinodal_statistics(storage):
    c = _q5(cases.spinodal(256, seed=0))
    ref = run_oracle(c, 2000)
    with lbm.Simulation(c, storage=storage) as sim:
        d0 = sim.reduce()
        sim.step(2000)
        d = sim.reduce()
    o = diag.diagnostics(ref, c["rho_l"], c["rho_g"], c["mask"])
    L_gpu = 2 * 256 * 256 / d["interface_crossings"]
    L_ref = 2 * 256 * 256 / o["interface_crossings"]
    drift = abs(d["sum_phi"] - d0["sum_phi"]) / d0["sum_phi"]
    print("[statistics] d2q5 spinodal %s: L %.3f vs oracle %.3f, sum phi drift %.1e"
          % (storage, L_gpu, L_ref, drift), flush=True)
    assert abs(L_gpu / L_ref - 1) < 0.05
    assert drift < {"f32": 1e-6, "f16": 1e-4}[storage]


def test_d2q5_batch_against_oracle():
    batch = [_q5(c) for c in cases.batch_ensemble(n=6, seed=5, lo=32, hi=96)]
    with lbm.Simulation(batch, storage="f64") as sim:
        sim.step(200)
        got = [sim.moments(k) for k in range(len(batch))]
    for k, c in enumerate(batch):
        ref = run_oracle(c, 200)
        for key in ref:
            assert np.array_equal(ref[key], got[k][key]), (k, key)
