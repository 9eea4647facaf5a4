"""GPU parity of the local non-equilibrium normal (Eq. 29, grad_scheme = LOCAL_NEQ) against
the FP64 CPU oracle: the FP64 format bit for bit, FP32 and FP16-deviation storage within
the same tolerances as the isotropic scheme."""
import numpy as np
import pytest

from paper_1710_09541_amd import cases, lbm
from tests.parity import TOL, errors, report, run_hip, run_oracle

pytestmark = pytest.mark.gpu


def _neq(c):
    c["grad_scheme"] = cases.GRAD_LOCAL_NEQ
    return c


def _bitwise(name, c, steps, **kw):
    ref = run_oracle(c, steps)
    got = run_hip(c, steps, "f64", **kw)
    ndiff = sum(int(np.count_nonzero(got[k] != ref[k])) for k in ref)
    print("[bitwise] eq29 %s f64 %d steps: %d differing values" % (name, steps, ndiff),
          flush=True)
    assert ndiff == 0


@pytest.mark.parametrize("name,make,steps", [
    ("static drop 64^2", lambda: cases.static_drop(), 2000),
    ("poiseuille 16x512", lambda: cases.layered_poiseuille(), 1000),
    ("impact 512x128 Re20", lambda: cases.droplet_impact(512, 128, D=64, Re=20), 300),
    ("spinodal 256^2", lambda: cases.spinodal(256, seed=0), 200)])
def test_eq29_f64_bitwise_equal_to_oracle(name, make, steps):
    _bitwise(name, _neq(make()), steps)


@pytest.mark.parametrize("nx,ny,bc,seed", [(100, 37, cases.PERIODIC, 0), (70, 45, cases.WALL, 1),
                                           (3, 5, cases.WALL, 2), (130, 6, cases.OPEN, 3)])
def test_eq29_f64_ragged_and_boundaries(nx, ny, bc, seed):
    c = _neq(cases.random_state_case(nx, ny, bc=bc, seed=seed))
    _bitwise("random %dx%d bc%d" % (nx, ny, bc), c, 30)


def test_eq29_f64_variants_bitwise():
    """Fused tile heights, the split kernel and graph replay give the same bits."""
    c = _neq(cases.droplet_impact(256, 96, D=40, Re=20))
    ref = run_hip(c, 40, "f64", kernel="fused", tile_rows=4)
    for kw in (dict(kernel="fused", tile_rows=8), dict(kernel="split", tile_rows=4),
               dict(kernel="fused", tile_rows=4, use_graph=False)):
        got = run_hip(c, 40, "f64", **kw)
        for k in ref:
            assert np.array_equal(ref[k], got[k]), kw


@pytest.mark.parametrize("storage,fields", [("f32", ("phi", "u")), ("f16", ("u",))])
def test_eq29_static_drop_reduced_storage(storage, fields):
    c = _neq(cases.static_drop())
    e = errors(c, run_hip(c, 1000, storage), run_oracle(c, 1000))
    report("eq29 static_drop 64^2", storage, e)
    for f in fields:
        assert e[f] <= TOL[storage]


@pytest.mark.parametrize("storage,fields", [("f32", ("phi", "u")), ("f16", ("u",))])
def test_eq29_poiseuille_reduced_storage(storage, fields):
    c = _neq(cases.layered_poiseuille())
    e = errors(c, run_hip(c, 1000, storage), run_oracle(c, 1000))
    report("eq29 poiseuille 16x512", storage, e)
    for f in fields:
        assert e[f] <= TOL[storage]


@pytest.mark.parametrize("storage,fields", [("f32", ("phi", "u")), ("f16", ("u",))])
def test_eq29_impact_reduced_storage(storage, fields):
    c = _neq(cases.droplet_impact(512, 128, D=64, Re=100))
    e = errors(c, run_hip(c, 10, storage), run_oracle(c, 10))
    report("eq29 impact 512x128 Re100", storage, e)
    for f in fields:
        assert e[f] <= TOL[storage]


def test_eq29_mixed_batch_f64():
    """The scheme is a per-instance parameter: a batch mixing both schemes matches the
    oracle instance by instance, bit for bit."""
    batch = cases.batch_ensemble(n=4, seed=3, lo=32, hi=80)
    for k, c in enumerate(batch):
        c["grad_scheme"] = k % 2
    with lbm.Simulation(batch, storage="f64") as sim:
        sim.step(100)
        got = [sim.moments(k) for k in range(len(batch))]
    for k, c in enumerate(batch):
        ref = run_oracle(c, 100)
        for key in ref:
            assert np.array_equal(ref[key], got[k][key]), (k, key)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_eq29_paper_static_drop_spurious_velocity(storage):
    """Sec. 3.1 at the paper's set-up (200 x 200 periodic, R = 50, W = 5, sigma = 1e-3,
    density ratio 1000, nu = 0.1, M = 0.1, local normal of Eq. 29): the largest spurious
    speed after 100,000 steps within a factor 2 of the 1.6e-9 the paper prints (it states
    no step count; measured 1.39e-9 after 1e5 steps and 1.90e-9 after 2e5).  The FP64
    format repeats the oracle's arithmetic bit for bit, so this pins the method itself over a
    horizon the oracle cannot afford in a test."""
    from tests.parity import paper_value
    c = _neq(cases.static_drop(200, 200, R=50.0, W=5.0, ratio=1000.0, sigma=0.001, nu=0.1,
                               M=0.1))
    with lbm.Simulation(c, storage=storage) as sim:
        sim.step(100000)
        d = sim.reduce()
    u_paper = paper_value("static_drop_max_spurious_velocity")
    print("[spurious] 200x200 drop, Eq. 29, %s, 1e5 steps: max |u| %.3e (paper %.1e)"
          % (storage, d["max_u"], u_paper), flush=True)
    assert d["nonfinite"] == 0
    assert 0.5 < d["max_u"] / u_paper < 2.0
