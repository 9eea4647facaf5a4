"""Host-only checks of the region where the GPU parity tests replace the FP32 tolerance by a
conditioning bound (tests/parity.drop_interior_mask): it must hold the nodes where the
oracle cannot be followed to that tolerance, and nothing it is needed for must lie outside.
Both are properties of the oracle alone, under relative input noise of the 32-bit unit
roundoff; no GPU result enters."""
import numpy as np

from paper_1710_09541_amd import cases
from tests.parity import drop_interior_mask, perturbed, run_oracle

STEPS = 41


def _spread(case, steps):
    ref = run_oracle(case, steps)
    d = np.zeros_like(ref["phi"])
    for seed in (5, 6, 7):
        p = perturbed(case, steps, eps=2.0 ** -23, seed=seed)
        d = np.maximum(d, np.abs(p["phi"] - ref["phi"]))
    return d


def test_interior_mask_holds_the_oracle_ill_conditioned_nodes():
    """A ratio-10 drop of radius 21 centred on a node (instance 160 of the 256-instance
    batch, 165 x 67): the oracle moves itself by more than the FP32 tolerance inside the
    mask, 8 to 10 nodes from the centre, and by less than a tenth of it outside."""
    c = cases.batch_ensemble(256, seed=1)[160]
    assert (c["nx"], c["ny"], c["name"]) == (165, 67, "static_drop")
    m = drop_interior_mask(c, STEPS)
    d = _spread(c, STEPS)
    assert d[m].max() > 1e-5
    assert d[~m].max() < 1e-6


def test_interior_mask_is_fixed_by_the_case_and_grows_with_time():
    c = cases.static_drop(64, 64, R=16.0, W=4.0)
    a, b = drop_interior_mask(c, 10), drop_interior_mask(c, 100)
    assert a.sum() < b.sum() and np.all(b[a])
    # centred: symmetric under both reflections of the periodic grid
    assert np.array_equal(a, a[::-1, :]) and np.array_equal(a, a[:, ::-1])
    assert drop_interior_mask(cases.spinodal(64), 10) is None
