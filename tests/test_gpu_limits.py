"""The largest grid one instance may have in each storage format (9 population planes just
below 4 GiB, where the 32-bit byte offsets of the buffer addressing come closest to their
limit), checked by a property that holds at any size: a periodic grid that repeats a
64 x 64 drop evolves as that drop does, so every 64 x 64 copy, the first and the last in
memory included, must equal the small run bit for bit (the per-node arithmetic does not
depend on the position).  The small run itself is held to the oracle by the other tests."""
import numpy as np
import pytest

from paper_1710_09541_amd import cases
from tests.parity import run_hip

pytestmark = pytest.mark.gpu

# largest multiple of 64 whose 9 planes (n^2 + 192 elements) stay below 4 GiB
LARGEST = {"f64": 7680, "f32": 10880, "f16": 15424}


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_largest_instance_repeats_the_small_drop(storage):
    n = LARGEST[storage]
    esize = {"f64": 8, "f32": 4, "f16": 2}[storage]
    assert 9 * (n * n + 192) * esize < 1 << 32
    small = cases.static_drop(64, 64, R=16)
    big = dict(small)
    reps = n // 64
    big["nx"] = big["ny"] = n
    for k in ("phi0", "ux0", "uy0"):
        big[k] = np.tile(small[k], (reps, reps))
    steps = 10
    ref = run_hip(small, steps, storage)
    got = run_hip(big, steps, storage)
    print("[limits] %s %dx%d: %.2f GB of populations per buffer"
          % (storage, n, n, 18 * n * n * esize / 1e9), flush=True)
    last = (reps - 1) * 64
    for y0, x0 in ((0, 0), (last, last), (last, 0), (0, last), (reps // 2 * 64, reps // 3 * 64)):
        for key in ref:
            tile = got[key][y0:y0 + 64, x0:x0 + 64]
            assert np.array_equal(tile, ref[key]), (storage, y0, x0, key)
