"""lbm_reduce_noalloc (the reduction through the library's fixed device scratch, for callers
that cannot allocate) against lbm_reduce, both through the C-ABI, on one MI355X."""
import pytest

from paper_1710_09541_amd import cases, lbm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage", ["f32", "f64", "f16"])
def test_noalloc_reduce_equals_lbm_reduce_on_two_calls(storage):
    """Two calls in a row, the second on a smaller instance (the scratch keeps the first
    call's larger planes), then the first again and a second context on the same GPU: every
    diagnostic equal, bit for bit, to lbm_reduce's on the same state."""
    big = cases.droplet_impact(512, 128, D=64, Re=100)      # 65,536 nodes
    small = cases.static_drop(48, 40, R=10)                  # 1,920 nodes
    with lbm.Simulation([big, small], storage=storage) as sim:
        sim.step(37)
        for k in (0, 1, 0):
            ref = lbm.lbm_reduce(sim.ctx, k, sim.cases[k]["mask"])
            got = lbm.lbm_reduce_noalloc(sim.ctx, k, sim.cases[k]["mask"])
            print("[noalloc] %s inst %d: %s" % (storage, k, got), flush=True)
            assert got == ref, (k, got, ref)
        with lbm.Simulation(cases.spinodal(64, seed=4), storage=storage) as other:
            other.step(5)
            ref = lbm.lbm_reduce(other.ctx, 0)
            got = lbm.lbm_reduce_noalloc(other.ctx, 0)
            assert got == ref
        # and the first context's result is unchanged by the other context's call
        assert lbm.lbm_reduce_noalloc(sim.ctx, 1, sim.cases[1]["mask"]) == \
            lbm.lbm_reduce(sim.ctx, 1, sim.cases[1]["mask"])


def test_noalloc_reduce_refuses_an_instance_beyond_its_scratch():
    """An instance of more than 1,048,576 nodes is refused with LBM_ERR_RANGE and a message;
    lbm_reduce still serves it, and the context goes on working."""
    c = cases.spinodal(1040, seed=1)                         # 1,081,600 nodes
    with lbm.Simulation(c, storage="f32", kernel="fused", tile_rows=4) as sim:
        sim.step(2)
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_reduce_noalloc(sim.ctx, 0)
        assert e.value.code == lbm.LBM_ERR_RANGE
        assert "1048576" in str(e.value)
        d = lbm.lbm_reduce(sim.ctx, 0)
        assert d["nonfinite"] == 0 and d["step"] == 2
