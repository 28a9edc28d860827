"""The interleaved layout (one lane per cell, the paper's one-cell-per-thread GPU ordering, Sec. 4.4) against the
oracle, with the parity bars of the level layout: identical spike (gid, step) lists and FP64 voltages within
max(1e-10, 10 s(t)); a split run equals the uninterrupted one bitwise; the FP32-mechanism path keeps every spike
within one step of the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1901_10975_amd import synth
from tests.test_gpu_parity import _edge_model, assert_spikes_equal, lockstep
from tests.progress import say

pytestmark = pytest.mark.gpu

IL = dict(layout="interleaved")


def test_clamped_cells_interleaved():
    m = synth.clamped_cells()
    say("interleaved: clamped_cells 100 ms, plain bar")
    orc, eng, worst = lockstep(m, range(40, 4001, 40), sensitivity=False, **IL)
    assert eng.info()["layout"] == 2
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=10)


def test_ring_network_interleaved_50ms():
    m = synth.ring_network(n_cells=300, n_comp=200, seed=41, tstop=50.0)
    m.nc_weight = m.nc_weight * 4
    say("interleaved: ring network 300 x 200, 50 ms")
    orc, eng, worst = lockstep(m, range(100, 2001, 100), **IL)
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=20)


def test_cortex_recipe_interleaved():
    """uneven cell sizes (groups padded to their largest cell), Poisson background, NetCon events"""
    m = synth.cortex_50k(n_cells=400)
    say("interleaved: cortex_50k recipe, 400 cells, 20 ms")
    orc, eng, worst = lockstep(m, range(40, 801, 40), **IL)
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=50)


def test_edge_shapes_interleaved():
    m = _edge_model()
    say("interleaved: edge shapes")
    orc, eng, worst = lockstep(m, range(10, 1201, 10), **IL)
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=3)


@pytest.mark.parametrize("cells_per_type", [1, 64])
def test_ring_types_interleaved_and_level(cells_per_type):
    """the node-ordering workload (random types of 83 compartments) on both layouts against the oracle"""
    m = synth.ring_types(n_cells=1024, cells_per_type=cells_per_type)
    say(f"ring_types 1024 cells, {cells_per_type} per type, both layouts")
    for layout in ("interleaved", "level"):
        orc, eng, worst = lockstep(m, range(40, 401, 40), layout=layout)
        assert worst <= 1.0, (layout, worst)
        assert_spikes_equal(orc, eng, min_count=16)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mech"])
def test_split_run_interleaved(precision):
    from paper_1901_10975_amd import cn
    m = synth.cortex_50k(n_cells=300, seed=23)
    say(f"interleaved restore, {precision}")
    whole = cn.Engine(m, precision=precision, **IL)
    whole.run_to_step(1200)
    a = cn.Engine(m, precision=precision, **IL)
    a.run_to_step(610)
    ck = a.checkpoint()
    b = cn.Engine(m, precision=precision, **IL)
    b.restore(ck)
    b.run_to_step(1200)
    cw, cb = whole.checkpoint(), b.checkpoint()
    assert np.array_equal(cw["v"], cb["v"])
    for k in cw["states"]:
        assert np.array_equal(cw["states"][k], cb["states"][k]), k
    gw, sw, tw = whole.spikes()
    gb, sb, tb = b.spikes()
    keep = sw > 610
    assert np.array_equal(gw[keep], gb) and np.array_equal(sw[keep], sb) and np.array_equal(tw[keep], tb)


def test_fp32_mech_interleaved_spikes_within_one_step():
    from paper_1901_10975_amd import cn
    m = synth.cortex_50k(n_cells=400, seed=29)
    say("interleaved fp32_mech against the FP64 oracle")
    orc = O.OracleSim(m, n_threads=16)
    eng = cn.Engine(m, precision="fp32_mech", **IL)
    orc.run(20.0)
    eng.run(20.0)
    go, so, _ = orc.spikes()
    gg, sg, _ = eng.spikes()
    assert go.size > 50
    co, cg = np.bincount(go, minlength=m.n_cells), np.bincount(gg, minlength=m.n_cells)
    assert np.array_equal(co, cg)
    oo, og = np.lexsort((so, go)), np.lexsort((sg, gg))
    assert int(np.abs(so[oo] - sg[og]).max()) <= 1


def test_per_compartment_parameters_interleaved():
    """per-compartment parameters (the table path of the general kernels) in the interleaved layout"""
    m = synth.ring_network(n_cells=120, n_comp=150, seed=31)
    rng = np.random.default_rng(31)
    hh = m.mechs["hh"]
    k = m.n_comp if hh.node is None else hh.node.size
    hh.params["gnabar"] = rng.uniform(0.08, 0.16, k)
    hh.params["gkbar"] = rng.uniform(0.02, 0.05, k)
    hh.params["gl"] = rng.uniform(1e-4, 5e-4, k)
    hh.params["el"] = rng.uniform(-60.0, -50.0, k)
    m.nc_weight = m.nc_weight * 4
    say("interleaved: per-compartment parameters")
    orc, eng, worst = lockstep(m, range(100, 1001, 100), **IL)
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=20)

