"""Gap junctions (electrical coupling as pairs of half-gap point processes, the semi-implicit reading of Sec. 2's
coupled cable system) on the GPU against the oracle, on both layouts: identical spike (gid, step) lists and FP64
voltages within max(1e-10, 10 s(t)); zero-conductance junctions leave every result bitwise unchanged; a split run
equals the uninterrupted one bitwise; the FP32-mechanism path keeps every spike within one step of the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1901_10975_amd import synth
from tests.test_gpu_parity import assert_spikes_equal, lockstep
from tests.progress import say

pytestmark = pytest.mark.gpu

LAYOUTS = ["level", "interleaved"]


def _ring(g=0.05, cluster=3, per_pair=2, n_cells=300, n_comp=200):
    m = synth.ring_network(n_cells=n_cells, n_comp=n_comp, seed=41, tstop=50.0)
    m.nc_weight = m.nc_weight * 4
    return synth.add_gap_junctions(m, cluster=cluster, per_pair=per_pair, g=g)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_ring_with_gap_clusters(layout):
    m = _ring()
    say(f"gap junctions, ring 300 x 200, clusters of 3, {m.n_gap} half-gaps, {layout}, 50 ms")
    orc, eng, worst = lockstep(m, range(100, 2001, 100), layout=layout)
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=20)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_cortex_recipe_with_gap_pairs(layout):
    """uneven cell sizes (pairs of up to 2,000 compartments), Poisson background and NetCons, three junctions per
    pair"""
    m = synth.add_gap_junctions(synth.cortex_50k(n_cells=400), cluster=2, per_pair=3, g=0.02, seed=5)
    say(f"gap junctions, cortex recipe 400 cells, pairs, {m.n_gap} half-gaps, {layout}, 20 ms")
    orc, eng, worst = lockstep(m, range(40, 801, 40), layout=layout)
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=50)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_ring_types_with_gap_clusters_of_eight(layout):
    """clusters of eight 83-compartment cells, every pair joined (28 junctions per cluster)"""
    m = synth.add_gap_junctions(synth.ring_types(n_cells=512, cells_per_type=4), cluster=8, g=0.01, seed=9)
    say(f"gap junctions, ring_types 512 cells, clusters of 8, {m.n_gap} half-gaps, {layout}, 10 ms")
    orc, eng, worst = lockstep(m, range(40, 401, 40), layout=layout)
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=16)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_zero_conductance_junctions_change_nothing(layout):
    """junctions with g = 0 add exact zeros to every sum; the packing that keeps clusters together changes the
    grouping only, which never changes a compartment's arithmetic"""
    from paper_1901_10975_amd import cn
    plain = synth.cortex_50k(n_cells=300, seed=31)
    gapped = synth.add_gap_junctions(synth.cortex_50k(n_cells=300, seed=31), cluster=2, per_pair=3, g=0.0)
    say(f"zero-conductance junctions, {layout}")
    a = cn.Engine(plain, layout=layout)
    b = cn.Engine(gapped, layout=layout)
    a.run(10.0)
    b.run(10.0)
    assert np.array_equal(a.voltages(), b.voltages())
    for x, y in zip(a.spikes(), b.spikes()):
        assert np.array_equal(x, y)
    assert a.spikes()[0].size > 0


@pytest.mark.parametrize("layout", LAYOUTS)
def test_split_run_with_gaps(layout):
    from paper_1901_10975_amd import cn
    m = _ring(n_cells=120, n_comp=60)
    say(f"gap junctions, split run, {layout}")
    whole = cn.Engine(m, layout=layout)
    whole.run_to_step(1200)
    a = cn.Engine(m, layout=layout)
    a.run_to_step(610)
    b = cn.Engine(m, layout=layout)
    b.restore(a.checkpoint())
    b.run_to_step(1200)
    assert np.array_equal(whole.voltages(), b.voltages())
    gw, sw, _ = whole.spikes()
    gb, sb, _ = b.spikes()
    keep = sw > 610
    assert np.array_equal(gw[keep], gb) and np.array_equal(sw[keep], sb)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_fp32_mech_with_gaps_spikes_within_one_step(layout):
    from paper_1901_10975_amd import cn
    m = synth.add_gap_junctions(synth.cortex_50k(n_cells=400, seed=29), cluster=2, per_pair=2, g=0.02)
    say(f"gap junctions, fp32_mech against the FP64 oracle, {layout}")
    orc = O.OracleSim(m, n_threads=16)
    eng = cn.Engine(m, precision="fp32_mech", layout=layout)
    orc.run(20.0)
    eng.run(20.0)
    go, so, _ = orc.spikes()
    gg, sg, _ = eng.spikes()
    assert go.size > 50
    co, cg = np.bincount(go, minlength=m.n_cells), np.bincount(gg, minlength=m.n_cells)
    assert np.array_equal(co, cg)
    oo, og = np.lexsort((so, go)), np.lexsort((sg, gg))
    assert int(np.abs(so[oo] - sg[og]).max()) <= 1


@pytest.mark.parametrize("layout", LAYOUTS)
def test_junctions_inside_one_cell_and_between_cells(layout):
    """a half-gap may join two compartments of the same cell (a shunt across its tree) as well as two cells"""
    m = _ring(n_cells=120, n_comp=60, cluster=2, per_pair=1, g=0.05)
    rng = np.random.default_rng(77)
    cells = rng.choice(m.n_cells, 40, replace=False)
    a = m.cell_offset[cells] + rng.integers(0, 60, 40)
    b = m.cell_offset[cells] + (a - m.cell_offset[cells] + rng.integers(1, 60, 40)) % 60
    m.gap_node = np.concatenate([m.gap_node, a, b])
    m.gap_partner = np.concatenate([m.gap_partner, b, a])
    m.gap_g = np.concatenate([m.gap_g, np.full(80, 0.02)])
    say(f"gap junctions inside cells and between them, {m.n_gap} half-gaps, {layout}")
    orc, eng, worst = lockstep(m, range(100, 2001, 100), layout=layout)
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=10)


def test_autotune_on_a_gap_model_keeps_the_results():
    """the autotuner's candidates that cannot hold a joined pair are skipped; its choice gives the default shape's
    results bitwise"""
    from paper_1901_10975_amd import cn
    m = synth.add_gap_junctions(synth.cortex_50k(n_cells=600, seed=13), cluster=2, per_pair=2, g=0.02)
    say("autotune on a model with gap junctions")
    ref = cn.Engine(m)
    ref.run(5.0)
    e = cn.Engine(m, autotune=True, tune_budget_ms=60000.0)
    t = e.tune
    say(f"  chose {t['layout']} {t['group_threads']}x{t['group_slots']} fill {t['group_fill_pct']} of "
        f"{len(t['candidates'])} candidates")
    e.run(5.0)
    assert np.array_equal(ref.voltages(), e.voltages())
    for x, y in zip(ref.spikes(), e.spikes()):
        assert np.array_equal(x, y)
