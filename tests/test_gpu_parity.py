"""Parity of the HIP path (through the C-ABI) with the oracle, element by element on the same seeded inputs.

FP64 path, at every checkpoint:
  * spike (gid, step) lists identical (exact);
  * voltage metric dev(t) = max over compartments of |v_gpu - v_oracle| / max(|v_oracle|, 1 mV) must satisfy
    dev(t) <= max(1e-10, 10 * s(t)), where s(t) is the largest value of the same metric between the oracle and an
    ensemble of rounding-level variants of itself: v_init moved one ulp up and down, every NetCon weight moved one
    ulp, the oracle built with fused multiply-add contraction, and the oracle whose potentials move by -1, 0 or +1 ulp
    after every step (the rounding probe, three seeds). s(t) is the problem's own sensitivity to rounding: spike
    upstrokes and near-threshold inputs amplify rounding differences (on the ring network a one-ulp change of the
    weights alone grows to 4e-9 by 40 ms), so two correctly rounded implementations that round differently cannot
    stay within 1e-10 of each other on an active network. The rounding probe stands for an implementation that
    evaluates every step with other (correctly rounded) operations, which is what the GPU path is: its deviation
    from the oracle is of the probe's size (median ratio near one on the ring network), while single perturbations
    at the start underestimate it. Where the dynamics do not amplify, s(t) stays below 1e-11 and the bar is 1e-10.
  * interpolated spike times within max(1e-9 ms, 10 * the ensemble's spike-time sensitivity).
"""
import copy

import numpy as np
import pytest

from oracle import oracle as O
from paper_1901_10975_amd import synth
from tests import models as TM
from tests.progress import say

pytestmark = pytest.mark.gpu

VTOL = 1e-10
THREADS = 16


def _engine(m, **kw):
    from paper_1901_10975_amd import cn
    return cn.Engine(m, **kw)


def vrel(a, ref):
    return float(np.max(np.abs(a - ref) / np.maximum(np.abs(ref), 1.0))) if ref.size else 0.0


KSENS = 10.0
JITTER_SEEDS = (1, 2, 3)


def _ensemble(m):
    """rounding-level variants of the oracle on model m"""
    out = []
    for v in (np.nextafter(m.v_init, np.inf), np.nextafter(m.v_init, -np.inf)):
        mp = copy.copy(m)
        mp.v_init = float(v)
        out.append(O.OracleSim(mp, n_threads=THREADS))
    if m.nc_weight.size:
        mp = copy.copy(m)
        mp.nc_weight = np.nextafter(m.nc_weight, np.inf)
        out.append(O.OracleSim(mp, n_threads=THREADS))
    out.append(O.OracleSim(m, n_threads=THREADS, fma=True))
    out += [O.OracleSim(m, n_threads=THREADS, jitter=seed) for seed in JITTER_SEEDS]
    return out


def lockstep(m, checkpoints, precision="fp64", sensitivity=True, spikes_each=False, **kw):
    """run the oracle, its rounding-level variants and the GPU in lockstep; returns the oracle, the engine and the
    worst ratio dev(t) / bar(t) (<= 1 passes). sensitivity: True for the whole ensemble, "fma" for the FMA-built
    oracle and one rounding-probe member (large models), False for the plain 1e-10 bar. spikes_each: compare the spike lists at every
    checkpoint."""
    orc = O.OracleSim(m, n_threads=THREADS)
    if sensitivity == "fma":
        ens = [O.OracleSim(m, n_threads=THREADS, fma=True), O.OracleSim(m, n_threads=THREADS, jitter=JITTER_SEEDS[0])]
    else:
        ens = _ensemble(m) if sensitivity else []
    eng = _engine(m, precision=precision, **kw)
    worst, ratios = 0.0, []
    for n in checkpoints:
        orc.run_to_step(n)
        eng.run_to_step(n)
        v = orc.v()
        s = 0.0
        for e in ens:
            e.run_to_step(n)
            s = max(s, vrel(e.v(), v))
        bar = max(VTOL, KSENS * s)
        dev = vrel(eng.voltages(), v)
        if dev / bar > worst or m.n_comp >= 1_000_000:  # full-size models report every boundary
            say(f"  step {n}: dev {dev:.2e} sensitivity {s:.2e} bar {bar:.2e}")
        worst = max(worst, dev / bar)
        if s > 0.0:
            ratios.append(dev / s)
        if spikes_each:
            go, so, _ = orc.spikes()
            gg, sg, _ = eng.spikes()
            assert np.array_equal(go, gg) and np.array_equal(so, sg), f"spike lists differ at step {n}"
    if ratios:
        say(f"  worst dev/s(t) {max(ratios):.2f}, median {float(np.median(ratios)):.2f}")
    orc.sens_t = 0.0
    g1, s1, t1 = orc.spikes()
    for e in ens:
        g2, s2, t2 = e.spikes()
        if np.array_equal(g1, g2) and np.array_equal(s1, s2) and t1.size:
            orc.sens_t = max(orc.sens_t, float(np.abs(t1 - t2).max()))
    return orc, eng, worst


def assert_spikes_equal(orc, eng, min_count=1):
    go, so, to = orc.spikes()
    gg, sg, tg = eng.spikes()
    assert go.size >= min_count
    assert np.array_equal(go, gg) and np.array_equal(so, sg), (go[:10], gg[:10], so[:10], sg[:10])
    np.testing.assert_allclose(tg, to, rtol=0, atol=max(1e-9, KSENS * getattr(orc, "sens_t", 0.0)))


def test_clamped_cells_full():
    m = synth.clamped_cells()
    say("clamped_cells 64x32 100 ms")
    orc, eng, worst = lockstep(m, range(40, 4001, 40), sensitivity=False)  # plain 1e-10 bar throughout
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=10)


def test_ring_network_200ms():
    """the ring network over its full 200 ms"""
    m = synth.ring_network()
    say("ring_network 1000x200 200 ms")
    orc, eng, worst = lockstep(m, range(200, 8001, 200))
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=100)


def test_ring_network_plain_bar_first_25ms():
    """over the window in which the network's rounding sensitivity stays far below 1e-10, the plain bar: voltages
    within 1e-10 relative at every interval boundary, spikes identical"""
    m = synth.ring_network()
    say("ring_network 1000x200, 25 ms, plain 1e-10 bar")
    orc, eng, worst = lockstep(m, range(40, 1001, 40), sensitivity=False, spikes_each=True)
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=5)


@pytest.mark.timeout(900)
def test_full_size_cortex_50k_20ms_every_compartment():
    """cortex_50k at full size (50,000 cells, 15.9M compartments, 5M synapses, Poisson background) in the
    benchmark's launch configuration over 20 ms (20 minimum-delay intervals, NetCon events crossing groups): every
    compartment and the whole spike list against the oracle at every interval boundary. The rounding sensitivity
    comes from the FMA-built oracle and one rounding-probe member (the full ensemble would take eight oracle runs of
    the whole network)."""
    m = synth.cortex_50k()
    say(f"cortex_50k full size, {m.n_comp} compartments, 20 ms, every interval boundary")
    orc, eng, worst = lockstep(m, range(40, 801, 40), sensitivity="fma", spikes_each=True)
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=1)
    say(f"  {orc.spikes()[0].size} spikes identical")


@pytest.mark.parametrize("threads", [0, 512])
def test_cortex_50k_recipe_400_cells(threads):
    """the cortex_50k recipe on 400 cells; threads=512 is the launch shape the full-size workload takes (512 threads,
    two register slots, 1024-compartment groups)"""
    m = synth.cortex_50k(n_cells=400)
    say(f"cortex_50k recipe, 400 cells, 20 ms, group_threads {threads}")
    orc, eng, worst = lockstep(m, range(40, 801, 40), group_threads=threads)
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=50)
    info = eng.info()
    assert info["interval_steps"] == 40
    if threads:
        assert info["group_threads"] == 512 and info["group_slots"] == 2


def test_cortex_200k_recipe_60_cells():
    m = synth.cortex_200k(n_cells=60)
    say("cortex_200k recipe, 60 cells, 10 ms")
    orc, eng, worst = lockstep(m, range(20, 401, 20))
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=1)
    assert eng.info()["interval_steps"] == 20


@pytest.mark.parametrize("threads", [0, 512])
def test_per_compartment_parameters(threads):
    """density-mechanism parameters that differ between compartments (the per-node parameter table path), over
    25 ms of an active network (weights x4): beyond that, rounding differences grow chaotically on this network"""
    m = synth.ring_network(n_cells=120, n_comp=150, seed=31)
    rng = np.random.default_rng(31)
    hh = m.mechs["hh"]
    k = m.n_comp if hh.node is None else hh.node.size
    hh.params["gnabar"] = rng.uniform(0.08, 0.16, k)
    hh.params["gkbar"] = rng.uniform(0.02, 0.05, k)
    hh.params["gl"] = rng.uniform(1e-4, 5e-4, k)
    hh.params["el"] = rng.uniform(-60.0, -50.0, k)
    m.nc_weight = m.nc_weight * 4
    say(f"per-compartment parameters, group_threads {threads}")
    orc, eng, worst = lockstep(m, range(100, 1001, 100), group_threads=threads)
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=20)


def test_irregular_run_lengths_and_graph_off():
    m = synth.ring_network(n_cells=80, n_comp=60, seed=21)
    m.nc_weight = m.nc_weight * 10
    steps = np.cumsum([1, 6, 13, 40, 41, 2, 80, 39, 120, 7, 300])
    say("irregular chunks")
    orc, eng, worst = lockstep(m, steps, use_graph=False)
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=5)


def test_graph_and_direct_launches_bitwise_equal():
    m = synth.cortex_50k(n_cells=120, seed=5)
    say("graph vs direct")
    a = _engine(m, use_graph=True)
    b = _engine(m, use_graph=False)
    a.run(10.0)
    b.run(10.0)
    assert np.array_equal(a.voltages(), b.voltages())
    for x, y in zip(a.spikes(), b.spikes()):
        assert np.array_equal(x, y)


def test_determinism_two_runs():
    m = synth.cortex_50k(n_cells=150, seed=6)
    say("determinism")
    runs = []
    for _ in range(2):
        e = _engine(m)
        e.run(15.0)
        runs.append((e.voltages(), e.spikes(), e.mech_state("expsyn")))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][2], runs[1][2])
    for x, y in zip(runs[0][1], runs[1][1]):
        assert np.array_equal(x, y)


def _edge_model():
    """single compartments, a deep chain, a wide star and random trees, with synapses and kicks at later steps"""
    rng = np.random.default_rng(4)
    parents = [[-1], [-1], TM.chain(700), [-1] + [0] * 99]
    for n in (2, 3, 17, 250):
        parents.append([-1] + [int(rng.integers(0, i)) for i in range(1, n)])
    sizes = [len(p) for p in parents]
    n = sum(sizes)
    diam = rng.uniform(0.5, 2.0, n)
    length = rng.uniform(10, 50, n)
    area = np.pi * diam * length
    ri = 1e-2 * 100.0 * length / (np.pi * diam * diam / 4)
    n_cells = len(parents)
    off = np.concatenate([[0], np.cumsum(sizes)])
    syn_node = np.concatenate([off[c] + rng.integers(0, sizes[c], 3) for c in range(n_cells)])
    syn = synth.MechTable(node=syn_node, params={"tau": rng.uniform(1, 5, syn_node.size), "e": 0.0})
    src = np.array([(s // 3 + 1) % n_cells for s in range(syn_node.size)], np.int32)
    mechs = {"hh": TM.hh(), "expsyn": syn,
             "iclamp": TM.iclamp(off[:-1][[0, 2]], [0.3, 1.5], dl=2.0, dur=5.0)}
    return TM.make(parents, area, ri, mechs, nc_src=src, nc_syn=np.arange(syn_node.size, dtype=np.int64),
                   nc_weight=rng.uniform(0.02, 0.08, syn_node.size), nc_delay=rng.uniform(0.6, 3.0, syn_node.size),
                   kick_step=np.array([0, 0, 57, 57, 300], np.int64), kick_syn=np.array([3, 3, 9, 10, 20], np.int64),
                   kick_weight=np.array([0.05, 0.07, 0.2, 0.1, 0.3]))


def test_edge_shapes_kicks_and_clamps():
    m = _edge_model()
    say("edge shapes")
    orc, eng, worst = lockstep(m, range(10, 1201, 10))
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=3)


@pytest.mark.parametrize("threads", [0, 512])
def test_groups_of_many_small_cells(threads):
    """400 two-compartment HH cells driven by somatic IClamps: groups of more than 64 cells, whose threshold tests
    run on several waves (the chunk's spike count is read after all of them)"""
    rng = np.random.default_rng(12)
    n_cells = 400
    parents = [[-1, 0]] * n_cells
    diam = rng.uniform(0.5, 2.0, 2 * n_cells)
    length = rng.uniform(10, 50, 2 * n_cells)
    area = np.pi * diam * length
    ri = TM.ri_uniform(diam, length)
    soma = np.arange(0, 2 * n_cells, 2)
    m = TM.make(parents, area, ri, {"hh": TM.hh(), "iclamp": TM.iclamp(soma, rng.uniform(0.002, 0.01, n_cells))})
    say(f"400 two-compartment cells, 20 ms, group_threads {threads}")
    orc, eng, worst = lockstep(m, range(40, 801, 40), group_threads=threads)
    assert eng.info()["n_groups"] * 64 < n_cells  # more than 64 cells per group on average
    assert worst <= 1.0, worst
    assert_spikes_equal(orc, eng, min_count=200)


def test_states_parity():
    m = synth.cortex_50k(n_cells=50, seed=8)
    say("states")
    orc = O.OracleSim(m, n_threads=THREADS)
    eng = _engine(m)
    for n in (0, 1, 77, 400):
        orc.run_to_step(n)
        eng.run_to_step(n)
        st = orc.states()
        for mech, which, key in (("hh", 0, "hh_m"), ("hh", 1, "hh_h"), ("hh", 2, "hh_n"), ("km", 0, "km_n"),
                                 ("cahi", 0, "cahi_m"), ("cahi", 1, "cahi_cai"), ("expsyn", 0, "syn_g")):
            got = eng.mech_state(mech, which)
            ref = st[key]
            scale = max(np.abs(ref).max(), 1e-30)
            assert np.max(np.abs(got - ref)) <= 1e-9 * scale, (n, key)


def test_event_capacity_overflow_is_reported():
    from paper_1901_10975_amd import cn
    m = synth.ring_network(n_cells=40, n_comp=20, seed=3)
    m.nc_weight = m.nc_weight * 20
    m.kick_step = np.zeros(40, np.int64)
    m.kick_syn = np.arange(40, dtype=np.int64) * 10
    m.kick_weight = np.full(40, 0.5)
    say("capacity overflow")
    eng = _engine(m, event_capacity=2)
    with pytest.raises(cn.CnError) as e:
        eng.run(20.0)
    assert e.value.code == cn.CN_E_CAPACITY
    with pytest.raises(cn.CnError) as e:
        eng.run(30.0)
    assert e.value.code == cn.CN_E_STATE


def test_state_errors():
    from paper_1901_10975_amd import cn
    m = synth.clamped_cells(n_cells=4)
    eng = _engine(m)
    eng.run(1.0)
    from paper_1901_10975_amd.cn import lib
    assert lib().cn_run(eng._h, 2.0, 0.05) == cn.CN_E_STATE
    assert lib().cn_run(eng._h, 0.5, 0.025) == cn.CN_E_STATE
    eng.run(1.0)  # same time: no-op


def test_full_size_cortex_50k_first_interval_sampled():
    """cortex_50k at full size in the benchmark's launch configuration: within the first interval no NetCon event
    can arrive, so each sampled cell evolves alone and the oracle can compute it on its own."""
    m = synth.cortex_50k()
    say("cortex_50k full size, first interval, 300 sampled cells")
    eng = _engine(m)
    M = 40
    eng.run_to_step(M)
    assert eng.info()["interval_steps"] == M
    v = eng.voltages()
    rng = np.random.default_rng(0)
    cells = np.sort(rng.choice(m.n_cells, 300, replace=False))
    sub = synth.subset_cells(m, cells)
    orc = O.OracleSim(sub, n_threads=THREADS)
    orc.run_to_step(M)
    nodes = np.concatenate([np.arange(m.cell_offset[c], m.cell_offset[c + 1]) for c in cells])
    assert vrel(v[nodes], orc.v()) <= VTOL
    gg, sg, _ = eng.spikes()
    keep = np.isin(gg, cells)
    go, so, _ = orc.spikes()
    assert np.array_equal(cells[go], gg[keep]) and np.array_equal(so, sg[keep])
    assert np.all(np.isfinite(v))


def test_full_size_cortex_200k_first_interval_sampled():
    """cortex_200k at full size (200,000 cells, about 127M compartments, 20-step interval, 512-thread groups of up to
    2048 compartments): within the first interval each sampled cell evolves alone, so the oracle computes it alone"""
    m = synth.cortex_200k()
    say(f"cortex_200k full size: {m.n_cells} cells, {m.n_comp} compartments; first interval, 100 sampled cells")
    eng = _engine(m)
    eng.run_to_step(20)
    assert eng.info()["interval_steps"] == 20
    v = eng.voltages()
    rng = np.random.default_rng(1)
    cells = np.sort(rng.choice(m.n_cells, 100, replace=False))
    sub = synth.subset_cells(m, cells)
    orc = O.OracleSim(sub, n_threads=THREADS)
    orc.run_to_step(20)
    nodes = np.concatenate([np.arange(m.cell_offset[c], m.cell_offset[c + 1]) for c in cells])
    assert vrel(v[nodes], orc.v()) <= VTOL
    assert np.all(np.isfinite(v))
