"""FP32-mechanism path (reading R12) against the FP64 oracle: every spike of the oracle is matched by the same cell's
spike of the same rank at most one step away (and no extra spikes), and the voltage deviation is bounded. The
deviations measured here are the figures stated for each config."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1901_10975_amd import synth
from tests.progress import say

pytestmark = pytest.mark.gpu


def _run(m, checkpoints, cells=None, **kw):
    from paper_1901_10975_amd import cn
    orc = O.OracleSim(m, n_threads=16)
    eng = cn.Engine(m, precision="fp32_mech", **kw)
    nodes = None if cells is None else np.concatenate(
        [np.arange(m.cell_offset[c], m.cell_offset[c + 1]) for c in cells])
    linf, med = 0.0, []
    for n in checkpoints:
        orc.run_to_step(n)
        eng.run_to_step(n)
        vo, vg = orc.v(), eng.voltages()
        if nodes is not None:
            vo, vg = vo[nodes], vg[nodes]
        d = np.abs(vo - vg)
        linf = max(linf, float(d.max()))
        med.append(float(np.median(d)))
    return orc, eng, linf, float(np.median(med))


def _spike_steps_within_one(orc, eng, cells):
    """each listed cell has as many spikes on the GPU as in the oracle, the k-th of each within one step"""
    go, so, _ = orc.spikes()
    gg, sg, _ = eng.spikes()
    keep_o, keep_g = np.isin(go, cells), np.isin(gg, cells)
    go, so, gg, sg = go[keep_o], so[keep_o], gg[keep_g], sg[keep_g]
    n_cells = int(max(cells.max() + 1, 1))
    co, cg = np.bincount(go, minlength=n_cells), np.bincount(gg, minlength=n_cells)
    bad = np.nonzero(co != cg)[0]
    assert bad.size == 0, (bad[:5], co[bad[:5]], cg[bad[:5]])
    oo, og = np.lexsort((so, go)), np.lexsort((sg, gg))  # by cell, then step: the k-th spikes align
    worst = int(np.abs(so[oo] - sg[og]).max()) if so.size else 0
    assert worst <= 1, worst
    return int(so.size), worst


def test_ring_network_fp32_mech_100ms():
    """the ring network in the FP32-mechanism path, 100 ms, errors on cells 0-499"""
    m = synth.ring_network(tstop=100.0)
    cells = np.arange(500)
    say("ring_network fp32_mech 100 ms")
    orc, eng, linf, med = _run(m, list(range(400, 4001, 400)), cells=cells)
    n, worst = _spike_steps_within_one(orc, eng, cells)
    say(f"  cells 0-499: {n} spikes, max |step difference| {worst}, voltage Linf {linf:.3g} mV, median {med:.3g} mV")
    assert n >= 1000
    assert med < 1e-3
    assert linf < 50.0  # a spike one step early or late moves v by tens of mV during the upstroke


@pytest.mark.parametrize("threads", [0, 512])
def test_cortex_50k_recipe_fp32_mech(threads):
    m = synth.cortex_50k(n_cells=400)
    cells = np.arange(m.n_cells)
    say(f"cortex_50k recipe fp32_mech, 400 cells, 20 ms, group_threads {threads}")
    orc, eng, linf, med = _run(m, list(range(40, 801, 40)), group_threads=threads)
    n, worst = _spike_steps_within_one(orc, eng, cells)
    say(f"  {n} spikes, max |step difference| {worst}, voltage Linf {linf:.3g} mV, median {med:.3g} mV")
    assert n >= 50
    assert med < 1e-3


def test_cortex_200k_recipe_fp32_mech():
    m = synth.cortex_200k(n_cells=60)
    cells = np.arange(m.n_cells)
    say("cortex_200k recipe fp32_mech, 60 cells, 10 ms")
    orc, eng, linf, med = _run(m, list(range(20, 401, 20)))
    n, worst = _spike_steps_within_one(orc, eng, cells)
    say(f"  {n} spikes, max |step difference| {worst}, voltage Linf {linf:.3g} mV, median {med:.3g} mV")
    assert med < 1e-3


@pytest.mark.timeout(900)
def test_full_size_cortex_200k_fp32_mech_four_intervals():
    """cortex_200k at full size (200,000 cells, about 127M compartments, 20M synapses, Poisson background) in the
    FP32-mechanism path over four 20-step intervals against the FP64 oracle of the whole network: every compartment
    compared at each interval boundary, spikes matched within one step"""
    m = synth.cortex_200k()
    say(f"cortex_200k full size fp32_mech: {m.n_comp} compartments, 4 intervals")
    orc, eng, linf, med = _run(m, [20, 40, 60, 80])
    n, worst = _spike_steps_within_one(orc, eng, np.arange(m.n_cells))
    say(f"  {n} spikes, max |step difference| {worst}, voltage Linf {linf:.3g} mV, median {med:.3g} mV")
    assert med < 1e-3
    assert linf < 1.0
