"""Checkpoint-restart on the GPU (Sec. 3.4): a run saved at step s and continued in a fresh model equals the
uninterrupted run bitwise, with the events in flight at s rebuilt from the spikes that sent them; a restart with a new
background key follows the oracle restarted the same way.

A checkpoint is the readouts at step s (cn_voltages, cn_mech_state of every state, cn_spikes); cn_restore writes them
into a model that has not run and queues again every NetCon event of the listed spikes due at or after s."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1901_10975_amd import synth
from tests.progress import say

pytestmark = pytest.mark.gpu

THREADS = 16


def _engine(m, **kw):
    from paper_1901_10975_amd import cn
    return cn.Engine(m, **kw)


def _in_flight(m, gid, step, s):
    """number of NetCon events of the spikes (gid, step) that are due at or after step s"""
    D = np.floor(m.nc_delay / m.dt + 0.5).astype(np.int64)
    n = 0
    for g, k in zip(gid, step):
        n += int(np.count_nonzero(k + D[m.nc_src == g] >= s))
    return n


def _assert_same(a, b, after=None):
    """bitwise equality of potentials, every mechanism state and the spikes (those after step `after` of a)"""
    ca, cb = a.checkpoint(), b.checkpoint()
    assert ca["step"] == cb["step"]
    assert np.array_equal(ca["v"], cb["v"])
    for k in ca["states"]:
        assert np.array_equal(ca["states"][k], cb["states"][k]), k
    ga, sa, ta = a.spikes()
    gb, sb, tb = b.spikes()
    if after is not None:
        keep = sa > after
        ga, sa, ta = ga[keep], sa[keep], ta[keep]
    assert np.array_equal(ga, gb) and np.array_equal(sa, sb) and np.array_equal(ta, tb)
    return ga.size


def _ring():
    return synth.ring_network(n_cells=200, n_comp=40, seed=7, tstop=60.0)


def _cortex():
    return synth.cortex_50k(n_cells=400, seed=11)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mech"])
@pytest.mark.parametrize("split", [800, 830])
@pytest.mark.parametrize("recipe", ["ring", "cortex"])
def test_split_run_equals_uninterrupted(recipe, split, precision):
    """split at an interval boundary (800 = 20 intervals of 40 steps) and inside an interval (830)"""
    m = _ring() if recipe == "ring" else _cortex()
    end = 2000
    say(f"restore: {recipe} {m.n_cells} cells, {precision}, split at step {split}, end {end}")
    whole = _engine(m, precision=precision)
    whole.run_to_step(end)
    first = _engine(m, precision=precision)
    first.run_to_step(split)
    ck = first.checkpoint()
    first.close()
    flying = _in_flight(m, ck["gid"], ck["spike_step"], split)
    say(f"  {ck['gid'].size} spikes before the split, {flying} events in flight")
    assert ck["gid"].size > 0 and flying > 0
    second = _engine(m, precision=precision)
    second.restore(ck)
    assert second.info()["step"] == split
    second.run_to_step(end)
    n_after = _assert_same(whole, second, after=split)
    say(f"  {n_after} spikes after the split, identical")
    assert n_after > 0


def test_restore_matches_the_restored_oracle():
    """the GPU restored from the oracle's own checkpoint follows the oracle restored from it (FP64 bar)"""
    m = _ring()
    s, end = 820, 1600
    say(f"restore from the oracle's checkpoint at step {s}")
    pre = O.OracleSim(m, n_threads=THREADS)
    pre.run_to_step(s)
    ck = pre.checkpoint()
    orc = O.OracleSim(m, n_threads=THREADS)
    orc.restore(ck)
    eng = _engine(m, precision="fp64")
    eng.restore(ck)
    for n in range(840, end + 1, 40):
        orc.run_to_step(n)
        eng.run_to_step(n)
        vo = orc.v()
        dev = float(np.max(np.abs(eng.voltages() - vo) / np.maximum(np.abs(vo), 1.0)))
        assert dev <= 1e-10, (n, dev)
    go, so, _ = orc.spikes()
    gg, sg, _ = eng.spikes()
    assert go.size > 0
    assert np.array_equal(go, gg) and np.array_equal(so, sg)


def test_reseeded_restart_follows_the_reseeded_oracle():
    """a restart under a new background key: it follows the oracle restarted under that key (spikes identical,
    voltages within the FP64 parity bar, whose sensitivity comes from rounding-level variants of the oracle restarted
    the same way: the FMA-built oracle and three rounding-probe seeds), and departs from the run that kept the old
    key"""
    m = _cortex()
    s, end, seed2 = 400, 1200, 987654321
    say(f"reseeded restart at step {s}")
    pre = O.OracleSim(m, n_threads=THREADS)
    pre.run_to_step(s)
    ck = pre.checkpoint()
    orc = O.OracleSim(m, n_threads=THREADS)
    ens = [O.OracleSim(m, n_threads=THREADS, fma=True)] + [O.OracleSim(m, n_threads=THREADS, jitter=j)
                                                          for j in (1, 2, 3)]
    for o in [orc] + ens:
        o.restore(ck)
        o.set_seed(seed2)
    eng = _engine(m, precision="fp64")
    eng.restore(ck)
    eng.set_seed(seed2)
    same_key = _engine(m, precision="fp64")
    same_key.restore(ck)
    for n in range(440, end + 1, 40):
        orc.run_to_step(n)
        eng.run_to_step(n)
        vo = orc.v()
        sens = 0.0
        for o in ens:
            o.run_to_step(n)
            sens = max(sens, float(np.max(np.abs(o.v() - vo) / np.maximum(np.abs(vo), 1.0))))
        dev = float(np.max(np.abs(eng.voltages() - vo) / np.maximum(np.abs(vo), 1.0)))
        assert dev <= max(1e-10, 10.0 * sens), (n, dev, sens)
    same_key.run_to_step(end)
    go, so, _ = orc.spikes()
    gg, sg, _ = eng.spikes()
    assert np.array_equal(go, gg) and np.array_equal(so, sg)
    assert not np.array_equal(same_key.voltages(), eng.voltages())
    ga, gs = same_key.mech_state("expsyn"), eng.mech_state("expsyn")
    assert not np.array_equal(ga, gs)


def test_restore_refuses_a_model_that_has_run():
    from paper_1901_10975_amd import cn
    m = _ring()
    a = _engine(m)
    a.run_to_step(80)
    ck = a.checkpoint()
    with pytest.raises(cn.CnError) as e:
        a.restore(ck)
    assert e.value.code == cn.CN_E_STATE
    b = _engine(m)
    bad = dict(ck)
    bad["spike_step"] = ck["spike_step"] + 10_000
    if bad["gid"].size:
        with pytest.raises(cn.CnError) as e:
            b.restore(bad)
        assert e.value.code == cn.CN_E_INVALID
    b.restore(ck)  # an invalid checkpoint leaves the model untouched
    b.run_to_step(120)
    a.run_to_step(120)
    _assert_same(a, b, after=80)
