"""cn_mech_state_noalloc, the state readout for callers that cannot allocate device memory, against cn_mech_state:
bitwise the same values on two calls in a row (the second on a smaller input), in both precisions, for every
state of every mechanism; requests beyond the static buffer are refused."""
import numpy as np
import pytest

from paper_1901_10975_amd import synth
from tests.progress import say

pytestmark = pytest.mark.gpu

STATES = (("hh", 0), ("hh", 1), ("hh", 2), ("km", 0), ("cahi", 0), ("cahi", 1), ("expsyn", 0))


@pytest.mark.parametrize("precision", ["fp64", "fp32_mech"])
def test_noalloc_equals_mech_state_two_calls_second_smaller(precision):
    from paper_1901_10975_amd import cn
    cases = ((synth.cortex_50k(n_cells=500, seed=9), 330), (synth.ring_network(n_cells=60, n_comp=30, seed=5), 170))
    sizes = []
    for m, steps in cases:
        e = cn.Engine(m, precision=precision)
        say(f"noalloc readout, {precision}: {m.n_cells} cells, {m.n_comp} compartments, {steps} steps")
        # before the first run: initial values
        for mech, which in STATES:
            if mech in m.mechs:
                assert np.array_equal(e.mech_state(mech, which), e.mech_state_noalloc(mech, which))
        e.run_to_step(steps)
        n = 0
        for mech, which in STATES:
            if mech not in m.mechs:
                continue
            a = e.mech_state(mech, which)
            b = e.mech_state_noalloc(mech, which)
            assert a.size > 0 and np.array_equal(a, b), (mech, which)
            n = max(n, a.size)
        sizes.append(n)
        e.close()
    assert sizes[1] < sizes[0]


def test_noalloc_refuses_more_than_its_buffer():
    from paper_1901_10975_amd import cn
    m = synth.cortex_50k(n_cells=14000, seed=3)
    assert m.n_comp > cn.NOALLOC_STATE_MAX
    e = cn.Engine(m)
    with pytest.raises(cn.CnError) as err:
        e.mech_state_noalloc("hh", 0)
    assert err.value.code == cn.CN_E_CAPACITY
    assert e.mech_state("expsyn").size == m.n_syn  # the allocating readout still serves it
    assert e.mech_state_noalloc("expsyn").size == m.n_syn  # 1.4M synapses fit the buffer
