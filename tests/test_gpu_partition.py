"""The sharded form of the path on one GPU (the spike exchange once per minimum-delay interval, Sec. 2): cells split
into K partitions, each a model of its own on the device whose remote inputs arrive as kicks at step k + D, give
bitwise the voltages and spikes of the single device run. This is what each GPU of a multi-GPU run computes between
exchanges; the exchange itself (an all-gather of the interval's spike records) is not built here."""
import numpy as np
import pytest

from tests.test_oracle_pins import _partitioned_run, _small_ring
from tests.progress import say

pytestmark = pytest.mark.gpu


class _Device:
    """the engine behind the interface the partitioned driver uses"""

    def __init__(self, m):
        from paper_1901_10975_amd import cn
        self.e = cn.Engine(m)

    def run_to_step(self, n):
        self.e.run_to_step(n)

    def spikes(self):
        return self.e.spikes()

    def v(self):
        return self.e.voltages()


@pytest.mark.parametrize("k_parts", [2, 3])
def test_partitions_on_the_device_equal_the_single_run(k_parts):
    m = _small_ring(n_cells=40, n_comp=20, seed=5)
    say(f"{k_parts} partitions of a 40-cell ring on the device, 30 ms")
    whole = _Device(m)
    whole.run_to_step(int(round(30.0 / m.dt)))
    g, k, t = whole.spikes()
    ref = sorted(zip(k.tolist(), g.tolist(), t.tolist()))
    assert len(ref) > 10
    parts = [np.arange(j, m.n_cells, k_parts) for j in range(k_parts)]
    spikes, v, passes = _partitioned_run(m, parts, 30.0, make=_Device)
    say(f"  settled after {passes} passes, {len(spikes)} spikes")
    assert passes >= 3
    assert sorted((s[1], s[0], s[2]) for s in spikes) == ref
    assert np.array_equal(v, whole.v())
