"""Error paths of cn_run on the GPU, forced from the host so that every kernel still exits normally.

* A device failure reported after work was queued leaves the device state ahead of the host's step counter: the
  model must refuse every later run (CN_E_STATE) instead of re-running from a stale step.
* A failure during the graph capture must end the capture: the caller's stream is usable afterwards.
* A non-finite membrane potential (a current far beyond any physiological value) is reported as CN_E_NUMERIC.
"""
import numpy as np
import pytest

from paper_1901_10975_amd import synth
from tests import models as TM
from tests.progress import say

pytestmark = pytest.mark.gpu


def test_failure_after_queued_work_breaks_the_model():
    from paper_1901_10975_amd import cn
    m = synth.ring_network(n_cells=40, n_comp=20, seed=3)
    say("injected drain failure")
    eng = cn.Engine(m, fault_inject=1)
    with pytest.raises(cn.CnError) as e:
        eng.run(5.0)
    assert e.value.code == cn.CN_E_DEVICE
    with pytest.raises(cn.CnError) as e:
        eng.run(10.0)
    assert e.value.code == cn.CN_E_STATE
    # readouts still answer
    assert np.all(np.isfinite(eng.voltages()))


@pytest.mark.parametrize("use_graph", [True, False])
def test_failed_capture_leaves_the_stream_usable(use_graph):
    import torch
    from paper_1901_10975_amd import cn
    m = synth.ring_network(n_cells=40, n_comp=20, seed=3)
    say(f"injected capture failure, use_graph {use_graph}")
    eng = cn.Engine(m, fault_inject=2, use_graph=use_graph)
    if use_graph:
        with pytest.raises(cn.CnError) as e:
            eng.run(5.0)
        assert e.value.code == cn.CN_E_DEVICE
        assert not torch.cuda.is_current_stream_capturing()
        x = torch.arange(1000, device="cuda", dtype=torch.float64)
        assert float(x.sum().item()) == 499500.0
        with pytest.raises(cn.CnError) as e:
            eng.run(5.0)
        assert e.value.code == cn.CN_E_STATE
    else:
        eng.run(5.0)  # no capture, nothing to fail
        assert eng.info()["step"] == 200


def test_nonfinite_voltage_is_reported():
    from paper_1901_10975_amd import cn
    m = TM.make([[-1], [-1, 0]], 1000.0, 10.0, {"hh": TM.hh(), "iclamp": TM.iclamp([0], 1e300, dl=0.0)})
    say("non-finite voltage")
    eng = cn.Engine(m)
    with pytest.raises(cn.CnError) as e:
        eng.run(2.0)
    assert e.value.code == cn.CN_E_NUMERIC
    with pytest.raises(cn.CnError) as e:
        eng.run(3.0)
    assert e.value.code == cn.CN_E_STATE
