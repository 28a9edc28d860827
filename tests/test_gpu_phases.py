"""The profiling build (libcn_phase.so, CN_PHASE_CLOCKS): bench.py --phase-clocks loads it in a process of its own,
and every phase of the interval kernel gets clock time on a small cortex recipe in both precisions."""
import json
import os
import subprocess
import sys

import pytest

from tests.progress import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_phase_clocks_cover_every_phase():
    from paper_1901_10975_amd import build as B, cn
    assert os.path.exists(B.LIB_PHASE), "build the profiling library first"
    say("phase clocks: cortex_50k recipe, 2000 cells, 3 intervals")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--phase-clocks", "--n-cells", "2000",
                        "--steps", "3", "--warmup", "1"], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["library"] == "libcn_phase.so"
    for prec in ("fp64", "fp32_mech"):
        share = out[prec]["share"]
        assert set(share) == set(cn.PHASES)
        assert all(v > 0.0 for v in share.values()), share
        assert abs(sum(share.values()) - 1.0) < 1e-9
        say(prec, {k: round(v, 3) for k, v in share.items()})
