"""The host runtime (validation, cell packing, level and interleaved layouts, node and event tables, gap-junction
records) under AddressSanitizer, on the CPU: cn_host.cpp is built with ASan on its host code only, linked with the
ordinary kernel objects, and a child process loads that library with the ASan runtime preloaded and builds every
layout the ABI tests build, in validate-only mode (no device), plus the refusal paths. Any out-of-bounds access or
use-after-free in the host code ends the child with an ASan report."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1901_10975_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ASAN_RT = sorted(glob.glob("/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))

COMMON = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wno-unused-function",
          "-Wno-unused-variable"]
# ASan on the host pass only (each -fsanitize after -Xarch_host); the device code is built as usual
HOST_ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]

CHILD = r"""
import sys
sys.modules["torch"] = None  # the validate-only path needs no HIP runtime from torch
sys.path.insert(0, ROOT)
import numpy as np
from paper_1901_10975_amd import cn, synth
cn.LIB_PATH = LIB
from tests import models as TM
from tests.test_abi import _tiny
from tests.test_gpu_parity import _edge_model

def build(m, **kw):
    e = cn.Engine(m, use_torch=False, validate_only=True, **kw)
    assert e.info()["n_comp"] == m.n_comp
    e.close()

models = [synth.clamped_cells(), synth.ring_network(n_cells=100, n_comp=200), synth.cortex_50k(n_cells=2000),
          synth.cortex_200k(n_cells=200), _edge_model(), synth.ring_types(n_cells=700, cells_per_type=4),
          synth.add_gap_junctions(synth.ring_network(n_cells=130, n_comp=60), cluster=5, per_pair=2),
          synth.add_gap_junctions(synth.cortex_50k(n_cells=300), cluster=2, per_pair=3)]
for m in models:
    for layout in ("level", "interleaved"):
        build(m, layout=layout)
for T, K, fill in ((128, 8, 100), (256, 4, 90), (512, 2, 100), (512, 4, 100)):
    build(synth.cortex_50k(n_cells=600, seed=19), group_threads=T, group_slots=K, group_fill_pct=fill)
refused = 0
for mutate in ("parent", "area", "gap_range", "gap_self", "gap_cluster"):
    m = _tiny() if not mutate.startswith("gap") else synth.add_gap_junctions(
        synth.ring_network(n_cells=12, n_comp=30), cluster=12 if mutate == "gap_cluster" else 2)
    if mutate == "parent":
        m.parent[2] = 3
    elif mutate == "area":
        m.area[1] = 0.0
    elif mutate == "gap_range":
        m.gap_partner[1] = 10 ** 6
    elif mutate == "gap_self":
        m.gap_partner[0] = m.gap_node[0]
    try:
        build(m, group_threads=128, group_slots=2)
    except cn.CnError as e:
        assert e.code == cn.CN_E_INVALID, e
        refused += 1
assert refused == 5, refused
print("host runtime clean under ASan", flush=True)
"""


@pytest.mark.skipif(not ASAN_RT or not os.path.exists(HIPCC), reason="hipcc or the ASan runtime is missing")
def test_host_runtime_under_asan(tmp_path):
    objs, procs = [], []
    for src in ("cn_host.cpp", "cn_kernels.hip", "cn_noalloc.hip"):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        extra = HOST_ASAN if src == "cn_host.cpp" else []
        procs.append(subprocess.Popen([HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    for p in procs:
        out = p.communicate()[0]
        assert p.returncode == 0, out.decode()[-2000:]
    lib = str(tmp_path / "libcn_asan.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                    "-shared-libsan", "-o", lib] + objs, check=True, capture_output=True)
    env = dict(os.environ, LD_PRELOAD=ASAN_RT[-1], ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23")
    code = f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + CHILD
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-6000:])
    assert "host runtime clean under ASan" in r.stdout
