"""The C-ABI library loads, exports every entry point include/cn.h declares, and rejects bad models through the
boundary before touching a device (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1901_10975_amd import cn, synth
from tests import models as TM

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cn_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    names = _declared()
    assert "cn_model_create" in names and "cn_run" in names
    L = cn.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(cn.EXPORTS) == set(names)


def _expect_invalid(model, **kw):
    with pytest.raises(cn.CnError) as e:
        cn.Engine(model, use_torch=False, **kw)
    assert e.value.code == cn.CN_E_INVALID, str(e.value)
    return str(e.value)


def _tiny():
    return TM.make([TM.chain(4), [-1, 0]], 500.0, 10.0, {"hh": TM.hh(), "expsyn": synth.MechTable(
        node=np.array([1, 4], np.int64), params={"tau": 2.0, "e": 0.0})}, nc_src=[0, 1],
        nc_syn=np.array([1, 0], np.int64), nc_weight=np.array([0.01, 0.01]), nc_delay=np.array([1.0, 2.0]))


def test_rejects_parent_order():
    m = _tiny()
    m.parent[2] = 3
    assert "parent" in _expect_invalid(m)


def test_rejects_bad_root():
    m = _tiny()
    m.parent[0] = 0
    _expect_invalid(m)


def test_rejects_nonpositive_area_and_ri():
    m = _tiny()
    m.area[1] = 0.0
    _expect_invalid(m)
    m = _tiny()
    m.ri[2] = -1.0
    _expect_invalid(m)
    m = _tiny()
    m.cm[3] = float("nan")
    _expect_invalid(m)


def test_rejects_bad_mechanisms_and_network():
    m = _tiny()
    m.mechs["pas"] = synth.MechTable(node=np.array([1, 1], np.int64), params={"g": 1e-4, "e": -65.0})
    assert "two instances" in _expect_invalid(m)
    m = _tiny()
    m.mechs["expsyn"].node[0] = 99
    _expect_invalid(m)
    m = _tiny()
    m.nc_syn[0] = 5
    _expect_invalid(m)
    m = _tiny()
    m.nc_src[1] = 7
    _expect_invalid(m)
    m = _tiny()
    m.mechs["hh"].params["gnabar"] = np.array([0.12] * 5 + [float("inf")])
    _expect_invalid(m)


def test_null_arguments_are_errors_not_crashes():
    L = cn.lib()
    n = C.c_int64()
    assert L.cn_spikes(None, C.byref(n), None, None, None, 0) == cn.CN_E_INVALID
    assert L.cn_run(None, 1.0, 0.025) == cn.CN_E_INVALID
    assert L.cn_voltages(None, None, 0) == cn.CN_E_INVALID
    assert L.cn_model_create(None, None, 0, None, None, None) == cn.CN_E_INVALID
    out = C.c_void_p()
    assert L.cn_model_create(None, None, 0, None, None, C.byref(out)) == cn.CN_E_INVALID
    assert b"NULL" in L.cn_last_error()
    L.cn_model_destroy(None)


@pytest.mark.parametrize("layout", ["level", "interleaved"])
@pytest.mark.parametrize("name", ["clamped_cells", "ring_small", "cortex_50k_small", "cortex_200k_small", "edge",
                                  "ring_types", "ring_gap"])
def test_host_layout_checks_pass(name, layout):
    """the device layout (cell groups, level or interleaved order, instance ranges, event targets) satisfies every
    invariant the kernels index by; built and checked on the host only"""
    from tests.test_gpu_parity import _edge_model
    model = {"clamped_cells": lambda: synth.clamped_cells(),
             "ring_small": lambda: synth.ring_network(n_cells=100, n_comp=200),
             "cortex_50k_small": lambda: synth.cortex_50k(n_cells=3000),
             "cortex_200k_small": lambda: synth.cortex_200k(n_cells=300),
             "edge": _edge_model,
             "ring_types": lambda: synth.ring_types(n_cells=700, cells_per_type=4),
             "ring_gap": lambda: synth.add_gap_junctions(synth.ring_network(n_cells=130, n_comp=60), cluster=5,
                                                         per_pair=2)}[name]()
    e = cn.Engine(model, use_torch=False, validate_only=True, layout=layout)
    info = e.info()
    assert info["n_comp"] == model.n_comp
    assert info["layout"] == cn.LAYOUT[layout]
    assert info["max_group_nodes"] <= info["group_threads"] * info["group_slots"]
    assert info["n_groups"] >= 1
    with pytest.raises(cn.CnError) as err:
        e.run(1.0)
    assert err.value.code == cn.CN_E_STATE


def test_restore_and_seed_argument_checks():
    """checkpoint-restart entry points reject NULL arguments and models without a device, before any device work"""
    L = cn.lib()
    assert L.cn_restore(None, 0.025, None) == cn.CN_E_INVALID
    assert L.cn_set_seed(None, 1) == cn.CN_E_INVALID
    e = cn.Engine(_tiny(), use_torch=False, validate_only=True)
    ck = dict(step=40, v=np.full(6, -65.0), states={k: np.zeros(0) for _, _, k in cn.STATE_KEYS},
              gid=np.zeros(0, np.int32), spike_step=np.zeros(0, np.int64))
    with pytest.raises(cn.CnError) as err:
        e.restore(ck)
    assert err.value.code == cn.CN_E_STATE


def _gapped(**kw):
    return synth.add_gap_junctions(synth.ring_network(n_cells=12, n_comp=30), **kw)


def test_rejects_bad_gap_junctions():
    """a half-gap names two distinct compartments in range and a finite conductance >= 0"""
    for field, k, val, what in (("gap_node", 0, -1, "range"), ("gap_partner", 1, 10 ** 6, "range"),
                                ("gap_g", 2, -0.1, "conductance"), ("gap_g", 0, np.nan, "conductance")):
        m = _gapped()
        getattr(m, field)[k] = val
        assert what in _expect_invalid(m)
    m = _gapped()
    m.gap_partner[0] = m.gap_node[0]
    assert "own partner" in _expect_invalid(m)


def test_rejects_gap_clusters_larger_than_a_group():
    """cells joined by junctions share a cell group: a cluster larger than the group, or more than 64 cells for the
    interleaved layout, or more than 15 half-gaps on one compartment, is refused"""
    m = _gapped(cluster=12)  # 360 compartments joined
    assert "gap junctions" in _expect_invalid(m, group_threads=128, group_slots=2, validate_only=True)
    m = synth.add_gap_junctions(synth.ring_network(n_cells=70, n_comp=3), cluster=70, per_pair=0)
    m.gap_node = np.arange(69, dtype=np.int64) * 3
    m.gap_partner = m.gap_node + 3
    m.gap_g = np.full(69, 0.001)
    assert "64 cells" in _expect_invalid(m, layout="interleaved", validate_only=True)
    m = _gapped()
    m.gap_node = np.zeros(16, np.int64)
    m.gap_partner = np.arange(16, dtype=np.int64) + 30
    m.gap_g = np.full(16, 0.001)
    assert "15 gap" in _expect_invalid(m, validate_only=True)
    m = _gapped(cluster=12)
    info = cn.Engine(m, use_torch=False, validate_only=True).info()
    assert info["n_groups"] == 1 and info["group_threads"] * info["group_slots"] >= 360  # default shape holds it


@pytest.mark.parametrize("layout", ["level", "interleaved"])
def test_gap_clusters_share_a_group(layout):
    """the packing keeps every junction's two ends in one group (the host layout check refuses anything else),
    with clusters of several sizes"""
    for cluster in (2, 7):
        m = synth.add_gap_junctions(synth.ring_network(n_cells=200, n_comp=40), cluster=cluster)
        e = cn.Engine(m, use_torch=False, validate_only=True, layout=layout)
        assert e.info()["n_comp"] == m.n_comp
    # chains of 64 cells (the most one interleaved group holds), junctions between neighbours' somata
    m = synth.ring_network(n_cells=200, n_comp=3)
    a = np.array([c for c in range(199) if c % 64 != 63], np.int64) * 3
    m.gap_node, m.gap_partner = np.concatenate([a, a + 3]), np.concatenate([a + 3, a])
    m.gap_g = np.full(m.gap_node.shape[0], 0.002)
    e = cn.Engine(m, use_torch=False, validate_only=True, layout=layout)
    assert e.info()["n_comp"] == m.n_comp


def test_phase_clocks_need_the_profiling_build():
    """cn_phase_clocks answers only in the CN_PHASE_CLOCKS build; the ordinary library refuses it, and NULL or a short
    buffer is an argument error"""
    L = cn.lib()
    out = (C.c_uint64 * len(cn.PHASES))()
    assert L.cn_phase_clocks(None, out, len(cn.PHASES)) == cn.CN_E_INVALID
    e = cn.Engine(_tiny(), use_torch=False, validate_only=True)
    assert L.cn_phase_clocks(e._h, out, len(cn.PHASES) - 1) == cn.CN_E_INVALID
    assert L.cn_phase_clocks(e._h, out, len(cn.PHASES)) == cn.CN_E_STATE
    assert "without phase clocks" in L.cn_last_error().decode()
