"""Thin ctypes binding of libcn.so (include/cn.h): argument marshalling only.

Every step of the simulation runs in the library's HIP kernels. PyTorch supplies device memory (through the
library's allocation callbacks, so tensors from torch's caching allocator back every device buffer) and the stream.
There is no fallback: if libcn.so is missing or fails to load, constructing an Engine raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

from . import synth

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcn.so")

CN_OK, CN_E_INVALID, CN_E_NOMEM, CN_E_DEVICE, CN_E_STATE, CN_E_CAPACITY, CN_E_NUMERIC = range(7)
MECH_ID = {"hh": 0, "pas": 1, "km": 2, "cahi": 3, "expsyn": 4, "iclamp": 5}
PRECISION = {"fp64": 0, "fp32_mech": 1}
LAYOUT = {"auto": 0, "level": 1, "interleaved": 2}
EXPORTS = ("cn_model_create", "cn_run", "cn_spikes", "cn_voltages", "cn_mech_state", "cn_mech_state_noalloc",
           "cn_restore", "cn_set_seed", "cn_autotune", "cn_model_info", "cn_stats", "cn_phase_clocks",
           "cn_model_destroy", "cn_last_error")
PHASES = ("chunk", "events", "mechanisms", "elimination", "roots", "substitution")
NOALLOC_STATE_MAX = 4194304
STATE_KEYS = (("hh", 0, "hh_m"), ("hh", 1, "hh_h"), ("hh", 2, "hh_n"), ("km", 0, "km_n"), ("cahi", 0, "cahi_m"),
              ("cahi", 1, "cahi_cai"), ("expsyn", 0, "syn_g"))

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)


class CnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cn error {code}: {msg}")
        self.code = code


class Topology(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("n_comp", C.c_int64), ("cell_offset", _i64p), ("parent", _i32p),
                ("area", _dp), ("ri", _dp), ("cm", _dp), ("v_init", C.c_double), ("celsius", C.c_double)]


class MechTable(C.Structure):
    _fields_ = [("type", C.c_int32), ("n", C.c_int64), ("node", _i64p), ("param", _dp * 4),
                ("param_scalar", C.c_double * 4)]


class Network(C.Structure):
    _fields_ = [("n_netcon", C.c_int64), ("src_cell", _i32p), ("target_syn", _i64p), ("weight", _dp),
                ("delay", _dp), ("threshold", _dp), ("threshold_scalar", C.c_double), ("n_kick", C.c_int64),
                ("kick_step", _i64p), ("kick_syn", _i64p), ("kick_weight", _dp), ("poisson_rate_hz", C.c_double),
                ("poisson_weight", _dp), ("seed", C.c_uint64), ("poisson_key", _i64p), ("n_gap", C.c_int64),
                ("gap_node", _i64p), ("gap_partner", _i64p), ("gap_g", _dp)]


class Checkpoint(C.Structure):
    _fields_ = [("step", C.c_int64), ("v", _dp), ("hh_m", _dp), ("hh_h", _dp), ("hh_n", _dp), ("km_n", _dp),
                ("cahi_m", _dp), ("cahi_cai", _dp), ("syn_g", _dp), ("n_spikes", C.c_int64), ("spike_gid", _i32p),
                ("spike_step", _i64p)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("layout", C.c_int32), ("stream", C.c_void_p), ("dev_alloc", ALLOC_FN),
                ("dev_free", FREE_FN), ("alloc_ctx", C.c_void_p), ("event_capacity", C.c_int32),
                ("max_interval", C.c_int32), ("group_threads", C.c_int32), ("use_graph", C.c_int32),
                ("timing", C.c_int32), ("validate_only", C.c_int32), ("fault_inject", C.c_int32),
                ("group_slots", C.c_int32), ("group_fill_pct", C.c_int32), ("reserved", C.c_int32 * 3)]


TUNE_MAX = 16


class TuneResult(C.Structure):
    _fields_ = [("group_threads", C.c_int32), ("group_slots", C.c_int32), ("group_fill_pct", C.c_int32),
                ("default_threads", C.c_int32), ("default_slots", C.c_int32), ("n_candidates", C.c_int32),
                ("from_cache", C.c_int32), ("layout", C.c_int32), ("interval_ms", C.c_double),
                ("default_ms", C.c_double), ("signature", C.c_uint64), ("cand_threads", C.c_int32 * TUNE_MAX),
                ("cand_slots", C.c_int32 * TUNE_MAX), ("cand_fill", C.c_int32 * TUNE_MAX),
                ("cand_layout", C.c_int32 * TUNE_MAX), ("cand_ms", C.c_double * TUNE_MAX)]


class Info(C.Structure):
    _fields_ = [("n_comp", C.c_int64), ("n_syn", C.c_int64), ("n_netcon", C.c_int64), ("n_groups", C.c_int64),
                ("step", C.c_int64), ("device_bytes", C.c_int64), ("n_cells", C.c_int32),
                ("interval_steps", C.c_int32), ("group_threads", C.c_int32), ("group_slots", C.c_int32),
                ("max_group_nodes", C.c_int32), ("max_levels", C.c_int32), ("ring_slots", C.c_int32),
                ("event_capacity", C.c_int32), ("precision", C.c_int32), ("lds_bytes", C.c_int32),
                ("dt", C.c_double), ("layout", C.c_int32), ("groups_per_cu", C.c_int32)]


_lib = None


def lib():
    """Load libcn.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1901_10975_amd/build.py")
        # PyTorch ships its own HIP runtime with the same SONAME as the system one. Loading torch first lets the
        # dynamic loader bind libcn.so to that runtime, so one process never holds two HIP runtimes.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        L.cn_last_error.restype = C.c_char_p
        L.cn_model_create.argtypes = [C.POINTER(Topology), C.POINTER(MechTable), C.c_int32, C.POINTER(Network),
                                      C.POINTER(Options), C.POINTER(C.c_void_p)]
        L.cn_run.argtypes = [C.c_void_p, C.c_double, C.c_double]
        L.cn_spikes.argtypes = [C.c_void_p, _i64p, _i32p, _i64p, _dp, C.c_int64]
        L.cn_voltages.argtypes = [C.c_void_p, _dp, C.c_int64]
        L.cn_mech_state.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _dp, C.c_int64]
        L.cn_mech_state_noalloc.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _dp, C.c_int64]
        L.cn_restore.argtypes = [C.c_void_p, C.c_double, C.POINTER(Checkpoint)]
        L.cn_set_seed.argtypes = [C.c_void_p, C.c_uint64]
        L.cn_autotune.argtypes = [C.POINTER(Topology), C.POINTER(MechTable), C.c_int32, C.POINTER(Network),
                                  C.POINTER(Options), C.c_double, C.c_double, C.POINTER(TuneResult)]
        L.cn_model_info.argtypes = [C.c_void_p, C.POINTER(Info)]
        L.cn_stats.argtypes = [C.c_void_p, _dp, _i64p]
        L.cn_phase_clocks.argtypes = [C.c_void_p, C.POINTER(C.c_uint64), C.c_int32]
        L.cn_model_destroy.argtypes = [C.c_void_p]
        L.cn_model_destroy.restype = None
        for f in ("cn_model_create", "cn_run", "cn_spikes", "cn_voltages", "cn_mech_state", "cn_mech_state_noalloc",
                  "cn_restore", "cn_set_seed", "cn_autotune", "cn_model_info", "cn_stats", "cn_phase_clocks"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(code):
    if code != CN_OK:
        raise CnError(code, lib().cn_last_error().decode())


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t)) if a is not None and a.size else C.POINTER(t)()


class _TorchMemory:
    """Device allocations served by torch's caching allocator and kept alive until the library frees them."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.live: Dict[int, object] = {}
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
        except Exception:
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _free(self, ptr, ctx):
        self.live.pop(int(ptr or 0), None)


def _describe(model: "synth.Model", keep: list):
    """the model description of cn_model_create (topology, mechanism tables, network) as ctypes structures; arrays
    are appended to `keep`, which the caller holds for the duration of the call"""

    def arr(x, dtype):
        a = np.ascontiguousarray(np.asarray(x), dtype=dtype)
        keep.append(a)
        return a

    n = model.n_comp
    topo = Topology(model.n_cells, n, _ptr(arr(model.cell_offset, np.int64), C.c_int64),
                    _ptr(arr(model.parent, np.int32), C.c_int32), _ptr(arr(model.area, np.float64), C.c_double),
                    _ptr(arr(model.ri, np.float64), C.c_double), _ptr(arr(model.cm, np.float64), C.c_double),
                    model.v_init, model.celsius)
    tables = []
    for name, t in model.mechs.items():
        mt = MechTable()
        mt.type = MECH_ID[name]
        mt.n = t.count(n)
        mt.node = _ptr(arr(t.node, np.int64), C.c_int64) if t.node is not None else _i64p()
        for j, pname in enumerate(synth.MECH_PARAMS[name]):
            v = t.params[pname]
            if np.isscalar(v):
                mt.param[j] = _dp()
                mt.param_scalar[j] = float(v)
            else:
                mt.param[j] = _ptr(arr(v, np.float64), C.c_double)
        tables.append(mt)
    mtab = (MechTable * max(1, len(tables)))(*tables)
    keep.append(mtab)
    pw = model.poisson_weight if model.poisson_weight.shape[0] else None
    net = Network(model.nc_src.shape[0], _ptr(arr(model.nc_src, np.int32), C.c_int32),
                  _ptr(arr(model.nc_syn, np.int64), C.c_int64), _ptr(arr(model.nc_weight, np.float64), C.c_double),
                  _ptr(arr(model.nc_delay, np.float64), C.c_double),
                  _ptr(arr(model.threshold, np.float64), C.c_double), 0.0, model.kick_step.shape[0],
                  _ptr(arr(model.kick_step, np.int64), C.c_int64), _ptr(arr(model.kick_syn, np.int64), C.c_int64),
                  _ptr(arr(model.kick_weight, np.float64), C.c_double), float(model.poisson_rate_hz),
                  _ptr(arr(pw, np.float64), C.c_double) if pw is not None else _dp(),
                  int(model.seed) & 0xFFFFFFFFFFFFFFFF,
                  _ptr(arr(model.poisson_key, np.int64), C.c_int64) if model.poisson_key is not None
                  else _i64p())
    ng = int(getattr(model, "n_gap", 0))
    net.n_gap = ng
    if ng:
        net.gap_node = _ptr(arr(model.gap_node, np.int64), C.c_int64)
        net.gap_partner = _ptr(arr(model.gap_partner, np.int64), C.c_int64)
        net.gap_g = _ptr(arr(model.gap_g, np.float64), C.c_double)
    return topo, mtab, len(tables), net


def _tune_dict(r: TuneResult) -> dict:
    k = r.n_candidates
    names = {v: n for n, v in LAYOUT.items()}
    return {"layout": names[r.layout], "group_threads": r.group_threads, "group_slots": r.group_slots,
            "group_fill_pct": r.group_fill_pct, "interval_ms": r.interval_ms, "default_threads": r.default_threads,
            "default_slots": r.default_slots, "default_ms": r.default_ms, "from_cache": bool(r.from_cache),
            "signature": f"{r.signature:016x}",
            "candidates": [{"layout": names[r.cand_layout[i]], "threads": r.cand_threads[i], "slots": r.cand_slots[i],
                            "fill_pct": r.cand_fill[i], "interval_ms": r.cand_ms[i]} for i in range(k)]}


class Engine:
    """A cn model on the GPU, built from a ``synth.Model``. ``autotune``: choose the cell-group shape with
    cn_autotune first (timed on this model's description; cached in the library by the model's signature), with a
    wall-time budget of ``tune_budget_ms``; the choice is kept in ``self.tune``."""

    def __init__(self, model: "synth.Model", precision: str = "fp64", use_graph: bool = True, timing: bool = False,
                 event_capacity: int = 0, max_interval: int = 0, group_threads: int = 0, group_slots: int = 0,
                 group_fill_pct: int = 0, use_torch: bool = True, stream=None, validate_only: bool = False,
                 fault_inject: int = 0, autotune: bool = False, tune_budget_ms: float = 60000.0,
                 layout: str = "auto"):
        L = lib()
        self.model = model
        self.dt = float(model.dt)
        keep = []
        topo, mtab, n_tables, net = _describe(model, keep)
        opt = Options()
        opt.precision = PRECISION[precision]
        opt.layout = LAYOUT[layout]
        opt.event_capacity = int(event_capacity)
        opt.max_interval = int(max_interval)
        opt.group_threads = int(group_threads)
        opt.group_slots = int(group_slots)
        opt.group_fill_pct = int(group_fill_pct)
        opt.use_graph = 1 if use_graph else 0
        opt.timing = 1 if timing else 0
        opt.validate_only = 1 if validate_only else 0
        opt.fault_inject = int(fault_inject)
        self._mem = None
        if use_torch and not validate_only:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("cn: no GPU visible to torch")
            self._mem = _TorchMemory(torch.device("cuda", torch.cuda.current_device()))
            opt.dev_alloc = self._mem.alloc_cb
            opt.dev_free = self._mem.free_cb
            s = stream if stream is not None else torch.cuda.current_stream()
            opt.stream = C.c_void_p(s.cuda_stream)
            self._stream = s
        self.tune = None
        if autotune:
            r = TuneResult()
            _check(L.cn_autotune(C.byref(topo), mtab, n_tables, C.byref(net), C.byref(opt), self.dt,
                                 float(tune_budget_ms), C.byref(r)))
            self.tune = _tune_dict(r)
            opt.layout = r.layout
            opt.group_threads, opt.group_slots, opt.group_fill_pct = r.group_threads, r.group_slots, r.group_fill_pct
        h = C.c_void_p()
        _check(L.cn_model_create(C.byref(topo), mtab, n_tables, C.byref(net), C.byref(opt), C.byref(h)))
        self._h = h
        self.precision = precision

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().cn_model_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, tstop: float):
        _check(lib().cn_run(self._h, float(tstop), self.dt))

    def run_to_step(self, n: int):
        self.run(n * self.dt)

    def voltages(self) -> np.ndarray:
        out = np.empty(self.model.n_comp)
        _check(lib().cn_voltages(self._h, _ptr(out, C.c_double), self.model.n_comp))
        return out

    def spikes(self):
        n = C.c_int64()
        _check(lib().cn_spikes(self._h, C.byref(n), _i32p(), _i64p(), _dp(), 0))
        k = n.value
        gid = np.empty(k, np.int32)
        step = np.empty(k, np.int64)
        t = np.empty(k)
        if k:
            _check(lib().cn_spikes(self._h, C.byref(n), _ptr(gid, C.c_int32), _ptr(step, C.c_int64),
                                   _ptr(t, C.c_double), k))
        return gid, step, t

    def mech_state(self, mech: str, which: int = 0) -> np.ndarray:
        cnt = self.model.mechs[mech].count(self.model.n_comp)
        out = np.empty(cnt)
        _check(lib().cn_mech_state(self._h, MECH_ID[mech], which, _ptr(out, C.c_double), cnt))
        return out

    def mech_state_noalloc(self, mech: str, which: int = 0) -> np.ndarray:
        """as mech_state, through the entry point that allocates no device memory (cn_mech_state_noalloc)"""
        cnt = self.model.mechs[mech].count(self.model.n_comp)
        out = np.empty(cnt)
        _check(lib().cn_mech_state_noalloc(self._h, MECH_ID[mech], which, _ptr(out, C.c_double), cnt))
        return out

    def checkpoint(self) -> dict:
        """what a restart needs (cn_checkpoint): step, potentials, every mechanism state at this step, the spikes so far"""
        gid, step, _ = self.spikes()
        states = {key: (self.mech_state(mech, which) if mech in self.model.mechs else np.zeros(0))
                  for mech, which, key in STATE_KEYS}
        return dict(step=int(self.info()["step"]), v=self.voltages(), states=states, gid=gid, spike_step=step)

    def restore(self, ck: dict):
        """continue from a checkpoint (cn_restore); this engine must not have run"""
        keep = []

        def p(a, dt, ct):
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return _ptr(a, ct)

        st = ck["states"]
        c = Checkpoint()
        c.step = int(ck["step"])
        c.v = p(ck["v"], np.float64, C.c_double)
        for _, _, key in STATE_KEYS:
            setattr(c, key, p(st[key], np.float64, C.c_double) if np.asarray(st[key]).size else _dp())
        c.n_spikes = int(np.asarray(ck["gid"]).size)
        c.spike_gid = p(ck["gid"], np.int32, C.c_int32)
        c.spike_step = p(ck["spike_step"], np.int64, C.c_int64)
        _check(lib().cn_restore(self._h, self.dt, C.byref(c)))

    def set_seed(self, seed: int):
        """key of the background streams from the current step on (cn_set_seed)"""
        _check(lib().cn_set_seed(self._h, int(seed) & 0xFFFFFFFFFFFFFFFF))

    def info(self) -> dict:
        i = Info()
        _check(lib().cn_model_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in Info._fields_}

    def stats(self):
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().cn_stats(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def phase_clocks(self) -> dict:
        """shader clocks of the interval kernel per phase (a library built with CN_PHASE_CLOCKS only)"""
        out = (C.c_uint64 * len(PHASES))()
        _check(lib().cn_phase_clocks(self._h, out, len(PHASES)))
        return dict(zip(PHASES, (int(x) for x in out)))
