"""ctypes wrapper of the oracle library (orc.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the benchmark's CPU-baseline leg, never by
the product path. It takes a ``synth.Model`` (the shared seeded input) and expands scalar parameters and dense
mechanism tables into the full per-instance arrays the C oracle requires.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")
# The same source compiled with fused multiply-add contraction: an equally valid oracle that rounds differently at
# every step. Tests use it to measure how strongly a network amplifies rounding-level differences.
LIB_FMA_PATH = os.path.join(HERE, "liborc_fma.so")
# The same source optimised for the host that times it (-O3 -march=native, still without FMA contraction): used only
# to time the oracle beside the GPU. It is compiled on the timing host itself; the CPU model it was built for is
# recorded next to it and a different host rebuilds it.
LIB_FAST_PATH = os.path.join(HERE, "liborc_fast.so")

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)


class OrcSpec(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int32), ("n_comp", C.c_int64), ("cell_offset", _i64p), ("parent", _i32p),
        ("area", _dp), ("ri", _dp), ("cm", _dp), ("v_init", C.c_double), ("celsius", C.c_double),
        ("n_hh", C.c_int64), ("hh_node", _i64p), ("hh_gnabar", _dp), ("hh_gkbar", _dp), ("hh_gl", _dp),
        ("hh_el", _dp),
        ("n_pas", C.c_int64), ("pas_node", _i64p), ("pas_g", _dp), ("pas_e", _dp),
        ("n_km", C.c_int64), ("km_node", _i64p), ("km_gbar", _dp),
        ("n_cahi", C.c_int64), ("cahi_node", _i64p), ("cahi_gbar", _dp),
        ("n_syn", C.c_int64), ("syn_node", _i64p), ("syn_tau", _dp), ("syn_e", _dp),
        ("n_icl", C.c_int64), ("icl_node", _i64p), ("icl_del", _dp), ("icl_dur", _dp), ("icl_amp", _dp),
        ("n_gap", C.c_int64), ("gap_node", _i64p), ("gap_partner", _i64p), ("gap_g", _dp),
        ("n_nc", C.c_int64), ("nc_src", _i32p), ("nc_syn", _i64p), ("nc_w", _dp), ("nc_delay", _dp),
        ("threshold", _dp),
        ("n_kick", C.c_int64), ("kick_step", _i64p), ("kick_syn", _i64p), ("kick_w", _dp),
        ("poisson_rate_hz", C.c_double), ("poisson_w", _dp), ("poisson_key", _i64p), ("seed", C.c_uint64),
        ("dt", C.c_double), ("batch_steps", C.c_int32), ("n_threads", C.c_int32), ("keep_matrix", C.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile liborc.so with gcc: plain -O2, no FMA contraction, OpenMP over cells; and liborc_fma.so, the same
    source with FMA contraction."""
    for path, fp in ((LIB_PATH, ["-ffp-contract=off"]), (LIB_FMA_PATH, ["-mfma", "-ffp-contract=fast"])):
        if force or not os.path.exists(path):
            cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp"] + fp + [
                "-Wall", "-Wno-unused-function", os.path.join(HERE, "orc.c"), "-o", path + ".tmp", "-lm"]
            subprocess.run(cmd, check=True)
            os.replace(path + ".tmp", path)
    return LIB_PATH


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def build_fast() -> str:
    """Compile liborc_fast.so for this host unless it was already built here."""
    tag = LIB_FAST_PATH + ".cpu"
    want = cpu_model()
    if os.path.exists(LIB_FAST_PATH) and os.path.exists(tag) and open(tag).read() == want:
        return LIB_FAST_PATH
    cmd = ["gcc", "-O3", "-march=native", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wno-unused-function", os.path.join(HERE, "orc.c"), "-o", LIB_FAST_PATH + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_FAST_PATH + ".tmp", LIB_FAST_PATH)
    with open(tag, "w") as fh:
        fh.write(want)
    return LIB_FAST_PATH


_libs = {}


def lib(fma: bool = False, fast: bool = False):
    path = LIB_FAST_PATH if fast else (LIB_FMA_PATH if fma else LIB_PATH)
    if path not in _libs:
        if fast:
            build_fast()
        elif not os.path.exists(path):
            build(force=False)
        L = C.CDLL(path)
        L.orc_error.restype = C.c_char_p
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(OrcSpec)]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_run.argtypes = [C.c_void_p, C.c_int64]
        L.orc_run.restype = C.c_int
        L.orc_step.argtypes = [C.c_void_p]
        L.orc_step.restype = C.c_int64
        L.orc_n_spikes.argtypes = [C.c_void_p]
        L.orc_n_spikes.restype = C.c_int64
        L.orc_n_delivered.argtypes = [C.c_void_p]
        L.orc_n_delivered.restype = C.c_int64
        L.orc_get_spikes.argtypes = [C.c_void_p, _i32p, _i64p, _dp]
        L.orc_get_v.argtypes = [C.c_void_p, _dp]
        L.orc_get_states.argtypes = [C.c_void_p] + [_dp] * 7
        L.orc_get_last_matrix.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_hines.argtypes = [C.c_int32, _i32p, _dp, _dp, _dp, _dp]
        L.orc_hines.restype = C.c_int64
        L.orc_poisson_draw.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        L.orc_poisson_draw.restype = C.c_uint32
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_restore.argtypes = [C.c_void_p, C.c_int64] + [_dp] * 8 + [C.c_int64, _i32p, _i64p]
        L.orc_restore.restype = C.c_int
        L.orc_set_seed.argtypes = [C.c_void_p, C.c_uint64]
        L.orc_set_jitter.argtypes = [C.c_void_p, C.c_uint64]
        _libs[path] = L
    return _libs[path]


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t)) if a is not None and a.size else C.POINTER(t)()


class OracleSim:
    """One oracle simulation of a ``synth.Model``. ``batch_steps``: 0 inserts a spike's events at once; M > 0
    inserts them at the end of each M-step interval."""

    def __init__(self, model, dt=None, batch_steps=0, n_threads=1, keep_matrix=False, fma=False, fast=False,
                 jitter=0):
        self.model = model
        self._L = lib(fma, fast)
        dt = float(model.dt if dt is None else dt)
        n = model.n_comp
        keep = []

        def arr(x, dtype):
            a = np.ascontiguousarray(np.asarray(x), dtype=dtype)
            keep.append(a)
            return a

        s = OrcSpec()
        s.n_cells = model.n_cells
        s.n_comp = n
        s.cell_offset = _p(arr(model.cell_offset, np.int64), C.c_int64)
        s.parent = _p(arr(model.parent, np.int32), C.c_int32)
        s.area = _p(arr(model.area, np.float64), C.c_double)
        s.ri = _p(arr(model.ri, np.float64), C.c_double)
        s.cm = _p(arr(model.cm, np.float64), C.c_double)
        s.v_init = model.v_init
        s.celsius = model.celsius
        mech_fields = {
            "hh": ("n_hh", "hh_node", [("gnabar", "hh_gnabar"), ("gkbar", "hh_gkbar"), ("gl", "hh_gl"),
                                       ("el", "hh_el")]),
            "pas": ("n_pas", "pas_node", [("g", "pas_g"), ("e", "pas_e")]),
            "km": ("n_km", "km_node", [("gbar", "km_gbar")]),
            "cahi": ("n_cahi", "cahi_node", [("gbar", "cahi_gbar")]),
            "expsyn": ("n_syn", "syn_node", [("tau", "syn_tau"), ("e", "syn_e")]),
            "iclamp": ("n_icl", "icl_node", [("del", "icl_del"), ("dur", "icl_dur"), ("amp", "icl_amp")]),
        }
        for name, (nf, nodef, cols) in mech_fields.items():
            t = model.mechs.get(name)
            if t is None:
                setattr(s, nf, 0)
                continue
            setattr(s, nf, t.count(n))
            setattr(s, nodef, _p(arr(t.nodes(n), np.int64), C.c_int64))
            for pname, field in cols:
                setattr(s, field, _p(arr(t.column(pname, n), np.float64), C.c_double))
        ng = int(getattr(model, "n_gap", 0))
        s.n_gap = ng
        s.gap_node = _p(arr(model.gap_node if ng else np.zeros(0), np.int64), C.c_int64)
        s.gap_partner = _p(arr(model.gap_partner if ng else np.zeros(0), np.int64), C.c_int64)
        s.gap_g = _p(arr(model.gap_g if ng else np.zeros(0), np.float64), C.c_double)
        s.n_nc = model.nc_src.shape[0]
        s.nc_src = _p(arr(model.nc_src, np.int32), C.c_int32)
        s.nc_syn = _p(arr(model.nc_syn, np.int64), C.c_int64)
        s.nc_w = _p(arr(model.nc_weight, np.float64), C.c_double)
        s.nc_delay = _p(arr(model.nc_delay, np.float64), C.c_double)
        s.threshold = _p(arr(model.threshold, np.float64), C.c_double)
        s.n_kick = model.kick_step.shape[0]
        s.kick_step = _p(arr(model.kick_step, np.int64), C.c_int64)
        s.kick_syn = _p(arr(model.kick_syn, np.int64), C.c_int64)
        s.kick_w = _p(arr(model.kick_weight, np.float64), C.c_double)
        s.poisson_rate_hz = model.poisson_rate_hz
        pw = model.poisson_weight if model.poisson_weight.shape[0] else np.zeros(model.n_syn)
        s.poisson_w = _p(arr(pw, np.float64), C.c_double)
        pk = model.poisson_key if getattr(model, "poisson_key", None) is not None else np.arange(model.n_syn)
        s.poisson_key = _p(arr(pk, np.int64), C.c_int64)
        s.seed = int(model.seed) & 0xFFFFFFFFFFFFFFFF
        s.dt = dt
        s.batch_steps = int(batch_steps)
        s.n_threads = int(n_threads)
        s.keep_matrix = 1 if keep_matrix else 0
        self.dt = dt
        self._h = self._L.orc_create(C.byref(s))
        if not self._h:
            raise ValueError("oracle: " + self._L.orc_error().decode())
        if jitter:
            self._L.orc_set_jitter(self._h, int(jitter) & 0xFFFFFFFFFFFFFFFF)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.orc_destroy(h)
            self._h = None

    @property
    def step(self) -> int:
        return int(self._L.orc_step(self._h))

    def run_to_step(self, n: int):
        if self._L.orc_run(self._h, int(n)) != 0:
            raise RuntimeError("oracle: " + self._L.orc_error().decode())

    def run(self, tstop: float):
        self.run_to_step(int(round(tstop / self.dt)))

    def v(self) -> np.ndarray:
        out = np.empty(self.model.n_comp)
        self._L.orc_get_v(self._h, _p(out, C.c_double))
        return out

    def spikes(self):
        n = int(self._L.orc_n_spikes(self._h))
        gid = np.empty(n, np.int32)
        step = np.empty(n, np.int64)
        t = np.empty(n)
        if n:
            self._L.orc_get_spikes(self._h, _p(gid, C.c_int32), _p(step, C.c_int64), _p(t, C.c_double))
        return gid, step, t

    def n_delivered(self) -> int:
        return int(self._L.orc_n_delivered(self._h))

    def states(self) -> dict:
        n = self.model.n_comp
        cnt = {k: (self.model.mechs[k].count(n) if k in self.model.mechs else 0)
               for k in ("hh", "km", "cahi", "expsyn")}
        out = {"hh_m": np.empty(cnt["hh"]), "hh_h": np.empty(cnt["hh"]), "hh_n": np.empty(cnt["hh"]),
               "km_n": np.empty(cnt["km"]), "cahi_m": np.empty(cnt["cahi"]), "cahi_cai": np.empty(cnt["cahi"]),
               "syn_g": np.empty(cnt["expsyn"])}
        self._L.orc_get_states(self._h, *[_p(out[k], C.c_double) for k in
                                        ("hh_m", "hh_h", "hh_n", "km_n", "cahi_m", "cahi_cai", "syn_g")])
        return out

    def checkpoint(self) -> dict:
        """the state a restart needs: step, potentials, mechanism states, conductances and the spikes so far"""
        gid, step, t = self.spikes()
        return dict(step=self.step, v=self.v(), states=self.states(), gid=gid, spike_step=step)

    def restore(self, ck: dict):
        """continue from `ck` (as checkpoint() returns it) in this model, which must not have run yet"""
        st = ck["states"]
        keys = ("hh_m", "hh_h", "hh_n", "km_n", "cahi_m", "cahi_cai", "syn_g")
        arrs = [np.ascontiguousarray(st[k], np.float64) for k in keys]
        v = np.ascontiguousarray(ck["v"], np.float64)
        gid = np.ascontiguousarray(ck["gid"], np.int32)
        stp = np.ascontiguousarray(ck["spike_step"], np.int64)
        rc = self._L.orc_restore(self._h, int(ck["step"]), _p(v, C.c_double), *[_p(a, C.c_double) for a in arrs],
                                 int(gid.size), _p(gid, C.c_int32), _p(stp, C.c_int64))
        if rc != 0:
            raise RuntimeError("oracle: " + self._L.orc_error().decode())

    def set_seed(self, seed: int):
        """key of the background streams from the current step on"""
        self._L.orc_set_seed(self._h, int(seed) & 0xFFFFFFFFFFFFFFFF)

    def last_matrix(self):
        n = self.model.n_comp
        d, rhs, dv = np.empty(n), np.empty(n), np.empty(n)
        self._L.orc_get_last_matrix(self._h, _p(d, C.c_double), _p(rhs, C.c_double), _p(dv, C.c_double))
        return d, rhs, dv


def hines(parent, a, b, d, rhs):
    """Solve one tree system in place with the oracle's Hines elimination; returns (solution, flop count)."""
    parent = np.ascontiguousarray(parent, np.int32)
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    d = np.array(d, np.float64)
    x = np.array(rhs, np.float64)
    fl = lib().orc_hines(int(parent.shape[0]), _p(parent, C.c_int32), _p(a, C.c_double), _p(b, C.c_double),
                         _p(d, C.c_double), _p(x, C.c_double))
    return x, int(fl)


def poisson_draw(seed: int, syn: int, step: int) -> int:
    return int(lib().orc_poisson_draw(seed & 0xFFFFFFFFFFFFFFFF, syn, step))


def philox(counter, key):
    c = (C.c_uint32 * 4)(*counter)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)
