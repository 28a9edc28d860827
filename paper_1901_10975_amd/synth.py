"""Seeded synthetic networks of multi-compartment cells.

This module is the one input source shared by the oracle tests and the HIP path. It draws topologies, geometry,
mechanism tables, connectivity and stimuli; it holds none of the time-stepping method's arithmetic. The only
arithmetic here is model building (compartment area and centre-to-centre axial resistance from diameter and
length), which a simulator does before the engine starts: the engine's boundary takes area and axial resistance
as given inputs.

Units follow the cable equation of Sec. 2 (Eq. 1): mV, ms, um, um^2, MOhm, uF/cm^2, S/cm^2, nA, uS.

Workload recipes (each draws its cells from ``numpy.random.default_rng`` with a fixed per-recipe seed):

* ``clamped_cells``: 64 cells x 32 compartments, hh at the soma, pas on the dendrites, an IClamp at each soma.
* ``ring_network``: 1,000 cells x 200 compartments, hh everywhere, 10 ExpSyn per cell each fed by one NetCon from
  a random other cell, 5 cells kicked at step 0 (a ring-style network, the shape of the paper's Ring model,
  Table 1); 200 ms by default, 100 ms where it exercises the FP32-mechanism path.
* ``cortex_50k``: 50,000 cells with log-uniform 50..1000 compartments, hh + km + cahi everywhere, 100 ExpSyn per
  cell, Poisson background at 5 Hz per synapse (a cortex-like shape, Table 1).
* ``cortex_200k``: 200,000 cells with log-uniform 100..2000 compartments, hh + pas + km + cahi everywhere, 100
  ExpSyn per cell, NetCon delays U(0.5, 10) ms, Poisson 5 Hz.

Every recipe takes ``n_cells`` to build a smaller network the same way (tests use this).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional, Union

import numpy as np

MECH_TYPES = ("hh", "pas", "km", "cahi", "expsyn", "iclamp")
# parameter columns per mechanism type, in the order the C boundary takes them
MECH_PARAMS = {
    "hh": ("gnabar", "gkbar", "gl", "el"),
    "pas": ("g", "e"),
    "km": ("gbar",),
    "cahi": ("gbar",),
    "expsyn": ("tau", "e"),
    "iclamp": ("del", "dur", "amp"),
}

Column = Union[float, np.ndarray]


@dataclasses.dataclass
class MechTable:
    """Instances of one mechanism type. ``node`` is a global compartment index per instance, or None when the
    mechanism is dense (instance i sits at compartment i). Each parameter is a scalar (same for every instance)
    or a float64 array with one value per instance."""

    node: Optional[np.ndarray]
    params: Dict[str, Column]

    def count(self, n_comp: int) -> int:
        return n_comp if self.node is None else int(self.node.shape[0])

    def nodes(self, n_comp: int) -> np.ndarray:
        return np.arange(n_comp, dtype=np.int64) if self.node is None else self.node

    def column(self, name: str, n_comp: int) -> np.ndarray:
        v = self.params[name]
        if np.isscalar(v):
            return np.full(self.count(n_comp), float(v))
        return np.asarray(v, dtype=np.float64)


@dataclasses.dataclass
class Model:
    n_cells: int
    cell_offset: np.ndarray  # int64 [n_cells+1]
    parent: np.ndarray  # int32 [n_comp], cell-local parent index, -1 at each root, parent[i] < i
    area: np.ndarray  # float64 [n_comp], um^2
    ri: np.ndarray  # float64 [n_comp], MOhm to the parent (ignored at roots)
    cm: np.ndarray  # float64 [n_comp], uF/cm^2
    v_init: float
    celsius: float
    mechs: Dict[str, MechTable]
    nc_src: np.ndarray  # int32 [n_nc] source cell
    nc_syn: np.ndarray  # int64 [n_nc] target ExpSyn instance
    nc_weight: np.ndarray  # float64 [n_nc] uS
    nc_delay: np.ndarray  # float64 [n_nc] ms
    threshold: np.ndarray  # float64 [n_cells] mV
    kick_step: np.ndarray  # int64 [n_kick]
    kick_syn: np.ndarray  # int64 [n_kick]
    kick_weight: np.ndarray  # float64 [n_kick] uS
    poisson_rate_hz: float
    poisson_weight: np.ndarray  # float64 [n_syn] uS (empty when there is no background)
    seed: int
    dt: float = 0.025
    tstop: float = 100.0
    name: str = ""
    poisson_key: Optional[np.ndarray] = None  # int64 [n_syn] background stream ids (None: instance index)
    # gap junctions as half-gap instances: current g (v_node - v_partner) nA at gap_node
    gap_node: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int64))
    gap_partner: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.int64))
    gap_g: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))  # uS

    @property
    def n_gap(self) -> int:
        return int(self.gap_node.shape[0])

    @property
    def n_comp(self) -> int:
        return int(self.cell_offset[-1])

    @property
    def n_syn(self) -> int:
        t = self.mechs.get("expsyn")
        return 0 if t is None else t.count(self.n_comp)

    def cell_sizes(self) -> np.ndarray:
        return np.diff(self.cell_offset)


RA = 100.0  # axial resistivity, ohm*cm
CM = 1.0  # uF/cm^2
V_INIT = -65.0
CELSIUS = 6.3
HH_PARAMS = {"gnabar": 0.12, "gkbar": 0.036, "gl": 3e-4, "el": -54.3}
PAS_PARAMS = {"g": 1e-4, "e": -65.0}
KM_GBAR = 2e-4
CAHI_GBAR = 1e-4


def _random_trees(rng: np.random.Generator, sizes: np.ndarray):
    """Random recursive trees: parent[i] uniform in [0, i) within each cell, root parent -1; per-compartment
    diameter U(0.5, 2) um and length U(10, 50) um. Returns offsets, local parents, area and axial resistance."""
    sizes = np.asarray(sizes, dtype=np.int64)
    off = np.zeros(sizes.shape[0] + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    n = int(off[-1])
    local = np.arange(n, dtype=np.int64) - np.repeat(off[:-1], sizes)
    u = rng.random(n)
    parent = np.floor(u * local).astype(np.int64)
    parent[local == 0] = -1
    diam = rng.uniform(0.5, 2.0, n)
    length = rng.uniform(10.0, 50.0, n)
    area = np.pi * diam * length
    # half-cylinder series resistance centre to centre; Ra in ohm*cm, lengths in um -> MOhm
    half = (length / 2.0) / (np.pi * diam * diam / 4.0)
    pg = np.where(parent >= 0, parent + np.repeat(off[:-1], sizes), 0)
    ri = 1e-2 * RA * (half + half[pg])
    ri[parent < 0] = 0.0
    return off, parent.astype(np.int32), area, ri


def _log_uniform_sizes(rng, n_cells, lo, hi):
    n = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), n_cells))).astype(np.int64)
    return np.clip(n, lo, hi)


def _synapses(rng, off, per_cell, tau, e):
    """``per_cell`` ExpSyn per cell at uniformly drawn compartments of that cell; instance c*per_cell + j."""
    n_cells = off.shape[0] - 1
    sizes = np.diff(off)
    cell = np.repeat(np.arange(n_cells, dtype=np.int64), per_cell)
    node = off[:-1][cell] + np.floor(rng.random(cell.shape[0]) * sizes[cell]).astype(np.int64)
    return cell, MechTable(node=node, params={"tau": float(tau), "e": float(e)})


def _netcons(rng, syn_cell, n_cells, w_hi, d_lo, d_hi):
    """One NetCon per synapse from a uniformly drawn other cell; weight U(0, w_hi) uS, delay U(d_lo, d_hi) ms."""
    n = syn_cell.shape[0]
    if n_cells > 1:
        src = (syn_cell + 1 + np.floor(rng.random(n) * (n_cells - 1)).astype(np.int64)) % n_cells
    else:
        src = np.zeros(n, dtype=np.int64)
    w = rng.uniform(0.0, w_hi, n)
    d = rng.uniform(d_lo, d_hi, n)
    return src.astype(np.int32), np.arange(n, dtype=np.int64), w, d


def _empty_i64():
    return np.zeros(0, dtype=np.int64)


def _base(off, parent, area, ri, mechs, **kw) -> Model:
    n = int(off[-1])
    n_cells = off.shape[0] - 1
    d = dict(
        n_cells=n_cells, cell_offset=off, parent=parent, area=area, ri=ri, cm=np.full(n, CM), v_init=V_INIT,
        celsius=CELSIUS, mechs=mechs, nc_src=np.zeros(0, np.int32), nc_syn=_empty_i64(), nc_weight=np.zeros(0),
        nc_delay=np.zeros(0), threshold=np.zeros(n_cells), kick_step=_empty_i64(), kick_syn=_empty_i64(),
        kick_weight=np.zeros(0), poisson_rate_hz=0.0, poisson_weight=np.zeros(0), seed=0)
    d.update(kw)
    return Model(**d)


def clamped_cells(n_cells: int = 64, seed: Optional[int] = None) -> Model:
    rng = np.random.default_rng(10975 + 1 if seed is None else seed)
    sizes = np.full(n_cells, 32, dtype=np.int64)
    off, parent, area, ri = _random_trees(rng, sizes)
    n = int(off[-1])
    soma = off[:-1].copy()
    dend = np.setdiff1d(np.arange(n, dtype=np.int64), soma)
    amp = rng.uniform(0.1, 0.5, n_cells)
    mechs = {
        "hh": MechTable(node=soma, params=dict(HH_PARAMS)),
        "pas": MechTable(node=dend, params=dict(PAS_PARAMS)),
        "iclamp": MechTable(node=soma.copy(), params={"del": 1.0, "dur": 100.0, "amp": amp}),
    }
    return _base(off, parent, area, ri, mechs, tstop=100.0, name="clamped_cells")


def _ring(n_cells, n_comp, seed, tstop, name) -> Model:
    rng = np.random.default_rng(seed)
    sizes = np.full(n_cells, n_comp, dtype=np.int64)
    off, parent, area, ri = _random_trees(rng, sizes)
    syn_cell, syn = _synapses(rng, off, 10, 2.0, 0.0)
    src, tgt, w, d = _netcons(rng, syn_cell, n_cells, 0.01, 1.0, 5.0)
    mechs = {"hh": MechTable(node=None, params=dict(HH_PARAMS)), "expsyn": syn}
    nk = min(5, n_cells)
    return _base(off, parent, area, ri, mechs, nc_src=src, nc_syn=tgt, nc_weight=w, nc_delay=d,
                 kick_step=np.zeros(nk, np.int64), kick_syn=np.arange(nk, dtype=np.int64) * 10,
                 kick_weight=np.full(nk, 0.1), tstop=tstop, name=name)


def ring_network(n_cells: int = 1000, n_comp: int = 200, seed: Optional[int] = None,
                 tstop: float = 200.0) -> Model:
    return _ring(n_cells, n_comp, 10975 + 2 if seed is None else seed, tstop, "ring_network")


def _cortex(n_cells, lo, hi, mech_names, d_lo, d_hi, seed, tstop, name) -> Model:
    rng = np.random.default_rng(seed)
    sizes = _log_uniform_sizes(rng, n_cells, lo, hi)
    off, parent, area, ri = _random_trees(rng, sizes)
    syn_cell, syn = _synapses(rng, off, 100, 2.0, 0.0)
    src, tgt, w, d = _netcons(rng, syn_cell, n_cells, 0.01, d_lo, d_hi)
    mechs = {}
    if "hh" in mech_names:
        mechs["hh"] = MechTable(node=None, params=dict(HH_PARAMS))
    if "pas" in mech_names:
        mechs["pas"] = MechTable(node=None, params=dict(PAS_PARAMS))
    if "km" in mech_names:
        mechs["km"] = MechTable(node=None, params={"gbar": KM_GBAR})
    if "cahi" in mech_names:
        mechs["cahi"] = MechTable(node=None, params={"gbar": CAHI_GBAR})
    mechs["expsyn"] = syn
    return _base(off, parent, area, ri, mechs, nc_src=src, nc_syn=tgt, nc_weight=w, nc_delay=d,
                 poisson_rate_hz=5.0, poisson_weight=w.copy(), seed=int(seed), tstop=tstop, name=name)


def cortex_50k(n_cells: int = 50000, seed: Optional[int] = None) -> Model:
    return _cortex(n_cells, 50, 1000, ("hh", "km", "cahi"), 1.0, 5.0, 10975 + 3 if seed is None else seed,
                   100.0, "cortex_50k")


def cortex_200k(n_cells: int = 200000, seed: Optional[int] = None) -> Model:
    return _cortex(n_cells, 100, 2000, ("hh", "pas", "km", "cahi"), 0.5, 10.0,
                   10975 + 5 if seed is None else seed, 50.0, "cortex_200k")


def ring_types(n_cells: int = 131072, n_comp: int = 83, cells_per_type: int = 1, ring_len: int = 128,
               seed: Optional[int] = None, tstop: float = 10.0) -> Model:
    """Rings of identical-size cells with a given number of identical cells per morphological type, the shape of the
    paper's node-ordering experiment (Sec. 4.4: 131,072 cells of 83 compartments, random branching per type, 1 to 32
    identical cells per type, 10 ms). Each type is a random recursive tree with its own geometry (a 20 x 20 um soma);
    cell c has type
    c // cells_per_type, so identical cells are adjacent. hh at the soma, pas elsewhere (a Ring-like cell: active
    soma, passive dendrites); one ExpSyn (tau 2 ms, e 0 mV) at compartment 1, driven by the previous cell of its ring
    of ring_len cells (weight 0.1 uS, delay 1 ms); the first cell of each ring is kicked at step 0."""
    rng = np.random.default_rng(10975 + 6 if seed is None else seed)
    n_types = -(-n_cells // cells_per_type)
    # per type: a random recursive tree, dendrites of diameter U(0.5, 2) um and length U(10, 50) um, a 20 x 20 um soma
    nt = n_types * n_comp
    local = np.tile(np.arange(n_comp, dtype=np.int64), n_types)
    t_parent = np.floor(rng.random(nt) * local).astype(np.int64)
    t_parent[local == 0] = -1
    diam = rng.uniform(0.5, 2.0, nt)
    length = rng.uniform(10.0, 50.0, nt)
    diam[local == 0] = 20.0
    length[local == 0] = 20.0
    t_area = np.pi * diam * length
    half = (length / 2.0) / (np.pi * diam * diam / 4.0)
    base = np.repeat(np.arange(n_types, dtype=np.int64) * n_comp, n_comp)
    t_ri = 1e-2 * RA * (half + half[np.where(t_parent >= 0, t_parent + base, 0)])
    t_ri[t_parent < 0] = 0.0
    t_parent = t_parent.astype(np.int32)
    typ = np.arange(n_cells, dtype=np.int64) // cells_per_type
    idx = (typ[:, None] * n_comp + np.arange(n_comp, dtype=np.int64)[None, :]).ravel()
    off = np.arange(n_cells + 1, dtype=np.int64) * n_comp
    parent, area, ri = t_parent[idx].copy(), t_area[idx].copy(), t_ri[idx].copy()
    soma = off[:-1].copy()
    dend = np.setdiff1d(np.arange(n_cells * n_comp, dtype=np.int64), soma)
    syn = MechTable(node=off[:-1] + 1, params={"tau": 2.0, "e": 0.0})
    cells = np.arange(n_cells, dtype=np.int64)
    ring0 = cells - cells % ring_len
    nxt = ring0 + (cells - ring0 + 1) % np.minimum(ring_len, n_cells - ring0)
    mechs = {"hh": MechTable(node=soma, params=dict(HH_PARAMS)), "pas": MechTable(node=dend, params=dict(PAS_PARAMS)),
             "expsyn": syn}
    kicks = np.arange(0, n_cells, ring_len, dtype=np.int64)
    return _base(off, parent, area, ri, mechs, nc_src=cells.astype(np.int32), nc_syn=nxt, nc_weight=np.full(n_cells, 0.1),
                 nc_delay=np.full(n_cells, 1.0), kick_step=np.zeros(kicks.size, np.int64), kick_syn=kicks,
                 kick_weight=np.full(kicks.size, 0.1), tstop=tstop, name="ring_types")


def add_gap_junctions(m: Model, cluster: int = 2, per_pair: int = 1, g: float = 0.005,
                      seed: Optional[int] = None) -> Model:
    """Electrical coupling (gap junctions) within clusters of `cluster` consecutive cells: every pair of cells of a
    cluster gets `per_pair` junctions between uniformly drawn compartments, conductance g uS, each junction as two
    half-gap instances (one at each end). Returns the model with its gap arrays set."""
    rng = np.random.default_rng(10975 + 7 if seed is None else seed)
    off = m.cell_offset
    sizes = np.diff(off)
    nodes, partners = [], []
    for c0 in range(0, m.n_cells, cluster):
        members = list(range(c0, min(c0 + cluster, m.n_cells)))
        for ia in range(len(members)):
            for ib in range(ia + 1, len(members)):
                a, b = members[ia], members[ib]
                for _ in range(per_pair):
                    na = off[a] + int(rng.integers(0, sizes[a]))
                    nb = off[b] + int(rng.integers(0, sizes[b]))
                    nodes += [na, nb]
                    partners += [nb, na]
    m.gap_node = np.asarray(nodes, np.int64)
    m.gap_partner = np.asarray(partners, np.int64)
    m.gap_g = np.full(m.gap_node.shape[0], float(g))
    return m


WORKLOADS = {"clamped_cells": clamped_cells, "ring_network": ring_network, "cortex_50k": cortex_50k,
             "cortex_200k": cortex_200k}


def subset_cells(m: Model, cells: np.ndarray) -> Model:
    """The sub-network on ``cells`` (sorted, unique): their compartments, mechanisms and synapses, the NetCons
    whose source and target both lie inside, and their kicks. Poisson streams keep their original synapse ids only
    if the caller passes ``seed`` through unchanged: the subset renumbers synapses, so its background draws differ
    from the full network's. Used to time the oracle on a bounded sample."""
    cells = np.asarray(cells, dtype=np.int64)
    sizes = m.cell_sizes()[cells]
    off = np.zeros(cells.shape[0] + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    old_nodes = np.concatenate([np.arange(m.cell_offset[c], m.cell_offset[c + 1]) for c in cells]) \
        if cells.shape[0] else _empty_i64()
    node_map = np.full(m.n_comp, -1, dtype=np.int64)
    node_map[old_nodes] = np.arange(old_nodes.shape[0])
    cell_map = np.full(m.n_cells, -1, dtype=np.int64)
    cell_map[cells] = np.arange(cells.shape[0])
    mechs = {}
    syn_map = None
    for k, t in m.mechs.items():
        nodes = t.nodes(m.n_comp)
        keep = np.nonzero(node_map[nodes] >= 0)[0]
        params = {p: (v if np.isscalar(v) else np.asarray(v)[keep]) for p, v in t.params.items()}
        node = None if (t.node is None) else node_map[nodes[keep]]
        if t.node is None:
            params = {p: (v if np.isscalar(v) else np.asarray(v)[old_nodes]) for p, v in t.params.items()}
        mechs[k] = MechTable(node=node, params=params)
        if k == "expsyn":
            syn_map = np.full(nodes.shape[0], -1, dtype=np.int64)
            syn_map[keep] = np.arange(keep.shape[0])
    if syn_map is None:
        syn_map = _empty_i64()
    nck = (cell_map[m.nc_src] >= 0) & (syn_map[m.nc_syn] >= 0) if m.nc_src.shape[0] else np.zeros(0, bool)
    kk = syn_map[m.kick_syn] >= 0 if m.kick_syn.shape[0] else np.zeros(0, bool)
    pw = m.poisson_weight[syn_map >= 0] if m.poisson_weight.shape[0] else m.poisson_weight
    old_key = m.poisson_key if m.poisson_key is not None else np.arange(syn_map.shape[0], dtype=np.int64)
    pkey = old_key[syn_map >= 0]
    gk = (node_map[m.gap_node] >= 0) & (node_map[m.gap_partner] >= 0) if m.n_gap else np.zeros(0, bool)
    return Model(
        n_cells=int(cells.shape[0]), cell_offset=off, parent=m.parent[old_nodes], area=m.area[old_nodes],
        ri=m.ri[old_nodes], cm=m.cm[old_nodes], v_init=m.v_init, celsius=m.celsius, mechs=mechs,
        nc_src=cell_map[m.nc_src[nck]].astype(np.int32), nc_syn=syn_map[m.nc_syn[nck]],
        nc_weight=m.nc_weight[nck], nc_delay=m.nc_delay[nck], threshold=m.threshold[cells],
        kick_step=m.kick_step[kk], kick_syn=syn_map[m.kick_syn[kk]], kick_weight=m.kick_weight[kk],
        poisson_rate_hz=m.poisson_rate_hz, poisson_weight=pw, seed=m.seed, dt=m.dt, tstop=m.tstop,
        name=m.name + "-subset", poisson_key=pkey, gap_node=node_map[m.gap_node[gk]],
        gap_partner=node_map[m.gap_partner[gk]], gap_g=m.gap_g[gk])
