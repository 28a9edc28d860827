"""Small hand-built models for the oracle pins (chains, single compartments, tiny trees)."""
import numpy as np

from paper_1901_10975_amd.synth import MechTable, Model


def ri_uniform(diam, length, ra=100.0):
    """axial resistance between centres of two equal cylinders, MOhm (Ra ohm*cm, um)"""
    return 1e-2 * ra * length / (np.pi * diam * diam / 4.0)


def make(parent_lists, area, ri, mechs, cm=1.0, v_init=-65.0, dt=0.025, **net):
    sizes = np.array([len(p) for p in parent_lists], dtype=np.int64)
    off = np.zeros(len(sizes) + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    n = int(off[-1])
    parent = np.concatenate([np.asarray(p, np.int32) for p in parent_lists])
    d = dict(n_cells=len(sizes), cell_offset=off, parent=parent, area=np.broadcast_to(area, n).astype(float).copy(),
             ri=np.broadcast_to(ri, n).astype(float).copy(), cm=np.broadcast_to(cm, n).astype(float).copy(),
             v_init=v_init, celsius=6.3, mechs=mechs, nc_src=np.zeros(0, np.int32), nc_syn=np.zeros(0, np.int64),
             nc_weight=np.zeros(0), nc_delay=np.zeros(0), threshold=np.zeros(len(sizes)),
             kick_step=np.zeros(0, np.int64), kick_syn=np.zeros(0, np.int64), kick_weight=np.zeros(0),
             poisson_rate_hz=0.0, poisson_weight=np.zeros(0), seed=0, dt=dt)
    d.update(net)
    for k in list(d):
        if k in ("nc_src",):
            d[k] = np.asarray(d[k], np.int32)
    return Model(**d)


def chain(n):
    return [-1] + list(range(n - 1))


def hh(node=None):
    return MechTable(node=node, params={"gnabar": 0.12, "gkbar": 0.036, "gl": 3e-4, "el": -54.3})


def pas(node=None, g=1e-4, e=-65.0):
    return MechTable(node=node, params={"g": g, "e": e})


def iclamp(node, amp, dl=0.0, dur=1e9):
    node = np.asarray(node, np.int64)
    return MechTable(node=node, params={"del": dl, "dur": dur, "amp": np.broadcast_to(amp, node.shape).astype(float)})
