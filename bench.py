"""Benchmark: compartment-timesteps per second of the fixed-step cable engine on one MI355X.

Main workload (the metric's configuration): cortex_50k - 50,000 cells with log-uniform 50..1000 compartments (15.93M
compartments), hh + km + cahi in every compartment, 100 ExpSyn per cell fed by NetCons with delays U(1, 5) ms (1 ms
minimum-delay interval, 40 steps of 0.025 ms) and 5 Hz Poisson background per synapse. Synthetic, seeded inputs
(synth.cortex_50k).

One benchmark step = one minimum-delay interval (40 time steps: delivery, mechanisms, assembly, tree solve,
threshold detection, and the interval's spike fan-out). Inputs are resident in HBM before the timed region. The
main line reports the FP64 path; beside it: the FP32-mechanism path on the same workload, the other workloads
(clamped_cells, ring_network in both precisions, cortex_200k in both precisions) as microseconds per time step, the
roofline of the dominant kernel and the oracle timed on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# vector ALU lane-operation peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one wave64 instruction issues over four
# cycles; FP64 and unpacked FP32 instructions alike). The FP64 FLOP peak (78.6 TFLOP/s) counts an FMA as two.
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
PROFILE = os.path.join(ROOT, "profiles", "cn_interval_cortex50k_traffic.json")
VALU_PROFILE = os.path.join(ROOT, "profiles", "cn_interval_cortex50k_valu.json")


def bytes_per_step(m, fp32: bool) -> float:
    """Algorithmic HBM bytes one time step of the per-step method must move: per compartment v read+write (16) and
    read-only parent index, a, b and the diagonal constant (28); per mechanism state a read and a write; per synapse
    g read+write, its compartment index and scale (12). Events are negligible and not counted."""
    s = 4 if fp32 else 8
    n = m.n_comp
    states = {"hh": 3, "km": 1, "cahi": 2}
    b = n * (16 + 28)
    for name, k in states.items():
        if name in m.mechs:
            b += m.mechs[name].count(n) * 2 * s * k
    b += m.n_syn * (2 * s + 12)
    return float(b)


def kernel_sources_sha256() -> str:
    h = hashlib.sha256()
    for f in ("cn_kernels.hip", "cn_internal.h", "cn_host.cpp"):
        with open(os.path.join(ROOT, "paper_1901_10975_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _profile(path, precision, info=None):
    """one kernel's record of a committed counter profile, or None when the kernel sources changed since it was
    taken, or when the run (its cn_model_info) used another group shape than the profiled kernel"""
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("source_sha256") != kernel_sources_sha256():
        return None
    k = rec.get("kernels", {}).get(precision)
    if k is not None and info is not None:
        shape = f"cn_interval<{info['group_threads']}, {info['group_slots']},"
        if info.get("layout") != 1 or shape not in k.get("kernel", ""):
            return None
    return k


def run_gpu(m, precision, steps, warmup, log, **kw):
    import torch
    from paper_1901_10975_amd import cn

    t0 = time.time()
    eng = cn.Engine(m, precision=precision, timing=True, use_graph=True, **kw)
    tune = eng.tune
    if tune is not None:
        log(f"[bench] {m.name} {precision}: autotuned in {time.time() - t0:.1f} s: {tune['layout']} "
            f"{tune['group_threads']}x{tune['group_slots']} fill {tune['group_fill_pct']} at {tune['interval_ms']:.3f} ms "
            f"per interval (default {tune['default_threads']}x{tune['default_slots']} {tune['default_ms']:.3f} ms, "
            f"{len(tune['candidates'])} candidates)")
    log(f"[bench] {m.name} {precision}: model {'tuned and ' if tune is not None else ''}built in "
        f"{time.time() - t0:.1f} s")
    eng.run_to_step(1)  # fixes dt, hence the interval length, and captures the interval graph
    M = eng.info()["interval_steps"]
    eng.run_to_step(max(1, warmup) * M)
    info = eng.info()
    n0 = info["step"]
    ms0, l0 = eng.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eng.run_to_step(n0 + steps * M)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms1, l1 = eng.stats()
    launches = l1 - l0
    kernel_ms = (ms1 - ms0) / max(1, launches)
    g, s, _ = eng.spikes()
    res = dict(wall=wall, M=M, steps=steps, kernel_ms=kernel_ms, launches=launches, info=info,
               n_spikes=int(g.size), comp_steps=float(m.n_comp) * steps * M, tune=tune)
    res["value"] = res["comp_steps"] / wall
    res["us_per_step"] = wall / (steps * M) * 1e6
    log(f"[bench] {m.name} {precision}: {steps} intervals x {M} steps in {wall:.3f} s -> {res['value']:.4e} "
        f"comp-steps/s ({res['us_per_step']:.2f} us/step); interval kernel {kernel_ms:.3f} ms avg over {launches}; "
        f"spikes so far {g.size}")
    eng.close()
    return res


def _oracle_rate(sub, threads, budget_s, M):
    """compartment-steps/s of the oracle on `sub`, advanced interval by interval until the time budget is used"""
    from oracle import oracle as O

    orc = O.OracleSim(sub, n_threads=threads, fast=True)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        n += M
        orc.run_to_step(n)
    el = time.perf_counter() - t0
    return sub.n_comp * n / el, n, el


def host_threads() -> int:
    """the host cores this process may use: the OpenMP thread count the environment grants, else the affinity set"""
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        cores = min(cores, int(env))
    return max(1, int(cores))


def cpu_baseline(m, M, log, budget_s=15.0, budget_1_s=8.0):
    """The oracle, as it stands, on every host core granted to this process over a bounded sample of the same
    workload: a random 5% of the cells (with their synapses, background streams and the NetCons among them),
    advanced interval by interval until the time budget is used; and on one core over a random 1% of the cells.
    Timed with the oracle compiled -O3 -march=native for this host (no FMA contraction)."""
    import numpy as np

    from oracle import oracle as O
    from paper_1901_10975_amd import synth

    O.build_fast()
    cores = host_threads()
    rng = np.random.default_rng(0)
    cells = np.sort(rng.choice(m.n_cells, max(1, m.n_cells // 20), replace=False))
    sub = synth.subset_cells(m, cells)
    val, n, el = _oracle_rate(sub, cores, budget_s, M)
    log(f"[bench] oracle: {sub.n_cells} cells / {sub.n_comp} compartments x {n} steps in {el:.1f} s on {cores} "
        f"threads -> {val:.3e} comp-steps/s")
    cells1 = np.sort(rng.choice(m.n_cells, max(1, m.n_cells // 100), replace=False))
    sub1 = synth.subset_cells(m, cells1)
    val1, n1, el1 = _oracle_rate(sub1, 1, budget_1_s, M)
    log(f"[bench] oracle: {sub1.n_cells} cells / {sub1.n_comp} compartments x {n1} steps in {el1:.1f} s on 1 "
        f"thread -> {val1:.3e} comp-steps/s")
    return {"value": val, "unit": "compartment-timesteps/s", "cores": cores, "kind": "oracle",
            "sample": f"{sub.n_cells} random cells of the workload ({sub.n_comp} compartments, their synapses, "
                      f"background streams and internal NetCons), {n} steps of 0.025 ms, FP64, {cores} threads, "
                      f"oracle built -O3 -march=native -ffp-contract=off",
            "cpu_model": O.cpu_model(), "host_cpus_visible": os.cpu_count(),
            "single_core": {"value": val1, "cores": 1,
                            "sample": f"{sub1.n_cells} random cells ({sub1.n_comp} compartments), {n1} steps, FP64"}}


def roofline(m, r64, fp32_res=None):
    """Roofline object of the dominant kernel (the FP64 interval kernel). achieved = the per-step method's
    algorithmic HBM bytes of one launch (bytes_per_step x steps per launch) / the launch's mean duration, against the
    8 TB/s HBM peak; traffic = measured HBM bytes per launch from the committed counter passes (null once the kernel
    changed). The kernel keeps a group on chip for a whole interval, so it moves far fewer bytes than the byte model
    counts; the vector-ALU view (measured VALU lane instructions against the lane-operation peak) is reported beside
    it and becomes the bound if the byte-model fraction would exceed one."""
    per_launch = bytes_per_step(m, False) * r64["M"]
    kern_s = r64["kernel_ms"] * 1e-3
    eff_gbs = per_launch / kern_s / 1e9
    tr = _profile(PROFILE, "fp64", r64["info"])
    traffic = None if tr is None else float(tr["traffic_bytes"])
    cnt = _profile(VALU_PROFILE, "fp64", r64["info"])
    alu = None
    if cnt is not None:
        lane = float(cnt["valu_lane_insts_per_comp_step"]) * m.n_comp * r64["M"] / kern_s
        alu = {"bound": "alu", "achieved": lane / 1e12, "peak": VALU_PEAK_LANE_OPS / 1e12,
               "unit": "T VALU lane-instructions/s", "frac": lane / VALU_PEAK_LANE_OPS,
               "valu_busy": cnt["valu_busy"], "fp64_tflops_counted": cnt["fp64_tflops"],
               "valu_lane_instr_per_comp_step": cnt["valu_lane_insts_per_comp_step"]}
    hbm = {"bound": "hbm", "achieved": eff_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": eff_gbs / HBM_PEAK_GBS,
           "traffic": traffic, "algorithmic_bytes_per_launch": per_launch,
           "bytes_per_unit": "140 B per compartment-step + 28 B per synapse-step (FP64)"}
    out = dict(hbm)
    if hbm["frac"] > 1.0 and alu is not None:
        out = dict(alu)
        out["traffic"] = traffic
        out["hbm_byte_model"] = hbm
    else:
        out["alu"] = alu
    out["kernel"] = "cn_interval<%d,%d,double>" % (r64["info"]["group_threads"], r64["info"]["group_slots"])
    out["kernel_ms"] = r64["kernel_ms"]
    out["measured_hbm_GBs"] = None if traffic is None else traffic / kern_s / 1e9
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed minimum-delay intervals of the main workload")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-cells", type=int, default=50000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run the main workload at the default cell-group shape instead of the autotuner's choice")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip clamped_cells, ring_network and cortex_200k")
    ap.add_argument("--only", choices=["cortex_50k", "cortex_200k"], default=None,
                    help="run one workload in both precisions and print its line only")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a plain 256 MiB device-to-device copy (calibrates HBM byte counters)")
    ap.add_argument("--ordering-study", action="store_true",
                    help="the node-ordering study: ring_types (131,072 cells x 83 compartments, 10 ms) with 1-64 "
                         "identical cells per type on the level and the interleaved layout; prints its own line")
    ap.add_argument("--study-cells", type=int, default=131072)
    ap.add_argument("--study-rows", default="1,2,4,8,16,32,64",
                    help="identical cells per type of the ordering study's rows (comma-separated)")
    ap.add_argument("--restart-study", action="store_true",
                    help="checkpoint-restart at full size (cortex_50k, both precisions): time the checkpoint and the "
                         "restore, and check that the split run equals the uninterrupted one bitwise; prints its own "
                         "line")
    ap.add_argument("--phase-clocks", action="store_true",
                    help="load the profiling build (libcn_phase.so) and print where the interval kernel's time goes "
                         "on cortex_50k, per phase, in both precisions; prints its own line")
    args = ap.parse_args()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this engine has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        sys.exit(1)
    from paper_1901_10975_amd import synth

    if args.copy_probe:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {a.numel() * 4} bytes read and written")
        del a, b

    if args.ordering_study:
        rows = tuple(int(x) for x in args.study_rows.split(","))
        print(json.dumps(ordering_study(log, synth, args.study_cells, rows)), flush=True)
        return

    if args.restart_study:
        print(json.dumps(restart_study(log, synth, args.n_cells)), flush=True)
        return

    if args.phase_clocks:
        print(json.dumps(phase_clocks(log, synth, args.n_cells, args.steps, args.warmup)), flush=True)
        return

    if args.only == "cortex_200k":
        m = synth.cortex_200k()
        log(f"[bench] cortex_200k: {m.n_cells} cells, {m.n_comp} compartments, {m.n_syn} synapses")
        r64 = run_gpu(m, "fp64", args.steps, args.warmup, log)
        r32 = run_gpu(m, "fp32_mech", args.steps, args.warmup, log)
        print(json.dumps({"workload": "cortex_200k", "n_comp": m.n_comp, "fp64": _brief(r64, m),
                          "fp32_mech": _brief(r32, m, True)}), flush=True)
        return

    t0 = time.time()
    m = synth.cortex_50k(n_cells=args.n_cells)
    log(f"[bench] cortex_50k: {m.n_cells} cells, {m.n_comp} compartments, {m.n_syn} synapses "
        f"(generated in {time.time() - t0:.1f} s)")
    tkw = {} if args.no_autotune else {"autotune": True, "tune_budget_ms": 60000.0}
    r64 = run_gpu(m, "fp64", args.steps, args.warmup, log, **tkw)
    r32 = None if args.no_fp32 else run_gpu(m, "fp32_mech", args.steps, args.warmup, log, **tkw)

    out = {
        "metric": "compartment-timesteps/sec at 50k cells (FP64 vs FP32-mech); HBM GB/s fraction",
        "value": r64["value"],
        "unit": "compartment-timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "cortex_50k: 50000 cells, log-uniform 50-1000 compartments (%d total), hh+km+cahi, "
                               "100 ExpSyn/cell, NetCon delay U(1,5) ms, Poisson 5 Hz, dt 0.025 ms; one step = one "
                               "1 ms min-delay interval (40 time steps)" % m.n_comp,
                   "n_cells": m.n_cells, "n_comp": m.n_comp, "n_syn": m.n_syn, "interval_steps": r64["M"],
                   "group_threads": r64["info"]["group_threads"], "group_slots": r64["info"]["group_slots"],
                   "layout": "interleaved" if r64["info"]["layout"] == 2 else "level",
                   "autotune": _tune_brief(r64["tune"])},
        "us_per_time_step": r64["us_per_step"],
        "roofline": roofline(m, r64),
    }
    if r32 is not None:
        out["fp32_mech"] = _brief(r32, m, True)
        out["fp32_mech"]["group_shape"] = [r32["info"]["group_threads"], r32["info"]["group_slots"]]
        out["fp32_mech"]["autotune"] = _tune_brief(r32["tune"])
        out["fp32_mech"]["speedup_vs_fp64"] = r32["value"] / r64["value"]
        out["fp32_mech"]["meets_1p5x_target"] = bool(r32["value"] / r64["value"] >= 1.5)
    if not args.no_other_configs and args.only is None:
        out["other_configs"] = other_configs(log, synth)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m, r64["M"], log)
        out["cpu_baseline"]["gpu_over_oracle"] = r64["value"] / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


def _tune_brief(t):
    """the autotuner's choice for a bench line (None when the default shape ran)"""
    if t is None:
        return None
    return {"chosen": f"{t['layout']} {t['group_threads']}x{t['group_slots']} fill {t['group_fill_pct']}",
            "interval_ms": t["interval_ms"], "default": f"level {t['default_threads']}x{t['default_slots']} fill 100",
            "default_ms": t["default_ms"], "gain_over_default": t["default_ms"] / t["interval_ms"],
            "candidates": [f"{c['layout']} {c['threads']}x{c['slots']} fill {c['fill_pct']}: {c['interval_ms']:.3f} ms"
                           for c in t["candidates"]]}


def _brief(r, m, fp32=False):
    bps = bytes_per_step(m, fp32)
    return {"value": r["value"], "unit": "compartment-timesteps/s", "us_per_time_step": r["us_per_step"],
            "interval_steps": r["M"], "kernel_ms": r["kernel_ms"],
            "effective_hbm_frac": bps * r["M"] / (r["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "counters": _profile(VALU_PROFILE, "fp32_mech" if fp32 else "fp64", r["info"])}


def other_configs(log, synth):
    """the remaining workloads: clamped_cells (64 x 32, 100 ms), ring_network (1000 x 200, 200 ms FP64; 100 ms in the
    FP32-mechanism path), cortex_200k (200,000 cells, 50 ms, both precisions), and the ring_types workload with and
    without gap junctions (FP64). The small ones fit in L2 or the Infinity Cache: their figure is microseconds per
    time step."""
    res = {}
    for name, make, prec, tstop in (("clamped_cells", synth.clamped_cells, "fp64", 100.0),
                                    ("ring_network", synth.ring_network, "fp64", 200.0),
                                    ("ring_network_fp32_mech", synth.ring_network, "fp32_mech", 100.0)):
        m = make()
        r = run_gpu_whole(m, prec, tstop, log)
        res[name] = r
    m = synth.cortex_200k()
    log(f"[bench] cortex_200k: {m.n_cells} cells, {m.n_comp} compartments, {m.n_syn} synapses")
    for prec in ("fp64", "fp32_mech"):
        r = run_gpu(m, prec, 100, 2, log)
        res["cortex_200k_" + prec] = _brief(r, m, prec == "fp32_mech")
    res["cortex_200k_fp32_mech"]["speedup_vs_fp64"] = (res["cortex_200k_fp32_mech"]["value"]
                                                       / res["cortex_200k_fp64"]["value"])
    # gap junctions: the node-ordering workload (131,072 cells x 83 compartments, 8 identical cells per type) with
    # and without electrical coupling inside clusters of four cells (every pair joined once, 0.01 uS; three joined
    # sets of 332 compartments fill a 1,024-compartment group as well as the single cells do)
    for name, gap in (("ring_types_fp64", False), ("ring_types_gap_fp64", True)):
        m = synth.ring_types(n_cells=131072, cells_per_type=8)
        if gap:
            m = synth.add_gap_junctions(m, cluster=4, per_pair=1, g=0.01)
        log(f"[bench] {name}: {m.n_cells} cells, {m.n_comp} compartments, {m.n_gap} half-gap junctions")
        r = run_gpu(m, "fp64", 20, 1, log)
        res[name] = _brief(r, m)
        res[name]["n_half_gaps"] = int(m.n_gap)
    res["ring_types_gap_fp64"]["relative_to_uncoupled"] = (res["ring_types_gap_fp64"]["value"]
                                                           / res["ring_types_fp64"]["value"])
    return res


def ordering_study(log, synth, n_cells, per_type=(1, 2, 4, 8, 16, 32, 64)):
    """Sec. 4.4's node-ordering experiment on this engine: ring_types (n_cells x 83 compartments, random branching
    per type, hh soma, pas dendrites) for 1 to 64 identical cells per type, 10 ms of simulated time after a one-
    interval warm-up, FP64, on the level layout (constant-depth order, level-parallel solve on chip) and the
    interleaved layout (one lane per cell, serial solve in global memory). Wall time of the 10 ms and the mean
    interval-kernel time from HIP events."""
    import torch
    from paper_1901_10975_amd import cn

    rows = []
    for k in per_type:
        m = synth.ring_types(n_cells=n_cells, cells_per_type=k)
        row = {"cells_per_type": k}
        for layout in ("level", "interleaved"):
            eng = cn.Engine(m, precision="fp64", timing=True, layout=layout)
            eng.run_to_step(40)
            ms0, l0 = eng.stats()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eng.run_to_step(40 + 400)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ms1, l1 = eng.stats()
            g, _, _ = eng.spikes()
            row[layout] = {"wall_ms_10ms": wall * 1e3, "kernel_ms_per_interval": (ms1 - ms0) / max(1, l1 - l0),
                           "us_per_step": wall / 400 * 1e6, "comp_steps_per_s": m.n_comp * 400 / wall,
                           "spikes": int(g.size)}
            log(f"[study] {k} per type, {layout}: 10 ms in {wall * 1e3:.1f} ms ({wall / 400 * 1e6:.1f} us/step), "
                f"interval kernel {row[layout]['kernel_ms_per_interval']:.3f} ms, {g.size} spikes")
            eng.close()
        row["interleaved_over_level"] = row["interleaved"]["wall_ms_10ms"] / row["level"]["wall_ms_10ms"]
        rows.append(row)
    return {"study": "node ordering (Sec. 4.4)", "workload": f"ring_types: {n_cells} cells x 83 compartments, "
            "hh soma, pas dendrites, one ExpSyn per cell in rings of 128, 10 ms at dt 0.025 ms, FP64",
            "n_comp": n_cells * 83, "rows": rows}


def restart_study(log, synth, n_cells, n_split=6, n_end=12):
    """Checkpoint-restart (Sec. 3.4) on the benchmark workload: run to interval n_split, take the checkpoint (the
    readouts: potentials, every state, the spikes), restore it into a fresh model and continue to interval n_end;
    the continued run must equal the uninterrupted one bitwise (potentials, states, the spikes after the split)."""
    import numpy as np
    import torch
    from paper_1901_10975_amd import cn

    m = synth.cortex_50k(n_cells=n_cells)
    out = {"study": "checkpoint-restart", "workload": f"cortex_50k: {m.n_cells} cells, {m.n_comp} compartments"}
    for prec in ("fp64", "fp32_mech"):
        whole = cn.Engine(m, precision=prec)
        whole.run_to_step(1)
        M = whole.info()["interval_steps"]
        whole.run_to_step(n_end * M)
        a = cn.Engine(m, precision=prec)
        a.run_to_step(n_split * M + M // 2)  # inside an interval: events in flight, a pending state update
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ck = a.checkpoint()
        t_ck = time.perf_counter() - t0
        nbytes = sum(np.asarray(x).nbytes for x in (ck["v"], ck["gid"], ck["spike_step"])) + \
            sum(x.nbytes for x in ck["states"].values())
        a.close()
        t0 = time.perf_counter()
        b = cn.Engine(m, precision=prec)
        t_build = time.perf_counter() - t0
        t0 = time.perf_counter()
        b.restore(ck)
        torch.cuda.synchronize()
        t_restore = time.perf_counter() - t0
        b.run_to_step(n_end * M)
        cw, cb = whole.checkpoint(), b.checkpoint()
        same = bool(np.array_equal(cw["v"], cb["v"]) and all(np.array_equal(cw["states"][k], cb["states"][k])
                                                            for k in cw["states"]))
        gw, sw, tw = whole.spikes()
        gb, sb, tb = b.spikes()
        keep = sw > ck["step"]
        same_spikes = bool(np.array_equal(gw[keep], gb) and np.array_equal(sw[keep], sb) and
                           np.array_equal(tw[keep], tb))
        rec = {"split_step": int(ck["step"]), "end_step": n_end * M, "checkpoint_s": t_ck, "checkpoint_bytes": nbytes,
               "model_build_s": t_build, "restore_s": t_restore, "spikes_before_split": int(ck["gid"].size),
               "spikes_after_split": int(gb.size), "identical_state": same, "identical_spikes": same_spikes}
        log(f"[restart] {prec}: checkpoint at step {ck['step']} in {t_ck:.2f} s ({nbytes / 1e6:.0f} MB), restore "
            f"{t_restore:.2f} s after a {t_build:.1f} s build; {gb.size} spikes after the split; identical "
            f"{same and same_spikes}")
        out[prec] = rec
        for e in (whole, b):
            e.close()
    return out


def phase_clocks(log, synth, n_cells, steps, warmup):
    """Per-phase shader clocks of the interval kernel (profiling build) on cortex_50k: the first wave of every group
    sums the clock between the barriers that close each phase; the sums over the timed intervals, per group-step and
    as shares. The kernel time from HIP events is printed beside them: the profiling marks cost a few scalar
    instructions per phase."""
    import torch
    from paper_1901_10975_amd import build as B, cn

    if not os.path.exists(B.LIB_PHASE):
        raise SystemExit(f"{B.LIB_PHASE} is missing: build it with paper_1901_10975_amd/build.py --phase-clocks")
    if cn._lib is not None and cn.LIB_PATH != B.LIB_PHASE:
        raise SystemExit("the ordinary library is already loaded in this process; run --phase-clocks on its own")
    cn.LIB_PATH = B.LIB_PHASE
    m = synth.cortex_50k(n_cells=n_cells)
    out = {"study": "interval-kernel phases", "workload": f"cortex_50k: {m.n_cells} cells, {m.n_comp} compartments",
           "library": os.path.basename(B.LIB_PHASE), "phases": list(cn.PHASES)}
    for prec in ("fp64", "fp32_mech"):
        eng = cn.Engine(m, precision=prec, timing=True, use_graph=True)
        eng.run_to_step(1)
        M = eng.info()["interval_steps"]
        eng.run_to_step(max(1, warmup) * M)
        c0, (ms0, l0) = eng.phase_clocks(), eng.stats()
        n0 = eng.info()["step"]
        eng.run_to_step(n0 + steps * M)
        torch.cuda.synchronize()
        c1, (ms1, l1) = eng.phase_clocks(), eng.stats()
        info = eng.info()
        d = {k: c1[k] - c0[k] for k in c1}
        tot = sum(d.values())
        gs = info["n_groups"] * steps * M
        rec = {"kernel_ms": (ms1 - ms0) / max(1, l1 - l0), "group_shape": [info["group_threads"], info["group_slots"]],
               "groups_per_cu": info["groups_per_cu"], "n_groups": info["n_groups"],
               "cycles_per_group_step": {k: v / gs for k, v in d.items()},
               "share": {k: v / tot for k, v in d.items()}}
        log(f"[phases] {prec}: interval kernel {rec['kernel_ms']:.3f} ms; per group-step cycles "
            + ", ".join(f"{k} {v:.0f}" for k, v in rec["cycles_per_group_step"].items()))
        out[prec] = rec
        eng.close()
    return out


def run_gpu_whole(m, precision, tstop, log):
    """a whole run of a small workload (warm-up: a short throw-away run), timed end to end"""
    import torch
    from paper_1901_10975_amd import cn

    w = cn.Engine(m, precision=precision)
    w.run(2.0)
    w.close()
    eng = cn.Engine(m, precision=precision, timing=True)
    eng.run_to_step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eng.run(tstop)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n = int(round(tstop / m.dt)) - 1
    g, _, _ = eng.spikes()
    ms, launches = eng.stats()
    r = {"us_per_time_step": wall / n * 1e6, "steps": n, "value": m.n_comp * n / wall,
         "unit": "compartment-timesteps/s", "precision": precision, "n_comp": m.n_comp, "spikes": int(g.size),
         "interval_steps": eng.info()["interval_steps"], "kernel_ms_mean": ms / max(1, launches)}
    log(f"[bench] {m.name} {precision}: {tstop} ms = {n} steps in {wall:.3f} s -> {r['us_per_time_step']:.2f} "
        f"us/step, {g.size} spikes")
    eng.close()
    return r


if __name__ == "__main__":
    main()
