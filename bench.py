"""Benchmark: compartment-timesteps per second of the fixed-step cable engine on one MI355X.

Workload: cortex_50k - 50,000 cells with log-uniform 50..1000 compartments (15.93M compartments), hh + km + cahi in
every compartment, 100 ExpSyn per cell fed by NetCons with delays U(1, 5) ms (1 ms minimum-delay interval, 40 steps
of 0.025 ms) and 5 Hz Poisson background per synapse. Synthetic, seeded inputs (synth.cortex_50k).

One benchmark step = one minimum-delay interval (40 time steps: delivery, mechanisms, assembly, tree solve,
threshold detection, and the interval's spike fan-out). Inputs are resident in HBM before the timed region.
The main line reports the FP64 path; the FP32-mechanism path is reported beside it.
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
# FP64 vector peak: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2 flops (FMA) x 2.4 GHz
FP64_PEAK_TFLOPS = 78.6
# algorithmic FP64 work per compartment-step of cortex_50k (hh, km, cahi rates and gates, currents, assembly and the
# tree solve): about 500 lane operations, each exponential or divide counted as the operations it takes
FLOPS_PER_COMP_STEP = 500.0
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


def profiled_traffic(precision: str):
    """HBM bytes per interval launch from the committed counter passes, or None when the kernel sources changed
    since they were taken"""
    try:
        with open(PROFILE) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("source_sha256") != kernel_sources_sha256():
        return None
    k = rec.get("kernels", {}).get(precision)
    return None if k is None else float(k["traffic_bytes"])


def profiled_valu(precision: str):
    """VALU busy fraction and measured FP64 TFLOP/s of the interval kernel from the committed counter passes, or
    None when the kernel sources changed since they were taken"""
    try:
        with open(VALU_PROFILE) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("source_sha256") != kernel_sources_sha256():
        return None
    k = rec.get("kernels", {}).get(precision)
    return None if k is None else {"valu_busy": k["valu_busy"], "measured_fp64_tflops": k["fp64_tflops"]}


def run_gpu(m, precision, steps, warmup, log):
    import torch
    from paper_1901_10975_amd import cn

    t0 = time.time()
    eng = cn.Engine(m, precision=precision, timing=True, use_graph=True)
    log(f"[bench] {precision}: model built in {time.time() - t0:.1f} s")
    dt = m.dt
    # warm-up (also fixes dt and captures the interval graph)
    eng.run_to_step(0 + max(1, warmup) * 40)
    info = eng.info()
    M = info["interval_steps"]
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
               n_spikes=int(g.size), comp_steps=float(m.n_comp) * steps * M)
    res["value"] = res["comp_steps"] / wall
    log(f"[bench] {precision}: {steps} intervals x {M} steps in {wall:.3f} s -> {res['value']:.4e} comp-steps/s; "
        f"interval kernel {kernel_ms:.3f} ms avg over {launches}; spikes so far {g.size}")
    eng.close()
    return res


def _oracle_rate(sub, threads, budget_s):
    """compartment-steps/s of the oracle on `sub`, advanced interval by interval until the time budget is used"""
    from oracle import oracle as O

    orc = O.OracleSim(sub, n_threads=threads)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        n += 40
        orc.run_to_step(n)
    el = time.perf_counter() - t0
    return sub.n_comp * n / el, n, el


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(m, log, budget_s=12.0, budget_1_s=8.0):
    """The oracle, as it stands, on the host cores over a bounded sample of the same workload: a random 5% of the
    cells (with their synapses, background streams and the NetCons among them), advanced interval by interval until
    the time budget is used; and on one core over a random 1% of the cells."""
    import numpy as np

    from paper_1901_10975_amd import synth

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(int(cores), 16))
    rng = np.random.default_rng(0)
    cells = np.sort(rng.choice(m.n_cells, max(1, m.n_cells // 20), replace=False))
    sub = synth.subset_cells(m, cells)
    val, n, el = _oracle_rate(sub, cores, budget_s)
    log(f"[bench] oracle: {sub.n_cells} cells / {sub.n_comp} compartments x {n} steps in {el:.1f} s on {cores} "
        f"threads -> {val:.3e} comp-steps/s")
    cells1 = np.sort(rng.choice(m.n_cells, max(1, m.n_cells // 100), replace=False))
    sub1 = synth.subset_cells(m, cells1)
    val1, n1, el1 = _oracle_rate(sub1, 1, budget_1_s)
    log(f"[bench] oracle: {sub1.n_cells} cells / {sub1.n_comp} compartments x {n1} steps in {el1:.1f} s on 1 "
        f"thread -> {val1:.3e} comp-steps/s")
    return {"value": val, "unit": "compartment-timesteps/s", "cores": cores, "kind": "oracle",
            "sample": f"{sub.n_cells} random cells of the workload ({sub.n_comp} compartments, their synapses, "
                      f"background streams and internal NetCons), {n} steps of 0.025 ms, FP64, {cores} threads",
            "cpu_model": _cpu_model(),
            "single_core": {"value": val1, "cores": 1,
                            "sample": f"{sub1.n_cells} random cells ({sub1.n_comp} compartments), {n1} steps, FP64"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed minimum-delay intervals (40 steps each)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-cells", type=int, default=50000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a plain 256 MiB device-to-device copy (calibrates HBM byte counters)")
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

    t0 = time.time()
    m = synth.cortex_50k(n_cells=args.n_cells)
    log(f"[bench] cortex_50k: {m.n_cells} cells, {m.n_comp} compartments, {m.n_syn} synapses "
        f"(generated in {time.time() - t0:.1f} s)")
    r64 = run_gpu(m, "fp64", args.steps, args.warmup, log)
    r32 = None if args.no_fp32 else run_gpu(m, "fp32_mech", args.steps, args.warmup, log)

    bps = bytes_per_step(m, False)
    per_launch = bps * r64["M"]
    kern_s = r64["kernel_ms"] * 1e-3
    eff_gbs = per_launch / kern_s / 1e9  # the per-step method's bytes at this rate
    flops_launch = FLOPS_PER_COMP_STEP * m.n_comp * r64["M"]
    achieved = flops_launch / kern_s / 1e12
    traffic = profiled_traffic("fp64")
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
                   "n_cells": m.n_cells, "n_comp": m.n_comp, "n_syn": m.n_syn, "interval_steps": r64["M"]},
        # The interval kernel keeps a group's potentials, states and constants on chip for all M steps, so it moves
        # far fewer HBM bytes than the per-step method: the bound is FP64 vector arithmetic and the latency of the
        # tree sweeps, not HBM. traffic = measured HBM bytes per launch (calibrated counters).
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": "cn_interval<%d,%d,double>" % (r64["info"]["group_threads"], r64["info"]["group_slots"]),
                     "kernel_ms": r64["kernel_ms"], "flops_per_launch": flops_launch,
                     "measured_hbm_GBs": None if traffic is None else traffic / kern_s / 1e9,
                     "effective_hbm_GBs": eff_gbs, "effective_hbm_frac": eff_gbs / HBM_PEAK_GBS,
                     "per_step_method_bytes_per_launch": per_launch,
                     "counters": profiled_valu("fp64")},
    }
    if r32 is not None:
        bps32 = bytes_per_step(m, True)
        out["fp32_mech"] = {"value": r32["value"], "ms_per_step": r32["wall"] / args.steps * 1e3,
                            "kernel_ms": r32["kernel_ms"],
                            "speedup_vs_fp64": r32["value"] / r64["value"],
                            "effective_GBs": bps32 * r32["M"] / (r32["kernel_ms"] * 1e-3) / 1e9,
                            "traffic": profiled_traffic("fp32_mech"), "counters": profiled_valu("fp32_mech")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m, log)
        out["cpu_baseline"]["gpu_over_oracle"] = r64["value"] / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
