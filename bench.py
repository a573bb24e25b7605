"""Benchmark of the D2V16 multi-component DBM step on one MI355X.

Workload (default): the three-species reacting premix on a 256x256 periodic
grid (fuel/oxidiser/product, molar masses 2, 32, 18; one-step Arrhenius
reaction k = 1e3 exp(-10/T); hot Gaussian kernel T = 3, sigma = 10 cells;
+-1% seeded density noise; dt = 1e-5, tau = 2e-5), FP32-bulk storage, forward
Euler + NND (the paper's scheme).  A "step" is one full time step of the
update: convection, moments, equilibrium, BGK + reaction + force, combine.

Prints ONE JSON line.  `value` is cell-species updates per second over the K
timed steps (graph-replayed, inputs resident in HBM).  `roofline` is for the
one-pass stage kernel, the only kernel of a step: algorithmic bytes (32
values of f read+written per cell-species per Euler step) over its mean
launch duration, which is the HIP-event time of the timed region (events
recorded on the library's stream) divided by the launches in it.
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same
workload on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --mode traffic --workload c4   (for rocprofv3 --pmc)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell·species updates/s + % HBM peak, FP32-bulk vs FP64 at stated L∞ error"
UNIT = "cell-species updates/s"

# HBM bytes per launch of the one-pass stage kernel, from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE runs (profiles/fused_stage_traffic.md), keyed by
# workload, with the hash of the kernel code they were taken at (source
# without comments, see code_text).  Changed kernel code makes the entry stale
# and `traffic` is reported as null.
MEASURED_TRAFFIC = {
    "c1/fp32": {"source": "a12b2d61298798f0", "bytes_per_launch": 26489788},
    "c4/fp32": {"source": "a12b2d61298798f0", "bytes_per_launch": 9607444038},
}


def code_text(src: str) -> str:
    """Source text without // comments and blank lines, trailing spaces
    stripped: what the compiler sees of the kernel, so that a comment edit
    does not mark the traffic measurement stale."""
    lines = []
    for line in src.splitlines():
        line = re.sub(r"//.*$", "", line).rstrip()
        if line:
            lines.append(line)
    return "\n".join(lines)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("dbm_kernels.hip", "dbm_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2006_15932_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def workload(name: str, precision: str):
    from paper_2006_15932_amd import workloads as W
    if name == "c1":
        return W.reacting(n=256, steps=5000, precision=precision), (
            "C1: 3-species reacting premix, 256x256 periodic, Euler+NND, dt=1e-5, tau=2e-5")
    if name == "c2":
        return W.rayleigh_taylor(n=1024, steps=20000, precision=precision), (
            "C2: 4-species Rayleigh-Taylor, 1024x1024, walls in y, g=(0,-0.1), Euler+NND")
    if name == "c4":
        return W.shear_layer(n=4096, steps=5000, precision=precision), (
            "C4: 4-species reacting supersonic double shear layer, 4096x4096 periodic, Euler+NND")
    raise SystemExit("unknown workload " + name)


def bytes_per_csu(precision: str, scheme: int) -> int:
    es = 4 if precision == "fp32" else 8
    return es * (32 if scheme == 0 else 128)


def gpu_run(p, precision, steps, warmup, tile_rows=0, pipeline=0, rounding=0, chain_wave=0):
    import torch
    from paper_2006_15932_amd import dbm as D
    sim = D.Simulation(p, precision=precision)
    assert sim.get_option(D.DBM_OPT_PATH) == 0, "one-pass HIP path not active"
    if rounding:
        sim.set_option(D.DBM_OPT_ROUNDING, rounding)
    if tile_rows:
        sim.set_option(D.DBM_OPT_TILE_ROWS, tile_rows)
    if pipeline:
        sim.set_option(D.DBM_OPT_PIPELINE, pipeline)
    if chain_wave:
        sim.set_option(D.DBM_OPT_CHAIN_WAVE, chain_wave)
    sim.set_fields()
    sim.step(warmup)
    sim.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(sim.stream)
    sim.step(steps)
    stop.record(sim.stream)
    stop.synchronize()
    ms = start.elapsed_time(stop)
    launches = steps * (1 if p.scheme == 0 else 3)
    kern_ms = ms / launches
    rows = sim.get_option(D.DBM_OPT_TILE_ROWS)
    sim.pipeline_in_use = sim.get_option(D.DBM_OPT_PIPELINE)
    sim.chain_wave_in_use = sim.get_option(D.DBM_OPT_CHAIN_WAVE)
    return sim, ms, kern_ms, rows


def errors_vs_oracle(n=64, steps=200):
    """FP32-bulk (round to nearest and stochastic rounding), FP32X and FP64
    runs of the same setup on an n x n instance against the FP64 CPU oracle
    (relative L-infinity per field)."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_helpers import field_errors, oracle_run
    from paper_2006_15932_amd import dbm as D
    from paper_2006_15932_amd import workloads as W
    p = W.reacting(n=n, steps=steps)
    o, fo = oracle_run(p, steps)
    mo = o.moments(fo)
    out = {}
    for key, prec, rnd in (("fp32", "fp32", 0), ("fp32_stochastic_rounding", "fp32", 1),
                           ("fp32x", "fp32x", 0), ("fp64", "fp64", 0)):
        sim = D.Simulation(p, precision=prec)
        if rnd:
            sim.set_option(D.DBM_OPT_ROUNDING, rnd)
        sim.set_fields()
        sim.step(steps)
        e = field_errors(p, sim.moments(), mo)
        out[key] = {k: float("%.3e" % v) for k, v in e.items()}
        sim.close()
    return out


def batched(steps=200):
    """C3: 64 independent reacting instances of uneven size (64^2 .. 512^2,
    per-instance tau and hot-spot T), FP32-bulk: one persistent launch per
    stage for all instances vs one launch per instance, both graph-replayed."""
    import torch
    from paper_2006_15932_amd import dbm as D
    from paper_2006_15932_amd import workloads as W
    probs = W.batch(count=64, steps=steps, precision="fp32")
    csu = sum(p.S * p.cells for p in probs)
    out = {"workload": "C3: 64 reacting instances, sizes in {64,128,256,512}^2, FP32-bulk, Euler",
           "instances": len(probs), "cell_species_per_step": csu}
    for mode, key in ((0, "persistent"), (1, "per_instance")):
        sim = D.Simulation(probs, precision="fp32")
        sim.set_option(D.DBM_OPT_BATCH_MODE, mode)
        for k in range(len(probs)):
            sim.set_fields(k)
        sim.step(10)
        sim.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(sim.stream)
        sim.step(steps)
        b.record(sim.stream)
        b.synchronize()
        out[key] = csu * steps / (a.elapsed_time(b) * 1e-3)
        sim.close()
    out["speedup"] = out["persistent"] / out["per_instance"]
    return out


def plain_fp64(p, steps=200):
    """The unfused FP64 GPU step (equilibrium kernel + convection/combine
    kernel) on the same workload, graph-replayed."""
    import torch
    from paper_2006_15932_amd import dbm as D
    sim = D.Simulation(p.with_(precision="fp64"), precision="fp64")
    sim.set_option(D.DBM_OPT_PATH, 1)
    sim.set_fields()
    sim.step(5)
    sim.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(sim.stream)
    sim.step(steps)
    b.record(sim.stream)
    b.synchronize()
    v = p.S * p.cells * steps / (a.elapsed_time(b) * 1e-3)
    sim.close()
    return v


def _oracle_rate(p, threads, target_s):
    from oracle import oracle as O
    from paper_2006_15932_amd import workloads as W
    O.set_threads(threads)
    o = O.Oracle(p)
    f = o.init_equilibrium(*W.fields(p))
    t0 = time.perf_counter()
    f = o.run(f, 2)
    est = (time.perf_counter() - t0) / 2
    n = max(2, int(target_s / max(est, 1e-6)))
    t0 = time.perf_counter()
    o.run(f, n)
    dt = time.perf_counter() - t0
    return p.S * p.cells * n / dt, n, dt


def _oracle_rate_large(threads, steps=2):
    """The oracle on the full 4096^2 shear layer: a fixed few steps."""
    from oracle import oracle as O
    from paper_2006_15932_amd import workloads as W
    p = W.shear_layer(n=4096, steps=steps, precision="fp64")
    O.set_threads(threads)
    o = O.Oracle(p)
    f = o.init_equilibrium(*W.fields(p))
    t0 = time.perf_counter()
    o.run(f, steps)
    dt = time.perf_counter() - t0
    return p.S * p.cells * steps / dt, dt


def cpu_baseline(p, target_s=10.0, large=True):
    threads = max(1, min(16, os.cpu_count() or 1))
    v, n, dt = _oracle_rate(p, threads, target_s)
    v1, n1, dt1 = _oracle_rate(p, 1, target_s / 3)
    out = {"value": v, "unit": UNIT, "cores": threads, "kind": "oracle",
           "sample": "FP64 oracle, %d Euler steps of the full %dx%d, %d-species workload "
                     "(%.1f s, OpenMP over rows)" % (n, p.nx, p.ny, p.S, dt),
           "single_thread_value": v1,
           "single_thread_sample": "%d steps on 1 thread (%.1f s)" % (n1, dt1)}
    if large:
        vl, dtl = _oracle_rate_large(threads)
        out["large_grid_value"] = vl
        out["large_grid_sample"] = ("FP64 oracle, 2 Euler steps of the 4096x4096 4-species shear "
                                    "layer on %d threads (%.1f s)" % (threads, dtl))
    return out


def traffic_mode(args):
    """Eager launches of the stage kernel plus a copy of known size, for
    rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs."""
    import torch
    p, _ = workload(args.workload, args.precision)
    sim, _, _, rows = gpu_run(p, args.precision, 2, 2, args.tile_rows, args.pipeline,
                              chain_wave=args.chain_wave)
    sim.time_stage_kernel(args.steps)
    sim.close()
    n = 256 << 20
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "traffic", "workload": args.workload, "rows": rows,
                      "copy_bytes_each_way": n, "launches": args.steps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="c1", choices=["c1", "c2", "c4"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--mode", default="bench", choices=["bench", "traffic"])
    ap.add_argument("--tile-rows", type=int, default=0, help="pin rows per tile (0 = autotune)")
    ap.add_argument("--chain-wave", type=int, default=0, choices=[0, 1, 2],
                    help="FP32 chain wavefront (S <= 3): 0 autotune, 1 off, 2 on")
    ap.add_argument("--pipeline", type=int, default=0, choices=[0, 1, 2],
                    help="FP32 row pipeline: 0 autotune, 1 off, 2 on (with --tile-rows)")
    ap.add_argument("--rounding", type=int, default=0, choices=[0, 1],
                    help="FP32 stores: 0 round to nearest, 1 stochastic")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: one GPU only (the library has no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.mode == "traffic":
        return traffic_mode(args)

    p, desc = workload(args.workload, args.precision)
    assert p.scheme == 0, "one launch per step is assumed below"
    sim, ms, kern_ms, rows = gpu_run(p, args.precision, args.steps, args.warmup, args.tile_rows,
                                     args.pipeline, args.rounding, args.chain_wave)
    pipeline = sim.pipeline_in_use
    chain_wave = sim.chain_wave_in_use
    csu_step = p.S * p.cells
    value = csu_step * args.steps / (ms * 1e-3)
    bpl = csu_step * bytes_per_csu(args.precision, p.scheme)
    achieved = bpl / (kern_ms * 1e-3) / 1e9
    tr = MEASURED_TRAFFIC.get(args.workload + "/" + args.precision)
    traffic = None
    if tr and tr.get("source") == kernel_source_hash():
        traffic = tr["bytes_per_launch"]
    sim.close()
    from paper_2006_15932_amd import dbm as D
    # achievable HBM rate: the faster of two sizes of the library's streaming copy
    copy_gbs = max(D.copy_rate_gbs(1 << 30), D.copy_rate_gbs(1 << 32, reps=4))
    line = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": desc, "grid": [p.nx, p.ny], "species": p.S,
                   "precision": "FP32-bulk (FP64 moments/T and conserved-row collision)"
                   if args.precision == "fp32" else "FP64", "scheme": "euler",
                   "tile_rows": rows, "row_pipeline": pipeline == 2,
                   "chain_wavefront": chain_wave == 2,
                   "rounding": "stochastic" if args.rounding else "nearest"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_fused_stage", "bytes_per_launch": bpl,
                     "ms_per_launch": kern_ms,
                     "achievable_copy_gbs": copy_gbs,
                     "frac_of_achievable": achieved / copy_gbs},
    }
    if traffic:
        # measured HBM bytes (rocprofv3 counters, calibrated) over the launch time
        line["roofline"]["traffic_gbs"] = traffic / (kern_ms * 1e-3) / 1e9
        line["roofline"]["traffic_frac"] = line["roofline"]["traffic_gbs"] / HBM_PEAK_GBS
    if not args.no_extra:
        extra = {}
        p64, _ = workload(args.workload, "fp64")
        s64, ms64, k64, _ = gpu_run(p64, "fp64", max(1, args.steps // 5), 20)
        extra["fp64_value"] = csu_step * max(1, args.steps // 5) / (ms64 * 1e-3)
        s64.close()
        px, _ = workload(args.workload, "fp32x")
        sx, msx, _, _ = gpu_run(px, "fp32x", max(1, args.steps // 5), 20)
        extra["fp32x_value"] = csu_step * max(1, args.steps // 5) / (msx * 1e-3)
        sx.close()
        # the same workload with the TVD-RK3 time scheme (three stage launches per step)
        pr3 = p.with_(scheme=1)
        n3 = max(1, args.steps // 5)
        sr3, ms3, k3, _ = gpu_run(pr3, args.precision, n3, 10)
        extra["rk3"] = {"value": csu_step * n3 / (ms3 * 1e-3), "ms_per_step": ms3 / n3,
                        "ms_per_stage_launch": k3,
                        "algorithmic_gbs": csu_step * bytes_per_csu(args.precision, 1)
                        / 3 / (k3 * 1e-3) / 1e9}
        sr3.close()
        extra["plain_fp64_value"] = plain_fp64(p)
        extra["speedup_fp32_fused_vs_plain_fp64"] = value / extra["plain_fp64_value"]
        extra["batched"] = batched()
        extra["linf_vs_oracle"] = {"sample": "64x64 instance of the same setup, 200 steps; "
                                             "u normalised by max(|u|, c_s), u_strict by "
                                             "max(|u|, 0.01 c_s)",
                                   **errors_vs_oracle()}
        pl, dl = workload("c4", "fp32")
        sl, msl, kl, rl = gpu_run(pl, "fp32", 50, 5)
        bl = pl.S * pl.cells * 128
        extra["large_grid"] = {"workload": dl, "value": pl.S * pl.cells * 50 / (msl * 1e-3),
                               "roofline": {"achieved": bl / (kl * 1e-3) / 1e9,
                                            "frac": bl / (kl * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                            "frac_of_achievable": bl / (kl * 1e-3) / 1e9 / copy_gbs,
                                            "ms_per_launch": kl, "tile_rows": rl}}
        sl.close()
        pr, dr = workload("c2", "fp32")
        sr, msr, kr, rr = gpu_run(pr, "fp32", 200, 10)
        br = pr.S * pr.cells * 128
        extra["rt_grid"] = {"workload": dr, "value": pr.S * pr.cells * 200 / (msr * 1e-3),
                            "roofline": {"achieved": br / (kr * 1e-3) / 1e9,
                                         "frac": br / (kr * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                         "frac_of_achievable": br / (kr * 1e-3) / 1e9 / copy_gbs,
                                         "ms_per_launch": kr, "tile_rows": rr}}
        sr.close()
        sr, msr, kr, _ = gpu_run(pr, "fp32", 200, 10, rounding=1)
        extra["rt_grid"]["value_stochastic_rounding"] = pr.S * pr.cells * 200 / (msr * 1e-3)
        sr.close()
        b = extra["batched"]
        b["persistent_hbm_frac"] = b["persistent"] * 128 / 1e9 / HBM_PEAK_GBS
        line["extra"] = extra
    if not args.no_cpu:
        from paper_2006_15932_amd import workloads as W
        line["cpu_baseline"] = cpu_baseline(p.with_(precision="fp64"))
    print(json.dumps(line))


if __name__ == "__main__":
    main()
