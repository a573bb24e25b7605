"""Benchmark of the D2V16 multi-component DBM step on one MI355X.

Workload (default, the largest single-GPU configuration): the four-species
reacting supersonic double shear layer on a 4096x4096 periodic grid (C1's
one-step Arrhenius chemistry plus an inert diluent of molar mass 28 at mass
fraction 0.7; u_x = +-1.5 with tanh profile width 8 cells, +-1% seeded
transverse velocity noise; rho = 1, T = 1; dt = 1e-5, tau = 2e-5), FP32-bulk
(OM storage), forward Euler + NND (the paper's scheme).  A "step" is one full
time step of the update: convection, moments, equilibrium, BGK + reaction +
force, combine -- one launch of the one-pass stage kernel.

Prints ONE JSON line.  `value` is cell-species updates per second over the K
timed steps (inputs resident in HBM; graph-replayed, one step per graph, the
graphs captured during the W warm-up steps; the first ten or so launches of
the stage kernel on C4 run up to 15% slower than the rest, so W defaults to
20; C4 runs at 256 rows per tile, the autotuner's choice, pinned).
`roofline` is for the one-pass stage kernel: algorithmic bytes (32 values of
f read and written per cell-species per Euler step) over its mean launch
duration, which is the HIP-event time of the timed region (events recorded
on the library's stream) divided by the launches in it; `traffic` is the
measured HBM bytes per launch (FETCH_SIZE / WRITE_SIZE) while the kernel
code is the one they were measured on.  `cpu_baseline` times the FP64 CPU oracle on a bounded sample
of the same workload on this host.  `extra` holds the other configurations
(C0-C3), other precisions and schemes, the plain FP64 GPU step, speedups at
equal accuracy and the achievable-copy sweep.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4]
       python bench.py --mode traffic --workload c4   (for rocprofv3 --pmc)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell·species updates/s + % HBM peak, FP32-bulk vs FP64 at stated L∞ error"
UNIT = "cell-species updates/s"

# HBM bytes per launch of the one-pass stage kernel, from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE runs (profiles/fused_om_c4_counters.md), keyed by
# workload, with the hash of the kernel code they were taken at (source
# without comments, see code_text) and the rows per tile.  Changed kernel
# code or other tile rows make the entry stale and `traffic` is reported as
# null.
MEASURED_TRAFFIC = {
    # FETCH_SIZE x 2 (the copy calibration) + WRITE_SIZE, KiB x 1024, medians
    # of the last 20 of the eager launches at the rows per tile given
    # (C4: the pinned rows; C2: the autotuner's)
    "c4/fp32/OM": {"source": "a2d2decc886a98e8", "tile_rows": 512,
        "fetch_kib": 2335371.0, "write_kib": 4194304.125,
        "bytes_per_launch": 1024 * (2 * 2335371.0 + 4194304.125)},
    "c4/fp32/OM+AR": {"source": "a2d2decc886a98e8", "tile_rows": 512,
        "fetch_kib": 2669747.0, "write_kib": 4718592.0625,
        "bytes_per_launch": 1024 * (2 * 2669747.0 + 4718592.0625)},
    "c4/fp32/f": {"source": "a2d2decc886a98e8", "tile_rows": 512,
        "fetch_kib": 2636329.53125, "write_kib": 4194304.0,
        "bytes_per_launch": 1024 * (2 * 2636329.53125 + 4194304.0)},
    "c4/fp64/f": {"source": "a2d2decc886a98e8", "tile_rows": 512,
        "fetch_kib": 4895516.25, "write_kib": 8388612.5,
        "bytes_per_launch": 1024 * (2 * 4895516.25 + 8388612.5)},
    "c2/fp32/OM": {"source": "a2d2decc886a98e8", "tile_rows": 32,
        "fetch_kib": 146490.9375, "write_kib": 262144.125,
        "bytes_per_launch": 1024 * (2 * 146490.9375 + 262144.125)},
    "c2/fp32/OM+AR": {"source": "a2d2decc886a98e8", "tile_rows": 16,
        "fetch_kib": 174840.15625, "write_kib": 294912.0625,
        "bytes_per_launch": 1024 * (2 * 174840.15625 + 294912.0625)},
}


# Rows per tile of the timed run (0 = the library's autotuner).  On C4 the
# autotuner's best are 256 and 512 rows, within 0.3% of each other; 512
# gives each of the 512 resident workgroups one tile and reads 0.7% fewer
# bytes (the 4-row y-halo of each tile).  Pinning it keeps the tuner's trial
# launches of the stage kernel out of the run, so that a kernel trace of the
# run averages the timed configuration only.
DEFAULT_TILE_ROWS = {"c4": 512}


def progress(what: str) -> None:
    """One line on stderr per finished part of the run (the JSON line alone
    goes to stdout)."""
    print("bench: %s done (%.0f s)" % (what, time.time() - T0), file=sys.stderr, flush=True)


T0 = time.time()


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


def stored_traffic(workload: str, precision: str, storage: str, tile_rows: int):
    """HBM bytes per launch measured for this configuration, or None when
    none was taken at the current kernel code and these rows per tile."""
    tr = MEASURED_TRAFFIC.get(workload + "/" + precision + "/" + storage)
    if tr and tr.get("source") == kernel_source_hash() and tr.get("tile_rows") == tile_rows:
        return tr["bytes_per_launch"]
    return None


WORKLOADS = {
    "c0": "C0: 2-species Sod tube, 400x1, outflow x, FP64, Euler+NND, dt=1e-5, tau=2e-5",
    "c1": "C1: 3-species reacting premix, 256x256 periodic, Euler+NND, dt=1e-5, tau=2e-5",
    "c2": "C2: 4-species Rayleigh-Taylor, 1024x1024, walls in y, g=(0,-0.1), Euler+NND",
    "c4": "C4: 4-species reacting supersonic double shear layer, 4096x4096 periodic, Euler+NND",
}


def workload(name: str, precision: str):
    from paper_2006_15932_amd import workloads as W
    if name == "c0":
        return W.sod(steps=1000, precision=precision), WORKLOADS[name]
    if name == "c1":
        return W.reacting(n=256, steps=5000, precision=precision), WORKLOADS[name]
    if name == "c2":
        return W.rayleigh_taylor(n=1024, steps=20000, precision=precision), WORKLOADS[name]
    if name == "c4":
        return W.shear_layer(n=4096, steps=5000, precision=precision), WORKLOADS[name]
    raise SystemExit("unknown workload " + name)


def bytes_per_csu(precision: str, scheme: int, storage: str = "") -> int:
    """Algorithmic bytes per cell-species update of one step: the 16 stored
    values read and written once (Euler), 128 values moved over the three
    stages of TVD-RK3; OM storage with A-block residuals also reads and
    writes four 2-byte residuals per step (Euler)."""
    es = {"fp32": 4, "fp64": 8, "fp32x": 6}[precision]
    if storage == "OM+AR":
        assert scheme == 0, "A-block residual bytes are counted for Euler steps"
        return es * 32 + 16
    return es * (32 if scheme == 0 else 128)


STORAGE_NAMES = {0: "OM", 1: "f", 2: "OM+AR"}


def gpu_run(p, precision, steps, warmup, tile_rows=0, rounding=0, chain_wave=0, storage=None,
            chunk=1, path=0):
    """Time `steps` steps after `warmup` untimed ones.  With chunk = 1 every
    step is one replay of one of two cached one-step graphs (both parities are
    captured during a warm-up of two or more steps), so the timed region
    replays exactly the graphs the warm-up built."""
    import torch
    from paper_2006_15932_amd import dbm as D
    sim = D.Simulation(p, precision=precision)
    if path:
        sim.set_option(D.DBM_OPT_PATH, 1)
    else:
        assert sim.get_option(D.DBM_OPT_PATH) == 0, "one-pass HIP path not active"
    if storage is not None:
        sim.set_option(D.DBM_OPT_STORAGE, storage)
    if rounding:
        sim.set_option(D.DBM_OPT_ROUNDING, rounding)
    if tile_rows:
        sim.set_option(D.DBM_OPT_TILE_ROWS, tile_rows)
    if chain_wave:
        sim.set_option(D.DBM_OPT_CHAIN_WAVE, chain_wave)
    sim.set_option(D.DBM_OPT_GRAPH_CHUNK, chunk)
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
    info = {"tile_rows": sim.get_option(D.DBM_OPT_TILE_ROWS),
            "chain_wavefront": sim.get_option(D.DBM_OPT_CHAIN_WAVE) == 2,
            "storage": STORAGE_NAMES[sim.get_option(D.DBM_OPT_STORAGE)],
            "drain": sim.get_option(D.DBM_OPT_DRAIN) == 2,
            "path": "one-pass" if sim.get_option(D.DBM_OPT_PATH) == 0 else "plain"}
    return sim, ms, ms / launches, info


def rate(p, steps, ms):
    return p.S * p.cells * steps / (ms * 1e-3)


def errors_vs_oracle(n=64, steps=200):
    """FP32-bulk (OM storage; f storage; stochastic rounding), FP32X and FP64
    runs of the reacting premix on an n x n instance against the FP64 CPU
    oracle (relative L-infinity per field, u gated by max(max|u|, 0.01 c_s))."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_helpers import field_errors, oracle_run
    from paper_2006_15932_amd import dbm as D
    from paper_2006_15932_amd import workloads as W
    p = W.reacting(n=n, steps=steps)
    o, fo = oracle_run(p, steps)
    mo = o.moments(fo)
    out = {}
    for key, prec, opts in (("fp32_om", "fp32", {}),
                            ("fp32_om_residuals", "fp32", {D.DBM_OPT_STORAGE: 2}),
                            ("fp32_f_storage", "fp32", {D.DBM_OPT_STORAGE: 1}),
                            ("fp32_om_stochastic_rounding", "fp32", {D.DBM_OPT_ROUNDING: 1}),
                            ("fp32x", "fp32x", {}), ("fp64", "fp64", {})):
        sim = D.Simulation(p, precision=prec)
        for k, v in opts.items():
            sim.set_option(k, v)
        sim.set_fields()
        sim.step(steps)
        e = field_errors(p, sim.moments(), mo)
        out[key] = {k: float("%.3e" % e[k]) for k in ("rho", "u", "u_cs", "T")}
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
        sim.set_option(D.DBM_OPT_GRAPH_CHUNK, steps)
        for k in range(len(probs)):
            sim.set_fields(k)
        sim.step(steps)                 # captures the timed graphs
        sim.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(sim.stream)
        sim.step(steps)
        b.record(sim.stream)
        b.synchronize()
        out[key] = csu * steps / (a.elapsed_time(b) * 1e-3)
        sim.close()
    out["speedup"] = out["persistent"] / out["per_instance"]
    out["persistent_hbm_frac"] = out["persistent"] * 128 / 1e9 / HBM_PEAK_GBS
    return out


def small_config(name, precision, steps, **kw):
    """A whole-grid rate on a smaller configuration: graphs of `steps` steps,
    the same graph replayed in the warm-up and in the timed region."""
    p, desc = workload(name, precision)
    kw.setdefault("chunk", steps)
    sim, ms, kern, info = gpu_run(p, precision, steps, steps, **kw)
    sim.close()
    bpl = p.S * p.cells * bytes_per_csu(precision, p.scheme, info["storage"]) / (
        1 if p.scheme == 0 else 3)
    return {"workload": desc, "precision": precision, "value": rate(p, steps, ms),
            "ms_per_step": ms / steps, "ms_per_launch": kern,
            "algorithmic_gbs": bpl / (kern * 1e-3) / 1e9,
            "frac": bpl / (kern * 1e-3) / 1e9 / HBM_PEAK_GBS, **info}


def copy_sweep():
    """Achievable copy rate: the library's streaming copy over grid sizes and
    16-byte words in flight per thread, and torch's device-to-device copy,
    on 4 GiB buffers."""
    import torch
    from paper_2006_15932_amd import dbm as D
    n = 4 << 30
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    res = []
    for grid in (1024, 2048, 4096, 8192, 16384):
        for words in (1, 2, 4, 8):
            ms = D.dbm_copy_rate(a.data_ptr(), b.data_ptr(), n, grid, 3, st.cuda_stream, words)
            res.append({"grid": grid, "words": words, "gbs": 2.0 * n / (ms * 1e-3) / 1e9})
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    torch_gbs = 3 * 2.0 * n / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    best = max(res, key=lambda r: r["gbs"])
    return {"bytes_each_way": n, "best": best, "torch_copy_gbs": torch_gbs, "sweep": res}


def host_info():
    info = {"nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"), "machine": platform.machine()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
            if line.startswith("Socket(s):"):
                info["sockets"] = line.split(":", 1)[1].strip()
            if line.startswith("Core(s) per socket:"):
                info["cores_per_socket"] = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(p, target_s=15.0):
    """The FP64 oracle, as it stands, on the same workload: whole-grid Euler
    steps on every CPU this process may run on (OpenMP over rows), for about
    target_s seconds."""
    from oracle import oracle as O
    from paper_2006_15932_amd import workloads as W
    host = host_info()
    threads = host["affinity_cpus"]
    O.set_threads(threads)
    o = O.Oracle(p)
    f = o.init_equilibrium(*W.fields(p))
    t0 = time.perf_counter()
    f = o.run(f, 1)
    est = time.perf_counter() - t0
    n = max(1, min(50, int(target_s / max(est, 1e-6))))
    t0 = time.perf_counter()
    o.run(f, n)
    dt = time.perf_counter() - t0
    return {"value": p.S * p.cells * n / dt, "unit": UNIT, "cores": O.get_threads(),
            "kind": "oracle",
            "sample": "FP64 oracle, %d Euler step(s) of the full %dx%d %d-species grid of the "
                      "benchmarked workload (%.1f s, OpenMP over rows on %d threads)"
                      % (n, p.nx, p.ny, p.S, dt, O.get_threads()),
            "host": host}


def traffic_mode(args):
    """Eager launches of the stage kernel plus a copy of known size, for
    rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs."""
    import torch
    p, _ = workload(args.workload, args.precision)
    sim, _, _, info = gpu_run(p, args.precision, 2, 2, args.tile_rows, args.rounding,
                              args.chain_wave, None if args.storage < 0 else args.storage)
    sim.time_stage_kernel(args.steps)
    sim.close()
    n = 256 << 20
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "traffic", "workload": args.workload, "info": info,
                      "copy_bytes_each_way": n, "launches": args.steps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c4"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "fp32x"])
    ap.add_argument("--mode", default="bench", choices=["bench", "traffic"])
    ap.add_argument("--tile-rows", type=int, default=-1,
                    help="rows per tile: 0 autotune, -1 the workload's default (C4: 256, the "
                         "autotuner's choice there, pinned so that every launch of the stage "
                         "kernel in the run is a launch of the timed configuration)")
    ap.add_argument("--chain-wave", type=int, default=0, choices=[0, 1, 2],
                    help="chain wavefront (S <= 3): 0 autotune, 1 off, 2 on")
    ap.add_argument("--rounding", type=int, default=0, choices=[0, 1],
                    help="FP32 stores: 0 round to nearest, 1 stochastic")
    ap.add_argument("--storage", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="FP32-bulk storage: -1 library default, 0 OM, 1 f itself, 2 OM with "
                         "A-block residuals")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: one GPU only (the library has no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.tile_rows < 0:
        args.tile_rows = DEFAULT_TILE_ROWS.get(args.workload, 0)
    if args.mode == "traffic":
        return traffic_mode(args)

    p, desc = workload(args.workload, args.precision)
    assert p.scheme == 0, "one launch per step is assumed below"
    sim, ms, kern_ms, info = gpu_run(p, args.precision, args.steps, args.warmup, args.tile_rows,
                                     args.rounding, args.chain_wave,
                                     None if args.storage < 0 else args.storage)
    sim.close()
    progress("timed run")
    value = rate(p, args.steps, ms)
    bpl = p.S * p.cells * bytes_per_csu(args.precision, p.scheme, info["storage"])
    achieved = bpl / (kern_ms * 1e-3) / 1e9
    traffic = stored_traffic(args.workload, args.precision, info["storage"], info["tile_rows"])
    line = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "fp32x": "f32x (f32 + bf16 residual)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": desc, "grid": [p.nx, p.ny], "species": p.S,
                   "precision": {"fp32": "FP32-bulk (FP64 moments/T and conserved-row collision)",
                                 "fp64": "FP64", "fp32x": "FP32X"}[args.precision],
                   "scheme": "euler", "rounding": "stochastic" if args.rounding else "nearest",
                   **info},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_fused_om" if info["storage"] == "OM" else "k_fused_stage",
                     "bytes_per_launch": bpl, "ms_per_launch": kern_ms},
    }
    if traffic:
        line["roofline"]["traffic_per_algorithmic"] = traffic / bpl
    if not args.no_extra:
        extra = {}
        cs = copy_sweep()
        line["roofline"]["achievable_copy_gbs"] = cs["best"]["gbs"]
        line["roofline"]["frac_of_achievable"] = achieved / cs["best"]["gbs"]
        extra["copy"] = cs
        progress("copy sweep")
        # the same grid in other precisions and storages, and with TVD-RK3
        for key, prec, kw in (("fp32_f_storage", "fp32", {"storage": 1}),
                              ("fp32_om_residuals", "fp32", {"storage": 2}),
                              ("fp32_om_stochastic_rounding", "fp32", {"rounding": 1}),
                              ("fp64", "fp64", {}), ("fp32x", "fp32x", {})):
            q, _ = workload(args.workload, prec)
            s2, ms2, k2, i2 = gpu_run(q, prec, 10, 2, **kw)
            s2.close()
            extra[key] = {"value": rate(q, 10, ms2), "ms_per_launch": k2,
                          "frac": q.S * q.cells * bytes_per_csu(prec, 0, i2["storage"])
                          / (k2 * 1e-3) / 1e9 / HBM_PEAK_GBS, **i2}
            progress(key)
        q = p.with_(scheme=1)
        s3, ms3, k3, i3 = gpu_run(q, args.precision, 10, 2)
        s3.close()
        extra["rk3"] = {"value": rate(q, 10, ms3), "ms_per_step": ms3 / 10,
                        "ms_per_stage_launch": k3,
                        "frac": q.S * q.cells * bytes_per_csu(args.precision, 1) / 3
                        / (k3 * 1e-3) / 1e9 / HBM_PEAK_GBS}
        q, _ = workload(args.workload, "fp64")
        sp_, msp, kp, ip = gpu_run(q, "fp64", 5, 2, path=1)
        sp_.close()
        extra["plain_fp64"] = {"value": rate(q, 5, msp), "ms_per_step": msp / 5, **ip}
        progress("rk3, plain fp64")
        extra["speedup_at_equal_accuracy"] = {
            "fp64_one_pass_vs_plain_fp64": extra["fp64"]["value"] / extra["plain_fp64"]["value"],
        }
        # smaller configurations (whole-grid rates, long graphs)
        extra["c1"] = small_config("c1", "fp32", 2000)
        extra["c1_fp64"] = small_config("c1", "fp64", 1000)
        extra["c1_plain_fp64"] = small_config("c1", "fp64", 500, path=1)
        progress("c1")
        extra["speedup_at_equal_accuracy"]["c1_fp32_om_vs_plain_fp64"] = (
            extra["c1"]["value"] / extra["c1_plain_fp64"]["value"])
        extra["speedup_at_equal_accuracy"]["c1_fp64_one_pass_vs_plain_fp64"] = (
            extra["c1_fp64"]["value"] / extra["c1_plain_fp64"]["value"])
        extra["c2"] = small_config("c2", "fp32", 500)
        extra["c2_om_residuals"] = small_config("c2", "fp32", 500, storage=2)
        extra["c2_stochastic_rounding"] = small_config("c2", "fp32", 500, rounding=1)
        extra["c2_plain_fp64"] = small_config("c2", "fp64", 50, path=1)
        extra["speedup_at_equal_accuracy"]["c2_fp32_om_residuals_vs_plain_fp64"] = (
            extra["c2_om_residuals"]["value"] / extra["c2_plain_fp64"]["value"])
        extra["speedup_at_equal_accuracy"]["note"] = (
            "pairs only precisions that both meet their bar at the stated step count: FP64 "
            "(one-pass and plain) always; FP32-bulk OM on C1 (256^2, 5000 steps within 1e-5); "
            "FP32-bulk OM with A-block residuals on C2 (its 128^2 crop, 20000 steps within "
            "1e-5; tests/test_gpu_stated_steps.py); the shear layer has no full-size oracle "
            "at 5000 steps, so FP32-bulk is not paired there")
        extra["c0_fp64"] = small_config("c0", "fp64", 1000)
        extra["c3"] = batched()
        progress("c2, c0, c3")
        extra["linf_vs_oracle"] = {"sample": "64x64 reacting premix, 200 steps; u gated by "
                                             "max(max|u|, 0.01 c_s), u_cs by max(max|u|, c_s)",
                                   **errors_vs_oracle()}
        progress("errors vs oracle")
        line["extra"] = extra
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(p.with_(precision="fp64"))
        progress("cpu baseline")
    print(json.dumps(line))


if __name__ == "__main__":
    main()
