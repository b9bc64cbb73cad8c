"""Throughput benchmark of the bulk-microphysics column step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c1] [--mode fp64]

One step = one casim_step over the whole synthetic domain (saturation
adjustment, the 12 process rates with limiter, sedimentation, tendency and
surface writes) with the state already resident in HBM.  The default workload
is the LES-like domain: 256 x 256 columns x 100 levels, 50 % clustered cloud,
dt = 2 s, seed 1, all arithmetic in binary64.

Prints one JSON line: grid-point updates/s, the roofline position of the
sweep kernel (algorithmic HBM bytes per launch / mean kernel time from HIP
events on the launch stream) and the CPU oracle's throughput on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
KERNEL_SOURCES = ["casim_sweep.hip", "casim_internal.h", "casim_math.h", "casim_math_tables.h", "casim_defaults.h"]
B_CLOUDY, B_CLEAR, B_COLUMN = 208, 160, 64   # algorithmic bytes per point / column
B_CLOUDY_WARM, B_CLEAR_WARM = 160, 136       # warm configuration: no ice-phase inputs


def algorithmic_bytes(cfg, mask, warm=False) -> int:
    """Bytes a step must move: 14 reads + 12 writes (FP64) per point of a
    cloudy column, 8 reads + 12 writes per point of a clear column, 8 surface
    writes per column.  The warm configuration reads 8 and 5 fields (no ice,
    snow or graupel) and still writes all 12 tendencies."""
    ncloudy = int(mask.sum())
    nclear = cfg.ncol - ncloudy
    bc, bl = (B_CLOUDY_WARM, B_CLEAR_WARM) if warm else (B_CLOUDY, B_CLEAR)
    return cfg.nlev * (ncloudy * bc + nclear * bl) + cfg.ncol * B_COLUMN


def sweep_source_digest() -> str:
    """SHA-256 over the sources the sweep kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2010_14823_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(cfg_name, mode):
    """HBM bytes per sweep launch measured by the FETCH_SIZE / WRITE_SIZE
    counters (already scaled by the copy-kernel calibration), read from the
    profile summary of this workload; None when there is none or when it was
    taken on kernel sources other than the current ones."""
    path = os.path.join(ROOT, "profiles", "sweep_kernel_%s_%s_hbm_counters.md" % (cfg_name, mode))
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"^\s*-?\s*`?(source_sha256|hbm_bytes_per_launch)`?\s*[:=]\s*`?([0-9a-fA-F.eE+]+)`?", line)
            if m:
                rec[m.group(1)] = m.group(2)
    if rec.get("source_sha256") != sweep_source_digest() or "hbm_bytes_per_launch" not in rec:
        return None
    return float(rec["hbm_bytes_per_launch"])


def cpu_baseline(st, dz, dt, budget_s=10.0):
    import oracle
    nthreads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    nthreads = min(nthreads, 16)
    oracle.build(force=False)
    oracle.step(st[:, :, :64], dz, dt, nthreads=nthreads)      # warm the library
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        oracle.step(st, dz, dt, nthreads=nthreads)
        times.append(time.perf_counter() - t0)
        # about 10 s of CPU work, at least 3 steps
        if (time.perf_counter() - t_start > budget_s and len(times) >= 3) or len(times) >= 500:
            break
    t = float(np.median(times))
    pts = st.shape[1] * st.shape[2]
    # one thread on the first 1/16 of the columns (about 2-3 s)
    sub = np.ascontiguousarray(st[:, :, :max(64, st.shape[2] // 16)])
    t1 = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.step(sub, dz, dt, nthreads=1)
        t1.append(time.perf_counter() - t0)
    t1m = float(np.median(t1))
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": pts / t, "unit": "grid-point updates/s", "cores": nthreads, "kind": "oracle",
            "sample": "%d columns x %d levels of the same workload, median of %d full steps "
                      "(%.3f s each, %.1f s in all)" % (st.shape[2], st.shape[1], len(times), t, sum(times)),
            "single_core": {"value": sub.shape[1] * sub.shape[2] / t1m, "cores": 1,
                            "sample": "first %d columns, median of 3 steps (%.2f s each)" % (sub.shape[2], t1m)},
            "host": {"cpu": model, "nproc": os.cpu_count()}}


def compare_with_plain(torch, casim, dev, dz, cfg, tend, sfc, mode, warm=0):
    """Per-field error of one step of `mode` against one plain binary64 step on
    the same state, both on the GPU: normwise max|d|/max|plain| and RMS."""
    casim.step(dev, dz, cfg.dt, tend, sfc)
    t_mode, s_mode = tend.clone(), sfc.clone()
    casim.init(casim.default_constants(mode=casim.MODE_FP64, warm=warm))
    casim.step(dev, dz, cfg.dt, tend, sfc)
    torch.cuda.synchronize()
    out = {}
    names = casim.TEND_NAMES + casim.SFC_NAMES
    pairs = [(t_mode[j], tend[j]) for j in range(12)] + [(s_mode[j], sfc[j]) for j in range(8)]
    for name, (a, b) in zip(names, pairs):
        d = (a - b).abs()
        den = b.abs().max().item()
        out[name] = {"max_rel": (d.max().item() / den) if den > 0 else (0.0 if d.max().item() == 0 else None),
                     "rms_rel": ((d.pow(2).mean().sqrt().item() / b.pow(2).mean().sqrt().item())
                                 if den > 0 else None)}
    casim.init(casim.default_constants(mode=mode, warm=warm))
    return out


def copy_probe(torch, nbytes=2 << 30, reps=5):
    """Achieved bandwidth of a plain 2 GiB device-to-device copy (read + write)."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    return {"bytes_read": nbytes, "bytes_written": nbytes, "ms": ms, "GBps": 2 * nbytes / (ms * 1e-3) / 1e9}


def host_pipeline(torch, casim, st, dz, dt, nblocks=0, reps=3):
    """casim_step_host on page-locked host copies of the workload: time per
    step including both PCIe directions, and the same step overlapped with a
    host workload (the parent model's other components) of similar length."""
    nf, nlev, ncol = st.shape
    hin, hout, hsfc = casim.HostArray(st.shape), casim.HostArray((12, nlev, ncol)), casim.HostArray((8, ncol))
    hin.array[:] = st
    casim.step_host(hin.array, dz, dt, hout.array, hsfc.array, nblocks=nblocks)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        casim.step_host(hin.array, dz, dt, hout.array, hsfc.array, nblocks=nblocks)
        torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / reps
    # a host workload of about the same length: dense products on the CPU
    a = np.random.default_rng(0).standard_normal((600, 600))
    n_mm = 1
    while True:
        t0 = time.perf_counter()
        for _ in range(n_mm):
            a = np.tanh(a @ a * 1e-3)
        t_host = time.perf_counter() - t0
        if t_host >= t_step or n_mm > 4096:
            break
        n_mm *= 2
    t0 = time.perf_counter()
    casim.step_host(hin.array, dz, dt, hout.array, hsfc.array, nblocks=nblocks)
    for _ in range(n_mm):
        a = np.tanh(a @ a * 1e-3)
    torch.cuda.synchronize()
    t_both = time.perf_counter() - t0
    h2d = st.nbytes
    d2h = 12 * nlev * ncol * 8 + 8 * ncol * 8
    for h in (hin, hout, hsfc):
        h.free()
    return {"ms_per_step": t_step * 1e3, "points_per_s": nlev * ncol / t_step, "nblocks": nblocks or 4,
            "bytes_h2d": h2d, "bytes_d2h": d2h, "pcie_GBps_both_directions": (h2d + d2h) / t_step / 1e9,
            "overlap": {"host_work_ms": t_host * 1e3, "step_ms": t_step * 1e3,
                        "concurrent_ms": t_both * 1e3, "serial_ms": (t_host + t_step) * 1e3}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--config", default="c1")
    ap.add_argument("--mode", default="fp64", choices=["fp64", "fp32mix", "surrogate", "fp64compact"])
    ap.add_argument("--checkpoint", default=None, help="surrogate checkpoint (casim_mlp_save blob)")
    ap.add_argument("--compare", action="store_true",
                    help="also run one plain binary64 step and report the per-field error of this mode")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--warm", action="store_true",
                    help="warm configuration (ice, snow and graupel processes off and not read)")
    ap.add_argument("--host-pipeline", action="store_true",
                    help="also time casim_step_host (state in page-locked host memory, both PCIe "
                         "directions included) alone and overlapped with a host workload")
    ap.add_argument("--no-copy", action="store_true",
                    help="skip the plain device-to-device copy of 2 GiB that is timed after the step "
                         "(the achievable-bandwidth reference and the scale for the HBM byte counters)")
    ap.add_argument("--with-copy", action="store_true", help="(the default; kept for older command lines)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the column step needs no exchange between GPUs "
              "and this benchmark runs on a single MI355X; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2010_14823_amd import casim, synth

    cfg = synth.CONFIGS[args.config]
    print("bench: generating %s (%d columns x %d levels)" % (cfg.name, cfg.ncol, cfg.nlev),
          file=sys.stderr, flush=True)
    fields, dz, cols = synth.generate(cfg)
    st = synth.stack(fields)
    mask = synth.cloud_mask(cfg)
    del fields
    dev = torch.from_numpy(st).cuda()
    tend = torch.empty((12, cfg.nlev, cfg.ncol), dtype=torch.float64, device="cuda")
    sfc = torch.empty((8, cfg.ncol), dtype=torch.float64, device="cuda")
    mode = {"fp64": casim.MODE_FP64, "fp32mix": casim.MODE_FP32MIX, "surrogate": casim.MODE_SURROGATE,
            "fp64compact": casim.MODE_FP64_COMPACT}[args.mode]
    if args.mode == "surrogate":
        if not args.checkpoint:
            print("--mode surrogate needs --checkpoint", file=sys.stderr)
            sys.exit(2)
        casim.init()
        casim.mlp_load(open(args.checkpoint, "rb").read())
        casim.surrogate_load()
    casim.init(casim.default_constants(mode=mode, warm=1 if args.warm else 0))
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        casim.step(dev, dz, cfg.dt, tend, sfc)
    torch.cuda.synchronize()
    status = casim.status()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        casim.step(dev, dz, cfg.dt, tend, sfc)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    status = casim.status()

    points = cfg.ncol * cfg.nlev
    ms_per_step = wall * 1e3 / args.steps
    alg = algorithmic_bytes(cfg, mask, args.warm)
    achieved = alg / (kern_ms * 1e-3) / 1e9
    traffic = recorded_traffic(cfg.name, args.mode) if args.mode in ("fp64", "fp32mix") and not args.warm else None
    line = {
        "metric": "grid-point updates/s: FP64 plain vs FP32-mixed vs MLP surrogate @ stated error",
        "value": points / (wall / args.steps),
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.mode in ("fp64", "fp64compact") else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "%s %s%s step: %d columns x %d levels, %s cloudy columns, dt=%g s, seed %d"
                               % (cfg.name, args.mode, " warm" if args.warm else "", cfg.ncol, cfg.nlev,
                                  "all" if cfg.cloud_frac is None else "%d%%" % round(100 * cfg.cloud_frac),
                                  cfg.dt, cfg.seed),
                   "columns": cfg.ncol, "levels": cfg.nlev, "points": points, "mode": args.mode,
                   "configuration": "warm" if args.warm else "cold"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": ("sweep_kernel (HIP events around the step: the ~7 us tile-order kernel "
                                "that precedes it is included)") if args.mode in ("fp64", "fp32mix")
                               else "whole step: point pass, rate kernel, sweep",
                     "kernel_ms": kern_ms, "algorithmic_bytes": alg},
        "status": status,
    }
    print("bench: %.4f ms/step on the GPU" % ms_per_step, file=sys.stderr, flush=True)
    if args.mode == "surrogate":
        line["surrogate"] = {"fallback_points_per_step": status["fallback"] / args.steps,
                             "inferred_points_per_step": status["inferred"] / args.steps}
    if args.compare and args.mode != "fp64":
        line["error_vs_fp64_plain"] = compare_with_plain(torch, casim, dev, dz, cfg, tend, sfc, mode,
                                                           1 if args.warm else 0)
    if not args.no_copy:
        line["copy_probe"] = copy_probe(torch)
        line["roofline"]["frac_of_copy"] = achieved / line["copy_probe"]["GBps"]
    if args.host_pipeline:
        line["host_pipeline"] = host_pipeline(torch, casim, st, dz, cfg.dt)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(st, dz, cfg.dt)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
