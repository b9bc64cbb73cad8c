"""Throughput benchmark of the bulk-microphysics column step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one casim_step over the whole synthetic domain (clean-up and
phase changes, saturation adjustment, the 12 process rates with limiter,
sedimentation, tendency and surface writes) with the state already resident
in HBM.  The default run measures the three paths of the metric on the
1024 x 1024 columns x 120 levels domains, each for exactly K timed steps
after W untimed ones:

* binary64 plain on 50 % clustered cloud, seed 3 -- the JSON line's ``value``
  (grid-point updates/s from the wall clock around the K steps);
* FP32-mixed on the same state, with its per-field error against the
  binary64 step (one step, and the state and tendencies after 10 coupled
  steps in which each path evolves its own state);
* the learned surrogate: trained in this run on plain-path samples of ten
  256 x 256 x 100 domains (seeds 10-19, 400,000 samples each, a stated epoch
  budget), then stepped on the 50 %-cloud inference domain (seed 4) with its
  per-field error against the binary64 step on that domain;

plus the binary64 step on the sparse deep-convection domain (10 % cloud,
seed 2), the HBM roofline position of the sweep kernel, a plain device copy
for the achievable bandwidth, and the CPU oracle on a bounded sample of the
headline workload.  Prints one JSON line.

``--config`` / ``--mode`` time one configuration and mode only (the
smaller domains are test cases; this is for profiling).
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

METRIC = "grid-point updates/s: FP64 plain vs FP32-mixed vs MLP surrogate @ stated error"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
BF16_PEAK_TFLOPS = 2500.0      # MI355X dense bf16 matrix peak
NET_FLOP_PER_POINT = 2 * (12 * 128 + 128 * 128 + 128 * 128 + 128 * 12)   # 71,680: 35,840 multiply-adds
KERNEL_SOURCES = ["casim_sweep.hip", "casim_internal.h", "casim_math.h", "casim_math_tables.h", "casim_defaults.h"]
B_CLOUDY, B_CLEAR, B_COLUMN = 208, 160, 64   # algorithmic bytes per point / column
B_CLOUDY_WARM, B_CLEAR_WARM = 160, 136       # warm configuration: no ice-phase inputs
MODES = {"fp64": 0, "fp32mix": 1, "surrogate": 2, "fp64compact": 3}
STATE_NAMES = ("T", "qv", "qc", "nc", "qr", "nr", "qi", "ni", "qs", "ns", "qg", "ng")


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


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


def host_threads():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(n, 16))


def cpu_baseline(cfg, rows, budget_s=12.0):
    """The oracle as it stands, on the host cores: one full step over the
    listed grid rows of the workload (a bounded sample; columns are
    independent), median over repeated steps within about budget_s."""
    import oracle
    from paper_2010_14823_amd import synth
    nthreads = host_threads()
    f, dz, _ = synth.generate(cfg, rows)
    st = synth.stack(f)
    del f
    oracle.build(force=False)
    oracle.step(np.ascontiguousarray(st[:, :, :64]), dz, cfg.dt, nthreads=nthreads)      # warm the library
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        oracle.step(st, dz, cfg.dt, nthreads=nthreads)
        times.append(time.perf_counter() - t0)
        if (time.perf_counter() - t_start > budget_s and len(times) >= 3) or len(times) >= 500:
            break
    t = float(np.median(times))
    pts = st.shape[1] * st.shape[2]
    sub = np.ascontiguousarray(st[:, :, :4096])
    t1 = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.step(sub, dz, cfg.dt, nthreads=1)
        t1.append(time.perf_counter() - t0)
    t1m = float(np.median(t1))
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": pts / t, "unit": "grid-point updates/s", "cores": nthreads, "kind": "oracle",
            "sample": "grid rows %d-%d of the %s workload (%d columns x %d levels), median of %d full oracle "
                      "steps (%.3f s each, %.1f s in all)" % (rows[0], rows[-1], cfg.name, st.shape[2], st.shape[1],
                                                             len(times), t, sum(times)),
            "single_core": {"value": sub.shape[1] * sub.shape[2] / t1m, "cores": 1,
                            "sample": "first 4096 of those columns, median of 3 steps (%.2f s each)" % t1m},
            "host": {"cpu": model, "nproc": os.cpu_count()}}


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


def stream_ceiling(torch, casim, nbytes=2 << 30, reps=5):
    """The library's hand-written streaming kernels (non-temporal accesses of
    8 or 16 bytes per lane, grids of 1024 to 16384 blocks of 256 threads) on
    2 GiB: copy (bytes read + written), read-only, write-only; each the best
    of the sweep, with the width and grid that reached it."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    out = {"bytes": nbytes, "sweep": []}
    for kind, name, moved in ((0, "copy", 2 * nbytes), (1, "read", nbytes), (2, "write", nbytes)):
        best = None
        for width in (8, 16):
            for blocks in (1024, 4096, 16384):
                casim.debug_bandwidth(src, dst, nbytes, kind, width, blocks, stream)
                s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                s.record(stream)
                for _ in range(reps):
                    casim.debug_bandwidth(src, dst, nbytes, kind, width, blocks, stream)
                e.record(stream)
                torch.cuda.synchronize()
                gbps = moved / (s.elapsed_time(e) / reps * 1e-3) / 1e9
                out["sweep"].append({"kind": name, "width": width, "blocks": blocks, "GBps": gbps})
                if best is None or gbps > best[0]:
                    best = (gbps, width, blocks)
        out[name + "_GBps"] = best[0]
        out[name + "_at"] = {"width": best[1], "blocks": best[2]}
    del src, dst
    return out


def time_steps(torch, casim, dev, dz, dt, tend, sfc, steps, warmup, fn=None):
    """W untimed steps, then exactly K steps between two synchronisations:
    wall-clock ms per step, and per-step HIP-event times on the launch
    stream (median, min, max, mean).  fn replaces casim.step (same
    arguments), e.g. by the streaming-floor diagnostic."""
    step = fn or casim.step
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        step(dev, dz, dt, tend, sfc)
    torch.cuda.synchronize()
    casim.status()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        step(dev, dz, dt, tend, sfc)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    status = casim.status()
    return {"ms_per_step": wall * 1e3 / steps, "event_ms": {"median": float(np.median(ms)), "min": float(ms.min()),
                                                            "max": float(ms.max()), "mean": float(ms.mean())},
            "status": status}


def field_errors(test_t, test_s, ref_t, ref_s):
    """Per field: normwise max |test - ref| / max |ref| and RMS |test - ref| /
    RMS ref, over the whole domain (torch tensors on the GPU)."""
    from paper_2010_14823_amd import casim
    out = {}
    pairs = [(casim.TEND_NAMES[j], test_t[j], ref_t[j]) for j in range(12)] + \
            [(casim.SFC_NAMES[j], test_s[j], ref_s[j]) for j in range(8)]
    for name, a, b in pairs:
        d = (a - b).abs()
        den = b.abs().max().item()
        rms = b.pow(2).mean().sqrt().item()
        out[name] = {"max": d.max().item() / den if den > 0 else (0.0 if d.max().item() == 0 else None),
                     "rms": d.pow(2).mean().sqrt().item() / rms if rms > 0 else None}
    return out


def state_errors(test, ref):
    out = {}
    for j, f in enumerate([0] + list(range(3, 14))):
        a, b = test[f], ref[f]
        d = (a - b).abs()
        den = b.abs().max().item()
        rms = b.pow(2).mean().sqrt().item()
        out[STATE_NAMES[j]] = {"max": d.max().item() / den if den > 0 else 0.0,
                               "rms": d.pow(2).mean().sqrt().item() / rms if rms > 0 else 0.0}
    return out


def worst(errs):
    vals = [v["max"] for v in errs.values() if v["max"] is not None]
    rms = [v["rms"] for v in errs.values() if v["rms"] is not None]
    return {"max": max(vals) if vals else 0.0, "rms": max(rms) if rms else 0.0}


def device_fields(torch, casim, host):
    """Host fields (nf, nlev, ncol) float64 on the device in the layout the
    library recommends: rows padded to casim_padded_ld (8 MiB + 2 KiB per
    level row of a 1024 x 1024 domain instead of 8 MiB)."""
    nf, nlev, ncol = host.shape
    dev = casim.empty_fields(nf, nlev, ncol)
    dev.copy_(torch.from_numpy(host))
    return dev


def outputs(torch, casim, cfg):
    """Tendencies (padded like the state) and surface sums for cfg."""
    return (casim.empty_fields(12, cfg.nlev, cfg.ncol),
            torch.empty((8, cfg.ncol), dtype=torch.float64, device="cuda"))


def upload(torch, casim, synth, cfg, workers):
    t0 = time.perf_counter()
    st, dz = synth.generate_stacked(cfg, workers=workers)
    dev = device_fields(torch, casim, st)
    del st
    log("%s generated and uploaded in %.1f s" % (cfg.name, time.perf_counter() - t0))
    return dev, dz


def workload_name(cfg):
    return "%dx%d columns x %d levels, %s cloudy columns%s, dt=%g s, seed %d" % (
        cfg.nx, cfg.ny, cfg.nlev, "all" if cfg.cloud_frac is None else "%d%%" % round(100 * cfg.cloud_frac),
        ", deep convection to 14 km" if cfg.deep else "", cfg.dt, cfg.seed)


def mode_record(cfg, mask, t, warm=False):
    pts = cfg.ncol * cfg.nlev
    alg = algorithmic_bytes(cfg, mask, warm)
    return {"workload": workload_name(cfg), "ms_per_step": t["ms_per_step"], "points_per_s": pts / (t["ms_per_step"] * 1e-3),
            "event_ms": t["event_ms"], "hbm_GBps_algorithmic": alg / (t["event_ms"]["mean"] * 1e-3) / 1e9,
            "frac_of_hbm_peak": alg / (t["event_ms"]["mean"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes": alg, "status": t["status"]}


def train_surrogate(torch, casim, budget_epochs, per_seed):
    """Samples of the plain binary64 path from ten LES-like domains, then
    Adam on the library's float32 kernels; returns the training record."""
    from paper_2010_14823_amd import surrogate
    t0 = time.perf_counter()
    casim.init()
    data = surrogate.generate_samples(range(10, 20), per_seed, log=lambda m: log(m))
    n_samples = int(data["n"])
    t1 = time.perf_counter()
    tr = surrogate.Trainer(data, seed=0, log=lambda m: log(m))
    untrained = tr.eval_loss(tr.val_idx)
    y = tr.y.cpu().numpy()[tr.val_idx]
    m = tr.m.cpu().numpy()[tr.val_idx]
    y0 = -np.array(tr.stats.y_mean) / np.array(tr.stats.y_std)
    zero = float(np.sum(m * (y0 - y) ** 2) / np.sum(m))
    hist = tr.fit(epochs=budget_epochs, batch=4096, lr=2e-3)
    t2 = time.perf_counter()
    casim.surrogate_load()
    del data, tr
    torch.cuda.empty_cache()
    return {"samples": n_samples, "validation_fraction": 0.1, "seeds": "10-19", "per_seed": per_seed,
            "epochs": budget_epochs, "batch": 4096, "sample_seconds": t1 - t0, "train_seconds": t2 - t1,
            "val_loss": min(h["val_loss"] for h in hist), "untrained_val_loss": untrained,
            "zero_predictor_val_loss": zero, "final_train_batch_loss": hist[-1]["train_batch_loss"]}


def coupled_errors(torch, casim, dev, dz, dt, nsteps=10):
    """Ten coupled steps of FP32-mixed and of binary64 plain, each evolving its
    own state with the parent-model update (X += dt tend, clip at 0): per
    field error of the state after nsteps - 1 updates and of the tendencies
    of step nsteps, FP32-mixed against binary64."""
    nf, nlev, ncol = dev.shape
    x64, x32 = casim.empty_fields(nf, nlev, ncol), casim.empty_fields(nf, nlev, ncol)
    x64.copy_(dev)
    x32.copy_(dev)
    t64, t32 = casim.empty_fields(12, nlev, ncol), casim.empty_fields(12, nlev, ncol)
    s64 = torch.empty((8, ncol), dtype=torch.float64, device="cuda")
    s32 = torch.empty_like(s64)
    for s in range(nsteps):
        for mode, x, t, sf in ((0, x64, t64, s64), (1, x32, t32, s32)):
            casim.init(casim.default_constants(mode=mode))
            casim.step(x, dz, dt, t, sf)
            if s + 1 < nsteps:
                casim.apply_tendencies(x, dz, dt, t, sf)
    torch.cuda.synchronize()
    out = {"state": state_errors(x32, x64), "tendencies": field_errors(t32, s32, t64, s64)}
    del x64, x32, t64, t32, s64, s32
    torch.cuda.empty_cache()
    return out


def timeindata(torch, casim, st, dz, cfg, reps=3):
    """The paper's per-step split (Sec. III-C table: copy-on, kernel, copy-off)
    for a state held in host memory: casim_step_host with one column block
    (copy in, step, copy out in sequence) and with four (the blocks' copies
    and steps overlap), from events on the library's three internal streams,
    beside the wall time per step."""
    nf, nlev, ncol = st.shape
    hin, hout, hsfc = casim.HostArray(st.shape), casim.HostArray((12, nlev, ncol)), casim.HostArray((8, ncol))
    hin.array[:] = st
    casim.init()
    out = {"workload": workload_name(cfg), "bytes_h2d": int(st.nbytes), "bytes_d2h": int(8 * (12 * nlev + 8) * ncol)}
    for nb in (1, 4):
        casim.step_host(hin.array, dz, cfg.dt, hout.array, hsfc.array, nblocks=nb)
        torch.cuda.synchronize()
        walls, splits = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            casim.step_host(hin.array, dz, cfg.dt, hout.array, hsfc.array, nblocks=nb)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            splits.append(casim.host_times()[:3])
        h2d, kern, d2h = (float(np.median([sp[k] for sp in splits])) for k in range(3))
        tot = h2d + kern + d2h
        out["blocks_%d" % nb] = {"wall_ms_per_step": float(np.median(walls)) * 1e3, "h2d_ms": h2d, "kernel_ms": kern,
                                 "d2h_ms": d2h, "h2d_share": h2d / tot, "kernel_share": kern / tot,
                                 "d2h_share": d2h / tot,
                                 "pcie_GBps_both_directions": (out["bytes_h2d"] + out["bytes_d2h"]) /
                                 float(np.median(walls)) / 1e9}
    for h in (hin, hout, hsfc):
        h.free()
    return out


def _shared_worker(rank, nranks, cfg_key, steps, warmup, barrier, queue):
    """One of nranks processes sharing the GPU: its own library context and
    stream, the grid rows rank, rank + nranks, ... of the workload (an
    interleaved share, so clustered cloud spreads over the ranks)."""
    try:
        import torch
        from paper_2010_14823_amd import casim, synth
        cfg = synth.CONFIGS[cfg_key]
        rows = list(range(rank, cfg.ny, nranks))
        f, dz, _ = synth.generate(cfg, rows)
        st = synth.stack(f)
        del f
        dev = device_fields(torch, casim, st)
        ncol = st.shape[2]
        tend = casim.empty_fields(12, cfg.nlev, ncol)
        sfc = torch.empty((8, ncol), dtype=torch.float64, device="cuda")
        casim.init()
        for _ in range(warmup):
            casim.step(dev, dz, cfg.dt, tend, sfc)
        torch.cuda.synchronize()
        barrier.wait()
        t0 = time.perf_counter()
        for _ in range(steps):
            casim.step(dev, dz, cfg.dt, tend, sfc)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        barrier.wait()
        queue.put((rank, ncol * cfg.nlev, t0, t1, None))
    except Exception as e:          # reported to the parent, which fails loudly
        queue.put((rank, 0, 0.0, 0.0, repr(e)))
        try:
            barrier.abort()
        except Exception:
            pass


def shared_gpu(cfg_key="c1", counts=(1, 2, 4, 8), steps=50, warmup=5):
    """Several parent-model ranks sharing the one GPU (as the paper's ranks
    shared a P100 through MPS): each rank a separate process with its own
    context stepping its share of the columns concurrently.  Aggregate
    grid-point updates/s = all points / the slowest rank's time."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    out = {}
    for n in counts:
        barrier, queue = ctx.Barrier(n), ctx.Queue()
        procs = [ctx.Process(target=_shared_worker, args=(r, n, cfg_key, steps, warmup, barrier, queue))
                 for r in range(n)]
        for p in procs:
            p.start()
        res = [queue.get(timeout=600) for _ in range(n)]
        for p in procs:
            p.join(timeout=120)
        errs = [r[4] for r in res if r[4]]
        if errs:
            raise RuntimeError("shared-GPU rank failed: %s" % errs[0])
        pts = sum(r[1] for r in res)
        t0, t1 = min(r[2] for r in res), max(r[3] for r in res)
        out[str(n)] = {"ranks": n, "points_per_s": pts * steps / (t1 - t0), "seconds": t1 - t0,
                       "ms_per_step_slowest_rank": max((r[3] - r[2]) for r in res) * 1e3 / steps}
        log("shared GPU, %d ranks: %.3g points/s" % (n, out[str(n)]["points_per_s"]))
    base = out[str(counts[0])]["points_per_s"]
    for v in out.values():
        v["relative_to_one_rank"] = v["points_per_s"] / base
    return {"workload": "c1 shares: grid rows r, r+N, ... per rank", "steps": steps, "per_rank_count": out}


def single_mode(args, torch, casim, synth):
    """Time one configuration in one mode (for profiling)."""
    cfg = synth.CONFIGS[args.config]
    workers = host_threads()
    dev, dz = upload(torch, casim, synth, cfg, workers)
    mask = synth.cloud_mask(cfg)
    tend, sfc = outputs(torch, casim, cfg)
    # "stream": the step's streaming floor (casim_debug_stream), no physics
    mode = MODES.get(args.mode, 0)
    if mode == 2:
        if not args.checkpoint:
            print("--mode surrogate needs --checkpoint (or run the default benchmark, which trains one)",
                  file=sys.stderr)
            sys.exit(2)
        casim.init()
        casim.mlp_load(open(args.checkpoint, "rb").read())
        casim.surrogate_load()
    casim.init(casim.default_constants(mode=mode, warm=1 if args.warm else 0))
    t = time_steps(torch, casim, dev, dz, cfg.dt, tend, sfc, args.steps, args.warmup,
                   casim.debug_stream if args.mode == "stream" else None)
    rec = mode_record(cfg, mask, t, args.warm)
    pts = cfg.ncol * cfg.nlev
    line = {"metric": METRIC, "value": pts / (t["ms_per_step"] * 1e-3), "unit": "grid-point updates/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64" if mode in (0, 3) else "f32+f64", "data": "synthetic",
            "config": {"workload": "%s %s step: %s" % (cfg.name, args.mode, workload_name(cfg)),
                       "columns": cfg.ncol, "levels": cfg.nlev, "points": pts, "mode": args.mode,
                       "configuration": "warm" if args.warm else "cold"},
            "mode_record": rec}
    if not args.no_copy:
        line["copy_probe"] = copy_probe(torch)
    print(json.dumps(line), flush=True)


def infer_rows(args, torch, casim):
    """Time the surrogate's inference kernel alone (casim_surrogate_infer) on
    N rows of seeded standard-normal features with random gates, statistics
    fitted to the first 200,000 rows and seeded random parameters (N(0, 0.1)):
    the kernel's cost does not depend on what the network learned."""
    n = args.infer_rows
    rng = np.random.default_rng(0)
    casim.init()
    feat = torch.from_numpy(rng.normal(size=(n, 12)).astype(np.float32)).cuda()
    gates = torch.from_numpy(rng.integers(0, 1 << 13, n).astype(np.int16)).cuda()
    rates = torch.zeros((n, 12), dtype=torch.float32, device="cuda")
    fb = torch.empty((n,), dtype=torch.uint8, device="cuda")
    m = min(n, 200_000)
    casim.mlp_fit_stats(feat[:m], rates[:m], gates[:m], m)
    casim.mlp_set_params(rng.normal(0.0, 0.1, casim.MLP_NPARAMS).astype(np.float32))
    casim.surrogate_load()
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        casim.surrogate_infer(feat, gates, n, rates, fb, stream)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        casim.surrogate_infer(feat, gates, n, rates, fb, stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    med = ms[len(ms) // 2]
    tf = n * NET_FLOP_PER_POINT / (med * 1e-3) / 1e12
    print(json.dumps({"kernel": "surrogate_infer_kernel", "rows": n, "launches": args.steps,
                      "ms_median": med, "ms_min": ms[0], "ms_max": ms[-1], "TFLOPs": tf,
                      "frac_bf16_peak": tf / BF16_PEAK_TFLOPS, "fallback": int(fb.sum().item())}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default=None, help="time one configuration only (c0..c4)")
    ap.add_argument("--mode", default="fp64", choices=sorted(MODES) + ["stream"])
    ap.add_argument("--warm", action="store_true", help="warm configuration (with --config)")
    ap.add_argument("--checkpoint", default=None, help="surrogate checkpoint for --config ... --mode surrogate")
    ap.add_argument("--epochs", type=int, default=40, help="surrogate training budget in epochs")
    ap.add_argument("--per-seed", type=int, default=400_000, help="surrogate training samples per seed")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-copy", action="store_true", help="skip the 2 GiB device copy probe")
    ap.add_argument("--no-c2", action="store_true", help="skip the sparse deep-convection domain")
    ap.add_argument("--no-surrogate", action="store_true", help="skip training and timing the surrogate")
    ap.add_argument("--no-shared", action="store_true", help="skip the several-ranks-on-one-GPU measurement")
    ap.add_argument("--no-pipeline", action="store_true",
                    help="skip the host-resident step (copy-in / step / copy-out split, c1 and c3)")
    ap.add_argument("--infer-rows", type=int, default=0,
                    help="time only the surrogate inference kernel on this many synthetic rows")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the column step needs no exchange between GPUs, and this benchmark "
              "runs on a single MI355X (sharding across GPUs is described, not built); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2010_14823_amd import casim, synth

    if args.infer_rows:
        infer_rows(args, torch, casim)
        return
    if args.config:
        single_mode(args, torch, casim, synth)
        return

    t_begin = time.perf_counter()
    workers = host_threads()
    K, W = args.steps, args.warmup
    c3, c4, c2 = synth.CONFIGS["c3"], synth.CONFIGS["c4"], synth.CONFIGS["c2"]

    # ---- binary64 plain and FP32-mixed on the headline domain ----------------
    t0 = time.perf_counter()
    st3, dz = synth.generate_stacked(c3, workers=workers)
    dev = device_fields(torch, casim, st3)
    log("%s generated and uploaded in %.1f s" % (c3.name, time.perf_counter() - t0))
    mask3 = synth.cloud_mask(c3)
    tend, sfc = outputs(torch, casim, c3)
    casim.init(casim.default_constants(mode=0))
    t64 = time_steps(torch, casim, dev, dz, c3.dt, tend, sfc, K, W)
    log("fp64 %s: %.4f ms/step (events: median %.4f)" % (c3.name, t64["ms_per_step"], t64["event_ms"]["median"]))
    ref_t, ref_s = tend.clone(), sfc.clone()
    # the step's own memory traffic without its physics (same tiles, order,
    # activity test and loads; zeros stored): its streaming floor
    stream = torch.cuda.current_stream()
    for _ in range(W):
        casim.debug_stream(dev, dz, c3.dt, tend, sfc)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for a, b in ev:
        a.record(stream)
        casim.debug_stream(dev, dz, c3.dt, tend, sfc)
        b.record(stream)
    torch.cuda.synchronize()
    floor_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    log("streaming floor of the step's access pattern: %.4f ms" % floor_ms)
    casim.init(casim.default_constants(mode=1))
    t32 = time_steps(torch, casim, dev, dz, c3.dt, tend, sfc, K, W)
    log("fp32mix %s: %.4f ms/step" % (c3.name, t32["ms_per_step"]))
    err32 = field_errors(tend, sfc, ref_t, ref_s)
    del ref_t, ref_s
    torch.cuda.empty_cache()
    err32_10 = coupled_errors(torch, casim, dev, dz, c3.dt, 10)
    del dev, tend, sfc
    torch.cuda.empty_cache()

    modes = {"fp64": mode_record(c3, mask3, t64), "fp32mix": mode_record(c3, mask3, t32)}
    modes["fp32mix"]["speedup_vs_fp64"] = t64["ms_per_step"] / t32["ms_per_step"]
    modes["fp32mix"]["error_vs_fp64_plain"] = {
        "one_step": err32, "worst_one_step": worst(err32),
        "ten_coupled_steps": err32_10,
        "worst_ten_steps": {"state": worst(err32_10["state"]), "tendencies": worst(err32_10["tendencies"])},
        "metric": "normwise: max |fp32mix - fp64| / max |fp64| and RMS(fp32mix - fp64) / RMS(fp64) per field "
                  "over the whole domain; the binary64 GPU path equals the oracle to 1e-12 per field (tests)"}

    # ---- the learned surrogate --------------------------------------------------
    if not args.no_surrogate:
        train = train_surrogate(torch, casim, args.epochs, args.per_seed)
        log("surrogate trained: val loss %.4f (untrained %.4f, zero predictor %.4f)"
            % (train["val_loss"], train["untrained_val_loss"], train["zero_predictor_val_loss"]))
        dev, dz = upload(torch, casim, synth, c4, workers)
        mask4 = synth.cloud_mask(c4)
        tend, sfc = outputs(torch, casim, c4)
        casim.init(casim.default_constants(mode=0))
        t64_4 = time_steps(torch, casim, dev, dz, c4.dt, tend, sfc, K, W)
        ref_t, ref_s = tend.clone(), sfc.clone()
        casim.init(casim.default_constants(mode=2))
        tsur = time_steps(torch, casim, dev, dz, c4.dt, tend, sfc, K, W)
        log("surrogate %s: %.4f ms/step (fp64 on this domain %.4f)" % (c4.name, tsur["ms_per_step"],
                                                                        t64_4["ms_per_step"]))
        errs = field_errors(tend, sfc, ref_t, ref_s)
        pts4 = c4.ncol * c4.nlev
        st_s = tsur["status"]
        rec = mode_record(c4, mask4, tsur)
        rec.update({"fp64_ms_per_step_same_domain": t64_4["ms_per_step"],
                    "speedup_vs_fp64": t64_4["ms_per_step"] / tsur["ms_per_step"],
                    "error_vs_fp64_plain": {"one_step": errs, "worst": worst(errs),
                                            "metric": "normwise per field over the whole domain, one step from "
                                                      "the same state"},
                    "inferred_points_per_step": st_s["inferred"] / K, "fallback_points_per_step": st_s["fallback"] / K,
                    "fallback_fraction_of_slotted": st_s["fallback"] / max(1, st_s["inferred"] + st_s["fallback"]),
                    "network_flop_per_inferred_point": NET_FLOP_PER_POINT, "training": train})
        rec["network_flop_per_step"] = NET_FLOP_PER_POINT * (st_s["inferred"] + st_s["fallback"]) / K
        modes["surrogate"] = rec
        del dev, tend, sfc, ref_t, ref_s
        torch.cuda.empty_cache()

    # ---- binary64 on the sparse deep-convection domain ---------------------------
    extra = {}
    if not args.no_c2:
        dev, dz = upload(torch, casim, synth, c2, workers)
        tend, sfc = outputs(torch, casim, c2)
        casim.init(casim.default_constants(mode=0))
        t2 = time_steps(torch, casim, dev, dz, c2.dt, tend, sfc, K, W)
        log("fp64 %s: %.4f ms/step" % (c2.name, t2["ms_per_step"]))
        extra["c2_fp64"] = mode_record(c2, synth.cloud_mask(c2), t2)
        del dev, tend, sfc
        torch.cuda.empty_cache()

    pts = c3.ncol * c3.nlev
    alg = algorithmic_bytes(c3, mask3)
    kern_ms = t64["event_ms"]["mean"]
    achieved = alg / (kern_ms * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": pts / (t64["ms_per_step"] * 1e-3),
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": t64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c3: " + workload_name(c3) + "; binary64 plain step (value); FP32-mixed on the "
                               "same domain and the surrogate on c4 (the same distribution, seed 4) in 'modes'",
                   "columns": c3.ncol, "levels": c3.nlev, "points": pts, "mode": "fp64", "configuration": "cold"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(c3.name, "fp64"),
                     "kernel": "sweep_kernel, binary64 (HIP events around each step on the launch stream; the "
                               "tile-order kernel of ~20 us that precedes it is included)",
                     "kernel_ms": kern_ms, "algorithmic_bytes": alg,
                     "streaming_floor_ms": floor_ms,
                     "streaming_floor_GBps": alg / (floor_ms * 1e-3) / 1e9,
                     "frac_of_streaming_floor": floor_ms / kern_ms,
                     "streaming_floor": "casim_debug_stream: the same sweep (tiles, launch order, activity test, "
                                        "the loads of busy chunks) storing zeros, no physics",
                     "bytes_per_point": {"cloudy_column": B_CLOUDY, "clear_column": B_CLEAR,
                                         "per_column": B_COLUMN}},
        "modes": modes,
    }
    line.update(extra)
    if not args.no_pipeline:
        c1 = synth.CONFIGS["c1"]
        st1, dz1 = synth.generate_stacked(c1, workers=workers)
        line["timeindata"] = {"c1": timeindata(torch, casim, st1, dz1, c1), "c3": timeindata(torch, casim, st3, dz, c3, 2)}
        del st1
        log("host pipeline split measured")
    del st3
    if not args.no_shared:
        torch.cuda.synchronize()
        line["shared_gpu"] = shared_gpu("c1", (1, 2, 4, 8), steps=50, warmup=5)
    if not args.no_copy:
        line["copy_probe"] = copy_probe(torch)
        line["roofline"]["frac_of_copy"] = achieved / line["copy_probe"]["GBps"]
        line["stream_ceiling"] = stream_ceiling(torch, casim)
        line["roofline"]["frac_of_stream_copy"] = achieved / line["stream_ceiling"]["copy_GBps"]
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(c3, list(range(0, 64)))
    line["bench_seconds"] = time.perf_counter() - t_begin
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
