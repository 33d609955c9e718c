"""Throughput benchmark: Kalman-filter track building and fitting on one GPU.

Workload (fit_scale): 200 events x 20 000 tracks, 17 barrel layers at
r = 4..68 cm, Bz = 3.8 T, seeded synthetic events (inputs resident in HBM
before timing).  One step = one pass of the hot path over the whole batch:
  hit_bin (all 200 events) -> kf_build (all 4 M seeds, one persistent launch)
  -> kf_fit (all 4 M tracks over their hit lists).
value = tracks per second through the step (each track built and fitted).

Prints one JSON line.  Per-kernel durations are measured with HIP events on
the stream the kernels run on.  The CPU baseline is the FP64 oracle timed on
a bounded sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "KF tracks/s (fit & build) on 1 GPU; learned-window vs plain at equal efficiency"

# Algorithmic work per candidate-layer of the fit formulation (see kfdev.h):
# propagate 60, transport + scattering 550, innovation 37, chi2 10, update 165
FIT_FLOP_PER_TRACK_LAYER = 822
# bytes per fitted track: 14 hit rows of 9 floats, seed (27 floats + q),
# outputs (27 floats + chi2 + ndof + status)
FIT_BYTES_PER_TRACK_14 = 14 * 36 + (27 * 4 + 1) + (27 * 4 + 12)
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (published)
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=None, help="override the number of events (testing)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--arith", choices=["f32", "f64"], default="f64",
                    help="arithmetic of the fit and build kernels (storage is FP32)")
    return ap.parse_args()


def cpu_baseline(w, fb, seconds):
    """FP64 oracle on a bounded sample of the same tracks (single thread)."""
    import oracle
    L = w.geometry.n_layers
    chunk = 2000
    done = 0
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < seconds:
        lo = (k * 7919 * chunk) % max(fb.n - chunk, 1)
        H = np.ascontiguousarray(fb.hits[:, :, lo:lo + chunk])
        so = oracle.seed(w.geometry, H, chunk)
        oracle.fit(w.geometry, 3, H, so["par"], so["cov"], so["q"], chunk)
        done += chunk
        k += 1
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "tracks/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} fit_scale tracks (seed + fit, {L} layers), FP64 oracle, single thread, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_1711_06571_amd import kftrack, presets, workloads

    dev = "cuda:0"
    w = presets.fit_scale()
    t_gen = time.perf_counter()
    fb = workloads.fit_batch(w, n_events=args.events)
    t_gen = time.perf_counter() - t_gen
    n = fb.n
    Hd = torch.from_numpy(fb.hits).to(dev)
    seeds = kftrack.kf_seed(w.geometry, n, Hd)
    out = None
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()

    arith = kftrack.ARITH_F64 if args.arith == "f64" else kftrack.ARITH_F32

    def step(evs=None, ar=None):
        nonlocal out
        if evs is not None:
            evs[0].record(stream)
        out = kftrack.kf_fit(w.geometry, n, 3, Hd, seeds["par"], seeds["cov"], seeds["q"], out=out,
                             arith=arith if ar is None else ar)
        if evs is not None:
            evs[1].record(stream)

    # the other arithmetic, timed separately for reference
    other = kftrack.ARITH_F32 if arith == kftrack.ARITH_F64 else kftrack.ARITH_F64
    step(ar=other)
    oe = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
    for e in oe:
        step(e, ar=other)
    torch.cuda.synchronize()
    other_ms = float(np.mean([a.elapsed_time(b) for a, b in oe]))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fit_ms = np.array([a.elapsed_time(b) for a, b in evs])
    ms_per_step = wall * 1e3 / args.steps
    value = n / (ms_per_step * 1e-3)

    L = w.geometry.n_layers
    flop = n * (L - 3) * FIT_FLOP_PER_TRACK_LAYER
    fit_avg = float(fit_ms.mean())
    achieved = flop / (fit_avg * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None, "kernel": "fit_kernel",
            "avg_ms": round(fit_avg, 4),
            "hbm_GBs_algorithmic": round(n * FIT_BYTES_PER_TRACK_14 / (fit_avg * 1e-3) / 1e9, 1)}
    res = {
        "metric": METRIC, "value": round(value, 1), "unit": "tracks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.arith, "data": "synthetic",
        "config": {"workload": w.name, "tracks": n, "events": n // w.n_tracks, "layers": L,
                   "step": "kf_fit"},
        "roofline": roof,
        "stages_ms": {"kf_fit": round(fit_avg, 4)},
        "other_arith": {"arith": "f32" if args.arith == "f64" else "f64", "kf_fit_ms": round(other_ms, 4)},
        "gen_s": round(t_gen, 2),
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(w, fb, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
