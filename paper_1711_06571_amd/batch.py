"""Batched building of many uneven events in one persistent, graph-captured
launch, with per-event completion latencies, and the autotuner over launch
shape and candidate cap.  Orchestration only: the work runs in libkftrack.

Seeds are handed out largest event first (a longest-processing-time order,
so the biggest events do not finish last), and within an event in index
order.  Per-event latency = the device wall-clock tick when the event's last
seed finished minus the earliest tick of the launch.
"""
from __future__ import annotations

import json
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import kftrack as kf
from . import presets, workloads

DEV = "cuda:0"


@dataclass
class Batch:
    w: presets.Workload
    eb: workloads.EventBatch
    layer: torch.Tensor
    xyz: torch.Tensor
    cov: torch.Tensor
    hoff: torch.Tensor
    sev: torch.Tensor
    seeds: dict
    order: torch.Tensor
    n_per_event: torch.Tensor
    ticks: torch.Tensor = None
    t0: torch.Tensor = None


def load(w=None, events=None) -> Batch:
    w = presets.batch() if w is None else w
    events = range(w.n_events) if events is None else events
    eb = workloads.event_batch(w, events, seed_layers=3)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    seeds = kf.kf_seed(w.geometry, eb.n_seeds, T(eb.seed_hits))
    counts = np.diff(eb.seed_offsets).astype(np.int32)
    ev_rank = np.argsort(-counts, kind="stable")
    order = np.concatenate([np.arange(eb.seed_offsets[e], eb.seed_offsets[e + 1]) for e in ev_rank]).astype(np.int32)
    b = Batch(w, eb, T(eb.layer), T(eb.xyz), T(eb.cov), T(eb.hit_offsets), T(eb.seed_event), seeds, T(order),
              T(counts))
    b.ticks = torch.zeros(len(counts), dtype=torch.int64, device=DEV)
    b.t0 = torch.zeros(1, dtype=torch.int64, device=DEV)
    return b


def extra_for(b: Batch, timestamps=True) -> kf.BuildExtra:
    ex = kf.BuildExtra()
    ex.seed_event = b.sev.data_ptr()
    ex.seed_order = b.order.data_ptr()
    if timestamps:
        ex.event_n_seeds = b.n_per_event.data_ptr()
        ex.event_done_ticks = b.ticks.data_ptr()
        ex.start_tick = b.t0.data_ptr()
    return ex


def plan(b: Batch, cap=None, lanes=0, blocks=0, arith=kf.ARITH_F32, window_mode=0, mlp_block=None, refine=0,
         fit=False, state=kf.STATE_CARTESIAN, tuned=False):
    """The batch's graph: binning and build, and with fit=True also the
    gather and the final fit of the built lists (in the same arithmetic and
    state).  tuned=True takes the launch parameters left at 0 from the
    autotuner's cached choice."""
    cuts = b.w.cuts
    bp = kf.build_params(cuts, cap=cap, lanes_per_block=lanes, persistent_blocks=blocks, arith=arith,
                         window_mode=window_mode, mlp_block=mlp_block, phi_refine=refine, state=state, tuned=tuned)
    keep = (b.sev, b.order, b.n_per_event, b.ticks, b.t0) + ((mlp_block,) if mlp_block is not None else ())
    return kf.BatchPlan(b.w.geometry, bp, b.layer, b.xyz, b.cov, b.hoff, cuts.n_phi_bins, cuts.n_z_bins,
                        b.eb.n_seeds, b.seeds["par"], b.seeds["cov"], b.seeds["q"], extra=extra_for(b),
                        fit_arith=arith if fit else None, keep=keep)


def run(p: kf.BatchPlan, reps=5) -> float:
    """Replay the graph; returns the median ms per launch."""
    p.launch()
    p.stream.synchronize()
    ts = []
    for _ in range(reps):
        a, c = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(p.stream)
        p.launch()
        c.record(p.stream)
        p.stream.synchronize()
        ts.append(a.elapsed_time(c))
    return float(np.median(ts))


def latencies_ms(b: Batch):
    khz = kf.wall_clock_khz()
    t = b.ticks.cpu().numpy().astype(np.float64)
    t0 = float(b.t0.cpu().numpy()[0])
    return (t - t0) / khz


def efficiency(b: Batch, out) -> float:
    F = b.w.cuts.first_layer
    n = b.eb.n_seeds
    hits = out["hits"].cpu().numpy()[:, :n]
    return float(np.mean((hits == b.eb.true_hits[F:, :n]).mean(axis=0) >= 0.75))


@dataclass
class TunePoint:
    lanes: int
    blocks_per_cu: int
    cap: int
    refine: int
    ms: float
    eff: float
    p50: float
    p99: float


@dataclass
class TuneResult:
    points: list = field(default_factory=list)
    best: TunePoint = None
    gpu: str = ""


def autotune(b: Batch, lanes_set=(64, 128, 256), bpcu_set=(1, 2, 0), caps=(4, 6, 8), refines=(8, 32, 64), reps=3,
             eff_tol=0.001, log=None, arith=kf.ARITH_F32) -> TuneResult:
    """Sweep launch shape x candidate cap x granularity of the fine phi index
    (the hit-search structure: sub-bins per phi bin).  Launch shape and
    granularity never change the results; the cap does, so the chosen point
    is the fastest whose efficiency is within eff_tol of the cap-6
    efficiency.  blocks_per_cu 0 means as many as fit."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    res = TuneResult(gpu=torch.cuda.get_device_name(0))
    for cap in caps:
        for refine in refines:
            for lanes in lanes_set:
                for bpcu in bpcu_set:
                    p = plan(b, cap=cap, lanes=lanes, blocks=bpcu * cus, refine=refine, arith=arith)
                    ms = run(p, reps=reps)
                    lat = latencies_ms(b)
                    eff = efficiency(b, p.out)
                    pt = TunePoint(lanes, bpcu, cap, refine, ms, eff, float(np.percentile(lat, 50)),
                                   float(np.percentile(lat, 99)))
                    res.points.append(pt)
                    if log:
                        log(pt)
                    p.close()
    res.best = choose(res.points, eff_tol)
    return res


def choose(points, eff_tol=0.001):
    """The fastest point whose efficiency is within eff_tol of the cap-6
    efficiency (the best efficiency seen if no cap-6 point was measured)."""
    ref = [q for q in points if q.cap == 6]
    eff6 = ref[0].eff if ref else max(q.eff for q in points)
    ok = [q for q in points if eff6 - q.eff <= eff_tol]
    return min(ok, key=lambda q: q.ms)


def save(res: TuneResult, path, workload):
    data = {"gpu": res.gpu, "workload": workload, "best": res.best.__dict__,
            "points": [q.__dict__ for q in res.points]}
    with open(path, "w") as f:
        json.dump(data, f, indent=1)


def save_cache(res: TuneResult, arith, path, workload):
    """Merge the chosen launch parameters into the cache kftrack reads
    (kftrack.TUNE_CACHE layout): kf_build -> arithmetic -> lanes_per_block,
    blocks_per_cu, phi_refine, plus the measurement they came from.  The cap
    is a parameter of the method, not of the launch, and is not cached."""
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    b = res.best
    data.setdefault("kf_build", {})["f64" if arith == kf.ARITH_F64 else "f32"] = {
        "lanes_per_block": b.lanes, "blocks_per_cu": b.blocks_per_cu, "phi_refine": b.refine,
        "ms": round(b.ms, 4), "cap_of_the_measurement": b.cap, "efficiency": round(b.eff, 4),
        "gpu": res.gpu, "workload": workload, "points": len(res.points)}
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
