"""Throughput benchmark: Kalman-filter track building and fitting on one GPU.

Workload (fit_scale): 200 events x 20 000 tracks, 17 barrel layers at
r = 4..68 cm, Bz = 3.8 T, seeded synthetic events; inputs resident in HBM
before timing.  One step = one pass of the hot path over the whole batch:
  hit_bin (all 200 events) -> kf_build (all 4 M seeds, one persistent launch)
  -> kf_gather_hits -> kf_fit (all 4 M built tracks).
value = tracks per second through the step (each track built and fitted).

Prints one JSON line.  Per-kernel durations come from HIP events recorded on
the stream the kernels run on.  The CPU baseline is the FP64 oracle (brute-
force build, then fit) timed on a bounded sample of the same workload.
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

# Algorithmic FP work (FMA = 2 flops) of the formulation in kfdev.h
FLOP_PREDICT = 610      # helix crossing 60 + surface Jacobian, transport and scattering noise 550
FLOP_WINDOW = 25        # window half-widths from the predicted covariance
FLOP_WINDOW_TEST = 8    # exact phi/z test of one scanned hit
FLOP_CHI2 = 47          # innovation + chi2 of one in-window hit
FLOP_UPDATE = 202       # innovation + Kalman gain and state/covariance update
# the general detector's build (two-step propagation): step 1 per candidate
# step is FLOP_PREDICT + FLOP_WINDOW; per in-window hit, step 2 (helix step
# 40, measured rows of the surface Jacobian 60, S = M P M^T + V 170) and chi2
FLOP_STEP2_CHI2 = 310
# a chosen hit: step 2 with the full transport and scattering, then the update
FLOP_STEP2_UPDATE = FLOP_PREDICT + FLOP_UPDATE
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}   # MI355X vector peaks (published)
# algorithmic bytes of one fitted track (14 layers): hit rows 14 x 36 B, seed
# (27 FP32 + charge) 109 B, outputs (27 FP32, chi2, ndof, status) 120 B
FIT_BYTES_PER_TRACK = 14 * 36 + 109 + 120
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--events", type=int, default=None, help="override the number of events (testing)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=25.0)
    ap.add_argument("--arith", choices=["f32", "f64"], default="f64",
                    help="arithmetic of the fit and build kernels (storage is FP32)")
    ap.add_argument("--no-other-arith", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-plain window comparison")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched uneven-events measurement")
    ap.add_argument("--no-lids", action="store_true", help="skip the general-detector (endcap disks) measurement")
    ap.add_argument("--autotune", action="store_true", help="sweep the batched build's launch parameters")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes 5 times (counter calibration)")
    return ap.parse_args()


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_build_kernel_fit_scale_f64.md")


def measured_traffic(kernel_name):
    """HBM bytes per launch of the build kernel from the committed counter
    summary, if it was taken on the kernel sources as they are now."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
        d = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        h = hashlib.sha256()
        for f in d["kernel_sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != d["source_sha256"] or d["kernel"] != kernel_name:
            return None
        return d["traffic_bytes_per_launch"]
    except (OSError, AttributeError, KeyError, ValueError):
        return None


def copy_only(nbytes):
    """A plain device-to-device copy of known size: what the HBM traffic
    counters read for it calibrates their reading for the kernels."""
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4, "reps": 5}), flush=True)


TRAIN_ROWS = 2_000_000


def learned_vs_plain(ariths, log):
    """Learned search window against the plain one on the learned workload
    (the build workload's generator, other events): 2 M rows dumped by the
    plain build of train events 0..2, gates at a quantile of their plain
    widths, GPU training on the gated rows (and, beside it, an ungated
    network trained on all rows), kappa calibrated on event 3 to keep the
    plain efficiency within 0.1 %, comparison on events 4..35, in each
    arithmetic and in both states (the network reads the Cartesian
    prediction; in the hybrid state it is trained on rows of the hybrid-state
    build, whose plain windows are narrower)."""
    import torch
    from paper_1711_06571_amd import kftrack as kf
    from paper_1711_06571_amd import presets, window
    w = presets.learned()
    t0 = time.perf_counter()
    tr = window.load_events(w, [0, 1, 2])
    rows = window.dump_rows(w, tr)[:TRAIN_ROWS]
    t = window.train_gated(w, rows, epochs=4)
    tu = window.train_gated(w, rows, quantile=0.0, epochs=4)
    rows_h = window.dump_rows(w, tr, state=kf.STATE_HYBRID)[:TRAIN_ROWS]
    t_h = window.train_gated(w, rows_h, epochs=4)
    del tr
    val = window.load_events(w, [3])
    # 32 events (640 k seeds, ~30 seed groups per wave): with only a few groups
    # per wave the build time is the slowest group's, not the throughput
    test = window.load_events(w, list(range(4, 36)))
    n = test.eb.n_seeds
    res = {"workload": f"{w.name}: 32 test events x {n // 32} tracks + noise", "train_rows": int(rows.shape[0]),
           "train_events": [0, 1, 2], "validation_event": 3,
           "gate_quantile": window.GATE_QUANTILE, "gates_cm": [round(v, 5) for v in t.gates],
           "rows_gated": int(t.rows_used), "train_seconds": round(t.seconds, 3), "loss_initial": round(t.loss0, 5),
           "loss_final": round(t.losses[-1], 5),
           "ungated_network": {"rows": int(tu.rows_used), "loss_initial": round(tu.loss0, 5),
                               "loss_final": round(tu.losses[-1], 5)},
           "hybrid_state_network": {"train_rows": int(rows_h.shape[0]), "gates_cm": [round(v, 5) for v in t_h.gates],
                                    "rows_gated": int(t_h.rows_used), "loss_initial": round(t_h.loss0, 5),
                                    "loss_final": round(t_h.losses[-1], 5)}}

    def compare(net, arith, state, outp, ep, tp, cp):
        out_v, _ = window.build(w, val, arith=arith, state=state)
        eff_val = window.efficiency(w, val, out_v)
        kap, trace = window.calibrate(w, net, val, eff_val, target=0.001, arith=arith, state=state)
        kf.mlp_set_header(net.block, kappa=kap)
        outl, cl = window.build(w, test, window_mode=1, block=net.block, counters=True, arith=arith, state=state)
        torch.cuda.synchronize()
        el = window.efficiency(w, test, outl)
        tl = window.time_build(w, test, 1, net.block, arith=arith, state=state)
        lost, lost_frac = window.lost_hits(w, test, outp, outl)
        cl = cl.cpu().numpy()
        return {"kappa": kap, "calibration": trace,
                "learned": {"build_ms": round(tl, 4), "seeds_per_s": round(n / (tl * 1e-3), 1),
                            "efficiency": round(el, 4),
                            "hits_tested_per_cand_layer": round(float(cl[1]) / max(float(cl[0]), 1), 3),
                            "lost_hits": lost, "lost_hit_fraction": round(lost_frac, 6)},
                "speedup": round(tp / tl, 3), "efficiency_loss": round(ep - el, 4)}

    for arith, state in [(a, kf.STATE_CARTESIAN) for a in ariths] + [(a, kf.STATE_HYBRID) for a in ariths]:
        name = ("f64" if arith == kf.ARITH_F64 else "f32") + ("_hybrid" if state == kf.STATE_HYBRID else "")
        outp, cp = window.build(w, test, counters=True, arith=arith, state=state)
        torch.cuda.synchronize()
        ep = window.efficiency(w, test, outp)
        tp = window.time_build(w, test, 0, arith=arith, state=state)
        cp = cp.cpu().numpy()
        r = compare(t_h if state == kf.STATE_HYBRID else t, arith, state, outp, ep, tp, cp)
        r["plain"] = {"build_ms": round(tp, 4), "seeds_per_s": round(n / (tp * 1e-3), 1), "efficiency": round(ep, 4),
                      "hits_tested_per_cand_layer": round(float(cp[1]) / max(float(cp[0]), 1), 3)}
        if state == kf.STATE_CARTESIAN:
            # the same comparison with the ungated network (consulted for every candidate)
            u = compare(tu, arith, state, outp, ep, tp, cp)
            r["ungated"] = {"kappa": u["kappa"], **u["learned"], "speedup": u["speedup"],
                            "efficiency_loss": u["efficiency_loss"]}
        log(f"learned {name}: kappa {r['kappa']}, eff plain {ep:.4f} learned {r['learned']['efficiency']:.4f}, "
            f"ms {tp:.3f} vs {r['learned']['build_ms']:.3f}, lost hits {r['learned']['lost_hit_fraction']:.5f}")
        res[name] = r
    res["total_seconds"] = round(time.perf_counter() - t0, 1)
    return res


def batched(arith, autotune, log):
    """64 events of uneven size (log-uniform 500..50 000 tracks, 5..30 %
    noise per layer) built in one persistent launch replayed as a HIP graph
    (binning of every event + the build)."""
    import numpy as np
    from paper_1711_06571_amd import batch, presets
    from paper_1711_06571_amd import kftrack as kf
    w = presets.batch()
    b = batch.load(w)
    if autotune:
        # sweep in the benchmark's arithmetic; the choice goes into the cache
        # (kftrack.TUNE_CACHE layout) written beside the other outputs
        tr = batch.autotune(b, log=lambda q: log(f"tune {q}"), arith=arith)
        os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
        batch.save_cache(tr, arith, os.path.join(ROOT, "gpurun_out", "autotune.json"), w.name)
        batch.save(tr, os.path.join(ROOT, "gpurun_out", "autotune_points.json"), w.name)
    # the default launch shape, then the autotuner's cached choice
    p = batch.plan(b, arith=arith)
    ms_default = batch.run(p, reps=5)
    p.close()
    cached = kf.tuned_launch(arith)
    p = batch.plan(b, arith=arith, tuned=True)
    ms = batch.run(p, reps=5)
    lat = batch.latencies_ms(b)
    eff = batch.efficiency(b, p.out)
    p.close()
    # the whole step (binning, build, gather, final fit) as one graph
    pf = batch.plan(b, arith=arith, fit=True, tuned=True)
    ms_fit = batch.run(pf, reps=5)
    pf.close()
    res = {"workload": f"{w.name}: {w.n_events} events, {b.eb.n_seeds} seeds", "ms_per_launch": round(ms, 4),
           "events_per_s": round(w.n_events / (ms * 1e-3), 2), "seeds_per_s": round(b.eb.n_seeds / (ms * 1e-3), 1),
           "latency_ms_p50": round(float(np.percentile(lat, 50)), 4),
           "latency_ms_p99": round(float(np.percentile(lat, 99)), 4), "efficiency": round(eff, 4),
           "ms_per_launch_with_fit": round(ms_fit, 4), "ms_per_launch_default_shape": round(ms_default, 4),
           "launch": "autotuned (cached choice)" if cached else "default (no cached choice)",
           "tuned": cached}
    log(f"batch: {ms:.3f} ms per launch")
    return res


def practical_peaks():
    """What the device sustains on the two roofline axes: a plain 1 GiB
    device copy (bytes read + written per second) and FMA chains in FP64 and
    FP32 (packed FP32 disabled, as in the library's kernels)."""
    import torch
    from paper_1711_06571_amd import kftrack as kf
    st = torch.cuda.current_stream()
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(5):
        dst.copy_(src)
    b.record(st)
    torch.cuda.synchronize()
    copy_gbs = 2 * n * 4 * 5 / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    res = {"hbm_copy_gbs": round(copy_gbs, 1)}
    blocks, iters = 8192, 4096
    for name, ar, dt in (("f64", kf.ARITH_F64, torch.float64), ("f32", kf.ARITH_F32, torch.float32)):
        out = torch.empty(blocks * 256, dtype=dt, device="cuda:0")
        kf.kf_peak_fma(ar, blocks, iters, out)
        a.record(st)
        kf.kf_peak_fma(ar, blocks, iters, out)
        b.record(st)
        torch.cuda.synchronize()
        res[f"fma_{name}_tflops"] = round(blocks * 256.0 * iters * 8 * 2 / (a.elapsed_time(b) * 1e-3) / 1e12, 2)
    return res


def fit_latency(arith, reps=50):
    """Latency of one kf_fit call on the small fit workload (1 event, 1 000
    tracks, 10 layers, fit over layers 4..10): median of HIP-event times
    around single calls on an idle stream."""
    import torch
    from paper_1711_06571_amd import datagen, kftrack as kf, presets
    w = presets.fit_small()
    ev = datagen.generate(w.geometry, w.gen, 0, w.n_tracks)
    n = ev.n_tracks
    H = torch.from_numpy(datagen.track_hits(ev)).to("cuda:0")
    s = kf.kf_seed(w.geometry, n, H)
    out = kf.kf_fit(w.geometry, n, 3, H, s["par"], s["cov"], s["q"], arith=arith)
    torch.cuda.synchronize()
    ts = []
    st = torch.cuda.current_stream()
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        kf.kf_fit(w.geometry, n, 3, H, s["par"], s["cov"], s["q"], out=out, arith=arith)
        b.record(st)
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b) * 1e3)
    return {"workload": w.name, "tracks": n, "us_median": round(float(np.median(ts)), 2),
            "us_min": round(float(np.min(ts)), 2)}


def lids(arith, log, n_events=16, fit_events=50):
    """The general detector (section 4.1: the barrel closed by endcap disks,
    modules off the average surfaces): 16 events x 20 000 tracks (|eta| <= 2,
    20 % noise per layer) through hit_bin_det -> kf_build_det (two-step
    propagation, one persistent launch) -> kf_gather_hits -> kf_fit_det, and
    the fit alone over 50 events x 20 000 tracks (lids_fit)."""
    import torch
    from paper_1711_06571_amd import kftrack as kf
    from paper_1711_06571_amd import presets, workloads
    dev = "cuda:0"
    w = presets.lids()
    d = w.detector
    cuts = w.cuts
    L, F = d.n_layers, cuts.first_layer
    t0 = time.perf_counter()
    eb = workloads.det_event_batch(w, range(n_events))
    n = eb.n_seeds
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    layer, xyz, cov, hoff, sev = T(eb.layer), T(eb.xyz), T(eb.cov), T(eb.hit_offsets), T(eb.seed_event)
    seeds = kf.kf_seed(d.seed_geometry(), n, T(eb.track_rows[:3]))
    binned = kf.BinnedHits(n_events, L, cuts.n_phi_bins, cuts.n_z_bins, xyz.shape[1], dev)
    ws_bin = torch.empty(kf.hit_bin_workspace_bytes(n_events, L, cuts.n_phi_bins, cuts.n_z_bins, xyz.shape[1]),
                         dtype=torch.uint8, device=dev)
    bp = kf.build_params(cuts, arith=arith)
    ws_build = torch.empty(kf.kf_build_workspace_bytes(bp, binned, n), dtype=torch.uint8, device=dev)
    ld = seeds["par"].shape[1]
    fit_hits = torch.zeros((L, 9, ld), dtype=torch.float32, device=dev)
    hole = torch.zeros(ld, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    state = {}

    def step(evs=None, counters=None):
        rec = (lambda i: evs[i].record(stream)) if evs is not None else (lambda i: None)
        ex = kf.BuildExtra()
        ex.seed_event = sev.data_ptr()
        if counters is not None:
            ex.counters = counters.data_ptr()
        rec(0)
        kf.hit_bin_det(d, cuts.n_phi_bins, cuts.n_z_bins, layer, xyz, cov, event_offsets=hoff, out=binned, ws=ws_bin)
        rec(1)
        state["b"] = kf.kf_build_det(d, bp, binned, n, seeds["par"], seeds["cov"], seeds["q"], extra=ex,
                                     out=state.get("b"), ws=ws_build)
        rec(2)
        kf.kf_gather_hits(L, F, n, state["b"]["hits"], xyz, cov, seed_event=sev, event_offsets=hoff,
                          fit_hits=fit_hits, hole_mask=hole)
        rec(3)
        state["f"] = kf.kf_fit_det(d, n, F, fit_hits, state["b"]["visit"], seeds["par"], seeds["cov"], seeds["q"],
                                   hole_mask=hole, out=state.get("f"), arith=arith)
        rec(4)

    step()
    reps = 5
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(reps)]
    torch.cuda.synchronize()
    tw = time.perf_counter()
    for k in range(reps):
        step(evs[k])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - tw) * 1e3 / reps
    st = np.array([[evs[k][i].elapsed_time(evs[k][i + 1]) for i in range(4)] for k in range(reps)]).mean(axis=0)
    cnt = torch.zeros(4, dtype=torch.int64, device=dev)
    step(counters=cnt)
    torch.cuda.synchronize()
    n_pred, n_scan, n_chi2, n_upd = [int(v) for v in cnt.cpu().numpy()]
    build_flop = (n_pred * (FLOP_PREDICT + FLOP_WINDOW) + n_scan * FLOP_WINDOW_TEST + n_chi2 * FLOP_STEP2_CHI2 +
                  n_upd * FLOP_STEP2_UPDATE)
    hits = state["b"]["hits"].cpu().numpy()[:, :n]
    true = eb.true_hits[F:, :n]
    found = ((hits == true) & (true >= 0)).sum(axis=0)
    eff = float(np.mean(found >= 0.75 * (true >= 0).sum(axis=0)))
    fst = state["f"]["status"].cpu().numpy()[:n]
    names = ["hit_bin_det", "kf_build_det", "kf_gather_hits", "kf_fit_det"]
    res = {"workload": f"{w.name}; {n_events} events in one launch, {n} seeds, {eb.xyz.shape[1]} hits",
           "ms_per_step": round(ms, 4), "tracks_per_s": round(n / (ms * 1e-3), 1),
           "stages_ms": {k: round(float(v), 4) for k, v in zip(names, st)},
           "efficiency_75pct": round(eff, 4), "fit_status_ok": round(float(np.mean(fst == 0)), 4),
           "tracks_reaching_disks": round(float(np.mean(eb.visit[:n] >= (1 << 10))), 4),
           "work": {"steps": n_pred, "hits_scanned": n_scan, "step2_chi2": n_chi2, "updates": n_upd,
                    "build_gflop": round(build_flop / 1e9, 3),
                    "build_tflops": round(build_flop / (float(st[1]) * 1e-3) / 1e12, 3)}}
    del binned, ws_bin, ws_build, fit_hits, state, seeds, layer, xyz, cov
    # the fit alone at scale over the tracks' own hit lists
    wf = presets.lids_fit()
    fb = workloads.det_event_batch(wf, range(fit_events))
    nf = fb.n_seeds
    Hd = T(fb.track_rows)
    vis = T(fb.visit.view(np.int32))
    sf = kf.kf_seed(d.seed_geometry(), nf, T(fb.track_rows[:3]))
    out = kf.kf_fit_det(d, nf, F, Hd, vis, sf["par"], sf["cov"], sf["q"], arith=arith)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        kf.kf_fit_det(d, nf, F, Hd, vis, sf["par"], sf["cov"], sf["q"], out=out, arith=arith)
    e1.record(stream)
    torch.cuda.synchronize()
    fms = e0.elapsed_time(e1) / reps
    nd = out["ndof"].cpu().numpy()[:nf]
    vb = np.array([bin(int(v)).count("1") for v in fb.visit[:nf]])
    fit_flop = int(np.sum(vb - np.array([bin(int(v) & 7).count("1") for v in fb.visit[:nf]]))) * FLOP_PREDICT + \
        int(nd.sum() // 2) * FLOP_UPDATE
    res["fit_at_scale"] = {"workload": f"{wf.name}: {nf} tracks", "kf_fit_det_ms": round(fms, 4),
                           "tracks_per_s": round(nf / (fms * 1e-3), 1),
                           "tflops": round(fit_flop / (fms * 1e-3) / 1e12, 3),
                           "fit_status_ok": round(float(np.mean(out["status"].cpu().numpy()[:nf] == 0)), 4)}
    res["total_seconds"] = round(time.perf_counter() - t0, 1)
    log(f"lids: step {ms:.3f} ms ({res['stages_ms']}), fit at scale {fms:.3f} ms")
    return res


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, eb, seconds, max_threads=16):
    """FP64 oracle on the host cores: brute-force build (every hit of a layer
    is window-tested, no binning), then the fit of the built lists, seed by
    seed.  Single thread on event 0, then one thread per event (events 0..T-1)
    on all usable cores (capped at the machine's CPU share of 16); the oracle's C
    calls release the interpreter lock.  Seeding is outside the timed loops,
    as on the GPU."""
    import threading
    import oracle
    L = w.geometry.n_layers
    F = w.cuts.first_layer

    def event_inputs(e):
        h0, h1 = int(eb.hit_offsets[e]), int(eb.hit_offsets[e + 1])
        s0, s1 = int(eb.seed_offsets[e]), int(eb.seed_offsets[e + 1])
        ne = s1 - s0
        xyz = np.ascontiguousarray(eb.xyz[:, h0:h1])
        cov = np.ascontiguousarray(eb.cov[:, h0:h1])
        layer = np.ascontiguousarray(eb.layer[h0:h1])
        ld = ((ne + 63) // 64) * 64
        Hs = np.zeros((3, 9, ld), dtype=np.float32)
        Hs[:, :, :ne] = eb.seed_hits[:, :, s0:s1]
        return xyz, cov, layer, ne, oracle.seed(w.geometry, Hs, ne)

    kept = []

    def chunk(inp, k, chunk_n=8, keep=False):
        xyz, cov, layer, ne, so = inp
        lst = (np.arange(chunk_n) * 2503 + k * chunk_n * 7919) % ne
        ob = oracle.build(w.geometry, w.cuts, layer, xyz, cov, so["par"], so["cov"], so["q"], ne, seed_list=lst)
        m = lst.size
        if keep:
            kept.append((lst, ob["hits"][:, :m].copy(), ob["nhits"][:m].copy(), ob["status"][:m].copy(),
                         ob["margin"][:, :m].copy()))
        hb = ob["hits"][:, :m]
        Hf = np.zeros((L, 9, 64), dtype=np.float32)
        hm = np.zeros(64, dtype=np.uint32)
        for l in range(F, L):
            h = hb[l - F]
            have = h >= 0
            Hf[l, 0:3, :m][:, have] = xyz[:, h[have]]
            Hf[l, 3:9, :m][:, have] = cov[:, h[have]]
            hm[:m] |= np.where(have, 0, 1 << l).astype(np.uint32)
        sp = np.zeros((6, 64), np.float32)
        sc = np.zeros((21, 64), np.float32)
        q = np.ones(64, np.int8)
        sp[:, :m] = so["par"][:, lst]
        sc[:, :m] = so["cov"][:, lst]
        q[:m] = so["q"][lst]
        oracle.fit(w.geometry, F, Hf, sp, sc, q, m, hole_mask=hm)
        return m

    # single core
    inp0 = event_inputs(0)
    t_single = 0.4 * seconds
    done1, k, t0 = 0, 0, time.perf_counter()
    while time.perf_counter() - t0 < t_single:
        done1 += chunk(inp0, k, keep=True)
        k += 1
    dt1 = time.perf_counter() - t0
    # all cores: one event per thread
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    T = max(1, min(usable, max_threads, w.n_events))
    inputs = [None] * T
    done = [0] * T
    ready = threading.Barrier(T + 1)
    t_all = 0.6 * seconds
    stop = [0.0]

    def worker(t):
        inputs[t] = event_inputs(t)
        ready.wait()
        kk = 0
        while time.perf_counter() < stop[0]:
            done[t] += chunk(inputs[t], kk)
            kk += 1

    th = [threading.Thread(target=worker, args=(t,)) for t in range(T)]
    for x in th:
        x.start()
    stop[0] = float("inf")
    ready.wait()
    tA = time.perf_counter()
    stop[0] = tA + t_all
    for x in th:
        x.join()
    dtA = time.perf_counter() - tA
    rate_all = sum(done) / dtA
    return kept, {"value": round(rate_all, 2), "unit": "tracks/s", "cores": T, "kind": "oracle",
            "host_cores": os.cpu_count(), "usable_cores": usable, "cpu_model": _cpu_model(),
            "single_core": {"value": round(done1 / dt1, 2), "seeds": done1, "seconds": round(dt1, 1)},
            "sample": f"fit_scale events 0..{T - 1} (20000 tracks each), {sum(done)} seeds in {dtA:.1f} s on "
                      f"{T} threads (one event per thread), seeds spread over each event; per seed a brute-force "
                      f"FP64 oracle build over {L} layers (every hit of a layer window-tested; the GPU path "
                      f"searches binned hits) then the FP64 oracle fit of the built list; single core: "
                      f"{done1} seeds of event 0 in {dt1:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "libkftrack runs on one GPU; --gpus must be 1 (events would be split across GPUs, one process each)"}))
        sys.exit(2)
    if args.copy_bytes:
        copy_only(args.copy_bytes)
        return
    import torch
    from paper_1711_06571_amd import kftrack as kf
    from paper_1711_06571_amd import presets, workloads

    dev = "cuda:0"
    w = presets.fit_scale()
    g = w.geometry
    cuts = w.cuts
    E = w.n_events if args.events is None else args.events
    t_gen = time.perf_counter()
    eb = workloads.event_batch(w, range(E), seed_layers=3)
    t_gen = time.perf_counter() - t_gen
    n = eb.n_seeds
    L = g.n_layers
    F = cuts.first_layer
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    layer, xyz, cov = T(eb.layer), T(eb.xyz), T(eb.cov)
    hoff, sev = T(eb.hit_offsets), T(eb.seed_event)
    seeds = kf.kf_seed(g, n, T(eb.seed_hits))
    nb = cuts.n_phi_bins * cuts.n_z_bins
    binned = kf.BinnedHits(E, L, cuts.n_phi_bins, cuts.n_z_bins, xyz.shape[1], dev)
    ws_bin = torch.empty(kf.hit_bin_workspace_bytes(E, L, cuts.n_phi_bins, cuts.n_z_bins, xyz.shape[1]),
                         dtype=torch.uint8, device=dev)
    ws_build = torch.empty(kf.kf_build_workspace_bytes(kf.build_params(cuts), binned, n), dtype=torch.uint8,
                           device=dev)
    ld = seeds["par"].shape[1]
    bout = dict(hits=torch.empty((L - F, ld), dtype=torch.int32, device=dev),
                par=torch.empty((6, ld), dtype=torch.float32, device=dev),
                cov=torch.empty((21, ld), dtype=torch.float32, device=dev),
                chi2=torch.empty(ld, dtype=torch.float32, device=dev),
                nhits=torch.empty(ld, dtype=torch.int32, device=dev),
                status=torch.empty(ld, dtype=torch.int32, device=dev))
    fit_hits = torch.zeros((L, 9, ld), dtype=torch.float32, device=dev)
    hole = torch.zeros(ld, dtype=torch.int32, device=dev)
    fout = None
    ex = kf.BuildExtra()
    ex.seed_event = sev.data_ptr()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def step(arith, ev=None, extra=ex, state=kf.STATE_CARTESIAN):
        nonlocal fout
        rec = (lambda i: ev[i].record(stream)) if ev is not None else (lambda i: None)
        rec(0)
        kf.hit_bin(g, cuts.n_phi_bins, cuts.n_z_bins, layer, xyz, cov, event_offsets=hoff, out=binned, ws=ws_bin)
        rec(1)
        bp = kf.build_params(cuts, arith=arith, state=state)
        kf.kf_build(g, bp, binned, n, seeds["par"], seeds["cov"], seeds["q"], extra=extra, out=bout, ws=ws_build)
        rec(2)
        kf.kf_gather_hits(L, F, n, bout["hits"], xyz, cov, seed_event=sev, event_offsets=hoff, fit_hits=fit_hits,
                          hole_mask=hole)
        rec(3)
        fit = kf.kf_fit_hybrid if state == kf.STATE_HYBRID else kf.kf_fit
        fout = fit(g, n, F, fit_hits, seeds["par"], seeds["cov"], seeds["q"], hole_mask=hole, out=fout, arith=arith)
        rec(4)

    def timed(arith, steps, state=kf.STATE_CARTESIAN):
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            step(arith, evs[k], state=state)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        st = np.array([[evs[k][i].elapsed_time(evs[k][i + 1]) for i in range(4)] for k in range(steps)])
        return wall * 1e3 / steps, st.mean(axis=0)

    arith = kf.ARITH_F64 if args.arith == "f64" else kf.ARITH_F32
    for _ in range(args.warmup):
        step(arith)
    ms_per_step, stages = timed(arith, args.steps)
    value = n / (ms_per_step * 1e-3)

    # work counters (separate, untimed pass)
    cnt = torch.zeros(4, dtype=torch.int64, device=dev)
    exc = kf.BuildExtra()
    exc.seed_event = sev.data_ptr()
    exc.counters = cnt.data_ptr()
    step(arith, extra=exc)
    torch.cuda.synchronize()
    n_pred, n_scan, n_chi2, n_upd = [int(v) for v in cnt.cpu().numpy()]
    build_flop = (n_pred * (FLOP_PREDICT + FLOP_WINDOW) + n_scan * FLOP_WINDOW_TEST + n_chi2 * FLOP_CHI2 +
                  n_upd * FLOP_UPDATE)
    ndof = fout["ndof"].cpu().numpy()[:n]
    st = fout["status"].cpu().numpy()[:n]
    n_upd_fit = int(ndof.sum() // 2)
    n_pred_fit = n * (L - F)  # upper bound: frozen tracks stop early
    fit_flop = n_pred_fit * FLOP_PREDICT + n_upd_fit * FLOP_UPDATE
    names = ["hit_bin", "kf_build", "kf_gather_hits", "kf_fit"]
    stage_ms = {k: round(float(v), 4) for k, v in zip(names, stages)}
    dom = names[int(np.argmax(stages))]
    peak = PEAK_TFLOPS[args.arith]
    flop_of = {"kf_build": build_flop, "kf_fit": fit_flop}
    if dom in flop_of:
        ach = flop_of[dom] / (stage_ms[dom] * 1e-3) / 1e12
        kname = f"build_kernel<{'double' if args.arith == 'f64' else 'float'}, false, false>" if dom == "kf_build" else dom
        roof = {"bound": "alu", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 4), "traffic": measured_traffic(kname), "kernel": dom,
                "avg_ms": stage_ms[dom]}
    else:
        roof = {"bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": None,
                "traffic": None, "kernel": dom, "avg_ms": stage_ms[dom]}
    # physics: fraction of seeds whose built list holds >= 75 % of their true hits
    hits = bout["hits"].cpu().numpy()[:, :n]
    nhits_g = bout["nhits"].cpu().numpy()[:n]
    eff = float(np.mean((hits == eb.true_hits[F:, :n]).mean(axis=0) >= 0.75))
    res = {
        "metric": METRIC, "value": round(value, 1), "unit": "tracks/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.arith, "data": "synthetic",
        "config": {"workload": w.name, "tracks": n, "events": E, "layers": L,
                   "step": "hit_bin -> kf_build -> kf_gather_hits -> kf_fit", "window": "plain",
                   "cand_cap": cuts.cand_cap, "chi2_cut": cuts.chi2_cut, "storage": "f32"},
        "roofline": roof,
        "stages_ms": stage_ms,
        "work": {"build_cand_layers": n_pred, "build_hits_tested": n_scan, "build_chi2": n_chi2,
                 "build_updates": n_upd, "build_gflop": round(build_flop / 1e9, 3),
                 "fit_gflop": round(fit_flop / 1e9, 3),
                 "fit_algorithmic_gb": round(n * FIT_BYTES_PER_TRACK / 1e9, 3),
                 "fit_gbs": round(n * FIT_BYTES_PER_TRACK / (stage_ms["kf_fit"] * 1e-3) / 1e9, 1),
                 "build_tflops": round(build_flop / (stage_ms["kf_build"] * 1e-3) / 1e12, 3),
                 "fit_tflops": round(fit_flop / (stage_ms["kf_fit"] * 1e-3) / 1e12, 3)},
        "efficiency_75pct": round(eff, 4),
        "fit_status_ok": round(float(np.mean(st == 0)), 4),
        "gen_s": round(t_gen, 2),
    }
    if not args.no_other_arith:
        other = "f32" if args.arith == "f64" else "f64"
        oa = kf.ARITH_F32 if other == "f32" else kf.ARITH_F64
        step(oa)
        oms, ost = timed(oa, max(2, args.steps // 2))
        res["other_arith"] = {"arith": other, "ms_per_step": round(oms, 4), "tracks_per_s": round(n / (oms * 1e-3), 1),
                              "stages_ms": {k: round(float(v), 4) for k, v in zip(names, ost)}}
    # the whole step in the hybrid state (build and fit; section 3's coordinates)
    step(arith, state=kf.STATE_HYBRID)
    hms, hst = timed(arith, max(2, args.steps // 2), state=kf.STATE_HYBRID)
    hh = bout["hits"].cpu().numpy()[:, :n]
    heff = float(np.mean((hh == eb.true_hits[F:, :n]).mean(axis=0) >= 0.75))
    res["hybrid_state"] = {"ms_per_step": round(hms, 4), "tracks_per_s": round(n / (hms * 1e-3), 1),
                           "stages_ms": {k: round(float(v), 4) for k, v in zip(names, hst)},
                           "efficiency_75pct": round(heff, 4),
                           "fit_status_ok": round(float(np.mean(fout["status"].cpu().numpy()[:n] == 0)), 4)}
    log = lambda m: print(m, file=sys.stderr, flush=True)
    res["fit_small_latency"] = fit_latency(arith)
    res["practical_peaks"] = practical_peaks()
    if not args.no_learned:
        res["learned_vs_plain"] = learned_vs_plain([kf.ARITH_F32, kf.ARITH_F64], log)
    if not args.no_batch:
        res["batched"] = batched(arith, args.autotune, log)
    if not args.no_lids:
        res["lids"] = lids(arith, log)
    if not args.no_cpu_baseline:
        kept, res["cpu_baseline"] = cpu_baseline(w, eb, args.cpu_seconds)
        # the oracle's builds of the single-core sample against the timed
        # step's lists (event 0 is seeds 0..19 999): identical on every
        # decidable seed, and how many are decidable
        import oracle
        lst = np.concatenate([k_[0] for k_ in kept]) if kept else np.zeros(0, np.int64)
        if lst.size:
            oh = np.concatenate([k_[1] for k_ in kept], axis=1)
            on = np.concatenate([k_[2] for k_ in kept])
            om = np.concatenate([k_[4] for k_ in kept], axis=1)
            dec = oracle.decidable(om)
            same = np.all(hits[:, lst] == oh, axis=0) & (nhits_g[lst] == on)
            res["parity_sample"] = {"seeds": int(lst.size), "decidable": round(float(dec.mean()), 4),
                                    "identical_on_decidable": round(float(same[dec].mean()), 4),
                                    "identical_overall": round(float(same.mean()), 4),
                                    "what": "oracle build of the CPU baseline's single-core seeds vs the timed "
                                            "FP64 step's hit lists and nhits (event 0)"}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
