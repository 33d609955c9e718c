"""Learned search window: data collection with the plain builder, training
with the library's GPU kernels, calibration, and the plain-vs-learned
comparison.  Orchestration only: every network and build computation runs in
libkftrack's kernels.

Data: for every candidate of the plain build whose hits so far are its
track's true hits or holes, and whose track has a hit on the layer, one row
of 27 features (predicted state and covariance) and the two labels (|arc| at
the layer radius and |dz| from the prediction to the true hit).

Training: asymmetric quantile loss (a missed true hit costs 20 times a unit
of extra width), Adam on FP32 master weights, BF16 working weights.

Gating: the network is consulted only where the plain window is wide (a
plain half-width above its gate, a quantile of the training rows' plain
widths), where it saves most of the scanned hits; elsewhere the plain window
stays.  The network is trained on the rows the gates pass.

Calibration: the widths are multiplied by kappa, chosen on validation events
as the smallest value whose build efficiency stays within the target of the
plain window's; predictions below the floors fall back to the plain window
(floors: one hit resolution, 0.01 cm arc and 0.1 cm in z).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import kftrack as kf
from . import presets, workloads

DEV = "cuda:0"
SCALE = np.array([0.01, 0.1])   # output scales: arc cm, z cm
FLOOR = (0.01, 0.1)
# the network is consulted where a plain half-width lies above this quantile
# of the training rows' (about 4 % of them): the widest windows, which scan
# most of the hits.  Rarely gated candidates leave most waves without a
# network tile to run (at the 0.9 quantile almost every wave ran one per
# layer); much higher quantiles leave the network too few training rows.
GATE_QUANTILE = 0.97
# kappa values the calibration tries, smallest first (the first that keeps
# the plain efficiency wins)
KAPPAS = [round(0.3 + 0.05 * i, 2) for i in range(19)] + [1.35, 1.5, 1.75, 2.0, 2.5, 3.0]


@dataclass
class EventOnGPU:
    eb: workloads.EventBatch
    binned: kf.BinnedHits
    seeds: dict
    xyz: torch.Tensor
    cov: torch.Tensor
    hoff: torch.Tensor
    sev: torch.Tensor


def load_events(w, events, n_tracks=None) -> EventOnGPU:
    eb = workloads.event_batch(w, events, n_tracks=n_tracks, seed_layers=3)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    xyz, cov, layer, hoff = T(eb.xyz), T(eb.cov), T(eb.layer), T(eb.hit_offsets)
    binned = kf.hit_bin(w.geometry, w.cuts.n_phi_bins, w.cuts.n_z_bins, layer, xyz, cov, event_offsets=hoff)
    seeds = kf.kf_seed(w.geometry, eb.n_seeds, T(eb.seed_hits))
    return EventOnGPU(eb, binned, seeds, xyz, cov, hoff, T(eb.seed_event))


def build(w, e: EventOnGPU, window_mode=0, block=None, counters=False, arith=kf.ARITH_F32,
          state=kf.STATE_CARTESIAN):
    bp = kf.build_params(w.cuts, window_mode=window_mode, mlp_block=block, arith=arith, state=state)
    ex = kf.BuildExtra()
    ex.seed_event = e.sev.data_ptr()
    cnt = None
    if counters:
        cnt = torch.zeros(4, dtype=torch.int64, device=DEV)
        ex.counters = cnt.data_ptr()
    out = kf.kf_build(w.geometry, bp, e.binned, e.eb.n_seeds, e.seeds["par"], e.seeds["cov"], e.seeds["q"], extra=ex)
    return out, cnt


def efficiency(w, e: EventOnGPU, out) -> float:
    """Fraction of seeds whose best candidate carries >= 75 % of its track's
    hits on the searched layers."""
    F = w.cuts.first_layer
    n = e.eb.n_seeds
    hits = out["hits"].cpu().numpy()[:, :n]
    return float(np.mean((hits == e.eb.true_hits[F:, :n]).mean(axis=0) >= 0.75))


def lost_hits(w, e: EventOnGPU, out_plain, out_learned):
    """True hits on the plain build's best candidates that the learned
    build's best candidates miss: (count, fraction of the plain build's true
    hits)."""
    F = w.cuts.first_layer
    n = e.eb.n_seeds
    t = e.eb.true_hits[F:, :n]
    hp = out_plain["hits"].cpu().numpy()[:, :n]
    hl = out_learned["hits"].cpu().numpy()[:, :n]
    found_p = (hp == t) & (t >= 0)
    lost = int(np.sum(found_p & (hl != t)))
    return lost, lost / max(int(found_p.sum()), 1)


def dump_rows(w, e: EventOnGPU, capacity=3_000_000, state=kf.STATE_CARTESIAN) -> np.ndarray:
    """Training rows from the plain FP32 build in the given state (the
    features are the Cartesian prediction in either state)."""
    eb = e.eb
    L = w.geometry.n_layers
    n = eb.n_seeds
    # true hit positions per seed and layer
    txyz = np.zeros((L, 3, eb.ld), dtype=np.float32)
    for l in range(L):
        idx = eb.true_hits[l, :n].astype(np.int64) + eb.hit_offsets[eb.seed_event].astype(np.int64)
        txyz[l, :, :n] = eb.xyz[:, idx]
    th = torch.from_numpy(eb.true_hits).to(DEV)
    tx = torch.from_numpy(txyz).to(DEV)
    dump = torch.empty((capacity, kf.MLP_ROW), dtype=torch.float32, device=DEV)
    cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
    bp = kf.build_params(w.cuts, state=state)
    ex = kf.BuildExtra()
    ex.seed_event = e.sev.data_ptr()
    ex.true_hits = th.data_ptr()
    ex.true_xyz = tx.data_ptr()
    ex.dump = dump.data_ptr()
    ex.dump_count = cnt.data_ptr()
    ex.dump_capacity = capacity
    kf.kf_build(w.geometry, bp, e.binned, n, e.seeds["par"], e.seeds["cov"], e.seeds["q"], extra=ex)
    torch.cuda.synchronize()
    k = min(int(cnt.item()), capacity)
    rows = dump[:k].cpu().numpy()
    # a deterministic order (the dump order depends on scheduling): by the
    # row's (seed, layer, slot) word
    return rows[np.argsort(rows[:, 31].view(np.uint32), kind="stable")]


def row_ids(rows):
    """(seed, layer, slot) of dumped rows."""
    v = rows[:, 31].view(np.uint32)
    return (v >> 8).astype(np.int64), ((v >> 3) & 31).astype(np.int64), (v & 7).astype(np.int64)


def plain_widths(w, rows):
    """Plain half-widths (arc at the layer radius, z; cm) of dumped rows, as
    the builder formed them (it writes them into each row).  A nearly
    singular FP32 covariance can round H P H^T below zero, which gives the
    builder an undefined width, i.e. a window that admits no hit: those count
    as the narrowest window."""
    wr, wz = rows[:, 29].astype(np.float64), rows[:, 30].astype(np.float64)
    return np.where(np.isfinite(wr), wr, 0.0), np.where(np.isfinite(wz), wz, 0.0)


def gates(w, rows, quantile):
    """Gate half-widths (arc, z) at the given quantile of the rows' plain
    widths: the network is consulted where either plain width lies above its
    gate (quantile 0: nearly everywhere)."""
    wr, wz = plain_widths(w, rows)
    if quantile <= 0:
        return 0.0, 0.0
    return float(np.quantile(wr, quantile)), float(np.quantile(wz, quantile))


def init_master(rng):
    W1 = rng.normal(0, np.sqrt(2.0 / 27), (64, 27))
    W2 = rng.normal(0, np.sqrt(2.0 / 64), (64, 64))
    W3 = rng.normal(0, np.sqrt(1.0 / 64), (2, 64))
    p = {"W1": W1, "b1": np.zeros(64), "W2": W2, "b2": np.zeros(64), "W3": W3, "b3": np.zeros(2)}
    m = kf.mlp_join(p).astype(np.float32)
    # the master starts on BF16 values, so the working copy equals it
    return (kf._bf16_bits(m).astype(np.uint32) << 16).view(np.float32).copy()


def standardisation(rows):
    x = rows[:, :27].astype(np.float64)
    mu = x.mean(axis=0)
    sd = x.std(axis=0)
    sd[sd <= 0] = 1.0
    return mu.astype(np.float32), sd.astype(np.float32)


@dataclass
class Trained:
    master: torch.Tensor
    block: torch.Tensor
    mu: np.ndarray
    sd: np.ndarray
    losses: list      # mean training loss of each epoch
    seconds: float
    steps: int
    loss0: float = 0.0  # mean loss of the initial network over the first batches
    gates: tuple = (0.0, 0.0)  # plain half-widths (arc, z) above which the network is consulted
    rows_used: int = 0


def train(rows: np.ndarray, epochs=4, batch=4096, lr=1e-3, seed=1711065715, log=None) -> Trained:
    rng = np.random.default_rng(seed)
    mu, sd = standardisation(rows)
    master_np = init_master(rng)
    block = kf.mlp_block(master_np, mu, sd, SCALE, kappa=1.0, floor_rphi=FLOOR[0], floor_z=FLOOR[1])
    master = torch.from_numpy(master_np).to(DEV)
    m = torch.zeros_like(master)
    v = torch.zeros_like(master)
    data = torch.from_numpy(np.ascontiguousarray(rows)).to(DEV)
    n = data.shape[0]
    grad = torch.empty(kf.MLP_NPARAM + 1, dtype=torch.float32, device=DEV)
    ws = torch.empty(int(kf.lib().kf_mlp_grad_workspace_bytes(batch)) // 4 + 1, dtype=torch.float32, device=DEV)
    gen = torch.Generator(device=DEV)
    gen.manual_seed(seed)
    losses = []
    step = 0
    # loss of the initial network (gradients computed, no step taken)
    acc0 = torch.zeros((), dtype=torch.float32, device=DEV)
    nb0 = max(1, min(16, n // batch))
    for b in range(nb0):
        kf.kf_mlp_grad(block, data[b * batch:(b + 1) * batch], grad=grad, ws=ws)
        acc0 += grad[-1]
    loss0 = float(acc0.item()) / nb0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen, device=DEV)
        shuf = data[perm]
        acc = torch.zeros((), dtype=torch.float32, device=DEV)
        nb = n // batch
        for b in range(nb):
            chunk = shuf[b * batch:(b + 1) * batch]
            kf.kf_mlp_grad(block, chunk, grad=grad, ws=ws)
            step += 1
            kf.kf_mlp_adam(block, master, m, v, grad, step, lr=lr)
            acc += grad[-1]
        losses.append(float(acc.item()) / max(nb, 1))
        if log:
            log(f"epoch {ep} loss {losses[-1]:.5f}")
    torch.cuda.synchronize()
    return Trained(master, block, mu, sd, losses, time.perf_counter() - t0, step, loss0, (0.0, 0.0), n)


def train_gated(w, rows: np.ndarray, quantile=GATE_QUANTILE, epochs=4, **kw) -> Trained:
    """Gates at `quantile` of the rows' plain widths, then training on the
    rows the gates pass (the population the network will see), for as many
    optimiser steps as `epochs` over all rows would take."""
    gr, gz = gates(w, rows, quantile)
    wr, wz = plain_widths(w, rows)
    sel = (wr > gr) | (wz > gz)
    n_sel = max(int(sel.sum()), 1)
    t = train(rows[sel], epochs=max(epochs, int(round(epochs * rows.shape[0] / n_sel))), **kw)
    kf.mlp_set_header(t.block, gate_rphi=gr, gate_z=gz)
    t.gates = (gr, gz)
    return t


def calibrate(w, t: Trained, val: EventOnGPU, eff_plain: float, target=0.001, kappas=None, arith=kf.ARITH_F32,
              state=kf.STATE_CARTESIAN):
    """Smallest kappa whose efficiency on the validation events is within
    `target` of the plain window's."""
    kappas = kappas or KAPPAS
    res = []
    for kap in kappas:
        kf.mlp_set_header(t.block, kappa=kap)
        out, _ = build(w, val, window_mode=1, block=t.block, arith=arith, state=state)
        torch.cuda.synchronize()
        eff = efficiency(w, val, out)
        res.append((kap, eff))
        if eff_plain - eff <= target:
            return kap, res
    return kappas[-1], res


def time_build(w, e: EventOnGPU, window_mode, block=None, reps=5, arith=kf.ARITH_F32, state=kf.STATE_CARTESIAN):
    build(w, e, window_mode, block, arith=arith, state=state)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        build(w, e, window_mode, block, arith=arith, state=state)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))
