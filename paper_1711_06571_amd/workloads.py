"""Assemble the synthetic inputs of each workload in the layouts the library
takes.  Input generation only (the seeded generator plus array plumbing)."""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import datagen
from .presets import Workload


@dataclass
class FitBatch:
    hits: np.ndarray      # [L][9][ld] float32, per track
    n: int                # tracks
    event_of: np.ndarray  # [n] event index
    ld: int


def fit_batch(w: Workload, n_events: int | None = None, n_tracks: int | None = None) -> FitBatch:
    """All events of a fit workload flattened into one track axis."""
    E = w.n_events if n_events is None else n_events
    T = w.n_tracks if n_tracks is None else n_tracks
    n = E * T
    ld = datagen.padded(n)
    L = w.geometry.n_layers
    H = np.zeros((L, 9, ld), dtype=np.float32)
    ev_of = np.zeros(n, dtype=np.int32)
    for e in range(E):
        ev = datagen.generate(w.geometry, w.gen, e, T)
        sl = slice(e * T, (e + 1) * T)
        for l in range(L):
            idx = ev.trk_hits[l]
            H[l, 0:3, sl] = ev.xyz[:, idx]
            H[l, 3:9, sl] = ev.cov[:, idx]
        ev_of[sl] = e
    return FitBatch(H, n, ev_of, ld)


@dataclass
class EventBatch:
    """Several events concatenated for hit_bin / kf_build."""
    xyz: np.ndarray          # [3][n_hits] float32
    cov: np.ndarray          # [6][n_hits] float32
    layer: np.ndarray        # [n_hits] int32
    hit_offsets: np.ndarray  # [E+1] int32
    seed_hits: np.ndarray    # [L][9][ld] float32 per seed (true hits; seeds use layers 0..2)
    true_hits: np.ndarray    # [L][ld] int32 event-local original index of each seed's true hit
    seed_event: np.ndarray   # [n_seeds] int32
    seed_offsets: np.ndarray  # [E+1]
    n_seeds: int
    ld: int
    track_of_hit: np.ndarray  # [n_hits] int32 (-1 noise), event-local track index


def _event_tracks(w: Workload, e: int, n_tracks=None) -> int:
    if n_tracks is not None:
        return n_tracks
    return w.n_tracks if w.tracks_hi == 0 else datagen.event_tracks(w.gen, e, w.tracks_lo, w.tracks_hi)


def event_batch(w: Workload, events, n_tracks=None, seed_layers=None) -> EventBatch:
    """Generate events into concatenated FP32 arrays, one event at a time.
    seed_hits keeps the first `seed_layers` layers of each track's hits (all
    layers by default)."""
    import ctypes
    events = list(events)
    L = w.geometry.n_layers
    SL = L if seed_layers is None else seed_layers
    nts = [_event_tracks(w, e, n_tracks) for e in events]
    cfg = datagen._cfg(w.geometry, w.gen)
    nh = []
    cnt = np.zeros(32, dtype=np.int64)
    for e, T in zip(events, nts):
        datagen.lib().kfg_layer_counts(ctypes.byref(cfg), e, T, cnt.ctypes.data)
        nh.append(int(cnt[:L].sum()))
    hoff = np.concatenate([[0], np.cumsum(nh)]).astype(np.int64)
    soff = np.concatenate([[0], np.cumsum(nts)]).astype(np.int64)
    if hoff[-1] >= 2 ** 31:
        raise ValueError("too many hits for int32 offsets")
    n_seeds = int(soff[-1])
    ld = datagen.padded(n_seeds)
    xyz = np.zeros((3, hoff[-1]), dtype=np.float32)
    cov = np.zeros((6, hoff[-1]), dtype=np.float32)
    layer = np.zeros(hoff[-1], dtype=np.int32)
    trk = np.zeros(hoff[-1], dtype=np.int32)
    H = np.zeros((SL, 9, ld), dtype=np.float32)
    TH = np.full((L, ld), -1, dtype=np.int32)
    sev = np.zeros(n_seeds, dtype=np.int32)
    for k, (e, T) in enumerate(zip(events, nts)):
        ev = datagen.generate(w.geometry, w.gen, e, T)
        hs = slice(hoff[k], hoff[k + 1])
        xyz[:, hs] = ev.xyz
        cov[:, hs] = ev.cov
        layer[hs] = ev.layer
        trk[hs] = ev.track
        sl = slice(soff[k], soff[k + 1])
        for l in range(L):
            idx = ev.trk_hits[l]
            if l < SL:
                H[l, 0:3, sl] = ev.xyz[:, idx]
                H[l, 3:9, sl] = ev.cov[:, idx]
            TH[l, sl] = idx
        sev[sl] = k
        del ev
    return EventBatch(xyz, cov, layer, hoff.astype(np.int32), H, TH, sev, soff.astype(np.int32), n_seeds, ld, trk)


@dataclass
class DetEventBatch:
    """Several events of a general detector concatenated for hit_bin_det /
    kf_build_det, with the per-track rows the fit takes."""
    xyz: np.ndarray          # [3][n_hits] float32
    cov: np.ndarray          # [6][n_hits] float32
    layer: np.ndarray        # [n_hits] int32
    hit_offsets: np.ndarray  # [E+1] int32
    track_rows: np.ndarray   # [L][9][ld] float32 each track's hits (zeros where it crosses no module)
    visit: np.ndarray        # [ld] uint32 layers each track has a hit on
    true_hits: np.ndarray    # [L][ld] int32 event-local original index of each track's hit (-1 none)
    seed_event: np.ndarray   # [n_seeds] int32
    seed_offsets: np.ndarray  # [E+1] int32
    n_seeds: int
    ld: int


def det_event_batch(w, events, n_tracks=None) -> DetEventBatch:
    """Generate events of a general-detector workload into concatenated FP32
    arrays (one event at a time)."""
    events = list(events)
    T = w.n_tracks if n_tracks is None else n_tracks
    L = w.detector.n_layers
    evs = [datagen.generate_det(w.detector, w.gen, e, T) for e in events]
    hoff = np.concatenate([[0], np.cumsum([ev.n_hits for ev in evs])]).astype(np.int64)
    soff = np.concatenate([[0], np.cumsum([ev.n_tracks for ev in evs])]).astype(np.int64)
    if hoff[-1] >= 2 ** 31:
        raise ValueError("too many hits for int32 offsets")
    n_seeds = int(soff[-1])
    ld = datagen.padded(n_seeds)
    xyz = np.concatenate([ev.xyz for ev in evs], axis=1).astype(np.float32)
    cov = np.concatenate([ev.cov for ev in evs], axis=1).astype(np.float32)
    layer = np.concatenate([ev.layer for ev in evs]).astype(np.int32)
    rows = np.zeros((L, 9, ld), dtype=np.float32)
    visit = np.zeros(ld, dtype=np.uint32)
    TH = np.full((L, ld), -1, dtype=np.int32)
    sev = np.zeros(n_seeds, dtype=np.int32)
    for k, ev in enumerate(evs):
        sl = slice(soff[k], soff[k + 1])
        r, v = datagen.det_track_rows(ev)
        rows[:, :, sl] = r[:, :, :ev.n_tracks]
        visit[sl] = v[:ev.n_tracks]
        TH[:, sl] = ev.trk_hits
        sev[sl] = k
    return DetEventBatch(np.ascontiguousarray(xyz), np.ascontiguousarray(cov), layer, hoff.astype(np.int32), rows,
                         visit, TH, sev, soff.astype(np.int32), n_seeds, ld)
