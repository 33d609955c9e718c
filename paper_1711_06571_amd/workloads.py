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


def event_batch(w: Workload, events, n_tracks=None) -> EventBatch:
    events = list(events)
    evs = []
    for e in events:
        T = n_tracks if n_tracks is not None else (
            w.n_tracks if w.tracks_hi == 0 else datagen.event_tracks(w.gen, e, w.tracks_lo, w.tracks_hi))
        evs.append(datagen.generate(w.geometry, w.gen, e, T))
    L = w.geometry.n_layers
    nh = [ev.n_hits for ev in evs]
    ns = [ev.n_tracks for ev in evs]
    hoff = np.concatenate([[0], np.cumsum(nh)]).astype(np.int64)
    soff = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    if hoff[-1] >= 2 ** 31:
        raise ValueError("too many hits for int32 offsets")
    n_seeds = int(soff[-1])
    ld = datagen.padded(n_seeds)
    xyz = np.concatenate([ev.xyz for ev in evs], axis=1).astype(np.float32)
    cov = np.concatenate([ev.cov for ev in evs], axis=1).astype(np.float32)
    layer = np.concatenate([ev.layer for ev in evs]).astype(np.int32)
    trk = np.concatenate([ev.track for ev in evs]).astype(np.int32)
    H = np.zeros((L, 9, ld), dtype=np.float32)
    TH = np.full((L, ld), -1, dtype=np.int32)
    sev = np.zeros(n_seeds, dtype=np.int32)
    for k, ev in enumerate(evs):
        sl = slice(soff[k], soff[k + 1])
        for l in range(L):
            idx = ev.trk_hits[l]
            H[l, 0:3, sl] = ev.xyz[:, idx]
            H[l, 3:9, sl] = ev.cov[:, idx]
            TH[l, sl] = idx
        sev[sl] = k
    return EventBatch(xyz, cov, layer, hoff.astype(np.int32), H, TH, sev, soff.astype(np.int32), n_seeds, ld, trk)
