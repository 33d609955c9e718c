"""Seeded synthetic event generator (ctypes binding of kfgen.c).

Input generation only: it simulates particles and hits and holds none of
the reconstruction arithmetic.  The GPU library and the oracle both consume
what it produces.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from ..presets import Geometry, GenSettings

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kfgen.c")
_LIB = os.path.join(_HERE, "libkfgen.so")


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("n_layers", ctypes.c_int32), ("smear", ctypes.c_int32), ("r", ctypes.c_double * 32),
        ("z_half", ctypes.c_double), ("bz", ctypes.c_double), ("x_over_x0", ctypes.c_double),
        ("mass", ctypes.c_double), ("sig_rphi", ctypes.c_double), ("sig_z", ctypes.c_double),
        ("pt_min", ctypes.c_double), ("pt_max", ctypes.c_double), ("eta_max", ctypes.c_double),
        ("vtx_sxy", ctypes.c_double), ("vtx_sz", ctypes.c_double), ("noise_lo", ctypes.c_double),
        ("noise_hi", ctypes.c_double), ("seed", ctypes.c_uint64),
    ]


class _DetCfg(ctypes.Structure):
    _fields_ = [
        ("n_layers", ctypes.c_int32), ("smear", ctypes.c_int32), ("kind", ctypes.c_int32 * 32),
        ("pos", ctypes.c_double * 32), ("lo", ctypes.c_double * 32), ("hi", ctypes.c_double * 32),
        ("dmod", ctypes.c_double * 32), ("n_mod", ctypes.c_int32), ("n_seed_layers", ctypes.c_int32),
        ("bz", ctypes.c_double), ("x_over_x0", ctypes.c_double), ("mass", ctypes.c_double),
        ("sig_rphi", ctypes.c_double), ("sig_w", ctypes.c_double), ("pt_min", ctypes.c_double),
        ("pt_max", ctypes.c_double), ("eta_max", ctypes.c_double), ("vtx_sxy", ctypes.c_double),
        ("vtx_sz", ctypes.c_double), ("noise_lo", ctypes.c_double), ("noise_hi", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


def build_lib() -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError(f"{_LIB} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.kfg_event.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_uint64, ctypes.c_int32] + [P] * 11 + [ctypes.c_int64]
        L.kfg_event.restype = ctypes.c_int
        L.kfg_layer_counts.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_uint64, ctypes.c_int32, P]
        L.kfg_layer_counts.restype = ctypes.c_int
        L.kfg_event_tracks.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32]
        L.kfg_event_tracks.restype = ctypes.c_int32
        L.kfg_philox4x32_10.argtypes = [P, P, P]
        L.kfg_philox4x32_10.restype = None
        L.kfg_splitmix64.argtypes = [ctypes.c_uint64]
        L.kfg_splitmix64.restype = ctypes.c_uint64
        L.kfg_det_event.argtypes = [ctypes.POINTER(_DetCfg), ctypes.c_uint64, ctypes.c_int32] + [P] * 10 + [
            ctypes.c_int64, P]
        L.kfg_det_event.restype = ctypes.c_int
        _lib = L
    return _lib


def _cfg(geom: Geometry, gen: GenSettings, x_over_x0=None) -> _Cfg:
    c = _Cfg()
    c.n_layers = geom.n_layers
    c.smear = 1 if gen.smear else 0
    for i, v in enumerate(geom.r):
        c.r[i] = v
    c.z_half = geom.z_half
    c.bz = geom.bz
    c.x_over_x0 = geom.x_over_x0 if x_over_x0 is None else x_over_x0
    c.mass = geom.mass
    c.sig_rphi, c.sig_z = gen.sig_rphi, gen.sig_z
    c.pt_min, c.pt_max, c.eta_max = gen.pt_min, gen.pt_max, gen.eta_max
    c.vtx_sxy, c.vtx_sz = gen.vtx_sxy, gen.vtx_sz
    c.noise_lo, c.noise_hi = gen.noise_lo, gen.noise_hi
    c.seed = gen.seed & 0xFFFFFFFFFFFFFFFF
    return c


@dataclass
class Event:
    """One generated event.  Hits are grouped by layer and shuffled within a
    layer; a hit's position in these arrays is its original index."""
    xyz: np.ndarray        # (3, n_hits) float64
    cov: np.ndarray        # (6, n_hits) float64: xx, xy, xz, yy, yz, zz
    layer: np.ndarray      # (n_hits,) int32
    track: np.ndarray      # (n_hits,) int32, -1 for noise
    trk_hits: np.ndarray   # (L, n_tracks) int32 original index of each track's hit
    q: np.ndarray          # (n_tracks,) int8
    truth: np.ndarray | None  # (L, 6, n_tracks) float64 state leaving each layer
    vertex: np.ndarray | None  # (6, n_tracks) float64 production state

    @property
    def n_hits(self) -> int:
        return self.xyz.shape[1]

    @property
    def n_tracks(self) -> int:
        return self.q.shape[0]


def event_tracks(gen: GenSettings, event: int, lo: int, hi: int) -> int:
    return int(lib().kfg_event_tracks(gen.seed, event, lo, hi))


def generate(geom: Geometry, gen: GenSettings, event: int, n_tracks: int, truth: bool = False,
             x_over_x0=None) -> Event:
    L = lib()
    cfg = _cfg(geom, gen, x_over_x0)
    counts = np.zeros(32, dtype=np.int64)
    if L.kfg_layer_counts(ctypes.byref(cfg), event, n_tracks, counts.ctypes.data):
        raise ValueError("bad generator configuration")
    nh = int(counts[: geom.n_layers].sum())
    hx = np.zeros(nh)
    hy = np.zeros(nh)
    hz = np.zeros(nh)
    hcov = np.zeros((6, nh))
    hl = np.zeros(nh, dtype=np.int32)
    ht = np.zeros(nh, dtype=np.int32)
    th = np.zeros((geom.n_layers, n_tracks), dtype=np.int32)
    q = np.zeros(n_tracks, dtype=np.int8)
    tr = np.zeros((geom.n_layers, 6, n_tracks)) if truth else None
    vt = np.zeros((6, n_tracks)) if truth else None
    rc = L.kfg_event(ctypes.byref(cfg), event, n_tracks, hx.ctypes.data, hy.ctypes.data, hz.ctypes.data,
                     hcov.ctypes.data, hl.ctypes.data, ht.ctypes.data, th.ctypes.data, q.ctypes.data,
                     tr.ctypes.data if tr is not None else None, vt.ctypes.data if vt is not None else None,
                     None, nh)
    if rc:
        raise RuntimeError(f"kfg_event failed with code {rc}")
    return Event(np.stack([hx, hy, hz]), hcov, hl, ht, th, q, tr, vt)


def padded(n: int, mult: int = 64) -> int:
    return max(mult, ((n + mult - 1) // mult) * mult)


def track_hits(ev: Event, ld: int | None = None, dtype=np.float32) -> np.ndarray:
    """Per-track hit rows in the fit layout [L][9][ld]: x, y, z, then the six
    covariance entries, for each track's own hit on each layer."""
    L, n = ev.trk_hits.shape
    ld = padded(n) if ld is None else ld
    out = np.zeros((L, 9, ld), dtype=dtype)
    for l in range(L):
        idx = ev.trk_hits[l]
        out[l, 0:3, :n] = ev.xyz[:, idx]
        out[l, 3:9, :n] = ev.cov[:, idx]
    return out


# ------------------------------------------------------------ general detector

def _det_cfg(det, gen: GenSettings, x_over_x0=None) -> _DetCfg:
    c = _DetCfg()
    c.n_layers = det.n_layers
    c.smear = 1 if gen.smear else 0
    for i in range(det.n_layers):
        c.kind[i] = det.kind[i]
        c.pos[i], c.lo[i], c.hi[i], c.dmod[i] = det.pos[i], det.lo[i], det.hi[i], det.dmod[i]
    c.n_mod = det.n_mod
    c.n_seed_layers = det.n_seed_layers
    c.bz, c.mass = det.bz, det.mass
    c.x_over_x0 = det.x_over_x0 if x_over_x0 is None else x_over_x0
    c.sig_rphi, c.sig_w = gen.sig_rphi, gen.sig_z
    c.pt_min, c.pt_max, c.eta_max = gen.pt_min, gen.pt_max, gen.eta_max
    c.vtx_sxy, c.vtx_sz = gen.vtx_sxy, gen.vtx_sz
    c.noise_lo, c.noise_hi = gen.noise_lo, gen.noise_hi
    c.seed = gen.seed & 0xFFFFFFFFFFFFFFFF
    return c


def generate_det(det, gen: GenSettings, event: int, n_tracks: int, truth: bool = False, x_over_x0=None) -> Event:
    """One event over a general detector (barrel cylinders and disks).  A
    track's hit index on a layer it does not cross is -1 (trk_hits); truth is
    NaN there."""
    L = lib()
    cfg = _det_cfg(det, gen, x_over_x0)
    nl = det.n_layers
    cap = int(nl * n_tracks * (1.0 + max(gen.noise_hi, gen.noise_lo)) + nl + 16)
    hx, hy, hz = np.zeros(cap), np.zeros(cap), np.zeros(cap)
    hcov = np.zeros((6, cap))
    hl = np.zeros(cap, dtype=np.int32)
    ht = np.zeros(cap, dtype=np.int32)
    th = np.zeros((nl, n_tracks), dtype=np.int32)
    q = np.zeros(n_tracks, dtype=np.int8)
    tr = np.zeros((nl, 6, n_tracks)) if truth else None
    vt = np.zeros((6, n_tracks)) if truth else None
    nh = ctypes.c_int64(0)
    rc = L.kfg_det_event(ctypes.byref(cfg), event, n_tracks, hx.ctypes.data, hy.ctypes.data, hz.ctypes.data,
                         hcov.ctypes.data, hl.ctypes.data, ht.ctypes.data, th.ctypes.data, q.ctypes.data,
                         tr.ctypes.data if tr is not None else None, vt.ctypes.data if vt is not None else None,
                         cap, ctypes.byref(nh))
    if rc:
        raise RuntimeError(f"kfg_det_event failed with code {rc}")
    n = int(nh.value)
    return Event(np.stack([hx[:n], hy[:n], hz[:n]]), np.ascontiguousarray(hcov[:, :n]), hl[:n].copy(), ht[:n].copy(),
                 th, q, tr, vt)


def det_track_rows(ev: Event, ld: int | None = None, dtype=np.float32):
    """Per-track hit rows [L][9][ld] over a general detector (zeros where the
    track does not cross a layer) and the visit masks [ld] (bit l: the track
    has a hit on layer l)."""
    L, n = ev.trk_hits.shape
    ld = padded(n) if ld is None else ld
    out = np.zeros((L, 9, ld), dtype=dtype)
    visit = np.zeros(ld, dtype=np.uint32)
    for l in range(L):
        idx = ev.trk_hits[l]
        have = idx >= 0
        cols = np.where(have)[0]
        out[l, 0:3, cols] = ev.xyz[:, idx[have]].T
        out[l, 3:9, cols] = ev.cov[:, idx[have]].T
        visit[:n] |= np.where(have, np.uint32(1 << l), np.uint32(0)).astype(np.uint32)
    return out, visit
