"""Python binding of libkftrack (ctypes).  Argument marshalling only: every
step runs in the library's HIP kernels.  Tensors are torch CUDA (HIP)
tensors; calls are enqueued on torch's current stream unless one is given.

The library must be built (see build_lib.py); importing this module on a
machine without it raises immediately instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkftrack.so")

KF_OK = 0
KF_E_INVALID_ARG = 1
KF_E_WORKSPACE = 2
KF_E_HIP = 3
KF_E_UNSUPPORTED = 4

ARITH_F32 = 0
ARITH_F64 = 1

TRK_NO_CROSSING = 1
TRK_OUT_OF_Z = 2
TRK_NONFINITE = 4
TRK_S_NOT_PD = 8
TRK_CAP_TRUNC = 16
TRK_EVENT_TOO_LARGE = 32


class Geometry(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("r", ctypes.c_float * 32), ("z_half", ctypes.c_float),
                ("bz", ctypes.c_float), ("x_over_x0", ctypes.c_float), ("mass", ctypes.c_float)]


class Hits(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_int32), ("n_layers", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("n_z", ctypes.c_int32), ("n_hits", ctypes.c_int32), ("offsets", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p), ("phi", ctypes.c_void_p),
                ("cov", ctypes.c_void_p), ("orig", ctypes.c_void_p)]


class BuildParams(ctypes.Structure):
    _fields_ = [("chi2_cut", ctypes.c_float), ("max_holes", ctypes.c_int32), ("cand_cap", ctypes.c_int32),
                ("nsigma", ctypes.c_float), ("win_sig_rphi", ctypes.c_float), ("win_sig_z", ctypes.c_float),
                ("first_layer", ctypes.c_int32), ("window_mode", ctypes.c_int32), ("mlp", ctypes.c_void_p),
                ("lanes_per_block", ctypes.c_int32), ("persistent_blocks", ctypes.c_int32),
                ("arith", ctypes.c_int32), ("phi_refine", ctypes.c_int32), ("state", ctypes.c_int32)]


class Detector(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("kind", ctypes.c_int32 * 32), ("pos", ctypes.c_float * 32),
                ("lo", ctypes.c_float * 32), ("hi", ctypes.c_float * 32), ("dmod", ctypes.c_float * 32),
                ("bz", ctypes.c_float), ("x_over_x0", ctypes.c_float), ("mass", ctypes.c_float)]


LAYER_BARREL = 0
LAYER_DISK = 1


class LaunchInfo(ctypes.Structure):
    _fields_ = [("lanes_per_block", ctypes.c_int32), ("blocks", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("resident_blocks_per_cu", ctypes.c_int32), ("max_lds_per_block", ctypes.c_int32)]


class FitStage(ctypes.Structure):
    _fields_ = [("arith", ctypes.c_int32), ("fit_hits", ctypes.c_void_p), ("hole_mask", ctypes.c_void_p),
                ("out_par", ctypes.c_void_p), ("out_cov", ctypes.c_void_p), ("out_chi2", ctypes.c_void_p),
                ("out_ndof", ctypes.c_void_p), ("out_status", ctypes.c_void_p)]


class BuildExtra(ctypes.Structure):
    _fields_ = [("seed_event", ctypes.c_void_p), ("seed_order", ctypes.c_void_p),
                ("event_n_seeds", ctypes.c_void_p), ("event_done_ticks", ctypes.c_void_p),
                ("start_tick", ctypes.c_void_p), ("true_hits", ctypes.c_void_p), ("true_xyz", ctypes.c_void_p),
                ("dump", ctypes.c_void_p),
                ("dump_count", ctypes.c_void_p), ("dump_capacity", ctypes.c_int32), ("counters", ctypes.c_void_p)]


class KFError(RuntimeError):
    pass


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise KFError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int32
        L.kf_status_string.restype = ctypes.c_char_p
        L.kf_status_string.argtypes = [ctypes.c_int]
        L.kf_last_error.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
        L.kf_seed.argtypes = [ctypes.POINTER(Geometry), I, I, P, ctypes.c_float, P, P, P, P, P]
        L.kf_fit.argtypes = [ctypes.POINTER(Geometry), I, I, I, P, P, P, P, P, P, P, P, P, P, I, P]
        L.kf_fit_hybrid.argtypes = L.kf_fit.argtypes
        L.hit_bin_workspace_bytes.restype = ctypes.c_size_t
        L.hit_bin_workspace_bytes.argtypes = [I, I, I, I, I]
        L.hit_bin.argtypes = [ctypes.POINTER(Geometry), I, P, I, I, I, P, P, P, P, P, P, P, P, P,
                              ctypes.c_size_t, P]
        L.kf_gather_hits.argtypes = [I, I, I, I, P, P, I, P, I, P, P, P, P, P]
        L.kf_batch_plan_create.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(BuildParams), I, P, I, P, P, P,
                                           ctypes.POINTER(Hits), P, P, P, P, P, ctypes.c_size_t, I, I, P, P, P, P, P,
                                           P, P, P, P, ctypes.POINTER(BuildExtra), P, ctypes.c_size_t, P,
                                           ctypes.POINTER(ctypes.c_void_p)]
        L.kf_step_plan_create.argtypes = list(L.kf_batch_plan_create.argtypes[:-2]) + [
            ctypes.POINTER(FitStage), P, ctypes.POINTER(ctypes.c_void_p)]
        L.kf_batch_plan_launch.argtypes = [P, P]
        L.kf_batch_plan_destroy.argtypes = [P]
        L.kf_wall_clock_khz.argtypes = [P]
        L.kf_mlp_block_bytes.restype = ctypes.c_size_t
        L.kf_mlp_grad_workspace_bytes.restype = ctypes.c_size_t
        L.kf_mlp_grad_workspace_bytes.argtypes = [I]
        L.kf_mlp_forward.argtypes = [P, I, P, P, P, P]
        L.kf_mlp_grad.argtypes = [P, I, P, P, P, ctypes.c_size_t, P]
        L.kf_mlp_adam.argtypes = [P, P, P, P, P, I, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, P]
        L.kf_build_workspace_bytes.restype = ctypes.c_size_t
        L.kf_build_workspace_bytes.argtypes = [ctypes.POINTER(BuildParams), ctypes.POINTER(Hits), I]
        L.kf_build.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(BuildParams), ctypes.POINTER(Hits), I,
                               I, P, P, P, P, P, P, P, P, P, ctypes.POINTER(BuildExtra), P, ctypes.c_size_t, P]
        L.kf_build_noalloc.argtypes = list(L.kf_build.argtypes[:15]) + [P]
        L.kf_build_noalloc_max_bytes.restype = ctypes.c_size_t
        L.kf_build_noalloc_max_bytes.argtypes = []
        L.kf_peak_fma.argtypes = [I, I, I, P, P]
        L.hit_bin_det.argtypes = [ctypes.POINTER(Detector)] + list(L.hit_bin.argtypes[1:])
        L.kf_fit_det.argtypes = [ctypes.POINTER(Detector), I, I, I, P, P, P, P, P, P, P, P, P, P, P, I, P]
        L.kf_build_det.argtypes = [ctypes.POINTER(Detector), ctypes.POINTER(BuildParams), ctypes.POINTER(Hits), I,
                                   I, P, P, P, P, P, P, P, P, P, P, ctypes.POINTER(BuildExtra), P, ctypes.c_size_t,
                                   P]
        _lib = L
    return _lib


def exported_symbols():
    return lib()


def _check(rc):
    if rc != KF_OK:
        msg = lib().kf_status_string(rc).decode()
        if rc == KF_E_HIP:
            buf = ctypes.create_string_buffer(512)
            lib().kf_last_error(buf, 512)
            msg += ": " + buf.value.decode()
        raise KFError(f"libkftrack status {rc}: {msg}")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise KFError("tensors passed to libkftrack must live on the GPU")
    if not t.is_contiguous():
        raise KFError("tensors passed to libkftrack must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def geometry(g) -> Geometry:
    """From a presets.Geometry."""
    o = Geometry()
    o.n_layers = g.n_layers
    for i, v in enumerate(g.r):
        o.r[i] = v
    o.z_half, o.bz, o.x_over_x0, o.mass = g.z_half, g.bz, g.x_over_x0, g.mass
    return o


def kf_seed(g, n, hits, beam_sigma=None, stream=None):
    """hits: [L][9][ld] float32 -> dict(q, par [6][ld], cov [21][ld], status).
    beam_sigma: beam-spot width (cm) of the seed convention, default the
    geometry's; 0 seeds from the three hits alone."""
    bs = float(getattr(g, "beam_sigma", 0.0)) if beam_sigma is None else float(beam_sigma)
    ld = hits.shape[2]
    dev = hits.device
    out = dict(q=torch.zeros(ld, dtype=torch.int8, device=dev),
               par=torch.zeros((6, ld), dtype=torch.float32, device=dev),
               cov=torch.zeros((21, ld), dtype=torch.float32, device=dev),
               status=torch.zeros(ld, dtype=torch.int32, device=dev))
    gg = geometry(g)
    _check(lib().kf_seed(ctypes.byref(gg), n, ld, _ptr(hits), ctypes.c_float(bs), _ptr(out["q"]), _ptr(out["par"]),
                         _ptr(out["cov"]), _ptr(out["status"]), _stream(stream)))
    return out


def _fit(fn, g, n, first_layer, hits, seed_par, seed_cov, q, hole_mask, out, arith, stream):
    ld = hits.shape[2]
    dev = hits.device
    if out is None:
        out = dict(par=torch.empty((6, ld), dtype=torch.float32, device=dev),
                   cov=torch.empty((21, ld), dtype=torch.float32, device=dev),
                   chi2=torch.empty(ld, dtype=torch.float32, device=dev),
                   ndof=torch.empty(ld, dtype=torch.int32, device=dev),
                   status=torch.empty(ld, dtype=torch.int32, device=dev))
    gg = geometry(g)
    _check(fn(ctypes.byref(gg), n, ld, first_layer, _ptr(hits), _ptr(hole_mask), _ptr(seed_par), _ptr(seed_cov),
              _ptr(q), _ptr(out["par"]), _ptr(out["cov"]), _ptr(out["chi2"]), _ptr(out["ndof"]),
              _ptr(out["status"]), arith, _stream(stream)))
    return out


def kf_fit(g, n, first_layer, hits, seed_par, seed_cov, q, hole_mask=None, out=None, arith=ARITH_F32, stream=None):
    return _fit(lib().kf_fit, g, n, first_layer, hits, seed_par, seed_cov, q, hole_mask, out, arith, stream)


def kf_fit_hybrid(g, n, first_layer, hits, seed_par, seed_cov, q, hole_mask=None, out=None, arith=ARITH_F32,
                  stream=None):
    """Fit in the hybrid state; outputs (x, y, z, q/pT, phi, theta) and their
    covariance."""
    return _fit(lib().kf_fit_hybrid, g, n, first_layer, hits, seed_par, seed_cov, q, hole_mask, out, arith, stream)


# ----------------------------------------------------------------- binning

class BinnedHits:
    """Device buffers produced by hit_bin (the kf_hits descriptor)."""

    def __init__(self, n_events, n_layers, n_phi, n_z, n_hits, device):
        nb = n_phi * n_z
        self.n_events, self.n_layers, self.n_phi, self.n_z, self.n_hits = n_events, n_layers, n_phi, n_z, n_hits
        self.offsets = torch.zeros((n_events, n_layers, nb + 1), dtype=torch.int32, device=device)
        self.xyzphi = torch.zeros((4, max(n_hits, 1)), dtype=torch.float32, device=device)
        self.cov = torch.zeros((6, max(n_hits, 1)), dtype=torch.float32, device=device)
        self.orig = torch.zeros(max(n_hits, 1), dtype=torch.int32, device=device)
        self.bad = torch.zeros(1, dtype=torch.int32, device=device)

    def descriptor(self) -> Hits:
        h = Hits()
        h.n_events, h.n_layers, h.n_phi, h.n_z, h.n_hits = (self.n_events, self.n_layers, self.n_phi, self.n_z,
                                                            self.n_hits)
        h.offsets = self.offsets.data_ptr()
        stride = self.xyzphi.shape[1] * 4
        base = self.xyzphi.data_ptr()
        h.x, h.y, h.z, h.phi = base, base + stride, base + 2 * stride, base + 3 * stride
        h.cov = self.cov.data_ptr()
        h.orig = self.orig.data_ptr()
        return h


def hit_bin_workspace_bytes(n_events, n_layers, n_phi, n_z, n_hits):
    return int(lib().hit_bin_workspace_bytes(n_events, n_layers, n_phi, n_z, n_hits))


def hit_bin(g, n_phi, n_z, layer, xyz, cov, event_offsets=None, out=None, ws=None, stream=None):
    """layer [n] int32, xyz [3][n], cov [6][n] float32 on the GPU; several
    events are concatenated and delimited by event_offsets [E+1] int32."""
    n = layer.shape[0]
    E = 1 if event_offsets is None else event_offsets.shape[0] - 1
    dev = layer.device
    if out is None:
        out = BinnedHits(E, g.n_layers, n_phi, n_z, n, dev)
    need = hit_bin_workspace_bytes(E, g.n_layers, n_phi, n_z, n)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    gg = geometry(g)
    _check(lib().hit_bin(ctypes.byref(gg), E, _ptr(event_offsets), n_phi, n_z, n, _ptr(layer), _ptr(xyz), _ptr(cov),
                         _ptr(out.offsets), _ptr(out.xyzphi), _ptr(out.cov), _ptr(out.orig), _ptr(out.bad),
                         _ptr(ws), ctypes.c_size_t(need), _stream(stream)))
    return out


# ------------------------------------------------------------------- build

STATE_CARTESIAN = 0
STATE_HYBRID = 1


# Launch parameters chosen by the autotuner (batch.autotune) per arithmetic,
# read once; a missing file means the library's defaults.
TUNE_CACHE = os.path.join(_HERE, "autotune.json")
_tune = None


def tuned_launch(arith):
    """The cached launch choice for kf_build in this arithmetic: dict with
    lanes_per_block, blocks_per_cu (0: as many as fit), phi_refine; or None."""
    global _tune
    if _tune is None:
        try:
            import json
            with open(TUNE_CACHE) as f:
                _tune = json.load(f)
        except (OSError, ValueError):
            _tune = {}
    return _tune.get("kf_build", {}).get("f64" if arith == ARITH_F64 else "f32")


def build_params(cuts, window_mode=0, mlp_block=None, lanes_per_block=0, persistent_blocks=0, cap=None,
                 arith=ARITH_F32, phi_refine=0, state=STATE_CARTESIAN, tuned=False):
    """kf_build_params from the cuts.  tuned=True fills the launch parameters
    left at 0 (lanes per block, persistent blocks, fine-index granularity)
    from the autotuner's cached choice for the arithmetic, if there is one."""
    if tuned and lanes_per_block == 0 and persistent_blocks == 0 and phi_refine == 0:
        t = tuned_launch(arith)
        if t:
            lanes_per_block = int(t["lanes_per_block"])
            cus = torch.cuda.get_device_properties(0).multi_processor_count
            persistent_blocks = int(t["blocks_per_cu"]) * cus
            phi_refine = int(t["phi_refine"])
    bp = BuildParams()
    bp.chi2_cut = cuts.chi2_cut
    bp.max_holes = cuts.max_holes
    bp.cand_cap = cuts.cand_cap if cap is None else cap
    bp.nsigma = cuts.nsigma
    bp.win_sig_rphi = cuts.win_sig_rphi
    bp.win_sig_z = cuts.win_sig_z
    bp.first_layer = cuts.first_layer
    bp.window_mode = window_mode
    bp.mlp = None if mlp_block is None else mlp_block.data_ptr()
    bp.lanes_per_block = lanes_per_block
    bp.persistent_blocks = persistent_blocks
    bp.arith = arith
    bp.phi_refine = phi_refine
    bp.state = state
    return bp


def kf_build_workspace_bytes(bp, binned: "BinnedHits", n_seeds):
    hd = binned.descriptor()
    return int(lib().kf_build_workspace_bytes(ctypes.byref(bp), ctypes.byref(hd), n_seeds))


def kf_build(g, bp, binned: BinnedHits, n_seeds, seed_par, seed_cov, q, extra=None, out=None, ws=None,
             stream=None):
    ld = seed_par.shape[1]
    dev = seed_par.device
    F = bp.first_layer
    if out is None:
        out = dict(hits=torch.empty((g.n_layers - F, ld), dtype=torch.int32, device=dev),
                   par=torch.empty((6, ld), dtype=torch.float32, device=dev),
                   cov=torch.empty((21, ld), dtype=torch.float32, device=dev),
                   chi2=torch.empty(ld, dtype=torch.float32, device=dev),
                   nhits=torch.empty(ld, dtype=torch.int32, device=dev),
                   status=torch.empty(ld, dtype=torch.int32, device=dev))
    need = kf_build_workspace_bytes(bp, binned, n_seeds)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    gg = geometry(g)
    hd = binned.descriptor()
    ex = extra if extra is not None else BuildExtra()
    _check(lib().kf_build(ctypes.byref(gg), ctypes.byref(bp), ctypes.byref(hd), n_seeds, ld, _ptr(seed_par),
                          _ptr(seed_cov), _ptr(q), _ptr(out["hits"]), _ptr(out["par"]), _ptr(out["cov"]),
                          _ptr(out["chi2"]), _ptr(out["nhits"]), _ptr(out["status"]), ctypes.byref(ex), _ptr(ws),
                          ctypes.c_size_t(need), _stream(stream)))
    return out


# ------------------------------------------------------- general detector

def detector(d) -> Detector:
    """From a presets.Detector (barrel cylinders and endcap disks)."""
    o = Detector()
    o.n_layers = d.n_layers
    for i in range(d.n_layers):
        o.kind[i] = d.kind[i]
        o.pos[i], o.lo[i], o.hi[i], o.dmod[i] = d.pos[i], d.lo[i], d.hi[i], d.dmod[i]
    o.bz, o.x_over_x0, o.mass = d.bz, d.x_over_x0, d.mass
    return o


def hit_bin_det(d, n_phi, n_w, layer, xyz, cov, event_offsets=None, out=None, ws=None, stream=None):
    """hit_bin over a general detector: rows in z on barrel layers, in r on
    disks (the descriptor's n_z is n_w)."""
    n = layer.shape[0]
    E = 1 if event_offsets is None else event_offsets.shape[0] - 1
    dev = layer.device
    if out is None:
        out = BinnedHits(E, d.n_layers, n_phi, n_w, n, dev)
    need = hit_bin_workspace_bytes(E, d.n_layers, n_phi, n_w, n)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    dd = detector(d)
    _check(lib().hit_bin_det(ctypes.byref(dd), E, _ptr(event_offsets), n_phi, n_w, n, _ptr(layer), _ptr(xyz),
                             _ptr(cov), _ptr(out.offsets), _ptr(out.xyzphi), _ptr(out.cov), _ptr(out.orig),
                             _ptr(out.bad), _ptr(ws), ctypes.c_size_t(need), _stream(stream)))
    return out


def kf_fit_det(d, n, first_layer, hits, visit, seed_par, seed_cov, q, hole_mask=None, out=None, arith=ARITH_F32,
               stream=None):
    """Fit over a general detector: hits [L][9][ld], visit [ld] (int32 view
    of the uint32 masks: bit l, the track crossed layer l)."""
    ld = hits.shape[2]
    dev = hits.device
    if out is None:
        out = dict(par=torch.empty((6, ld), dtype=torch.float32, device=dev),
                   cov=torch.empty((21, ld), dtype=torch.float32, device=dev),
                   chi2=torch.empty(ld, dtype=torch.float32, device=dev),
                   ndof=torch.empty(ld, dtype=torch.int32, device=dev),
                   status=torch.empty(ld, dtype=torch.int32, device=dev))
    dd = detector(d)
    _check(lib().kf_fit_det(ctypes.byref(dd), n, ld, first_layer, _ptr(hits), _ptr(visit), _ptr(hole_mask),
                            _ptr(seed_par), _ptr(seed_cov), _ptr(q), _ptr(out["par"]), _ptr(out["cov"]),
                            _ptr(out["chi2"]), _ptr(out["ndof"]), _ptr(out["status"]), arith, _stream(stream)))
    return out


def kf_build_det(d, bp, binned: BinnedHits, n_seeds, seed_par, seed_cov, q, extra=None, out=None, ws=None,
                 stream=None):
    """Two-step build over a general detector; outputs as kf_build plus
    visit [ld] (int32 view of the uint32 masks of visited layers)."""
    ld = seed_par.shape[1]
    dev = seed_par.device
    F = bp.first_layer
    if out is None:
        out = dict(hits=torch.empty((d.n_layers - F, ld), dtype=torch.int32, device=dev),
                   visit=torch.empty(ld, dtype=torch.int32, device=dev),
                   par=torch.empty((6, ld), dtype=torch.float32, device=dev),
                   cov=torch.empty((21, ld), dtype=torch.float32, device=dev),
                   chi2=torch.empty(ld, dtype=torch.float32, device=dev),
                   nhits=torch.empty(ld, dtype=torch.int32, device=dev),
                   status=torch.empty(ld, dtype=torch.int32, device=dev))
    need = kf_build_workspace_bytes(bp, binned, n_seeds)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    dd = detector(d)
    hd = binned.descriptor()
    ex = extra if extra is not None else BuildExtra()
    _check(lib().kf_build_det(ctypes.byref(dd), ctypes.byref(bp), ctypes.byref(hd), n_seeds, ld, _ptr(seed_par),
                              _ptr(seed_cov), _ptr(q), _ptr(out["hits"]), _ptr(out["visit"]), _ptr(out["par"]),
                              _ptr(out["cov"]), _ptr(out["chi2"]), _ptr(out["nhits"]), _ptr(out["status"]),
                              ctypes.byref(ex), _ptr(ws), ctypes.c_size_t(need), _stream(stream)))
    return out


def kf_build_det_last_launch() -> dict:
    info = LaunchInfo()
    _check(lib().kf_build_det_last_launch(ctypes.byref(info)))
    return {k: int(getattr(info, k)) for k, _ in LaunchInfo._fields_}


def kf_build_noalloc(g, bp, binned: BinnedHits, n_seeds, seed_par, seed_cov, q, extra=None, out=None, stream=None):
    """kf_build with the library's static workspace (no workspace argument;
    the call allocates no device memory when `out` is given)."""
    ld = seed_par.shape[1]
    dev = seed_par.device
    F = bp.first_layer
    if out is None:
        out = dict(hits=torch.empty((g.n_layers - F, ld), dtype=torch.int32, device=dev),
                   par=torch.empty((6, ld), dtype=torch.float32, device=dev),
                   cov=torch.empty((21, ld), dtype=torch.float32, device=dev),
                   chi2=torch.empty(ld, dtype=torch.float32, device=dev),
                   nhits=torch.empty(ld, dtype=torch.int32, device=dev),
                   status=torch.empty(ld, dtype=torch.int32, device=dev))
    gg = geometry(g)
    hd = binned.descriptor()
    ex = extra if extra is not None else BuildExtra()
    _check(lib().kf_build_noalloc(ctypes.byref(gg), ctypes.byref(bp), ctypes.byref(hd), n_seeds, ld, _ptr(seed_par),
                                  _ptr(seed_cov), _ptr(q), _ptr(out["hits"]), _ptr(out["par"]), _ptr(out["cov"]),
                                  _ptr(out["chi2"]), _ptr(out["nhits"]), _ptr(out["status"]), ctypes.byref(ex),
                                  _stream(stream)))
    return out


def kf_build_noalloc_max_bytes() -> int:
    return int(lib().kf_build_noalloc_max_bytes())


def kf_peak_fma(arith, blocks, iters, out, stream=None):
    """Launch the FMA-chain kernel (8 chains x iters x 2 flops per lane)."""
    _check(lib().kf_peak_fma(arith, blocks, iters, _ptr(out), _stream(stream)))


def kf_build_last_launch() -> dict:
    """Launch shape of the last kf_build call of this thread."""
    info = LaunchInfo()
    _check(lib().kf_build_last_launch(ctypes.byref(info)))
    return {k: int(getattr(info, k)) for k, _ in LaunchInfo._fields_}


def kf_gather_hits(n_layers, first_layer, n_seeds, built_hits, xyz, cov, seed_event=None, event_offsets=None,
                   fit_hits=None, hole_mask=None, stream=None):
    """Built hit lists -> fit rows [L][9][ld] and hole mask [ld] (int32 view)."""
    ld = built_hits.shape[1]
    dev = built_hits.device
    if fit_hits is None:
        fit_hits = torch.zeros((n_layers, 9, ld), dtype=torch.float32, device=dev)
    if hole_mask is None:
        hole_mask = torch.zeros(ld, dtype=torch.int32, device=dev)
    E = 1 if event_offsets is None else event_offsets.shape[0] - 1
    n_hits = xyz.shape[1]
    _check(lib().kf_gather_hits(n_layers, first_layer, n_seeds, ld, _ptr(built_hits), _ptr(seed_event), E,
                                _ptr(event_offsets), n_hits, _ptr(xyz), _ptr(cov), _ptr(fit_hits), _ptr(hole_mask),
                                _stream(stream)))
    return fit_hits, hole_mask


# ------------------------------------------------------------ window network

MLP_NPARAM = 64 * 27 + 64 + 64 * 64 + 64 + 2 * 64 + 2
MLP_ROW = 32
_MLP_HDR = 192


def _bf16_bits(a):
    """FP32 -> bfloat16 bit patterns, round to nearest even (packing only)."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def mlp_split(master):
    """FP32 master vector -> dict of W1 (64,27), b1, W2 (64,64), b2, W3 (2,64), b3."""
    m = np.asarray(master, dtype=np.float32)
    o = 0
    out = {}
    for k, shp in (("W1", (64, 27)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (2, 64)),
                   ("b3", (2,))):
        n = int(np.prod(shp))
        out[k] = m[o:o + n].reshape(shp)
        o += n
    return out


def mlp_join(p):
    return np.concatenate([np.asarray(p[k], dtype=np.float32).ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def _packed(Wm):
    """W [rows][64 hidden units] in the inference's operand order: entry
    (out, unit) at ((((out >> 4) * 2 + (unit >> 5)) * 16 + (out & 15)) * 32)
    + ((unit & 15) >> 2) * 8 + ((unit >> 4) & 1) * 4 + (unit & 3)."""
    rows = Wm.shape[0]
    out = np.arange(rows)[:, None]
    unit = np.arange(64)[None, :]
    idx = ((((out >> 4) * 2 + (unit >> 5)) * 16 + (out & 15)) * 32) + ((unit & 15) >> 2) * 8 + \
        ((unit >> 4) & 1) * 4 + (unit & 3)
    P = np.zeros(rows * 64, dtype=np.float32)
    P[idx.ravel()] = np.asarray(Wm, dtype=np.float32).ravel()
    return P


def mlp_block(master, mu, sd, scale, kappa=1.0, floor_rphi=0.01, floor_z=0.1, gate_rphi=0.0, gate_z=0.0,
              device="cuda:0"):
    """Pack the device block: FP32 header then BF16 weights (W1 padded to 32
    inputs, W2, W3 padded to 16 rows, W2 transposed, then W2 and W3 in the
    inference's operand order)."""
    p = mlp_split(master)
    hdr = np.zeros(_MLP_HDR, dtype=np.float32)
    hdr[0:27] = mu
    hdr[27:54] = 1.0 / np.asarray(sd, dtype=np.float64)
    hdr[54:118] = p["b1"]
    hdr[118:182] = p["b2"]
    hdr[182:184] = p["b3"]
    hdr[184:186] = scale
    hdr[186] = kappa
    hdr[187] = floor_rphi
    hdr[188] = floor_z
    hdr[189] = gate_rphi
    hdr[190] = gate_z
    W1 = np.zeros((64, 32), dtype=np.float32)
    W1[:, :27] = p["W1"]
    W3 = np.zeros((16, 64), dtype=np.float32)
    W3[:2] = p["W3"]
    w = np.concatenate([_bf16_bits(W1).ravel(), _bf16_bits(p["W2"]).ravel(), _bf16_bits(W3).ravel(),
                        _bf16_bits(np.ascontiguousarray(p["W2"].T)).ravel(),
                        _bf16_bits(_packed(p["W2"])).ravel(), _bf16_bits(_packed(W3)).ravel()])
    raw = np.concatenate([hdr.view(np.uint8), w.view(np.uint8)])
    assert raw.size == int(lib().kf_mlp_block_bytes())
    return torch.from_numpy(raw.view(np.float32).copy()).to(device)


def mlp_set_header(block, kappa=None, floor_rphi=None, floor_z=None, gate_rphi=None, gate_z=None):
    """Rewrite header words of a device block in place (None leaves a word);
    gates: the network is consulted only where the plain arc or z half-width
    exceeds them (0: everywhere)."""
    if gate_rphi is not None:
        block[189] = gate_rphi
    if gate_z is not None:
        block[190] = gate_z
    if kappa is not None:
        block[186] = kappa
    if floor_rphi is not None:
        block[187] = floor_rphi
    if floor_z is not None:
        block[188] = floor_z


def kf_mlp_forward(block, rows, n=None, logits=False, stream=None):
    n = rows.shape[0] if n is None else n
    out = torch.empty((max(n, 1), 2), dtype=torch.float32, device=rows.device)
    lo = torch.empty((max(n, 1), 2), dtype=torch.float32, device=rows.device) if logits else None
    _check(lib().kf_mlp_forward(_ptr(block), n, _ptr(rows), _ptr(out), _ptr(lo), _stream(stream)))
    return (out, lo) if logits else out


def kf_mlp_grad(block, rows, n=None, grad=None, ws=None, stream=None):
    n = rows.shape[0] if n is None else n
    if grad is None:
        grad = torch.empty(MLP_NPARAM + 1, dtype=torch.float32, device=rows.device)
    need = int(lib().kf_mlp_grad_workspace_bytes(n))
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need // 4 + 1, dtype=torch.float32, device=rows.device)
    _check(lib().kf_mlp_grad(_ptr(block), n, _ptr(rows), _ptr(grad), _ptr(ws), ctypes.c_size_t(need),
                             _stream(stream)))
    return grad


def kf_mlp_adam(block, master, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().kf_mlp_adam(_ptr(block), _ptr(master), _ptr(m), _ptr(v), _ptr(grad), step, ctypes.c_float(lr),
                             ctypes.c_float(beta1), ctypes.c_float(beta2), ctypes.c_float(eps), _stream(stream)))


# ------------------------------------------------------------ batched graph

class BatchPlan:
    """hit_bin + kf_build of a batch of events captured as one HIP graph;
    with fit_arith set, also kf_gather_hits + kf_fit of the built lists (the
    whole step), fit outputs in self.fit.  The graph bakes in raw device
    pointers: the plan holds references to the buffers it allocates and to
    the inputs it is given, and `keep` must list the tensors behind the raw
    pointers of `extra` (seed_event, seed_order, counters, ticks, ...) and of
    bp.mlp (the network block), so none is freed while the plan lives."""

    def __init__(self, g, bp, layer, xyz, cov, event_offsets, n_phi, n_z, n_seeds, seed_par, seed_cov, q,
                 extra=None, stream=None, fit_arith=None, keep=()):
        dev = layer.device
        n_hits = layer.shape[0]
        E = event_offsets.shape[0] - 1
        self.binned = BinnedHits(E, g.n_layers, n_phi, n_z, n_hits, dev)
        self.bin_ws = torch.empty(max(hit_bin_workspace_bytes(E, g.n_layers, n_phi, n_z, n_hits), 1),
                                  dtype=torch.uint8, device=dev)
        self.build_ws = torch.empty(max(kf_build_workspace_bytes(bp, self.binned, n_seeds), 1), dtype=torch.uint8,
                                    device=dev)
        ld = seed_par.shape[1]
        F = bp.first_layer
        self.out = dict(hits=torch.empty((g.n_layers - F, ld), dtype=torch.int32, device=dev),
                        par=torch.empty((6, ld), dtype=torch.float32, device=dev),
                        cov=torch.empty((21, ld), dtype=torch.float32, device=dev),
                        chi2=torch.empty(ld, dtype=torch.float32, device=dev),
                        nhits=torch.empty(ld, dtype=torch.int32, device=dev),
                        status=torch.empty(ld, dtype=torch.int32, device=dev))
        self._keep = (layer, xyz, cov, event_offsets, seed_par, seed_cov, q) + tuple(keep)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.g = geometry(g)
        self.bp = bp
        self.extra = extra if extra is not None else BuildExtra()
        self.hd = self.binned.descriptor()
        h = ctypes.c_void_p()
        b = self.binned
        base = b.xyzphi
        args = [
            ctypes.byref(self.g), ctypes.byref(self.bp), E, _ptr(event_offsets), n_hits, _ptr(layer), _ptr(xyz),
            _ptr(cov), ctypes.byref(self.hd), _ptr(b.offsets), _ptr(base), _ptr(b.cov), _ptr(b.orig),
            _ptr(self.bin_ws), ctypes.c_size_t(self.bin_ws.numel()), n_seeds, ld, _ptr(seed_par), _ptr(seed_cov),
            _ptr(q), _ptr(self.out["hits"]), _ptr(self.out["par"]), _ptr(self.out["cov"]), _ptr(self.out["chi2"]),
            _ptr(self.out["nhits"]), _ptr(self.out["status"]), ctypes.byref(self.extra), _ptr(self.build_ws),
            ctypes.c_size_t(self.build_ws.numel())]
        self.fit = None
        torch.cuda.synchronize()
        if fit_arith is None:
            _check(lib().kf_batch_plan_create(*args, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        else:
            L = g.n_layers
            self.fit = dict(hits=torch.zeros((L, 9, ld), dtype=torch.float32, device=dev),
                            hole=torch.zeros(ld, dtype=torch.int32, device=dev),
                            par=torch.empty((6, ld), dtype=torch.float32, device=dev),
                            cov=torch.empty((21, ld), dtype=torch.float32, device=dev),
                            chi2=torch.empty(ld, dtype=torch.float32, device=dev),
                            ndof=torch.empty(ld, dtype=torch.int32, device=dev),
                            status=torch.empty(ld, dtype=torch.int32, device=dev))
            f = self.fit
            self.fs = FitStage(fit_arith, _ptr(f["hits"]), _ptr(f["hole"]), _ptr(f["par"]), _ptr(f["cov"]),
                               _ptr(f["chi2"]), _ptr(f["ndof"]), _ptr(f["status"]))
            torch.cuda.synchronize()
            _check(lib().kf_step_plan_create(*args, ctypes.byref(self.fs), ctypes.c_void_p(self.stream.cuda_stream),
                                             ctypes.byref(h)))
        self.handle = h

    def launch(self):
        _check(lib().kf_batch_plan_launch(self.handle, ctypes.c_void_p(self.stream.cuda_stream)))

    def close(self):
        if self.handle:
            lib().kf_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wall_clock_khz() -> int:
    v = ctypes.c_int32()
    _check(lib().kf_wall_clock_khz(ctypes.byref(v)))
    return int(v.value)
