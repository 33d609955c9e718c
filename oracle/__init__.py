"""FP64 CPU oracle (ctypes binding of kforacle.c, plus the network oracle in
mlp.py).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg may use it; the GPU product path never imports it.  It
shares no code with the GPU library: the structures below mirror the C
header of this directory only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libkforacle.so")

TRK_NO_CROSSING = 1
TRK_OUT_OF_Z = 2
TRK_NONFINITE = 4
TRK_S_NOT_PD = 8
TRK_CAP_TRUNC = 16

# rows of the build's decision margins (smallest distance of a decision of
# that kind from its threshold, per seed)
MARGIN_CHI2, MARGIN_WINDOW, MARGIN_GEOMETRY, MARGIN_GATE, MARGIN_LEARNED = range(5)
N_MARGIN = 5


def build_lib() -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-o", _LIB,
           os.path.join(_HERE, "kforacle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


class Geom(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("r", ctypes.c_float * 32), ("z_half", ctypes.c_float),
                ("bz", ctypes.c_float), ("x_over_x0", ctypes.c_float), ("mass", ctypes.c_float)]


class BuildParams(ctypes.Structure):
    _fields_ = [("chi2_cut", ctypes.c_float), ("max_holes", ctypes.c_int32), ("cand_cap", ctypes.c_int32),
                ("nsigma", ctypes.c_float), ("win_sig_rphi", ctypes.c_float), ("win_sig_z", ctypes.c_float),
                ("first_layer", ctypes.c_int32), ("window_mode", ctypes.c_int32), ("mlp", ctypes.c_void_p),
                ("state", ctypes.c_int32)]


class Detector(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("kind", ctypes.c_int32 * 32), ("pos", ctypes.c_float * 32),
                ("lo", ctypes.c_float * 32), ("hi", ctypes.c_float * 32), ("dmod", ctypes.c_float * 32),
                ("bz", ctypes.c_float), ("x_over_x0", ctypes.c_float), ("mass", ctypes.c_float)]


BARREL, DISK = 0, 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError(f"{_LIB} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        L.orc_propagate.argtypes = [P, I, D, D, P, P, P]
        L.orc_state_at.argtypes = [P, I, D, D, P]
        L.orc_state_at.restype = None
        L.orc_jacobian.argtypes = [P, I, D, D, P]
        L.orc_jacobian.restype = None
        L.orc_ms_cov.argtypes = [P, D, D, P]
        L.orc_ms_cov.restype = None
        L.orc_update.argtypes = [P, P, P, P, P, P]
        L.orc_predict.argtypes = [ctypes.POINTER(Geom), I, P, I, P, P, P, P]
        L.orc_seed.argtypes = [ctypes.POINTER(Geom), I, I, P, D, P, P, P, P, P, P]
        L.orc_seed64.argtypes = [ctypes.POINTER(Geom), I, I, P, D, P, P, P, P]
        L.orc_beam_d0.argtypes = [P, I, D, P, P]
        L.orc_fit.argtypes = [ctypes.POINTER(Geom), I, I, I] + [P] * 10
        L.orc_fit64.argtypes = [ctypes.POINTER(Geom), I, I, I] + [P] * 9
        L.orc_hit_bin.argtypes = [ctypes.POINTER(Geom), I, I, I, P, P, P, P, P]
        L.orc_hyb_from_cart.argtypes = [P, I, P]
        L.orc_hyb_from_cart.restype = None
        L.orc_cart_from_hyb.argtypes = [P, P]
        L.orc_hyb_jac_cart_from_hyb.argtypes = [P, P]
        L.orc_hyb_jac_cart_from_hyb.restype = None
        L.orc_hyb_jac_hyb_from_cart.argtypes = [P, I, P]
        L.orc_hyb_jac_hyb_from_cart.restype = None
        L.orc_predict_hyb.argtypes = [ctypes.POINTER(Geom), I, P, P, P, P, P]
        L.orc_fit_hybrid.argtypes = [ctypes.POINTER(Geom), I, I, I] + [P] * 10
        L.orc_fit_hybrid64.argtypes = [ctypes.POINTER(Geom), I, I, I] + [P] * 9
        L.orc_build.argtypes = [ctypes.POINTER(Geom), ctypes.POINTER(BuildParams), I, P, P, P, I, I, P, P, P, I,
                                P, P, P, P, P, P, P, P]
        L.orc_mlp_forward.argtypes = [P, P, P]
        L.orc_mlp_blob_size.argtypes = []
        DP = ctypes.POINTER(Detector)
        L.orc_cyl_path.argtypes = [P, I, D, D, I, P, P]
        L.orc_plane_path.argtypes = [P, D, I, P]
        L.orc_jacobian_surf.argtypes = [P, I, D, D, I, P]
        L.orc_jacobian_surf.restype = None
        L.orc_ms_cov_surf.argtypes = [P, I, D, D, P]
        L.orc_ms_cov_surf.restype = None
        L.orc_step_surf.argtypes = [DP, I, D, I, I, P, I, P, P, P, P]
        L.orc_update_disk.argtypes = [P, P, P, P, P, P]
        L.orc_fit_det.argtypes = [DP, I, I, I] + [P] * 11
        L.orc_fit_det64.argtypes = [DP, I, I, I] + [P] * 10
        L.orc_hit_bin_det.argtypes = [DP, I, I, I, P, P, P, P, P]
        L.orc_build_det.argtypes = [DP, ctypes.POINTER(BuildParams), I, P, P, P, I, I, P, P, P, I, P] + [P] * 8
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def geom(g) -> Geom:
    """From a presets.Geometry."""
    o = Geom()
    o.n_layers = g.n_layers
    for i, v in enumerate(g.r):
        o.r[i] = v
    o.z_half, o.bz, o.x_over_x0, o.mass = g.z_half, g.bz, g.x_over_x0, g.mass
    return o


# ------------------------------------------------------------------ primitives

def propagate(X, q, R, bz):
    X = np.ascontiguousarray(X, dtype=np.float64)
    Xo = np.zeros(6)
    s = np.zeros(1)
    disc = np.zeros(1)
    rc = lib().orc_propagate(_p(X), int(q), float(R), float(bz), _p(Xo), _p(s), _p(disc))
    return rc, Xo, float(s[0]), float(disc[0])


def state_at(X, q, bz, s):
    X = np.ascontiguousarray(X, dtype=np.float64)
    Xo = np.zeros(6)
    lib().orc_state_at(_p(X), int(q), float(bz), float(s), _p(Xo))
    return Xo


def jacobian(X, q, bz, s):
    X = np.ascontiguousarray(X, dtype=np.float64)
    J = np.zeros(36)
    lib().orc_jacobian(_p(X), int(q), float(bz), float(s), _p(J))
    return J.reshape(6, 6)


def ms_cov(X, x_over_x0, mass):
    X = np.ascontiguousarray(X, dtype=np.float64)
    Q = np.zeros(36)
    lib().orc_ms_cov(_p(X), float(x_over_x0), float(mass), _p(Q))
    return Q.reshape(6, 6)


def update(X, P, hit):
    X = np.ascontiguousarray(X, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(36)
    hit = np.ascontiguousarray(hit, dtype=np.float64)
    Xo = np.zeros(6)
    Po = np.zeros(36)
    c2 = np.zeros(1)
    rc = lib().orc_update(_p(X), _p(P), _p(hit), _p(Xo), _p(Po), _p(c2))
    return rc, Xo, Po.reshape(6, 6), float(c2[0])


def predict(g, layer, X, q, P):
    X = np.ascontiguousarray(X, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(36)
    Xo = np.zeros(6)
    Po = np.zeros(36)
    disc = np.zeros(1)
    gg = geom(g)
    rc = lib().orc_predict(ctypes.byref(gg), int(layer), _p(X), int(q), _p(P), _p(Xo), _p(Po), _p(disc))
    return rc, Xo, Po.reshape(6, 6)


# ------------------------------------------------------------------ batches

def beam_d0(X, q, bz):
    """Impact parameter |c| - rho of the helix of X and its gradient."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    f = np.zeros(1)
    H = np.zeros(6)
    rc = lib().orc_beam_d0(_p(X), int(q), float(bz), _p(f), _p(H))
    return rc, float(f[0]), H


def _beam(g, beam_sigma):
    return float(getattr(g, "beam_sigma", 0.0)) if beam_sigma is None else float(beam_sigma)


def seed(g, hits, n, beam_sigma=None):
    """hits: [L][9][ld] float32.  Returns dict of FP32 seeds (the values both
    sides consume), their FP64 originals, q and status.  beam_sigma: the
    beam-spot width (cm) of the seed convention, default the geometry's;
    0 for the three-hit-only convention."""
    ld = hits.shape[2]
    hits = np.ascontiguousarray(hits, dtype=np.float32)
    q = np.zeros(ld, dtype=np.int8)
    par = np.zeros((6, ld), dtype=np.float32)
    cov = np.zeros((21, ld), dtype=np.float32)
    par64 = np.zeros((6, ld))
    cov64 = np.zeros((21, ld))
    st = np.zeros(ld, dtype=np.int32)
    gg = geom(g)
    rc = lib().orc_seed(ctypes.byref(gg), n, ld, _p(hits), _beam(g, beam_sigma), _p(q), _p(par), _p(cov), _p(par64),
                        _p(cov64), _p(st))
    if rc:
        raise ValueError("orc_seed: bad arguments")
    return dict(q=q, par=par, cov=cov, par64=par64, cov64=cov64, status=st)


def seed64(g, hits, n, beam_sigma=None):
    """FP64 hits [L][9][ld] -> FP64 seeds (no rounding anywhere)."""
    ld = hits.shape[2]
    hits = np.ascontiguousarray(hits, dtype=np.float64)
    q = np.zeros(ld, dtype=np.int8)
    par64 = np.zeros((6, ld))
    cov64 = np.zeros((21, ld))
    st = np.zeros(ld, dtype=np.int32)
    gg = geom(g)
    rc = lib().orc_seed64(ctypes.byref(gg), n, ld, _p(hits), _beam(g, beam_sigma), _p(q), _p(par64), _p(cov64),
                          _p(st))
    if rc:
        raise ValueError("orc_seed64: bad arguments")
    return dict(q=q, par64=par64, cov64=cov64, status=st)


def fit(g, first_layer, hits, seed_par, seed_cov, q, n, hole_mask=None):
    ld = hits.shape[2]
    out = dict(par=np.zeros((6, ld)), cov=np.zeros((21, ld)), chi2=np.zeros(ld), ndof=np.zeros(ld, np.int32),
               status=np.zeros(ld, np.int32))
    hits = np.ascontiguousarray(hits, dtype=np.float32)
    sp = np.ascontiguousarray(seed_par, dtype=np.float32)
    sc = np.ascontiguousarray(seed_cov, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.int8)
    hm = None if hole_mask is None else np.ascontiguousarray(hole_mask, dtype=np.uint32)
    gg = geom(g)
    rc = lib().orc_fit(ctypes.byref(gg), n, ld, first_layer, _p(hits), _p(hm), _p(sp), _p(sc), _p(q),
                       _p(out["par"]), _p(out["cov"]), _p(out["chi2"]), _p(out["ndof"]), _p(out["status"]))
    if rc:
        raise ValueError("orc_fit: bad arguments")
    return out


def hyb_from_cart(X, q):
    """Hybrid state (x, y, z, q/pT, phi, theta) of a Cartesian state."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.zeros(6)
    lib().orc_hyb_from_cart(_p(X), int(q), _p(Y))
    return Y


def cart_from_hyb(Y):
    """(Cartesian state, charge) of a hybrid state."""
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    X = np.zeros(6)
    q = lib().orc_cart_from_hyb(_p(Y), _p(X))
    return X, int(q)


def hyb_jacobians(Y):
    """(d cart / d hyb at Y, d hyb / d cart at the Cartesian image of Y)."""
    X, q = cart_from_hyb(Y)
    A = np.zeros(36)
    B = np.zeros(36)
    lib().orc_hyb_jac_cart_from_hyb(_p(np.ascontiguousarray(Y, dtype=np.float64)), _p(A))
    lib().orc_hyb_jac_hyb_from_cart(_p(X), q, _p(B))
    return A.reshape(6, 6), B.reshape(6, 6)


def predict_hyb(g, layer, Y, P):
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64)
    Yo = np.zeros(6)
    Po = np.zeros(36)
    gg = geom(g)
    rc = lib().orc_predict_hyb(ctypes.byref(gg), int(layer), _p(Y), _p(P), _p(Yo), _p(Po), None)
    return rc, Yo, Po.reshape(6, 6)


def fit_hybrid(g, first_layer, hits, seed_par, seed_cov, q, n, hole_mask=None):
    """Fit in the hybrid state from Cartesian seeds; outputs (x, y, z, q/pT,
    phi, theta) and their covariance."""
    ld = hits.shape[2]
    out = dict(par=np.zeros((6, ld)), cov=np.zeros((21, ld)), chi2=np.zeros(ld), ndof=np.zeros(ld, np.int32),
               status=np.zeros(ld, np.int32))
    hits = np.ascontiguousarray(hits, dtype=np.float32)
    sp = np.ascontiguousarray(seed_par, dtype=np.float32)
    sc = np.ascontiguousarray(seed_cov, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.int8)
    hm = None if hole_mask is None else np.ascontiguousarray(hole_mask, dtype=np.uint32)
    gg = geom(g)
    rc = lib().orc_fit_hybrid(ctypes.byref(gg), n, ld, first_layer, _p(hits), _p(hm), _p(sp), _p(sc), _p(q),
                              _p(out["par"]), _p(out["cov"]), _p(out["chi2"]), _p(out["ndof"]), _p(out["status"]))
    if rc:
        raise ValueError("orc_fit_hybrid: bad arguments")
    return out


def fit_hybrid64(g, first_layer, hits, seed_par, seed_cov, q, n):
    ld = hits.shape[2]
    out = dict(par=np.zeros((6, ld)), cov=np.zeros((21, ld)), chi2=np.zeros(ld), ndof=np.zeros(ld, np.int32),
               status=np.zeros(ld, np.int32))
    hits = np.ascontiguousarray(hits, dtype=np.float64)
    sp = np.ascontiguousarray(seed_par, dtype=np.float64)
    sc = np.ascontiguousarray(seed_cov, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.int8)
    gg = geom(g)
    rc = lib().orc_fit_hybrid64(ctypes.byref(gg), n, ld, first_layer, _p(hits), _p(sp), _p(sc), _p(q),
                                _p(out["par"]), _p(out["cov"]), _p(out["chi2"]), _p(out["ndof"]), _p(out["status"]))
    if rc:
        raise ValueError("orc_fit_hybrid64: bad arguments")
    return out


def fit64(g, first_layer, hits, seed_par, seed_cov, q, n):
    ld = hits.shape[2]
    out = dict(par=np.zeros((6, ld)), cov=np.zeros((21, ld)), chi2=np.zeros(ld), ndof=np.zeros(ld, np.int32),
               status=np.zeros(ld, np.int32))
    hits = np.ascontiguousarray(hits, dtype=np.float64)
    sp = np.ascontiguousarray(seed_par, dtype=np.float64)
    sc = np.ascontiguousarray(seed_cov, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.int8)
    gg = geom(g)
    rc = lib().orc_fit64(ctypes.byref(gg), n, ld, first_layer, _p(hits), _p(sp), _p(sc), _p(q),
                         _p(out["par"]), _p(out["cov"]), _p(out["chi2"]), _p(out["ndof"]), _p(out["status"]))
    if rc:
        raise ValueError("orc_fit64: bad arguments")
    return out


def hit_bin(g, n_phi, n_z, layer, xyz):
    n = layer.shape[0]
    L = g.n_layers
    nb = n_phi * n_z
    offsets = np.zeros((L, nb + 1), dtype=np.int32)
    order = np.zeros(n, dtype=np.int32)
    phi = np.zeros(n, dtype=np.float32)
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    layer = np.ascontiguousarray(layer, dtype=np.int32)
    gg = geom(g)
    rc = lib().orc_hit_bin(ctypes.byref(gg), n_phi, n_z, n, _p(layer), _p(xyz), _p(offsets), _p(order), _p(phi))
    if rc:
        raise ValueError("orc_hit_bin: bad arguments")
    return dict(offsets=offsets, order=order, phi=phi)


def build(g, cuts, layer, xyz, cov, seed_par, seed_cov, q, n_seeds, seed_list=None, cap=None,
          window_mode=0, mlp_blob=None, first_layer=None, state=0):
    """Brute-force combinatorial build.  seed_list selects seeds; outputs are
    indexed by position in the list (first len(seed_list) columns).  state 1
    builds in the hybrid state (Cartesian seeds converted; hybrid outputs)."""
    ld = seed_par.shape[1]
    lst = None if seed_list is None else np.ascontiguousarray(seed_list, dtype=np.int32)
    nl = n_seeds if lst is None else lst.shape[0]
    if nl > ld:
        raise ValueError("seed list longer than the leading dimension")
    F = cuts.first_layer if first_layer is None else first_layer
    L = g.n_layers
    o = dict(hits=np.zeros((L - F, ld), np.int32), par=np.zeros((6, ld)), cov=np.zeros((21, ld)),
             chi2=np.zeros(ld), nhits=np.zeros(ld, np.int32), status=np.zeros(ld, np.int32),
             margin=np.zeros((N_MARGIN, ld)))
    bp = BuildParams()
    bp.chi2_cut = cuts.chi2_cut
    bp.max_holes = cuts.max_holes
    bp.cand_cap = cuts.cand_cap if cap is None else cap
    bp.nsigma = cuts.nsigma
    bp.win_sig_rphi = cuts.win_sig_rphi
    bp.win_sig_z = cuts.win_sig_z
    bp.first_layer = F
    bp.window_mode = window_mode
    bp.state = state
    blob = None
    if window_mode == 1:
        blob = np.ascontiguousarray(mlp_blob, dtype=np.float64)
        bp.mlp = blob.ctypes.data
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    cov = np.ascontiguousarray(cov, dtype=np.float32)
    layer = np.ascontiguousarray(layer, dtype=np.int32)
    sp = np.ascontiguousarray(seed_par, dtype=np.float32)
    sc = np.ascontiguousarray(seed_cov, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.int8)
    gg = geom(g)
    rc = lib().orc_build(ctypes.byref(gg), ctypes.byref(bp), layer.shape[0], _p(layer), _p(xyz), _p(cov), n_seeds,
                         ld, _p(sp), _p(sc), _p(q), nl, _p(lst), _p(o["hits"]), _p(o["par"]), _p(o["cov"]),
                         _p(o["chi2"]), _p(o["nhits"]), _p(o["status"]), _p(o["margin"]))
    if rc:
        raise ValueError("orc_build: bad arguments")
    del blob
    return {k: (v[..., :nl]) for k, v in o.items()}


# Parity rule of the build: a seed is decidable when every decision of its
# search lies further from its threshold than the GPU's arithmetic can move
# it.  The GPU's hit tests and hit chi2 run in FP32 (positions rounded to
# ~1e-5 cm, chi2 ~3e-5 at the cut of 30), crossings and state in the mode's
# arithmetic; the network's widths carry BF16 activations.  The tolerances
# are about ten times those effects.  A gate decision compares a plain
# half-width (3 sqrt(S) from the covariance, ~1e-7 cm rounding even in FP32)
# with a constant: 1e-5 cm.
MARGIN_TOL = {MARGIN_CHI2: 1e-3, MARGIN_WINDOW: 1e-4, MARGIN_GEOMETRY: 1e-3, MARGIN_GATE: 1e-5,
              MARGIN_LEARNED: 1e-3}


def decidable(margin):
    """Per-seed mask: every margin row above its tolerance (MARGIN_TOL)."""
    m = np.asarray(margin)
    ok = np.ones(m.shape[1], dtype=bool)
    for row, tol in MARGIN_TOL.items():
        ok &= m[row] > tol
    return ok


def undecidable_by_row(margin):
    """Fraction of seeds each margin row alone makes undecidable."""
    m = np.asarray(margin)
    names = {MARGIN_CHI2: "chi2", MARGIN_WINDOW: "window", MARGIN_GEOMETRY: "geometry", MARGIN_GATE: "gate",
             MARGIN_LEARNED: "learned"}
    return {names[r]: float(np.mean(m[r] <= t)) for r, t in MARGIN_TOL.items()}


def mlp_forward(blob, x):
    blob = np.ascontiguousarray(blob, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.zeros(2)
    lib().orc_mlp_forward(_p(blob), _p(x), _p(w))
    return w


def mlp_blob_size() -> int:
    return int(lib().orc_mlp_blob_size())


# ------------------------------------------------------------ general detector

def detector(d) -> Detector:
    """From a presets.Detector."""
    o = Detector()
    o.n_layers = d.n_layers
    for i in range(d.n_layers):
        o.kind[i] = d.kind[i]
        o.pos[i], o.lo[i], o.hi[i], o.dmod[i] = d.pos[i], d.lo[i], d.hi[i], d.dmod[i]
    o.bz, o.x_over_x0, o.mass = d.bz, d.x_over_x0, d.mass
    return o


def cyl_path(X, q, R, bz, nearest=False):
    """Path s to the crossing with r = R (first ahead, or the nearest either
    way); None when the circles do not meet."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    s = ctypes.c_double(0)
    dsc = ctypes.c_double(0)
    rc = lib().orc_cyl_path(_p(X), int(q), float(R), float(bz), int(nearest), ctypes.byref(s), ctypes.byref(dsc))
    return None if rc else s.value


def plane_path(X, Z, nearest=False):
    X = np.ascontiguousarray(X, dtype=np.float64)
    s = ctypes.c_double(0)
    rc = lib().orc_plane_path(_p(X), float(Z), int(nearest), ctypes.byref(s))
    return None if rc else s.value


def jacobian_surf(X, q, bz, s, kind):
    X = np.ascontiguousarray(X, dtype=np.float64)
    J = np.zeros(36)
    lib().orc_jacobian_surf(_p(X), int(q), float(bz), float(s), int(kind), _p(J))
    return J.reshape(6, 6)


def ms_cov_surf(X, kind, x_over_x0, mass):
    X = np.ascontiguousarray(X, dtype=np.float64)
    Q = np.zeros(36)
    lib().orc_ms_cov_surf(_p(X), int(kind), float(x_over_x0), float(mass), _p(Q))
    return Q.reshape(6, 6)


def step_surf(d, kind, value, X, q, P, nearest=False, material=True):
    """One step to a surface (cylinder r = value or plane z = value): state,
    transported covariance (+ scattering); None on failure."""
    dd = detector(d)
    X = np.ascontiguousarray(X, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(36)
    Xo, Po = np.zeros(6), np.zeros(36)
    rc = lib().orc_step_surf(ctypes.byref(dd), int(kind), float(value), int(nearest), int(material), _p(X), int(q),
                             _p(P), _p(Xo), _p(Po), None)
    return None if rc else (Xo, Po.reshape(6, 6))


def update_disk(X, P, hit):
    X = np.ascontiguousarray(X, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64).reshape(36)
    hit = np.ascontiguousarray(hit, dtype=np.float64)
    Xo, Po, c2 = np.zeros(6), np.zeros(36), ctypes.c_double(0)
    rc = lib().orc_update_disk(_p(X), _p(P), _p(hit), _p(Xo), _p(Po), ctypes.byref(c2))
    return None if rc else (Xo, Po.reshape(6, 6), c2.value)


def _fit_out(ld):
    return dict(par=np.zeros((6, ld)), cov=np.zeros((21, ld)), chi2=np.zeros(ld), ndof=np.zeros(ld, np.int32),
                status=np.zeros(ld, np.int32))


def fit_det(d, first_layer, hits, visit, seed_par, seed_cov, q, n, hole_mask=None):
    """Fit over a general detector: hits [L][9][ld] FP32, visit [ld] uint32
    (bit l: the track crosses layer l), hole_mask (bit l: no hit there)."""
    dd = detector(d)
    hits = np.ascontiguousarray(hits, dtype=np.float32)
    ld = hits.shape[2]
    o = _fit_out(ld)
    visit = np.ascontiguousarray(visit, dtype=np.uint32)
    hm = None if hole_mask is None else np.ascontiguousarray(hole_mask, dtype=np.uint32)
    sp = np.ascontiguousarray(seed_par, dtype=np.float32)
    sc = np.ascontiguousarray(seed_cov, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.int8)
    rc = lib().orc_fit_det(ctypes.byref(dd), n, ld, first_layer, _p(hits), _p(visit), _p(hm), _p(sp), _p(sc), _p(q),
                           _p(o["par"]), _p(o["cov"]), _p(o["chi2"]), _p(o["ndof"]), _p(o["status"]))
    if rc:
        raise ValueError("orc_fit_det: bad arguments")
    return o


def fit_det64(d, first_layer, hits, visit, seed_par, seed_cov, q, n):
    dd = detector(d)
    hits = np.ascontiguousarray(hits, dtype=np.float64)
    ld = hits.shape[2]
    o = _fit_out(ld)
    visit = np.ascontiguousarray(visit, dtype=np.uint32)
    sp = np.ascontiguousarray(seed_par, dtype=np.float64)
    sc = np.ascontiguousarray(seed_cov, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.int8)
    rc = lib().orc_fit_det64(ctypes.byref(dd), n, ld, first_layer, _p(hits), _p(visit), _p(sp), _p(sc), _p(q),
                             _p(o["par"]), _p(o["cov"]), _p(o["chi2"]), _p(o["ndof"]), _p(o["status"]))
    if rc:
        raise ValueError("orc_fit_det64: bad arguments")
    return o


def hit_bin_det(d, n_phi, n_w, layer, xyz):
    dd = detector(d)
    layer = np.ascontiguousarray(layer, dtype=np.int32)
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    n = layer.shape[0]
    offsets = np.zeros((d.n_layers, n_phi * n_w + 1), np.int32)
    order = np.zeros(max(n, 1), np.int32)
    phi = np.zeros(max(n, 1), np.float32)
    rc = lib().orc_hit_bin_det(ctypes.byref(dd), n_phi, n_w, n, _p(layer), _p(xyz), _p(offsets), _p(order), _p(phi))
    if rc:
        raise ValueError("orc_hit_bin_det: bad arguments")
    return dict(offsets=offsets, order=order[:n], phi=phi[:n])


def build_det(d, cuts, layer, xyz, cov, seed_par, seed_cov, q, n_seeds, seed_list=None, cap=None):
    """Brute-force combinatorial build over a general detector (two-step
    propagation, next layer per candidate).  Outputs indexed by position in
    seed_list; hits [L - F][.] per layer, visit masks."""
    dd = detector(d)
    ld = seed_par.shape[1]
    lst = None if seed_list is None else np.ascontiguousarray(seed_list, dtype=np.int32)
    nl = n_seeds if lst is None else lst.shape[0]
    F = cuts.first_layer
    L = d.n_layers
    o = dict(hits=np.zeros((L - F, ld), np.int32), visit=np.zeros(ld, np.uint32), par=np.zeros((6, ld)),
             cov=np.zeros((21, ld)), chi2=np.zeros(ld), nhits=np.zeros(ld, np.int32), status=np.zeros(ld, np.int32),
             margin=np.zeros((N_MARGIN, ld)))
    bp = BuildParams()
    bp.chi2_cut = cuts.chi2_cut
    bp.max_holes = cuts.max_holes
    bp.cand_cap = cuts.cand_cap if cap is None else cap
    bp.nsigma = cuts.nsigma
    bp.win_sig_rphi = cuts.win_sig_rphi
    bp.win_sig_z = cuts.win_sig_z
    bp.first_layer = F
    bp.window_mode = 0
    bp.state = 0
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    cov = np.ascontiguousarray(cov, dtype=np.float32)
    layer = np.ascontiguousarray(layer, dtype=np.int32)
    sp = np.ascontiguousarray(seed_par, dtype=np.float32)
    sc = np.ascontiguousarray(seed_cov, dtype=np.float32)
    q = np.ascontiguousarray(q, dtype=np.int8)
    rc = lib().orc_build_det(ctypes.byref(dd), ctypes.byref(bp), layer.shape[0], _p(layer), _p(xyz), _p(cov),
                             n_seeds, ld, _p(sp), _p(sc), _p(q), nl, _p(lst), _p(o["hits"]), _p(o["visit"]),
                             _p(o["par"]), _p(o["cov"]), _p(o["chi2"]), _p(o["nhits"]), _p(o["status"]),
                             _p(o["margin"]))
    if rc:
        raise ValueError("orc_build_det: bad arguments")
    return {k: (v[..., :nl]) for k, v in o.items()}
