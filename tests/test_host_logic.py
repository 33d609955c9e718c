"""Host-side logic that needs no GPU: workspace-size queries of the C ABI,
the plain-window widths and gates of the learned window, and the
autotuner's choice rule."""
import ctypes

import numpy as np
import pytest

from paper_1711_06571_amd import presets


@pytest.fixture(scope="module")
def kf():
    from paper_1711_06571_amd import kftrack
    return kftrack


def test_hit_bin_workspace_bytes(kf):
    q = kf.hit_bin_workspace_bytes
    assert q(0, 17, 63, 16, 10) == 0 and q(1, 17, 0, 16, 10) == 0 and q(1, 17, 63, 16, -1) == 0
    NB = 3 * 17 * 63 * 16
    a, b = q(3, 17, 63, 16, 1000), q(3, 17, 63, 16, 2000)
    # per hit: bin, arrival index, phi (4 bytes each) and a 48-byte record
    assert b - a == pytest.approx(1000 * 60, abs=4 * 256)
    assert a >= 1000 * 60 + 2 * NB * 4 and a % 256 == 0  # bin counts and starts
    assert q(3, 17, 63, 16, 0) >= 2 * NB * 4


def test_kf_build_workspace_bytes(kf):
    w = presets.build()
    bp = kf.build_params(w.cuts)
    hd = kf.Hits()
    hd.n_events, hd.n_layers, hd.n_phi, hd.n_z = 2, 17, 63, 16
    hd.n_hits = 1000
    lib = kf.lib()
    a = lib.kf_build_workspace_bytes(ctypes.byref(bp), ctypes.byref(hd), 100)
    hd.n_hits = 2000
    b = lib.kf_build_workspace_bytes(ctypes.byref(bp), ctypes.byref(hd), 100)
    # the packed hit copy: 48 bytes per hit
    assert b - a == pytest.approx(48 * 1000, abs=256)
    # the fine index: n_phi * refine + 1 entries per (event, layer, z row)
    bp64, bp8 = kf.build_params(w.cuts, phi_refine=64), kf.build_params(w.cuts, phi_refine=8)
    f64 = lib.kf_build_workspace_bytes(ctypes.byref(bp64), ctypes.byref(hd), 100)
    f8 = lib.kf_build_workspace_bytes(ctypes.byref(bp8), ctypes.byref(hd), 100)
    assert f64 - f8 == pytest.approx(2 * 17 * 16 * 63 * 56 * 4, abs=512)
    assert lib.kf_build_workspace_bytes(ctypes.byref(bp), ctypes.byref(hd), 100) == f64  # 0 means 64
    hd.n_hits = -1
    assert lib.kf_build_workspace_bytes(ctypes.byref(bp), ctypes.byref(hd), 100) == 0


def test_plain_widths_and_gates():
    from paper_1711_06571_amd import window
    w = presets.learned()
    c = w.cuts
    rng = np.random.default_rng(3)
    n = 1000
    rows = np.zeros((n, 32), dtype=np.float32)
    phi = rng.uniform(0, 2 * np.pi, n)
    r = rng.uniform(4, 60, n)
    rows[:, 0], rows[:, 1], rows[:, 2] = r * np.cos(phi), r * np.sin(phi), rng.uniform(-50, 50, n)
    # an isotropic transverse position covariance s2 I and a z variance v
    s2, v = rng.uniform(1e-6, 1e-2, n), rng.uniform(1e-4, 1.0, n)
    rows[:, 6], rows[:, 12], rows[:, 17] = s2, s2, v  # P_xx, P_yy, P_zz in the row layout
    wr, wz = window.plain_widths(w, rows)
    assert np.allclose(wr, c.nsigma * np.sqrt(s2 + c.win_sig_rphi ** 2), rtol=1e-5)
    assert np.allclose(wz, c.nsigma * np.sqrt(v + c.win_sig_z ** 2), rtol=1e-5)
    assert window.gates(w, rows, 0.0) == (0.0, 0.0)
    gr, gz = window.gates(w, rows, 0.9)
    assert np.mean(wr > gr) == pytest.approx(0.1, abs=0.01) and np.mean(wz > gz) == pytest.approx(0.1, abs=0.01)


def test_autotune_choice():
    from paper_1711_06571_amd.batch import TunePoint, choose
    pts = [TunePoint(256, 2, 6, 32, 19.3, 0.8028, 15.8, 16.9), TunePoint(256, 2, 6, 64, 19.2, 0.8028, 15.5, 16.7),
           TunePoint(256, 2, 4, 64, 12.8, 0.7982, 9.4, 10.2), TunePoint(128, 0, 8, 64, 26.5, 0.8041, 22.0, 23.9)]
    assert choose(pts, 0.001) is pts[1]  # cap 4 loses 0.46 % > 0.1 %
    assert choose(pts, 0.01) is pts[2]
    assert choose(pts[2:], 0.001) is pts[3]  # no cap-6 point: the best efficiency is the reference
