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


def test_gates_from_the_dumped_plain_widths():
    """The gates are quantiles of the plain half-widths the builder writes
    into each dumped row (columns 29 and 30); quantile 0 consults the network
    everywhere."""
    from paper_1711_06571_amd import window
    w = presets.learned()
    rng = np.random.default_rng(3)
    n = 1000
    rows = np.zeros((n, 32), dtype=np.float32)
    rows[:, 29] = rng.uniform(0.01, 0.5, n)
    rows[:, 30] = rng.uniform(0.3, 3.0, n)
    rows[:, 31] = ((np.arange(n, dtype=np.uint32) << 8) | (5 << 3) | 2).view(np.float32)
    wr, wz = window.plain_widths(w, rows)
    assert np.array_equal(wr, rows[:, 29].astype(np.float64)) and np.array_equal(wz, rows[:, 30].astype(np.float64))
    assert window.gates(w, rows, 0.0) == (0.0, 0.0)
    gr, gz = window.gates(w, rows, 0.9)
    assert np.mean(wr > gr) == pytest.approx(0.1, abs=0.01) and np.mean(wz > gz) == pytest.approx(0.1, abs=0.01)
    seed, layer, slot = window.row_ids(rows)
    assert np.array_equal(seed, np.arange(n)) and np.all(layer == 5) and np.all(slot == 2)


def test_autotune_choice():
    from paper_1711_06571_amd.batch import TunePoint, choose
    pts = [TunePoint(256, 2, 6, 32, 19.3, 0.8028, 15.8, 16.9), TunePoint(256, 2, 6, 64, 19.2, 0.8028, 15.5, 16.7),
           TunePoint(256, 2, 4, 64, 12.8, 0.7982, 9.4, 10.2), TunePoint(128, 0, 8, 64, 26.5, 0.8041, 22.0, 23.9)]
    assert choose(pts, 0.001) is pts[1]  # cap 4 loses 0.46 % > 0.1 %
    assert choose(pts, 0.01) is pts[2]
    assert choose(pts[2:], 0.001) is pts[3]  # no cap-6 point: the best efficiency is the reference


def test_autotune_cache_round_trip(tmp_path, monkeypatch):
    """The autotuner's choice is written to the cache per arithmetic (merged
    with what is there) and read back by the binding; the cap stays out of
    the launch parameters."""
    from paper_1711_06571_amd import kftrack as kf
    from paper_1711_06571_amd.batch import TunePoint, TuneResult, save_cache
    path = str(tmp_path / "autotune.json")
    r64 = TuneResult(points=[TunePoint(256, 2, 6, 64, 24.1, 0.803, 21.0, 22.0)], gpu="gfx950")
    r64.best = r64.points[0]
    r32 = TuneResult(points=[TunePoint(128, 0, 6, 32, 19.0, 0.803, 15.0, 16.0)], gpu="gfx950")
    r32.best = r32.points[0]
    save_cache(r64, kf.ARITH_F64, path, "batch")
    save_cache(r32, kf.ARITH_F32, path, "batch")
    monkeypatch.setattr(kf, "TUNE_CACHE", path)
    monkeypatch.setattr(kf, "_tune", None)
    t64, t32 = kf.tuned_launch(kf.ARITH_F64), kf.tuned_launch(kf.ARITH_F32)
    assert (t64["lanes_per_block"], t64["blocks_per_cu"], t64["phi_refine"]) == (256, 2, 64)
    assert (t32["lanes_per_block"], t32["blocks_per_cu"], t32["phi_refine"]) == (128, 0, 32)
    assert "cap" not in t64
    monkeypatch.setattr(kf, "TUNE_CACHE", str(tmp_path / "missing.json"))
    monkeypatch.setattr(kf, "_tune", None)
    assert kf.tuned_launch(kf.ARITH_F64) is None
