"""Input generator: counter-based RNG known answers and event invariants."""
import dataclasses
import os

import numpy as np

from paper_1711_06571_amd import datagen, presets


def _philox(ctr, key):
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    datagen.lib().kfg_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return [int(v) for v in o]


def _golden(name):
    """Rows of hexadecimal words of a fixture under tests/golden (its header
    cites the source)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    rows = []
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([int(v, 16) for v in line.split()])
    return rows


def test_philox_known_answers():
    rows = _golden("philox4x32_10_kat.txt")
    assert len(rows) == 3
    for r in rows:
        assert _philox(r[0:4], r[4:6]) == r[6:10], r


def test_splitmix64_known_answer():
    rows = _golden("splitmix64_kat.txt")
    assert len(rows) == 1
    for state, out in rows:
        assert int(datagen.lib().kfg_splitmix64(state)) == out


def test_event_layout_and_truth():
    w = presets.build()
    ev = datagen.generate(w.geometry, w.gen, 3, 500, truth=True)
    L = w.geometry.n_layers
    r = np.array(w.geometry.r)
    assert ev.n_hits == L * (500 + 100)
    # layer-major grouping, each layer a contiguous block
    assert np.all(np.diff(ev.layer) >= 0)
    assert np.all(np.bincount(ev.layer) == 600)
    # every track hit sits on its layer, belongs to its track
    for l in range(L):
        idx = ev.trk_hits[l]
        assert np.all(ev.layer[idx] == l)
        assert np.all(ev.track[idx] == np.arange(500))
        rr = np.hypot(ev.xyz[0, idx], ev.xyz[1, idx])
        assert np.allclose(rr, r[l], rtol=0, atol=1e-9)
        # truth crossings lie on the cylinder and within the barrel
        rt = np.hypot(ev.truth[l, 0], ev.truth[l, 1])
        assert np.allclose(rt, r[l], rtol=0, atol=1e-9)
        assert np.all(np.abs(ev.truth[l, 2]) <= w.geometry.z_half)
    # noise hits are flagged and uniform in z within the barrel
    noise = ev.track < 0
    assert noise.sum() == L * 100
    assert np.all(np.abs(ev.xyz[2, noise]) <= w.geometry.z_half)
    # hit covariance: rank 2, no radial component, nominal resolutions
    for i in range(0, ev.n_hits, 97):
        c = ev.cov[:, i]
        V = np.array([[c[0], c[1], c[2]], [c[1], c[3], c[4]], [c[2], c[4], c[5]]])
        n = np.array([ev.xyz[0, i], ev.xyz[1, i], 0.0]) / np.hypot(ev.xyz[0, i], ev.xyz[1, i])
        assert abs(n @ V @ n) < 1e-15
        assert np.isclose(np.trace(V), w.gen.sig_rphi ** 2 + w.gen.sig_z ** 2, rtol=1e-12)


def test_kinematic_ranges_and_determinism():
    w = presets.fit_small()
    a = datagen.generate(w.geometry, w.gen, 0, 2000, truth=True)
    b = datagen.generate(w.geometry, w.gen, 0, 2000, truth=True)
    assert np.array_equal(a.xyz, b.xyz) and np.array_equal(a.trk_hits, b.trk_hits)
    c = datagen.generate(w.geometry, w.gen, 1, 2000, truth=True)
    assert not np.array_equal(a.xyz, c.xyz)
    pt = np.hypot(a.vertex[3], a.vertex[4])
    assert pt.min() >= 0.5 and pt.max() <= 10.0
    eta = np.arcsinh(a.vertex[5] / pt)
    assert np.abs(eta).max() <= 1.0 + 1e-12
    assert 0.45 < np.mean(a.q == 1) < 0.55
    # smearing: residual of the hit from the truth crossing
    r = np.array(w.geometry.r)
    dphi = []
    dz = []
    for l in range(w.geometry.n_layers):
        idx = a.trk_hits[l]
        ph = np.arctan2(a.xyz[1, idx], a.xyz[0, idx])
        pht = np.arctan2(a.truth[l, 1], a.truth[l, 0])
        dphi.append(np.angle(np.exp(1j * (ph - pht))) * r[l])
        dz.append(a.xyz[2, idx] - a.truth[l, 2])
    dphi = np.concatenate(dphi)
    dz = np.concatenate(dz)
    assert abs(np.std(dphi) / w.gen.sig_rphi - 1) < 0.03
    assert abs(np.std(dz) / w.gen.sig_z - 1) < 0.03


def test_uneven_batch_counts():
    w = presets.batch()
    n = [datagen.event_tracks(w.gen, e, w.tracks_lo, w.tracks_hi) for e in range(2000)]
    n = np.array(n)
    assert n.min() >= 500 and n.max() <= 50000
    # log-uniform: median near sqrt(500 * 50000) = 5000
    assert 4000 < np.median(n) < 6200
    g = dataclasses.replace(w.gen)
    cnt = np.zeros(32, dtype=np.int64)
    cfg = datagen._cfg(w.geometry, g)
    datagen.lib().kfg_layer_counts(datagen.ctypes.byref(cfg), 5, 1000, cnt.ctypes.data)
    f = cnt[: w.geometry.n_layers] / 1000.0 - 1.0
    assert np.all(f >= 0.05 - 1e-9) and np.all(f <= 0.30 + 1e-9) and np.std(f) > 0.01
