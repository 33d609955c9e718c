"""GPU hit_bin vs the oracle's counting sort: offsets and order bit-exact."""
import numpy as np
import pytest

import oracle
from paper_1711_06571_amd import datagen, presets, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from gpu_common import host, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def kf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_06571_amd import kftrack
    return kftrack


def _check_event(w, b_gpu, e, ev_xyz, ev_cov, ev_layer, base, n_phi=63, n_z=16):
    """Compare event e of a binned batch with the oracle's binning of that event."""
    o = oracle.hit_bin(w.geometry, n_phi, n_z, ev_layer, ev_xyz)
    off_g = host(b_gpu.offsets)[e] - base
    assert np.array_equal(off_g, o["offsets"])
    n = ev_layer.shape[0]
    orig = host(b_gpu.orig)[base:base + n]
    assert np.array_equal(orig, o["order"])
    xyzphi = host(b_gpu.xyzphi)[:, base:base + n]
    assert np.array_equal(xyzphi[3], o["phi"])
    assert np.array_equal(xyzphi[:3], ev_xyz[:, o["order"]])
    assert np.array_equal(host(b_gpu.cov)[:, base:base + n], ev_cov[:, o["order"]])


def test_hit_bin_single_event(kf):
    w = presets.build()
    ev = datagen.generate(w.geometry, w.gen, 0, w.n_tracks)
    xyz = ev.xyz.astype(np.float32)
    cov = ev.cov.astype(np.float32)
    b = kf.hit_bin(w.geometry, 63, 16, to_dev(ev.layer), to_dev(xyz), to_dev(cov))
    torch.cuda.synchronize()
    assert int(host(b.bad)[0]) == 0
    _check_event(w, b, 0, xyz, cov, ev.layer, 0)


def test_hit_bin_batch_of_uneven_events(kf):
    w = presets.batch()
    eb = workloads.event_batch(w, range(6))
    eoff = eb.hit_offsets
    b = kf.hit_bin(w.geometry, 63, 16, to_dev(eb.layer), to_dev(eb.xyz), to_dev(eb.cov), event_offsets=to_dev(eoff))
    torch.cuda.synchronize()
    for e in range(6):
        sl = slice(eoff[e], eoff[e + 1])
        _check_event(w, b, e, np.ascontiguousarray(eb.xyz[:, sl]), np.ascontiguousarray(eb.cov[:, sl]),
                     np.ascontiguousarray(eb.layer[sl]), int(eoff[e]))


def test_hit_bin_edge_cases(kf):
    w = presets.build()
    g = w.geometry
    # empty input
    b = kf.hit_bin(g, 63, 16, torch.zeros(0, dtype=torch.int32, device="cuda:0"),
                   torch.zeros((3, 0), device="cuda:0"), torch.zeros((6, 0), device="cuda:0"))
    torch.cuda.synchronize()
    assert np.all(host(b.offsets) == 0)
    # hits on bin edges, phi = 0 and near 2 pi, z at the barrel ends, one bad layer
    R = g.r[4]
    ph = np.array([0.0, 2 * np.pi / 63, 2 * np.pi - 1e-7, np.pi, 1.0, 1.0], dtype=np.float64)
    z = np.array([-100.0, 100.0, 0.0, 12.5, -87.5, 3.0])
    xyz = np.stack([R * np.cos(ph), R * np.sin(ph), z]).astype(np.float32)
    cov = np.ones((6, 6), dtype=np.float32)
    layer = np.array([4, 4, 4, 4, 4, 99], dtype=np.int32)
    b = kf.hit_bin(g, 63, 16, to_dev(layer), to_dev(xyz), to_dev(cov))
    torch.cuda.synchronize()
    assert int(host(b.bad)[0]) == 1
    o = oracle.hit_bin(g, 63, 16, layer, xyz)
    assert np.array_equal(host(b.offsets)[0], o["offsets"])
    assert np.array_equal(host(b.orig)[:5], o["order"][:5])


# ---- the two sorting paths -------------------------------------------------
# Input grouped by layer (all valid) is sorted by one block per (event,
# layer); any other input by the general kernels.  The workspace's last 256
# bytes hold the path flag (0: grouped path).  The grouped path is tried
# when there are enough (event, layer) ranges, or when the environment asks
# for it (as the tests below do, whatever the size).


@pytest.fixture
def grouped(monkeypatch):
    monkeypatch.setenv("KFTRACK_HIT_BIN_PATH", "grouped")

def _bin(kf, g, n_phi, n_z, layer, xyz, cov, eoff=None):
    E = 1 if eoff is None else len(eoff) - 1
    need = kf.hit_bin_workspace_bytes(E, g.n_layers, n_phi, n_z, layer.shape[0])
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    b = kf.hit_bin(g, n_phi, n_z, to_dev(layer), to_dev(np.ascontiguousarray(xyz)), to_dev(np.ascontiguousarray(cov)),
                   event_offsets=None if eoff is None else to_dev(np.asarray(eoff, np.int32)), ws=ws)
    torch.cuda.synchronize()
    flag = int(ws[need - 256:need - 252].view(torch.int32).cpu()[0])
    return b, flag


def _event(seed=0):
    w = presets.build()
    ev = datagen.generate(w.geometry, w.gen, seed, w.n_tracks)
    return w, ev.layer.astype(np.int32), ev.xyz.astype(np.float32), ev.cov.astype(np.float32)


def test_grouped_input_takes_the_block_path(kf, grouped):
    w, layer, xyz, cov = _event()
    assert np.all(np.diff(layer) >= 0)
    b, flag = _bin(kf, w.geometry, 63, 16, layer, xyz, cov)
    assert flag == 0
    assert int(host(b.bad)[0]) == 0
    _check_event(w, b, 0, xyz, cov, layer, 0)


def test_shuffled_input_takes_the_general_path(kf, grouped):
    """The same hits in a random order: general kernels, oracle order (the
    original index is the shuffled position)."""
    w, layer, xyz, cov = _event()
    perm = np.random.default_rng(5).permutation(layer.shape[0])
    layer, xyz, cov = layer[perm], np.ascontiguousarray(xyz[:, perm]), np.ascontiguousarray(cov[:, perm])
    b, flag = _bin(kf, w.geometry, 63, 16, layer, xyz, cov)
    assert flag == 1
    _check_event(w, b, 0, xyz, cov, layer, 0)


def test_layers_in_descending_order_take_the_general_path(kf, grouped):
    w, layer, xyz, cov = _event()
    order = np.argsort(-layer, kind="stable")
    layer, xyz, cov = layer[order], np.ascontiguousarray(xyz[:, order]), np.ascontiguousarray(cov[:, order])
    b, flag = _bin(kf, w.geometry, 63, 16, layer, xyz, cov)
    assert flag == 1
    _check_event(w, b, 0, xyz, cov, layer, 0)


def test_bin_above_the_tile_takes_the_general_path(kf, grouped):
    """One bin per layer (more than 2048 hits each): the grouped path gives way."""
    w, layer, xyz, cov = _event()
    assert np.bincount(layer).min() > 2048
    b, flag = _bin(kf, w.geometry, 1, 1, layer, xyz, cov)
    assert flag == 1
    _check_event(w, b, 0, xyz, cov, layer, 0, n_phi=1, n_z=1)


def test_many_bins_take_the_general_path(kf, grouped):
    w, layer, xyz, cov = _event()
    b, flag = _bin(kf, w.geometry, 128, 64, layer, xyz, cov)
    assert flag == 1
    _check_event(w, b, 0, xyz, cov, layer, 0, n_phi=128, n_z=64)


def test_block_path_with_empty_layers_and_events(kf, grouped):
    """Grouped events where some layers (and one whole event) hold no hits;
    small bins (a tile of 2048 positions spans many bins), coarse bins (a
    tile ends inside a layer's range)."""
    w, layer, xyz, cov = _event()
    keep = (layer != 3) & (layer != 9)
    l2, x2, c2 = layer[keep], np.ascontiguousarray(xyz[:, keep]), np.ascontiguousarray(cov[:, keep])
    n1 = l2.shape[0]
    lay = np.concatenate([l2, l2[:0], layer])
    X = np.concatenate([x2, x2[:, :0], xyz], axis=1)
    C = np.concatenate([c2, c2[:, :0], cov], axis=1)
    eoff = [0, n1, n1, lay.shape[0]]
    for n_phi, n_z in ((63, 16), (8, 2)):
        b, flag = _bin(kf, w.geometry, n_phi, n_z, lay, X, C, eoff=eoff)
        assert flag == 0
        for e in (0, 1, 2):
            sl = slice(eoff[e], eoff[e + 1])
            _check_event(w, b, e, np.ascontiguousarray(X[:, sl]), np.ascontiguousarray(C[:, sl]),
                         np.ascontiguousarray(lay[sl]), eoff[e], n_phi=n_phi, n_z=n_z)


def test_batch_of_events_takes_the_block_path(kf, grouped):
    w = presets.batch()
    eb = workloads.event_batch(w, range(6))
    b, flag = _bin(kf, w.geometry, 63, 16, eb.layer, eb.xyz, eb.cov, eoff=eb.hit_offsets)
    assert flag == 0
    eoff = eb.hit_offsets
    for e in range(6):
        sl = slice(eoff[e], eoff[e + 1])
        _check_event(w, b, e, np.ascontiguousarray(eb.xyz[:, sl]), np.ascontiguousarray(eb.cov[:, sl]),
                     np.ascontiguousarray(eb.layer[sl]), int(eoff[e]))


def test_path_choice_follows_the_number_of_ranges(kf, monkeypatch):
    """Without the override: one event (17 ranges) goes to the general
    kernels; many small events (at least six ranges per compute unit) to the
    grouped path; =general forces the general kernels.  Results equal the
    oracle either way."""
    monkeypatch.delenv("KFTRACK_HIT_BIN_PATH", raising=False)
    w, layer, xyz, cov = _event()
    b, flag = _bin(kf, w.geometry, 63, 16, layer, xyz, cov)
    assert flag == 1
    _check_event(w, b, 0, xyz, cov, layer, 0)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    E = -(-6 * cus // w.geometry.n_layers)
    eb = workloads.event_batch(w, range(E), n_tracks=100)
    b, flag = _bin(kf, w.geometry, 63, 16, eb.layer, eb.xyz, eb.cov, eoff=eb.hit_offsets)
    assert flag == 0
    eoff = eb.hit_offsets
    for e in (0, E // 2, E - 1):
        sl = slice(eoff[e], eoff[e + 1])
        _check_event(w, b, e, np.ascontiguousarray(eb.xyz[:, sl]), np.ascontiguousarray(eb.cov[:, sl]),
                     np.ascontiguousarray(eb.layer[sl]), int(eoff[e]))
    monkeypatch.setenv("KFTRACK_HIT_BIN_PATH", "general")
    b, flag = _bin(kf, w.geometry, 63, 16, eb.layer, eb.xyz, eb.cov, eoff=eb.hit_offsets)
    assert flag == 1
    sl = slice(eoff[1], eoff[2])
    _check_event(w, b, 1, np.ascontiguousarray(eb.xyz[:, sl]), np.ascontiguousarray(eb.cov[:, sl]),
                 np.ascontiguousarray(eb.layer[sl]), int(eoff[1]))
