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


def _check_event(w, b_gpu, e, ev_xyz, ev_cov, ev_layer, base):
    """Compare event e of a binned batch with the oracle's binning of that event."""
    o = oracle.hit_bin(w.geometry, 63, 16, ev_layer, ev_xyz)
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
