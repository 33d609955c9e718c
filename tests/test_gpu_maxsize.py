"""The largest sizes the library accepts, against the oracle: 32 layers
(every bit of the fit's hole mask, the longest per-wave history tables of
the build) for the fit and the build, and the build at the largest
candidate cap (8)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1711_06571_amd import datagen, presets

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from gpu_common import assert_fit_parity_converged, host, to_dev  # noqa: E402
from test_gpu_build import compare, gpu_build_event  # noqa: E402


@pytest.fixture(scope="module")
def kf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_06571_amd import kftrack
    return kftrack


def workload32(noise):
    # a longer barrel so that tracks of |eta| up to ~1 reach r = 128 cm
    g = presets.barrel(32, z_half=250.0)
    gen = presets.GenSettings(seed=presets.SEED_BASE + 9, noise_lo=noise, noise_hi=noise)
    return presets.Workload(f"32 layers r=4..128 cm, |z|<250 cm, {noise:.0%} noise", g, gen, 1, 300)


def test_fit_32_layers(kf):
    """Tracks with hits on all 32 layers, some layers dropped to holes (the
    hole mask's high bits included): FP64 fit against the oracle's."""
    w = workload32(0.0)
    g = w.geometry
    ev = datagen.generate(g, w.gen, 0, w.n_tracks)
    n = ev.n_tracks
    H = datagen.track_hits(ev)
    so = oracle.seed(g, H, n)
    ld = H.shape[2]
    rng = np.random.default_rng(32)
    hm = np.zeros(ld, dtype=np.uint32)
    for l in (5, 17, 30, 31):
        hm[:n] |= np.where(rng.random(n) < 0.3, np.uint32(1) << np.uint32(l), np.uint32(0))
    par, cov, q = so["par"].astype(np.float32), so["cov"].astype(np.float32), so["q"].astype(np.int8)
    o = oracle.fit(g, 3, H, par, cov, q, n, hole_mask=hm)
    out = kf.kf_fit(g, n, 3, to_dev(H), to_dev(par), to_dev(cov), to_dev(q), hole_mask=to_dev(hm.view(np.int32)),
                    arith=kf.ARITH_F64)
    gg = {k: host(v) for k, v in out.items()}
    errs = assert_fit_parity_converged(gg, o, n, "fit 32 layers")
    nd = 2 * (32 - 3 - np.array([bin(int(v)).count("1") for v in hm[:n]]))
    ok = gg["status"][:n] == 0
    assert np.array_equal(gg["ndof"][:n][ok], nd[ok])
    print("fit, 32 layers:", errs)


@pytest.mark.parametrize("cap", [6, 8])
def test_build_32_layers(kf, cap):
    """Build over 29 searched layers with 20 % noise, cap 6 and the largest
    cap 8: hit lists on every decidable seed against the oracle's."""
    w = workload32(0.2)
    ev = datagen.generate(w.geometry, w.gen, 1, w.n_tracks)
    n = ev.n_tracks
    gb, _ = gpu_build_event(kf, w, ev, kf.ARITH_F64, cap=cap)
    H = datagen.track_hits(ev)
    so = oracle.seed(w.geometry, H, n)
    cuts = dataclasses.replace(w.cuts, cand_cap=cap)
    o = oracle.build(w.geometry, cuts, ev.layer, ev.xyz, ev.cov, so["par"], so["cov"], so["q"], n)
    r = compare(gb, o, n, ctx=f"32 layers cap {cap}")
    assert gb["hits"].shape[0] == 29
    print(f"build, 32 layers, cap {cap}:", r)
