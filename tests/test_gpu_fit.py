"""GPU parity of kf_seed and kf_fit against the FP64 oracle, through the C ABI."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1711_06571_amd import datagen, presets

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def kf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_06571_amd import kftrack
    kftrack.lib()
    return kftrack


from gpu_common import (DEV, assert_fit_parity_converged, fit_agreement, fit_inputs, host,  # noqa: E402
                        seed_rel_sigma_p, to_dev)


def _seed_both(kf, g, H, n):
    so = oracle.seed(g, H, n)
    sg = kf.kf_seed(g, n, to_dev(H))
    sg = {k: host(v) for k, v in sg.items()}
    return so, sg


def _assert_seed_parity(so, sg, n):
    assert np.array_equal(so["q"][:n], sg["q"][:n])
    assert np.array_equal(so["status"][:n], sg["status"][:n])
    # both compute in FP64 and round to FP32: equal up to one FP32 rounding step
    d = np.abs(so["par"][:, :n].astype(np.float64) - sg["par"][:, :n])
    assert np.all(d <= 2.5e-7 * np.abs(so["par"][:, :n]) + 1e-30)
    dc = np.abs(so["cov"][:, :n].astype(np.float64) - sg["cov"][:, :n])
    scale = np.abs(so["cov"][:, :n]).max(axis=0, keepdims=True)
    assert np.all(dc <= 1e-6 * scale + 1e-30)


def test_seed_and_fit_parity_small(kf):
    """FP64 arithmetic: every track within the parity tolerances."""
    w = presets.fit_small()
    ev = datagen.generate(w.geometry, w.gen, 0, w.n_tracks)
    n = ev.n_tracks
    H = fit_inputs(ev)
    so, sg = _seed_both(kf, w.geometry, H, n)
    _assert_seed_parity(so, sg, n)
    o = oracle.fit(w.geometry, 3, H, so["par"], so["cov"], so["q"], n)
    g = kf.kf_fit(w.geometry, n, 3, to_dev(H), to_dev(sg["par"]), to_dev(sg["cov"]), to_dev(sg["q"]),
                  arith=kf.ARITH_F64)
    g = {k: host(v) for k, v in g.items()}
    errs = assert_fit_parity_converged(g, o, n, "fit_small f64")
    print("fit_small parity (f64 arithmetic)", errs)


def test_fit_fp32_arithmetic_agreement(kf):
    """FP32 arithmetic (hardware reciprocals, 1 ulp): tracks whose seed is
    well conditioned (relative momentum uncertainty below 0.1) within the
    tolerances but for a rare rounding casualty (at most 1 in 1000); the
    agreement fraction over all tracks is reported."""
    w = presets.fit_scale()
    ev = datagen.generate(w.geometry, w.gen, 1, 20000)
    n = ev.n_tracks
    H = fit_inputs(ev)
    so, sg = _seed_both(kf, w.geometry, H, n)
    o = oracle.fit(w.geometry, 3, H, so["par"], so["cov"], so["q"], n)
    g = kf.kf_fit(w.geometry, n, 3, to_dev(H), to_dev(sg["par"]), to_dev(sg["cov"]), to_dev(sg["q"]),
                  arith=kf.ARITH_F32)
    g = {k: host(v) for k, v in g.items()}
    agree = fit_agreement(g, o, n)
    well = seed_rel_sigma_p(so["par"], so["cov"], n) < 0.1
    print(f"fp32 arithmetic: agreement {agree.mean():.4f} overall, {agree[well].mean():.4f} on "
          f"{well.mean():.3f} well-conditioned seeds")
    assert agree[well].mean() >= 0.999
    # FP32 arithmetic meets the tolerances on well-conditioned seeds only; over
    # all tracks it agrees on 0.8895 (measured), FP64 arithmetic is the parity
    # mode
    assert agree.mean() >= 0.87


@pytest.mark.parametrize("n", [1, 63, 64, 65, 777])
def test_fit_ragged_sizes(kf, n):
    w = presets.fit_scale()
    ev = datagen.generate(w.geometry, w.gen, 3, n)
    H = fit_inputs(ev)
    so, sg = _seed_both(kf, w.geometry, H, n)
    _assert_seed_parity(so, sg, n)
    o = oracle.fit(w.geometry, 3, H, so["par"], so["cov"], so["q"], n)
    g = kf.kf_fit(w.geometry, n, 3, to_dev(H), to_dev(sg["par"]), to_dev(sg["cov"]), to_dev(sg["q"]),
                  arith=kf.ARITH_F64)
    assert_fit_parity_converged({k: host(v) for k, v in g.items()}, o, n, f"n={n}")


def test_fit_zero_noise_returns_generating_helix(kf):
    w = presets.fit_scale()
    g0 = w.geometry.replace(x_over_x0=0.0)
    gen = dataclasses.replace(w.gen, smear=False, vtx_sxy=0.0)
    ev = datagen.generate(g0, gen, 0, 2000, truth=True)
    n = ev.n_tracks
    H = fit_inputs(ev)
    sg = kf.kf_seed(g0, n, to_dev(H))
    g = kf.kf_fit(g0, n, 3, to_dev(H), sg["par"], sg["cov"], sg["q"], arith=kf.ARITH_F32)
    par = host(g["par"])[:, :n].astype(np.float64)
    tr = ev.truth[-1]
    ep = np.linalg.norm(par[:3] - tr[:3], axis=0) / np.linalg.norm(tr[:3], axis=0)
    # FP32 inputs: hits are off the helix by one rounding; momentum from a
    # three-point curvature amplifies that at high pT, so use low pT for p
    pt = np.hypot(ev.vertex[3], ev.vertex[4])
    em = np.linalg.norm(par[3:] - tr[3:], axis=0) / np.linalg.norm(tr[3:], axis=0)
    assert ep.max() < 1e-5
    assert em[pt < 2].max() < 1e-4
    assert host(g["chi2"])[:n].max() < 1e-2


def test_fit_status_paths(kf):
    w = presets.fit_small()
    ev = datagen.generate(w.geometry, w.gen, 0, 128)
    n = ev.n_tracks
    H = fit_inputs(ev)
    so = oracle.seed(w.geometry, H, n)
    sp = so["par"].copy()
    sp[3:6, 0] = np.float32([0.01, 0.0, 0.0])  # cannot reach the next layer
    sp[0:3, 0] = np.float32([12.0, 0.0, 0.0])
    H[5, 0, 1] = np.nan  # non-finite hit on layer 5
    sp[2, 2] = np.float32(99.9)  # leaves the barrel in z
    sp[5, 2] = np.float32(50.0)
    hm = np.zeros(H.shape[2], dtype=np.uint32)
    hm[3] = (1 << 4) | (1 << 8)
    o = oracle.fit(w.geometry, 3, H, sp, so["cov"], so["q"], n, hole_mask=hm)
    g = kf.kf_fit(w.geometry, n, 3, to_dev(H), to_dev(sp), to_dev(so["cov"]), to_dev(so["q"]),
                  hole_mask=to_dev(hm.view(np.int32)), arith=kf.ARITH_F64)
    gh = {k: host(v) for k, v in g.items()}
    assert gh["status"][0] == oracle.TRK_NO_CROSSING
    assert gh["status"][1] == oracle.TRK_NONFINITE
    assert gh["status"][2] == oracle.TRK_OUT_OF_Z
    assert gh["ndof"][3] == 2 * (w.geometry.n_layers - 5)
    assert_fit_parity_converged(gh, o, n, "status paths")


@pytest.mark.parametrize("hybrid", [False, True])
def test_fit_empty_and_invalid(kf, hybrid):
    w = presets.fit_small()
    fit = kf.kf_fit_hybrid if hybrid else kf.kf_fit
    H = torch.zeros((10, 9, 64), dtype=torch.float32, device=DEV)
    sp = torch.zeros((6, 64), device=DEV)
    sc = torch.zeros((21, 64), device=DEV)
    q = torch.ones(64, dtype=torch.int8, device=DEV)
    fit(w.geometry, 0, 3, H, sp, sc, q)  # n = 0: nothing to do
    with pytest.raises(kf.KFError):
        fit(w.geometry, -1, 3, H, sp, sc, q)
    with pytest.raises(kf.KFError):
        fit(w.geometry, 10, 11, H, sp, sc, q)
    bad = w.geometry.replace(bz=0.0)
    with pytest.raises(kf.KFError):
        fit(bad, 10, 3, H, sp, sc, q)
    with pytest.raises(kf.KFError):
        fit(w.geometry, 10, 3, H, sp, sc, q, arith=7)
    if hybrid:
        # a zero seed (no momentum) has no hybrid state: flagged, not crashed
        out = fit(w.geometry, 10, 3, H, sp, sc, q)
        torch.cuda.synchronize()
        assert np.all(host(out["status"])[:10] & kf.TRK_NONFINITE)
