"""Oracle pins for the hybrid state (Cartesian position, polar momentum
(q/pT, phi, theta)): the changes of variables and their Jacobians against
round trips and central differences, the linearised prediction against
central differences of the propagation map, zero-noise exactness of the fit,
consistency with the Cartesian fit where both linearisations agree, and the
reason for the state: a seed of the wrong charge can be corrected."""
import dataclasses

import numpy as np

import oracle
from paper_1711_06571_amd import datagen, presets

from conftest import full_from_upper


def _random_cart(rng, n):
    X = np.zeros((n, 6))
    phi = rng.uniform(-np.pi, np.pi, n)
    r = rng.uniform(4, 60, n)
    X[:, 0], X[:, 1], X[:, 2] = r * np.cos(phi), r * np.sin(phi), rng.uniform(-50, 50, n)
    pt = rng.uniform(0.5, 10, n)
    pphi = phi + rng.normal(0, 0.3, n)
    eta = rng.uniform(-1, 1, n)
    X[:, 3], X[:, 4], X[:, 5] = pt * np.cos(pphi), pt * np.sin(pphi), pt * np.sinh(eta)
    q = rng.choice([-1, 1], n)
    return X, q


def test_round_trip_and_definitions():
    rng = np.random.default_rng(11)
    X, q = _random_cart(rng, 200)
    for i in range(200):
        Y = oracle.hyb_from_cart(X[i], q[i])
        pt = np.hypot(X[i, 3], X[i, 4])
        assert abs(Y[3] - q[i] / pt) <= 1e-15 * abs(Y[3])
        assert abs(np.cos(Y[4]) * pt - X[i, 3]) < 1e-12 and abs(np.sin(Y[4]) * pt - X[i, 4]) < 1e-12
        p = np.linalg.norm(X[i, 3:])
        assert abs(np.cos(Y[5]) * p - X[i, 5]) < 1e-12 * p
        Xb, qb = oracle.cart_from_hyb(Y)
        assert qb == q[i]
        assert np.allclose(Xb, X[i], rtol=1e-13, atol=1e-12)


def test_change_of_variable_jacobians():
    rng = np.random.default_rng(12)
    X, q = _random_cart(rng, 40)
    for i in range(40):
        Y = oracle.hyb_from_cart(X[i], q[i])
        A, B = oracle.hyb_jacobians(Y)
        # central differences of both maps
        FA = np.zeros((6, 6))
        FB = np.zeros((6, 6))
        for j in range(6):
            h = 1e-6 * max(1.0, abs(Y[j]))
            e = np.zeros(6)
            e[j] = h
            FA[:, j] = (oracle.cart_from_hyb(Y + e)[0] - oracle.cart_from_hyb(Y - e)[0]) / (2 * h)
            h = 1e-6 * max(1.0, abs(X[i, j]))
            e = np.zeros(6)
            e[j] = h
            FB[:, j] = (oracle.hyb_from_cart(X[i] + e, q[i]) - oracle.hyb_from_cart(X[i] - e, q[i])) / (2 * h)
        assert np.allclose(A, FA, rtol=1e-6, atol=1e-8 * np.abs(FA).max())
        assert np.allclose(B, FB, rtol=1e-6, atol=1e-8 * np.abs(FB).max())
        # inverse maps: inverse Jacobians
        assert np.allclose(B @ A, np.eye(6), atol=1e-10)


def test_prediction_linearisation_matches_differences():
    """Without material, the predicted covariance of P = I is J J^T with J
    the central-difference Jacobian of the map Y -> predicted Y."""
    g = presets.fit_scale().geometry.replace(x_over_x0=0.0)
    rng = np.random.default_rng(13)
    X, q = _random_cart(rng, 30)
    done = 0
    for i in range(30):
        X[i, :2] *= 4.0 / np.hypot(X[i, 0], X[i, 1])  # start on the first layer
        Y = oracle.hyb_from_cart(X[i], q[i])
        rc, Yo, Po = oracle.predict_hyb(g, 3, Y, np.eye(6))
        if rc:
            continue
        J = np.zeros((6, 6))
        ok = True
        for j in range(6):
            h = 1e-7 * max(1.0, abs(Y[j]))
            e = np.zeros(6)
            e[j] = h
            r1, Y1, _ = oracle.predict_hyb(g, 3, Y + e, np.zeros((6, 6)))
            r2, Y2, _ = oracle.predict_hyb(g, 3, Y - e, np.zeros((6, 6)))
            ok = ok and r1 == 0 and r2 == 0
            d = Y1 - Y2
            d[4] = (d[4] + np.pi) % (2 * np.pi) - np.pi
            J[:, j] = d / (2 * h)
        if not ok:
            continue
        assert np.allclose(Po, J @ J.T, rtol=2e-5, atol=2e-6 * np.abs(Po).max())
        done += 1
    assert done >= 20


def _zero_noise_event(w, n):
    gen = dataclasses.replace(w.gen, smear=False, vtx_sxy=0.0)
    g = w.geometry.replace(x_over_x0=0.0)
    return g, datagen.generate(g, gen, 0, n, truth=True)


def test_zero_noise_hybrid_fit_returns_generating_helix():
    w = presets.fit_scale()
    g, ev = _zero_noise_event(w, 300)
    n = ev.n_tracks
    H = datagen.track_hits(ev, dtype=np.float64)
    sd = oracle.seed64(g, H, n)
    o = oracle.fit_hybrid64(g, 3, H, sd["par64"], sd["cov64"], sd["q"], n)
    assert np.all(o["status"][:n] == 0)
    tr = ev.truth[-1]
    for i in range(n):
        Yt = oracle.hyb_from_cart(tr[:, i], ev.q[i])
        d = o["par"][:, i] - Yt
        d[4] = (d[4] + np.pi) % (2 * np.pi) - np.pi
        assert np.all(np.abs(d[:3]) < 1e-9 * 70) and abs(d[3]) < 1e-9 * abs(Yt[3]) and np.all(np.abs(d[4:]) < 1e-9)
    assert o["chi2"][:n].max() < 1e-12


def test_hybrid_and_cartesian_fits_agree_on_well_measured_tracks():
    """Both filters linearise the same model; on tracks whose seed is well
    measured they reach the same estimate within a fraction of its error
    (the linearisations differ at second order)."""
    w = presets.fit_scale()
    ev = datagen.generate(w.geometry, w.gen, 3, 600, truth=True)
    n = ev.n_tracks
    H = datagen.track_hits(ev)
    sd = oracle.seed(w.geometry, H, n)
    oc = oracle.fit(w.geometry, 3, H, sd["par"], sd["cov"], sd["q"], n)
    oh = oracle.fit_hybrid(w.geometry, 3, H, sd["par"], sd["cov"], sd["q"], n)
    # well-measured seeds: momentum error below 10 % of the momentum
    Ps = full_from_upper(sd["cov"][:, :n].astype(np.float64))
    p = np.linalg.norm(sd["par"][3:, :n].astype(np.float64), axis=0)
    well = np.sqrt(np.trace(Ps[:, 3:, 3:], axis1=1, axis2=2)) < 0.1 * p
    ok = well & (oc["status"][:n] == 0) & (oh["status"][:n] == 0) & (oc["chi2"][:n] < 3 * oc["ndof"][:n])
    assert ok.sum() > 50
    Pc = full_from_upper(oh["cov"][:, :n])
    diffs = []
    for i in np.where(ok)[0]:
        Yc = oracle.hyb_from_cart(oc["par"][:, i], 1 if oh["par"][3, i] > 0 else -1)
        d = oh["par"][:, i] - Yc
        d[4] = (d[4] + np.pi) % (2 * np.pi) - np.pi
        sig = np.sqrt(np.maximum(np.diag(Pc[i]), 1e-30))
        diffs.append(np.abs(d[3:]) / sig[3:])
    diffs = np.array(diffs)
    print(f"hybrid vs Cartesian fit, momentum difference / sigma: median {np.median(diffs):.3f}, "
          f"99 % {np.percentile(diffs, 99):.3f}")
    assert np.median(diffs) < 0.05 and np.percentile(diffs, 99) < 1.0


def test_wrong_charge_seed_is_corrected():
    """High-pT tracks seeded with the wrong charge (same momentum vector,
    seed covariance broad in curvature): the hybrid fit moves q/pT through
    zero to the true sign, which a fixed-charge Cartesian state cannot."""
    w = presets.fit_scale()
    g = w.geometry
    gen = dataclasses.replace(w.gen, pt_min=6.0, pt_max=10.0)
    ev = datagen.generate(g, gen, 4, 300, truth=True)
    n = ev.n_tracks
    H = datagen.track_hits(ev)
    sd = oracle.seed(g, H, n)
    # the truth at layer 2 with the opposite charge, and a covariance broad
    # enough in curvature to allow the flip: the seed's own, with the momentum
    # block inflated to (|p|)^2 in every direction
    par = np.zeros_like(sd["par"])
    cov = np.array(sd["cov"])
    par[:, :n] = ev.truth[2].astype(np.float32)
    qf = np.zeros_like(sd["q"])
    qf[:n] = -ev.q
    P = full_from_upper(cov[:, :n].astype(np.float64))
    p2 = (ev.truth[2][3:] ** 2).sum(axis=0)
    for i in range(n):
        P[i, 3:, 3:] += np.eye(3) * p2[i]
    iu = np.triu_indices(6)
    cov[:, :n] = P[:, iu[0], iu[1]].T.astype(np.float32)
    oh = oracle.fit_hybrid(g, 3, H, par, cov, qf, n)
    oc = oracle.fit(g, 3, H, par, cov, qf, n)
    okh = oh["status"][:n] == 0
    right = np.sign(oh["par"][3, :n]) == ev.q
    good_h = okh & right & (oh["chi2"][:n] < 3 * np.maximum(oh["ndof"][:n], 1))
    good_c = (oc["status"][:n] == 0) & (oc["chi2"][:n] < 3 * np.maximum(oc["ndof"][:n], 1))
    print(f"wrong-charge seeds: hybrid corrected {good_h.mean():.3f}, Cartesian acceptable {good_c.mean():.3f}")
    assert good_h.mean() > 0.8
    assert good_h.mean() > good_c.mean() + 0.3
