"""Oracle pins for multiple scattering and the Kalman update."""
import dataclasses

import numpy as np

import oracle
from paper_1711_06571_amd import datagen, presets


def test_highland_width_against_generator_kicks():
    """Sample covariance of the simulated scattering kicks (the generator's own
    code) vs the oracle's process noise, at normal incidence, 1 GeV pions."""
    geom = presets.barrel(2)
    gen = dataclasses.replace(presets.GenSettings(seed=99), pt_min=1.0, pt_max=1.0, eta_max=0.0, smear=False,
                              vtx_sxy=0.0, vtx_sz=0.0)
    n = 400_000
    ev = datagen.generate(geom, gen, 0, n, truth=True)
    # all tracks share pT and eta and start at the origin; the pre-kick
    # momentum is the vertex momentum turned by one angle per charge
    p_after = ev.truth[0, 3:]  # (3, n)
    # rotation angle of the momentum from vertex to layer 0 (same for all tracks of one charge)
    dth = {}
    for qq in (1, -1):
        t = int(np.where(ev.q == qq)[0][0])
        rc, Xo, _, _ = oracle.propagate(ev.vertex[:, t], qq, geom.r[0], geom.bz)
        a0 = np.arctan2(ev.vertex[4, t], ev.vertex[3, t])
        dth[qq] = np.arctan2(Xo[4], Xo[3]) - a0
    a = np.arctan2(ev.vertex[4], ev.vertex[3]) + np.where(ev.q == 1, dth[1], dth[-1])
    u = np.stack([np.cos(a), np.sin(a), np.zeros(n)])  # unit pre-kick direction (eta = 0)
    e1 = np.stack([-np.sin(a), np.cos(a), np.zeros(n)])
    e2 = np.stack([np.zeros(n), np.zeros(n), np.ones(n)])
    p = 1.0
    k1 = (p_after * e1).sum(0) / p
    k2 = (p_after * e2).sum(0) / p
    # oracle theta0^2 = trace(Q) / (2 |p|^2) at the crossing state
    Xs = np.array([geom.r[0], 0.0, 0.0, 1.0, 0.0, 0.0])
    Q = oracle.ms_cov(Xs, geom.x_over_x0, geom.mass)
    th2 = np.trace(Q) / 2.0
    assert abs(np.var(k1) / th2 - 1) < 0.01
    assert abs(np.var(k2) / th2 - 1) < 0.01
    assert abs(np.mean(k1 * k2)) < 0.01 * th2
    # Q annihilates the momentum direction and is PSD
    assert np.abs(Q @ Xs).max() < 1e-18
    assert np.linalg.eigvalsh(Q).min() > -1e-18


def test_highland_closed_form_values():
    """theta0 = 13.6 MeV/(beta c p) sqrt(x/X0) (1 + 0.038 ln(x/(X0 beta^2)))
    (PDG), evaluated by hand for three (p, psi) points: x/X0 = 0.02, pion."""
    m = 0.13957
    cases = [  # p [GeV], incidence psi [rad], theta0 [rad] evaluated separately
        (1.0, 0.0, 0.001654709159),
        (0.5, 0.0, 0.003411408229),
        (2.0, np.pi / 4, 0.0009912896166),
    ]
    for p, psi, th_expected in cases:
        X = np.array([10.0, 0.0, 0.0, p * np.cos(psi), p * np.sin(psi), 0.0])
        Q = oracle.ms_cov(X, 0.02, m)
        th = np.sqrt(np.trace(Q) / (2 * p * p))
        assert abs(th / th_expected - 1) < 1e-9, (p, psi, th)


def _rand_spd(rng, n=6, scale=None):
    A = rng.normal(size=(n, n))
    P = A @ A.T + n * np.eye(n)
    if scale is not None:
        D = np.diag(scale)
        P = D @ P @ D
    return P


def _state_on_cylinder(rng, R=20.0):
    ph = rng.uniform(0, 2 * np.pi)
    return np.array([R * np.cos(ph), R * np.sin(ph), rng.uniform(-20, 20),
                     rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(-3, 3)])


def _hit_near(rng, X, srphi=0.01, sz=0.1):
    R = np.hypot(X[0], X[1])
    ph = np.arctan2(X[1], X[0]) + rng.normal(0, 0.05) / R
    t = np.array([-np.sin(ph), np.cos(ph), 0.0])
    V = srphi ** 2 * np.outer(t, t)
    V[2, 2] = sz ** 2
    return np.array([R * np.cos(ph), R * np.sin(ph), X[2] + rng.normal(0, 0.3),
                     V[0, 0], V[0, 1], V[0, 2], V[1, 1], V[1, 2], V[2, 2]])


def _frame(X, hit):
    r = np.hypot(X[0], X[1])
    t = np.array([-X[1] / r, X[0] / r, 0.0])
    H = np.zeros((2, 6))
    H[0, :3] = t
    H[1, 2] = 1.0
    V = np.array([[hit[3], hit[4], hit[5]], [hit[4], hit[6], hit[7]], [hit[5], hit[7], hit[8]]])
    F = np.array([t, [0, 0, 1.0]])
    V2 = F @ V @ F.T
    res = np.array([t @ (hit[:3] - X[:3]), hit[2] - X[2]])
    return H, V2, res


def test_update_scalar_weighted_mean(rng):
    """No correlations: each measured coordinate becomes the inverse-variance
    weighted mean of prediction and hit (textbook one-dimensional case)."""
    X = np.array([20.0, 0.0, 3.0, 1.0, 0.5, 0.2])
    P = np.diag([1e-3, 4e-4, 2e-2, 1e-2, 1e-2, 1e-2])
    hit = np.array([20.0, 0.02, 3.1, 0, 0, 0, 1e-4, 0, 1e-2])  # on the tangent at (20, 0)
    rc, Xo, Po, c2 = oracle.update(X, P, hit)
    assert rc == 0
    w = 4e-4 / (4e-4 + 1e-4)
    assert np.isclose(Xo[1], 0.0 + w * 0.02, rtol=1e-14)
    assert np.isclose(Po[1, 1], 4e-4 * 1e-4 / (4e-4 + 1e-4), rtol=1e-13)
    wz = 2e-2 / (2e-2 + 1e-2)
    assert np.isclose(Xo[2], 3.0 + wz * 0.1, rtol=1e-14)
    assert np.isclose(Po[2, 2], 2e-2 * 1e-2 / 3e-2, rtol=1e-13)
    assert np.isclose(c2, 0.02 ** 2 / 5e-4 + 0.1 ** 2 / 3e-2, rtol=1e-13)
    assert Xo[0] == X[0] and np.array_equal(Xo[3:], X[3:])


def test_update_information_form_and_joseph(rng):
    for _ in range(50):
        X = _state_on_cylinder(rng)
        P = _rand_spd(rng, scale=np.array([0.1, 0.1, 0.3, 0.05, 0.05, 0.05]))
        hit = _hit_near(rng, X)
        rc, Xo, Po, c2 = oracle.update(X, P, hit)
        assert rc == 0
        H, V2, res = _frame(X, hit)
        # information form: Po^-1 = P^-1 + H^T V2^-1 H
        lhs = np.linalg.inv(Po)
        rhs = np.linalg.inv(P) + H.T @ np.linalg.inv(V2) @ H
        assert np.allclose(lhs, rhs, rtol=1e-8, atol=1e-8 * np.abs(rhs).max())
        # Joseph form equals the standard form
        S = H @ P @ H.T + V2
        K = P @ H.T @ np.linalg.inv(S)
        I = np.eye(6)
        Pj = (I - K @ H) @ P @ (I - K @ H).T + K @ V2 @ K.T
        assert np.allclose(Pj, Po, rtol=1e-10, atol=1e-12 * np.abs(P).max())
        # chi2 identity: predicted form = posterior residual + state-change form
        post = res - H @ (Xo - X)
        c2b = post @ np.linalg.inv(V2) @ post + (Xo - X) @ np.linalg.inv(P) @ (Xo - X)
        assert np.isclose(c2, c2b, rtol=1e-8)


def test_update_keeps_radial_null_vector(rng):
    for _ in range(20):
        X = _state_on_cylinder(rng)
        n = np.array([X[0], X[1], 0, 0, 0, 0]) / np.hypot(X[0], X[1])
        B = np.linalg.svd(np.eye(6) - np.outer(n, n))[0][:, :5]
        A = rng.normal(size=(5, 5))
        P = B @ (A @ A.T + np.eye(5)) @ B.T * 0.01
        hit = _hit_near(rng, X)
        rc, Xo, Po, c2 = oracle.update(X, P, hit)
        assert rc == 0
        assert np.abs(Po @ n).max() < 1e-14 * np.abs(Po).max()
        ev = np.linalg.eigvalsh(Po)
        assert ev.min() > -1e-14 * ev.max() and np.sort(ev)[1] > 0


def test_update_rejects_non_positive_S():
    X = np.array([20.0, 0.0, 3.0, 1.0, 0.5, 0.2])
    P = np.zeros((6, 6))
    hit = np.array([20.0, 0.0, 3.0, 0, 0, 0, 0, 0, 0])
    rc, _, _, _ = oracle.update(X, P, hit)
    assert rc == oracle.TRK_S_NOT_PD
