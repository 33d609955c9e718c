"""Oracle pins for propagation (helix in a uniform solenoidal field, crossing
with a cylinder) and its Jacobian.  The pins are independent of the oracle's
closed form: numerical integration of the Lorentz force, bisection, finite
differences, reversibility and the straight-line limit."""
import numpy as np
import pytest

import oracle

KAPPA = 0.299792458e-2
BZ = float(np.float32(3.8))


def _random_states(rng, n, r0=4.0):
    """States on the cylinder r = r0, moving outward, pT in [0.5, 10]."""
    out = []
    while len(out) < n:
        ph = rng.uniform(0, 2 * np.pi)
        pt = rng.uniform(0.5, 10)
        dirn = ph + rng.uniform(-0.6, 0.6)
        pz = pt * np.sinh(rng.uniform(-1, 1))
        out.append(np.array([r0 * np.cos(ph), r0 * np.sin(ph), rng.uniform(-10, 10),
                             pt * np.cos(dirn), pt * np.sin(dirn), pz]))
    return np.array(out)


def _rk4_lorentz(X, q, bz, S, nstep):
    """Integrate dx/dS = p/|p|, dp/dS = q*KAPPA*(p/|p|) x B over 3-D path S."""
    x = X[:3].astype(float).copy()
    p = X[3:].astype(float).copy()
    h = S / nstep
    B = np.array([0.0, 0.0, bz])

    def f(x, p):
        u = p / np.linalg.norm(p)
        return u, q * KAPPA * np.cross(u, B)

    for _ in range(nstep):
        k1x, k1p = f(x, p)
        k2x, k2p = f(x + 0.5 * h * k1x, p + 0.5 * h * k1p)
        k3x, k3p = f(x + 0.5 * h * k2x, p + 0.5 * h * k2p)
        k4x, k4p = f(x + h * k3x, p + h * k3p)
        x = x + h / 6 * (k1x + 2 * k2x + 2 * k3x + k4x)
        p = p + h / 6 * (k1p + 2 * k2p + 2 * k3p + k4p)
    return np.concatenate([x, p])


def test_helix_matches_lorentz_force_integration(rng):
    for X in _random_states(rng, 6):
        for q in (1, -1):
            rc, Xo, s, _ = oracle.propagate(X, q, 40.0, BZ)
            assert rc == 0
            pt = np.hypot(X[3], X[4])
            S = s * np.linalg.norm(X[3:]) / pt  # 3-D path length
            Xr = _rk4_lorentz(X, q, BZ, S, 4000)
            assert np.allclose(Xr[:3], Xo[:3], rtol=0, atol=1e-9)
            assert np.allclose(Xr[3:], Xo[3:], rtol=1e-10, atol=1e-12)


def test_crossing_is_first_root_by_bisection(rng):
    for X in _random_states(rng, 20):
        q = 1 if rng.uniform() < 0.5 else -1
        R = 36.0
        rc, Xo, s, _ = oracle.propagate(X, q, R, BZ)
        assert rc == 0
        assert abs(np.hypot(Xo[0], Xo[1]) - R) <= 1e-12 * R

        def rad(t):
            Y = oracle.state_at(X, q, BZ, t)
            return np.hypot(Y[0], Y[1]) - R
        # scan for the first sign change of r(t) - R, then bisect
        ts = np.linspace(0, 400, 40001)
        vals = np.array([rad(t) for t in ts[:4000]])
        k = int(np.argmax(vals > 0))
        assert k > 0
        lo, hi = ts[k - 1], ts[k]
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if rad(mid) > 0:
                hi = mid
            else:
                lo = mid
        assert abs(0.5 * (lo + hi) - s) <= 1e-11 * R


def test_reversibility(rng):
    for X in _random_states(rng, 20):
        q = 1 if rng.uniform() < 0.5 else -1
        rc, Xo, _, _ = oracle.propagate(X, q, 60.0, BZ)
        assert rc == 0
        back = Xo.copy()
        back[3:] *= -1
        rc, Xb, _, _ = oracle.propagate(back, -q, 4.0, BZ)
        assert rc == 0
        assert np.allclose(Xb[:3], X[:3], rtol=0, atol=1e-9)
        assert np.allclose(-Xb[3:], X[3:], rtol=1e-10, atol=1e-12)


def test_straight_line_limit(rng):
    # at bz = 1e-5 T the radius of curvature exceeds 1e7 cm; the sagitta over
    # the path is below 1e-5 cm, so the crossing approaches the line-circle one
    bz = 1e-5
    for X in _random_states(rng, 10):
        rc, Xo, s, _ = oracle.propagate(X, 1, 50.0, bz)
        assert rc == 0
        pt = np.hypot(X[3], X[4])
        t = X[3:5] / pt
        b = X[0:2] @ t
        c = X[0:2] @ X[0:2] - 50.0 ** 2
        sl = -b + np.sqrt(b * b - c)
        assert abs(s - sl) < 1e-4
        assert np.allclose(Xo[:2], X[0:2] + sl * t, atol=1e-4)
        assert abs(Xo[2] - (X[2] + X[5] / pt * sl)) < 1e-4


def test_no_crossing_for_curlers():
    # pT = 0.1 GeV: 2 rho = 17.5 cm < 40 cm, the circle never reaches r = 40
    X = np.array([4.0, 0.0, 0.0, 0.1, 0.0, 0.0])
    rc, _, _, _ = oracle.propagate(X, 1, 40.0, BZ)
    assert rc == oracle.TRK_NO_CROSSING


def _prop_end(X, q, R):
    rc, Xo, _, _ = oracle.propagate(X, q, R, BZ)
    assert rc == 0
    return Xo


def test_jacobian_matches_central_differences(rng):
    for X in _random_states(rng, 12):
        q = 1 if rng.uniform() < 0.5 else -1
        R = 28.0
        rc, Xo, s, _ = oracle.propagate(X, q, R, BZ)
        J = oracle.jacobian(X, q, BZ, s)
        Jn = np.zeros((6, 6))
        for j in range(6):
            h = 1e-6 * max(abs(X[j]), 1.0)
            d = np.zeros(6)
            d[j] = h
            Jn[:, j] = (_prop_end(X + d, q, R) - _prop_end(X - d, q, R)) / (2 * h)
        scale = np.maximum(np.abs(Jn).max(axis=1, keepdims=True), 1e-3)
        assert np.all(np.abs(J - Jn) / scale < 1e-7), np.abs(J - Jn) / scale
        # the radial direction at the crossing is a left null vector
        n = np.array([Xo[0], Xo[1], 0, 0, 0, 0]) / np.hypot(Xo[0], Xo[1])
        assert np.abs(n @ J).max() < 1e-12 * np.abs(J).max()
