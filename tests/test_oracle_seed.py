"""Oracle pins for the beam-spot part of the seed convention: the impact
parameter function is the distance of closest approach of the helix to the z
axis (brute force along the helix), its gradient matches central finite
differences, it vanishes for tracks generated from the axis, and the
constraint does what it is for (fewer seeds with the wrong charge)."""
import dataclasses

import numpy as np

import oracle
from paper_1711_06571_amd import datagen, presets


def _random_states(rng, n, bz):
    out = []
    for _ in range(n):
        phi = rng.uniform(0, 2 * np.pi)
        r = rng.uniform(4.0, 40.0)
        pt = rng.uniform(0.5, 10.0)
        dirn = phi + rng.uniform(-0.5, 0.5)
        X = np.array([r * np.cos(phi), r * np.sin(phi), rng.uniform(-50, 50), pt * np.cos(dirn), pt * np.sin(dirn),
                      pt * rng.uniform(-1.2, 1.2)])
        out.append((X, int(rng.choice([-1, 1]))))
    return out


def _closest_approach(X, q, bz):
    """Smallest transverse distance of the helix from the z axis, by a grid
    over the transverse path and golden-section refinement (both directions
    of motion, one full turn)."""
    pt = np.hypot(X[3], X[4])
    rho = pt / (0.299792458e-2 * abs(bz))
    L = 2 * np.pi * rho
    ss = np.linspace(-L, L, 20001)
    rr = np.array([np.hypot(*oracle.state_at(X, q, bz, s)[:2]) for s in ss])
    k = int(np.argmin(rr))
    a, b = ss[max(k - 1, 0)], ss[min(k + 1, len(ss) - 1)]
    f = lambda s: np.hypot(*oracle.state_at(X, q, bz, s)[:2])
    gr = (np.sqrt(5) - 1) / 2
    for _ in range(200):
        c, d = b - gr * (b - a), a + gr * (b - a)
        if f(c) < f(d):
            b = d
        else:
            a = c
    return f(0.5 * (a + b))


def test_beam_d0_is_distance_of_closest_approach():
    rng = np.random.default_rng(7)
    bz = 3.8
    for X, q in _random_states(rng, 12, bz):
        rc, f, _ = oracle.beam_d0(X, q, bz)
        assert rc == 0
        assert abs(abs(f) - _closest_approach(X, q, bz)) < 1e-7


def test_beam_d0_gradient_matches_finite_differences():
    rng = np.random.default_rng(8)
    bz = 3.8
    for X, q in _random_states(rng, 20, bz):
        rc, f, H = oracle.beam_d0(X, q, bz)
        num = np.zeros(6)
        for j in range(6):
            h = 1e-6 * max(1.0, abs(X[j]))
            Xp, Xm = X.copy(), X.copy()
            Xp[j] += h
            Xm[j] -= h
            num[j] = (oracle.beam_d0(Xp, q, bz)[1] - oracle.beam_d0(Xm, q, bz)[1]) / (2 * h)
        assert np.allclose(H, num, rtol=1e-6, atol=1e-8), (H, num)
        assert H[2] == 0.0 and H[5] == 0.0


def test_beam_d0_vanishes_for_tracks_from_the_axis():
    """Without material the generated helix is the one that left the axis."""
    w = presets.build()
    g = w.geometry.replace(x_over_x0=0.0)
    gen = dataclasses.replace(w.gen, vtx_sxy=0.0)
    ev = datagen.generate(g, gen, 5, 300, truth=True)
    for l in (0, 2, 9):
        T = ev.truth[l]
        d = [oracle.beam_d0(T[:, i], int(ev.q[i]), g.bz)[1] for i in range(ev.n_tracks)]
        assert np.abs(d).max() < 1e-9


def test_beam_spot_reduces_wrong_charge_seeds():
    """At high pT the sagitta over hits 0..2 is comparable to the hit
    resolution; the beam line doubles the lever arm."""
    w = presets.build()
    ev = datagen.generate(w.geometry, w.gen, 6, 3000)
    H = datagen.track_hits(ev)
    n = ev.n_tracks
    wrong_beam = np.mean(oracle.seed(w.geometry, H, n)["q"][:n] != ev.q)
    wrong_three = np.mean(oracle.seed(w.geometry, H, n, beam_sigma=0.0)["q"][:n] != ev.q)
    assert wrong_beam < 0.035 and wrong_three > 0.06, (wrong_beam, wrong_three)
