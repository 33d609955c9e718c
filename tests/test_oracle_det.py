"""Oracle pins for the general detector (section 4.1): endcap disks (the
"cylinder with lids") and modules off a layer's average surface, with the
two-step propagation of track building.  Each pin is independent of the
closed forms it checks: numerical integration of the Lorentz force,
bisection, finite differences, composition of steps, textbook special cases
of the update, exact recovery of noise-free tracks, chi2 statistics and
exhaustive search on tiny events."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1711_06571_amd import datagen, presets

from conftest import full_from_upper, upper_from_full
from test_oracle_helix import BZ, _rk4_lorentz

TWO_PI = 2 * np.pi


def _states_on_cylinder(rng, n, R=20.0, eta=(0.6, 2.0)):
    """States on r = R moving outward and forward in z (pz > 0)."""
    out = []
    for _ in range(n):
        ph = rng.uniform(0, TWO_PI)
        pt = rng.uniform(0.5, 10)
        d = ph + rng.uniform(-0.5, 0.5)
        out.append(np.array([R * np.cos(ph), R * np.sin(ph), rng.uniform(20, 40), pt * np.cos(d), pt * np.sin(d),
                             pt * np.sinh(rng.uniform(*eta))]))
    return out


def test_plane_crossing_matches_lorentz_force_integration(rng):
    for X in _states_on_cylinder(rng, 6):
        for q in (1, -1):
            Z = 70.0
            s = oracle.plane_path(X, Z)
            assert s is not None and s > 0
            Xo = oracle.state_at(X, q, BZ, s)
            assert abs(Xo[2] - Z) <= 1e-12 * Z
            S = s * np.linalg.norm(X[3:]) / np.hypot(X[3], X[4])
            Xr = _rk4_lorentz(X, q, BZ, S, 4000)
            assert np.allclose(Xr[:3], Xo[:3], rtol=0, atol=1e-9)
            assert np.allclose(Xr[3:], Xo[3:], rtol=1e-10, atol=1e-12)
            # a plane behind the track has no forward crossing; the nearest
            # crossing goes backwards
            assert oracle.plane_path(X, X[2] - 5.0) is None
            sb = oracle.plane_path(X, X[2] - 5.0, nearest=True)
            assert sb < 0 and abs(oracle.state_at(X, q, BZ, sb)[2] - (X[2] - 5.0)) < 1e-12 * 40


def test_nearest_cylinder_crossing_by_bisection_and_reversibility(rng):
    for X in _states_on_cylinder(rng, 10):
        q = 1 if rng.uniform() < 0.5 else -1
        for R in (19.5, 20.5):
            s = oracle.cyl_path(X, q, R, BZ, nearest=True)
            assert s is not None and (s < 0) == (R < 20.0)
            Xo = oracle.state_at(X, q, BZ, s)
            assert abs(np.hypot(Xo[0], Xo[1]) - R) <= 1e-12 * R

            def f(t):
                Y = oracle.state_at(X, q, BZ, t)
                return np.hypot(Y[0], Y[1]) - R
            # the nearest sign change of r(t) - R scanning outwards from t = 0
            ts = np.linspace(0, 40, 4001) * (1 if R > 20 else -1)
            vals = np.array([f(t) for t in ts])
            k = int(np.argmax(np.sign(vals) != np.sign(vals[0])))
            lo, hi = ts[k - 1], ts[k]
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if np.sign(f(mid)) == np.sign(f(lo)):
                    lo = mid
                else:
                    hi = mid
            assert abs(0.5 * (lo + hi) - s) < 1e-9
            # reversibility: from the crossing, the nearest crossing of the start
            # cylinder is the start
            s2 = oracle.cyl_path(Xo, q, 20.0, BZ, nearest=True)
            assert np.allclose(oracle.state_at(Xo, q, BZ, s2), X, rtol=1e-11, atol=1e-10)


def _fd_jacobian(f, X, rel=1e-6):
    J = np.zeros((6, 6))
    for j in range(6):
        h = rel * max(abs(X[j]), 1.0)
        e = np.zeros(6)
        e[j] = h
        J[:, j] = (f(X + e) - f(X - e)) / (2 * h)
    return J


def test_plane_jacobian_against_finite_differences(rng):
    for X in _states_on_cylinder(rng, 8):
        for q in (1, -1):
            Z = 80.0
            s = oracle.plane_path(X, Z)
            J = oracle.jacobian_surf(X, q, BZ, s, oracle.DISK)

            def f(Y):
                return oracle.state_at(Y, q, BZ, oracle.plane_path(Y, Z))
            Jfd = _fd_jacobian(f, X)
            scale = np.abs(Jfd).max(axis=1, keepdims=True) + 1e-12
            assert np.all(np.abs(J - Jfd) <= 1e-6 * scale + 1e-7), np.abs(J - Jfd).max()
            # the end point stays on the plane: the z row vanishes, so every
            # transported covariance has the null vector (zhat, 0)
            assert np.abs(J[2]).max() < 1e-12


def test_cylinder_surface_jacobian_is_the_barrel_jacobian(rng):
    for X in _states_on_cylinder(rng, 5):
        s = oracle.cyl_path(X, 1, 30.0, BZ)
        assert np.array_equal(oracle.jacobian_surf(X, 1, BZ, s, oracle.BARREL), oracle.jacobian(X, 1, BZ, s))


def _det(**kw):
    return presets.cylinder_with_lids(**kw)


@pytest.mark.parametrize("kind,avg,hits", [(0, 24.0, (24.5, 23.5)), (1, 70.0, (71.0, 69.0))])
def test_two_step_equals_direct_propagation(rng, kind, avg, hits):
    """Step 1 to the average surface, step 2 (nearest crossing) to the hit's
    surface equals one step to the hit's surface: same state, and the
    transported covariance (the Jacobians compose to the direct one)."""
    d = _det().replace(x_over_x0=0.0)
    for X in _states_on_cylinder(rng, 6):
        q = 1 if rng.uniform() < 0.5 else -1
        P = np.diag([1e-4, 1e-4, 1e-2, 1e-4, 1e-4, 1e-4]) + 1e-6
        a = oracle.step_surf(d, kind, avg, X, q, P, material=False)
        assert a is not None
        for v in hits:
            two = oracle.step_surf(d, kind, v, a[0], q, a[1], nearest=True, material=False)
            one = oracle.step_surf(d, kind, v, X, q, P, material=False)
            assert np.allclose(two[0], one[0], rtol=1e-12, atol=1e-10)
            assert np.allclose(two[1], one[1], rtol=1e-8, atol=1e-12 * np.abs(one[1]).max())


def test_disk_update_weighted_mean_information_and_joseph(rng):
    # no correlations: x and y become inverse-variance weighted means
    X = np.array([20.0, 5.0, 70.0, 1.0, 0.5, 2.0])
    P = np.diag([4e-4, 9e-4, 0.0, 1e-2, 1e-2, 1e-2])
    hit = np.array([20.02, 4.97, 70.0, 1e-4, 0.0, 0.0, 2e-4, 0.0, 0.0])
    Xo, Po, c2 = oracle.update_disk(X, P, hit)
    wx, wy = 4e-4 / 5e-4, 9e-4 / 11e-4
    assert np.isclose(Xo[0], 20.0 + wx * 0.02, rtol=1e-14) and np.isclose(Xo[1], 5.0 - wy * 0.03, rtol=1e-14)
    assert np.isclose(Po[0, 0], 4e-4 * 1e-4 / 5e-4, rtol=1e-13)
    assert np.isclose(c2, 0.02 ** 2 / 5e-4 + 0.03 ** 2 / 11e-4, rtol=1e-13)
    assert Xo[2] == X[2] and np.array_equal(Xo[3:], X[3:])
    for _ in range(30):
        A = rng.normal(size=(6, 6))
        P = (A @ A.T + 6 * np.eye(6)) * 1e-3
        ph = rng.uniform(0, TWO_PI)
        t, r = np.array([-np.sin(ph), np.cos(ph)]), np.array([np.cos(ph), np.sin(ph)])
        V = 1e-4 * np.outer(t, t) + 1e-2 * np.outer(r, r)
        X = np.array([20 * np.cos(ph), 20 * np.sin(ph), 70.0, 1.0, 0.5, 2.0])
        hit = np.array([X[0] + rng.normal(0, 0.05), X[1] + rng.normal(0, 0.05), 70.0, V[0, 0], V[0, 1], 0.0,
                        V[1, 1], 0.0, 0.0])
        Xo, Po, c2 = oracle.update_disk(X, P, hit)
        H = np.zeros((2, 6))
        H[0, 0] = H[1, 1] = 1.0
        lhs = np.linalg.inv(Po)
        rhs = np.linalg.inv(P) + H.T @ np.linalg.inv(V) @ H
        assert np.allclose(lhs, rhs, rtol=1e-8, atol=1e-8 * np.abs(rhs).max())
        S = H @ P @ H.T + V
        K = P @ H.T @ np.linalg.inv(S)
        I6 = np.eye(6)
        Pj = (I6 - K @ H) @ P @ (I6 - K @ H).T + K @ V @ K.T
        assert np.allclose(Pj, Po, rtol=1e-10, atol=1e-12 * np.abs(P).max())
        res = hit[:2] - X[:2]
        assert np.isclose(c2, res @ np.linalg.inv(S) @ res, rtol=1e-10)


def test_disk_scattering_uses_the_plane_normal():
    p = np.array([0.6, 0.8, 3.0])
    X = np.concatenate([[10.0, 0.0, 70.0], p])
    Q = oracle.ms_cov_surf(X, oracle.DISK, 0.02, 0.13957)
    pn = np.linalg.norm(p)
    xe = 0.02 / (3.0 / pn)  # incidence from zhat
    beta = pn / np.hypot(pn, 0.13957)
    th0 = 0.0136 / (beta * pn) * np.sqrt(xe) * (1 + 0.038 * np.log(xe / beta ** 2))
    assert np.allclose(Q[3:, 3:], th0 ** 2 * (pn ** 2 * np.eye(3) - np.outer(p, p)), rtol=1e-12)
    assert np.abs(Q[:3]).max() == 0


def _det_event(w, n, event=0, smear=True, x0=None, truth=True):
    gen = dataclasses.replace(w.gen, smear=smear)
    if not smear:
        gen = dataclasses.replace(gen, vtx_sxy=0.0)
    return datagen.generate_det(w.detector, gen, event, n, truth=truth, x_over_x0=x0)


def test_det_fit_zero_noise_returns_generating_helix():
    """No smearing and no material: seeded from exact hits, the fit over
    barrel layers, displaced modules and disks returns the generating helix
    at the track's last layer."""
    w = presets.lids()
    d = w.detector.replace(x_over_x0=0.0)
    ev = _det_event(w, 400, smear=False, x0=0.0)
    n = ev.n_tracks
    H, visit = datagen.det_track_rows(ev, dtype=np.float64)
    sg = d.seed_geometry()
    sd = oracle.seed64(sg.replace(x_over_x0=0.0), H[:3], n, beam_sigma=0.0)
    o = oracle.fit_det64(d, 3, H, visit, sd["par64"], sd["cov64"], sd["q"], n)
    assert np.all(o["status"][:n] == 0)
    last = np.array([int(v).bit_length() - 1 for v in visit[:n]])
    tr = ev.truth[last, :, np.arange(n)].T
    err = np.abs(o["par"][:, :n] - tr) / np.maximum(np.abs(tr), 1.0)
    assert err.max() < 1e-9, err.max()
    assert np.abs(o["chi2"][:n]).max() < 1e-10
    ndisk = np.array([sum((int(v) >> l) & 1 for l in range(10, 24)) for v in visit[:n]])
    assert (ndisk > 0).mean() > 0.3  # the pin covers disk updates


def _consistent_det_seeds(d, ev, rng, alpha):
    n = ev.n_tracks
    H, visit = datagen.det_track_rows(ev, dtype=np.float64)
    sd = oracle.seed64(d.seed_geometry(), H[:3], n)
    P = full_from_upper(sd["cov64"][:, :n]) * alpha
    tr = ev.truth[2]
    X = np.zeros_like(sd["par64"])
    for t in range(n):
        w_, V = np.linalg.eigh(P[t])
        X[:, t] = tr[:, t] + V @ (np.sqrt(np.clip(w_, 0, None)) * rng.normal(size=6))
    C = np.zeros_like(sd["cov64"])
    C[:, :n] = upper_from_full(P)
    q = np.zeros_like(sd["q"])
    q[:n] = ev.q
    return H, visit, X, C, q


@pytest.mark.parametrize("x0", [0.0, float(np.float32(0.02))])
def test_det_chi2_averages_ndof(x0, rng):
    """Seeds drawn from the truth with their stated covariance: the summed
    chi2 of the fit over barrel layers, displaced modules and disks averages
    its degrees of freedom (2 per hit)."""
    w = presets.lids()
    d = w.detector.replace(x_over_x0=x0)
    gen = dataclasses.replace(w.gen, pt_max=2.0)
    ev = datagen.generate_det(d, gen, 5, 5000, truth=True, x_over_x0=x0)
    n = ev.n_tracks
    H, visit, X, C, q = _consistent_det_seeds(d, ev, rng, 0.01)
    o = oracle.fit_det64(d, 3, H, visit, X, C, q, n)
    ok = o["status"][:n] == 0
    assert ok.mean() > 0.999
    c2 = o["chi2"][:n][ok]
    nd = o["ndof"][:n][ok]
    sig = np.sqrt(2.0 * nd.sum())
    assert abs(c2.sum() - nd.sum()) < 3.5 * sig, (c2.sum(), nd.sum(), sig)
    # the disks alone too
    last_disk = np.array([int(v) >= (1 << 10) for v in visit[:n]])[ok]
    assert last_disk.mean() > 0.3


def test_det_fit_on_a_plain_barrel_equals_barrel_fit():
    """A detector of exact cylinders (no disks, no module offsets) and the
    barrel fit of the same tracks agree (the detector fit steps to each hit's
    own radius, which is the layer radius up to the FP32 rounding of the
    hit)."""
    w = presets.fit_small()
    g = w.geometry
    d = presets.Detector([0] * g.n_layers, g.r[:g.n_layers], [-g.z_half] * g.n_layers, [g.z_half] * g.n_layers,
                         [0.0] * g.n_layers, bz=g.bz, x_over_x0=g.x_over_x0, mass=g.mass)
    ev = datagen.generate(g, w.gen, 0, 500)
    n = ev.n_tracks
    H = datagen.track_hits(ev)
    so = oracle.seed(g, H, n)
    ob = oracle.fit(g, 3, H, so["par"], so["cov"], so["q"], n)
    visit = np.full(H.shape[2], (1 << g.n_layers) - 1, dtype=np.uint32)
    od = oracle.fit_det(d, 3, H, visit, so["par"], so["cov"], so["q"], n)
    # (the barrel fit also stops a track beyond |z| = z_half; the detector fit
    # follows the list it is given)
    ok = ob["status"][:n] == 0
    good = ok & (ob["chi2"][:n] <= 5 * np.maximum(ob["ndof"][:n], 1))
    assert np.array_equal(od["ndof"][:n][ok], ob["ndof"][:n][ok]) and ok.mean() > 0.95
    e = np.abs(od["par"][:, :n] - ob["par"][:, :n]).max(axis=0) / np.abs(ob["par"][:, :n]).max(axis=0)
    assert np.median(e[good]) < 1e-6 and e[good].max() < 1e-3


def test_det_binning_definition():
    w = presets.lids()
    d = w.detector
    ev = _det_event(w, 2000)
    xyz = ev.xyz.astype(np.float32)
    nphi, nw = 63, 16
    b = oracle.hit_bin_det(d, nphi, nw, ev.layer, xyz)
    order, off, phi = b["order"], b["offsets"], b["phi"]
    assert np.array_equal(np.sort(order), np.arange(ev.n_hits))
    nb = nphi * nw
    for l in range(d.n_layers):
        row = off[l]
        assert np.all(np.diff(row) >= 0) and row[nb] - row[0] == np.sum(ev.layer == l)
        lo, hi = d.lo[l], d.hi[l]
        for bb in range(0, nb, 29):
            sl = order[row[bb]:row[bb + 1]]
            if len(sl) == 0:
                continue
            iw, ip = divmod(bb, nphi)
            x, y, z = (xyz[c, sl].astype(np.float64) for c in range(3))
            w_ = np.hypot(x, y) if d.kind[l] == oracle.DISK else z
            ph = np.mod(np.arctan2(y, x), TWO_PI)
            assert np.all(ph >= ip * TWO_PI / nphi - 1e-6) and np.all(ph < (ip + 1) * TWO_PI / nphi + 1e-6)
            wl = lo + iw * (hi - lo) / nw
            inner = (w_ >= lo) & (w_ <= hi)  # hits beyond the extent go to the edge bins
            assert np.all(w_[inner] >= wl - 1e-9) and np.all(w_[inner] < wl + (hi - lo) / nw + 1e-9)
            ps = phi[row[bb]:row[bb + 1]]
            assert np.all(np.diff(ps) >= 0)


def _dfs_det(d, cuts, ev, sd, t, greedy=False):
    """Exhaustive depth-first enumeration of the detector build's rules (next
    layer, two-step window and update, hole), written from the rules with the
    oracle's pinned primitives; greedy follows only the best child."""
    xyz = ev.xyz.astype(np.float32).astype(np.float64)
    cov = ev.cov.astype(np.float32).astype(np.float64)
    L = d.n_layers
    by_layer = [np.where(ev.layer == l)[0] for l in range(L)]
    q = int(sd["q"][t])
    X0 = sd["par"][:, t].astype(np.float64)
    P0 = full_from_upper(sd["cov"][:, t:t + 1].astype(np.float64))[0]
    leaves = []
    ns, sr, sw = cuts.nsigma, cuts.win_sig_rphi, cuts.win_sig_z

    def next_layer(cur, X, P):
        for j in range(cur + 1, L):
            a = oracle.step_surf(d, d.kind[j], d.pos[j], X, q, P, material=False)
            if a is None:
                continue
            Xa = a[0]
            if d.kind[j] == oracle.DISK:
                # within half a turn (the angle turned is KAPPA B dz / pz),
                # still moving outwards
                turn = abs(0.299792458e-2 * d.bz * (d.pos[j] - X[2]) / X[5])
                if not (turn < np.pi and Xa[0] * Xa[3] + Xa[1] * Xa[4] > 0):
                    continue
            w_ = np.hypot(Xa[0], Xa[1]) if d.kind[j] == oracle.DISK else Xa[2]
            if d.lo[j] <= w_ <= d.hi[j]:
                return j, Xa, a[1]
        return None

    def children(l, Xa, Pa, nhits, holes, chi2):
        kind = d.kind[l]
        r = np.hypot(Xa[0], Xa[1])
        tv, nv = np.array([-Xa[1], Xa[0]]) / r, np.array([Xa[0], Xa[1]]) / r
        Stt = tv @ Pa[:2, :2] @ tv + sr ** 2
        pr, pphi = nv @ Xa[3:5], tv @ Xa[3:5]
        if kind == oracle.DISK:
            Sww = nv @ Pa[:2, :2] @ nv + sw ** 2
            sl_w, sl_phi = pr / Xa[5], pphi / (r * Xa[5])
        else:
            Sww = Pa[2, 2] + sw ** 2
            sl_w, sl_phi = Xa[5] / pr, pphi / (r * pr)
        dphi = ns * np.sqrt(Stt) / r + d.dmod[l] * abs(sl_phi)
        dw = ns * np.sqrt(Sww) + d.dmod[l] * abs(sl_w)
        php = np.arctan2(Xa[1], Xa[0])
        wp = r if kind == oracle.DISK else Xa[2]
        out = []
        for hi in by_layer[l]:
            h = np.concatenate([xyz[:, hi], cov[:, hi]])
            dph = np.angle(np.exp(1j * (np.arctan2(h[1], h[0]) - php)))
            hw = np.hypot(h[0], h[1]) if kind == oracle.DISK else h[2]
            if abs(dph) > dphi or abs(hw - wp) > dw:
                continue
            surf = h[2] if kind == oracle.DISK else np.hypot(h[0], h[1])
            st = oracle.step_surf(d, kind, surf, Xa, q, Pa, nearest=True, material=True)
            if st is None:
                continue
            if kind == oracle.DISK:
                u = oracle.update_disk(st[0], st[1], h)
                if u is None:
                    continue
                Xu, Pu, c2 = u
            else:
                rc, Xu, Pu, c2 = oracle.update(st[0], st[1], h)
                if rc:
                    continue
            if c2 < cuts.chi2_cut:
                out.append((nhits + 1, chi2 + c2, int(hi), Xu, Pu, holes))
        if holes < cuts.max_holes:
            Q = oracle.ms_cov_surf(Xa, kind, d.x_over_x0, d.mass)
            out.append((nhits, chi2, -1, Xa, Pa + Q, holes + 1))
        out.sort(key=lambda c: (-c[0], c[1], c[2] if c[2] >= 0 else 1 << 30))
        return out

    def rec(cur, X, P, nhits, holes, chi2, hits):
        nl = next_layer(cur, X, P)
        if nl is None:
            leaves.append((nhits, chi2, list(hits)))
            return
        l, Xa, Pa = nl
        ch = children(l, Xa, Pa, nhits, holes, chi2)
        if not ch:
            leaves.append((nhits, chi2, list(hits)))
            return
        for (nh, c2, hi, Xc, Pc, ho) in (ch[:1] if greedy else ch):
            rec(l, Xc, Pc, nh, ho, c2, hits + [(l, hi)])

    rec(cuts.first_layer - 1, X0, P0, 0, 0, 0.0, [])
    best = min(leaves, key=lambda lf: (-lf[0], lf[1]))
    return best, len(leaves)


def _tiny_lids():
    """Seven layers: the three seed cylinders, two barrel layers with
    displaced modules (|z| <= 30 cm) and one disk on each side."""
    d = presets.Detector([0, 0, 0, 0, 0, 1, 1], [4.0, 8.0, 12.0, 16.0, 20.0, 36.0, -36.0],
                         [-100.0, -100.0, -100.0, -30.0, -30.0, 14.0, 14.0],
                         [100.0, 100.0, 100.0, 30.0, 30.0, 42.0, 42.0], [0, 0, 0, 0.5, 0.5, 1.0, 1.0])
    gen = presets.GenSettings(seed=4343, eta_max=1.8, noise_lo=1.0, noise_hi=1.0)
    return presets.DetWorkload("tiny lids", d, gen, 1, 3)


@pytest.mark.parametrize("wide", [False, True])
def test_det_unbounded_cap_equals_exhaustive_search(wide):
    w = _tiny_lids()
    d, cuts = w.detector, w.cuts
    if wide:
        cuts = dataclasses.replace(cuts, nsigma=1e3, chi2_cut=1e12)
    ev = _det_event(w, 3, event=1)
    n = ev.n_tracks
    H, visit = datagen.det_track_rows(ev)
    sd = oracle.seed(d.seed_geometry(), H[:3], n)
    most = 0
    for t in range(n):
        best, nleaves = _dfs_det(d, cuts, ev, sd, t)
        most = max(most, nleaves)
        o = oracle.build_det(d, cuts, ev.layer, ev.xyz, ev.cov, sd["par"], sd["cov"], sd["q"], n, seed_list=[t],
                             cap=1 << 20)
        assert o["nhits"][0] == best[0]
        assert abs(o["chi2"][0] - best[1]) <= 1e-9 * max(1.0, best[1])
        exp = np.full(d.n_layers - cuts.first_layer, -1)
        vis = 0
        for l, hi in best[2]:
            exp[l - cuts.first_layer] = hi
            vis |= 1 << l
        assert list(o["hits"][:, 0]) == list(exp)
        assert int(o["visit"][0]) == vis
    if wide:
        assert most > 10  # a branching tree: every hit of a layer and a hole


def test_det_cap_one_equals_greedy():
    w = presets.lids()
    d, cuts = w.detector, dataclasses.replace(w.cuts, cand_cap=1)
    ev = _det_event(w, 60, event=2)
    n = ev.n_tracks
    H, visit = datagen.det_track_rows(ev)
    sd = oracle.seed(d.seed_geometry(), H[:3], n)
    o = oracle.build_det(d, cuts, ev.layer, ev.xyz, ev.cov, sd["par"], sd["cov"], sd["q"], n)
    for t in range(0, n, 6):
        best, _ = _dfs_det(d, cuts, ev, sd, t, greedy=True)
        assert o["nhits"][t] == best[0]
        exp = np.full(d.n_layers - cuts.first_layer, -1)
        for l, hi in best[2]:
            exp[l - cuts.first_layer] = hi
        assert list(o["hits"][:, t]) == list(exp)


def test_det_noise_free_event_recovers_true_hits():
    """No noise hits, no smearing, no material: every seed's best candidate
    carries exactly its track's hits on every layer it crosses, chi2 ~ 0."""
    w = presets.lids()
    d = w.detector.replace(x_over_x0=0.0)
    gen = dataclasses.replace(w.gen, smear=False, vtx_sxy=0.0, noise_lo=0.0, noise_hi=0.0)
    ev = datagen.generate_det(d, gen, 3, 300, x_over_x0=0.0)
    n = ev.n_tracks
    H, visit = datagen.det_track_rows(ev)
    sd = oracle.seed(d.seed_geometry(), H[:3], n, beam_sigma=0.0)
    o = oracle.build_det(d, w.cuts, ev.layer, ev.xyz, ev.cov, sd["par"], sd["cov"], sd["q"], n)
    F = w.cuts.first_layer
    assert np.array_equal(o["hits"][:, :n], ev.trk_hits[F:, :n])
    assert np.array_equal(o["visit"][:n], visit[:n] & ~np.uint32((1 << F) - 1))
    assert np.abs(o["chi2"][:n]).max() < 1e-3


def test_det_build_on_plain_barrel_matches_barrel_build():
    """On a detector of exact cylinders the detector build and the barrel
    build choose the same hits for nearly every seed (the detector build
    steps to each hit's own radius: chi2 differs by the FP32 rounding of the
    hits)."""
    w = presets.build()
    g = w.geometry
    d = presets.Detector([0] * g.n_layers, g.r[:g.n_layers], [-g.z_half] * g.n_layers, [g.z_half] * g.n_layers,
                         [0.0] * g.n_layers, bz=g.bz, x_over_x0=g.x_over_x0, mass=g.mass)
    ev = datagen.generate(g, w.gen, 4, 2000)
    n = ev.n_tracks
    H = datagen.track_hits(ev)
    so = oracle.seed(g, H, n)
    lst = np.arange(0, n, 20)
    ob = oracle.build(g, w.cuts, ev.layer, ev.xyz, ev.cov, so["par"], so["cov"], so["q"], n, seed_list=lst)
    od = oracle.build_det(d, w.cuts, ev.layer, ev.xyz, ev.cov, so["par"], so["cov"], so["q"], n, seed_list=lst)
    same = np.all(ob["hits"] == od["hits"], axis=0)
    assert same.mean() > 0.97, same.mean()


def test_det_build_efficiency_and_margins():
    w = presets.lids()
    d = w.detector
    ev = _det_event(w, 20000, truth=False)
    n = ev.n_tracks
    H, visit = datagen.det_track_rows(ev)
    sd = oracle.seed(d.seed_geometry(), H[:3], n)
    lst = np.arange(0, n, 100)
    o = oracle.build_det(d, w.cuts, ev.layer, ev.xyz, ev.cov, sd["par"], sd["cov"], sd["q"], n, seed_list=lst)
    F = w.cuts.first_layer
    true = ev.trk_hits[F:, lst]
    found = ((o["hits"] == true) & (true >= 0)).sum(axis=0)
    eff = found >= 0.75 * (true >= 0).sum(axis=0)
    print(f"lids build: efficiency {eff.mean():.3f}, undecidable {1 - oracle.decidable(o['margin']).mean():.3f}")
    assert eff.mean() > 0.7
    assert oracle.decidable(o["margin"]).mean() > 0.85
