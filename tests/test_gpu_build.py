"""GPU kf_build (after GPU hit_bin) against the oracle's brute-force build.

Hit lists, nhits and status must be identical for every decidable seed: one
whose every decision during the oracle's search is further from its
threshold than the numerical noise can move it (chi2 gaps above 1e-3,
window edges further than 1e-4 cm, crossing and barrel-end tests further than
1e-3 relative).  chi2 within 1e-3 * max(1, chi2) and parameters within 1e-4
on decidable seeds whose best candidate converged (chi2/ndof <= 100)."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1711_06571_amd import datagen, presets, workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from gpu_common import host, rel_vec_err, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def kf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_06571_amd import kftrack
    return kftrack


def decidable(o):
    return oracle.decidable(o["margin"])


# Bounds on what the parity comparison excludes.  The fraction of undecidable
# seeds grows with the number of decisions a seed makes (about 70 predicted
# candidate-layers, 20-40 hits window-tested per candidate-layer): 8 % on 400
# seeds of the full build event (chi2 row 4.3 %, window row 3.8 %), 2-17 %
# over 63-seed samples of single events.  Seeds whose lists differ must be
# undecidable and stay rare: none has been seen in any run.
UNDECIDABLE_MAX = 0.15
UNDECIDABLE_MAX_SMALL_SAMPLE = 0.25  # fewer than 100 seeds
MISMATCH_MAX_FRACTION = 0.01


def gpu_build_event(kf, w, ev, arith, cap=None, lanes=0, blocks=0, order=None, seeds=None, refine=0, state=None):
    xyz = ev.xyz.astype(np.float32)
    cov = ev.cov.astype(np.float32)
    b = kf.hit_bin(w.geometry, w.cuts.n_phi_bins, w.cuts.n_z_bins, to_dev(ev.layer), to_dev(xyz), to_dev(cov))
    H = datagen.track_hits(ev)
    n = ev.n_tracks
    if seeds is None:
        seeds = kf.kf_seed(w.geometry, n, to_dev(H))
    bp = kf.build_params(w.cuts, cap=cap, lanes_per_block=lanes, persistent_blocks=blocks, arith=arith,
                         phi_refine=refine, **({} if state is None else {"state": state}))
    ex = kf.BuildExtra()
    keep = []
    if order is not None:
        od = to_dev(order.astype(np.int32))
        keep.append(od)
        ex.seed_order = od.data_ptr()
    out = kf.kf_build(w.geometry, bp, b, n, seeds["par"], seeds["cov"], seeds["q"], extra=ex)
    torch.cuda.synchronize()
    return {k: host(v) for k, v in out.items()}, seeds


def compare(g, o, n_cols, cols_g=None, ctx="", check_params=True, und_max=None):
    """g: GPU outputs (indexed by seed), o: oracle outputs for seeds cols_g;
    und_max overrides the bound on the undecidable fraction."""
    cols_g = np.arange(n_cols) if cols_g is None else cols_g
    dec = decidable(o)[:n_cols]
    gh = g["hits"][:, cols_g]
    same_hits = np.all(gh == o["hits"][:, :n_cols], axis=0)
    same_n = g["nhits"][cols_g] == o["nhits"][:n_cols]
    same_st = g["status"][cols_g] == o["status"][:n_cols]
    ok = same_hits & same_n & same_st
    bad = np.where(dec & ~ok)[0]
    assert bad.size == 0, f"{ctx}: {bad.size} decidable seeds differ, first {bad[:10]}"
    c2g = g["chi2"][cols_g].astype(np.float64)
    c2o = o["chi2"][:n_cols]
    e = np.abs(c2g - c2o) / np.maximum(1.0, c2o)
    sel = dec & ok
    assert e[sel].max(initial=0) <= 1e-3, f"{ctx}: chi2 {e[sel].max():.3g}"
    if check_params:
        conv = sel & (c2o <= 100 * np.maximum(2 * o["nhits"][:n_cols], 1))
        pg = g["par"][:, cols_g].astype(np.float64)
        po = o["par"][:, :n_cols]
        ep = rel_vec_err(pg[:3], po[:3])
        em = rel_vec_err(pg[3:], po[3:])
        assert ep[conv].max(initial=0) <= 1e-4 and em[conv].max(initial=0) <= 1e-4, \
            f"{ctx}: params {ep[conv].max():.3g} {em[conv].max():.3g}"
    rows = oracle.undecidable_by_row(o["margin"][:, :n_cols])
    und = float(1 - dec.mean()) if n_cols else 0.0
    mism = int((~ok).sum())
    # the exclusions are bounded: few undecidable seeds, and fewer still
    # whose lists differ
    bound = UNDECIDABLE_MAX if n_cols >= 100 else UNDECIDABLE_MAX_SMALL_SAMPLE
    bound = bound if und_max is None else und_max
    assert und <= bound, f"{ctx}: {und:.3f} undecidable (by row {rows})"
    assert mism <= max(1, int(MISMATCH_MAX_FRACTION * n_cols)), f"{ctx}: {mism} of {n_cols} seeds differ"
    return dict(undecidable=und, by_row=rows, mismatched=mism, n=int(n_cols))


def test_build_parity_small_event(kf):
    w = presets.build()
    ev = datagen.generate(w.geometry, w.gen, 11, 600)
    n = ev.n_tracks
    g, sg = gpu_build_event(kf, w, ev, kf.ARITH_F64)
    H = datagen.track_hits(ev)
    so = oracle.seed(w.geometry, H, n)
    o = oracle.build(w.geometry, w.cuts, ev.layer, ev.xyz, ev.cov, so["par"], so["cov"], so["q"], n)
    r = compare(g, o, n, ctx="small f64")
    print("build small f64", r)


def test_build_parity_full_event_sampled(kf):
    """The full build workload (20 000 tracks + 20 % noise per layer), in the
    launch configuration the benchmark uses; the oracle builds 240 sampled
    seeds one by one."""
    w = presets.build()
    ev = datagen.generate(w.geometry, w.gen, 0, w.n_tracks)
    n = ev.n_tracks
    g, sg = gpu_build_event(kf, w, ev, kf.ARITH_F64)
    H = datagen.track_hits(ev)
    so = oracle.seed(w.geometry, H, n)
    lst = np.concatenate([np.arange(0, n, 97)[:200], np.arange(n - 40, n)])
    o = oracle.build(w.geometry, w.cuts, ev.layer, ev.xyz, ev.cov, so["par"], so["cov"], so["q"], n, seed_list=lst)
    r = compare(g, o, lst.size, cols_g=lst, ctx="full f64")
    print("build full f64", r)


def test_build_fp32_arithmetic_agreement(kf):
    w = presets.build()
    ev = datagen.generate(w.geometry, w.gen, 12, 600)
    n = ev.n_tracks
    g, sg = gpu_build_event(kf, w, ev, kf.ARITH_F32)
    H = datagen.track_hits(ev)
    so = oracle.seed(w.geometry, H, n)
    o = oracle.build(w.geometry, w.cuts, ev.layer, ev.xyz, ev.cov, so["par"], so["cov"], so["q"], n)
    dec = decidable(o)
    same = np.all(g["hits"][:, :n] == o["hits"], axis=0) & (g["nhits"][:n] == o["nhits"])
    from gpu_common import seed_rel_sigma_p
    well = seed_rel_sigma_p(so["par"], so["cov"], n) < 0.1
    print(f"build fp32: identical lists {same.mean():.4f} overall, {same[dec].mean():.4f} decidable, "
          f"{same[dec & well].mean() if (dec & well).any() else 1.0:.4f} decidable well-conditioned")
    assert same[dec & well].all()
    assert same.mean() >= 0.97  # measured 0.990


@pytest.mark.parametrize("cap", [1, 3, 4, 5, 8])
def test_build_other_caps(kf, cap):
    w = presets.build()
    ev = datagen.generate(w.geometry, w.gen, 13, 300)
    n = ev.n_tracks
    g, sg = gpu_build_event(kf, w, ev, kf.ARITH_F64, cap=cap)
    H = datagen.track_hits(ev)
    so = oracle.seed(w.geometry, H, n)
    o = oracle.build(w.geometry, w.cuts, ev.layer, ev.xyz, ev.cov, so["par"], so["cov"], so["q"], n, cap=cap)
    print(f"cap {cap}", compare(g, o, n, ctx=f"cap {cap}"))


def test_build_launch_shape_and_order_invariance(kf):
    w = presets.build()
    ev = datagen.generate(w.geometry, w.gen, 14, 2000)
    n = ev.n_tracks
    ref, sg = gpu_build_event(kf, w, ev, kf.ARITH_F32)
    rng = np.random.default_rng(5)
    # launch shape, seed order and the granularity of the fine phi index
    # (an acceleration structure only) change no output
    for lanes, blocks, order, refine in [(64, 0, None, 0), (128, 7, None, 1), (256, 1, None, 32),
                                         (256, 0, rng.permutation(n), 3)]:
        g, _ = gpu_build_event(kf, w, ev, kf.ARITH_F32, lanes=lanes, blocks=blocks, order=order, seeds=sg,
                               refine=refine)
        for k in ref:
            assert np.array_equal(g[k][..., :n], ref[k][..., :n]), (k, lanes, blocks, refine)


@pytest.mark.parametrize("hybrid", [False, True])
def test_build_fp64_launch_shapes(kf, hybrid):
    """FP64 builds keep each candidate's state between layers in the block's
    LDS, at offsets that depend on the waves per block: blocks of one, two
    and four waves, and a fixed small grid, give the default launch's
    outputs bit for bit, in both states."""
    w = presets.build()
    ev = datagen.generate(w.geometry, w.gen, 15, 1500)
    n = ev.n_tracks
    st = kf.STATE_HYBRID if hybrid else kf.STATE_CARTESIAN
    ref, sg = gpu_build_event(kf, w, ev, kf.ARITH_F64, state=st)
    for lanes, blocks in [(64, 0), (128, 7), (256, 1)]:
        g, _ = gpu_build_event(kf, w, ev, kf.ARITH_F64, lanes=lanes, blocks=blocks, seeds=sg, state=st)
        for k in ref:
            assert np.array_equal(g[k][..., :n], ref[k][..., :n]), (k, lanes, blocks, hybrid)


@pytest.mark.parametrize("cap", [3, 8])
def test_hybrid_state_build_other_caps(kf, cap):
    """The hybrid FP64 build at other caps against the oracle (at cap 8 its
    LDS state takes one block per CU)."""
    w = presets.build()
    ev = datagen.generate(w.geometry, w.gen, 16, 300)
    n = ev.n_tracks
    g, _ = gpu_build_event(kf, w, ev, kf.ARITH_F64, cap=cap, state=kf.STATE_HYBRID)
    H = datagen.track_hits(ev)
    so = oracle.seed(w.geometry, H, n)
    o = oracle.build(w.geometry, w.cuts, ev.layer, ev.xyz, ev.cov, so["par"], so["cov"], so["q"], n, cap=cap,
                     state=1)
    print(f"hybrid cap {cap}", compare(g, o, n, ctx=f"hybrid cap {cap}", check_params=False))


def test_build_noise_free_recovers_true_hits(kf):
    w = presets.build()
    g0 = w.geometry.replace(x_over_x0=0.0)
    w0 = dataclasses.replace(w, geometry=g0)
    gen = dataclasses.replace(w.gen, smear=False, vtx_sxy=0.0, noise_lo=0.0, noise_hi=0.0, pt_max=3.0)
    ev = datagen.generate(g0, gen, 0, 1000)
    g, _ = gpu_build_event(kf, w0, ev, kf.ARITH_F32)
    F = w.cuts.first_layer
    assert np.array_equal(g["hits"][:, :1000], ev.trk_hits[F:])
    assert np.all(g["nhits"][:1000] == g0.n_layers - F)


def test_build_batch_of_events(kf):
    w = presets.batch()
    eb = workloads.event_batch(w, range(4), n_tracks=None)
    b = kf.hit_bin(w.geometry, 63, 16, to_dev(eb.layer), to_dev(eb.xyz), to_dev(eb.cov),
                   event_offsets=to_dev(eb.hit_offsets))
    sg = kf.kf_seed(w.geometry, eb.n_seeds, to_dev(eb.seed_hits))
    bp = kf.build_params(w.cuts, arith=kf.ARITH_F64)
    ex = kf.BuildExtra()
    sev = to_dev(eb.seed_event)
    ex.seed_event = sev.data_ptr()
    nps = to_dev(np.diff(eb.seed_offsets).astype(np.int32))
    ticks = torch.zeros(4, dtype=torch.int64, device="cuda:0")
    t0 = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    ex.event_n_seeds = nps.data_ptr()
    ex.event_done_ticks = ticks.data_ptr()
    ex.start_tick = t0.data_ptr()
    out = kf.kf_build(w.geometry, bp, b, eb.n_seeds, sg["par"], sg["cov"], sg["q"], extra=ex)
    torch.cuda.synchronize()
    g = {k: host(v) for k, v in out.items()}
    tk = host(ticks)
    assert np.all(tk > host(t0)[0])
    for e in range(4):
        s0, s1 = eb.seed_offsets[e], eb.seed_offsets[e + 1]
        h0, h1 = eb.hit_offsets[e], eb.hit_offsets[e + 1]
        m = s1 - s0
        lst = np.arange(0, m, max(1, m // 25))
        Hs = np.ascontiguousarray(eb.seed_hits[:, :, s0:s1])
        so = oracle.seed(w.geometry, Hs, m)
        o = oracle.build(w.geometry, w.cuts, eb.layer[h0:h1], eb.xyz[:, h0:h1], eb.cov[:, h0:h1], so["par"],
                         so["cov"], so["q"], m, seed_list=lst)
        print(f"event {e}", compare(g, o, lst.size, cols_g=s0 + lst, ctx=f"event {e}"))


def test_build_batch_with_empty_events(kf):
    """Four events in one launch: event 1 keeps its seeds but has no hits
    (every layer a hole), event 2 has hits but no seeds.  Events 0 and 3
    match the oracle on their sampled seeds, the seeds of event 1 find
    nothing, event 2's hits are binned and its completion tick is never
    written (it has no seed to finish)."""
    w = presets.batch()
    eb = workloads.event_batch(w, range(4))
    ho, so_ = eb.hit_offsets.astype(np.int64), eb.seed_offsets.astype(np.int64)
    keep_h = np.concatenate([np.arange(ho[0], ho[1]), np.arange(ho[2], ho[4])])
    keep_s = np.concatenate([np.arange(so_[0], so_[2]), np.arange(so_[3], so_[4])])
    nh = np.array([ho[1] - ho[0], 0, ho[3] - ho[2], ho[4] - ho[3]])
    hoff = np.concatenate([[0], np.cumsum(nh)]).astype(np.int32)
    ns = np.array([so_[1] - so_[0], so_[2] - so_[1], 0, so_[4] - so_[3]])
    soff = np.concatenate([[0], np.cumsum(ns)])
    n = int(ns.sum())
    ld = ((n + 63) // 64) * 64
    xyz, cov, layer = eb.xyz[:, keep_h], eb.cov[:, keep_h], eb.layer[keep_h]
    sh = np.zeros((eb.seed_hits.shape[0], 9, ld), dtype=np.float32)
    sh[:, :, :n] = eb.seed_hits[:, :, keep_s]
    sev = eb.seed_event[keep_s].astype(np.int32)
    b = kf.hit_bin(w.geometry, 63, 16, to_dev(layer), to_dev(xyz), to_dev(cov), event_offsets=to_dev(hoff))
    sg = kf.kf_seed(w.geometry, n, to_dev(sh))
    ex = kf.BuildExtra()
    sevd = to_dev(sev)
    ex.seed_event = sevd.data_ptr()
    nps = to_dev(ns.astype(np.int32))
    ticks = torch.zeros(4, dtype=torch.int64, device="cuda:0")
    t0 = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    ex.event_n_seeds = nps.data_ptr()
    ex.event_done_ticks = ticks.data_ptr()
    ex.start_tick = t0.data_ptr()
    out = kf.kf_build(w.geometry, kf.build_params(w.cuts, arith=kf.ARITH_F64), b, n, sg["par"], sg["cov"],
                      sg["q"], extra=ex)
    torch.cuda.synchronize()
    g = {k: host(v) for k, v in out.items()}
    offs = host(b.offsets).reshape(4, w.geometry.n_layers, -1)
    assert np.all(offs[1] == hoff[1]) and offs[2, -1, -1] == hoff[3]
    tk = host(ticks)
    assert tk[0] > host(t0)[0] and tk[1] > host(t0)[0] and tk[3] > host(t0)[0] and tk[2] == 0
    e1 = np.arange(soff[1], soff[2])
    assert np.all(g["nhits"][e1] == 0) and np.all(g["hits"][:, e1] == -1)
    for e in (0, 3):
        s0, s1 = int(soff[e]), int(soff[e + 1])
        h0, h1 = int(hoff[e]), int(hoff[e + 1])
        m = s1 - s0
        lst = np.arange(0, m, max(1, m // 25))
        Hs = np.zeros((sh.shape[0], 9, ((m + 63) // 64) * 64), dtype=np.float32)
        Hs[:, :, :m] = sh[:, :, s0:s1]
        so = oracle.seed(w.geometry, Hs, m)
        o = oracle.build(w.geometry, w.cuts, np.ascontiguousarray(layer[h0:h1]), np.ascontiguousarray(xyz[:, h0:h1]),
                         np.ascontiguousarray(cov[:, h0:h1]), so["par"], so["cov"], so["q"], m, seed_list=lst)
        print(f"event {e} beside empty events", compare(g, o, lst.size, cols_g=s0 + lst, ctx=f"event {e}"))


@pytest.mark.parametrize("state", [0, 1])
def test_build_edge_cases(kf, state):
    w = presets.build()
    g = w.geometry
    ev = datagen.generate(g, w.gen, 15, 64)
    xyz = ev.xyz.astype(np.float32)
    b = kf.hit_bin(g, 63, 16, to_dev(ev.layer), to_dev(xyz), to_dev(ev.cov.astype(np.float32)))
    H = datagen.track_hits(ev)
    sg = kf.kf_seed(g, 64, to_dev(H))
    par = sg["par"].clone()
    par[0, 5] = float("nan")  # a non-finite seed is returned as given, flagged
    bp = kf.build_params(w.cuts, state=state)
    out = kf.kf_build(g, bp, b, 64, par, sg["cov"], sg["q"])
    torch.cuda.synchronize()
    st = host(out["status"])
    assert st[5] & kf.TRK_NONFINITE and host(out["nhits"])[5] == 0
    assert np.all(host(out["hits"])[:, 5] == -1)
    # no seeds: nothing to do
    kf.kf_build(g, bp, b, 0, par, sg["cov"], sg["q"])
    # a cap the kernels do not implement; a state that does not exist
    with pytest.raises(kf.KFError):
        kf.kf_build(g, kf.build_params(w.cuts, cap=9, state=state), b, 64, par, sg["cov"], sg["q"])
    with pytest.raises(kf.KFError):
        kf.kf_build(g, kf.build_params(w.cuts, state=2), b, 64, par, sg["cov"], sg["q"])
    # a workspace that is not 256-byte aligned (the packed hits are read as
    # 16-byte vectors) is refused before any launch
    need = kf.kf_build_workspace_bytes(bp, b, 64)
    wsb = torch.empty(need + 256, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(kf.KFError, match="orkspace"):
        kf.kf_build(g, bp, b, 64, par, sg["cov"], sg["q"], ws=wsb[16:])
    # an event with no hits at all: every seed ends on holes and stops
    empty = kf.hit_bin(g, 63, 16, torch.zeros(0, dtype=torch.int32, device="cuda:0"),
                       torch.zeros((3, 0), device="cuda:0"), torch.zeros((6, 0), device="cuda:0"))
    out = kf.kf_build(g, bp, empty, 64, sg["par"], sg["cov"], sg["q"])
    torch.cuda.synchronize()
    assert np.all(host(out["nhits"])[:64] == 0)


def _hybrid_param_errors(g, o, cols_g, sel):
    gp = g["par"][:, cols_g][:, sel].astype(np.float64)
    op = o["par"][:, sel]
    ep = rel_vec_err(gp[:3], op[:3])
    ek = np.abs(gp[3] - op[3]) / np.abs(op[3])
    da = gp[4:] - op[4:]
    da[0] = (da[0] + np.pi) % (2 * np.pi) - np.pi
    return ep, ek, np.abs(da).max(axis=0)


@pytest.mark.parametrize("full", [False, True])
def test_hybrid_state_build_parity(kf, full):
    """The build in the hybrid state (FP64 arithmetic) against the oracle's:
    hit lists, nhits and status on every decidable seed; chi2, position,
    q/pT and angles on the converged ones."""
    w = presets.build()
    if full:
        ev = datagen.generate(w.geometry, w.gen, 0, w.n_tracks)
    else:
        ev = datagen.generate(w.geometry, w.gen, 13, 600)
    n = ev.n_tracks
    xyz = ev.xyz.astype(np.float32)
    b = kf.hit_bin(w.geometry, w.cuts.n_phi_bins, w.cuts.n_z_bins, to_dev(ev.layer), to_dev(xyz),
                   to_dev(ev.cov.astype(np.float32)))
    H = datagen.track_hits(ev)
    sg = kf.kf_seed(w.geometry, n, to_dev(H))
    bp = kf.build_params(w.cuts, arith=kf.ARITH_F64, state=kf.STATE_HYBRID)
    out = kf.kf_build(w.geometry, bp, b, n, sg["par"], sg["cov"], sg["q"])
    torch.cuda.synchronize()
    g = {k: host(v) for k, v in out.items()}
    so = oracle.seed(w.geometry, H, n)
    lst = np.concatenate([np.arange(0, n, 97)[:200], np.arange(n - 40, n)]) if full else np.arange(n)
    o = oracle.build(w.geometry, w.cuts, ev.layer, ev.xyz, ev.cov, so["par"], so["cov"], so["q"], n,
                     seed_list=lst, state=1)
    r = compare(g, o, lst.size, cols_g=lst, ctx=f"hybrid {'full' if full else 'small'}", check_params=False)
    dec = decidable(o)[:lst.size]
    same = np.all(g["hits"][:, lst] == o["hits"], axis=0) & (g["nhits"][lst] == o["nhits"])
    conv = dec & same & (o["chi2"] <= 100 * np.maximum(2 * o["nhits"], 1))
    sel = np.where(conv)[0]
    ep, ek, ea = _hybrid_param_errors(g, o, lst, sel)
    assert ep.max(initial=0) <= 1e-4 and ek.max(initial=0) <= 1e-4 and ea.max(initial=0) <= 1e-4, \
        (ep.max(), ek.max(), ea.max())
    print(f"build hybrid {'full' if full else 'small'} f64", r, f"params on {sel.size}: pos {ep.max(initial=0):.2g} "
          f"q/pT {ek.max(initial=0):.2g} angles {ea.max(initial=0):.2g}")


def test_hybrid_state_build_efficiency(kf):
    """On the full build event the hybrid state keeps the true hits of more
    seeds than the Cartesian state (seeds of the wrong charge recover)."""
    w = presets.build()
    ev = datagen.generate(w.geometry, w.gen, 0, w.n_tracks, truth=True)
    n = ev.n_tracks
    gc, sg = gpu_build_event(kf, w, ev, kf.ARITH_F64)
    xyz = ev.xyz.astype(np.float32)
    b = kf.hit_bin(w.geometry, w.cuts.n_phi_bins, w.cuts.n_z_bins, to_dev(ev.layer), to_dev(xyz),
                   to_dev(ev.cov.astype(np.float32)))
    bp = kf.build_params(w.cuts, arith=kf.ARITH_F64, state=kf.STATE_HYBRID)
    gh = {k: host(v) for k, v in kf.kf_build(w.geometry, bp, b, n, sg["par"], sg["cov"], sg["q"]).items()}
    F = w.cuts.first_layer
    true = ev.trk_hits[F:, :n]
    ec = ((gc["hits"][:, :n] == true).sum(axis=0) / true.shape[0] >= 0.75).mean()
    eh = ((gh["hits"][:, :n] == true).sum(axis=0) / true.shape[0] >= 0.75).mean()
    print(f"build efficiency, {n} seeds: Cartesian {ec:.4f}, hybrid {eh:.4f}")
    assert eh >= ec


def test_build_event_too_large(kf):
    """Event-local hit indices are 24 bits wide: a seed whose event holds
    2^24 binned hits is not built (status KF_TRK_EVENT_TOO_LARGE, no hits),
    while the seeds of a normal event in the same launch are built exactly as
    on their own."""
    w = presets.build()
    g = w.geometry
    ev = datagen.generate(g, w.gen, 3, 300)
    n0 = ev.n_tracks
    big = 1 << 24
    rng = np.random.default_rng(5)
    ph = rng.uniform(0, 2 * np.pi, big)
    R = g.r[5]
    xyz1 = np.stack([R * np.cos(ph), R * np.sin(ph), rng.uniform(-100, 100, big)]).astype(np.float32)
    del ph
    cov1 = np.zeros((6, big), np.float32)
    cov1[0] = cov1[3] = 1e-4
    cov1[5] = 1e-2
    xyz = np.concatenate([ev.xyz.astype(np.float32), xyz1], axis=1)
    cov = np.concatenate([ev.cov.astype(np.float32), cov1], axis=1)
    layer = np.concatenate([ev.layer, np.full(big, 5, np.int32)])
    hoff = np.array([0, ev.n_hits, ev.n_hits + big], np.int32)
    del xyz1, cov1
    b = kf.hit_bin(g, 63, 16, to_dev(layer), to_dev(xyz), to_dev(cov), event_offsets=to_dev(hoff))
    H = datagen.track_hits(ev)
    s = kf.kf_seed(g, n0, to_dev(H))
    ld = datagen.padded(n0 + 1)
    sp = torch.zeros((6, ld), device="cuda:0")
    sc = torch.zeros((21, ld), device="cuda:0")
    q = torch.ones(ld, dtype=torch.int8, device="cuda:0")
    sp[:, :n0], sc[:, :n0], q[:n0] = s["par"][:, :n0], s["cov"][:, :n0], s["q"][:n0]
    sp[:, n0], sc[:, n0], q[n0] = s["par"][:, 0], s["cov"][:, 0], s["q"][0]
    sev = torch.zeros(n0 + 1, dtype=torch.int32, device="cuda:0")
    sev[n0] = 1
    ex = kf.BuildExtra()
    ex.seed_event = sev.data_ptr()
    bp = kf.build_params(w.cuts, arith=kf.ARITH_F64)
    out = kf.kf_build(g, bp, b, n0 + 1, sp, sc, q, extra=ex)
    torch.cuda.synchronize()
    o = {k: host(v) for k, v in out.items()}
    del b
    assert o["status"][n0] == kf.TRK_EVENT_TOO_LARGE and o["nhits"][n0] == 0 and np.all(o["hits"][:, n0] == -1)
    ref, _ = gpu_build_event(kf, w, ev, kf.ARITH_F64, seeds=s)
    for k in ("hits", "nhits", "status", "chi2", "par"):
        assert np.array_equal(o[k][..., :n0], ref[k][..., :n0]), k
