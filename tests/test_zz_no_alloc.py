"""The allocation-free build (kf_build_noalloc: workspace in the library's
static device array) against kf_build with a caller-allocated workspace, on
two calls in a row (the second smaller), through the C ABI; and its clear
error when a call needs more than the static array holds."""
import ctypes

import numpy as np
import pytest

from paper_1711_06571_amd import datagen, presets

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from gpu_common import host, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def kf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_06571_amd import kftrack
    return kftrack


def _inputs(kf, w, ev):
    b = kf.hit_bin(w.geometry, w.cuts.n_phi_bins, w.cuts.n_z_bins, to_dev(ev.layer),
                   to_dev(ev.xyz.astype(np.float32)), to_dev(ev.cov.astype(np.float32)))
    H = datagen.track_hits(ev)
    s = kf.kf_seed(w.geometry, ev.n_tracks, to_dev(H))
    return b, s


@pytest.mark.parametrize("arith", ["f64", "f32"])
def test_noalloc_build_equals_build(kf, arith):
    w = presets.build()
    a = kf.ARITH_F64 if arith == "f64" else kf.ARITH_F32
    bp = kf.build_params(w.cuts, arith=a)
    # two calls in a row, the second on a smaller event: the static array
    # keeps the first call's contents, which must not leak into the second
    for e, nt in ((0, w.n_tracks), (1, 1500)):
        ev = datagen.generate(w.geometry, w.gen, e, nt)
        n = ev.n_tracks
        b, s = _inputs(kf, w, ev)
        need = kf.kf_build_workspace_bytes(bp, b, n)
        assert need <= kf.kf_build_noalloc_max_bytes()
        ref = kf.kf_build(w.geometry, bp, b, n, s["par"], s["cov"], s["q"])
        torch.cuda.synchronize()
        ref = {k: host(v) for k, v in ref.items()}
        # outputs preallocated and poisoned, so every entry must be written
        out = {k: torch.full_like(torch.from_numpy(v).to("cuda:0"), -7) for k, v in ref.items()}
        torch.cuda.synchronize()
        got = kf.kf_build_noalloc(w.geometry, bp, b, n, s["par"], s["cov"], s["q"], out=out)
        torch.cuda.synchronize()
        for k, v in ref.items():
            gv = host(got[k])
            assert np.array_equal(gv[..., :n], v[..., :n]), f"{arith} event {e}: {k} differs"
        print(f"noalloc {arith} event {e} ({n} seeds, workspace {need} B): identical to kf_build")


def test_noalloc_rejects_calls_beyond_the_static_array(kf):
    """A batch whose workspace exceeds the static array: KF_E_WORKSPACE with a
    message, nothing launched (the descriptor's arrays are never read)."""
    w = presets.build()
    ev = datagen.generate(w.geometry, w.gen, 0, 200)
    b, s = _inputs(kf, w, ev)
    big = kf.BinnedHits(400, w.geometry.n_layers, w.cuts.n_phi_bins, w.cuts.n_z_bins, 10, "cuda:0")
    bp = kf.build_params(w.cuts, arith=kf.ARITH_F64)
    assert kf.kf_build_workspace_bytes(bp, big, ev.n_tracks) > kf.kf_build_noalloc_max_bytes()
    ex = kf.BuildExtra()
    sev = torch.zeros(s["par"].shape[1], dtype=torch.int32, device="cuda:0")
    ex.seed_event = sev.data_ptr()
    with pytest.raises(kf.KFError, match="status 2"):
        kf.kf_build_noalloc(w.geometry, bp, big, ev.n_tracks, s["par"], s["cov"], s["q"], extra=ex)
    buf = ctypes.create_string_buffer(256)
    kf.lib().kf_last_error(buf, 256)
    assert b"static scratch" in buf.value
    torch.cuda.synchronize()
