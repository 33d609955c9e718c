"""GPU window-network kernels (BF16 MFMA, FP32 accumulation) against the FP64
network oracle: forward on BF16-rounded weights and activations, gradients
of the asymmetric quantile loss, and one Adam step."""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from gpu_common import host, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def kf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_06571_amd import kftrack
    return kftrack


def _setup(rng, n):
    mu = rng.normal(size=27).astype(np.float32).astype(np.float64)
    sd = rng.uniform(0.5, 2.0, size=27).astype(np.float32).astype(np.float64)
    p = omlp.init_params(rng, mu, sd, np.array([0.01, 0.1]))
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.1, p[k].shape).astype(np.float32).astype(np.float64)
    rows = np.zeros((n, 32), dtype=np.float32)
    rows[:, :27] = rng.normal(size=(n, 27)) * sd + mu
    rows[:, 27] = np.abs(rng.normal(size=n)) * 0.01
    rows[:, 28] = np.abs(rng.normal(size=n)) * 0.1
    return p, rows


def _oracle_params(p, sd_f32):
    q = dict(p)
    # the device standardises with 1/sd in FP32
    q["sd"] = 1.0 / np.float32(1.0 / sd_f32).astype(np.float64)
    return q


def test_forward_matches_oracle(kf, rng):
    p, rows = _setup(rng, 1000)  # ragged: 15 full waves and a partial one
    master = np.concatenate([p[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")]).astype(np.float32)
    blk = kf.mlp_block(master, p["mu"], p["sd"], p["scale"])
    w, o = kf.kf_mlp_forward(blk, to_dev(rows), logits=True)
    w, o = host(w), host(o)
    q = _oracle_params(p, p["sd"].astype(np.float32))
    ref = omlp.forward(q, rows[:, :27].astype(np.float64))
    assert np.allclose(o, ref["o"], rtol=0, atol=2e-3 * np.abs(ref["o"]).max())
    rel = np.abs(w - ref["w"]) / ref["w"]
    assert rel.max() < 5e-3, rel.max()
    assert np.median(rel) < 1e-4


def test_gradient_matches_oracle(kf, rng):
    p, rows = _setup(rng, 4096)
    master = np.concatenate([p[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")]).astype(np.float32)
    blk = kf.mlp_block(master, p["mu"], p["sd"], p["scale"])
    g = host(kf.kf_mlp_grad(blk, to_dev(rows)))
    q = _oracle_params(p, p["sd"].astype(np.float32))
    c = omlp.forward(q, rows[:, :27].astype(np.float64))
    d = rows[:, 27:29].astype(np.float64)
    ref = omlp.backward(q, c, d)
    loss = omlp.loss(c["w"], d)
    assert abs(g[-1] / loss - 1) < 1e-3
    gp = kf.mlp_split(g[:-1])
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        err = np.linalg.norm(gp[k] - ref[k]) / np.linalg.norm(ref[k])
        assert err < 2e-2, (k, err)


def test_adam_step_matches_oracle(kf, rng):
    p, rows = _setup(rng, 256)
    master = np.concatenate([p[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")]).astype(np.float32)
    blk = kf.mlp_block(master, p["mu"], p["sd"], p["scale"])
    grad = rng.normal(size=kf.MLP_NPARAM + 1).astype(np.float32) * 1e-2
    mst, m, v = to_dev(master), torch.zeros(kf.MLP_NPARAM, device="cuda:0"), torch.zeros(kf.MLP_NPARAM,
                                                                                         device="cuda:0")
    gd = to_dev(grad)
    for t in (1, 2, 3):
        kf.kf_mlp_adam(blk, mst, m, v, gd, t)
    ref_master = {k: v_.astype(np.float64) for k, v_ in kf.mlp_split(master).items()}
    om = {k: np.zeros_like(ref_master[k]) for k in ref_master}
    ov = {k: np.zeros_like(ref_master[k]) for k in ref_master}
    gsplit = {k: v_.astype(np.float64) for k, v_ in kf.mlp_split(grad[:-1]).items()}
    for t in (1, 2, 3):
        work = omlp.adam_step(ref_master, gsplit, om, ov, t)
    got = kf.mlp_split(host(mst))
    for k in ref_master:
        assert np.allclose(got[k], ref_master[k], rtol=1e-5, atol=1e-7), k
    # the block's BF16 weights are the rounded masters
    blk2 = kf.mlp_block(host(mst), p["mu"], p["sd"], p["scale"])
    assert np.array_equal(host(blk)[192:], host(blk2)[192:])
