"""Oracle pins for the search-window network: finite-difference gradients,
the closed-form optimum of the asymmetric loss, and agreement of the two
independent forward implementations (NumPy and C)."""
import numpy as np
from scipy.stats import norm

import oracle
from oracle import mlp


def _params(rng):
    mu = rng.normal(size=27)
    sd = rng.uniform(0.5, 2.0, size=27)
    p = mlp.init_params(rng, mu, sd, np.array([0.01, 0.1]))
    p["b1"] = rng.normal(0, 0.1, 64)
    p["b2"] = rng.normal(0, 0.1, 64)
    p["b3"] = rng.normal(0, 0.1, 2)
    return p


def test_backward_matches_central_differences(rng):
    p = _params(rng)
    x = rng.normal(size=(32, 27)) * p["sd"] + p["mu"]
    d = np.abs(rng.normal(size=(32, 2))) * np.array([0.01, 0.1])
    c = mlp.forward(p, x, round_bf16=False)
    g = mlp.backward(p, c, d)
    for k in mlp.TRAINABLE:
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            h = 1e-6
            old = flat[i]
            flat[i] = old + h
            lp = mlp.loss(mlp.forward(p, x, round_bf16=False)["w"], d)
            flat[i] = old - h
            lm = mlp.loss(mlp.forward(p, x, round_bf16=False)["w"], d)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-4), (k, i, fd, an)


def test_quantile_optimum():
    """Constant input, d = |N(0, s^2)|: training converges to the 20/21
    quantile of |N|, s * Phi^-1(41/42)."""
    rng = np.random.default_rng(3)
    s = np.array([0.02, 0.3])
    p = mlp.init_params(rng, np.zeros(27), np.ones(27), np.array([0.01, 0.1]))
    x = np.zeros((512, 27))
    master = {k: p[k].copy() for k in mlp.TRAINABLE}
    m = {k: np.zeros_like(master[k]) for k in mlp.TRAINABLE}
    v = {k: np.zeros_like(master[k]) for k in mlp.TRAINABLE}
    for t in range(1, 2501):
        d = np.abs(rng.normal(size=(512, 2))) * s
        c = mlp.forward(p, x, round_bf16=False)
        g = mlp.backward(p, c, d)
        work = mlp.adam_step(master, g, m, v, t, lr=3e-3 if t < 1500 else 2e-4)
        for k in mlp.TRAINABLE:
            p[k] = master[k].copy()
    w = mlp.forward(p, x[:1], round_bf16=False)["w"][0]
    expect = s * norm.ppf(41.0 / 42.0)
    assert np.all(np.abs(w / expect - 1) < 0.01), (w, expect)


def test_c_and_numpy_forward_agree(rng):
    p = _params(rng)
    b = mlp.blob(p)
    assert b.size == oracle.mlp_blob_size()
    x = rng.normal(size=(64, 27)) * p["sd"] + p["mu"]
    w_np = mlp.forward(p, x)["w"]
    for i in range(64):
        w_c = oracle.mlp_forward(b, x[i])
        assert np.allclose(w_c, w_np[i], rtol=1e-12, atol=0)


def test_bf16_rounding():
    # exact halfway cases round to even; values already representable stay
    v = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -7, -2.5, 3.0e38])
    r = mlp.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2.0 ** -6 and r[3] == 1.0 + 2.0 ** -7
    assert r[4] == -2.5
    assert np.isfinite(r[5]) or r[5] == np.inf
