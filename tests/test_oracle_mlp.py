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


def _adam_state():
    master = {k: np.zeros(1) for k in mlp.TRAINABLE}
    m = {k: np.zeros(1) for k in mlp.TRAINABLE}
    v = {k: np.zeros(1) for k in mlp.TRAINABLE}
    return master, m, v


def test_adam_steps_by_hand():
    """Adam (Kingma and Ba, Algorithm 1) worked by hand on scalars.

    Step 1: the bias-corrected moments are g and g^2, so every weight moves
    by lr * g / (|g| + eps) whatever beta1, beta2 are (lr * sign(g) when
    |g| >> eps, lr / 2 when |g| = eps: eps sits outside the square root).
    Step 2 after gradients g1, g2: the corrected moments are the weighted
    means (beta1 g1 + g2) / (1 + beta1) and (beta2 g1^2 + g2^2) / (1 + beta2).
    A constant gradient keeps moving by lr * g / (|g| + eps) at every step.
    Dropping the bias correction, squaring inside the wrong moment or moving
    eps under the root each fails one of these."""
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    g_vals = {"W1": 0.5, "b1": -2.0, "W2": 1e-8, "b2": 3.0, "W3": -1e-8, "b3": 0.25}
    master, m, v = _adam_state()
    grads = {k: np.array([g_vals[k]]) for k in mlp.TRAINABLE}
    work = mlp.adam_step(master, grads, m, v, 1, lr=lr, beta1=b1, beta2=b2, eps=eps)
    for k, g in g_vals.items():
        expect = -lr * g / (abs(g) + eps)
        assert abs(master[k][0] - expect) <= 1e-15, (k, master[k][0], expect)
    # |g| = eps: half a step, not lr * g / sqrt(g^2 + eps)
    assert abs(master["W2"][0] + lr / 2) < 1e-15
    # the working copy: BF16 weight matrices, FP32-exact biases
    assert work["W1"][0] == mlp.bf16(master["W1"])[0] and work["b1"][0] == master["b1"][0]

    # step 2 with a second gradient of opposite sign: (g1, g2) = (1, -1)
    master, m, v = _adam_state()
    for t, g in ((1, 1.0), (2, -1.0)):
        grads = {k: np.array([g]) for k in mlp.TRAINABLE}
        mlp.adam_step(master, grads, m, v, t, lr=lr, beta1=b1, beta2=b2, eps=eps)
    mhat = (b1 * 1.0 + (-1.0)) / (1 + b1)          # -0.0526...
    vhat = (b2 * 1.0 + 1.0) / (1 + b2)             # 1
    expect = -lr * 1.0 / (1.0 + eps) - lr * mhat / (np.sqrt(vhat) + eps)
    for k in mlp.TRAINABLE:
        assert abs(master[k][0] - expect) <= 1e-15, (k, master[k][0], expect)

    # constant gradient for five steps: five equal moves
    master, m, v = _adam_state()
    for t in range(1, 6):
        grads = {k: np.array([0.3]) for k in mlp.TRAINABLE}
        mlp.adam_step(master, grads, m, v, t, lr=lr, beta1=b1, beta2=b2, eps=eps)
    for k in mlp.TRAINABLE:
        assert abs(master[k][0] - (-5 * lr * 0.3 / (0.3 + eps))) <= 1e-14
