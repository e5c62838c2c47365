"""Pins of the training oracle: its analytic backward against central finite
differences of its own loss on the smooth (unrounded) path, and its rounded
forward against the integer inference oracle."""
import numpy as np

import oracle
from oracle import train
from tests.test_oracle_predictor import blob


def _setup(rng, n=40):
    theta = np.concatenate([rng.normal(0, 6, 768), rng.normal(0, 200, 64), rng.normal(0, 4, 4096),
                            rng.normal(0, 100, 64), rng.normal(0, 6, 256), rng.normal(0, 50, 4)])
    x = rng.integers(-600, 600, (n, 12)).astype(np.float64)
    x[:, 8:] = rng.integers(0, 20, (n, 4))
    t = rng.normal(0, 300, (n, 4))
    return theta, x, t


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    theta, x, t = _setup(rng)
    r = (6, 7, 5)
    _, g = train.loss_and_grad(theta, x, t, r, quantize=False)
    idx = rng.choice(train.N_PARAMS, 300, replace=False)
    checked = 0
    for i in idx:
        eps = 1e-5 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        lp, _ = train.loss_and_grad(tp, x, t, r, quantize=False)
        lm, _ = train.loss_and_grad(tm, x, t, r, quantize=False)
        fd = (lp - lm) / (2 * eps)
        # kinks (clamp edges, |.| at 0) make a few central differences meaningless
        c0 = train.forward(theta, x, r, quantize=False)
        cp = train.forward(tp, x, r, quantize=False)
        if not (np.array_equal(c0["m1"], cp["m1"]) and np.array_equal(c0["m2"], cp["m2"]) and
                np.array_equal(np.sign(c0["qc"] - t), np.sign(cp["qc"] - t))):
            continue
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
        checked += 1
    assert checked > 200


def test_rounded_forward_is_the_integer_network():
    rng = np.random.default_rng(4)
    theta, x, t = _setup(rng, 200)
    r = (6, 7, 5)
    c = train.forward(theta, x, r, quantize=True)
    w = train.rounded(train.unpack(theta))
    b = blob(w["W1"], w["W2"], w["W3"], w["b1"], w["b2"], w["b3"], *r)
    q_int = oracle.mlp_forward(oracle.mlp_struct(b), x.astype(np.int32))
    o = c["qc"] * 2.0 ** r[2]
    assert np.array_equal(np.clip(np.floor((o + 2 ** (r[2] - 1)) / 2 ** r[2]), -2**24, 2**24), q_int)
