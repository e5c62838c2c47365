"""fp64 reference of one training step of the learned predictor.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): the GPU trainer's
gradients are checked against it.  Plain numpy, written from the definition:

  parameters theta = W1 (64,12), b1 (64), W2 (64,64), b2 (64), W3 (4,64), b3 (4)
  (flattened in that order); the forward pass uses the rounded parameters
  (int8 weights, integer biases) exactly as the integer network does:
    z1 = floor((x W1q^T + b1q + 2^(r1-1)) / 2^r1), h1 = clamp(z1, 0, 127)
    z2 = floor((h1 W2q^T + b2q + 2^(r2-1)) / 2^r2), h2 = clamp(z2, 0, 127)
    o  = h2 W3q^T + b3q,  prediction qc = o / 2^r3 (in quanta of 2^-12 um)
  loss: mean over samples of sum_k |qc_k - t_k| (t: the true next move in
  quanta).  Backward: straight-through rounding (gradients pass the rounding
  of weights, biases and activations unchanged) and clamp masks 0 <= z <= 127.
  With quantize=False the rounding is left out (z = a / 2^r): a piecewise
  linear network whose gradient finite differences can check.
"""
import numpy as np

SHAPES = [("W1", (64, 12)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (4, 64)), ("b3", (4,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, at = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[at:at + n], np.float64).reshape(shape)
        at += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], np.float64).reshape(-1) for name, _ in SHAPES])


def rounded(p):
    q = {}
    for name, _ in SHAPES:
        v = np.rint(p[name])
        q[name] = np.clip(v, -128, 127) if name.startswith("W") else np.clip(v, -2**24, 2**24)
    return q


def forward(theta, x, r, quantize=True):
    p = unpack(theta)
    w = rounded(p) if quantize else p
    r1, r2, r3 = r
    x = np.asarray(x, np.float64)

    def layer(a, rr):
        if quantize:
            z = np.floor((a + (2.0 ** (rr - 1) if rr else 0.0)) / 2.0 ** rr)
        else:
            z = a / 2.0 ** rr
        return z, np.clip(z, 0, 127), ((z >= 0) & (z <= 127)).astype(np.float64)

    a1 = x @ w["W1"].T + w["b1"]
    z1, h1, m1 = layer(a1, r1)
    a2 = h1 @ w["W2"].T + w["b2"]
    z2, h2, m2 = layer(a2, r2)
    o = h2 @ w["W3"].T + w["b3"]
    return dict(w=w, x=x, h1=h1, m1=m1, h2=h2, m2=m2, qc=o / 2.0 ** r3)


def loss_and_grad(theta, x, t, r, quantize=True):
    """(loss, gradient of theta) for inputs x (n,12) and targets t (n,4)."""
    c = forward(theta, x, r, quantize)
    r1, r2, r3 = r
    n = x.shape[0]
    t = np.asarray(t, np.float64)
    diff = c["qc"] - t
    loss = np.abs(diff).sum() / n
    go = np.sign(diff) / 2.0 ** r3 / n
    w = c["w"]
    g = {"W3": go.T @ c["h2"], "b3": go.sum(0)}
    ga2 = (go @ w["W3"]) * c["m2"] / 2.0 ** r2
    g["W2"] = ga2.T @ c["h1"]
    g["b2"] = ga2.sum(0)
    ga1 = (ga2 @ w["W2"]) * c["m1"] / 2.0 ** r1
    g["W1"] = ga1.T @ c["x"]
    g["b1"] = ga1.sum(0)
    return loss, pack(g)
