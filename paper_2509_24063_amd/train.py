"""Training the learned predictor on the GPU.

harvest(): runs exchanges of a synthetic world through the library with the
  encoder's window tap on; each predicted slot yields one window (the 12
  predictor inputs and the true move of words 2..5 in quanta of 2^-12 um).
  A zero-weight predictor with the wanted cell side drives the encoder, so the
  windows are exactly the inputs a trained predictor will later see.
fit(): Adam on the library's quantisation-aware forward/backward kernels,
  mini-batches taken from a shuffled copy of the windows, cosine learning
  rate; returns the predictor blob (int8/int32 parameters, shifts, cell).

The network and its encoding are the learned-prediction rule of the exchange
(an addition to the paper's delta encoding, Sec. 2.3); nothing here is used
by an exchange itself.
"""
from __future__ import annotations

import math
import struct

import numpy as np
import torch

from . import native, synth

SHIFTS = (3, 7, 1)
BLOB_LEN = 5672


def zero_blob(cell: float = 24.0) -> bytes:
    head = struct.pack("<II", int.from_bytes(b"TAP1", "little"), 1)
    body = bytes(768 + 4096 + 256 + 4 * (64 + 64 + 4) + 8)
    return head + body + struct.pack("<d", cell)


def harvest(ctx: native.Context, world: synth.World, iterations: int, cap: int, cell: float = 24.0):
    """(inputs int32 [n,12], targets float32 [n,4]) on the device from
    `iterations` exchanges of `world` (advanced in place)."""
    cfg = world.cfg
    inputs = torch.empty((cap, 12), dtype=torch.int32, device="cuda")
    targets = torch.empty((cap, 4), dtype=torch.float32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    pred = native.Predictor(ctx, zero_blob(cell))
    ref, roff = native.empty_messages(cfg.ndirs * world.store.P)
    hist = native.History(0)
    ctx.set_window_tap(inputs, targets, count)
    try:
        for _ in range(iterations):
            ds = native.DeviceStore(world.store)
            idx, seg = ctx.select_aura(ds, cfg.w, cfg.ndirs)
            buf, moff = ctx.serialize(ds, idx, seg)
            nrec = int(seg[-1].item())
            hout = native.History(nrec)
            enc, eoff, nref, noff, _ = ctx.delta_encode(buf, moff, ref, roff, pred=pred, hist=hist, hist_out=hout)
            ctx.check("harvest")
            ref, roff, hist = nref[: int(noff[-1].item())].clone(), noff.clone(), hout
            world.step()
    finally:
        ctx.set_window_tap()
    n = int(count.item())
    if n > cap:
        raise RuntimeError(f"window capacity {cap} too small for {n} windows")
    return inputs[:n], targets[:n]


def init_params(seed: int = 1, scale: float = 8.0) -> np.ndarray:
    """Weights ~ N(0, scale^2) (in int8 units), biases 0; layout W1 b1 W2 b2 W3 b3."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, scale, 768), np.zeros(64), rng.normal(0, scale, 4096), np.zeros(64),
             rng.normal(0, scale, 256), np.zeros(4)]
    return np.concatenate(parts).astype(np.float32)


def fit(ctx: native.Context, inputs, targets, steps: int = 1500, batch: int = 4096, lr: float = 0.5,
        shifts=SHIFTS, cell: float = 24.0, seed: int = 1, log=None) -> bytes:
    n = inputs.shape[0]
    if n == 0:
        raise ValueError("no training windows")
    tr = native.Trainer(ctx, init_params(seed), shifts, cell)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    batch = min(batch, n)
    perm, at = None, n
    for k in range(1, steps + 1):
        if at + batch > n:  # reshuffle once per pass over the windows
            perm = torch.randperm(n, device="cuda", generator=g)
            xs, ts = inputs[perm].contiguous(), targets[perm].contiguous()
            at = 0
        lrk = lr * 0.5 * (1.0 + math.cos(math.pi * k / steps))
        tr.step(xs[at:at + batch], ts[at:at + batch], lr=lrk)
        at += batch
        if log and (k % 250 == 0 or k == steps):
            loss, _ = tr.grad(inputs, targets)
            log(f"step {k}: mean L1 loss {loss:.1f} quanta")
    blob = tr.export()
    tr.close()
    return blob
