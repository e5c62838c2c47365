"""Pins of the oracle's learned predictor (integer MLP 12->64->64->4).

Pins: the integer layers against numpy int64 matrix products; hand-set
weights with hand-computed outputs; zero weights give exactly the plain
encoding; a network that copies the last move predicts a uniformly moving
agent exactly, so its residual words vanish; the neighbour count against a
brute-force cell count; round-half-even input quantisation at half quanta.
"""
import struct

import numpy as np

import oracle
from tests.test_oracle_delta import rec, tam1

Q = 2.0 ** -12


def blob(w1, w2, w3, b1, b2, b3, r1, r2, r3, cell=24.0) -> bytes:
    """Predictor blob built from the format text (test helper)."""
    out = struct.pack("<II", int.from_bytes(b"TAP1", "little"), 1)
    out += np.asarray(w1, np.int8).tobytes() + np.asarray(w2, np.int8).tobytes() + np.asarray(w3, np.int8).tobytes()
    out += np.asarray(b1, np.int32).tobytes() + np.asarray(b2, np.int32).tobytes() + np.asarray(b3, np.int32).tobytes()
    out += bytes([r1, r2, r3]) + b"\0" * 5 + struct.pack("<d", cell)
    assert len(out) == 5672
    return out


def copy_last_move_blob():
    """q_k = in_k for |in_k| <= 127 via relu(in) - relu(-in)."""
    w1 = np.zeros((64, 12), np.int8)
    w2 = np.zeros((64, 64), np.int8)
    w3 = np.zeros((4, 64), np.int8)
    for k in range(4):
        w1[2 * k, k], w1[2 * k + 1, k] = 1, -1
        w3[k, 2 * k], w3[k, 2 * k + 1] = 1, -1
    for u in range(8):
        w2[u, u] = 1
    return blob(w1, w2, w3, np.zeros(64), np.zeros(64), np.zeros(4), 0, 0, 0)


def numpy_forward(w1, w2, w3, b1, b2, b3, r1, r2, r3, x):
    def rq(v, r):
        return np.floor_divide(v + ((1 << (r - 1)) if r else 0), 1 << r)
    x = x.astype(np.int64)
    h1 = np.clip(rq(x @ w1.astype(np.int64).T + b1, r1), 0, 127)
    h2 = np.clip(rq(h1 @ w2.astype(np.int64).T + b2, r2), 0, 127)
    return np.clip(rq(h2 @ w3.astype(np.int64).T + b3, r3), -(1 << 24), 1 << 24)


def test_integer_layers_match_int64_matmul():
    rng = np.random.default_rng(1)
    for r in [(0, 0, 0), (7, 9, 5), (12, 3, 20), (24, 24, 24)]:
        w1 = rng.integers(-128, 128, (64, 12))
        w2 = rng.integers(-128, 128, (64, 64))
        w3 = rng.integers(-128, 128, (4, 64))
        b1 = rng.integers(-2**24, 2**24, 64)
        b2 = rng.integers(-2**20, 2**20, 64)
        b3 = rng.integers(-2**24, 2**24, 4)
        m = oracle.mlp_struct(blob(w1, w2, w3, b1, b2, b3, *r))
        x = rng.integers(-32768, 32768, (300, 12))
        x[:, 8:] = rng.integers(0, 128, (300, 4))
        assert np.array_equal(oracle.mlp_forward(m, x), numpy_forward(w1, w2, w3, b1, b2, b3, *r, x))


def test_hand_set_weights():
    w1 = np.zeros((64, 12)); w2 = np.zeros((64, 64)); w3 = np.zeros((4, 64))
    w1[0, 0] = 1; w2[0, 0] = 1; w3[0, 0] = 1
    m = oracle.mlp_struct(blob(w1, w2, w3, np.zeros(64), np.zeros(64), np.zeros(4), 0, 0, 0))
    x = np.zeros((4, 12), np.int32)
    x[:, 0] = [5, -3, 300, 127]
    assert oracle.mlp_forward(m, x)[:, 0].tolist() == [5, 0, 127, 127]
    # r1 = 1: round half up of in/2 -> 5 -> 3, 4 -> 2, -3 -> 0 (relu)
    m = oracle.mlp_struct(blob(w1, w2, w3, np.zeros(64), np.zeros(64), np.zeros(4), 1, 0, 0))
    x[:, 0] = [5, 4, -3, 7]
    assert oracle.mlp_forward(m, x)[:, 0].tolist() == [3, 2, 0, 4]
    # output shift with negative values floors after adding half: (-5 + 1) >> 1 = -2
    w3[0, 0] = -1
    m = oracle.mlp_struct(blob(w1, w2, w3, np.zeros(64), np.zeros(64), np.zeros(4), 0, 0, 1))
    x[:, 0] = [5, 4, 3, 0]
    assert oracle.mlp_forward(m, x)[:, 0].tolist() == [-2, -2, -1, 0]


def _moving_pair(n=40, step=10):
    """Reference with history h1 = R - step*Q on x,y,z; current moved by step*Q again."""
    rng = np.random.default_rng(2)
    R, C = [], []
    h = oracle.History(n)
    for j in range(n):
        x = 100.0 + float(rng.integers(0, 1 << 20)) * Q
        r = rec(j + 1, x=x, words=9, fill=j)
        R.append(r)
        c = list(r)
        for k in range(3):
            v = np.array([r[2 + k]], np.uint64).view(np.float64)[0]
            c[2 + k] = int(np.array([v + step * Q], np.float64).view(np.uint64)[0])
            h.h1[j, k] = np.array([v - step * Q], np.float64).view(np.uint64)[0]
        h.h1[j, 3] = r[5]
        h.hlen[j] = 1
        C.append(c)
    return tam1(R), tam1(C), h


def test_zero_weights_give_the_plain_encoding():
    ref, cur, h = _moving_pair()
    z = oracle.mlp_struct(blob(*(np.zeros((64, 12)), np.zeros((64, 64)), np.zeros((4, 64))),
                               np.zeros(64), np.zeros(64), np.zeros(4), 0, 0, 0))
    st, enc_l, nref_l, mode, _ = oracle.delta_encode(cur, ref, z, h)
    st2, enc_p, nref_p, _, _ = oracle.delta_encode(cur, ref)
    assert st == st2 == 0 and mode == 0
    assert np.array_equal(enc_l, enc_p) and np.array_equal(nref_l, nref_p)


def test_exact_prediction_zeroes_the_residual():
    ref, cur, h = _moving_pair()
    m = oracle.mlp_struct(copy_last_move_blob())
    st, enc, nref, mode, hout = oracle.delta_encode(cur, ref, m, h)
    assert st == 0 and mode == 1
    hdr = struct.unpack_from("<IHBBIIIIQQQQQ", enc.tobytes(), 0)
    n, W, var_bytes = hdr[4], hdr[10], hdr[12]
    assert var_bytes == 0                        # every residual word is zero
    assert enc.size == 64 + 8 * ((n + 63) // 64) + 8 * ((W + 63) // 64) + ((W + 63) // 64 + 7) // 8 * 8
    st, dec, hdec = oracle.delta_decode(enc, ref, m, h)
    assert st == 0 and np.array_equal(dec, nref) and np.array_equal(nref, cur)
    # both sides advance the history identically: h2 <- h1, h1 <- R, hlen + 1
    assert np.array_equal(hout.h1, hdec.h1) and np.array_equal(hout.h2, hdec.h2)
    assert np.array_equal(hout.h2, h.h1) and np.all(hout.hlen == 2)
    # without history the same network predicts nothing
    st, enc0, _, mode0, _ = oracle.delta_encode(cur, ref, m, oracle.History(h.n))
    assert mode0 == 0


def test_neighbour_count_brute_force():
    rng = np.random.default_rng(4)
    cell = 24.0
    recs = [rec(j + 1, x=float(rng.integers(0, 5)) * 13.0 + 0.5) for j in range(60)]
    for r in recs:
        r[3] = int(np.array([float(rng.integers(0, 3)) * 30.0], np.float64).view(np.uint64)[0])
    ref = tam1(recs)
    h = oracle.History(60)
    h.hlen[:] = 1
    inp, pred = oracle.predictor_inputs(ref, h, cell)
    pos = [np.array(r[2:5], np.uint64).view(np.float64) for r in recs]
    for j in range(60):
        cj = tuple(np.floor(pos[j] / cell))
        cnt = sum(1 for p in pos if tuple(np.floor(p / cell)) == cj)
        assert inp[j, 8] == min(cnt, 127)
    assert np.all(pred == 1) and np.all(inp[:, 11] == 1)


def test_input_quantisation_rounds_half_to_even():
    deltas = [0.5, 1.5, 2.5, -0.5, -1.5, 40000.0, -40000.0, 3.25]
    expect = [0, 2, 2, 0, -2, 32767, -32768, 3]
    recs = [rec(j + 1, x=500.0) for j in range(len(deltas))]
    h = oracle.History(len(deltas))
    for j, d in enumerate(deltas):
        h.h1[j, 0] = np.array([500.0 - d * Q], np.float64).view(np.uint64)[0]
        h.h1[j, 1:] = recs[j][3:6]
        h.hlen[j] = 1
    inp, _ = oracle.predictor_inputs(tam1(recs), h, 24.0)
    assert inp[:, 0].tolist() == expect
    assert np.all(inp[:, 1:4] == 0) and np.all(inp[:, 4:8] == 0)
