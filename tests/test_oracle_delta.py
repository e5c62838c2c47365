"""Pins of the oracle's delta encoding (Sec. 2.3).

The paper: sender and receiver keep the same reference; agents present in
both are moved to their reference position, vanished ones leave a
placeholder, new ones are appended; the difference is written for matched
agents; the receiver restores the message from the reference and removes the
placeholders (the original order is not restored).  Pins: an O(n^2)
brute-force match, a hand-computed encoding, an independent spec decoder,
closed-form sizes for cur == ref and for an empty reference, the round trip
on adversarial inputs, and rejection of damaged or mismatched encodings.
"""
import struct

import numpy as np
import pytest

import oracle
from paper_2509_24063_amd import synth
from tests.specparse import decode_tad1, parse_tam1


def tam1(records):
    """Build a TAM1 message from records (lists of words) -- test helper."""
    n = len(records)
    offs, at = [], 0
    for r in records:
        offs.append(at)
        at += len(r)
    body = struct.pack(f"<{n}I", *offs) + (b"\0" * 4 if n % 2 else b"")
    area = b"".join(struct.pack(f"<{len(r)}Q", *r) for r in records)
    hdr = struct.pack("<IHHIIQQ", int.from_bytes(b"TAM1", "little"), 1, 0, n, 0, at, 0)
    return np.frombuffer(hdr + body + area, np.uint8).copy()


def rec(uid, x=1.0, words=7, cls=0, nb=0, fill=0):
    r = [uid, cls | (nb << 16) | (words << 32)]
    r += list(np.array([x, 2.0, 3.0, 10.0], np.float64).view(np.uint64))[: max(0, min(4, words - 2))]
    r += [fill] * (words - len(r))
    return [int(v) for v in r]


def brute_match(cur_recs, ref_recs):
    m = []
    for r in ref_recs:
        hit = [i for i, c in enumerate(cur_recs) if c[0] == r[0] and c[1] == r[1]]
        m.append(hit[0] if hit else -1)
    used = set(i for i in m if i >= 0)
    return m, [i for i in range(len(cur_recs)) if i not in used]


def roundtrip(cur, ref):
    st, enc, nref, mode, _ = oracle.delta_encode(cur, ref)
    assert st == 0
    st, dec, _ = oracle.delta_decode(enc, ref)
    assert st == 0
    assert np.array_equal(dec, nref)
    return enc, nref


def test_hand_computed_encoding():
    """One record whose x changed in its lowest byte: D = [0,0,1,0,0,0,0]."""
    r = rec(5, x=1.0)
    c = list(r)
    c[2] ^= 0x01
    ref, cur = tam1([r]), tam1([c])
    st, enc, nref, mode, _ = oracle.delta_encode(cur, ref)
    assert st == 0 and mode == 0
    expect = struct.pack("<IHBBIIIIQQQQQ", int.from_bytes(b"TAD1", "little"), 1, 0, 1, 1, 1, 0, 0, 7, 5, 7, 0, 8)
    expect += struct.pack("<Q", 1)          # presence: slot 0
    expect += struct.pack("<Q", 1 << 2)     # word bitmap: word 2
    expect += bytes([1]) + b"\0" * 7        # one group block of 8 bytes
    expect += bytes([0x01, 0x01]) + b"\0" * 6   # nibble len=1, byte 0x01, pad
    assert enc.tobytes() == expect
    assert nref.tobytes() == cur.tobytes()


def test_match_against_brute_force_and_canonical_order():
    rng = np.random.default_rng(3)
    for trial in range(20):
        uids = rng.choice(np.arange(1, 60), size=40, replace=False)
        ref_recs = [rec(int(u), x=float(rng.random()), words=int(rng.integers(2, 10))) for u in uids[:25]]
        cur_recs = []
        for r in ref_recs:
            if rng.random() < 0.8:
                c = list(r)
                if len(c) > 2:
                    c[2] ^= int(rng.integers(0, 1 << 40))
                if rng.random() < 0.1:       # same uid, other shape -> gone + new
                    c = rec(c[0], words=len(c) + 1)
                cur_recs.append(c)
        cur_recs += [rec(int(u), words=int(rng.integers(2, 10))) for u in uids[25:]]
        order = rng.permutation(len(cur_recs))
        cur_recs = [cur_recs[i] for i in order]
        enc, nref = roundtrip(tam1(cur_recs), tam1(ref_recs))
        m, new = brute_match(cur_recs, ref_recs)
        expect = [cur_recs[i] for i in m if i >= 0] + [cur_recs[i] for i in new]
        assert parse_tam1(nref.tobytes()) == expect
        assert decode_tad1(enc.tobytes(), ref_recs) == expect


def test_size_when_cur_equals_ref():
    cfg = synth.config(1)
    s = synth.World(cfg).store
    idx, seg = oracle.select_aura(s, cfg.w, 6)
    buf, off = oracle.serialize(s, cfg.schema, idx, seg)
    for k in range(6):
        msg = buf[off[k]:off[k + 1]]
        _, n, W = oracle.view(msg)
        enc, nref = roundtrip(msg, msg)
        G = (W + 63) // 64
        assert enc.size == 64 + 8 * ((n + 63) // 64) + 8 * G + (G + 7) // 8 * 8
        assert np.array_equal(nref, msg)


def test_size_against_empty_reference():
    cfg = synth.config(1)
    s = synth.World(cfg).store
    idx, seg = oracle.select_aura(s, cfg.w, 6)
    buf, off = oracle.serialize(s, cfg.schema, idx, seg)
    empty, _ = oracle.empty_messages(1)
    msg = buf[off[0]:off[1]]
    _, n, W = oracle.view(msg)
    enc, nref = roundtrip(msg, empty)
    assert enc.size == 64 + (4 * n + 7) // 8 * 8 + 8 * W
    assert np.array_equal(nref, msg)      # R empty: C' == C


def test_adversarial_roundtrips():
    a = [rec(u, x=float(u)) for u in range(1, 50)]
    empty = tam1([])
    cases = [
        (empty, empty), (tam1(a), empty), (empty, tam1(a)), (tam1(a), tam1(a)),
        (tam1([rec(u + 1000) for u in range(1, 50)]), tam1(a)),       # all new
        (tam1([rec(1, x=2.0)]), tam1([rec(1)])),                          # one record
    ]
    for words in (2, 3):                                                   # W = 64k +- 1
        n = 64 * 3 // words + 1
        r = [rec(u, words=words, fill=u) for u in range(1, n + 1)]
        c = [list(x) for x in r]
        for x in c:
            x[-1] ^= 0xFF00FF
        cases.append((tam1(c), tam1(r)))
    for cur, ref in cases:
        enc, nref = roundtrip(cur, ref)
        # C' holds the same records as C (as a multiset)
        assert sorted(map(tuple, parse_tam1(nref.tobytes()))) == sorted(map(tuple, parse_tam1(cur.tobytes())))


def test_cur_in_reference_order_restores_cur_exactly():
    cfg = synth.config(1)
    w = synth.World(cfg)
    s = w.store
    idx, seg = oracle.select_aura(s, cfg.w, 6)
    buf, off = oracle.serialize(s, cfg.schema, idx, seg)
    ref = buf[off[2]:off[3]]
    s2 = w.step()
    idx2, seg2 = oracle.select_aura(s2, cfg.w, 6)
    buf2, off2 = oracle.serialize(s2, cfg.schema, idx2, seg2)
    cur = buf2[off2[2]:off2[3]]
    _, _, cprime, _, _ = oracle.delta_encode(cur, ref)
    # encoding C' (already in reference order) against R returns C' itself
    _, enc, nref, _, _ = oracle.delta_encode(cprime, ref)
    st, dec, _ = oracle.delta_decode(enc, ref)
    assert st == 0 and np.array_equal(dec, cprime) and np.array_equal(nref, cprime)


def test_invalid_inputs():
    assert oracle.delta_encode(tam1([rec(1), rec(1)]), tam1([]))[0] == oracle.INVALID      # duplicate uid
    assert oracle.delta_encode(tam1([rec(0)]), tam1([]))[0] == oracle.INVALID              # uid 0
    assert oracle.delta_encode(tam1([]), tam1([rec(2), rec(2)]))[0] == oracle.INVALID      # bad reference


def test_damaged_or_mismatched_encodings_are_rejected():
    rng = np.random.default_rng(9)
    r = [rec(u, x=float(rng.random()), words=int(rng.integers(6, 11))) for u in range(1, 200)]
    c = [list(x) for x in r[10:]] + [rec(900 + u) for u in range(5)]
    for x in c:
        x[2] ^= int(rng.integers(1, 1 << 44))
    ref, cur = tam1(r), tam1(c)
    st, enc, nref, _, _ = oracle.delta_encode(cur, ref)
    assert st == 0
    assert oracle.delta_decode(enc[:-8], ref)[0] == oracle.CORRUPT                       # truncated
    other = tam1(r[:-1] + [rec(5000)])
    assert oracle.delta_decode(enc, other)[0] == oracle.REF_MISMATCH                     # other reference
    bad = enc.copy()
    bad[32] ^= 1                                                                           # uid fold
    assert oracle.delta_decode(bad, ref)[0] == oracle.REF_MISMATCH
    bad = enc.copy()
    bad[12] ^= 1                                                                           # n_match
    assert oracle.delta_decode(bad, ref)[0] == oracle.CORRUPT
    # the first group block starts after the new records; make its first nibble 0
    hdr = np.frombuffer(enc[:64].tobytes(), np.uint64)
    var_at = enc.size - int(hdr[7])
    bad = enc.copy()
    bad[var_at] &= 0xF0
    assert oracle.delta_decode(bad, ref)[0] == oracle.CORRUPT
    # arbitrary single-byte damage never crashes: either an error or some decode
    for _ in range(300):
        bad = enc.copy()
        bad[rng.integers(0, enc.size)] ^= np.uint8(1 << rng.integers(0, 8))
        st, out, _ = oracle.delta_decode(bad, ref)
        # INVALID: the operator field now names subtraction, which this receiver is not set to
        assert st in (0, oracle.CORRUPT, oracle.REF_MISMATCH, oracle.INVALID)


def test_multi_iteration_world_roundtrip_and_compression():
    cfg = synth.config(1)
    w = synth.World(cfg)
    ref, ref_off = oracle.empty_messages(6)
    for it in range(4):
        s = w.store
        idx, seg = oracle.select_aura(s, cfg.w, 6)
        buf, off = oracle.serialize(s, cfg.schema, idx, seg)
        enc, eoff, nref, noff, _, _ = oracle.encode_all(buf, off, ref, ref_off)
        dec, doff, _ = oracle.decode_all(enc, eoff, ref, ref_off)
        assert np.array_equal(dec, nref) and np.array_equal(doff, noff)
        for k in range(6):
            assert decode_tad1(enc[eoff[k]:eoff[k + 1]].tobytes(),
                               parse_tam1(ref[ref_off[k]:ref_off[k + 1]].tobytes())) == \
                parse_tam1(nref[noff[k]:noff[k + 1]].tobytes())
        if it > 0:
            assert enc.size < 0.4 * buf.size       # positions move ~0.1 um: most bytes vanish
        ref, ref_off = nref, noff
        w.step()


@pytest.mark.parametrize("op", [0, 1])
def test_packer_against_bitwise_encoder(op):
    """The whole plain encoding, byte for byte, against an encoder built bit
    by bit from the format (tests/specparse.encode_tad1): residual words of
    every significant-byte length 1..8 (and zero) at random word positions,
    several 64-word groups with a ragged last one, vanished and new records.
    A non-minimal length, a swapped nibble order or a misplaced byte in the
    oracle's packer changes the bytes."""
    from tests.specparse import _undiff, encode_tad1

    rng = np.random.default_rng(101 + op)
    seen = set()
    for trial in range(12):
        nref = int(rng.integers(1, 48))
        uids = rng.choice(np.arange(1, 5000), size=nref + 8, replace=False)
        ref_recs = [rec(int(u), x=float(rng.normal()), words=int(rng.integers(2, 24)),
                        fill=int(rng.integers(0, 1 << 63))) for u in uids[:nref]]
        cur_recs = []
        for r in ref_recs:
            if rng.random() < 0.15:  # vanished
                continue
            c = list(r)
            for q in range(2, len(c)):
                L = int(rng.integers(0, 9))
                if L == 0:
                    continue
                d = int(rng.integers(1 << (8 * (L - 1)), 1 << min(63, 8 * L))) if L < 8 else \
                    int(rng.integers(1 << 56, 1 << 63)) | (int(rng.integers(0, 2)) << 63)
                assert (d.bit_length() + 7) // 8 == L
                seen.add(L)
                c[q] = _undiff(r[q], d, op)
            cur_recs.append(c)
        for u in uids[nref:nref + int(rng.integers(0, 8))]:  # new
            cur_recs.append(rec(int(u), words=int(rng.integers(2, 12)), fill=7))
        order = rng.permutation(len(cur_recs))
        cur_recs = [cur_recs[i] for i in order]
        st, enc, nref_msg, mode, _ = oracle.delta_encode(tam1(cur_recs), tam1(ref_recs), op=op)
        assert st == 0 and mode == 0
        assert enc.tobytes() == encode_tad1(cur_recs, ref_recs, op)
    assert seen == set(range(1, 9))
