"""Pins of the byte-wise subtraction operator (the difference of Sec. 2.3,
which the paper leaves open; operator 1 in the TAD1 header, XOR is 0).

Each of a word's eight bytes is subtracted on its own modulo 256.  A byte
difference is zero exactly when the two bytes are equal, so the zero bytes
of the residual, and hence the word bitmap and every block size, are those
of the XOR encoding: only the significant bytes differ.  Pins: a
hand-computed encoding, identical layouts against XOR encodings of a walking
world (plain and learned), the spec decoder's byte-wise inversion of the
oracle's encodings, and the operator check on both sides."""
import struct

import numpy as np

import oracle
from paper_2509_24063_amd import synth
from tests.specparse import decode_tad1, parse_tam1
from tests.test_oracle_delta import rec, tam1
from tests.test_oracle_predictor import copy_last_move_blob


def test_hand_computed_subtraction_encoding():
    """Word 6 goes from 0x00FF to 0x0100: XOR would give 0x01FF; the byte
    differences are 0x00 - 0xFF = 0x01 and 0x01 - 0x00 = 0x01, so 0x0101,
    still two significant bytes."""
    r = rec(5, words=7, fill=0x00FF)
    c = list(r)
    c[6] = 0x0100
    ref, cur = tam1([r]), tam1([c])
    st, enc, nref, mode, _ = oracle.delta_encode(cur, ref, op=1)
    assert st == 0 and mode == 0
    expect = struct.pack("<IHBBIIIIQQQQQ", int.from_bytes(b"TAD1", "little"), 1, 0, 1, 1, 1, 0, 1, 7, 5, 7, 0, 8)
    expect += struct.pack("<Q", 1)          # presence: slot 0
    expect += struct.pack("<Q", 1 << 6)     # word bitmap: word 6
    expect += bytes([1]) + b"\0" * 7        # one group block of 8 bytes
    expect += bytes([0x02, 0x01, 0x01]) + b"\0" * 5   # nibble len=2, bytes 0x01 0x01, pad
    assert enc.tobytes() == expect
    assert nref.tobytes() == cur.tobytes()
    st, dec, _ = oracle.delta_decode(enc, ref, op=1)
    assert st == 0 and dec.tobytes() == cur.tobytes()
    # the XOR encoding of the same pair carries 0x01FF
    st, ex, _, _, _ = oracle.delta_encode(cur, ref)
    assert st == 0 and ex[-8:-5].tobytes() == bytes([0x02, 0xFF, 0x01])


def _layout_equal(a, b):
    """Same bytes except the operator field and the group blocks."""
    var = int(a[56:64].view(np.uint64)[0])
    assert a.size == b.size and int(b[56:64].view(np.uint64)[0]) == var
    assert a[:20].tobytes() == b[:20].tobytes() and a[24:a.size - var].tobytes() == b[24:b.size - var].tobytes()


def _world_pairs(persistent, iters=4):
    cfg = synth.config(1, median=3000.0, persistent=persistent)
    w = synth.World(cfg)
    for _ in range(iters):
        st = w.store
        idx, seg = oracle.select_aura(st, cfg.w, cfg.ndirs)
        yield cfg, oracle.serialize(st, cfg.schema, idx, seg)
        w.step()


def test_layout_equals_xor_and_spec_decoder_inverts():
    ref, ref_off = oracle.empty_messages(26)
    blocks_differ = 0
    for cfg, (buf, moff) in _world_pairs(False):
        ex, exo, xref, xoff, _, _ = oracle.encode_all(buf, moff, ref, ref_off)
        es, eso, sref, soff, _, _ = oracle.encode_all(buf, moff, ref, ref_off, op=1)
        assert np.array_equal(exo, eso) and np.array_equal(xref, sref) and np.array_equal(xoff, soff)
        for k in range(len(eso) - 1):
            a, b = ex[exo[k]:exo[k + 1]], es[eso[k]:eso[k + 1]]
            _layout_equal(a, b)
            assert int(b[20:24].view(np.uint32)[0]) == 1 and int(a[20:24].view(np.uint32)[0]) == 0
            blocks_differ += a.tobytes() != b.tobytes()
            assert decode_tad1(b.tobytes(), parse_tam1(ref[ref_off[k]:ref_off[k + 1]].tobytes())) == \
                parse_tam1(sref[soff[k]:soff[k + 1]].tobytes())
        dec, doff, _ = oracle.decode_all(es, eso, ref, ref_off, op=1)
        assert np.array_equal(dec, sref) and np.array_equal(doff, soff)
        ref, ref_off = sref, soff
    assert blocks_differ > 0


def test_learned_and_mixed_modes_keep_the_layout():
    m = oracle.mlp_struct(copy_last_move_blob())
    ref, ref_off = oracle.empty_messages(26)
    hist = oracle.History(0)
    seen = set()
    for persistent in (True, False):
        ref, ref_off = oracle.empty_messages(26)
        hist = oracle.History(0)
        for cfg, (buf, moff) in _world_pairs(persistent):
            ex, exo, xref, xoff, xm, xh = oracle.encode_all(buf, moff, ref, ref_off, m, hist)
            es, eso, sref, soff, sm, sh = oracle.encode_all(buf, moff, ref, ref_off, m, hist, op=1)
            assert np.array_equal(exo, eso) and np.array_equal(xm, sm) and np.array_equal(xref, sref)
            for k in range(len(eso) - 1):
                _layout_equal(ex[exo[k]:exo[k + 1]], es[eso[k]:eso[k + 1]])
            dec, doff, _ = oracle.decode_all(es, eso, ref, ref_off, m, hist, op=1)
            assert np.array_equal(dec, sref)
            seen |= set(int(v) for v in sm)
            ref, ref_off, hist = sref, soff, sh
    assert seen == {0, 1, 2}


def test_operator_checks():
    r = rec(5, words=7, fill=3)
    c = list(r)
    c[6] = 9
    ref, cur = tam1([r]), tam1([c])
    assert oracle.delta_encode(cur, ref, op=2)[0] == oracle.INVALID
    _, ex, _, _, _ = oracle.delta_encode(cur, ref)
    _, es, _, _, _ = oracle.delta_encode(cur, ref, op=1)
    assert oracle.delta_decode(ex, ref, op=1)[0] == oracle.INVALID    # made with XOR, receiver subtracts
    assert oracle.delta_decode(es, ref, op=0)[0] == oracle.INVALID
    bad = es.copy()
    bad[20] = 2                                                          # no operator 2
    assert oracle.delta_decode(bad, ref, op=1)[0] == oracle.CORRUPT
    assert oracle.delta_decode(bad, ref, op=0)[0] == oracle.CORRUPT
