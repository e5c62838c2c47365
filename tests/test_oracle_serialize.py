"""Pins of the oracle's TA IO serialization and view (Sec. 2.2.1).

The paper's example (Fig. 2) is a container of three agents with zero, one
and two behaviours, serialized by an in-order traversal that copies every
block and replaces the vtable pointer by a class id.  Pins: that example's
bytes assembled field by field from the TAM1 definition, an independent
parser that reads every record back into the agent's attributes, the size
identity, zero padding, and rejection of damaged messages.
"""
import os
import struct

import numpy as np
import pytest

import oracle
from paper_2509_24063_amd import synth
from tests.specparse import parse_tam1

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def fig2_store():
    """Three spheres with 0, 1 and 2 behaviours of 16 bytes."""
    f64 = np.array([[1.5, 2.5, 3.5], [4.0, 5.0, 6.0], [7.25, 8.25, 9.25], [10.0, 11.0, 12.0]])
    beh = [[], [(3, b"\x11" * 8)], [(4, b"\x22" * 8), (5, bytes(range(8)))]]
    return synth.make_store(uid=[101, 102, 103], cls=[0, 0, 0], nb=[0, 1, 2], f64=f64,
                            i32=[[7, -1, 2]], beh_blocks=beh, box=[0, 0, 0, 20, 20, 20])


def fig2_expected_bytes() -> bytes:
    """TAM1 of the three agents, built field by field from the format text."""
    recs = []
    fields = [(1.5, 4.0, 7.25, 10.0), (2.5, 5.0, 8.25, 11.0), (3.5, 6.0, 9.25, 12.0)]
    types = [7, -1, 2]
    behs = [b"", struct.pack("<II", 3, 8) + b"\x11" * 8,
            struct.pack("<II", 4, 8) + b"\x22" * 8 + struct.pack("<II", 5, 8) + bytes(range(8))]
    for i in range(3):
        words = 2 + 4 + 1 + len(behs[i]) // 8
        rec = struct.pack("<Q", 101 + i) + struct.pack("<HHI", 0, i, words)
        rec += struct.pack("<4d", *fields[i]) + struct.pack("<iI", types[i], 0) + behs[i]
        recs.append(rec)
    area = b"".join(recs)
    offs = struct.pack("<3I", 0, 7, 16) + b"\0" * 4
    hdr = struct.pack("<IHHIIQQ", int.from_bytes(b"TAM1", "little"), 1, 0, 3, 0, len(area) // 8, 0)
    return hdr + offs + area


def _golden_layout():
    vals = {}
    with open(os.path.join(GOLDEN, "fig2_layout.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split("=")
                vals[k.strip()] = [int(x) for x in v.split()]
    return vals


def test_fig2_example_bytes():
    s = fig2_store()
    idx = np.array([0, 1, 2], np.int32)
    buf, off = oracle.serialize(s, synth.Schema((4,), (1,)), idx, np.array([0, 3]))
    g = _golden_layout()
    assert buf.tobytes() == fig2_expected_bytes()
    assert buf.size == g["total_bytes"][0]
    assert list(np.frombuffer(buf[32:44].tobytes(), np.uint32)) == g["offsets"]
    recs = parse_tam1(buf.tobytes())
    assert [len(r) for r in recs] == g["record_words"]


def test_records_read_back_into_agent_attributes():
    cfg = synth.config(5, median=400.0, sigma=0.5, grid=(2, 1, 1))
    world = synth.World(cfg)
    s = world.store
    idx, seg_off = oracle.select_aura(s, cfg.w, 26)
    buf, msg_off = oracle.serialize(s, cfg.schema, idx, seg_off)
    for seg in range(seg_off.shape[0] - 1):
        msg = buf[msg_off[seg]:msg_off[seg + 1]].tobytes()
        recs = parse_tam1(msg)
        sel = idx[seg_off[seg]:seg_off[seg + 1]]
        assert len(recs) == sel.shape[0]
        words_total = 0
        for rec, a in zip(recs, sel):
            c = int(s.cls[a])
            F, I = cfg.n_f64[c], cfg.n_i32[c]
            assert rec[0] == int(s.uid[a])
            assert rec[1] & 0xFFFF == c and (rec[1] >> 16) & 0xFFFF == int(s.nb[a])
            assert rec[1] >> 32 == len(rec)
            got_f = np.array(rec[2:2 + F], np.uint64).view(np.float64)
            assert np.array_equal(got_f, s.f64[:F, a])
            ints = np.array(rec[2 + F:2 + F + (I + 1) // 2], np.uint64).view(np.int32)
            assert np.array_equal(ints[:I], s.i32[:I, a])
            if I % 2:
                assert ints[I] == 0
            beh = np.array(rec[2 + F + (I + 1) // 2:], np.uint64).view(np.uint8)
            assert np.array_equal(beh, s.beh[s.beh_off[a]:s.beh_off[a + 1]])
            words_total += len(rec)
        n = len(recs)
        assert len(msg) == 32 + 8 * ((n + 1) // 2) + 8 * words_total


def test_view_accepts_and_rejects():
    buf, off = oracle.serialize(fig2_store(), synth.Schema((4,), (1,)), np.array([0, 1, 2], np.int32),
                                np.array([0, 3]))
    st, n, rw = oracle.view(buf)
    assert (st, n, rw) == (0, 3, 27)
    bad = buf.copy()
    bad[0] ^= 1
    assert oracle.view(bad)[0] == oracle.INVALID
    assert oracle.view(buf[:-8])[0] == oracle.INVALID
    bad = buf.copy()
    bad[36] = 8                                   # second offset no longer the running sum
    assert oracle.view(bad)[0] == oracle.INVALID
    bad = buf.copy()
    bad[44] = 1                                   # offset table padding must be zero
    assert oracle.view(bad)[0] == oracle.INVALID
    bad = buf.copy()
    bad[48 + 12] = 6                              # first record claims 6 words instead of 7
    assert oracle.view(bad)[0] == oracle.INVALID
    empty, _ = oracle.empty_messages(1)
    assert oracle.view(empty)[:2] == (0, 0)


def test_empty_segments_and_multi_segment_offsets():
    s = fig2_store()
    idx = np.array([2, 0], np.int32)
    seg_off = np.array([0, 0, 1, 1, 2])
    buf, msg_off = oracle.serialize(s, synth.Schema((4,), (1,)), idx, seg_off)
    sizes = np.diff(msg_off)
    assert list(sizes) == [32, 32 + 8 + 88, 32, 32 + 8 + 56]
