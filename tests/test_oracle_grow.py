"""Pins of the oracle's growth of viewed records (Sec. 2.2.1 "Mutability":
a record used in place may grow past its room; it moves to a block outside
the message and the old block is given up).

Pins: compaction of serialized (canonical) messages is the identity;
growing records by z words and compacting equals serializing the store in
which those agents carry z more zero words of behaviour bytes (ties both
functions to the separately pinned serializer); a grown record read through
its redirected offset holds its old words and zeros; growing again from the
arena; error and capacity cases."""
import numpy as np
import pytest

import oracle
from paper_2509_24063_amd import synth


def _messages(seed=4, n=800, ndirs=26):
    cfg = synth.config(1, median=n, seed=seed, ndirs=ndirs, w=40.0)
    st = synth.World(cfg).store
    idx, so = oracle.select_aura(st, cfg.w, cfg.ndirs)
    buf, moff = oracle.serialize(st, cfg.schema, idx, so)
    return cfg, st, idx, so, buf, moff


def _with_arena(buf, extra):
    out = np.zeros(buf.shape[0] + extra, np.uint8)
    out[: buf.shape[0]] = buf
    return out


def _record(buf, moff, s, r):
    a = int(moff[s])
    n = int(buf[a + 8:a + 12].view(np.uint32)[0])
    recs = a + 32 + 8 * ((n + 1) // 2)
    off = int(buf[a + 32 + 4 * r:a + 36 + 4 * r].view(np.uint32)[0])
    p = recs + 8 * off
    w = int(buf[p + 8:p + 16].view(np.uint64)[0]) >> 32
    return buf[p:p + 8 * w].view(np.uint64)


def test_compact_of_canonical_messages_is_identity():
    cfg, st, idx, so, buf, moff = _messages()
    status, out, ooff = oracle.view_compact(_with_arena(buf, 4096), moff)
    assert status == oracle.OK
    assert np.array_equal(ooff, moff) and np.array_equal(out, buf)


def _grown_store(st, idx, so, picks, z):
    """The store in which the agents of the picked (segment, record) pairs have
    z[k] more zero words at the end of their behaviour bytes."""
    extra = np.zeros(st.n, np.int64)
    for (s, r), zz in zip(picks, z):
        extra[int(idx[so[s] + r])] = 8 * zz
    old = st.beh_off
    lens = np.diff(old) + extra
    new_off = np.zeros(st.n + 1, np.int64)
    np.cumsum(lens, out=new_off[1:])
    beh = np.zeros(int(new_off[-1]), np.uint8)
    for i in range(st.n):
        beh[new_off[i]:new_off[i] + old[i + 1] - old[i]] = st.beh[old[i]:old[i + 1]]
    return synth.Store(uid=st.uid, cls=st.cls, nb=st.nb, f64=st.f64, i32=st.i32, beh_off=new_off, beh=beh,
                       part_off=st.part_off, boxes=st.boxes)


def _picks(so, rng, count, idx=None):
    """Distinct (segment, record) pairs, ascending; with idx, only records of
    agents that appear in one segment alone (so that growing the agent in the
    store grows exactly that record)."""
    once = None
    if idx is not None:
        u, c = np.unique(idx, return_counts=True)
        once = set(int(a) for a in u[c == 1])
    nonempty = [s for s in range(len(so) - 1) if so[s + 1] > so[s]]
    pairs = set()
    while len(pairs) < count:
        s = int(rng.choice(nonempty))
        r = int(rng.integers(0, so[s + 1] - so[s]))
        if once is not None and int(idx[so[s] + r]) not in once:
            continue
        pairs.add((s, r))
    return sorted(pairs)


def test_grow_then_compact_equals_serializing_the_grown_store():
    cfg, st, idx, so, buf, moff = _messages(seed=6)
    rng = np.random.default_rng(1)
    picks = _picks(so, rng, 40, idx)
    z = rng.integers(0, 4, len(picks))
    words = []
    for (s, r), zz in zip(picks, z):
        words.append(len(_record(buf, moff, s, r)) + int(zz))
    b = _with_arena(buf, 8 * sum(words) + 64)
    status, used = oracle.view_grow(b, moff, [p[0] for p in picks], [p[1] for p in picks], words)
    assert status == oracle.OK and used == 8 * sum(words)
    for (s, r), zz, w in zip(picks, z, words):
        rec = _record(b, moff, s, r)
        old = _record(buf, moff, s, r)
        assert len(rec) == w and np.array_equal(rec[2:len(old)], old[2:]) and rec[0] == old[0]
        assert int(rec[1]) >> 32 == w and (int(rec[1]) & 0xFFFFFFFF) == (int(old[1]) & 0xFFFFFFFF)
        assert not rec[len(old):].any()
    status, out, ooff = oracle.view_compact(b, moff)
    assert status == oracle.OK
    want, woff = oracle.serialize(_grown_store(st, idx, so, picks, z), cfg.schema, idx, so)
    assert np.array_equal(ooff, woff) and np.array_equal(out, want)


def test_grow_twice_from_the_arena():
    cfg, st, idx, so, buf, moff = _messages(seed=8)
    rng = np.random.default_rng(2)
    picks = _picks(so, rng, 10, idx)
    b = _with_arena(buf, 1 << 16)
    used = 0
    total = np.zeros(len(picks), np.int64)
    for step in range(3):
        words = [len(_record(b, moff, s, r)) + 1 for (s, r) in picks]
        status, used = oracle.view_grow(b, moff, [p[0] for p in picks], [p[1] for p in picks], words, used)
        assert status == oracle.OK
        total += 1
    status, out, ooff = oracle.view_compact(b, moff)
    want, woff = oracle.serialize(_grown_store(st, idx, so, picks, total), cfg.schema, idx, so)
    assert status == oracle.OK and np.array_equal(out, want)


@pytest.mark.parametrize("case", ["order", "smaller", "seg", "rec", "capacity", "arena_free"])
def test_grow_errors(case):
    cfg, st, idx, so, buf, moff = _messages(seed=10)
    rng = np.random.default_rng(3)
    picks = _picks(so, rng, 3)
    seg = [p[0] for p in picks]
    rec = [p[1] for p in picks]
    words = [len(_record(buf, moff, s, r)) + 1 for s, r in picks]
    b = _with_arena(buf, 4096)
    used = 0
    if case == "order":
        seg, rec, words = seg[::-1], rec[::-1], words[::-1]
    elif case == "smaller":
        words[1] -= 2
    elif case == "seg":
        seg[2] = len(so) - 1
    elif case == "rec":
        rec[2] = int(so[seg[2] + 1] - so[seg[2]])
    elif case == "capacity":
        b = _with_arena(buf, 8)
    elif case == "arena_free":
        # a record redirected into the arena's free part
        s, r = picks[0]
        a = int(moff[s])
        n = int(b[a + 8:a + 12].view(np.uint32)[0])
        recs = a + 32 + 8 * ((n + 1) // 2)
        b[a + 32 + 4 * r:a + 36 + 4 * r] = np.frombuffer(np.uint32((buf.shape[0] - recs) // 8).tobytes(), np.uint8)
    before = b.copy()
    status, used2 = oracle.view_grow(b, moff, seg, rec, words, used)
    assert status == (oracle.CAPACITY if case == "capacity" else oracle.INVALID)
    assert np.array_equal(b, before) and used2 == used
