"""Pins of the oracle's agent migration (Sec. 2.1, "Agent Migration"; records
as serialized in Sec. 2.2.1).

The paper: an agent that moves out of the locally owned space is moved to the
rank that owns its new position, packed by the same serialization as the aura
exchange.  Pins: the owning box found geometrically (the neighbour box that
contains the position, in exact rationals), consistency with the separately
pinned aura selection at w = 0 (the migrant direction is the largest of the
directions the agent is within 0 of), conservation of every agent's whole row
through select -> serialize -> apply with grid routing, the ordering rule of
the rebuilt store, and the error and capacity cases.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2509_24063_amd import synth

DIRS = [(c % 3 - 1, (c // 3) % 3 - 1, c // 9 - 1) for c in range(27) if c != 13]


def _world(grid=(2, 2, 2), median=1500, sigma=3.0, steps=2, seed=7, **over):
    cfg = synth.config(1, grid=grid, median=median, step_sigma=sigma, walls="domain", side=60.0, seed=seed,
                       ndirs=26, **over)
    w = synth.World(cfg)
    for _ in range(steps):
        w.step()
    return cfg, w.store


def _direction_by_geometry(pos, boxes, p, grid):
    """The direction whose neighbour box (the own box moved by d * side)
    contains pos, in exact rationals; (0, 0, 0) for the own box."""
    lo = [Fraction(v) for v in boxes[p, :3]]
    hi = [Fraction(v) for v in boxes[p, 3:]]
    x = [Fraction(v) for v in pos]
    hits = []
    for d in [(0, 0, 0)] + DIRS:
        inside = True
        for a in range(3):
            side = hi[a] - lo[a]
            if not (lo[a] + d[a] * side <= x[a] < hi[a] + d[a] * side):
                inside = False
        if inside:
            hits.append(d)
    assert len(hits) == 1  # the 27 boxes tile the space around the own box
    return hits[0]


def test_migrants_match_box_geometry():
    cfg, st = _world()
    idx, so = oracle.select_migrants(st)
    assert len(idx) > 50
    seg_of = {}
    for s in range(len(so) - 1):
        for i in idx[so[s]:so[s + 1]]:
            assert int(i) not in seg_of  # at most one direction per agent
            seg_of[int(i)] = s
    for p in range(st.P):
        for i in range(st.part_off[p], st.part_off[p + 1]):
            d = _direction_by_geometry(st.f64[:3, i], st.boxes, p, cfg.grid)
            if d == (0, 0, 0):
                assert i not in seg_of
            else:
                assert seg_of[i] == p * 26 + DIRS.index(d)


def test_migrant_direction_is_the_largest_aura_direction_at_zero_width():
    cfg, st = _world(seed=11)
    idx, so = oracle.select_migrants(st)
    aidx, aso = oracle.select_aura(st, 0.0, 26)
    aura_dirs = {}
    for s in range(len(aso) - 1):
        for i in aidx[aso[s]:aso[s + 1]]:
            aura_dirs.setdefault(int(i), []).append(DIRS[s % 26])
    got = {}
    for s in range(len(so) - 1):
        for i in idx[so[s]:so[s + 1]]:
            got[int(i)] = DIRS[s % 26]
    assert set(got) == set(aura_dirs)
    for i, ds in aura_dirs.items():
        best = max(ds, key=lambda d: abs(d[0]) + abs(d[1]) + abs(d[2]))
        assert got[i] == best
        # every aura direction of the agent is a sub-direction of its migrant direction
        for d in ds:
            assert all(d[a] in (0, best[a]) for a in range(3))


def test_segments_ascending_and_partition_local():
    cfg, st = _world(seed=3)
    idx, so = oracle.select_migrants(st)
    assert so[0] == 0 and np.all(np.diff(so) >= 0)
    for s in range(len(so) - 1):
        seg = idx[so[s]:so[s + 1]]
        p = s // 26
        assert np.all(np.diff(seg) > 0)
        assert np.all((seg >= st.part_off[p]) & (seg < st.part_off[p + 1]))


def _rows(st, schema, nf, ni):
    """uid -> (cls, nb, class fp64 fields, class int32 attributes, behaviour bytes)."""
    out = {}
    for i in range(st.n):
        c = int(st.cls[i])
        out[int(st.uid[i])] = (c, int(st.nb[i]), st.f64[:schema.n_f64[c], i].tobytes(),
                               st.i32[:schema.n_i32[c], i].tobytes(),
                               st.beh[st.beh_off[i]:st.beh_off[i + 1]].tobytes(),
                               st.f64[schema.n_f64[c]:nf, i].tobytes(), st.i32[schema.n_i32[c]:ni, i].tobytes())
    return out


def _apply(cfg, st, dest=None):
    idx, so = oracle.select_migrants(st)
    msgs, moff = oracle.serialize(st, cfg.schema, idx, so)
    if dest is None:
        dest = synth.neighbour_table(cfg.grid)
    nf, ni = max(cfg.schema.n_f64), max(cfg.schema.n_i32)
    status, out = oracle.migrate_apply(st, cfg.schema, msgs, moff, dest, nf, ni)
    return idx, so, msgs, moff, status, out


@pytest.mark.parametrize("over", [{}, dict(cyl_frac=0.3, n_f64=(4, 7), n_i32=(1, 3), nb_max=3,
                                         payload_words=(1, 4))])
def test_rows_conserved_and_every_agent_in_its_box(over):
    cfg, st = _world(seed=5, **over)
    nf, ni = max(cfg.schema.n_f64), max(cfg.schema.n_i32)
    idx, so, msgs, moff, status, out = _apply(cfg, st)
    assert status == oracle.OK
    assert len(idx) > 0
    assert out["sizes"][0] == st.n and out["sizes"][1] == st.beh.shape[0]
    new = synth.Store(uid=out["uid"], cls=out["cls"], nb=out["nb"], f64=out["f64"], i32=out["i32"],
                      beh_off=out["beh_off"], beh=out["beh"], part_off=out["part_off"], boxes=st.boxes)
    assert _rows(new, cfg.schema, nf, ni) == _rows(st, cfg.schema, nf, ni)
    for q in range(new.P):
        for i in range(new.part_off[q], new.part_off[q + 1]):
            for a in range(3):
                assert new.boxes[q, a] <= new.f64[a, i] < new.boxes[q, 3 + a]
    # nobody left to migrate
    idx2, _ = oracle.select_migrants(new)
    assert len(idx2) == 0


def test_order_kept_agents_then_messages_in_order():
    cfg, st = _world(seed=9)
    idx, so, msgs, moff, status, out = _apply(cfg, st)
    assert status == oracle.OK
    dest = synth.neighbour_table(cfg.grid)
    leaving = set(int(i) for i in idx)
    for q in range(st.P):
        kept = [int(st.uid[i]) for i in range(st.part_off[q], st.part_off[q + 1]) if i not in leaving]
        incoming = []
        for s in range(len(so) - 1):
            if dest[s] == q:
                incoming += [int(st.uid[i]) for i in idx[so[s]:so[s + 1]]]
        got = [int(u) for u in out["uid"][out["part_off"][q]:out["part_off"][q + 1]]]
        assert got == kept + incoming


def test_skipped_messages_and_single_partition_receiver():
    cfg, st = _world(seed=13)
    idx, so = oracle.select_migrants(st)
    msgs, moff = oracle.serialize(st, cfg.schema, idx, so)
    dest = np.full(len(so) - 1, -1, np.int32)
    status, out = oracle.migrate_apply(st, cfg.schema, msgs, moff, dest, 4, 1)
    assert status == oracle.OK and out["sizes"][0] == st.n - len(idx)
    # a one-partition receiver takes every message addressed to partition 0
    recv = st.partition(0)
    recv.f64[:3] = np.clip(recv.f64[:3], recv.boxes[0, :3, None], np.nextafter(recv.boxes[0, 3:, None], -np.inf))
    dest0 = np.zeros(len(so) - 1, np.int32)
    status, out = oracle.migrate_apply(recv, cfg.schema, msgs, moff, dest0, 4, 1)
    assert status == oracle.OK
    assert out["sizes"][0] == recv.n + len(idx)
    assert list(out["uid"][recv.n:]) == [int(st.uid[i]) for i in idx]


def test_capacity_reports_sizes():
    cfg, st = _world(seed=17)
    idx, so, msgs, moff, status, out = _apply(cfg, st)
    need = out["sizes"].copy()
    dest = synth.neighbour_table(cfg.grid)
    st2, out2 = oracle.migrate_apply(st, cfg.schema, msgs, moff, dest, 4, 1, cap=int(need[0]) - 1,
                                     beh_cap=int(need[1]))
    assert st2 == oracle.CAPACITY and np.array_equal(out2["sizes"], need)
    assert np.array_equal(out2["part_off"], out["part_off"])
    st3, _ = oracle.migrate_apply(st, cfg.schema, msgs, moff, dest, 4, 1, cap=int(need[0]),
                                  beh_cap=int(need[1]) - 8)
    assert st3 == oracle.CAPACITY


def _damage(msgs, moff, which):
    m = msgs.copy()
    a = int(moff[which])
    n = int(m[a + 8:a + 12].view(np.uint32)[0])
    rec0 = a + 32 + 8 * ((n + 1) // 2)
    return m, rec0


@pytest.mark.parametrize("case", ["magic", "dest", "class", "short", "uid0", "offset"])
def test_invalid_inputs(case):
    cfg, st = _world(seed=19)
    idx, so = oracle.select_migrants(st)
    msgs, moff = oracle.serialize(st, cfg.schema, idx, so)
    dest = synth.neighbour_table(cfg.grid).copy()
    s = int(np.flatnonzero(np.diff(so) > 0)[0])
    m, rec0 = _damage(msgs, moff, s)
    if case == "magic":
        m[int(moff[s])] ^= 1
    elif case == "dest":
        dest[s] = st.P
    elif case == "class":
        m[rec0 + 8:rec0 + 10] = np.frombuffer(np.uint16(7).tobytes(), np.uint8)
    elif case == "short":
        _short_record_case()
        return
    elif case == "uid0":
        m[rec0:rec0 + 8] = 0
    elif case == "offset":
        bad = moff.copy()
        bad[s + 1] += 4
        status, _ = oracle.migrate_apply(st, cfg.schema, m, bad, dest, 4, 1)
        assert status == oracle.INVALID
        return
    status, _ = oracle.migrate_apply(st, cfg.schema, m, moff, dest, 4, 1)
    assert status == oracle.INVALID


def _short_record_case():
    """A consistent message whose record is shorter than its class's fixed part:
    a class-0 record without behaviours (2 + 4 + 1 words) relabelled as class 1
    (2 + 7 + 2 words needed)."""
    cfg, st = _world(seed=23, cyl_frac=0.3, n_f64=(4, 7), n_i32=(1, 3))
    idx, so = oracle.select_migrants(st)
    msgs, moff = oracle.serialize(st, cfg.schema, idx, so)
    dest = synth.neighbour_table(cfg.grid)
    status, _ = oracle.migrate_apply(st, cfg.schema, msgs, moff, dest, 7, 3)
    assert status == oracle.OK
    for s in range(len(so) - 1):
        a = int(moff[s])
        n = int(msgs[a + 8:a + 12].view(np.uint32)[0])
        offs = msgs[a + 32:a + 32 + 4 * n].view(np.uint32)
        recs = a + 32 + 8 * ((n + 1) // 2)
        for r in range(n):
            at = recs + 8 * int(offs[r])
            hdr = int(msgs[at + 8:at + 16].view(np.uint64)[0])
            if hdr & 0xFFFF == 0 and hdr >> 32 == 7:
                m = msgs.copy()
                m[at + 8:at + 10] = np.frombuffer(np.uint16(1).tobytes(), np.uint8)
                assert oracle.view(m[a:int(moff[s + 1])])[0] == oracle.OK
                status, _ = oracle.migrate_apply(st, cfg.schema, m, moff, dest, 7, 3)
                assert status == oracle.INVALID
                return
    raise AssertionError("no behaviour-less class-0 migrant in the sample")
