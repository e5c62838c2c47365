"""Pins of the oracle's aura selection (Sec. 2.1, "Aura Update").

The paper: agents whose interaction region reaches into a neighbouring
partition box are copied to that neighbour, and the copied region is narrower
than the box.  Pins: an exact geometric brute force (agent inside the
neighbour box grown by w, in rational arithmetic on dyadic positions), the
face/edge/corner consistency of the 26 directions, the closed-form expected
count for uniform positions, and ordering/partition rules.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2509_24063_amd import synth

FACE_CODES = [4, 10, 12, 14, 16, 22]


def _dirs(ndirs):
    out = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dx, dy, dz) == (0, 0, 0):
                    continue
                if ndirs == 6 and abs(dx) + abs(dy) + abs(dz) != 1:
                    continue
                out.append((dx, dy, dz))
    return out


def _store_from_positions(pos, box):
    n = pos.shape[1]
    f64 = np.zeros((4, n))
    f64[:3] = pos
    f64[3] = 10.0
    return synth.make_store(uid=np.arange(1, n + 1), cls=np.zeros(n), nb=np.zeros(n), f64=f64,
                            i32=np.zeros((1, n)), beh_blocks=[[] for _ in range(n)], box=box)


def _brute(pos, box, w, ndirs):
    """Agent i goes to neighbour d iff it lies inside that neighbour's box
    (the own box translated by d * side) grown by w on every side; computed
    with exact rationals.  Boxes are half-open [lo, hi)."""
    lo = [Fraction(v) for v in box[:3]]
    hi = [Fraction(v) for v in box[3:]]
    side = [hi[a] - lo[a] for a in range(3)]
    W = Fraction(w)
    segs = []
    for d in _dirs(ndirs):
        members = []
        for i in range(pos.shape[1]):
            ok = True
            for a in range(3):
                x = Fraction(float(pos[a, i]))
                nlo, nhi = lo[a] + d[a] * side[a], hi[a] + d[a] * side[a]
                if not (nlo - W <= x < nhi + W):
                    ok = False
            if ok:
                members.append(i)
        segs.append(members)
    return segs


@pytest.mark.parametrize("ndirs", [6, 26])
def test_select_matches_geometric_brute_force(ndirs):
    rng = np.random.default_rng(11)
    box = [0.0, 0.0, 0.0, 64.0, 48.0, 80.0]
    w = 8.0
    # dyadic positions (multiples of 1/8), including points exactly on thresholds
    pos = np.stack([rng.integers(0, 8 * int(box[3 + a]), 60) / 8.0 for a in range(3)])
    pos[:, 0] = [8.0, 40.0, 72.0]          # exactly lo+w: outside lower slabs; exactly hi-w: inside upper
    pos[:, 1] = [7.875, 40.0 - 0.125, 0.0]
    store = _store_from_positions(pos, box)
    idx, seg_off = oracle.select_aura(store, w, ndirs)
    want = _brute(pos, box, w, ndirs)
    got = [list(idx[seg_off[k]:seg_off[k + 1]]) for k in range(ndirs)]
    assert got == want


def test_edges_and_corners_are_intersections_of_faces():
    rng = np.random.default_rng(5)
    pos = rng.random((3, 4000)) * 100.0
    store = _store_from_positions(pos, [0, 0, 0, 100, 100, 100])
    idx, seg_off = oracle.select_aura(store, 20.0, 26)
    sets = {d: set(idx[seg_off[k]:seg_off[k + 1]].tolist()) for k, d in enumerate(_dirs(26))}
    for d, members in sets.items():
        expect = set(range(pos.shape[1]))
        for a in range(3):
            if d[a] != 0:
                face = [0, 0, 0]
                face[a] = d[a]
                expect &= sets[tuple(face)]
        assert members == expect, d


def test_expected_count_closed_form():
    """For uniform positions the count of direction d is Binomial(N, prod_a p_a)
    with p_a = w/L on the axes where d_a != 0."""
    rng = np.random.default_rng(7)
    N, L, w = 200_000, 200.0, 24.0
    pos = rng.random((3, N)) * L
    store = _store_from_positions(pos, [0, 0, 0, L, L, L])
    idx, seg_off = oracle.select_aura(store, w, 26)
    counts = np.diff(seg_off)
    for k, d in enumerate(_dirs(26)):
        p = (w / L) ** sum(1 for v in d if v)
        mean, sd = N * p, np.sqrt(N * p * (1 - p))
        assert abs(counts[k] - mean) < 6 * sd, (d, counts[k], mean)


def test_order_and_partitions():
    cfg = synth.config(3, median=300.0)
    world = synth.World(cfg)
    s = world.store
    idx, seg_off = oracle.select_aura(s, cfg.w, 26)
    assert seg_off.shape[0] == s.P * 26 + 1
    for seg in range(s.P * 26):
        part = seg // 26
        m = idx[seg_off[seg]:seg_off[seg + 1]]
        assert np.all(np.diff(m) > 0)
        assert np.all((m >= s.part_off[part]) & (m < s.part_off[part + 1]))


def test_face_mode_codes_and_capacity():
    pos = np.array([[1.0], [1.0], [1.0]])
    store = _store_from_positions(pos, [0, 0, 0, 100, 100, 100])
    idx, seg_off = oracle.select_aura(store, 10.0, 6)
    # a corner agent near lo on every axis is in the three lower faces: codes 4, 10, 12
    assert [int(seg_off[k + 1] - seg_off[k]) for k in range(6)] == [1, 1, 1, 0, 0, 0]
    assert [c for c in FACE_CODES[:3]] == [4, 10, 12]
