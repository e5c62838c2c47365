"""Seeded synthetic agent populations and their dynamics.

This module is the only code shared by the HIP path and the CPU oracle, and it
is shared as *input* only: it creates agent stores and advances them between
exchanges.  It contains none of the exchange arithmetic (aura selection,
serialization, matching, residuals, packing or prediction).

The workloads stand in for the paper's BioDynaMo benchmark simulations (cell
clustering / proliferation, Sec. 3.1), which are not available: spheres with a
position, a diameter, an integer type and 0..2 small behaviours, moving by a
Gaussian random walk with division and death (Sec. 2.3 notes that positions
change gradually while type and diameter stay constant).

Store layout (struct of arrays, all partitions concatenated):
  uid      u64[n]          unique agent id, ((origin_partition+1) << 40) | counter
  cls      u16[n]          class id (0 = sphere, 1 = cylinder)
  nb       u16[n]          number of behaviour blocks
  f64      f64[F, n]       column k = fp64 field k (0..2 position, 3 diameter)
  i32      i32[I, n]       column k = int32 attribute k (0 = type)
  beh_off  i64[n+1]        byte offsets of each agent's behaviour blocks in beh
  beh      u8[beh_off[n]]  blocks: u32 class, u32 payload bytes (multiple of 8), payload
  part_off i64[P+1]        agents of partition p are [part_off[p], part_off[p+1])
  boxes    f64[P, 6]       lo0 lo1 lo2 hi0 hi1 hi2 of each partition box
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

UID_SHIFT = 40


@dataclasses.dataclass
class Store:
    uid: np.ndarray
    cls: np.ndarray
    nb: np.ndarray
    f64: np.ndarray
    i32: np.ndarray
    beh_off: np.ndarray
    beh: np.ndarray
    part_off: np.ndarray
    boxes: np.ndarray

    @property
    def n(self) -> int:
        return int(self.uid.shape[0])

    @property
    def P(self) -> int:
        return int(self.part_off.shape[0] - 1)

    def partition(self, p: int) -> "Store":
        """A copy of partition p alone, as a one-partition store."""
        a, b = int(self.part_off[p]), int(self.part_off[p + 1])
        bo = self.beh_off[a:b + 1]
        return Store(
            uid=self.uid[a:b].copy(), cls=self.cls[a:b].copy(), nb=self.nb[a:b].copy(),
            f64=np.ascontiguousarray(self.f64[:, a:b]), i32=np.ascontiguousarray(self.i32[:, a:b]),
            beh_off=(bo - bo[0]).astype(np.int64), beh=self.beh[int(bo[0]):int(bo[-1])].copy(),
            part_off=np.array([0, b - a], dtype=np.int64), boxes=self.boxes[p:p + 1].copy())


@dataclasses.dataclass
class Schema:
    n_f64: tuple
    n_i32: tuple


@dataclasses.dataclass
class Config:
    name: str
    seed: int
    grid: tuple            # partitions per axis
    side: float            # partition box side length (um)
    median: float          # agents per partition (median; exact when sigma == 0)
    sigma: float           # lognormal sigma of the partition sizes
    ndirs: int             # 6 (faces) or 26
    w: float               # aura width (um)
    step_sigma: float      # Gaussian step per axis (um)
    p_div: float
    p_death: float
    iterations: int
    cyl_frac: float = 0.0  # fraction of cylinders
    n_f64: tuple = (4,)
    n_i32: tuple = (1,)
    nb_max: int = 2
    payload_words: tuple = (1, 1)   # payload size range in 8-byte words (inclusive)
    persistent: bool = False        # AR(1) velocity and growing diameter
    sort_cells: bool = True
    walls: str = "box"              # "box": reflect at every partition box; "domain": only at the
                                    # union of the boxes, so agents can leave their partition's box

    @property
    def schema(self) -> Schema:
        return Schema(self.n_f64, self.n_i32)


def config(index: int, **over) -> Config:
    """The five workloads: 1 small correctness case, 2 one large partition,
    3 many uneven partitions, 4 predictor training/evaluation (config 1/2
    geometry), 5 heterogeneous large batched run."""
    base = dict(w=24.0, step_sigma=0.1, p_div=0.01, p_death=0.005)
    if index == 1:
        c = Config("cfg1", 2, (1, 1, 1), 200.0, 1e4, 0.0, 6, iterations=10, **base)
    elif index == 2:
        c = Config("cfg2", 3, (1, 1, 1), 1000.0, 1e7, 0.0, 26, iterations=50, **base)
    elif index == 3:
        side = (2e5 / 0.01) ** (1.0 / 3.0)
        c = Config("cfg3", 4, (8, 8, 8), side, 2e5, 1.0, 26, iterations=100, **base)
    elif index == 4:
        c = Config("cfg4", 5, (1, 1, 1), 200.0, 1e5, 0.0, 6, iterations=13, **base)
    elif index == 5:
        med = 2e8 / (256 * math.exp(0.5))
        side = (med / 0.01) ** (1.0 / 3.0)
        c = Config("cfg5", 6, (8, 8, 4), side, med, 1.0, 26, iterations=20, w=24.0,
                   step_sigma=0.1, p_div=0.02, p_death=0.01, cyl_frac=0.2,
                   n_f64=(14, 14), n_i32=(1, 3), nb_max=4, payload_words=(1, 7))
    else:
        raise ValueError(index)
    return dataclasses.replace(c, **over)


def neighbour_table(grid: tuple) -> np.ndarray:
    """int32[P*26]: for partition p of a gx x gy x gz grid of boxes (p = ix + gx
    (iy + gy iz)) and the k-th of the 26 directions (dx, dy, dz) in ascending
    order of (dx+1) + 3(dy+1) + 9(dz+1), the partition of the neighbouring box,
    or -1 past the edge of the grid.  This is the rank lookup a caller does to
    route migration messages; it is geometry, not part of the exchange."""
    gx, gy, gz = grid
    P = gx * gy * gz
    dirs = [(c % 3 - 1, (c // 3) % 3 - 1, c // 9 - 1) for c in range(27) if c != 13]
    out = np.full(P * 26, -1, dtype=np.int32)
    for p in range(P):
        ix, iy, iz = p % gx, (p // gx) % gy, p // (gx * gy)
        for k, (dx, dy, dz) in enumerate(dirs):
            jx, jy, jz = ix + dx, iy + dy, iz + dz
            if 0 <= jx < gx and 0 <= jy < gy and 0 <= jz < gz:
                out[p * 26 + k] = jx + gx * (jy + gy * jz)
    return out


def _behaviours(rng, nb: np.ndarray, pw: tuple):
    """Behaviour blocks for agents with nb[i] blocks each: (beh_off, beh bytes)."""
    nblk = int(nb.sum())
    k = rng.integers(pw[0], pw[1] + 1, size=nblk, dtype=np.int64)      # payload words
    blk_words = 1 + k
    agent_words = np.zeros(nb.shape[0], dtype=np.int64)
    owner = np.repeat(np.arange(nb.shape[0]), nb.astype(np.int64))
    np.add.at(agent_words, owner, blk_words)
    beh_off = np.zeros(nb.shape[0] + 1, dtype=np.int64)
    np.cumsum(agent_words * 8, out=beh_off[1:])
    words = np.empty(int(beh_off[-1] // 8), dtype=np.uint64)
    blk_start = np.zeros(nblk, dtype=np.int64)
    if nblk:
        np.cumsum(blk_words[:-1], out=blk_start[1:])
    bcls = rng.integers(1, 8, size=nblk, dtype=np.uint64)
    words[blk_start] = bcls | ((k.astype(np.uint64) * np.uint64(8)) << np.uint64(32))
    is_payload = np.ones(words.shape[0], dtype=bool)
    is_payload[blk_start] = False
    words[is_payload] = rng.integers(0, 2**63, size=int(is_payload.sum()), dtype=np.uint64) * np.uint64(2) \
        + rng.integers(0, 2, size=int(is_payload.sum()), dtype=np.uint64)
    return beh_off, words.view(np.uint8)


def _gather_beh(beh_off: np.ndarray, beh: np.ndarray, sel: np.ndarray):
    """Behaviour CSR of the agents sel (in that order)."""
    w = beh.view(np.uint64)
    lo = beh_off[sel] // 8
    ln = (beh_off[sel + 1] - beh_off[sel]) // 8
    off = np.zeros(sel.shape[0] + 1, dtype=np.int64)
    np.cumsum(ln * 8, out=off[1:])
    tot = int(off[-1] // 8)
    if tot == 0:
        return off, np.zeros(0, dtype=np.uint8)
    src = np.repeat(lo - off[:-1] // 8, ln) + np.arange(tot, dtype=np.int64)
    return off, w[src].view(np.uint8).copy()


class World:
    """A population plus its generator state; step() advances one iteration."""

    def __init__(self, cfg: Config, max_agents: int | None = None):
        self.cfg = cfg
        self.rng = np.random.Generator(np.random.PCG64(cfg.seed))
        rng = self.rng
        gx, gy, gz = cfg.grid
        P = gx * gy * gz
        if cfg.sigma > 0:
            z = rng.standard_normal(P)
            counts = np.rint(cfg.median * np.exp(cfg.sigma * z)).astype(np.int64)
        else:
            counts = np.full(P, int(round(cfg.median)), dtype=np.int64)
        if max_agents is not None:
            counts = np.minimum(counts, max_agents)
        counts = np.maximum(counts, 1)
        boxes = np.zeros((P, 6))
        p = 0
        for iz in range(gz):
            for iy in range(gy):
                for ix in range(gx):
                    lo = np.array([ix, iy, iz], dtype=np.float64) * cfg.side
                    boxes[p, :3] = lo
                    boxes[p, 3:] = lo + cfg.side
                    p += 1
        self.counter = np.zeros(P, dtype=np.int64)
        parts = []
        for p in range(P):
            parts.append(self._new_partition(p, int(counts[p]), boxes[p]))
        self.store = _concat(parts, boxes)
        if cfg.persistent:
            self.vel = np.zeros((3, self.store.n))
        else:
            self.vel = None

    # -- creation -------------------------------------------------------------
    def _new_partition(self, p: int, n: int, box: np.ndarray):
        cfg, rng = self.cfg, self.rng
        F, I = max(cfg.n_f64), max(cfg.n_i32)
        pos = np.empty((3, n))
        for a in range(3):
            pos[a] = box[a] + (box[3 + a] - box[a]) * rng.random(n)
            np.minimum(pos[a], np.nextafter(box[3 + a], -np.inf), out=pos[a])
        if cfg.sort_cells:
            c = np.floor((pos - box[:3, None]) / cfg.w).astype(np.int64)
            nc = int(math.ceil(cfg.side / cfg.w)) + 1
            key = (c[2] * nc + c[1]) * nc + c[0]
            pos = pos[:, np.argsort(key, kind="stable")]
        cls = (rng.random(n) < cfg.cyl_frac).astype(np.uint16) if cfg.cyl_frac > 0 else np.zeros(n, np.uint16)
        f64 = np.zeros((F, n))
        f64[:3] = pos
        f64[3] = rng.uniform(8.0, 12.0, n)
        if F > 4:
            f64[4:] = rng.random((F - 4, n))
        i32 = np.zeros((I, n), dtype=np.int32)
        i32[0] = rng.integers(0, 4, n, dtype=np.int32)
        if I > 1:
            i32[1:] = rng.integers(-2**31, 2**31, (I - 1, n), dtype=np.int64).astype(np.int32)
            ncls_i32 = np.array(cfg.n_i32)
            for k in range(1, I):
                i32[k, ncls_i32[cls] <= k] = 0
        if len(cfg.n_f64) > 1:
            ncls_f = np.array(cfg.n_f64)
            for k in range(4, F):
                f64[k, ncls_f[cls] <= k] = 0.0
        nb = rng.integers(0, cfg.nb_max + 1, n).astype(np.uint16)
        beh_off, beh = _behaviours(rng, nb, cfg.payload_words)
        uid = self._uids(p, n)
        return uid, cls, nb, f64, i32, beh_off, beh

    def _uids(self, p: int, n: int) -> np.ndarray:
        c0 = int(self.counter[p])
        self.counter[p] += n
        return (np.uint64(p + 1) << np.uint64(UID_SHIFT)) | np.arange(c0, c0 + n, dtype=np.uint64)

    # -- dynamics -------------------------------------------------------------
    def _reflect(self, x: np.ndarray, lo: np.ndarray, hi: np.ndarray):
        for a in range(3):
            xa = x[a]
            m = xa < lo[a]
            xa[m] = 2 * lo[a][m] - xa[m] if np.ndim(lo[a]) else 2 * lo[a] - xa[m]
            m = xa >= hi[a]
            xa[m] = 2 * hi[a][m] - xa[m] if np.ndim(hi[a]) else 2 * hi[a] - xa[m]
            np.clip(xa, lo[a], np.nextafter(hi[a], -np.inf), out=xa)

    def step(self):
        """One iteration: walk, death (stable compaction), division (daughters appended
        per partition)."""
        cfg, rng, s = self.cfg, self.rng, self.store
        n = s.n
        part_of = np.repeat(np.arange(s.P), np.diff(s.part_off))
        if cfg.walls == "domain":
            dlo, dhi = s.boxes[:, :3].min(axis=0), s.boxes[:, 3:].max(axis=0)
            lo = np.repeat(dlo[:, None], n, axis=1)
            hi = np.repeat(dhi[:, None], n, axis=1)
        else:
            lo = s.boxes[part_of, :3].T
            hi = s.boxes[part_of, 3:].T
        if cfg.persistent:
            self.vel = 0.9 * self.vel + rng.normal(0.0, cfg.step_sigma, (3, n))
            s.f64[:3] += self.vel
            s.f64[3] += 0.01
        else:
            s.f64[:3] += rng.normal(0.0, cfg.step_sigma, (3, n))
        self._reflect(s.f64[:3], lo, hi)
        # death: uniform without replacement, stable compaction
        k_death = int(round(cfg.p_death * n))
        alive = np.ones(n, dtype=bool)
        if k_death:
            alive[rng.choice(n, size=k_death, replace=False)] = False
        # division among survivors
        surv = np.flatnonzero(alive)
        k_div = int(round(cfg.p_div * surv.shape[0]))
        parents = np.sort(rng.choice(surv, size=k_div, replace=False)) if k_div else np.zeros(0, np.int64)
        dpart = part_of[parents]
        dpos = s.f64[:3, parents] + rng.normal(0.0, cfg.step_sigma, (3, k_div))
        if cfg.walls == "domain":
            self._reflect(dpos, lo[:, :k_div], hi[:, :k_div])
        else:
            self._reflect(dpos, s.boxes[dpart, :3].T, s.boxes[dpart, 3:].T)
        # new order: per partition, survivors then that partition's daughters
        keys = np.concatenate([part_of[surv] * 2, dpart * 2 + 1])
        src = np.concatenate([surv, parents])
        order = np.argsort(keys, kind="stable")
        src = src[order]
        is_d = np.concatenate([np.zeros(surv.shape[0], bool), np.ones(k_div, bool)])[order]
        f64 = s.f64[:, src]
        # parents are ascending, so their partitions are non-decreasing and the
        # stable sort keeps the daughters in parent order
        d_src_idx = np.flatnonzero(is_d)
        f64[:3, d_src_idx] = dpos
        uid = s.uid[src].copy()
        newp = part_of[src]
        for p in np.unique(newp[is_d]):
            m = d_src_idx[newp[d_src_idx] == p]
            uid[m] = self._uids(int(p), m.shape[0])
        beh_off, beh = _gather_beh(s.beh_off, s.beh, src)
        counts = np.bincount(newp, minlength=s.P)
        part_off = np.zeros(s.P + 1, dtype=np.int64)
        np.cumsum(counts, out=part_off[1:])
        self.store = Store(uid=uid, cls=s.cls[src], nb=s.nb[src], f64=np.ascontiguousarray(f64),
                           i32=np.ascontiguousarray(s.i32[:, src]), beh_off=beh_off, beh=beh,
                           part_off=part_off, boxes=s.boxes)
        if self.vel is not None:
            self.vel = self.vel[:, src]
        return self.store


def _concat(parts, boxes) -> Store:
    uid = np.concatenate([p[0] for p in parts])
    cls = np.concatenate([p[1] for p in parts])
    nb = np.concatenate([p[2] for p in parts])
    f64 = np.ascontiguousarray(np.concatenate([p[3] for p in parts], axis=1))
    i32 = np.ascontiguousarray(np.concatenate([p[4] for p in parts], axis=1))
    offs, behs, base = [np.zeros(1, np.int64)], [], 0
    for p in parts:
        offs.append(p[5][1:] + base)
        base += int(p[5][-1])
        behs.append(p[6])
    beh_off = np.concatenate(offs)
    beh = np.concatenate(behs) if behs else np.zeros(0, np.uint8)
    counts = np.array([p[0].shape[0] for p in parts], dtype=np.int64)
    part_off = np.zeros(len(parts) + 1, dtype=np.int64)
    np.cumsum(counts, out=part_off[1:])
    return Store(uid, cls, nb, f64, i32, beh_off, beh, part_off, boxes)


def make_store(uid, cls, nb, f64, i32, beh_blocks, box, part_off=None) -> Store:
    """Small hand-built store. beh_blocks[i] is a list of (class, payload bytes)."""
    n = len(uid)
    offs = [0]
    buf = bytearray()
    for blocks in beh_blocks:
        for bc, payload in blocks:
            assert len(payload) % 8 == 0
            buf += int(bc).to_bytes(4, "little") + len(payload).to_bytes(4, "little") + bytes(payload)
        offs.append(len(buf))
    boxes = np.asarray(box, dtype=np.float64).reshape(-1, 6)
    if part_off is None:
        part_off = [0, n]
    return Store(uid=np.asarray(uid, np.uint64), cls=np.asarray(cls, np.uint16), nb=np.asarray(nb, np.uint16),
                 f64=np.ascontiguousarray(np.asarray(f64, np.float64).reshape(-1, n)),
                 i32=np.ascontiguousarray(np.asarray(i32, np.int32).reshape(-1, n)),
                 beh_off=np.asarray(offs, np.int64), beh=np.frombuffer(bytes(buf), np.uint8).copy(),
                 part_off=np.asarray(part_off, np.int64), boxes=boxes)
