"""Seeded synthetic populations generated and advanced on the GPU.

The workloads with 1.7e8 and 2e8 agents are too large for the host generator
(synth.World takes minutes per state at that size).  DeviceWorld follows the
same recipe on the GPU with torch, drawing from torch's seeded generator
instead of numpy's (so its states differ from World's, statistically alike):

  - a periodic grid of partition boxes with lognormal sizes (the partition
    sizes are drawn exactly as World draws them);
  - per partition, uniform positions sorted by aura-wide cell, diameters
    U[8,12], the class (sphere, or cylinder with probability cyl_frac), the
    class's further fp64 fields U[0,1) and int32 attributes, 0..nb_max
    behaviour blocks (u32 class 1..7, u32 payload bytes, 1..7 random payload
    words), uids ((partition + 1) << 40 | counter);
  - per iteration: a Gaussian walk reflected at the partition box, deaths
    uniform without replacement, divisions among the survivors (a daughter
    is a copy of its parent with a new uid and its own step), the store
    rebuilt per partition as survivors then daughters.

Input only: none of the exchange arithmetic is here.  The population lives
in the buffers of a fixed-capacity store (native.DeviceStore.alloc), which it
rewrites in place each iteration, so captured graphs stay valid.
"""
from __future__ import annotations

import math

import numpy as np

from . import synth


class DeviceWorld:
    def __init__(self, cfg: synth.Config, store, device="cuda", log=None):
        """store: a native.DeviceStore from DeviceStore.alloc with room for the
        population and its growth (see capacity())."""
        import torch
        self.torch = torch
        self.cfg, self.ds, self.dev = cfg, store, torch.device(device)
        self.gen = torch.Generator(device=self.dev)
        self.gen.manual_seed(cfg.seed)
        counts, boxes = partition_sizes(cfg)
        P = counts.shape[0]
        self.P = P
        self.boxes = torch.from_numpy(boxes).to(self.dev)
        n = int(counts.sum())
        if n > store.n:
            raise ValueError("store too small for the population")
        self.counter = torch.from_numpy(counts.astype(np.int64)).to(self.dev)
        self.n = n
        self._init_population(torch.from_numpy(counts).to(self.dev), log)

    # -- sizes ------------------------------------------------------------------
    @staticmethod
    def capacity(cfg: synth.Config, iterations: int, slack: float = 1.02):
        """(agents, behaviour bytes) a store needs for `iterations` steps of
        growth (division among survivors minus death) from the initial size."""
        counts, _ = partition_sizes(cfg)
        n = float(counts.sum())
        growth = ((1.0 - cfg.p_death) * (1.0 + cfg.p_div)) ** iterations
        agents = int(n * growth * slack) + 4096
        mean_blk = 8.0 * (1.0 + 0.5 * (cfg.payload_words[0] + cfg.payload_words[1]))
        beh = (int(agents * 0.5 * cfg.nb_max * mean_blk * 1.02) + (1 << 20)) // 8 * 8
        return agents, beh

    # -- helpers ------------------------------------------------------------------
    def _rand(self, *shape):
        return self.torch.rand(*shape, generator=self.gen, device=self.dev, dtype=self.torch.float64)

    def _randn(self, *shape):
        return self.torch.randn(*shape, generator=self.gen, device=self.dev, dtype=self.torch.float64)

    def _randint(self, lo, hi, n, dtype=None):
        torch = self.torch
        return torch.randint(lo, hi, (n,), generator=self.gen, device=self.dev, dtype=dtype or torch.int64)

    def _part_of(self, n):
        torch = self.torch
        po = self.ds.part_off
        return torch.repeat_interleave(torch.arange(self.P, device=self.dev), po[1:] - po[:-1], output_size=n)

    def _reflect(self, x, part):
        """Reflect positions x [3, m] of agents in partitions `part` at their boxes."""
        torch = self.torch
        for a in range(3):
            lo = self.boxes[part, a]
            hi = self.boxes[part, 3 + a]
            xa = x[a]
            xa.copy_(torch.where(xa < lo, 2 * lo - xa, xa))
            xa.copy_(torch.where(xa >= hi, 2 * hi - xa, xa))
            xa.copy_(torch.minimum(torch.maximum(xa, lo), torch.nextafter(hi, torch.full_like(hi, -math.inf))))

    # -- creation -------------------------------------------------------------------
    def _init_population(self, counts, log):
        torch, cfg, ds, n = self.torch, self.cfg, self.ds, self.n
        P = self.P
        F, I = max(cfg.n_f64), max(cfg.n_i32)
        part = torch.repeat_interleave(torch.arange(P, device=self.dev), counts, output_size=n)
        lo = self.boxes[part, :3].T
        pos = lo + cfg.side * self._rand(3, n)
        for a in range(3):
            hi = self.boxes[part, 3 + a]
            pos[a] = torch.minimum(pos[a], torch.nextafter(hi, torch.full_like(hi, -math.inf)))
        if cfg.sort_cells:
            nc = int(math.ceil(cfg.side / cfg.w)) + 1
            c = torch.floor((pos - lo) / cfg.w).to(torch.int64).clamp_(0, nc - 1)
            key = ((part * nc + c[2]) * nc + c[1]) * nc + c[0]
            order = torch.sort(key, stable=True).indices
            pos = pos[:, order]
            del key, c, order
        del lo
        cls = (self._rand(n) < cfg.cyl_frac).to(torch.int16) if cfg.cyl_frac > 0 else \
            torch.zeros(n, dtype=torch.int16, device=self.dev)
        ds.f64[:3, :n] = pos
        del pos
        ds.f64[3, :n] = 8.0 + 4.0 * self._rand(n)
        nf = torch.tensor(cfg.n_f64, device=self.dev)[cls.long()]
        for k in range(4, F):
            ds.f64[k, :n] = torch.where(nf > k, self._rand(n), torch.zeros((), dtype=torch.float64, device=self.dev))
        ni = torch.tensor(cfg.n_i32, device=self.dev)[cls.long()]
        ds.i32[0, :n] = self._randint(0, 4, n, torch.int32)
        for k in range(1, I):
            v = self._randint(-2**31, 2**31, n).to(torch.int32)
            ds.i32[k, :n] = torch.where(ni > k, v, torch.zeros((), dtype=torch.int32, device=self.dev))
        del nf, ni
        ds.cls[:n] = cls
        nb = self._randint(0, cfg.nb_max + 1, n)
        ds.nb[:n] = nb.to(torch.int16)
        # behaviour blocks: u32 class | u32 payload bytes, then the payload words
        nblk = int(nb.sum().item())
        k = self._randint(cfg.payload_words[0], cfg.payload_words[1] + 1, nblk)
        owner = torch.repeat_interleave(torch.arange(n, device=self.dev), nb, output_size=nblk)
        agent_words = torch.zeros(n, dtype=torch.int64, device=self.dev).index_add_(0, owner, 1 + k)
        del owner
        ds.beh_off[0] = 0
        torch.cumsum(agent_words * 8, 0, out=ds.beh_off[1:n + 1])
        total = int(ds.beh_off[n].item())
        if total > ds.beh.numel():
            raise ValueError("behaviour buffer too small for the population")
        words = ds.beh[:total].view(torch.int64)
        # random payload words, filled in chunks
        step = 1 << 27
        for a in range(0, words.numel(), step):
            b = min(words.numel(), a + step)
            words[a:b] = torch.randint(-2**63, 2**63 - 1, (b - a,), generator=self.gen, device=self.dev,
                                       dtype=torch.int64)
        start = torch.zeros(nblk, dtype=torch.int64, device=self.dev)
        if nblk:
            torch.cumsum(1 + k[:-1], 0, out=start[1:])
        bcls = self._randint(1, 8, nblk)
        words[start] = bcls | ((k * 8) << 32)
        del start, bcls, k, nb, agent_words
        if n < ds.n:
            ds.beh_off[n + 1:] = total
        # uids: partition + 1 above bit 40, a counter per partition
        first = torch.zeros(P, dtype=torch.int64, device=self.dev)
        torch.cumsum(counts[:-1], 0, out=first[1:])
        local = torch.arange(n, device=self.dev) - first[part]
        ds.uid[:n] = ((part + 1) << synth.UID_SHIFT) | local
        ds.part_off[0] = 0
        torch.cumsum(counts, 0, out=ds.part_off[1:])
        del part, local, first
        ds.live = n
        if self.dev.type == "cuda":
            torch.cuda.synchronize()
        if log:
            log(f"device population: {n} agents, {total} behaviour bytes")

    # -- dynamics --------------------------------------------------------------------
    def step(self):
        """One iteration: walk, deaths, divisions; the store rewritten in place."""
        torch, cfg, ds, n, P = self.torch, self.cfg, self.ds, self.n, self.P
        part = self._part_of(n)
        x = ds.f64[:3, :n]
        x += cfg.step_sigma * self._randn(3, n)
        self._reflect(x, part)
        k_death = int(round(cfg.p_death * n))
        alive = torch.ones(n, dtype=torch.bool, device=self.dev)
        if k_death:
            alive[torch.randperm(n, generator=self.gen, device=self.dev)[:k_death]] = False
        surv = torch.nonzero(alive).squeeze(1)
        del alive
        k_div = int(round(cfg.p_div * surv.shape[0]))
        pick = torch.randperm(surv.shape[0], generator=self.gen, device=self.dev)[:k_div]
        parents = torch.sort(surv[pick]).values
        del pick
        dpart = part[parents]
        dpos = ds.f64[:3, parents] + cfg.step_sigma * self._randn(3, k_div)
        self._reflect(dpos, dpart)
        keys = torch.cat([part[surv] * 2, dpart * 2 + 1])
        src = torch.cat([surv, parents])
        order = torch.sort(keys, stable=True).indices
        del keys
        src = src[order]
        is_d = torch.cat([torch.zeros(surv.shape[0], dtype=torch.bool, device=self.dev),
                          torch.ones(k_div, dtype=torch.bool, device=self.dev)])[order]
        del order, surv
        m = src.shape[0]
        if m > ds.n:
            raise ValueError(f"store capacity {ds.n} exceeded ({m} agents)")
        newpart = part[src]
        del part
        # behaviours of the new order (gathered word by word into a new buffer)
        old_off = ds.beh_off[: n + 1]
        lens = (old_off[src + 1] - old_off[src]) // 8
        new_off = torch.zeros(m + 1, dtype=torch.int64, device=self.dev)
        torch.cumsum(lens * 8, 0, out=new_off[1:])
        total = int(new_off[m].item())
        if total > ds.beh.numel():
            raise ValueError("behaviour buffer capacity exceeded")
        old_words = ds.beh.view(torch.int64)
        new_words = torch.empty(total // 8, dtype=torch.int64, device=self.dev)
        chunk = 1 << 24
        for a in range(0, m, chunk):
            b = min(m, a + chunk)
            ln = lens[a:b]
            w0, w1 = int(new_off[a].item()) // 8, int(new_off[b].item()) // 8
            if w1 == w0:
                continue
            base = old_off[src[a:b]] // 8 - new_off[a:b] // 8
            idx = torch.repeat_interleave(base, ln, output_size=w1 - w0) + torch.arange(w0, w1, device=self.dev)
            new_words[w0:w1] = old_words[idx]
            del idx, base, ln
        ds.beh[:total].view(torch.int64).copy_(new_words)
        del new_words, lens
        # columns of the new order
        for col in (ds.uid, ds.cls, ds.nb):
            col[:m] = col[src]
        for k in range(ds.f64.shape[0]):
            ds.f64[k, :m] = ds.f64[k, src]
        for k in range(ds.i32.shape[0]):
            ds.i32[k, :m] = ds.i32[k, src]
        d_idx = torch.nonzero(is_d).squeeze(1)
        ds.f64[:3, d_idx] = dpos
        del dpos, is_d
        # daughters' uids: per partition, the next counter values in parent order
        if k_div:
            firstd = torch.searchsorted(dpart, dpart)
            rank = torch.arange(k_div, device=self.dev) - firstd
            ds.uid[d_idx] = ((dpart + 1) << synth.UID_SHIFT) | (self.counter[dpart] + rank)
            self.counter += torch.bincount(dpart, minlength=P)
            del firstd, rank
        ds.beh_off[: m + 1] = new_off
        if m < ds.n:
            ds.beh_off[m + 1:] = total
        cnt = torch.bincount(newpart, minlength=P)
        ds.part_off[0] = 0
        torch.cumsum(cnt, 0, out=ds.part_off[1:])
        del newpart, src, parents, dpart, d_idx, new_off
        self.n = m
        ds.live = m

    # -- host copies ---------------------------------------------------------------------
    def partition_host(self, p: int) -> synth.Store:
        """Partition p's agents copied to the host, as a one-partition store."""
        ds = self.ds
        po = ds.part_off.cpu().numpy()
        a, b = int(po[p]), int(po[p + 1])
        bo = ds.beh_off[a:b + 1].cpu().numpy()
        return synth.Store(
            uid=ds.uid[a:b].cpu().numpy().view(np.uint64), cls=ds.cls[a:b].cpu().numpy().view(np.uint16),
            nb=ds.nb[a:b].cpu().numpy().view(np.uint16), f64=np.ascontiguousarray(ds.f64[:, a:b].cpu().numpy()),
            i32=np.ascontiguousarray(ds.i32[:, a:b].cpu().numpy()), beh_off=(bo - bo[0]).astype(np.int64),
            beh=ds.beh[int(bo[0]):int(bo[-1])].cpu().numpy(), part_off=np.array([0, b - a], np.int64),
            boxes=ds.boxes.cpu().numpy().reshape(-1, 6)[p:p + 1].copy())


def partition_sizes(cfg: synth.Config):
    """(agent counts per partition, boxes [P, 6]): the partition sizes and boxes
    World draws first from its seeded numpy generator."""
    rng = np.random.Generator(np.random.PCG64(cfg.seed))
    gx, gy, gz = cfg.grid
    P = gx * gy * gz
    if cfg.sigma > 0:
        z = rng.standard_normal(P)
        counts = np.rint(cfg.median * np.exp(cfg.sigma * z)).astype(np.int64)
    else:
        counts = np.full(P, int(round(cfg.median)), dtype=np.int64)
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
    return counts, boxes
