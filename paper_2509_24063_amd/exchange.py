"""Exchange iterations of one GPU's partitions with fixed device buffers.

A Pipeline owns everything an iteration writes -- selection, messages,
encodings -- and two copies of each side's reference state (messages and
predictor history): an iteration reads the reference copy and writes its C'
into the other copy.  Sender and receiver update their reference at regular
intervals (Sec. 2.3): after every `refresh`-th iteration (t = 0, refresh,
2 refresh, ...) the copy just written becomes the reference; in between, the
same reference serves several iterations and each iteration's C' is only an
output.  refresh = 1 makes every C' the next reference.  It runs each
iteration eagerly (Context.run_iteration), or replays one of two captured HIP
graphs (one per reference copy) when the agent store lives in fixed buffers
(DeviceStore with cap).
"""
from __future__ import annotations

import numpy as np
import torch

from . import native


class Pipeline:
    def __init__(self, ctx: native.Context, ds: native.DeviceStore, w: float, ndirs: int, idx_cap: int,
                 msgs_cap: int, pred: native.Predictor | None = None, decode: bool = True, device="cuda",
                 refresh: int = 1, shared_rx: bool = False, enc_cap: int | None = None, keys: bool = True):
        """shared_rx: the receiver, on the same GPU, decodes against the
        sender's reference and predictor history (byte-identical to its own
        copies) and writes its C' over the sender's message buffer, which the
        encoder has consumed by then: two message buffers and two histories
        less, for populations that would not fit otherwise (refresh 1 only).
        enc_cap: capacity of the encoding buffer (default: the worst-case
        bound).  keys: keep the record keys (uid and header word per record)
        of every message set beside it, so that the delta calls read them
        instead of the records."""
        if refresh < 1:
            raise ValueError("refresh interval must be >= 1")
        if shared_rx and (refresh != 1 or not decode):
            raise ValueError("a shared receiver needs refresh 1 and decoding")
        self.ctx, self.ds, self.w, self.ndirs, self.pred = ctx, ds, w, ndirs, pred
        self.refresh = refresh
        self.shared_rx = shared_rx
        self.nseg = nseg = ds.P * ndirs
        self.idx_cap, self.msgs_cap = idx_cap, msgs_cap
        self.enc_cap = int(native.lib().ta_delta_bound(nseg, msgs_cap, msgs_cap)) if enc_cap is None else enc_cap
        z8 = lambda n: torch.zeros(max(n, 8), dtype=torch.uint8, device=device)  # noqa: E731
        zo = lambda: torch.zeros(nseg + 1, dtype=torch.int64, device=device)  # noqa: E731
        self.idx = torch.zeros(max(idx_cap, 1), dtype=torch.int32, device=device)
        self.seg_off = zo()
        self.msgs, self.msg_off = z8(msgs_cap), zo()
        self.enc, self.enc_off = z8(self.enc_cap), zo()
        self.modes = torch.zeros(max(nseg, 1), dtype=torch.uint8, device=device)
        self.ref = [z8(msgs_cap), z8(msgs_cap)]
        self.ref_off = [zo(), zo()]
        # predictor history (learned mode only), per reference slot of each side
        hc = idx_cap if pred is not None else 0
        self.hist = [native.History(hc, device), native.History(hc, device)]
        zk = lambda: torch.zeros(2 * max(idx_cap, 1), dtype=torch.int64, device=device) if keys else None  # noqa
        self.msg_keys = zk()
        self.ref_keys = [zk(), zk()]
        if shared_rx:
            self.rx = [self.msgs, self.msgs]
            self.rx_off = [zo()] * 2
            self.rx_hist = [native.History(hc, device)] * 2
            self.rx_keys = [self.msg_keys] * 2
        else:
            self.rx = [z8(msgs_cap), z8(msgs_cap)] if decode else None
            self.rx_off = [zo(), zo()] if decode else None
            self.rx_hist = [native.History(hc, device), native.History(hc, device)] if decode else None
            self.rx_keys = [zk(), zk()] if decode else [None, None]
        self.decode = decode
        self.reset()
        self.graphs = [None, None]

    def reset(self):
        """Back to the first iteration: empty references, no history."""
        empty, off = native.empty_messages(self.nseg, self.ref[0].device)
        for bufs, offs in ((self.ref, self.ref_off), (None if self.shared_rx else self.rx, self.rx_off)):
            if bufs is None:
                continue
            bufs[0][:empty.numel()].copy_(empty)
            offs[0].copy_(off)
        for hs in (self.hist, self.rx_hist):
            if hs is not None:
                for h in hs:
                    h.hlen.zero_()
        self.t = 0
        self.r = 0  # the reference copy
        self.last = 1  # the copy the last iteration wrote

    def iteration(self, parity: int, ds: native.DeviceStore | None = None) -> native.Iteration:
        p, q = parity, 1 - parity
        ds = self.ds if ds is None else ds
        pred = self.pred
        keys = None
        if self.msg_keys is not None:
            keys = dict(msg=self.msg_keys, ref=self.ref_keys[p], newref=self.ref_keys[q])
            if self.decode:
                keys.update(rx_ref=self.ref_keys[p] if self.shared_rx else self.rx_keys[p], rx_out=self.rx_keys[q])
        if self.shared_rx:
            rx = dict(rx_ref=self.ref[p], rx_ref_off=self.ref_off[p], rx_out=self.rx[q], rx_out_off=self.rx_off[q],
                      rx_hist=self.hist[p] if pred else None, rx_hist_out=self.rx_hist[q] if pred else None)
        else:
            rx = dict(rx_ref=self.rx[p], rx_ref_off=self.rx_off[p], rx_out=self.rx[q], rx_out_off=self.rx_off[q],
                      rx_hist=self.rx_hist[p] if pred else None,
                      rx_hist_out=self.rx_hist[q] if pred else None) if self.decode else {}
        return native.Iteration(ds, self.w, self.ndirs, self.idx, self.seg_off, self.msgs, self.msg_off,
                                self.ref[p], self.ref_off[p], self.enc, self.enc_off, self.ref[q], self.ref_off[q],
                                self.modes, pred=pred, hist=self.hist[p] if pred else None,
                                hist_out=self.hist[q] if pred else None, keys=keys, **rx)

    def capture(self, stream=None):
        """Capture the two parities' iterations as graphs (store: self.ds)."""
        for p in (0, 1):
            if self.graphs[p] is None:
                self.graphs[p] = native.Graph(self.ctx, self.iteration(p), stream)

    def step(self, ds: native.DeviceStore | None = None, graph: bool = False):
        """Run one iteration on `ds` (default: the pipeline's store)."""
        p = self.r
        if graph:
            if ds is not None and ds is not self.ds:
                raise ValueError("graphs are bound to the pipeline's store")
            self.capture()
            self.graphs[p].launch()
        else:
            self.ctx.run_iteration(self.iteration(p, ds))
        self.last = 1 - p
        if self.t % self.refresh == 0:
            self.r = 1 - p
        self.t += 1

    def ran(self, n: int):
        """Bookkeeping after n iterations run outside step() (each one the
        iteration of its parity, t = 0 .. n-1, refresh interval 1)."""
        if self.refresh != 1:
            raise ValueError("iterations run outside step() assume refresh interval 1")
        self.t = n
        self.r = n % 2
        self.last = 1 - (n - 1) % 2

    # -- results of the last iteration -------------------------------------------
    def outputs(self):
        """(enc, enc_off, newref, newref_off, rx_out, rx_out_off) of the last iteration
        (newref: its C', the next reference only after a refresh iteration)."""
        q = self.last
        rx = (self.rx[q], self.rx_off[q]) if self.decode else (None, None)
        return (self.enc, self.enc_off, self.ref[q], self.ref_off[q]) + rx

    def close(self):
        for g in self.graphs:
            if g is not None:
                g.close()
        self.graphs = [None, None]


def capacities(ctx: native.Context, store, ndirs: int, w: float, slack: float = 1.25):
    """(idx_cap, msgs_cap) for a population like `store`, with slack for growth:
    the selection counted once on the device, and the TAM1 bound for it."""
    ds = native.DeviceStore(store)
    idx, seg = ctx.select_aura(ds, w, ndirs)
    ctx.check("capacity probe")
    nrec = int(seg[-1].item())
    idx_cap = int(nrec * slack) + 1024
    msgs_cap = ctx.serialize_bound(ds, store.P * ndirs, idx_cap)
    del ds, idx, seg
    return idx_cap, int(msgs_cap)


def sized_pipeline(ctx: native.Context, ds: native.DeviceStore, ndirs: int, w: float, growth: float,
                   pred: native.Predictor | None = None, slack: float = 1.03):
    """A shared-receiver Pipeline for a large population in a fixed-capacity
    store, its buffers sized from the present state's selection and message
    bytes (measured on the device: the serialization is sized without being
    written) times `growth`, the population's growth until the last
    iteration."""
    nseg = ds.P * ndirs
    dev = ds.uid.device
    idx = torch.empty(int(0.8 * ds.live) + 4096, dtype=torch.int32, device=dev)
    seg = torch.empty(nseg + 1, dtype=torch.int64, device=dev)
    ctx.select_aura(ds, w, ndirs, idx_cap=idx.numel(), out=(idx, seg))
    ctx.check("selection for sizing")
    records = int(seg[-1].item())
    tiny = torch.empty(8, dtype=torch.uint8, device=dev)
    moff = torch.empty(nseg + 1, dtype=torch.int64, device=dev)
    st = native.lib().ta_serialize(ctx.h, native.C.byref(ds.agents()), native._p(idx), native._p(seg), nseg,
                                   idx.numel(), native._p(tiny), 0, native._p(moff), None, 0, native._stream())
    if st or ctx.poll() not in (native.OK, native.CAPACITY):
        raise native.TAError(st or native.INVALID, "serialization for sizing")
    msg_bytes = int(moff[-1].item())
    del idx, seg, tiny, moff
    idx_cap = int(records * growth * slack) + 4096
    msgs_cap = (int(msg_bytes * growth * slack) + 64 * nseg) // 8 * 8
    enc_cap = (int(msgs_cap * 1.08) + 64 * nseg) // 8 * 8
    ctx.reserve(ds.n, nseg, idx_cap, msgs_cap)
    pl = Pipeline(ctx, ds, w, ndirs, idx_cap, msgs_cap, pred=pred, shared_rx=True, enc_cap=enc_cap)
    pl.sizing = dict(records=records, msg_bytes=msg_bytes, idx_cap=idx_cap, msgs_cap=msgs_cap, enc_cap=enc_cap)
    return pl


def segment_bytes(buf, off, s0: int, s1: int):
    """Host bytes of segments [s0, s1) of dense messages or encodings, and
    their offsets from the first one's start."""
    o = off[s0:s1 + 1].cpu().numpy()
    return buf[int(o[0]):int(o[-1])].cpu().numpy(), o - o[0]


def split_host(t, off):
    """Host bytes of dense messages/encodings: (buffer up to off[-1], offsets)."""
    o = off.cpu().numpy()
    return t[: int(o[-1])].cpu().numpy(), o


class OverlapPipeline:
    """One GPU's exchange as a three-stage pipeline on three streams, each
    stage with its own context (its own scratch memory): selection and
    serialization of iteration t + 1, encoding of t and decoding of t - 1
    run at the same time.  In a deployment the receiver works on other
    neighbours' messages and never waits for the sender; here it decodes the
    sender's own encodings, which only adds the wait for them.

    Messages and encodings are double-buffered (iteration t uses copy t % 2).
    Each hand-off records an event on the producing stream that the consumer
    waits for, and a producer waits for the consumer's event of t - 2 before
    it writes the same copy again.  References ping-pong on each side as in
    Pipeline (refresh interval 1).  Every stream has the default priority.

    The agent store is the caller's: step() orders the serialization after
    the work already enqueued on the caller's current stream (e.g. a
    DeviceStore.load() of this state), and returns with that stream ordered
    after the serialization, so the caller may load the next state into the
    same buffers right away.  The store's memory is marked as used by the
    serialization stream, so freeing the store early is safe too."""

    def __init__(self, schema, ds: native.DeviceStore, w: float, ndirs: int, idx_cap: int, msgs_cap: int,
                 device="cuda", keys: bool = True):
        self.ser, self.tx, self.rxc = native.Context(schema), native.Context(schema), native.Context(schema)
        self.s_ser, self.s_enc, self.s_dec = (torch.cuda.Stream(device=device) for _ in range(3))
        self.w, self.ndirs, self.ds = w, ndirs, ds
        self.nseg = nseg = ds.P * ndirs
        self.idx_cap, self.msgs_cap = idx_cap, msgs_cap
        self.enc_cap = int(native.lib().ta_delta_bound(nseg, msgs_cap, msgs_cap))
        z8 = lambda n: torch.zeros(max(n, 8), dtype=torch.uint8, device=device)  # noqa: E731
        zo = lambda: torch.zeros(nseg + 1, dtype=torch.int64, device=device)  # noqa: E731
        self.idx = [torch.zeros(max(idx_cap, 1), dtype=torch.int32, device=device) for _ in range(2)]
        self.seg_off = [zo(), zo()]
        self.msgs, self.msg_off = [z8(msgs_cap), z8(msgs_cap)], [zo(), zo()]
        self.modes = torch.zeros(max(nseg, 1), dtype=torch.uint8, device=device)
        self.enc, self.enc_off = [z8(self.enc_cap), z8(self.enc_cap)], [zo(), zo()]
        self.ref, self.ref_off = [z8(msgs_cap), z8(msgs_cap)], [zo(), zo()]
        self.rx, self.rx_off = [z8(msgs_cap), z8(msgs_cap)], [zo(), zo()]
        zk = lambda: torch.zeros(2 * max(idx_cap, 1), dtype=torch.int64, device=device) if keys else None  # noqa
        self.msg_keys, self.ref_keys, self.rx_keys = [zk(), zk()], [zk(), zk()], [zk(), zk()]
        self.ev_ser = [torch.cuda.Event(), torch.cuda.Event()]  # messages t % 2 written
        self.ev_enc = [torch.cuda.Event(), torch.cuda.Event()]  # messages read, encoding t % 2 written
        self.ev_dec = [torch.cuda.Event(), torch.cuda.Event()]  # encoding t % 2 read
        self.device = device
        self.reset()

    def reset(self):
        """Back to the first iteration (empty references on both sides), once
        every stage's earlier work has ended."""
        self.join()
        torch.cuda.synchronize()
        empty, off = native.empty_messages(self.nseg, self.device)
        for bufs, offs in ((self.ref, self.ref_off), (self.rx, self.rx_off)):
            bufs[0][:empty.numel()].copy_(empty)
            offs[0].copy_(off)
        torch.cuda.synchronize()
        self.t = 0

    def tune_streams(self, states, trials: int = 6, steps: int = 6) -> float:
        """Choose the stages' streams by timing.  Streams share the device's
        few hardware queues, and which stream lands on which queue is not
        exposed; some assignments let the stages overlap and others hold them
        back (up to 0.2 ms per step on the 1e7-agent exchange).  Each trial
        gives the three stages three consecutive streams of a fresh pool and
        times `steps` iterations over `states` (after two warm-up ones); the
        fastest trial's streams are kept, and the pipeline starts over at the
        first iteration.  Returns the chosen trial's seconds per step."""
        import time
        pool = [torch.cuda.Stream(device=self.device) for _ in range(trials + 2)]
        n = len(states)
        best, best_s = None, float("inf")
        for i in range(trials):
            self.s_ser, self.s_enc, self.s_dec = pool[i], pool[i + 1], pool[i + 2]
            self.reset()
            for k in range(2):
                self.step(states[k % n])
            self.join()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(2, 2 + steps):
                self.step(states[k % n])
            self.join()
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / steps
            if el < best_s:
                best, best_s = i, el
        self.check("stream tuning")
        self.s_ser, self.s_enc, self.s_dec = pool[best], pool[best + 1], pool[best + 2]
        self.reset()
        return best_s

    @property
    def streams(self):
        return (self.s_ser, self.s_enc, self.s_dec)

    def reserve(self, max_agents: int):
        for c in (self.ser, self.tx, self.rxc):
            c.reserve(max_agents, self.nseg, self.idx_cap, self.msgs_cap)

    def step(self, ds: native.DeviceStore | None = None):
        ds = self.ds if ds is None else ds
        t = self.t
        m = t % 2  # messages and encoding copy
        p, q = t % 2, 1 - t % 2  # reference copies read and written
        caller = torch.cuda.current_stream()
        with torch.cuda.stream(self.s_ser):
            self.s_ser.wait_stream(caller)  # the store as the caller wrote it
            if t >= 2:
                self.s_ser.wait_event(self.ev_enc[m])
            self.ser.select_aura(ds, self.w, self.ndirs, idx_cap=self.idx_cap, out=(self.idx[m], self.seg_off[m]))
            self.ser.serialize(ds, self.idx[m], self.seg_off[m], idx_cap=self.idx_cap,
                               out=(self.msgs[m], self.msg_off[m]), keys=self.msg_keys[m])
            self.ev_ser[m].record(self.s_ser)
            for x in ds.tensors():
                x.record_stream(self.s_ser)
        caller.wait_event(self.ev_ser[m])  # the store is free again after this point
        with torch.cuda.stream(self.s_enc):
            self.s_enc.wait_event(self.ev_ser[m])
            if t >= 2:
                self.s_enc.wait_event(self.ev_dec[m])
            self.tx.delta_encode(self.msgs[m], self.msg_off[m], self.ref[p], self.ref_off[p],
                                 out=(self.enc[m], self.enc_off[m], self.ref[q], self.ref_off[q], self.modes),
                                 keys=(self.msg_keys[m], self.ref_keys[p], self.ref_keys[q])
                                 if self.msg_keys[m] is not None else None)
            self.ev_enc[m].record(self.s_enc)
        with torch.cuda.stream(self.s_dec):
            self.s_dec.wait_event(self.ev_enc[m])
            self.rxc.delta_decode(self.enc[m], self.enc_off[m], self.rx[p], self.rx_off[p],
                                  out=(self.rx[q], self.rx_off[q]),
                                  keys=(self.rx_keys[p], self.rx_keys[q]) if self.rx_keys[p] is not None else None)
            self.ev_dec[m].record(self.s_dec)
        self.t += 1

    def join(self):
        """Make the current stream wait for every stage."""
        cur = torch.cuda.current_stream()
        for st in self.streams:
            cur.wait_stream(st)

    def check(self, what="pipelined exchange"):
        self.join()
        for c, side in ((self.ser, "select/serialize"), (self.tx, "encode"), (self.rxc, "decode")):
            c.check(f"{what} ({side})")

    def outputs(self):
        """(enc, enc_off, newref, newref_off, rx_out, rx_out_off) of the last iteration."""
        e, q = (self.t - 1) % 2, self.t % 2
        return self.enc[e], self.enc_off[e], self.ref[q], self.ref_off[q], self.rx[q], self.rx_off[q]

    def close(self):
        self.join()
        torch.cuda.synchronize()
        for c in (self.ser, self.tx, self.rxc):
            c.close()
