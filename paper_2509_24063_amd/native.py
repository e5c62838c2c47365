"""ctypes binding of libteraagent.so.

Argument marshalling only: torch CUDA tensors provide device memory and the
current stream; every step of the exchange runs in the library's HIP kernels.
The library must be built (``__graft_entry__.build()``); nothing here falls
back to another implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# TERAAGENT_LIB: load another build of the library (e.g. one with other
# compile-time launch shapes)
LIB = os.environ.get("TERAAGENT_LIB") or os.path.join(HERE, "lib", "libteraagent.so")

OK, INVALID, CAPACITY, CORRUPT, REF_MISMATCH, HIP = 0, 1, 2, 3, 4, 5
NAMES = {0: "ok", 1: "invalid", 2: "capacity", 3: "corrupt", 4: "ref_mismatch", 5: "hip"}


class TAError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__(f"{what}: {NAMES.get(code, code)}")
        self.code = code


class Agents(C.Structure):
    _fields_ = [("n", C.c_int64), ("uid", C.c_void_p), ("cls", C.c_void_p), ("nb", C.c_void_p),
                ("f64", C.c_void_p), ("f64_stride", C.c_int64), ("i32", C.c_void_p), ("i32_stride", C.c_int64),
                ("beh_off", C.c_void_p), ("beh", C.c_void_p)]


class StoreT(C.Structure):
    _fields_ = [("cap", C.c_int64), ("uid", C.c_void_p), ("cls", C.c_void_p), ("nb", C.c_void_p),
                ("f64", C.c_void_p), ("f64_stride", C.c_int64), ("i32", C.c_void_p), ("i32_stride", C.c_int64),
                ("beh_off", C.c_void_p), ("beh", C.c_void_p), ("beh_cap", C.c_int64)]


class ViewT(C.Structure):
    _fields_ = [("n", C.c_int64), ("rec_words", C.c_int64), ("off", C.c_void_p), ("records", C.c_void_p)]


class KeysT(C.Structure):
    _fields_ = [("cur", C.c_void_p), ("ref", C.c_void_p), ("out", C.c_void_p), ("out_cap", C.c_int64)]


class HistT(C.Structure):
    _fields_ = [("h1", C.c_void_p), ("h2", C.c_void_p), ("hlen", C.c_void_p), ("cap", C.c_int64)]


class IterationT(C.Structure):
    _fields_ = [("agents", C.c_void_p), ("P", C.c_int32), ("ndirs", C.c_int32), ("part_off", C.c_void_p),
                ("boxes", C.c_void_p), ("w", C.c_double), ("idx", C.c_void_p), ("idx_cap", C.c_int64),
                ("seg_off", C.c_void_p), ("msgs", C.c_void_p), ("msgs_cap", C.c_int64), ("msg_off", C.c_void_p),
                ("pred", C.c_void_p), ("ref", C.c_void_p), ("ref_len", C.c_int64), ("ref_off", C.c_void_p),
                ("hist_in", C.c_void_p), ("hist_out", C.c_void_p), ("enc", C.c_void_p), ("enc_cap", C.c_int64),
                ("enc_off", C.c_void_p), ("newref", C.c_void_p), ("newref_cap", C.c_int64),
                ("newref_off", C.c_void_p), ("modes", C.c_void_p), ("rx_ref", C.c_void_p),
                ("rx_ref_len", C.c_int64), ("rx_ref_off", C.c_void_p), ("rx_hist_in", C.c_void_p),
                ("rx_hist_out", C.c_void_p), ("rx_out", C.c_void_p), ("rx_out_cap", C.c_int64),
                ("rx_out_off", C.c_void_p), ("msg_keys", C.c_void_p), ("ref_keys", C.c_void_p),
                ("newref_keys", C.c_void_p), ("rx_ref_keys", C.c_void_p), ("rx_out_keys", C.c_void_p),
                ("keys_cap", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB)
        vp, i64, i32, st = C.c_void_p, C.c_int64, C.c_int32, C.c_int
        L.ta_create.argtypes = [C.POINTER(vp), C.c_uint32, vp, vp]
        L.ta_destroy.argtypes = [vp]
        L.ta_reserve.argtypes = [vp, i64, i64, i64, i64]
        L.ta_status_poll.argtypes = [vp, vp]
        L.ta_select_aura.argtypes = [vp, C.POINTER(Agents), i32, vp, vp, C.c_double, i32, vp, i64, vp, vp]
        L.ta_select_aura_static.argtypes = [vp, C.POINTER(Agents), i32, vp, vp, C.c_double, i32, vp, i64, vp, vp]
        L.ta_select_migrants.argtypes = [vp, C.POINTER(Agents), i32, vp, vp, vp, i64, vp, vp]
        L.ta_migrate_apply.argtypes = [vp, C.POINTER(Agents), i32, vp, vp, vp, i64, vp, i64, vp, C.POINTER(StoreT),
                                       vp, vp, vp]
        L.ta_view_grow.argtypes = [vp, vp, i64, vp, i64, vp, vp, vp, i64, vp, vp]
        L.ta_view_compact.argtypes = [vp, vp, i64, vp, i64, vp, i64, vp, vp]
        L.ta_serialize.argtypes = [vp, C.POINTER(Agents), vp, vp, i64, i64, vp, i64, vp, vp, i64, vp]
        L.ta_serialize_bound.argtypes = [i64, i64, i64]
        L.ta_serialize_bound.restype = i64
        L.ta_view.argtypes = [vp, i64, vp, C.POINTER(ViewT), vp]
        L.ta_view_validate.argtypes = [vp, vp, vp, i64, i64, vp]
        L.ta_predictor_load.argtypes = [vp, vp, C.c_size_t, C.POINTER(vp)]
        L.ta_predictor_free.argtypes = [vp]
        L.ta_predictor_free.restype = None
        L.ta_delta_encode.argtypes = [vp, i64, vp, i64, vp, vp, i64, vp, vp, C.POINTER(HistT), C.POINTER(HistT),
                                      vp, i64, vp, vp, i64, vp, vp, C.POINTER(KeysT), vp]
        L.ta_delta_bound.argtypes = [i64, i64, i64]
        L.ta_delta_bound.restype = i64
        L.ta_delta_decode.argtypes = [vp, i64, vp, i64, vp, vp, i64, vp, vp, C.POINTER(HistT), C.POINTER(HistT),
                                      vp, i64, vp, C.POINTER(KeysT), vp]
        L.ta_predictor_eval.argtypes = [vp, vp, vp, vp, i64, vp]
        L.ta_time_kernel.argtypes = [vp, C.c_char_p]
        L.ta_kernel_time.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.ta_kernel_time_of.argtypes = [vp, C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.ta_set_window_tap.argtypes = [vp, vp, vp, i64, vp]
        L.ta_trainer_create.argtypes = [vp, vp, C.c_uint32, C.c_uint32, C.c_uint32, C.c_double, C.POINTER(vp)]
        L.ta_trainer_free.argtypes = [vp]
        L.ta_trainer_free.restype = None
        L.ta_trainer_grad.argtypes = [vp, vp, vp, vp, i64, vp, vp]
        L.ta_trainer_step.argtypes = [vp, vp, vp, vp, i64, C.c_float, C.c_float, C.c_float, C.c_float, vp]
        L.ta_trainer_params.argtypes = [vp, vp]
        L.ta_trainer_export.argtypes = [vp, vp, C.c_size_t]
        L.ta_iteration_run.argtypes = [vp, C.POINTER(IterationT), vp]
        L.ta_graph_capture.argtypes = [vp, C.POINTER(IterationT), vp, C.POINTER(vp)]
        L.ta_graph_launch.argtypes = [vp, vp]
        L.ta_graph_free.argtypes = [vp]
        L.ta_graph_free.restype = None
        L.ta_get_grids.argtypes = [vp, vp]
        L.ta_set_grids.argtypes = [vp, vp]
        L.ta_set_difference_op.argtypes = [vp, C.c_int32]
        L.ta_tune.argtypes = [vp, C.POINTER(IterationT), C.c_char_p, i32, vp, C.POINTER(C.c_int32)]
        for f in ("ta_iteration_run", "ta_graph_capture", "ta_graph_launch", "ta_get_grids", "ta_set_grids",
                  "ta_tune", "ta_set_difference_op"):
            getattr(L, f).restype = st
        for f in ("ta_create", "ta_destroy", "ta_reserve", "ta_status_poll", "ta_select_aura", "ta_select_aura_static",
                  "ta_serialize", "ta_view",
                  "ta_view_validate", "ta_predictor_load", "ta_predictor_eval", "ta_delta_encode", "ta_delta_decode",
                  "ta_time_kernel", "ta_kernel_time", "ta_kernel_time_of", "ta_set_window_tap", "ta_trainer_create", "ta_trainer_grad",
                  "ta_trainer_step", "ta_trainer_params", "ta_trainer_export"):
            getattr(L, f).restype = st
        _lib = L
    return _lib


def _p(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr()) if t.numel() else None


def _keys(cur, ref, out):
    return KeysT(_p(cur), _p(ref), _p(out), out.numel() // 2 if out is not None else 0)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(code, what):
    if code:
        raise TAError(code, what)


class DeviceStore:
    """An agent store (see synth.Store) copied to device tensors.

    With `cap` (agents) and `beh_cap` (bytes) the buffers are allocated
    larger than the store, and load() copies later states of a population
    into the same memory: the library then sees n = cap agents, of which
    the partition table's part_off[P] are live (graphs stay valid)."""

    def __init__(self, store, device="cuda", cap: int | None = None, beh_cap: int | None = None):
        self.fixed = cap is not None
        cap = store.n if cap is None else cap
        bytes_ = store.beh.size if beh_cap is None else beh_cap
        if cap < store.n or bytes_ < store.beh.size:
            raise ValueError("store larger than the buffers")
        F, I = store.f64.shape[0], store.i32.shape[0]
        self.n = cap
        self.P = store.P
        self.uid = torch.zeros(max(cap, 1), dtype=torch.int64, device=device)
        self.cls = torch.zeros(max(cap, 1), dtype=torch.int16, device=device)
        self.nb = torch.zeros(max(cap, 1), dtype=torch.int16, device=device)
        self.f64 = torch.zeros((F, max(cap, 1)), dtype=torch.float64, device=device)
        self.i32 = torch.zeros((I, max(cap, 1)), dtype=torch.int32, device=device)
        self.beh_off = torch.zeros(cap + 1, dtype=torch.int64, device=device)
        self.beh = torch.zeros(max(bytes_, 8), dtype=torch.uint8, device=device)
        self.part_off = torch.zeros(store.P + 1, dtype=torch.int64, device=device)
        self.boxes = torch.from_numpy(np.ascontiguousarray(store.boxes, np.float64).reshape(-1)).to(device)
        self.max_beh_words = 0
        self.load(store)
        self._s = Agents(self.n, _p(self.uid), _p(self.cls), _p(self.nb), _p(self.f64), self.f64.shape[1],
                         _p(self.i32), self.i32.shape[1], _p(self.beh_off), _p(self.beh))

    def load(self, store):
        """Copy a state of the population (same partitions, n <= cap) in."""
        n = store.n
        if n > self.n or store.beh.size > self.beh.numel() or store.P != self.P:
            raise ValueError("state does not fit the buffers")

        def up(dst, a, dt):
            if a.size:
                dst.copy_(torch.from_numpy(np.ascontiguousarray(a).view(dt)))
        up(self.uid[:n], store.uid, np.int64)
        up(self.cls[:n], store.cls, np.int16)
        up(self.nb[:n], store.nb, np.int16)
        up(self.f64[:, :n], store.f64, np.float64)
        up(self.i32[:, :n], store.i32, np.int32)
        up(self.beh_off[:n + 1], store.beh_off, np.int64)
        if n < self.n:  # behaviour offsets of the dead tail: empty ranges
            self.beh_off[n + 1:] = int(store.beh_off[-1])
        up(self.beh[:store.beh.size], store.beh, np.uint8)
        up(self.part_off, store.part_off, np.int64)
        bw = np.diff(store.beh_off) // 8
        self.max_beh_words = max(self.max_beh_words, int(bw.max()) if bw.size else 0)
        self.live = n

    def agents(self):
        return self._s

    def tensors(self):
        """Every device tensor of the store (for stream bookkeeping)."""
        return (self.uid, self.cls, self.nb, self.f64, self.i32, self.beh_off, self.beh, self.part_off, self.boxes)

    @classmethod
    def alloc(cls, F: int, I: int, boxes, cap: int, beh_cap: int, device="cuda"):
        """An empty store (no live agents) with room for cap agents and beh_cap
        behaviour bytes, for ta_migrate_apply to write into."""
        boxes = np.ascontiguousarray(boxes, np.float64).reshape(-1, 6)
        P = boxes.shape[0]
        ds = cls.__new__(cls)
        ds.fixed = True
        ds.n, ds.P = cap, P
        ds.uid = torch.zeros(max(cap, 1), dtype=torch.int64, device=device)
        ds.cls = torch.zeros(max(cap, 1), dtype=torch.int16, device=device)
        ds.nb = torch.zeros(max(cap, 1), dtype=torch.int16, device=device)
        ds.f64 = torch.zeros((F, max(cap, 1)), dtype=torch.float64, device=device)
        ds.i32 = torch.zeros((I, max(cap, 1)), dtype=torch.int32, device=device)
        ds.beh_off = torch.zeros(cap + 1, dtype=torch.int64, device=device)
        ds.beh = torch.zeros(max(beh_cap, 8), dtype=torch.uint8, device=device)
        ds.beh_cap = beh_cap
        ds.part_off = torch.zeros(P + 1, dtype=torch.int64, device=device)
        ds.boxes = torch.from_numpy(boxes.reshape(-1).copy()).to(device)
        ds.max_beh_words = 0
        ds.live = 0
        ds._s = Agents(ds.n, _p(ds.uid), _p(ds.cls), _p(ds.nb), _p(ds.f64), ds.f64.shape[1], _p(ds.i32),
                       ds.i32.shape[1], _p(ds.beh_off), _p(ds.beh))
        return ds

    def store_struct(self):
        """The buffers as a ta_store (for calls that write a store)."""
        return StoreT(self.n, _p(self.uid), _p(self.cls), _p(self.nb), _p(self.f64), self.f64.shape[1],
                      _p(self.i32), self.i32.shape[1], _p(self.beh_off), _p(self.beh),
                      getattr(self, "beh_cap", self.beh.numel()))

    def numpy(self):
        """The live agents (part_off[P] of them) back on the host, as a synth.Store."""
        from . import synth
        po = self.part_off.cpu().numpy()
        n = int(po[-1])
        bo = self.beh_off[:n + 1].cpu().numpy()
        return synth.Store(uid=self.uid[:n].cpu().numpy().view(np.uint64), cls=self.cls[:n].cpu().numpy().view(np.uint16),
                           nb=self.nb[:n].cpu().numpy().view(np.uint16), f64=self.f64[:, :n].cpu().numpy(),
                           i32=self.i32[:, :n].cpu().numpy(), beh_off=bo,
                           beh=self.beh[:int(bo[-1]) if n else 0].cpu().numpy(), part_off=po,
                           boxes=self.boxes.cpu().numpy().reshape(-1, 6))


class History:
    """Predictor history on the device: h1, h2 int64[n,4] (fp64 bits), hlen uint8[n]."""

    def __init__(self, n, device="cuda"):
        self.h1 = torch.zeros((max(n, 1), 4), dtype=torch.int64, device=device)
        self.h2 = torch.zeros((max(n, 1), 4), dtype=torch.int64, device=device)
        self.hlen = torch.zeros(max(n, 1), dtype=torch.uint8, device=device)
        self.n = n

    def struct(self):
        return HistT(_p(self.h1), _p(self.h2), _p(self.hlen), self.n)

    @staticmethod
    def from_numpy(h1, h2, hlen, device="cuda"):
        n = int(hlen.shape[0])
        h = History(n, device)
        if n:
            h.h1[:n] = torch.from_numpy(np.ascontiguousarray(h1).view(np.int64)).to(device)
            h.h2[:n] = torch.from_numpy(np.ascontiguousarray(h2).view(np.int64)).to(device)
            h.hlen[:n] = torch.from_numpy(np.ascontiguousarray(hlen)).to(device)
        return h

    def numpy(self, n=None):
        n = self.n if n is None else n
        return (self.h1[:n].cpu().numpy().view(np.uint64), self.h2[:n].cpu().numpy().view(np.uint64),
                self.hlen[:n].cpu().numpy())


class Predictor:
    def __init__(self, ctx, blob: bytes):
        b = (C.c_uint8 * len(blob)).from_buffer_copy(blob)
        h = C.c_void_p()
        _check(lib().ta_predictor_load(ctx.h, b, len(blob), C.byref(h)), "ta_predictor_load")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ta_predictor_free(self.h)
            self.h = None


class Context:
    def __init__(self, schema):
        nf = (C.c_uint16 * len(schema.n_f64))(*schema.n_f64)
        ni = (C.c_uint16 * len(schema.n_i32))(*schema.n_i32)
        h = C.c_void_p()
        _check(lib().ta_create(C.byref(h), len(schema.n_f64), nf, ni), "ta_create")
        self.h = h
        self.max_f = max(schema.n_f64)
        self.max_i = max(schema.n_i32)

    def close(self):
        if getattr(self, "h", None):
            h, self.h = self.h, None
            _check(lib().ta_destroy(h), "ta_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, max_agents, max_segments, max_records, max_msg_bytes):
        _check(lib().ta_reserve(self.h, max_agents, max_segments, max_records, max_msg_bytes), "ta_reserve")

    def poll(self) -> int:
        return lib().ta_status_poll(self.h, _stream())

    def check(self, what="exchange"):
        _check(self.poll(), what)

    # -- the exchange --------------------------------------------------------
    def select_aura(self, ds: DeviceStore, w: float, ndirs: int, idx_cap: int | None = None, out=None):
        if idx_cap is None:
            idx_cap = max(64, 26 * ds.n)
        idx = out[0] if out is not None else torch.empty(max(idx_cap, 1), dtype=torch.int32, device=ds.uid.device)
        seg_off = out[1] if out is not None else torch.empty(ds.P * ndirs + 1, dtype=torch.int64,
                                                             device=ds.uid.device)
        _check(lib().ta_select_aura(self.h, C.byref(ds.agents()), ds.P, _p(ds.part_off), _p(ds.boxes), float(w),
                                    ndirs, _p(idx), idx_cap, _p(seg_off), _stream()), "ta_select_aura")
        return idx, seg_off

    def select_aura_static(self, ds: DeviceStore, w: float, ndirs: int, idx, seg_off):
        """ta_select_aura_static into caller-given idx (device int32) and
        seg_off (device int64[P*ndirs+1]): the selection without allocation."""
        _check(lib().ta_select_aura_static(self.h, C.byref(ds.agents()), ds.P, _p(ds.part_off), _p(ds.boxes),
                                           float(w), ndirs, _p(idx), idx.numel(), _p(seg_off), _stream()),
               "ta_select_aura_static")
        return idx, seg_off

    def select_migrants(self, ds: DeviceStore, idx_cap: int | None = None, out=None):
        if idx_cap is None:
            idx_cap = max(64, ds.n)
        idx = out[0] if out is not None else torch.empty(max(idx_cap, 1), dtype=torch.int32, device=ds.uid.device)
        seg_off = out[1] if out is not None else torch.empty(ds.P * 26 + 1, dtype=torch.int64, device=ds.uid.device)
        _check(lib().ta_select_migrants(self.h, C.byref(ds.agents()), ds.P, _p(ds.part_off), _p(ds.boxes), _p(idx),
                                        idx_cap, _p(seg_off), _stream()), "ta_select_migrants")
        return idx, seg_off

    def migrate_apply(self, ds: DeviceStore, msgs, msg_off, msg_part, out: DeviceStore, sizes=None):
        """Build out (a DeviceStore from DeviceStore.alloc) from ds and the
        migration messages; out.part_off receives the result's partitions.
        Returns the device int64[2] sizes (agents, behaviour bytes)."""
        nseg = msg_off.numel() - 1
        if sizes is None:
            sizes = torch.empty(2, dtype=torch.int64, device=ds.uid.device)
        so = out.store_struct()
        _check(lib().ta_migrate_apply(self.h, C.byref(ds.agents()), ds.P, _p(ds.part_off), _p(ds.boxes), _p(msgs),
                                      msgs.numel() if msgs is not None else 0, _p(msg_off), nseg, _p(msg_part),
                                      C.byref(so), _p(out.part_off), _p(sizes), _stream()), "ta_migrate_apply")
        return sizes

    def view_grow(self, buf, msg_off, seg, rec, words, arena_used):
        """Grow records in place (see ta_view_grow); arena_used: device int64[1]."""
        n = seg.numel()
        _check(lib().ta_view_grow(self.h, _p(buf), buf.numel(), _p(msg_off), msg_off.numel() - 1, _p(seg), _p(rec),
                                  _p(words), n, _p(arena_used), _stream()), "ta_view_grow")

    def view_compact(self, buf, msg_off, out, out_off):
        _check(lib().ta_view_compact(self.h, _p(buf), buf.numel(), _p(msg_off), msg_off.numel() - 1, _p(out),
                                     out.numel(), _p(out_off), _stream()), "ta_view_compact")

    def serialize_bound(self, ds: DeviceStore, nseg: int, idx_cap: int) -> int:
        words = 2 + self.max_f + (self.max_i + 1) // 2 + ds.max_beh_words
        return int(lib().ta_serialize_bound(nseg, idx_cap, words))

    def serialize(self, ds: DeviceStore, idx, seg_off, idx_cap: int | None = None, out_cap: int | None = None,
                  out=None, keys=None):
        """keys (optional): device int64 [>= 2 idx_cap] receiving the records' keys."""
        nseg = seg_off.numel() - 1
        if idx_cap is None:
            idx_cap = idx.numel()
        if out is None:
            if out_cap is None:
                out_cap = self.serialize_bound(ds, nseg, idx_cap)
            buf = torch.empty(max(out_cap, 8), dtype=torch.uint8, device=seg_off.device)
            msg_off = torch.empty(nseg + 1, dtype=torch.int64, device=seg_off.device)
        else:
            buf, msg_off = out
            out_cap = buf.numel()
        _check(lib().ta_serialize(self.h, C.byref(ds.agents()), _p(idx), _p(seg_off), nseg, idx_cap, _p(buf),
                                  out_cap, _p(msg_off), _p(keys), keys.numel() // 2 if keys is not None else 0,
                                  _stream()), "ta_serialize")
        return buf, msg_off

    def delta_encode(self, cur, cur_off, ref, ref_off, pred: Predictor | None = None, hist: History | None = None,
                     hist_out: History | None = None, out=None, enc_cap=None, keys=None):
        """keys (optional): (cur keys, ref keys, C' keys out), each a device
        int64 tensor or None."""
        nseg = cur_off.numel() - 1
        dev = cur.device
        if out is None:
            if enc_cap is None:
                enc_cap = int(lib().ta_delta_bound(nseg, cur.numel(), ref.numel()))
            enc = torch.empty(max(enc_cap, 8), dtype=torch.uint8, device=dev)
            enc_off = torch.empty(nseg + 1, dtype=torch.int64, device=dev)
            newref = torch.empty(max(cur.numel(), 8), dtype=torch.uint8, device=dev)
            newref_off = torch.empty(nseg + 1, dtype=torch.int64, device=dev)
            modes = torch.empty(max(nseg, 1), dtype=torch.uint8, device=dev)
        else:
            enc, enc_off, newref, newref_off, modes = out
        hs = hist.struct() if hist is not None else None
        ho = hist_out.struct() if hist_out is not None else None
        ks = _keys(*keys) if keys is not None else None
        _check(lib().ta_delta_encode(self.h, nseg, _p(cur), cur.numel(), _p(cur_off), _p(ref), ref.numel(),
                                     _p(ref_off), pred.h if pred is not None else None,
                                     C.byref(hs) if hs is not None else None, C.byref(ho) if ho is not None else None,
                                     _p(enc), enc.numel(), _p(enc_off), _p(newref), newref.numel(), _p(newref_off),
                                     _p(modes), C.byref(ks) if ks is not None else None, _stream()),
               "ta_delta_encode")
        return enc, enc_off, newref, newref_off, modes

    def delta_decode(self, enc, enc_off, ref, ref_off, pred: Predictor | None = None, hist: History | None = None,
                     hist_out: History | None = None, out=None, out_cap=None, keys=None):
        """keys (optional): (ref keys, C' keys out), each a device int64 tensor or None."""
        nseg = enc_off.numel() - 1
        dev = enc.device
        if out is None:
            if out_cap is None:
                out_cap = ref.numel() + enc.numel() + 8 * nseg + 64
            buf = torch.empty(max(out_cap, 8), dtype=torch.uint8, device=dev)
            off = torch.empty(nseg + 1, dtype=torch.int64, device=dev)
        else:
            buf, off = out
        hs = hist.struct() if hist is not None else None
        ho = hist_out.struct() if hist_out is not None else None
        ks = _keys(None, *keys) if keys is not None else None
        _check(lib().ta_delta_decode(self.h, nseg, _p(enc), enc.numel(), _p(enc_off), _p(ref), ref.numel(),
                                     _p(ref_off), pred.h if pred is not None else None,
                                     C.byref(hs) if hs is not None else None, C.byref(ho) if ho is not None else None,
                                     _p(buf), buf.numel(), _p(off), C.byref(ks) if ks is not None else None,
                                     _stream()), "ta_delta_decode")
        return buf, off

    def predictor_eval(self, pred: Predictor, inputs):
        """q = predictor(inputs) for device int32 [n,12] inputs -> int32 [n,4]."""
        inputs = inputs.contiguous()
        n = inputs.shape[0]
        q = torch.empty((max(n, 1), 4), dtype=torch.int32, device=inputs.device)
        _check(lib().ta_predictor_eval(self.h, pred.h, _p(inputs), _p(q), n, _stream()), "ta_predictor_eval")
        return q[:n]

    def view(self, buf, start: int, length: int, header: bytes | None = None):
        """ta_view of the message at buf[start:start+length]; header: its first
        32 bytes as the caller holds them (then the device is not read)."""
        v = ViewT()
        ptr = C.c_void_p(buf.data_ptr() + start)
        hb = (C.c_uint8 * 32).from_buffer_copy(header[:32]) if header is not None else None
        _check(lib().ta_view(ptr, length, hb, C.byref(v), _stream()), "ta_view")
        return v

    def validate(self, buf, off):
        nseg = off.numel() - 1
        _check(lib().ta_view_validate(self.h, _p(buf), _p(off), nseg, buf.numel(), _stream()), "ta_view_validate")

    def time_kernel(self, name: str | None):
        _check(lib().ta_time_kernel(self.h, name.encode() if name else None), "ta_time_kernel")

    def kernel_time(self, name: str | None = None):
        """(launches, total ms) of the timed launches of family `name`, or of
        every timed family."""
        n, ms = C.c_int64(0), C.c_double(0)
        if name is None:
            _check(lib().ta_kernel_time(self.h, C.byref(n), C.byref(ms)), "ta_kernel_time")
        else:
            _check(lib().ta_kernel_time_of(self.h, name.encode(), C.byref(n), C.byref(ms)), "ta_kernel_time_of")
        return n.value, ms.value


    # -- iterations, graphs, tuning ---------------------------------------------
    def run_iteration(self, it: Iteration):
        _check(lib().ta_iteration_run(self.h, C.byref(it.s), _stream()), "ta_iteration_run")

    def grids(self):
        g = (C.c_int32 * 4)()
        _check(lib().ta_get_grids(self.h, g), "ta_get_grids")
        return list(g)

    def set_difference_op(self, op: int):
        """0: XOR residuals (default); 1: byte-wise subtraction mod 256."""
        _check(lib().ta_set_difference_op(self.h, op), "ta_set_difference_op")

    def set_grids(self, grids=None):
        g = (C.c_int32 * 4)(*grids) if grids is not None else None
        _check(lib().ta_set_grids(self.h, g), "ta_set_grids")

    def tune(self, it: Iteration, cache_path: str | None = None, reps: int = 3) -> bool:
        """Tune the family grids on this iteration; True when taken from the cache."""
        fc = C.c_int32(0)
        _check(lib().ta_tune(self.h, C.byref(it.s), cache_path.encode() if cache_path else None, reps, _stream(),
                             C.byref(fc)), "ta_tune")
        return bool(fc.value)

    # -- training of the predictor ---------------------------------------------
    def set_window_tap(self, inputs=None, targets=None, count=None):
        """Collect training windows from every learned encode: inputs int32
        [cap,12], targets float32 [cap,4], count int64 [1] (zeroed by the
        caller; reads as the number of windows offered).  No arguments: off."""
        if inputs is None:
            _check(lib().ta_set_window_tap(self.h, None, None, 0, None), "ta_set_window_tap")
            self._tap = None
            return
        assert inputs.dtype == torch.int32 and targets.dtype == torch.float32 and count.dtype == torch.int64
        assert inputs.is_contiguous() and targets.is_contiguous() and inputs.shape[0] == targets.shape[0]
        self._tap = (inputs, targets, count)  # keep the buffers alive while the tap is set
        _check(lib().ta_set_window_tap(self.h, _p(inputs), _p(targets), inputs.shape[0], _p(count)),
               "ta_set_window_tap")


class Trainer:
    """Device trainer of the predictor's parameters (fp32, 5252 values)."""
    N_PARAMS = 5252

    def __init__(self, ctx: Context, init, shifts, cell: float):
        init = np.ascontiguousarray(init, np.float32)
        assert init.shape == (self.N_PARAMS,)
        h = C.c_void_p()
        r1, r2, r3 = shifts
        _check(lib().ta_trainer_create(ctx.h, init.ctypes.data_as(C.c_void_p), r1, r2, r3, float(cell), C.byref(h)),
               "ta_trainer_create")
        self.h, self.ctx = h, ctx

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ta_trainer_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def grad(self, inputs, targets):
        """(loss, gradient float32 [5252]) at the current parameters."""
        n = inputs.shape[0]
        out = torch.empty(self.N_PARAMS + 1, dtype=torch.float32, device=inputs.device)
        # contiguous copies stay referenced until the call has been enqueued (a
        # tensor freed earlier could be handed to another allocation first)
        x, y = inputs.contiguous(), targets.contiguous()
        _check(lib().ta_trainer_grad(self.ctx.h, self.h, _p(x), _p(y), n, _p(out), _stream()), "ta_trainer_grad")
        g = out.cpu().numpy()
        return float(g[-1]), g[:-1]

    def step(self, inputs, targets, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(lib().ta_trainer_step(self.ctx.h, self.h, _p(inputs), _p(targets), inputs.shape[0], lr, beta1, beta2,
                                     eps, _stream()), "ta_trainer_step")

    def params(self):
        out = np.zeros(self.N_PARAMS, np.float32)
        _check(lib().ta_trainer_params(self.h, out.ctypes.data_as(C.c_void_p)), "ta_trainer_params")
        return out

    def export(self) -> bytes:
        b = (C.c_uint8 * 5672)()
        _check(lib().ta_trainer_export(self.h, b, 5672), "ta_trainer_export")
        return bytes(b)


class Iteration:
    """One exchange iteration's arguments (select, serialize, encode and,
    with rx_out, decode), kept alive together with the tensors they point to."""

    def __init__(self, ds: DeviceStore, w: float, ndirs: int, idx, seg_off, msgs, msg_off, ref, ref_off, enc,
                 enc_off, newref, newref_off, modes, pred: Predictor | None = None, hist: History | None = None,
                 hist_out: History | None = None, rx_ref=None, rx_ref_off=None, rx_hist: History | None = None,
                 rx_hist_out: History | None = None, rx_out=None, rx_out_off=None, keys=None):
        """keys (optional): dict of record-key tensors msg, ref, newref, rx_ref,
        rx_out (any may be None), each holding `cap` records."""
        self._keep = [ds, idx, seg_off, msgs, msg_off, ref, ref_off, enc, enc_off, newref, newref_off, modes, pred,
                      hist, hist_out, rx_ref, rx_ref_off, rx_hist, rx_hist_out, rx_out, rx_out_off, keys]
        k = keys or {}
        kcap = min([t.numel() // 2 for n, t in k.items() if t is not None and n in ("msg", "newref", "rx_out")],
                   default=0)
        self._agents = ds.agents()
        hs = [h.struct() if h is not None else None for h in (hist, hist_out, rx_hist, rx_hist_out)]
        self._hs = hs
        ptr = lambda x: C.cast(C.pointer(x), C.c_void_p) if x is not None else None  # noqa: E731
        self.s = IterationT(
            ptr(self._agents), ds.P, ndirs, _p(ds.part_off), _p(ds.boxes), float(w), _p(idx), idx.numel(),
            _p(seg_off), _p(msgs), msgs.numel(), _p(msg_off), pred.h if pred is not None else None, _p(ref),
            ref.numel(), _p(ref_off), ptr(hs[0]), ptr(hs[1]), _p(enc), enc.numel(), _p(enc_off), _p(newref),
            newref.numel(), _p(newref_off), _p(modes), _p(rx_ref), rx_ref.numel() if rx_ref is not None else 0,
            _p(rx_ref_off), ptr(hs[2]), ptr(hs[3]), _p(rx_out), rx_out.numel() if rx_out is not None else 0,
            _p(rx_out_off), _p(k.get("msg")), _p(k.get("ref")), _p(k.get("newref")), _p(k.get("rx_ref")),
            _p(k.get("rx_out")), kcap)


class Graph:
    """An iteration captured as a HIP graph."""

    def __init__(self, ctx: "Context", it: Iteration, stream=None):
        self.ctx, self.it = ctx, it
        h = C.c_void_p()
        # capture needs a stream of its own (not the NULL stream); the graph
        # may be launched on any stream
        st = stream if stream is not None else torch.cuda.Stream()
        _check(lib().ta_graph_capture(ctx.h, C.byref(it.s), C.c_void_p(st.cuda_stream), C.byref(h)),
               "ta_graph_capture")
        self.h = h

    def launch(self):
        _check(lib().ta_graph_launch(self.h, _stream()), "ta_graph_launch")

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ta_graph_free(self.h)
            self.h = None

    def __del__(self):
        self.close()


def empty_messages(nseg: int, device="cuda"):
    """nseg empty TAM1 messages: the reference before the first exchange."""
    one = np.zeros(32, np.uint8)
    one[:4] = np.frombuffer(b"TAM1", np.uint8)
    one[4] = 1
    buf = torch.from_numpy(np.tile(one, max(nseg, 1))).to(device)
    off = torch.arange(nseg + 1, dtype=torch.int64, device=device) * 32
    return buf, off
