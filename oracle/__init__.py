"""Python face of the plain CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg are its only users.  It shares no code with the GPU library.
Every function works on host numpy arrays; multi-segment helpers run the
one-message C functions segment by segment and concatenate the results.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

OK, INVALID, CAPACITY, CORRUPT, REF_MISMATCH = 0, 1, 2, 3, 4


def build() -> str:
    """Compile oracle.c with gcc (no fast-math, no contraction)."""
    src = os.path.join(HERE, "oracle.c")
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fno-fast-math", "-Wall", "-o", tmp, src, "-lm"])
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        _declare(_lib)
    return _lib


class Agents(C.Structure):
    _fields_ = [("n", C.c_int64), ("uid", C.c_void_p), ("cls", C.c_void_p), ("nb", C.c_void_p),
                ("f64", C.c_void_p), ("f64_stride", C.c_int64), ("i32", C.c_void_p), ("i32_stride", C.c_int64),
                ("beh_off", C.c_void_p), ("beh", C.c_void_p)]


class OStore(C.Structure):
    _fields_ = [("cap", C.c_int64), ("uid", C.c_void_p), ("cls", C.c_void_p), ("nb", C.c_void_p),
                ("f64", C.c_void_p), ("f64_stride", C.c_int64), ("i32", C.c_void_p), ("i32_stride", C.c_int64),
                ("beh_off", C.c_void_p), ("beh", C.c_void_p), ("beh_cap", C.c_int64)]


class MLP(C.Structure):
    _fields_ = [("w1", C.c_int8 * 768), ("w2", C.c_int8 * 4096), ("w3", C.c_int8 * 256),
                ("b1", C.c_int32 * 64), ("b2", C.c_int32 * 64), ("b3", C.c_int32 * 4),
                ("r1", C.c_uint8), ("r2", C.c_uint8), ("r3", C.c_uint8), ("cell", C.c_double)]


class Hist(C.Structure):
    _fields_ = [("h1", C.c_void_p), ("h2", C.c_void_p), ("hlen", C.c_void_p)]


def _declare(L):
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int
    L.orc_select_aura.argtypes = [i64, vp, vp, i64, vp, C.c_double, i32, vp, i64, vp]
    L.orc_select_migrants.argtypes = [i64, vp, vp, i64, vp, vp, i64, vp]
    L.orc_migrate_apply.argtypes = [C.POINTER(Agents), i64, vp, vp, i32, vp, vp, i32, i32, vp, i64, vp, i64, vp,
                                    C.POINTER(OStore), vp, vp]
    L.orc_view_grow.argtypes = [vp, i64, vp, i64, vp, vp, vp, i64, C.POINTER(C.c_int64)]
    L.orc_view_compact.argtypes = [vp, i64, vp, i64, vp, i64, vp]
    L.orc_serialize.argtypes = [C.POINTER(Agents), i32, vp, vp, vp, vp, i64, vp, i64, vp]
    L.orc_view.argtypes = [vp, i64, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.orc_mlp_parse.argtypes = [vp, i64, C.POINTER(MLP)]
    L.orc_mlp_forward.argtypes = [C.POINTER(MLP), vp, vp]
    L.orc_mlp_forward.restype = None
    L.orc_delta_encode.argtypes = [vp, i64, vp, i64, C.POINTER(MLP), C.POINTER(Hist), C.POINTER(Hist), vp, i64,
                                   C.POINTER(C.c_int64), vp, i64, C.POINTER(C.c_int64), C.POINTER(C.c_int), C.c_int]
    L.orc_delta_decode.argtypes = [vp, i64, vp, i64, C.POINTER(MLP), C.POINTER(Hist), C.POINTER(Hist), vp, i64,
                                   C.POINTER(C.c_int64), C.c_int]
    L.orc_predictor_inputs.argtypes = [vp, i64, C.POINTER(Hist), C.c_double, vp, vp]


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a.size else C.c_void_p(a.ctypes.data)


# ---------------------------------------------------------------------------
def select_aura(store, w: float, ndirs: int):
    """(idx int32[S], seg_off int64[P*ndirs+1])."""
    L = lib()
    f64 = np.ascontiguousarray(store.f64)
    part_off = np.ascontiguousarray(store.part_off, dtype=np.int64)
    boxes = np.ascontiguousarray(store.boxes, dtype=np.float64)
    P = part_off.shape[0] - 1
    seg_off = np.zeros(P * ndirs + 1, dtype=np.int64)
    cap = max(1, 26 * store.n)
    idx = np.zeros(cap, dtype=np.int32)
    st = L.orc_select_aura(P, _p(part_off), _p(f64), f64.shape[1], _p(boxes), float(w), ndirs, _p(idx), cap,
                           _p(seg_off))
    if st:
        raise RuntimeError(f"orc_select_aura status {st}")
    return idx[: int(seg_off[-1])].copy(), seg_off


def select_migrants(store):
    """(idx int32[S], seg_off int64[P*26+1]): agents outside their partition box,
    by the direction they left it in."""
    L = lib()
    f64 = np.ascontiguousarray(store.f64)
    part_off = np.ascontiguousarray(store.part_off, dtype=np.int64)
    boxes = np.ascontiguousarray(store.boxes, dtype=np.float64)
    P = part_off.shape[0] - 1
    seg_off = np.zeros(P * 26 + 1, dtype=np.int64)
    cap = max(1, store.n)
    idx = np.zeros(cap, dtype=np.int32)
    st = L.orc_select_migrants(P, _p(part_off), _p(f64), f64.shape[1], _p(boxes), _p(idx), cap, _p(seg_off))
    if st:
        raise RuntimeError(f"orc_select_migrants status {st}")
    return idx[: int(seg_off[-1])].copy(), seg_off


def migrate_apply(store, schema, msgs: np.ndarray, msg_off: np.ndarray, dest: np.ndarray, nf_cols: int,
                  ni_cols: int, cap: int | None = None, beh_cap: int | None = None):
    """The store after a migration exchange: (status, out) with out a dict of
    uid, cls, nb, f64 [nf_cols, n], i32 [ni_cols, n], beh_off, beh, part_off and
    sizes (agents, behaviour bytes).  cap / beh_cap default to the sizes needed."""
    L = lib()
    a, keep = _agents(store)
    part_off = np.ascontiguousarray(store.part_off, np.int64)
    boxes = np.ascontiguousarray(store.boxes, np.float64)
    P = part_off.shape[0] - 1
    nf = np.asarray(schema.n_f64, np.uint16)
    ni = np.asarray(schema.n_i32, np.uint16)
    msgs = np.ascontiguousarray(msgs, np.uint8)
    if msgs.size == 0:
        msgs = np.zeros(8, np.uint8)
        msgs_len = 0
    else:
        msgs_len = msgs.shape[0]
    msg_off = np.ascontiguousarray(msg_off, np.int64)
    nseg = msg_off.shape[0] - 1
    dest = np.ascontiguousarray(dest, np.int32) if nseg else np.zeros(1, np.int32)
    sizes = np.zeros(2, np.int64)
    part_out = np.zeros(P + 1, np.int64)

    def run(c, bc):
        o = dict(uid=np.zeros(max(c, 1), np.uint64), cls=np.zeros(max(c, 1), np.uint16),
                 nb=np.zeros(max(c, 1), np.uint16), f64=np.zeros((max(nf_cols, 1), max(c, 1))),
                 i32=np.zeros((max(ni_cols, 1), max(c, 1)), np.int32), beh_off=np.zeros(c + 1, np.int64),
                 beh=np.zeros(max(bc, 8), np.uint8))
        st_ = OStore(c, _p(o["uid"]), _p(o["cls"]), _p(o["nb"]), _p(o["f64"]), o["f64"].shape[1], _p(o["i32"]),
                     o["i32"].shape[1], _p(o["beh_off"]), _p(o["beh"]), bc)
        r = L.orc_migrate_apply(C.byref(a), P, _p(part_off), _p(boxes), nf.shape[0], _p(nf), _p(ni), nf_cols,
                                ni_cols, _p(msgs), msgs_len, _p(msg_off), nseg, _p(dest), C.byref(st_),
                                _p(part_out), _p(sizes))
        return r, o

    st, o = run(0 if cap is None else cap, 0 if beh_cap is None else beh_cap)
    if st == CAPACITY and cap is None and beh_cap is None:
        st, o = run(int(sizes[0]), int(sizes[1]))
    del keep
    n = int(sizes[0])
    out = dict(part_off=part_out.copy(), sizes=sizes.copy())
    if st == OK:
        out.update(uid=o["uid"][:n], cls=o["cls"][:n], nb=o["nb"][:n], f64=o["f64"][:nf_cols, :n],
                   i32=o["i32"][:ni_cols, :n], beh_off=o["beh_off"][: n + 1], beh=o["beh"][: int(sizes[1])])
    return st, out


def view_grow(buf: np.ndarray, msg_off: np.ndarray, seg, rec, words, arena_used: int = 0):
    """Grow records in place (buf is modified): (status, arena_used)."""
    L = lib()
    assert buf.dtype == np.uint8 and buf.flags.c_contiguous
    msg_off = np.ascontiguousarray(msg_off, np.int64)
    seg = np.ascontiguousarray(seg, np.int32)
    rec = np.ascontiguousarray(rec, np.uint32)
    words = np.ascontiguousarray(words, np.uint32)
    n = seg.shape[0]
    pad = lambda a: a if a.size else np.zeros(1, a.dtype)  # noqa: E731
    used = C.c_int64(arena_used)
    st = L.orc_view_grow(_p(buf), buf.shape[0], _p(msg_off), msg_off.shape[0] - 1, _p(pad(seg)), _p(pad(rec)),
                         _p(pad(words)), n, C.byref(used))
    return st, int(used.value)


def view_compact(buf: np.ndarray, msg_off: np.ndarray, out_cap: int | None = None):
    """Canonical copies: (status, out bytes, out_off)."""
    L = lib()
    msg_off = np.ascontiguousarray(msg_off, np.int64)
    nseg = msg_off.shape[0] - 1
    out_off = np.zeros(nseg + 1, np.int64)
    b = np.ascontiguousarray(buf, np.uint8)
    if out_cap is None:
        st = L.orc_view_compact(_p(b), b.shape[0], _p(msg_off), nseg, None, 0, _p(out_off))
        if st not in (OK, CAPACITY):
            return st, None, out_off
        out_cap = int(out_off[-1])
    out = np.zeros(max(out_cap, 8), np.uint8)
    st = L.orc_view_compact(_p(b), b.shape[0], _p(msg_off), nseg, _p(out), out_cap, _p(out_off))
    return st, out[: int(out_off[-1])] if st == OK else None, out_off


def _agents(store):
    keep = dict(uid=np.ascontiguousarray(store.uid, np.uint64), cls=np.ascontiguousarray(store.cls, np.uint16),
                nb=np.ascontiguousarray(store.nb, np.uint16), f64=np.ascontiguousarray(store.f64, np.float64),
                i32=np.ascontiguousarray(store.i32, np.int32), beh_off=np.ascontiguousarray(store.beh_off, np.int64),
                beh=np.ascontiguousarray(store.beh, np.uint8))
    if keep["beh"].size == 0:
        keep["beh"] = np.zeros(8, np.uint8)
    a = Agents(store.n, _p(keep["uid"]), _p(keep["cls"]), _p(keep["nb"]), _p(keep["f64"]), keep["f64"].shape[1],
               _p(keep["i32"]), keep["i32"].shape[1], _p(keep["beh_off"]), _p(keep["beh"]))
    return a, keep


def serialize(store, schema, idx: np.ndarray, seg_off: np.ndarray):
    """(buffer uint8[], msg_off int64[nseg+1]) for every segment of idx/seg_off."""
    L = lib()
    a, keep = _agents(store)
    nf = np.asarray(schema.n_f64, np.uint16)
    ni = np.asarray(schema.n_i32, np.uint16)
    idx = np.ascontiguousarray(idx, np.int32)
    seg_off = np.ascontiguousarray(seg_off, np.int64)
    nseg = seg_off.shape[0] - 1
    msg_off = np.zeros(nseg + 1, np.int64)
    st = L.orc_serialize(C.byref(a), nf.shape[0], _p(nf), _p(ni), _p(idx if idx.size else np.zeros(1, np.int32)),
                         _p(seg_off), nseg, None, 0, _p(msg_off))
    cap = int(msg_off[-1])
    out = np.zeros(max(cap, 8), np.uint8)
    st = L.orc_serialize(C.byref(a), nf.shape[0], _p(nf), _p(ni), _p(idx if idx.size else np.zeros(1, np.int32)),
                         _p(seg_off), nseg, _p(out), cap, _p(msg_off))
    if st:
        raise RuntimeError(f"orc_serialize status {st}")
    del keep
    return out[:cap], msg_off


def view(msg: np.ndarray):
    """(status, n, rec_words) of one TAM1 message."""
    n, rw = C.c_int64(0), C.c_int64(0)
    m = np.ascontiguousarray(msg, np.uint8)
    st = lib().orc_view(_p(m) if m.size else None, m.size, C.byref(n), C.byref(rw))
    return st, n.value, rw.value


def mlp_struct(blob: bytes):
    m = MLP()
    b = np.frombuffer(bytes(blob), np.uint8).copy()
    st = lib().orc_mlp_parse(_p(b), b.size, C.byref(m))
    if st:
        raise ValueError(f"predictor blob rejected ({st})")
    return m


def mlp_forward(m: MLP, inp: np.ndarray) -> np.ndarray:
    inp = np.ascontiguousarray(inp, np.int32).reshape(-1, 12)
    out = np.zeros((inp.shape[0], 4), np.int32)
    L = lib()
    for r in range(inp.shape[0]):
        L.orc_mlp_forward(C.byref(m), _p(inp[r]), _p(out[r]))
    return out


class History:
    """Per-slot predictor history: h1, h2 uint64[n, 4] (fp64 bits), hlen uint8[n]."""

    def __init__(self, n: int):
        self.h1 = np.zeros((n, 4), np.uint64)
        self.h2 = np.zeros((n, 4), np.uint64)
        self.hlen = np.zeros(n, np.uint8)

    @property
    def n(self):
        return self.hlen.shape[0]

    def slice(self, a, b):
        h = History(0)
        h.h1, h.h2, h.hlen = self.h1[a:b], self.h2[a:b], self.hlen[a:b]
        return h

    def struct(self):
        for x in (self.h1, self.h2, self.hlen):
            assert x.flags.c_contiguous
        pad = np.zeros(8, np.uint64)
        self._keep = pad
        return Hist(_p(self.h1) if self.h1.size else _p(pad), _p(self.h2) if self.h2.size else _p(pad),
                    _p(self.hlen) if self.hlen.size else _p(pad))

    @staticmethod
    def concat(hs):
        h = History(0)
        h.h1 = np.concatenate([x.h1 for x in hs]) if hs else np.zeros((0, 4), np.uint64)
        h.h2 = np.concatenate([x.h2 for x in hs]) if hs else np.zeros((0, 4), np.uint64)
        h.hlen = np.concatenate([x.hlen for x in hs]) if hs else np.zeros(0, np.uint8)
        return h


def _buf(x):
    x = np.ascontiguousarray(x, np.uint8)
    return x if x.size else np.zeros(8, np.uint8), x.size


def delta_encode(cur: np.ndarray, ref: np.ndarray, mlp: MLP | None = None, hist: History | None = None,
                 want_hist: bool = False, op: int = 0):
    """Encode one message with difference operator op (0 XOR, 1 byte-wise
    subtraction mod 256).  Returns (status, enc, newref, mode, hist_out)."""
    L = lib()
    c, cl = _buf(cur)
    r, rl = _buf(ref)
    _, n_cur, _ = view(cur)
    cap = 64 + 16 * max(cl, 8) + 64
    ncap = cl + 64
    out = np.zeros(cap, np.uint8)
    nref = np.zeros(ncap, np.uint8)
    ol, nl, mode = C.c_int64(0), C.c_int64(0), C.c_int(0)
    hin = hist.struct() if hist is not None else None
    hout_obj = History(max(n_cur, 0)) if (want_hist or mlp is not None) else None
    hout = hout_obj.struct() if hout_obj is not None else None
    st = L.orc_delta_encode(_p(c), cl, _p(r), rl, C.byref(mlp) if mlp is not None else None,
                            C.byref(hin) if hin is not None else None, C.byref(hout) if hout is not None else None,
                            _p(out), cap, C.byref(ol), _p(nref), ncap, C.byref(nl), C.byref(mode), op)
    if st:
        return st, None, None, None, None
    return st, out[: ol.value].copy(), nref[: nl.value].copy(), mode.value, hout_obj


def delta_decode(enc: np.ndarray, ref: np.ndarray, mlp: MLP | None = None, hist: History | None = None,
                 want_hist: bool = False, cap: int | None = None, op: int = 0):
    """Decode one message with the receiver's operator op.  Returns
    (status, out, hist_out)."""
    L = lib()
    e, el = _buf(enc)
    r, rl = _buf(ref)
    if cap is None:
        cap = 64 + 2 * (el + rl) + 64
    out = np.zeros(max(cap, 8), np.uint8)
    ol = C.c_int64(0)
    hin = hist.struct() if hist is not None else None
    n_out = 0
    if el >= 64 and (want_hist or mlp is not None):
        hdr = np.frombuffer(e[:64].tobytes(), np.uint32)
        n_out = int(hdr[3]) + int(hdr[4])
    hout_obj = History(n_out) if (want_hist or mlp is not None) else None
    hout = hout_obj.struct() if hout_obj is not None else None
    st = L.orc_delta_decode(_p(e), el, _p(r), rl, C.byref(mlp) if mlp is not None else None,
                            C.byref(hin) if hin is not None else None, C.byref(hout) if hout is not None else None,
                            _p(out), cap, C.byref(ol), op)
    if st:
        return st, None, None
    return st, out[: ol.value].copy(), hout_obj


def predictor_inputs(ref: np.ndarray, hist: History, cell: float):
    """(inputs int32[n,12], predicted uint8[n]) for every slot of ref."""
    r, rl = _buf(ref)
    _, n, _ = view(ref)
    inp = np.zeros((max(n, 1), 12), np.int32)
    pred = np.zeros(max(n, 1), np.uint8)
    h = hist.struct()
    st = lib().orc_predictor_inputs(_p(r), rl, C.byref(h), float(cell), _p(inp), _p(pred))
    if st:
        raise RuntimeError(f"orc_predictor_inputs status {st}")
    return inp[:n], pred[:n]


# ---------------------------------------------------------------------------
# multi-segment helpers: messages concatenated densely, offsets [nseg+1]
def split(buf: np.ndarray, off: np.ndarray):
    return [buf[int(off[s]):int(off[s + 1])] for s in range(off.shape[0] - 1)]


def join(msgs):
    off = np.zeros(len(msgs) + 1, np.int64)
    np.cumsum([m.size for m in msgs], out=off[1:])
    buf = np.concatenate(msgs) if msgs else np.zeros(0, np.uint8)
    return buf, off


def empty_messages(nseg: int):
    """nseg empty TAM1 messages (the reference before the first exchange)."""
    one = np.zeros(32, np.uint8)
    one[:4] = np.frombuffer(b"TAM1", np.uint8)
    one[4] = 1
    return join([one.copy() for _ in range(nseg)])


def encode_all(cur, cur_off, ref, ref_off, mlp=None, hist=None, want_hist=False, op=0):
    """Encode every segment.  Returns (enc, enc_off, newref, newref_off, modes, hist_out)."""
    cs, rs = split(cur, cur_off), split(ref, ref_off)
    encs, nrefs, modes, hists = [], [], [], []
    base = 0
    for s in range(len(cs)):
        _, nr, _ = view(rs[s])
        hs = hist.slice(base, base + nr) if hist is not None else None
        base += nr
        st, e, n, m, h = delta_encode(cs[s], rs[s], mlp, hs, want_hist, op=op)
        if st:
            raise RuntimeError(f"orc_delta_encode segment {s}: status {st}")
        encs.append(e)
        nrefs.append(n)
        modes.append(m)
        hists.append(h)
    enc, enc_off = join(encs)
    nref, nref_off = join(nrefs)
    hout = History.concat(hists) if (want_hist or mlp is not None) else None
    return enc, enc_off, nref, nref_off, np.array(modes, np.uint8), hout


def decode_all(enc, enc_off, ref, ref_off, mlp=None, hist=None, want_hist=False, op=0):
    es, rs = split(enc, enc_off), split(ref, ref_off)
    outs, hists = [], []
    base = 0
    for s in range(len(es)):
        _, nr, _ = view(rs[s])
        hs = hist.slice(base, base + nr) if hist is not None else None
        base += nr
        st, o, h = delta_decode(es[s], rs[s], mlp, hs, want_hist, op=op)
        if st:
            raise RuntimeError(f"orc_delta_decode segment {s}: status {st}")
        outs.append(o)
        hists.append(h)
    out, off = join(outs)
    hout = History.concat(hists) if (want_hist or mlp is not None) else None
    return out, off, hout
