"""Helpers for the GPU parity tests: one exchange through the HIP library and
the same exchange through the oracle, and byte comparisons of every buffer."""
import numpy as np

import oracle


def host(t, off=None):
    if off is None:
        return t.cpu().numpy()
    end = int(off[-1])
    return t[:end].cpu().numpy()


class GpuSide:
    """Sender and receiver on the GPU: references kept on the device."""

    def __init__(self, ctx, nseg, device="cuda"):
        from paper_2509_24063_amd import native
        self.ctx = ctx
        self.ref, self.ref_off = native.empty_messages(nseg, device)
        self.rx_ref, self.rx_ref_off = self.ref, self.ref_off

    def step(self, ds, cfg, idx_cap=None):
        ctx = self.ctx
        idx, seg = ctx.select_aura(ds, cfg.w, cfg.ndirs, idx_cap=idx_cap)
        buf, moff = ctx.serialize(ds, idx, seg)
        enc, eoff, nref, noff, modes = ctx.delta_encode(buf, moff, self.ref, self.ref_off)
        dec, doff = ctx.delta_decode(enc, eoff, self.rx_ref, self.rx_ref_off)
        ctx.check("exchange")
        out = dict(idx=idx, seg=seg, buf=buf, moff=moff, enc=enc, eoff=eoff, nref=nref, noff=noff, dec=dec,
                   doff=doff)
        self.ref, self.ref_off = nref, noff
        self.rx_ref, self.rx_ref_off = dec, doff
        return out


class OracleSide:
    def __init__(self, nseg, op=0):
        self.ref, self.ref_off = oracle.empty_messages(nseg)
        self.op = op

    def step(self, store, cfg):
        idx, seg = oracle.select_aura(store, cfg.w, cfg.ndirs)
        buf, moff = oracle.serialize(store, cfg.schema, idx, seg)
        enc, eoff, nref, noff, modes, _ = oracle.encode_all(buf, moff, self.ref, self.ref_off, op=self.op)
        dec, doff, _ = oracle.decode_all(enc, eoff, self.ref, self.ref_off, op=self.op)
        assert np.array_equal(dec, nref)
        out = dict(idx=idx, seg=seg, buf=buf, moff=moff, enc=enc, eoff=eoff, nref=nref, noff=noff)
        self.ref, self.ref_off = nref, noff
        return out


def assert_same(g, o, tag=""):
    seg = host(g["seg"])
    assert np.array_equal(seg, o["seg"]), f"{tag}: segment offsets"
    assert np.array_equal(host(g["idx"])[: int(seg[-1])], o["idx"]), f"{tag}: selected indices"
    moff = host(g["moff"])
    assert np.array_equal(moff, o["moff"]), f"{tag}: message offsets"
    assert np.array_equal(host(g["buf"], moff), o["buf"]), f"{tag}: TAM1 messages"
    eoff = host(g["eoff"])
    assert np.array_equal(eoff, o["eoff"]), f"{tag}: encoding offsets"
    assert np.array_equal(host(g["enc"], eoff), o["enc"]), f"{tag}: TAD1 encodings"
    noff = host(g["noff"])
    assert np.array_equal(noff, o["noff"]), f"{tag}: C' offsets (sender)"
    assert np.array_equal(host(g["nref"], noff), o["nref"]), f"{tag}: C' (sender)"
    doff = host(g["doff"])
    assert np.array_equal(doff, o["noff"]), f"{tag}: C' offsets (receiver)"
    assert np.array_equal(host(g["dec"], doff), o["nref"]), f"{tag}: C' (receiver)"


class OracleLearnedSide:
    """The oracle's sender and receiver in learned mode: the reference (C' of
    the previous exchange) and its predictor history, the same on both sides;
    each step checks that the receiver's C' and history equal the sender's."""

    def __init__(self, nseg, mlp, op=0):
        self.ref, self.ref_off = oracle.empty_messages(nseg)
        self.hist = oracle.History(0)
        self.mlp, self.op = mlp, op

    def step(self, store, cfg):
        idx, seg = oracle.select_aura(store, cfg.w, cfg.ndirs)
        buf, moff = oracle.serialize(store, cfg.schema, idx, seg)
        enc, eoff, nref, noff, modes, h = oracle.encode_all(buf, moff, self.ref, self.ref_off, self.mlp, self.hist,
                                                            op=self.op)
        dec, doff, hd = oracle.decode_all(enc, eoff, self.ref, self.ref_off, self.mlp, self.hist, op=self.op)
        assert np.array_equal(dec, nref) and np.array_equal(doff, noff)
        assert np.array_equal(hd.h1, h.h1) and np.array_equal(hd.h2, h.h2) and np.array_equal(hd.hlen, h.hlen)
        out = dict(idx=idx, seg=seg, buf=buf, moff=moff, enc=enc, eoff=eoff, nref=nref, noff=noff, modes=modes,
                   hist=h)
        self.ref, self.ref_off, self.hist = nref, noff, h
        return out


def tied_learned_groups(enc, eoff, plain, plain_off):
    """Groups of learned (mode 1) segments whose learned and plain blocks
    have the same size but differ (the encoder must write the learned one):
    counted from the oracle's learned encodings and its plain encodings of
    the same messages."""
    from tests.specparse import group_blocks
    n = 0
    for s in range(len(eoff) - 1):
        mode, gl = group_blocks(enc[eoff[s]:eoff[s + 1]].tobytes())
        if mode != 1:
            continue
        _, gp = group_blocks(plain[plain_off[s]:plain_off[s + 1]].tobytes())
        for (sl, bl, xl), (sp, bp, xp) in zip(gl, gp):
            n += int((sl & 0x7F) == (sp & 0x7F) and (bl != bp or xl != xp))
    return n
