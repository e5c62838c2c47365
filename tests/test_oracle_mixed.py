"""Pins of the mixed encoding (mode 2: the learned/plain choice per 64-word
group instead of per segment).  For every segment encoded in mode 2 over
several exchanges of the random-walk world with a copy-last-move predictor: it decodes back to C'; a
group flagged plain has exactly the block size of the segment's plain
encoding (an independent call without a predictor); a group flagged learned
is strictly smaller than there; and the whole residual is smaller than both
the plain one and the encoding's own learned-only alternative would allow.
"""
import numpy as np

import oracle
from paper_2509_24063_amd import synth
from tests.test_oracle_predictor import copy_last_move_blob


def _groups(enc):
    n_ref = int(enc[8:12].view(np.uint32)[0])
    W = int(enc[40:48].view(np.uint64)[0])
    G = (W + 63) // 64
    at = 64 + 8 * ((n_ref + 63) // 64) + 8 * G
    return enc[at:at + G], int(enc[56:64].view(np.uint64)[0])


def test_mixed_mode_segments():
    # the copy-last-move network on a random walk: its prediction helps some
    # groups and hurts others
    cfg = synth.config(1, median=3000.0, persistent=False)
    world = synth.World(cfg)
    m = oracle.mlp_struct(copy_last_move_blob())
    ref, ref_off = oracle.empty_messages(cfg.ndirs)
    hist = oracle.History(0)
    mixed = 0
    for it in range(6):
        st = world.store
        idx, seg = oracle.select_aura(st, cfg.w, cfg.ndirs)
        buf, moff = oracle.serialize(st, cfg.schema, idx, seg)
        cs, rs = oracle.split(buf, moff), oracle.split(ref, ref_off)
        base = 0
        for s in range(len(cs)):
            _, nr, _ = oracle.view(rs[s])
            hs = hist.slice(base, base + nr)
            base += nr
            status, enc, nref, mode, _ = oracle.delta_encode(cs[s], rs[s], m, hs, True)
            assert status == 0
            if mode != 2:
                continue
            mixed += 1
            status, dec, _ = oracle.delta_decode(enc, rs[s], m, hs)
            assert status == 0 and np.array_equal(dec, nref)
            status, plain, pref, pmode, _ = oracle.delta_encode(cs[s], rs[s])
            assert status == 0 and pmode == 0 and np.array_equal(pref, nref)
            gm, var_m = _groups(enc)
            gp, var_p = _groups(plain)
            flags = gm >> 7
            assert flags.any() and not flags.all()
            assert np.array_equal((gm & 0x7F)[flags == 0], gp[flags == 0])
            assert np.all((gm & 0x7F)[flags == 1] < gp[flags == 1])
            assert var_m < var_p and var_m == 8 * int((gm & 0x7F).astype(np.int64).sum())
        enc_all = oracle.encode_all(buf, moff, ref, ref_off, m, hist)
        ref, ref_off, hist = enc_all[2], enc_all[3], enc_all[5]
        world.step()
    assert mixed > 0
