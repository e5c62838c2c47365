"""GPU parity of the byte-wise subtraction operator (operator 1 of the
difference of Sec. 2.3): encodings, C' on both sides and the modes, byte
for byte against the oracle over several exchanges, plain and with a
predictor (learned and mixed segments); an encoding made with the other
operator is rejected like the oracle rejects it."""
import numpy as np
import pytest

import oracle
from paper_2509_24063_amd import synth
from tests.exchange_util import host
from tests.test_oracle_predictor import copy_last_move_blob

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_24063_amd import native as n
    n.lib()
    return n


@pytest.mark.parametrize("learned", [False, True])
def test_subtraction_exchanges_match_oracle(native, learned):
    cfg = synth.config(1, median=3000.0, persistent=False)
    world = synth.World(cfg)
    ctx = native.Context(cfg.schema)
    ctx.set_difference_op(1)
    b = copy_last_move_blob()
    pred = native.Predictor(ctx, b) if learned else None
    m = oracle.mlp_struct(b) if learned else None
    nseg = cfg.ndirs
    ref, roff = native.empty_messages(nseg)
    rx, rxoff = ref, roff
    href, hrx = native.History(0), native.History(0)
    oref, ooff = oracle.empty_messages(nseg)
    ohist = oracle.History(0)
    modes_seen = set()
    for it in range(5):
        s = world.store
        print(f"[subtract learned={learned}] iteration {it}", flush=True)
        ds = native.DeviceStore(s)
        idx, seg = ctx.select_aura(ds, cfg.w, cfg.ndirs)
        buf, moff = ctx.serialize(ds, idx, seg)
        nrec = int(host(seg)[-1])
        hout, hrxo = native.History(nrec), native.History(nrec)
        kw = dict(pred=pred, hist=href, hist_out=hout) if learned else {}
        enc, eoff, nref, noff, modes = ctx.delta_encode(buf, moff, ref, roff, **kw)
        kw = dict(pred=pred, hist=hrx, hist_out=hrxo) if learned else {}
        dec, doff = ctx.delta_decode(enc, eoff, rx, rxoff, **kw)
        ctx.check(f"iteration {it}")
        obuf, omoff = oracle.serialize(s, cfg.schema, *oracle.select_aura(s, cfg.w, cfg.ndirs))
        oenc, oeoff, onref, onoff, omodes, onh = oracle.encode_all(obuf, omoff, oref, ooff, m, ohist if learned else None,
                                                                   op=1)
        assert np.array_equal(host(eoff), oeoff)
        assert np.array_equal(host(enc, host(eoff)), oenc)
        assert np.array_equal(host(modes)[:nseg], omodes)
        assert np.array_equal(host(nref, host(noff)), onref)
        assert np.array_equal(host(dec, host(doff)), onref)
        modes_seen |= set(int(v) for v in omodes)
        ref, roff = nref[: int(host(noff)[-1])].clone(), noff.clone()
        rx, rxoff = dec[: int(host(doff)[-1])].clone(), doff.clone()
        href, hrx = hout, hrxo
        oref, ooff = onref, onoff
        if learned:
            ohist = onh
        world.step()
    if learned:
        assert 2 in modes_seen
    ctx.close()


def test_operator_mismatch_and_bad_value(native):
    cfg = synth.config(1, median=3000.0)
    world = synth.World(cfg)
    s0 = world.store
    world.step()
    s1 = world.store
    nseg = cfg.ndirs
    sender, receiver = native.Context(cfg.schema), native.Context(cfg.schema)
    sender.set_difference_op(1)
    with pytest.raises(Exception):
        sender.set_difference_op(2)
    msgs = []
    for s in (s0, s1):
        ds = native.DeviceStore(s)
        idx, seg = sender.select_aura(ds, cfg.w, cfg.ndirs)
        msgs.append(sender.serialize(ds, idx, seg))
    ref, roff = native.empty_messages(nseg)
    _, _, r1, r1off, _ = sender.delta_encode(*msgs[0], ref, roff)
    sender.check("first encoding")
    enc, eoff, _, _, _ = sender.delta_encode(*msgs[1], r1[: int(host(r1off)[-1])].clone(), r1off.clone())
    sender.check("second encoding")
    rxref = r1[: int(host(r1off)[-1])].clone()
    receiver.delta_decode(enc, eoff, rxref, r1off.clone())   # receiver still on XOR
    assert receiver.poll() == native.INVALID
    oe, ooff = host(enc, host(eoff)), host(eoff)
    st, _, _ = oracle.delta_decode(oe[ooff[0]:ooff[1]], host(rxref, host(r1off))[host(r1off)[0]:host(r1off)[1]], op=0)
    assert st == oracle.INVALID
    receiver.set_difference_op(1)
    dec, doff = receiver.delta_decode(enc, eoff, rxref, r1off.clone())
    receiver.check("matching operator")
    sender.close()
    receiver.close()
