"""GPU parity of the learned predictor: the integer MLP (matrix-core layer
included) against the oracle bit for bit, and learned-mode exchanges --
encodings, the chosen mode per segment, C' and the predictor history --
byte-equal to the oracle on both sides."""
import numpy as np
import pytest

import oracle
from paper_2509_24063_amd import synth
from tests.exchange_util import host
from tests.test_oracle_predictor import _moving_pair, blob, copy_last_move_blob

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_24063_amd import native as n
    n.lib()
    return n


def _random_blob(rng, r=(7, 9, 5), cell=24.0, scale=128):
    w1 = rng.integers(-scale, scale, (64, 12))
    w2 = rng.integers(-scale, scale, (64, 64))
    w3 = rng.integers(-scale, scale, (4, 64))
    b1 = rng.integers(-2**20, 2**20, 64)
    b2 = rng.integers(-2**16, 2**16, 64)
    b3 = rng.integers(-2**20, 2**20, 4)
    return blob(w1, w2, w3, b1, b2, b3, *r, cell=cell)


def test_mlp_matches_oracle(native):
    import torch
    rng = np.random.default_rng(21)
    ctx = native.Context(synth.Schema((4,), (1,)))
    for r in [(0, 0, 0), (7, 9, 5), (12, 3, 20), (24, 24, 24), (10, 10, 2)]:
        b = _random_blob(rng, r)
        x = rng.integers(-32768, 32768, (1000, 12)).astype(np.int32)
        x[:, 8:] = rng.integers(0, 128, (1000, 4))
        # the full input ranges: moves at the int16 limits, behaviour count and
        # class up to the u16 limit
        x[:100, :8] = rng.choice([-32768, -32767, -16385, -16384, -1, 0, 16383, 16384, 32767], (100, 8))
        x[:200, 9:11] = rng.choice([0, 127, 128, 16383, 16384, 32767, 32768, 65535], (200, 2))
        print(f"[mlp] shifts {r}", flush=True)
        pred = native.Predictor(ctx, b)
        q = host(ctx.predictor_eval(pred, torch.from_numpy(x).cuda()))
        ctx.check("eval")
        assert np.array_equal(q, oracle.mlp_forward(oracle.mlp_struct(b), x)), r
    ctx.close()


def _upload(msgs):
    import torch
    buf, off = oracle.join([np.asarray(m, np.uint8) for m in msgs])
    return (torch.from_numpy(buf if buf.size else np.zeros(8, np.uint8)).cuda(), torch.from_numpy(off).cuda())


def test_learned_handmade_exact_prediction(native):
    ref, cur, h = _moving_pair()
    b = copy_last_move_blob()
    ctx = native.Context(synth.Schema((4,), (1,)))
    pred = native.Predictor(ctx, b)
    R, roff = _upload([ref])
    Cb, coff = _upload([cur])
    hd = native.History.from_numpy(h.h1, h.h2, h.hlen)
    ho = native.History(len(h.hlen))
    print("[learned] handmade", flush=True)
    enc, eoff, nref, noff, modes = ctx.delta_encode(Cb, coff, R, roff, pred=pred, hist=hd, hist_out=ho)
    ctx.check("encode")
    st, oenc, onref, omode, ohist = oracle.delta_encode(cur, ref, oracle.mlp_struct(b), h)
    assert st == 0 and omode == 1 and int(host(modes)[0]) == 1
    assert np.array_equal(host(enc, host(eoff)), oenc)
    assert np.array_equal(host(nref, host(noff)), onref)
    g1, g2, gl = ho.numpy()
    assert np.array_equal(g1, ohist.h1) and np.array_equal(g2, ohist.h2) and np.array_equal(gl, ohist.hlen)
    hr = native.History(len(h.hlen))
    dec, doff = ctx.delta_decode(enc, eoff, R, roff, pred=pred, hist=hd, hist_out=hr)
    ctx.check("decode")
    assert np.array_equal(host(dec, host(doff)), onref)
    r1, r2, rl = hr.numpy()
    assert np.array_equal(r1, ohist.h1) and np.array_equal(r2, ohist.h2) and np.array_equal(rl, ohist.hlen)
    ctx.close()


def test_history_smaller_than_reference_is_invalid(native):
    """A learned call whose history holds fewer slots than the reference has
    records is rejected with TA_ERR_INVALID, on either side; the same
    context then runs the full call correctly."""
    ref, cur, h = _moving_pair()
    b = copy_last_move_blob()
    ctx = native.Context(synth.Schema((4,), (1,)))
    pred = native.Predictor(ctx, b)
    R, roff = _upload([ref])
    Cb, coff = _upload([cur])
    n = len(h.hlen)
    full = native.History.from_numpy(h.h1, h.h2, h.hlen)
    short = native.History.from_numpy(h.h1[:n - 1], h.h2[:n - 1], h.hlen[:n - 1])
    print("[learned] short history", flush=True)
    ctx.delta_encode(Cb, coff, R, roff, pred=pred, hist=short, hist_out=native.History(n))
    assert ctx.poll() == native.INVALID
    enc, eoff, nref, noff, _ = ctx.delta_encode(Cb, coff, R, roff, pred=pred, hist=full, hist_out=native.History(n))
    ctx.check("encode")
    ctx.delta_decode(enc, eoff, R, roff, pred=pred, hist=short, hist_out=native.History(n))
    assert ctx.poll() == native.INVALID
    dec, doff = ctx.delta_decode(enc, eoff, R, roff, pred=pred, hist=full, hist_out=native.History(n))
    ctx.check("decode")
    st, _, onref, _, _ = oracle.delta_encode(cur, ref, oracle.mlp_struct(b), h)
    assert st == 0
    assert np.array_equal(host(nref, host(noff)), onref) and np.array_equal(host(dec, host(doff)), onref)
    ctx.close()


@pytest.mark.parametrize("persistent,which", [(True, "copy"), (False, "copy"), (False, "random"), (True, "zero")])
def test_learned_iterations_match_oracle(native, persistent, which):
    """Sender and receiver on the GPU, oracle beside them, over several
    exchanges with the history carried along."""
    import torch
    rng = np.random.default_rng(5)
    if which == "copy":
        b = copy_last_move_blob()
    elif which == "zero":
        b = blob(np.zeros((64, 12)), np.zeros((64, 64)), np.zeros((4, 64)), np.zeros(64), np.zeros(64),
                 np.zeros(4), 0, 0, 0)
    else:
        b = _random_blob(rng, (9, 9, 4), scale=8)
    cfg = synth.config(1, median=3000.0, persistent=persistent)
    world = synth.World(cfg)
    ctx = native.Context(cfg.schema)
    pred = native.Predictor(ctx, b)
    m = oracle.mlp_struct(b)
    nseg = cfg.ndirs
    ref, roff = native.empty_messages(nseg)
    rx, rxoff = ref, roff
    href, hrx = native.History(0), native.History(0)
    oref, ooff = oracle.empty_messages(nseg)
    ohist = oracle.History(0)
    learned_segments = mixed_segments = 0
    for it in range(6):
        s = world.store
        print(f"[learned {which}] iteration {it}", flush=True)
        ds = native.DeviceStore(s)
        idx, seg = ctx.select_aura(ds, cfg.w, cfg.ndirs)
        buf, moff = ctx.serialize(ds, idx, seg)
        nrec = int(host(seg)[-1])
        hout, hrxo = native.History(nrec), native.History(nrec)
        enc, eoff, nref, noff, modes = ctx.delta_encode(buf, moff, ref, roff, pred=pred, hist=href, hist_out=hout)
        dec, doff = ctx.delta_decode(enc, eoff, rx, rxoff, pred=pred, hist=hrx, hist_out=hrxo)
        ctx.check(f"iteration {it}")
        obuf, omoff = oracle.serialize(s, cfg.schema, *oracle.select_aura(s, cfg.w, cfg.ndirs))
        oenc, oeoff, onref, onoff, omodes, onh = oracle.encode_all(obuf, omoff, oref, ooff, m, ohist)
        assert np.array_equal(host(eoff), oeoff)
        assert np.array_equal(host(enc, host(eoff)), oenc)
        assert np.array_equal(host(modes)[:nseg], omodes)
        assert np.array_equal(host(nref, host(noff)), onref)
        assert np.array_equal(host(dec, host(doff)), onref)
        for hh in (hout, hrxo):
            a1, a2, al = hh.numpy()
            assert np.array_equal(a1, onh.h1) and np.array_equal(a2, onh.h2) and np.array_equal(al, onh.hlen)
        learned_segments += int(np.count_nonzero(omodes))
        mixed_segments += int(np.count_nonzero(omodes == 2))
        ref, roff, rx, rxoff = nref[: int(host(noff)[-1])].clone(), noff.clone(), dec[: int(host(doff)[-1])].clone(), doff.clone()
        href, hrx = hout, hrxo
        oref, ooff, ohist = onref, onoff, onh
        world.step()
    if which == "copy" and persistent:
        assert learned_segments > 0   # the copy-last-move network wins on persistent motion
    if which == "copy" and not persistent:
        assert mixed_segments > 0     # on a random walk it helps some groups and hurts others
    if which == "zero":
        assert learned_segments == 0  # zero weights never beat plain (ties go to plain)
    ctx.close()


def test_plain_exchange_with_history(native):
    """Plain encodings (no predictor) that still write the history of C',
    on both sides: encodings, C' and the histories equal the oracle's."""
    cfg = synth.config(1, median=3000.0)
    world = synth.World(cfg)
    ctx = native.Context(cfg.schema)
    nseg = cfg.ndirs
    ref, roff = native.empty_messages(nseg)
    rx, rxoff = ref, roff
    oref, ooff = oracle.empty_messages(nseg)
    for it in range(4):
        s = world.store
        print(f"[plain history] iteration {it}", flush=True)
        ds = native.DeviceStore(s)
        idx, seg = ctx.select_aura(ds, cfg.w, cfg.ndirs)
        buf, moff = ctx.serialize(ds, idx, seg)
        nrec = int(host(seg)[-1])
        hout, hrxo = native.History(nrec), native.History(nrec)
        enc, eoff, nref, noff, _ = ctx.delta_encode(buf, moff, ref, roff, hist_out=hout)
        dec, doff = ctx.delta_decode(enc, eoff, rx, rxoff, hist_out=hrxo)
        ctx.check(f"iteration {it}")
        obuf, omoff = oracle.serialize(s, cfg.schema, *oracle.select_aura(s, cfg.w, cfg.ndirs))
        oenc, oeoff, onref, onoff, _, onh = oracle.encode_all(obuf, omoff, oref, ooff, want_hist=True)
        assert np.array_equal(host(enc, host(eoff)), oenc)
        assert np.array_equal(host(nref, host(noff)), onref)
        assert np.array_equal(host(dec, host(doff)), onref)
        for hh in (hout, hrxo):
            a1, a2, al = hh.numpy()
            assert np.array_equal(a1, onh.h1) and np.array_equal(a2, onh.h2) and np.array_equal(al, onh.hlen)
        ref, roff = nref[: int(host(noff)[-1])].clone(), noff.clone()
        rx, rxoff = dec[: int(host(doff)[-1])].clone(), doff.clone()
        oref, ooff = onref, onoff
        world.step()
    ctx.close()
