"""The pipelined exchange (selection + serialization, encoding and decoding
on three streams, one context each) against the oracle: every iteration's
encoding and both sides' C' when each step is checked, and the final ones
when all steps run back to back with no host synchronisation in between
(iterations t - 1, t and t + 1 in flight together)."""
import numpy as np
import pytest

import oracle
from paper_2509_24063_amd import synth
from tests.exchange_util import host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_24063_amd import native as n
    n.lib()
    return n


def _states(cfg, n):
    world = synth.World(cfg)
    out = []
    for _ in range(n):
        out.append(world.store)
        world.step()
    return out


def _oracle(states, cfg):
    ref, ref_off = oracle.empty_messages(states[0].P * cfg.ndirs)
    out = []
    for st in states:
        idx, seg = oracle.select_aura(st, cfg.w, cfg.ndirs)
        buf, moff = oracle.serialize(st, cfg.schema, idx, seg)
        enc, eoff, nref, noff, _, _ = oracle.encode_all(buf, moff, ref, ref_off)
        out.append((enc, eoff, nref, noff))
        ref, ref_off = nref, noff
    return out


def _same(got, want, tag):
    enc, eoff, nref, noff, rx, rxoff = got
    we, weo, wn, wno = want
    assert np.array_equal(host(eoff), weo) and np.array_equal(host(enc, eoff), we), tag
    assert np.array_equal(host(noff), wno) and np.array_equal(host(nref, noff), wn), tag
    assert np.array_equal(host(rxoff), wno) and np.array_equal(host(rx, rxoff), wn), tag


@pytest.mark.parametrize("sync_each", [True, False])
def test_overlapped_exchange_matches_oracle(native, sync_each):
    from paper_2509_24063_amd.exchange import OverlapPipeline, capacities
    cfg = synth.config(3, median=300.0, grid=(2, 2, 2))
    states = _states(cfg, 7)
    want = _oracle(states, cfg)
    ctx = native.Context(cfg.schema)
    idx_cap, msgs_cap = capacities(ctx, states[0], cfg.ndirs, cfg.w, slack=1.5)
    ctx.close()
    dss = [native.DeviceStore(s) for s in states]
    pl = OverlapPipeline(cfg.schema, dss[0], cfg.w, cfg.ndirs, idx_cap, msgs_cap)
    pl.reserve(max(s.n for s in states))
    for t, ds in enumerate(dss):
        print(f"[overlap sync_each={sync_each}] iteration {t}", flush=True)
        pl.step(ds)
        if sync_each:
            pl.check(f"iteration {t}")
            _same(pl.outputs(), want[t], t)
    pl.check("end")
    _same(pl.outputs(), want[-1], "last")
    pl.close()


def test_overlapped_exchange_reusing_one_store(native):
    """One fixed-capacity store whose buffers receive every state by load()
    on the caller's stream right before each step, with no host
    synchronisation in between: each serialization must see its own state
    complete, and the next load must not overwrite a state still being
    serialized."""
    from paper_2509_24063_amd.exchange import OverlapPipeline, capacities
    cfg = synth.config(3, median=300.0, grid=(2, 2, 2))
    states = _states(cfg, 6)
    want = _oracle(states, cfg)
    ctx = native.Context(cfg.schema)
    idx_cap, msgs_cap = capacities(ctx, states[0], cfg.ndirs, cfg.w, slack=1.5)
    ctx.close()
    cap = max(s.n for s in states)
    ds = native.DeviceStore(states[0], cap=cap, beh_cap=max(s.beh.size for s in states))
    pl = OverlapPipeline(cfg.schema, ds, cfg.w, cfg.ndirs, idx_cap, msgs_cap)
    pl.reserve(cap)
    outs = []
    for t, st in enumerate(states):
        print(f"[overlap one store] iteration {t}", flush=True)
        ds.load(st)
        pl.step(ds)
        if t >= len(states) - 2:
            pl.check(f"iteration {t}")
            outs.append(tuple(x.clone() for x in pl.outputs()))
    pl.check("end")
    _same(outs[0], want[-2], "second to last")
    _same(outs[1], want[-1], "last")
    pl.close()


def test_stream_tuning_keeps_results(native):
    """Choosing the stages' streams by timing runs trial iterations and then
    starts over: the exchange that follows still equals the oracle's."""
    from paper_2509_24063_amd.exchange import OverlapPipeline, capacities
    cfg = synth.config(3, median=300.0, grid=(2, 2, 2))
    states = _states(cfg, 5)
    want = _oracle(states, cfg)
    ctx = native.Context(cfg.schema)
    idx_cap, msgs_cap = capacities(ctx, states[0], cfg.ndirs, cfg.w, slack=1.5)
    ctx.close()
    dss = [native.DeviceStore(s) for s in states]
    pl = OverlapPipeline(cfg.schema, dss[0], cfg.w, cfg.ndirs, idx_cap, msgs_cap)
    pl.reserve(max(s.n for s in states))
    print("[overlap] stream tuning", flush=True)
    sec = pl.tune_streams(dss[::-1], trials=3, steps=2)
    assert sec > 0 and pl.t == 0
    for t, ds in enumerate(dss):
        print(f"[overlap tuned] iteration {t}", flush=True)
        pl.step(ds)
    pl.check("end")
    _same(pl.outputs(), want[-1], "last")
    pl.close()
