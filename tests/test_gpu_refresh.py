"""GPU parity with a reference refresh interval k > 1 (Sec. 2.3: sender and
receiver update their reference at regular intervals).  Between refreshes
every iteration is encoded against the same reference; the pipeline's
encodings, C' and the receiver's C' equal the oracle's under the same
policy, byte for byte, eagerly and from captured graphs."""
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


def _oracle_run(states, cfg, k):
    nseg = states[0].P * cfg.ndirs
    ref, ref_off = oracle.empty_messages(nseg)
    out = []
    for t, st in enumerate(states):
        idx, seg = oracle.select_aura(st, cfg.w, cfg.ndirs)
        buf, moff = oracle.serialize(st, cfg.schema, idx, seg)
        enc, eoff, nref, noff, _, _ = oracle.encode_all(buf, moff, ref, ref_off)
        dec, doff, _ = oracle.decode_all(enc, eoff, ref, ref_off)
        assert np.array_equal(dec, nref) and np.array_equal(doff, noff)
        out.append((enc, eoff, nref, noff))
        if t % k == 0:
            ref, ref_off = nref, noff
    return out


@pytest.mark.parametrize("k,graph", [(2, False), (3, False), (3, True)])
def test_refresh_interval_matches_oracle(native, k, graph):
    from paper_2509_24063_amd.exchange import Pipeline, capacities
    cfg = synth.config(1)
    world = synth.World(cfg)
    states = []
    for _ in range(7):
        states.append(world.store)
        world.step()
    want = _oracle_run(states, cfg, k)
    ctx = native.Context(cfg.schema)
    idx_cap, msgs_cap = capacities(ctx, states[0], cfg.ndirs, cfg.w, slack=1.5)
    cap = max(s.n for s in states) + 64
    beh = max(s.beh.size for s in states) + 4096
    ds = native.DeviceStore(states[0], cap=cap, beh_cap=beh)
    ctx.reserve(cap, states[0].P * cfg.ndirs, idx_cap, msgs_cap)
    pl = Pipeline(ctx, ds, cfg.w, cfg.ndirs, idx_cap, msgs_cap, refresh=k)
    for t, st in enumerate(states):
        print(f"[refresh k={k} graph={graph}] iteration {t}", flush=True)
        ds.load(st)
        pl.step(graph=graph)
        ctx.check(f"iteration {t}")
        enc, eoff, nref, noff, rx, rxoff = pl.outputs()
        we, weo, wn, wno = want[t]
        assert np.array_equal(host(eoff), weo), t
        assert np.array_equal(host(enc, eoff), we), t
        assert np.array_equal(host(noff), wno), t
        assert np.array_equal(host(nref, noff), wn), t
        assert np.array_equal(host(rxoff), wno), t
        assert np.array_equal(host(rx, rxoff), wn), t
    pl.close()
    ctx.close()
