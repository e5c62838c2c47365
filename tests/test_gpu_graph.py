"""Batched iterations: the iteration entry point against the oracle, HIP
graph replays against eager runs, launch-shape invariance, tuning and its
cache.

Graph replays alternate with eager work (loading the next population state,
reading results back) and every replay is compared with an eager iteration
on the same inputs."""
import numpy as np
import pytest

import oracle
from paper_2509_24063_amd import synth
from tests.exchange_util import OracleSide, host
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


def _outputs(pl):
    enc, eoff, nref, noff, rx, rxoff = pl.outputs()
    e, n = host(eoff), host(noff)
    out = dict(eoff=e, enc=host(enc, e), noff=n, nref=host(nref, n), moff=host(pl.msg_off))
    out["msgs"] = host(pl.msgs, out["moff"])
    if rx is not None:
        r = host(rxoff)
        out["rxoff"], out["rx"] = r, host(rx, r)
    return out


def _same(a, b, tag):
    for k in a:
        assert np.array_equal(a[k], b[k]), f"{tag}: {k}"


@pytest.mark.parametrize("op", [0, 1])
def test_iteration_entry_matches_oracle(native, op):
    from paper_2509_24063_amd.exchange import Pipeline, capacities
    cfg = synth.config(3, median=300.0)
    world = synth.World(cfg)
    ctx = native.Context(cfg.schema)
    ctx.set_difference_op(op)
    idx_cap, msgs_cap = capacities(ctx, world.store, cfg.ndirs, cfg.w, slack=1.5)
    ds0 = native.DeviceStore(world.store)
    pl = Pipeline(ctx, ds0, cfg.w, cfg.ndirs, idx_cap, msgs_cap)
    orc = OracleSide(pl.nseg, op)
    for it in range(3):
        print(f"[iteration] cfg3-small op {op} {it}", flush=True)
        ds = native.DeviceStore(world.store)
        pl.step(ds)
        ctx.check(f"iteration {it}")
        o = orc.step(world.store, cfg)
        g = _outputs(pl)
        assert np.array_equal(g["moff"], o["moff"]) and np.array_equal(g["msgs"], o["buf"])
        assert np.array_equal(g["eoff"], o["eoff"]) and np.array_equal(g["enc"], o["enc"])
        assert np.array_equal(g["noff"], o["noff"]) and np.array_equal(g["nref"], o["nref"])
        assert np.array_equal(g["rxoff"], o["noff"]) and np.array_equal(g["rx"], o["nref"])
        world.step()
    ctx.close()


@pytest.mark.parametrize("learned,op", [(False, 0), (True, 0), (True, 1)])
def test_graph_replays_match_eager(native, learned, op):
    from paper_2509_24063_amd.exchange import Pipeline, capacities
    cfg = synth.config(3, median=500.0, persistent=learned)
    world = synth.World(cfg)
    ctx = native.Context(cfg.schema)
    ctx.set_difference_op(op)  # graphs captured under an operator replay it
    pred = native.Predictor(ctx, copy_last_move_blob()) if learned else None
    idx_cap, msgs_cap = capacities(ctx, world.store, cfg.ndirs, cfg.w, slack=1.5)
    cap = int(world.store.n * 1.3)
    beh_cap = int(world.store.beh.size * 1.3) + 64
    fixed = native.DeviceStore(world.store, cap=cap, beh_cap=beh_cap)
    gpl = Pipeline(ctx, fixed, cfg.w, cfg.ndirs, idx_cap, msgs_cap, pred=pred)
    epl = Pipeline(ctx, native.DeviceStore(world.store), cfg.w, cfg.ndirs, idx_cap, msgs_cap, pred=pred)
    gpl.capture()
    learned_segments = 0
    for it in range(6):
        print(f"[graph] learned={learned} iteration {it}", flush=True)
        fixed.load(world.store)           # eager work between replays
        gpl.step(graph=True)
        epl.step(native.DeviceStore(world.store))
        ctx.check(f"iteration {it}")
        _same(_outputs(gpl), _outputs(epl), f"iteration {it}")
        if learned:
            learned_segments += int(host(gpl.modes)[: gpl.nseg].sum())
        world.step()
    if learned:
        assert learned_segments > 0
    gpl.close()
    ctx.close()


def test_launch_shapes_do_not_change_results(native):
    from paper_2509_24063_amd.exchange import Pipeline, capacities
    cfg = synth.config(5, median=300.0, grid=(2, 2, 2))
    world = synth.World(cfg)
    ctx = native.Context(cfg.schema)
    idx_cap, msgs_cap = capacities(ctx, world.store, cfg.ndirs, cfg.w, slack=1.5)
    states = []
    for _ in range(3):
        states.append(native.DeviceStore(world.store))
        world.step()
    ref = None
    for grids in (None, [1, 1, 1, 1], [3, 5, 7, 2], [256, 4096, 512, 1024]):
        print(f"[shapes] grids {grids}", flush=True)
        ctx.set_grids(grids)
        pl = Pipeline(ctx, states[0], cfg.w, cfg.ndirs, idx_cap, msgs_cap)
        res = []
        for ds in states:
            pl.step(ds)
            ctx.check(f"grids {grids}")
            res.append(_outputs(pl))
        if ref is None:
            ref = res
        else:
            for a, b in zip(ref, res):
                _same(a, b, f"grids {grids}")
    ctx.set_grids(None)
    ctx.close()


def test_tune_and_cache(native, tmp_path):
    from paper_2509_24063_amd.exchange import Pipeline, capacities
    cfg = synth.config(3, median=300.0)
    world = synth.World(cfg)
    ctx = native.Context(cfg.schema)
    idx_cap, msgs_cap = capacities(ctx, world.store, cfg.ndirs, cfg.w, slack=1.5)
    ds = native.DeviceStore(world.store)
    pl = Pipeline(ctx, ds, cfg.w, cfg.ndirs, idx_cap, msgs_cap)
    pl.step()
    want = _outputs(pl)
    pl.reset()
    default = ctx.grids()
    cache = str(tmp_path / "tune.txt")
    print("[tune] timing", flush=True)
    assert ctx.tune(pl.iteration(0), cache, reps=2) is False
    tuned = ctx.grids()
    assert all(g % 256 == 0 or g == d for g, d in zip(tuned, default))
    lines = open(cache).read().split("\n")
    assert len([x for x in lines if x]) == 1
    ctx.set_grids(None)
    assert ctx.tune(pl.iteration(0), cache, reps=2) is True
    assert ctx.grids() == tuned
    pl.reset()
    pl.step()
    ctx.check("after tuning")
    _same(_outputs(pl), want, "tuned")
    ctx.close()
