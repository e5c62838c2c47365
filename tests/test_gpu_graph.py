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
from tests.exchange_util import OracleLearnedSide, OracleSide, host, tied_learned_groups
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


def _same_as_oracle(g, o, tag, pl=None):
    """Graph or eager pipeline outputs against the oracle's learned exchange:
    messages, encodings, modes, both sides' C' and the sender's history."""
    assert np.array_equal(g["moff"], o["moff"]) and np.array_equal(g["msgs"], o["buf"]), f"{tag}: messages"
    assert np.array_equal(g["eoff"], o["eoff"]) and np.array_equal(g["enc"], o["enc"]), f"{tag}: encodings"
    assert np.array_equal(g["noff"], o["noff"]) and np.array_equal(g["nref"], o["nref"]), f"{tag}: sender C'"
    assert np.array_equal(g["rxoff"], o["noff"]) and np.array_equal(g["rx"], o["nref"]), f"{tag}: receiver C'"
    if pl is not None:
        assert np.array_equal(host(pl.modes)[: pl.nseg], o["modes"]), f"{tag}: modes"
        h = o["hist"]
        for side in (pl.hist, pl.rx_hist):
            a1, a2, al = side[pl.last].numpy(h.hlen.shape[0])
            assert np.array_equal(a1, h.h1) and np.array_equal(a2, h.h2) and np.array_equal(al, h.hlen), \
                f"{tag}: history"


@pytest.mark.parametrize("learned,op", [(False, 0), (True, 0), (True, 1)])
def test_graph_replays_match_eager(native, learned, op):
    """Graph replays against eager iterations; learned replays (13,312
    segments: 512 partitions x 26) also against the oracle's learned
    exchange, with the predictor history carried along on both sides."""
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
    orc = OracleLearnedSide(gpl.nseg, oracle.mlp_struct(copy_last_move_blob()), op) if learned else None
    learned_segments = 0
    for it in range(6):
        print(f"[graph] learned={learned} op {op} iteration {it} ({gpl.nseg} segments)", flush=True)
        fixed.load(world.store)           # eager work between replays
        gpl.step(graph=True)
        epl.step(native.DeviceStore(world.store))
        ctx.check(f"iteration {it}")
        g = _outputs(gpl)
        _same(g, _outputs(epl), f"iteration {it}")
        if learned:
            learned_segments += int(np.count_nonzero(host(gpl.modes)[: gpl.nseg]))
            _same_as_oracle(g, orc.step(world.store, cfg), f"learned op {op} iteration {it}", gpl)
        world.step()
    if learned:
        assert learned_segments > 0
    gpl.close()
    ctx.close()


@pytest.mark.parametrize("op", [0, 1])
def test_heterogeneous_learned_matches_oracle(native, op):
    """The heterogeneous workload at reduced size (80/20 spheres and
    cylinders with 14 fp64 fields each, 0-4 behaviours of 1-7 payload words,
    2 % division, 1 % death; 2x2x2 partitions, 208 segments) in learned mode
    through the iteration entry: every buffer, the chosen modes and both
    sides' histories equal the oracle's."""
    from paper_2509_24063_amd.exchange import Pipeline, capacities
    cfg = synth.config(5, median=400.0, grid=(2, 2, 2), persistent=True)
    world = synth.World(cfg)
    ctx = native.Context(cfg.schema)
    ctx.set_difference_op(op)
    blob = copy_last_move_blob()
    pred = native.Predictor(ctx, blob)
    idx_cap, msgs_cap = capacities(ctx, world.store, cfg.ndirs, cfg.w, slack=1.5)
    pl = Pipeline(ctx, native.DeviceStore(world.store), cfg.w, cfg.ndirs, idx_cap, msgs_cap, pred=pred)
    orc = OracleLearnedSide(pl.nseg, oracle.mlp_struct(blob), op)
    modes, ties = [], 0
    for it in range(5):
        print(f"[cfg5 learned] op {op} iteration {it}", flush=True)
        pl.step(native.DeviceStore(world.store))
        ctx.check(f"iteration {it}")
        ref, ref_off = orc.ref, orc.ref_off
        o = orc.step(world.store, cfg)
        _same_as_oracle(_outputs(pl), o, f"cfg5 op {op} iteration {it}", pl)
        modes.append(o["modes"])
        pe, peo, _, _, _, _ = oracle.encode_all(o["buf"], o["moff"], ref, ref_off, op=op)
        ties += tied_learned_groups(o["enc"], o["eoff"], pe, peo)
        world.step()
    assert np.count_nonzero(np.concatenate(modes)) > 0  # the predictor wins some segments
    assert ties > 0  # learned segments with tied groups whose learned block differs were checked
    assert len(set(np.unique(world.store.cls))) == 2 and int(world.store.nb.max()) == 4
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


@pytest.mark.parametrize("learned", [False, True])
def test_shared_receiver_matches_own_copies(native, learned):
    """A receiver that decodes against the sender's reference and history and
    writes its C' over the consumed message buffer gives the same C' and
    history as one with copies of its own, eagerly and from graphs."""
    from paper_2509_24063_amd.exchange import Pipeline, capacities
    cfg = synth.config(5, median=400.0, grid=(2, 2, 2), persistent=True)
    world = synth.World(cfg)
    ctx = native.Context(cfg.schema)
    pred = native.Predictor(ctx, copy_last_move_blob()) if learned else None
    idx_cap, msgs_cap = capacities(ctx, world.store, cfg.ndirs, cfg.w, slack=1.5)
    cap = int(world.store.n * 1.3)
    fixed = native.DeviceStore(world.store, cap=cap, beh_cap=int(world.store.beh.size * 1.3) + 64)
    own = Pipeline(ctx, native.DeviceStore(world.store), cfg.w, cfg.ndirs, idx_cap, msgs_cap, pred=pred)
    shared = Pipeline(ctx, fixed, cfg.w, cfg.ndirs, idx_cap, msgs_cap, pred=pred, shared_rx=True,
                      enc_cap=int(msgs_cap * 1.1) + 64 * 208)
    shared.capture()
    for it in range(5):
        print(f"[shared rx] learned={learned} iteration {it}", flush=True)
        fixed.load(world.store)
        shared.step(graph=it % 2 == 1)
        own.step(native.DeviceStore(world.store))
        ctx.check(f"iteration {it}")
        a, b = _outputs(shared), _outputs(own)
        for k in ("eoff", "enc", "noff", "nref", "rxoff", "rx"):
            assert np.array_equal(a[k], b[k]), f"iteration {it}: {k}"
        if learned:  # the C' histories (records of C' of every segment)
            nrec = int(sum(np.frombuffer(b["nref"][o:o + 12].tobytes(), np.uint32)[2] for o in b["noff"][:-1]))
            x1, x2, xl = shared.rx_hist[0].numpy(nrec)
            y1, y2, yl = own.rx_hist[own.last].numpy(nrec)
            assert np.array_equal(x1, y1) and np.array_equal(x2, y2) and np.array_equal(xl, yl), f"history {it}"
        world.step()
    shared.close()
    ctx.close()
