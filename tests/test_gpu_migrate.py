"""GPU parity of agent migration (Sec. 2.1, "Agent Migration"): migrant
selection and the rebuilt store, through the C ABI, against the oracle.
Indices, segment offsets, messages and every column of the new store are
compared byte for byte."""
import numpy as np
import pytest

import oracle
from paper_2509_24063_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_24063_amd import native as n
    n.lib()
    return n


def _world(grid=(2, 2, 2), median=1500, sigma=3.0, steps=2, seed=7, side=60.0, **over):
    cfg = synth.config(1, grid=grid, median=median, step_sigma=sigma, walls="domain", side=side, seed=seed,
                       ndirs=26, **over)
    w = synth.World(cfg)
    for _ in range(steps):
        w.step()
    return cfg, w


def _cols(cfg):
    return max(cfg.schema.n_f64), max(cfg.schema.n_i32)


def _host(t):
    return t.cpu().numpy()


def _gpu_select(native, ctx, ds):
    idx, so = ctx.select_migrants(ds)
    ctx.check("select_migrants")
    so_h = _host(so)
    return idx, so, _host(idx)[: int(so_h[-1])], so_h


def _compare_store(tag, got, want, nf, ni):
    n = int(want["sizes"][0])
    assert np.array_equal(_host(got["sizes"]), want["sizes"]), tag
    assert np.array_equal(_host(got["part_off"]), want["part_off"]), tag
    ds = got["store"]
    assert np.array_equal(_host(ds.uid[:n]).view(np.uint64), want["uid"]), tag
    assert np.array_equal(_host(ds.cls[:n]).view(np.uint16), want["cls"]), tag
    assert np.array_equal(_host(ds.nb[:n]).view(np.uint16), want["nb"]), tag
    assert np.array_equal(_host(ds.f64[:nf, :n]).view(np.uint64), want["f64"].view(np.uint64)), tag
    assert np.array_equal(_host(ds.i32[:ni, :n]), want["i32"]), tag
    assert np.array_equal(_host(ds.beh_off[:n + 1]), want["beh_off"]), tag
    assert np.array_equal(_host(ds.beh[: int(want["sizes"][1])]), want["beh"]), tag


def _exchange(native, ctx, cfg, store, dest, tag, cap=None, beh_cap=None, msgs=None):
    """select -> serialize -> apply on the GPU and in the oracle; returns both results."""
    import torch
    nf, ni = _cols(cfg)
    ds = native.DeviceStore(store)
    print(f"[{tag}] {store.n} agents, {store.P} partitions", flush=True)
    idx, so, idx_h, so_h = _gpu_select(native, ctx, ds)
    oidx, oso = oracle.select_migrants(store)
    assert np.array_equal(idx_h, oidx) and np.array_equal(so_h, oso), tag
    if msgs is None:
        buf, moff = ctx.serialize(ds, idx, so)
        ctx.check("serialize")
        omsgs, omoff = oracle.serialize(store, cfg.schema, oidx, oso)
        assert np.array_equal(_host(moff), omoff) and np.array_equal(_host(buf)[: int(omoff[-1])], omsgs), tag
    else:
        omsgs, omoff = msgs
        buf = torch.from_numpy(np.concatenate([omsgs, np.zeros(8, np.uint8)])).cuda()
        moff = torch.from_numpy(omoff).cuda()
    status, want = oracle.migrate_apply(store, cfg.schema, omsgs, omoff, dest, nf, ni, cap=cap, beh_cap=beh_cap)
    need = want["sizes"]
    out = native.DeviceStore.alloc(nf, ni, store.boxes, int(need[0]) if cap is None else cap,
                                   int(need[1]) if beh_cap is None else beh_cap)
    dest_t = torch.from_numpy(np.ascontiguousarray(dest, np.int32)).cuda() if len(dest) else \
        torch.zeros(1, dtype=torch.int32, device="cuda")
    sizes = ctx.migrate_apply(ds, buf[: int(omoff[-1])] if int(omoff[-1]) else None, moff, dest_t, out)
    got_status = ctx.poll()
    return status, want, got_status, dict(sizes=sizes, part_off=out.part_off, store=out)


def test_select_migrants_matches_oracle(native):
    for seed, grid in [(3, (2, 2, 2)), (5, (3, 2, 1)), (8, (1, 1, 1))]:
        cfg, w = _world(grid=grid, seed=seed)
        ctx = native.Context(cfg.schema)
        ds = native.DeviceStore(w.store)
        _, _, idx, so = _gpu_select(native, ctx, ds)
        oidx, oso = oracle.select_migrants(w.store)
        assert np.array_equal(idx, oidx) and np.array_equal(so, oso), (seed, grid)
        ctx.close()


def test_select_migrants_many_tiles_and_ragged(native):
    # 2e5 agents over 4 uneven partitions: many 2048-agent tiles, ragged tails
    cfg, w = _world(grid=(2, 2, 1), median=5e4, sigma=0.5, seed=21, side=200.0, steps=1)
    ctx = native.Context(cfg.schema)
    ds = native.DeviceStore(w.store)
    _, _, idx, so = _gpu_select(native, ctx, ds)
    oidx, oso = oracle.select_migrants(w.store)
    assert len(oidx) > 100
    assert np.array_equal(idx, oidx) and np.array_equal(so, oso)
    ctx.close()


@pytest.mark.parametrize("over", [{}, dict(cyl_frac=0.3, n_f64=(4, 7), n_i32=(1, 3), nb_max=3,
                                         payload_words=(1, 4))])
def test_migrate_apply_matches_oracle(native, over):
    cfg, w = _world(seed=5, **over)
    ctx = native.Context(cfg.schema)
    dest = synth.neighbour_table(cfg.grid)
    nf, ni = _cols(cfg)
    store = w.store
    for it in range(3):
        st, want, gst, got = _exchange(native, ctx, cfg, store, dest, f"apply it {it}")
        assert st == oracle.OK and gst == native.OK
        _compare_store(f"it {it}", got, want, nf, ni)
        # the next iteration starts from the migrated store
        w.store = got["store"].numpy()
        w.step()
        store = w.store
    ctx.close()


def test_skipped_messages_and_single_partition_receiver(native):
    cfg, w = _world(seed=13)
    ctx = native.Context(cfg.schema)
    store = w.store
    nseg = store.P * 26
    st, want, gst, got = _exchange(native, ctx, cfg, store, np.full(nseg, -1, np.int32), "skipped")
    assert st == oracle.OK and gst == native.OK
    _compare_store("skipped", got, want, *_cols(cfg))
    # one-partition receiver: all messages of the 2x2x2 grid addressed to it
    oidx, oso = oracle.select_migrants(store)
    msgs = oracle.serialize(store, cfg.schema, oidx, oso)
    recv = store.partition(0)
    recv.f64[:3] = np.clip(recv.f64[:3], recv.boxes[0, :3, None], np.nextafter(recv.boxes[0, 3:, None], -np.inf))
    st, want, gst, got = _exchange(native, ctx, cfg, recv, np.zeros(nseg, np.int32), "receiver", msgs=msgs)
    assert st == oracle.OK and gst == native.OK
    assert int(want["sizes"][0]) == recv.n + len(oidx)
    _compare_store("receiver", got, want, *_cols(cfg))
    ctx.close()


def test_no_messages_and_empty_store(native):
    import torch
    cfg, w = _world(seed=29)
    ctx = native.Context(cfg.schema)
    nf, ni = _cols(cfg)
    store = w.store
    # no messages: the store only loses its migrants
    ds = native.DeviceStore(store)
    status, want = oracle.migrate_apply(store, cfg.schema, np.zeros(0, np.uint8), np.zeros(1, np.int64),
                                        np.zeros(0, np.int32), nf, ni)
    out = native.DeviceStore.alloc(nf, ni, store.boxes, int(want["sizes"][0]), int(want["sizes"][1]))
    sizes = ctx.migrate_apply(ds, None, torch.zeros(1, dtype=torch.int64, device="cuda"),
                              torch.zeros(1, dtype=torch.int32, device="cuda"), out)
    assert ctx.poll() == native.OK and status == oracle.OK
    _compare_store("no messages", dict(sizes=sizes, part_off=out.part_off, store=out), want, nf, ni)
    # empty store (every partition empty) taking in messages
    oidx, oso = oracle.select_migrants(store)
    msgs = oracle.serialize(store, cfg.schema, oidx, oso)
    empty = synth.Store(uid=np.zeros(0, np.uint64), cls=np.zeros(0, np.uint16), nb=np.zeros(0, np.uint16),
                        f64=np.zeros((nf, 0)), i32=np.zeros((ni, 0), np.int32), beh_off=np.zeros(1, np.int64),
                        beh=np.zeros(0, np.uint8), part_off=np.zeros(store.P + 1, np.int64), boxes=store.boxes)
    st, want, gst, got = _exchange(native, ctx, cfg, empty, synth.neighbour_table(cfg.grid), "empty", msgs=msgs)
    assert st == oracle.OK and gst == native.OK
    _compare_store("empty", got, want, nf, ni)
    ctx.close()


def test_capacity_reports_sizes(native):
    cfg, w = _world(seed=17)
    ctx = native.Context(cfg.schema)
    dest = synth.neighbour_table(cfg.grid)
    st, want, gst, got = _exchange(native, ctx, cfg, w.store, dest, "sizes")
    need = want["sizes"].copy()
    for cap, bcap in [(int(need[0]) - 1, int(need[1])), (int(need[0]), int(need[1]) - 8)]:
        st, want2, gst, got = _exchange(native, ctx, cfg, w.store, dest, "capacity", cap=cap, beh_cap=bcap)
        assert st == oracle.CAPACITY and gst == native.CAPACITY
        assert np.array_equal(_host(got["sizes"]), need)
        assert np.array_equal(_host(got["part_off"]), want["part_off"])
    ctx.close()


@pytest.mark.parametrize("case", ["magic", "dest", "class", "uid0", "offset"])
def test_invalid_inputs_match_oracle_status(native, case):
    cfg, w = _world(seed=19)
    ctx = native.Context(cfg.schema)
    store = w.store
    oidx, oso = oracle.select_migrants(store)
    msgs, moff = oracle.serialize(store, cfg.schema, oidx, oso)
    dest = synth.neighbour_table(cfg.grid).copy()
    s = int(np.flatnonzero(np.diff(oso) > 0)[0])
    a = int(moff[s])
    n = int(msgs[a + 8:a + 12].view(np.uint32)[0])
    rec0 = a + 32 + 8 * ((n + 1) // 2)
    m, mo = msgs.copy(), moff.copy()
    if case == "magic":
        m[a] ^= 1
    elif case == "dest":
        dest[s] = store.P
    elif case == "class":
        m[rec0 + 8:rec0 + 10] = np.frombuffer(np.uint16(7).tobytes(), np.uint8)
    elif case == "uid0":
        m[rec0:rec0 + 8] = 0
    elif case == "offset":
        mo[s + 1] += 4
    st, want, gst, got = _exchange(native, ctx, cfg, store, dest, case, msgs=(m, mo), cap=store.n + 64,
                                   beh_cap=store.beh.size + 4096)
    assert st == oracle.INVALID and gst == native.INVALID
    ctx.close()


def test_full_size_migration(native):
    """The bench's migration workload (1e7 agents in a 2x2x2 grid of 500 um
    boxes, walls at the domain only, one walk step): selection, messages and
    every column of the rebuilt store against the oracle."""
    cfg = synth.config(2, grid=(2, 2, 2), side=500.0, median=1e7 / 8, walls="domain")
    w = synth.World(cfg)
    w.step()
    ctx = native.Context(cfg.schema)
    st, want, gst, got = _exchange(native, ctx, cfg, w.store, synth.neighbour_table(cfg.grid), "full size")
    assert st == oracle.OK and gst == native.OK
    assert int(want["sizes"][0]) == w.store.n
    _compare_store("full size", got, want, *_cols(cfg))
    ctx.close()
