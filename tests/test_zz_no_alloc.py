"""The allocation-free selection entry point (ta_select_aura_static, scratch
in a static device array) against ta_select_aura on the same inputs: two
calls in a row, the second with a smaller store and fewer partitions, and the
host-side rejection of a store beyond the static array."""
import ctypes as C

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


def _both(native, ctx, store, cfg, tag):
    import torch
    ds = native.DeviceStore(store)
    cap = 26 * store.n + 64
    idx_a, seg_a = ctx.select_aura(ds, cfg.w, cfg.ndirs, idx_cap=cap)
    idx_b = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
    seg_b = torch.full((ds.P * cfg.ndirs + 1,), -7, dtype=torch.int64, device="cuda")
    print(f"[no-alloc] {tag}: {store.n} agents, {store.P} partitions, {cfg.ndirs} directions", flush=True)
    ctx.select_aura_static(ds, cfg.w, cfg.ndirs, idx_b, seg_b)
    ctx.check(tag)
    sa, sb = host(seg_a), host(seg_b)
    assert np.array_equal(sa, sb), tag
    S = int(sa[-1])
    assert np.array_equal(host(idx_a)[:S], host(idx_b)[:S]), tag
    oidx, oseg = oracle.select_aura(store, cfg.w, cfg.ndirs)
    assert np.array_equal(sb, oseg) and np.array_equal(host(idx_b)[:S], oidx), tag
    return S


def test_static_selection_matches_the_allocating_one(native):
    big = synth.config(3, median=20000.0, grid=(2, 2, 2))
    small = synth.config(1, median=3000.0)
    ctx = native.Context(big.schema)
    s1 = _both(native, ctx, synth.World(big).store, big, "first call, 8 partitions")
    s2 = _both(native, ctx, synth.World(small).store, small, "second call, smaller store")
    assert s1 > s2 > 0
    ctx.close()


def test_static_selection_rejects_stores_beyond_its_array(native):
    import torch
    n = (1 << 24) + (1 << 22)
    ctx = native.Context(synth.Schema((4,), (1,)))
    f64 = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    part_off = torch.tensor([0, n], dtype=torch.int64, device="cuda")
    boxes = torch.tensor([0, 0, 0, 1, 1, 1], dtype=torch.float64, device="cuda")
    idx = torch.empty(64, dtype=torch.int32, device="cuda")
    seg = torch.empty(27, dtype=torch.int64, device="cuda")
    ag = native.Agents(n, None, None, None, C.c_void_p(f64.data_ptr()), n, None, n, None, None)
    print(f"[no-alloc] {n} agents: rejected on the host", flush=True)
    st = native.lib().ta_select_aura_static(ctx.h, C.byref(ag), 1, C.c_void_p(part_off.data_ptr()),
                                            C.c_void_p(boxes.data_ptr()), 0.1, 26, C.c_void_p(idx.data_ptr()), 64,
                                            C.c_void_p(seg.data_ptr()), native._stream())
    assert st == native.CAPACITY
    assert ctx.poll() == native.OK
    ctx.close()
