"""GPU parity of record growth and compaction (Sec. 2.2.1, "Mutability")
through the C ABI: the whole buffer after growth (messages, redirected
offsets, arena), the arena use, compacted messages and their offsets, and
the statuses of bad lists, byte for byte against the oracle."""
import numpy as np
import pytest

import oracle
from tests.test_oracle_grow import _messages, _picks, _record, _with_arena

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_24063_amd import native as n
    n.lib()
    return n


def _dev(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a if dtype is None else np.asarray(a, dtype))
    if a.size == 0:
        a = np.zeros(1, a.dtype)
    return torch.from_numpy(a).cuda()


def _run_grow(native, ctx, buf, moff, seg, rec, words, used=0):
    """GPU growth of a copy of buf; returns (status, bytes, arena_used)."""
    import torch
    b = _dev(buf)
    au = torch.tensor([used], dtype=torch.int64, device="cuda")
    seg_t = _dev(np.asarray(seg, np.int32))
    rec_t = _dev(np.asarray(rec, np.uint32))
    words_t = _dev(np.asarray(words, np.uint32))
    mo = _dev(moff, np.int64)  # every argument tensor stays referenced until the call has run
    from paper_2509_24063_amd.native import lib, _p, _stream
    st = lib().ta_view_grow(ctx.h, _p(b), b.numel(), _p(mo), len(moff) - 1, _p(seg_t), _p(rec_t), _p(words_t),
                            len(seg), _p(au), _stream())
    assert st == 0
    status = ctx.poll()
    return status, b.cpu().numpy(), int(au.item())


def _run_compact(native, ctx, buf, moff, out_cap):
    import torch
    out = torch.zeros(max(out_cap, 8), dtype=torch.uint8, device="cuda")
    ooff = torch.zeros(len(moff), dtype=torch.int64, device="cuda")
    src, mo = _dev(buf), _dev(moff, np.int64)  # referenced until the call has run
    from paper_2509_24063_amd.native import lib, _p, _stream
    st = lib().ta_view_compact(ctx.h, _p(src), len(buf), _p(mo), len(moff) - 1, _p(out), out_cap, _p(ooff),
                               _stream())
    assert st == 0
    status = ctx.poll()
    o = ooff.cpu().numpy()
    return status, out.cpu().numpy()[: int(o[-1])] if status == 0 else None, o


def test_compact_canonical_is_identity(native):
    cfg, st, idx, so, buf, moff = _messages(seed=4)
    ctx = native.Context(cfg.schema)
    status, out, ooff = _run_compact(native, ctx, _with_arena(buf, 4096), moff, len(buf))
    assert status == native.OK and np.array_equal(ooff, moff) and np.array_equal(out, buf)
    ctx.close()


@pytest.mark.parametrize("count,rounds", [(40, 1), (300, 1), (12, 3)])
def test_grow_and_compact_match_oracle(native, count, rounds):
    cfg, st, idx, so, buf, moff = _messages(seed=6, n=3000)
    ctx = native.Context(cfg.schema)
    rng = np.random.default_rng(count)
    picks = _picks(so, rng, count)
    b_o = _with_arena(buf, 1 << 18)
    b_g = b_o.copy()
    used_o = used_g = 0
    for step in range(rounds):
        print(f"[grow] {count} records, round {step}", flush=True)
        words = [len(_record(b_o, moff, s, r)) + int(rng.integers(0, 5)) for s, r in picks]
        seg, rec = [p[0] for p in picks], [p[1] for p in picks]
        so_, used_o = oracle.view_grow(b_o, moff, seg, rec, words, used_o)
        assert so_ == oracle.OK
        status, b_g, used_g = _run_grow(native, ctx, b_g, moff, seg, rec, words, used_g)
        assert status == native.OK and used_g == used_o
        assert np.array_equal(b_g, b_o)
    so_, want, woff = oracle.view_compact(b_o, moff)
    status, got, goff = _run_compact(native, ctx, b_g, moff, int(woff[-1]))
    assert so_ == oracle.OK and status == native.OK
    assert np.array_equal(goff, woff) and np.array_equal(got, want)
    # too little room for the compacted messages: offsets still reported
    status, _, goff = _run_compact(native, ctx, b_g, moff, int(woff[-1]) - 8)
    assert status == native.CAPACITY and np.array_equal(goff, woff)
    ctx.close()


@pytest.mark.parametrize("case", ["order", "smaller", "seg", "rec", "capacity", "arena_free"])
def test_grow_errors_match_oracle(native, case):
    cfg, st, idx, so, buf, moff = _messages(seed=10)
    ctx = native.Context(cfg.schema)
    rng = np.random.default_rng(3)
    picks = _picks(so, rng, 3)
    seg = [p[0] for p in picks]
    rec = [p[1] for p in picks]
    words = [len(_record(buf, moff, s, r)) + 1 for s, r in picks]
    b = _with_arena(buf, 4096)
    if case == "order":
        seg, rec, words = seg[::-1], rec[::-1], words[::-1]
    elif case == "smaller":
        words[1] -= 2
    elif case == "seg":
        seg[2] = len(so) - 1
    elif case == "rec":
        rec[2] = int(so[seg[2] + 1] - so[seg[2]])
    elif case == "capacity":
        b = _with_arena(buf, 8)
    elif case == "arena_free":
        s, r = picks[0]
        a = int(moff[s])
        n = int(b[a + 8:a + 12].view(np.uint32)[0])
        recs = a + 32 + 8 * ((n + 1) // 2)
        b[a + 32 + 4 * r:a + 36 + 4 * r] = np.frombuffer(np.uint32((buf.shape[0] - recs) // 8).tobytes(), np.uint8)
    b_o = b.copy()
    so_, used_o = oracle.view_grow(b_o, moff, seg, rec, words, 0)
    status, b_g, used_g = _run_grow(native, ctx, b, moff, seg, rec, words, 0)
    want = oracle.CAPACITY if case == "capacity" else oracle.INVALID
    assert so_ == want and status == want
    assert np.array_equal(b_g, b) and used_g == 0
    ctx.close()
