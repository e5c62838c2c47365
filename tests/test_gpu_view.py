"""GPU parity of the view checks (Sec. 2.2.1 "Deserialization": one pass over
the received buffer, no allocation).  ta_view (O(1): header and size
identity) and ta_view_validate (the full O(n) check) are compared with the
oracle's orc_view over a sweep of damaged messages: header bytes, counts,
lengths, offsets, the offset table's pad entry, record sizes and uids."""
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


def _u32(b, at):
    return int(np.frombuffer(b[at:at + 4].tobytes(), np.uint32)[0])


def _set32(b, at, v):
    b[at:at + 4] = np.frombuffer(np.uint32(v & 0xFFFFFFFF).tobytes(), np.uint8)


def _set64(b, at, v):
    b[at:at + 8] = np.frombuffer(np.uint64(v & 0xFFFFFFFFFFFFFFFF).tobytes(), np.uint8)


def damages(msg, rng):
    """(tag, damaged copy) pairs of one TAM1 message."""
    n = _u32(msg, 8)
    rw = int(np.frombuffer(msg[16:24].tobytes(), np.uint64)[0])
    area = 32 + 8 * ((n + 1) // 2)
    yield "intact", msg.copy()
    for at in range(32):
        d = msg.copy()
        d[at] = (int(d[at]) + 1) & 0xFF
        yield f"header byte {at}", d
    for dn in (-1, 1, 2):
        d = msg.copy()
        _set32(d, 8, n + dn)
        yield f"n{dn:+d}", d
    for dw in (-1, 1):
        d = msg.copy()
        _set64(d, 16, rw + dw)
        yield f"rec_words{dw:+d}", d
    yield "short", msg[:-8].copy()
    yield "long", np.concatenate([msg, np.zeros(8, np.uint8)])
    if n % 2:
        d = msg.copy()
        d[32 + 4 * n] = 1
        yield "table pad", d
    for i in sorted(rng.choice(n, size=min(n, 12), replace=False)):
        o = _u32(msg, 32 + 4 * i)
        for tag, v in (("+1", o + 1), ("-1", o - 1), ("zero", 0), ("huge", 0xFFFFFFFF), ("end", rw)):
            if v == o:
                continue
            d = msg.copy()
            _set32(d, 32 + 4 * i, v)
            yield f"offset {i} {tag}", d
    for i in sorted(rng.choice(n, size=min(n, 12), replace=False)):
        at = area + 8 * _u32(msg, 32 + 4 * i)
        words = _u32(msg, at + 12)
        for tag, v in (("+1", words + 1), ("-1", words - 1), ("zero", 0), ("one", 1), ("huge", 0xFFFFFFFF)):
            d = msg.copy()
            _set32(d, at + 12, v)
            yield f"record {i} words {tag}", d
        d = msg.copy()
        _set64(d, at, 0)
        yield f"record {i} uid zero", d
        d = msg.copy()
        d[at + 8] ^= 1  # class: not a view check
        yield f"record {i} class", d
        if words > 2:
            d = msg.copy()
            d[at + 16] ^= 0x40  # a field value
            yield f"record {i} field", d


def test_view_statuses_match_oracle(native):
    import torch
    cfg = synth.config(1, median=2000.0)
    world = synth.World(cfg)
    idx, seg = oracle.select_aura(world.store, cfg.w, cfg.ndirs)
    buf, moff = oracle.serialize(world.store, cfg.schema, idx, seg)
    n0 = int(seg[1] - seg[0])
    n_odd = n0 if n0 % 2 else n0 - 1
    n_even = n0 - 1 if n0 % 2 else n0
    odd, _ = oracle.serialize(world.store, cfg.schema, idx[:n_odd], np.array([0, n_odd]))
    even, _ = oracle.serialize(world.store, cfg.schema, idx[:n_even], np.array([0, n_even]))
    empty, _ = oracle.empty_messages(1)
    pick = [odd, even, empty]
    assert _u32(odd, 8) % 2 == 1 and _u32(even, 8) % 2 == 0 and _u32(even, 8) > 0
    ctx = native.Context(cfg.schema)
    rng = np.random.default_rng(7)
    counts = {0: 0, 1: 0}
    for k, msg in enumerate(pick):
        for tag, d in damages(msg, rng):
            print(f"[view] message {k} ({_u32(msg, 8)} records): {tag}", flush=True)
            want = oracle.view(d)[0]
            dev = torch.from_numpy(d).cuda()
            off = torch.tensor([0, d.size], dtype=torch.int64, device="cuda")
            ctx.validate(dev, off)
            full = ctx.poll()
            assert full == want, f"message {k} {tag}: validate {full}, oracle {want}"
            quick = []
            for hdr in (None, d[:32].tobytes() if d.size >= 32 else None):
                try:
                    v = ctx.view(dev, 0, d.size, header=hdr)
                    quick.append(native.OK)
                    assert v.n == _u32(d, 8) and v.records - dev.data_ptr() == 32 + 8 * ((v.n + 1) // 2)
                except native.TAError as e:
                    quick.append(e.code)
            assert quick[0] == quick[1], f"message {k} {tag}: header given or read differ"
            # the O(1) view's checks are a subset of the full check
            if quick[0] != native.OK:
                assert quick[0] == native.INVALID and want == oracle.INVALID, f"message {k} {tag}"
            if tag in ("short", "long") or (tag.startswith("header byte") and int(tag.split()[-1]) not in range(8, 12)):
                assert quick[0] == want, f"message {k} {tag}: view {quick[0]}, oracle {want}"
            counts[min(want, 1)] += 1
    assert counts[0] >= 20 and counts[1] >= 100, counts
    ctx.close()
