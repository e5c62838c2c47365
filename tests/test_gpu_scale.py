"""The large batched workloads at their own scale against the oracle: 512
partitions of about 1.7e8 sphere agents (plain delta), and 256 partitions
of 2e8 heterogeneous agents (80/20 spheres and cylinders, 14 fp64 fields,
0-4 behaviours of 1-7 words, learned predictor), their states generated and
advanced on the GPU.  Every iteration runs as one graph replay over all
partitions, the receiver sharing the sender's reference copy; one sampled
partition's 26 segments (messages, encodings, modes, the sender's and the
receiver's C') are compared byte for byte with the oracle's exchange of that
partition, which keeps its own reference and history chain.

Minutes of GPU time and up to about 250 GB of device memory each: they run
only with TA_SCALE_TESTS=1 (e.g. TA_SCALE_TESTS=1 pytest -m gpu
tests/test_gpu_scale.py); TA_SCALE_AGENTS scales the median partition size
down, TA_SCALE_ITERATIONS sets the iterations (default 20)."""
import os

import numpy as np
import pytest

import oracle
from paper_2509_24063_amd import synth
from tests.exchange_util import OracleLearnedSide, OracleSide
from tests.test_oracle_predictor import copy_last_move_blob

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(os.environ.get("TA_SCALE_TESTS") != "1",
                                 reason="large-scale runs: set TA_SCALE_TESTS=1")]


@pytest.fixture(scope="module")
def native():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_24063_amd import native as n
    n.lib()
    return n


def _segments(buf, off, s0, s1):
    from paper_2509_24063_amd.exchange import segment_bytes
    return segment_bytes(buf, off, s0, s1)


@pytest.mark.parametrize("index", [3, 5])
def test_sampled_partition_every_iteration(native, index):
    import torch
    from paper_2509_24063_amd.exchange import sized_pipeline
    from paper_2509_24063_amd.synth_device import DeviceWorld, partition_sizes
    over = {"median": float(os.environ["TA_SCALE_AGENTS"])} if os.environ.get("TA_SCALE_AGENTS") else {}
    cfg = synth.config(index, **over)
    iterations = int(os.environ.get("TA_SCALE_ITERATIONS", "20"))
    cap, beh_cap = DeviceWorld.capacity(cfg, iterations + 1)
    counts, boxes = partition_sizes(cfg)
    ds = native.DeviceStore.alloc(max(cfg.n_f64), max(cfg.n_i32), boxes, cap, beh_cap)
    world = DeviceWorld(cfg, ds, log=lambda m: print(m, flush=True))
    P = world.P
    sample = int(np.argsort(counts)[P // 2])  # the median-sized partition
    ctx = native.Context(cfg.schema)
    learned = index == 5
    blob = copy_last_move_blob() if learned else None
    pred = native.Predictor(ctx, blob) if learned else None
    pl = sized_pipeline(ctx, ds, cfg.ndirs, cfg.w, cap / world.n, pred)
    pl.capture()
    orc = OracleLearnedSide(cfg.ndirs, oracle.mlp_struct(blob)) if learned else OracleSide(cfg.ndirs)
    s0, s1 = cfg.ndirs * sample, cfg.ndirs * (sample + 1)
    modes_seen = np.zeros(3, np.int64)
    for t in range(iterations):
        print(f"[scale cfg{index}] iteration {t}: {world.n} agents, sampled partition {sample}", flush=True)
        pl.step(graph=True)
        ctx.check(f"iteration {t}")
        o = orc.step(world.partition_host(sample), cfg)
        enc, eoff, nref, noff, rx, rxoff = pl.outputs()
        for (buf, off), (want, want_off), what in (
                ((enc, eoff), (o["enc"], o["eoff"]), "encodings"),
                ((nref, noff), (o["nref"], o["noff"]), "sender C'"),
                ((rx, rxoff), (o["nref"], o["noff"]), "receiver C'")):
            got, got_off = _segments(buf, off, s0, s1)
            assert np.array_equal(got_off, want_off), f"iteration {t}: {what} offsets"
            assert np.array_equal(got, want), f"iteration {t}: {what}"
        if learned:
            m = pl.modes[s0:s1].cpu().numpy()
            assert np.array_equal(m, o["modes"]), f"iteration {t}: modes"
            modes_seen += np.bincount(m, minlength=3)
        world.step()
    if learned:
        assert modes_seen[1:].sum() > 0  # the predictor was chosen somewhere in the sampled partition
    pl.close()
    ctx.close()
