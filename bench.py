"""Benchmark of the aura exchange on one MI355X.

Default workload: one step is one whole exchange of one iteration of the
1e7-agent world (1000^3 um box, 26 neighbour auras, spheres with 0..2
behaviours, Gaussian walk with division and death): aura selection,
serialization of all 26 messages, delta encoding against the previous
iteration's messages and decoding on the receive side.  Inputs are generated
up front (seeded, synthetic) and resident in HBM when the timed region
starts; the reference of step k is the C' of step k-1, exactly as in a
running simulation.  The steps are timed twice, as batched iteration calls
and as replays of one captured HIP graph per iteration; `value` comes from
the faster mode (named in `timed_mode`).

`--workload batched`: 512 partitions of uneven (lognormal) size in an 8x8x8
periodic grid, 26 segments each; the same iteration timed as batched calls,
as graph replays, and (--per-partition) as one set of calls per partition.

Prints one JSON line.  `value` is aura records (one agent sent to one
neighbour direction) exchanged per second over the whole step.  Also
reported:
- `steps_ms_GBps`: ms per step and algorithmic GB/s of select, serialize,
  match, xor_pack and decode, from one pass with events at the step
  boundaries and around the encoder's match kernels only;
- `serialize_delta`: serialize + delta-encode on their own (algorithmic
  bytes, fraction of the 8 TB/s HBM peak and of `copy_peak_GBps`, the rate
  of a plain device copy timed in the same run);
- `roofline` / `rooflines`: the measured kernel families' launches (HIP
  events on the library's stream around every launch), their algorithmic
  bytes and fractions of both peaks;
- `learned`: the same steps in learned mode (predictor trained on the GPU):
  ms per step, stage times, serialize + delta GB/s, the learned kernels;
- encoded bytes per record in plain and learned mode, the eager steps again
  with the byte-wise subtraction operator, growth and compaction, agent
  migration;
- `cpu_baseline`: the CPU oracle on a bounded sample of the same workload,
  on one host thread and with its one-message calls spread over the host
  threads, with the CPU model.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# timing families that span several kernels (the join: count, scan, scatter, bucket; the prediction:
# neighbour table and network): reported in `rooflines`, never as the one kernel of `roofline`
MULTI_KERNEL_FAMILIES = ("encode_join", "predict")
METRIC = "agents/s and GB/s (frac of HBM peak) serialize+delta; encoded bytes/agent learned vs plain"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["single", "batched", "batched-full", "hetero"], default="single",
                    help="single: 1e7 agents, one box; batched: 512 uneven partitions from host-generated states "
                         "(--agents scales them down); batched-full and hetero: 512 partitions of 1.7e8 agents and "
                         "256 partitions of 2e8 heterogeneous agents (learned), states advanced on the GPU, one "
                         "graph per iteration")
    ap.add_argument("--agents", type=float, default=None, help="agents (single) or median per partition (batched)")
    ap.add_argument("--roofline-kernels", default="encode_groups,decode_unpack,serialize_pack,select_count,encode_join",
                    help="kernel families timed with HIP events; the one with the largest time is `roofline`")
    ap.add_argument("--copy-peak-mib", type=float, default=1024.0, help="size of the copies timed for copy_peak_GBps")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="bound of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-migration", action="store_true", help="skip the agent-migration measurement")
    ap.add_argument("--migration-only", action="store_true",
                    help="only the agent-migration measurement (for profiling); prints its JSON object")
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--per-partition", action="store_true", help="batched: also time per-partition calls")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="MiB copied once by a plain device copy (reference for HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def generate(world, nstates, native):
    t0 = time.time()
    host_states, dev_states = [], []
    for k in range(nstates):
        host_states.append(world.store)
        dev_states.append(native.DeviceStore(world.store))
        world.step()
        log(f"generated state {k + 1}/{nstates} ({world.store.n} agents, {time.time() - t0:.0f}s)")
    return host_states, dev_states


def eager_pass(ctx, native, cfg, dev_states, host_states, warmup, idx_cap, ser_cap, enc_cap, kernels, pred=None):
    """Every step through the single calls, with events at the stage
    boundaries only (before select, serialize and encode, after encode and
    after decode) and the library's events around the kernel families named
    in `kernels` (comma-separated); the byte accounting of a step is read
    back after it, outside the events.  With `pred`, learned mode on both
    sides (the predictor history carried along)."""
    import numpy as np
    import torch
    nstates = len(dev_states)
    nseg = dev_states[0].P * cfg.ndirs
    dev = torch.device("cuda")
    u8 = dict(dtype=torch.uint8, device=dev)
    i64 = dict(dtype=torch.int64, device=dev)
    idx = torch.empty(idx_cap, dtype=torch.int32, device=dev)
    seg = torch.empty(nseg + 1, **i64)
    buf, moff = torch.empty(ser_cap, **u8), torch.empty(nseg + 1, **i64)
    enc, eoff = torch.empty(enc_cap, **u8), torch.empty(nseg + 1, **i64)
    refs = [torch.empty(ser_cap, **u8) for _ in range(2)]
    roffs = [torch.empty(nseg + 1, **i64) for _ in range(2)]
    rx = [torch.empty(ser_cap, **u8) for _ in range(2)]
    rxoffs = [torch.empty(nseg + 1, **i64) for _ in range(2)]
    hc = idx_cap if pred is not None else 0
    hist = [native.History(hc) for _ in range(2)]
    # record keys beside every message set (as the pipelines keep them)
    zk = lambda: torch.zeros(2 * idx_cap, dtype=torch.int64, device=dev)  # noqa: E731
    mkeys, rkeys, xkeys = zk(), [zk(), zk()], [zk(), zk()]
    rxhist = [native.History(hc) for _ in range(2)]
    modes = torch.empty(nseg, **u8)
    e0, e1 = native.empty_messages(nseg)
    refs[1][: e0.numel()].copy_(e0)
    roffs[1].copy_(e1)
    rx[1][: e0.numel()].copy_(e0)
    rxoffs[1].copy_(e1)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    spin = spin_cycles(3.0)
    acc = dict(records=0, ser=0, enc=0, match=0, dec=0, sel=0, W=0, var=0, matched=0, groups=0, tad=0, msg=0,
               sd_ms=0.0, step_ms=0.0, select_ms=0.0, serialize_ms=0.0, encode_ms=0.0, decode_ms=0.0,
               learned_segments=0)
    prev_msg, prev_S = 32 * nseg, 0
    for k in range(nstates):
        if k == warmup:
            ctx.check("eager warmup")
            ctx.time_kernel(kernels)
        ds = dev_states[k]
        cur_ref, nxt = (k + 1) % 2, k % 2
        lp = dict(pred=pred, hist=hist[cur_ref], hist_out=hist[nxt]) if pred is not None else {}
        lr = dict(pred=pred, hist=rxhist[cur_ref], hist_out=rxhist[nxt]) if pred is not None else {}
        # the GPU spins while the host enqueues the step, so that the events
        # time the kernels back to back, not the enqueue
        torch.cuda._sleep(spin)
        ev[0].record()
        ctx.select_aura(ds, cfg.w, cfg.ndirs, idx_cap=idx_cap, out=(idx, seg))
        ev[1].record()
        ctx.serialize(ds, idx, seg, idx_cap=idx_cap, out=(buf, moff), keys=mkeys)
        ev[2].record()
        ctx.delta_encode(buf, moff, refs[cur_ref], roffs[cur_ref], out=(enc, eoff, refs[nxt], roffs[nxt], modes),
                         keys=(mkeys, rkeys[cur_ref], rkeys[nxt]), **lp)
        ev[3].record()
        ctx.delta_decode(enc, eoff, rx[cur_ref], rxoffs[cur_ref], out=(rx[nxt], rxoffs[nxt]),
                         keys=(xkeys[cur_ref], xkeys[nxt]), **lr)
        ev[4].record()
        torch.cuda.synchronize()
        mo = moff.cpu().numpy()
        M = int(mo[-1])
        S = int(seg[-1].item())
        if k >= warmup:
            eo = eoff.cpu().numpy()
            T = int(eo[-1])
            hdr = enc[:T].cpu().numpy()
            heads = np.stack([np.frombuffer(hdr[eo[q]:eo[q] + 64].tobytes(), np.uint64) for q in range(nseg)])
            acc["records"] += S
            acc["W"] += int(heads[:, 5].sum())
            acc["var"] += int(heads[:, 7].sum())
            acc["matched"] += int((heads[:, 1] >> np.uint64(32)).sum())
            acc["groups"] += int(((heads[:, 5] + np.uint64(63)) // np.uint64(64)).sum())
            acc["learned_segments"] += int(np.count_nonzero(modes[:nseg].cpu().numpy()))
            acc["tad"] += T
            acc["msg"] += M
            R = prev_msg  # the reference is the previous step's C', the size of that step's messages
            acc["sel"] += 24 * host_states[k].n + 4 * S
            # serialize: indices, behaviour offsets, gathered source fields (about the record bytes), records + offsets
            acc["ser"] += 4 * S + 16 * S + M + M
            # match: a 16-byte (uid, item) entry built per reference record and probed per current record
            acc["match"] += 16 * (S + prev_S)
            # residual and packing: read C and R, write the encoding and C'
            acc["enc"] += M + R + T + M
            # decode: read the encoding and R, write C'
            acc["dec"] += T + R + M
            acc["select_ms"] += ev[0].elapsed_time(ev[1])
            acc["serialize_ms"] += ev[1].elapsed_time(ev[2])
            acc["encode_ms"] += ev[2].elapsed_time(ev[3])
            acc["decode_ms"] += ev[3].elapsed_time(ev[4])
            acc["sd_ms"] += ev[1].elapsed_time(ev[3])
            acc["step_ms"] += ev[0].elapsed_time(ev[4])
        prev_msg, prev_S = M, S
    fam = {}
    for name in [x for x in kernels.split(",") if x]:
        fam[name] = ctx.kernel_time(name)
    ctx.time_kernel(None)
    ctx.check("eager steps")
    last = (nstates - 1) % 2
    n_last = int(roffs[last][-1])
    assert torch.equal(rxoffs[last], roffs[last]) and torch.equal(rx[last][:n_last], refs[last][:n_last]), \
        "receiver C' differs from sender C'"
    final = dict(nref=refs[last][:n_last].clone(), noff=roffs[last].clone(), eoff=eoff.clone())
    return acc, fam, final


def graph_pass(ctx, native, cfg, dev_states, warmup, idx_cap, ser_cap, pred=None, hist_cap=None):
    """One captured graph per step (ping-pong references); the timed steps
    are graph launches only.  Returns (elapsed of the timed steps, pipeline)."""
    import torch
    from paper_2509_24063_amd.exchange import Pipeline
    pl = Pipeline(ctx, dev_states[0], cfg.w, cfg.ndirs, idx_cap, ser_cap, pred=pred)
    graphs = [native.Graph(ctx, pl.iteration(k % 2, ds)) for k, ds in enumerate(dev_states)]
    for k in range(warmup):
        graphs[k].launch()
    ctx.check("graph warmup")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(warmup, len(dev_states)):
        graphs[k].launch()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    ctx.check("graph steps")
    pl.ran(len(dev_states))
    for g in graphs:
        g.close()
    return elapsed, pl


def eager_timed_pass(ctx, native, cfg, dev_states, warmup, idx_cap, ser_cap, pred=None):
    """Every step as one batched iteration call (no host synchronisation
    between steps); wall clock over the timed steps."""
    import torch
    from paper_2509_24063_amd.exchange import Pipeline
    pl = Pipeline(ctx, dev_states[0], cfg.w, cfg.ndirs, idx_cap, ser_cap, pred=pred)
    its = [pl.iteration(k % 2, ds) for k, ds in enumerate(dev_states)]
    for k in range(warmup):
        ctx.run_iteration(its[k])
    ctx.check("eager timed warmup")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(warmup, len(dev_states)):
        ctx.run_iteration(its[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    ctx.check("eager timed steps")
    pl.ran(len(dev_states))
    return elapsed, pl


def overlap_pass(ctx, native, cfg, dev_states, warmup, idx_cap, ser_cap):
    """The exchange as a three-stage pipeline on three streams, a context each
    (OverlapPipeline): selection and serialization of iteration t + 1,
    encoding of t and decoding of t - 1 at the same time.  Same work per step
    as the other modes."""
    import torch
    from paper_2509_24063_amd.exchange import OverlapPipeline
    pl = OverlapPipeline(cfg.schema, dev_states[0], cfg.w, cfg.ndirs, idx_cap, ser_cap)
    pl.reserve(max(s.n for s in dev_states))
    # the stages' streams chosen by timing a few short trials (untimed here)
    pl.tune_streams(dev_states[:8])
    for k in range(warmup):
        pl.step(dev_states[k])
    pl.check("overlap warm-up")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(warmup, len(dev_states)):
        pl.step(dev_states[k])
    pl.join()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    pl.check("overlap steps")
    return elapsed, pl


def spin_cycles(ms):
    """The argument of torch.cuda._sleep that keeps the GPU busy for about
    `ms` milliseconds (calibrated once against events)."""
    import torch
    global _SPIN_PER_MS
    if _SPIN_PER_MS is None:
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda._sleep(1 << 20)
        ev[0].record()
        torch.cuda._sleep(1 << 22)
        ev[1].record()
        torch.cuda.synchronize()
        _SPIN_PER_MS = (1 << 22) / max(ev[0].elapsed_time(ev[1]), 1e-3)
    return int(_SPIN_PER_MS * ms)


_SPIN_PER_MS = None


def copy_peak(mib):
    """Device-to-device copy rate (read + write bytes per second) of a plain
    torch copy of `mib` MiB, the best of five."""
    import torch
    nb = int(mib * (1 << 20))
    src = torch.ones(nb, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    best = float("inf")
    for _ in range(5):
        ev[0].record()
        dst.copy_(src)
        ev[1].record()
        torch.cuda.synchronize()
        best = min(best, ev[0].elapsed_time(ev[1]))
    del src, dst
    return 2 * nb / (best / 1000.0) / 1e9


def stage_times(acc, fam, K):
    """ms per step and algorithmic GB/s of the five steps of an exchange."""
    m_launch, m_ms = fam.get("encode_match", (0, 0.0))
    match_ms = m_ms
    parts = {
        "select": (acc["select_ms"], acc["sel"]),
        "serialize": (acc["serialize_ms"], acc["ser"]),
        "match": (match_ms, acc["match"]),
        "xor_pack": (acc["encode_ms"] - match_ms, acc["enc"]),
        "decode": (acc["decode_ms"], acc["dec"]),
    }
    return {k: {"ms_per_step": ms / K, "GBps_algorithmic": b / (ms / 1000.0) / 1e9 if ms > 0 else None,
                "frac_hbm_peak": b / (ms / 1000.0) / 1e9 / HBM_PEAK_GBPS if ms > 0 else None}
            for k, (ms, b) in parts.items()}


def kernel_bytes(kname, acc):
    """Algorithmic bytes of one kernel family over the timed steps."""
    return {
        # plain mode: read C and R words of matched records and their starts and C/R words, write C' words,
        # the group blocks, bitmaps, sizes and offsets; read the group-to-segment and first-record maps
        "encode_groups": 24 * acc["W"] + 24 * acc["matched"] + acc["var"] + 25 * acc["groups"],
        # learned mode: the same, plus per matched record its four predicted words and flag, per group its
        # choice byte
        "encode_groups_learned": 24 * acc["W"] + 57 * acc["matched"] + acc["var"] + 26 * acc["groups"],
        # read the group blocks and their tables, R words and directory entries, write C' words
        "decode_unpack": 16 * acc["W"] + acc["var"] + 17 * acc["groups"] + 40 * acc["matched"],
        # gather the agents' fields (about the record bytes), indices, offsets; write records + offsets
        "serialize_pack": 2 * acc["msg"] + 32 * acc["records"],
        # read x, y, z of every agent, write one code byte per agent
        "select_count": acc["sel"] - 4 * acc["records"] + (acc["sel"] - 4 * acc["records"]) // 24,
        # the join's 16-byte entries, built and probed
        "encode_join": acc["match"],
    }.get(kname, float("nan"))


def roofline_entry(kname, launches, kernel_ms, total_bytes, copy_gbps, traffic):
    avg_ms = kernel_ms / max(launches, 1)
    kb = total_bytes / max(launches, 1)
    achieved = kb / (avg_ms / 1000.0) / 1e9 if avg_ms > 0 else 0.0
    return {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS, "frac_copy_peak": achieved / copy_gbps, "traffic": traffic,
            "launches": launches, "avg_ms": avg_ms, "algorithmic_bytes_per_launch": kb}


def same_as_final(pl, final, mode):
    """A timed mode's last iteration: its encoding offsets, the sender's C'
    and the receiver's C' equal the stage pass's."""
    import torch
    _, eoff, nref, noff, rx, rxoff = pl.outputs()
    n = int(final["noff"][-1])
    assert torch.equal(eoff, final["eoff"]), f"{mode} pass: encoding sizes differ from the stage pass"
    assert torch.equal(noff, final["noff"]) and torch.equal(nref[:n], final["nref"]), \
        f"{mode} pass: sender C' differs from the stage pass"
    if rx is not None:
        assert torch.equal(rxoff, final["noff"]) and torch.equal(rx[:n], final["nref"]), \
            f"{mode} pass: receiver C' differs from the stage pass"


def learned_mode(ctx, native, cfg, dev_states, host_states, args, idx_cap, ser_cap, enc_cap, pred, copy_gbps):
    """The same steps in learned mode: wall clock of the batched iteration
    calls, stage times and serialize + delta GB/s (same byte formula as plain
    mode), the learned kernels' times, and encoded bytes per record."""
    K = args.steps
    kern = "encode_match,predict,encode_groups,decode_unpack"
    acc, fam, final = eager_pass(ctx, native, cfg, dev_states, host_states, args.warmup, idx_cap, ser_cap, enc_cap,
                                 kern, pred=pred)
    el, pl = eager_timed_pass(ctx, native, cfg, dev_states, args.warmup, idx_cap, ser_cap, pred=pred)
    same_as_final(pl, final, "learned")
    pl.close()
    del pl
    sd_bytes = acc["ser"] + acc["match"] + acc["enc"]
    sd_gbps = sd_bytes / (acc["sd_ms"] / 1000.0) / 1e9
    return {
        "ms_per_step": 1000.0 * el / K,
        "steps_ms_GBps": stage_times(acc, fam, K),
        "serialize_delta": {"ms_per_step": acc["sd_ms"] / K, "GBps_algorithmic": sd_gbps,
                            "frac_hbm_peak": sd_gbps / HBM_PEAK_GBPS, "frac_copy_peak": sd_gbps / copy_gbps},
        "kernels_us_per_step": {k: 1000.0 * ms / K for k, (n, ms) in fam.items()},
        "rooflines": [roofline_entry(k, n, ms, kernel_bytes(k + "_learned" if k == "encode_groups" else k, acc),
                                     copy_gbps, None)
                      for k, (n, ms) in fam.items() if k in ("encode_groups", "decode_unpack")],
        "bytes_per_agent": acc["tad"] / acc["records"],
        "learned_segments": acc["learned_segments"],
    }


def train_predictor(native, synth, log_fn, which=("random_walk", "persistent")):
    """Predictor trained on the GPU on windows of the 1e5-agent, 13-iteration
    world (200^3 um box, 6 faces), like the exchange's own history."""
    from paper_2509_24063_amd import train
    tctx = native.Context(synth.Schema((4,), (1,)))
    out = {}
    for name, persistent in [x for x in (("random_walk", False), ("persistent", True)) if x[0] in which]:
        world = synth.World(synth.config(4, persistent=persistent))
        x, t = train.harvest(tctx, world, iterations=13, cap=2_000_000)
        losses = []
        blob = train.fit(tctx, x, t, steps=1500, log=losses.append)
        out[name] = (blob, int(x.shape[0]), losses[-1] if losses else "")
        log_fn(f"trained predictor on {x.shape[0]} windows ({name}): {out[name][2]}")
    tctx.close()
    return out


def persistent_variant(native, synth, blob, agents=1e6, iterations=8, skip=3):
    """Plain vs learned bytes per record on the persistent-motion world
    (velocity 0.9 v + N(0, 0.1) um, diameter +0.01 um per iteration), 26 auras."""
    from paper_2509_24063_amd.exchange import Pipeline, capacities
    cfg = synth.config(2, median=agents, persistent=True, seed=13)
    world = synth.World(cfg)
    ctx = native.Context(cfg.schema)
    pred = native.Predictor(ctx, blob)
    idx_cap, ser_cap = capacities(ctx, world.store, cfg.ndirs, cfg.w, slack=1.3)
    pls = {k: Pipeline(ctx, native.DeviceStore(world.store), cfg.w, cfg.ndirs, idx_cap, ser_cap,
                       pred=pred if k == "learned" else None, decode=False) for k in ("plain", "learned")}
    tot = {"plain": 0, "learned": 0}
    records = 0
    for it in range(iterations):
        ds = native.DeviceStore(world.store)
        for k, pl in pls.items():
            pl.step(ds)
            if it >= skip:
                tot[k] += int(pl.enc_off[-1].item())
        if it >= skip:
            records += int(pls["plain"].seg_off[-1].item())
        world.step()
    ctx.check("persistent variant")
    ctx.close()
    return {"agents": int(agents), "records": records, "plain": tot["plain"] / records,
            "learned": tot["learned"] / records, "ratio": tot["learned"] / tot["plain"]}


def per_partition_pass(native, cfg, host_states, warmup):
    """The same iterations as one set of calls per partition (26 segments
    each), every call prepared before the timed region."""
    import torch
    from paper_2509_24063_amd.exchange import Pipeline, capacities
    P = host_states[0].P
    ctx = native.Context(cfg.schema)
    parts = [[native.DeviceStore(s.partition(p)) for p in range(P)] for s in host_states]
    pls = []
    for p in range(P):
        idx_cap, ser_cap = capacities(ctx, host_states[0].partition(p), cfg.ndirs, cfg.w, slack=1.3)
        pls.append(Pipeline(ctx, parts[0][p], cfg.w, cfg.ndirs, idx_cap, ser_cap))
    its = [[pls[p].iteration(k % 2, parts[k][p]) for p in range(P)] for k in range(len(host_states))]
    run = native.lib().ta_iteration_run
    h = ctx.h
    import ctypes as C
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for k in range(warmup):
        for it in its[k]:
            run(h, C.byref(it.s), stream)
    ctx.check("per-partition warmup")
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(warmup, len(host_states)):
        for it in its[k]:
            run(h, C.byref(it.s), stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    ctx.check("per-partition steps")
    ctx.close()
    return elapsed


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures the exchange on one GPU only (asked for {args.gpus})", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2509_24063_amd import native, synth

    torch.cuda.set_device(0)
    if args.workload in ("batched-full", "hetero"):
        print(json.dumps(scale_pass(args, native, synth)), flush=True)
        return
    if args.migration_only:
        print(json.dumps({"migration": migration_pass(native, synth, args.warmup, args.steps)}), flush=True)
        return
    batched = args.workload == "batched"
    if batched:
        cfg = synth.config(3, **({"median": args.agents} if args.agents else {}))
    else:
        cfg = synth.config(2, median=args.agents or 1e7)
    nstates = args.warmup + args.steps
    world = synth.World(cfg)
    host_states, dev_states = generate(world, nstates, native)
    P = host_states[0].P
    nseg = P * cfg.ndirs
    n_agents = host_states[0].n

    if args.copy_probe > 0:
        nb = int(args.copy_probe * (1 << 20))
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {nb} bytes")
        del src, dst
    ctx = native.Context(cfg.schema)
    from paper_2509_24063_amd.exchange import capacities
    idx_cap, ser_cap = capacities(ctx, host_states[0], cfg.ndirs, cfg.w, slack=1.3)
    enc_cap = int(native.lib().ta_delta_bound(nseg, ser_cap, ser_cap))
    ctx.reserve(max(s.n for s in dev_states), nseg, idx_cap, ser_cap)

    tuned = None
    if not args.no_tune:
        from paper_2509_24063_amd.exchange import Pipeline
        pl = Pipeline(ctx, dev_states[0], cfg.w, cfg.ndirs, idx_cap, ser_cap)
        pl.step()  # a non-empty reference for the tuned iteration
        from_cache = ctx.tune(pl.iteration(1, dev_states[1]), args.tune_cache, reps=3)
        tuned = {"grids": dict(zip(["select", "serialize", "encode", "decode"], ctx.grids())),
                 "from_cache": from_cache}
        log(f"tuned launch grids {tuned}")
        pl.close()
        del pl

    copy_gbps = copy_peak(args.copy_peak_mib)
    log(f"device copy peak: {copy_gbps:.0f} GB/s ({args.copy_peak_mib} MiB copies)")

    # stage pass: events at the step boundaries and around the encoder's match part only
    acc, fam, final = eager_pass(ctx, native, cfg, dev_states, host_states, args.warmup, idx_cap, ser_cap, enc_cap,
                                 "encode_match")
    K = args.steps
    stages = stage_times(acc, fam, K)
    log("stage pass: " + ", ".join(f"{k} {v['ms_per_step']:.3f} ms" for k, v in stages.items()))
    # kernel pass: the library's events around every launch of the measured kernel families
    kernels = [k for k in args.roofline_kernels.split(",") if k]
    acc_k, ktimes, final_k = eager_pass(ctx, native, cfg, dev_states, host_states, args.warmup, idx_cap, ser_cap,
                                        enc_cap, ",".join(kernels))
    assert torch.equal(final_k["noff"], final["noff"]) and torch.equal(final_k["nref"], final["nref"])
    for kname, (launches, kernel_ms) in ktimes.items():
        log(f"kernel pass: {kname}: {kernel_ms / max(launches, 1) * 1000:.1f} us per launch")
    timings = {}
    modes = [("eager", eager_timed_pass), ("graph", graph_pass)]
    if not batched:  # three more contexts' scratch would not fit beside the batched states
        modes.append(("overlap", overlap_pass))
    for mode, fn in modes:
        el, pl = fn(ctx, native, cfg, dev_states, args.warmup, idx_cap, ser_cap)
        same_as_final(pl, final, mode)
        pl.close()
        del pl
        timings[mode] = el
        log(f"{mode} pass: {1000 * el / args.steps:.3f} ms/step")
    # the same eager steps with the byte-wise subtraction operator (not a candidate for `value`)
    ctx.set_difference_op(1)
    el, pl = eager_timed_pass(ctx, native, cfg, dev_states, args.warmup, idx_cap, ser_cap)
    same_as_final(pl, final, "subtraction")
    pl.close()
    del pl
    ctx.set_difference_op(0)
    subtraction_s = el
    log(f"eager pass, subtraction operator: {1000 * el / args.steps:.3f} ms/step")
    mode = min(timings, key=timings.get)
    best_s = timings[mode]

    records = acc["records"]
    value = records / best_s
    sd_bytes = acc["ser"] + acc["match"] + acc["enc"]
    sd_gbps = sd_bytes / (acc["sd_ms"] / 1000.0) / 1e9
    rooflines = []
    for kname, (launches, kernel_ms) in ktimes.items():
        rooflines.append(roofline_entry(kname, launches, kernel_ms, kernel_bytes(kname, acc_k), copy_gbps,
                                        measured_traffic(kname, f"{args.workload}:{n_agents}")))
    # the dominant kernel: the largest time per step
    rooflines.sort(key=lambda r: -r["avg_ms"] * r["launches"])
    if batched:
        workload = (f"{P} partitions (8x8x8 periodic, lognormal sizes, median {int(cfg.median)}), "
                    f"{n_agents} sphere agents, 26 auras each ({nseg} segments); select + serialize + "
                    "UID-matched XOR delta + zero-block pack + decode, one graph per iteration")
    else:
        workload = (f"{n_agents:.0e} sphere agents in a 1000^3 um box, 26 neighbour auras, 0-2 behaviours of 16 B, "
                    "Gaussian walk sigma 0.1 um, 1% division, 0.5% death; select + serialize + "
                    "UID-matched XOR delta + zero-block pack + decode")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "aura records/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * best_s / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded generator; the paper's BioDynaMo models are not available)",
        "config": {
            "workload": workload,
            "agents": int(n_agents),
            "partitions": P,
            "records_per_step": records // K,
            "record": "one agent sent to one neighbour direction (an agent near an edge or corner is sent "
                      "to several)",
            "segments": nseg,
        },
        "timed_mode": mode,
        "eager_ms_per_step": 1000.0 * timings["eager"] / K,
        "subtraction_eager_ms_per_step": 1000.0 * subtraction_s / K,
        "graph_ms_per_step": 1000.0 * timings["graph"] / K,
        "overlap_ms_per_step": 1000.0 * timings["overlap"] / K if "overlap" in timings else None,
        "launch_grids": tuned,
        "copy_peak_GBps": copy_gbps,
        "steps_ms_GBps": stages,
        "serialize_delta": {
            "ms_per_step": acc["sd_ms"] / K,
            "GBps_algorithmic": sd_gbps,
            "frac_hbm_peak": sd_gbps / HBM_PEAK_GBPS,
            "frac_copy_peak": sd_gbps / copy_gbps,
        },
        "bytes_per_agent": {
            "raw_record": acc["msg"] / records,
            "plain_delta": acc["tad"] / records,
            "learned_delta": None,
        },
        "step_algorithmic_GBps": (acc["sel"] + acc["ser"] + acc["match"] + acc["enc"] + acc["dec"]) / best_s / 1e9,
        # the dominant single kernel (a family of several kernels, as the join's, is listed in rooflines only)
        "roofline": next((r for r in rooflines if r["kernel"] not in MULTI_KERNEL_FAMILIES), None),
        "rooflines": rooflines,
    }
    if batched and args.per_partition:
        pp_s = per_partition_pass(native, cfg, host_states, args.warmup)
        out["per_partition_ms_per_step"] = 1000.0 * pp_s / K
        out["batched_speedup_vs_per_partition"] = pp_s / best_s
        log(f"per-partition pass: {1000 * pp_s / K:.3f} ms/step")
    if not args.no_learned:
        trained = train_predictor(native, synth, log)
        blob = trained["random_walk"][0]
        pred = native.Predictor(ctx, blob)
        out["learned"] = learned_mode(ctx, native, cfg, dev_states, host_states, args, idx_cap, ser_cap, enc_cap,
                                      pred, copy_gbps)
        lm = out["learned"]
        log(f"learned mode: {lm['ms_per_step']:.3f} ms/step, serialize+delta "
            f"{lm['serialize_delta']['GBps_algorithmic']:.0f} GB/s, {lm['bytes_per_agent']:.3f} B/record")
        out["bytes_per_agent"]["learned_delta"] = lm["bytes_per_agent"]
        out["bytes_per_agent"]["learned_segments"] = lm["learned_segments"]
        out["bytes_per_agent"]["learned_training"] = f"{trained['random_walk'][1]} windows of the 1e5-agent world"
        out["bytes_per_agent"]["persistent_variant"] = persistent_variant(native, synth, trained["persistent"][0])
    if not batched:
        out["growth"] = growth_pass(ctx, native, cfg, dev_states[0], idx_cap, ser_cap, args.warmup, K)
        log(f"growth of every 100th record by 2 words: grow {out['growth']['grow_ms']:.3f} ms, compact "
            f"{out['growth']['compact_ms']:.3f} ms ({out['growth']['compact_GBps']:.0f} GB/s)")
        rb = refresh_bytes(ctx, native, cfg, dev_states, args.warmup, idx_cap, ser_cap)
        out["bytes_per_agent"]["plain_delta_by_refresh_interval"] = {str(k): v / records for k, v in rb.items()}
        log("plain delta bytes/record by refresh interval: " +
            ", ".join(f"k={k}: {v / records:.2f}" for k, v in rb.items()))
    if not args.no_migration and not batched:
        del dev_states
        torch.cuda.empty_cache()
        out["migration"] = migration_pass(native, synth, args.warmup, args.steps)
        log(f"migration: {out['migration']['ms_per_step']:.3f} ms/step, "
            f"{out['migration']['migrants_per_step']} migrants, migrate_keep "
            f"{out['migration']['roofline']['achieved']:.0f} GB/s")
    if not args.no_cpu and not batched:
        per_rec = {"select": acc["sel"], "serialize": acc["ser"], "encode": acc["match"] + acc["enc"],
                   "decode": acc["dec"]}
        out["cpu_baseline"] = cpu_baseline(host_states, cfg, args.cpu_seconds,
                                           {k: v / acc["records"] for k, v in per_rec.items()})
        cb = out["cpu_baseline"]
        log(f"cpu baseline: {cb['value']:.3g} records/s on {cb['cores']} threads "
            f"({cb['single_core']['value']:.3g} on one core), {cb['cpu_model']}")
    print(json.dumps(out), flush=True)


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter measurement
    (profiles/traffic.json), or None when there is none for this kernel and
    workload or the kernel's source has changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path))[kernel]
    except (OSError, KeyError, ValueError):
        return None
    src = os.path.join(ROOT, "paper_2509_24063_amd", "csrc", rec["source"])
    try:
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    if digest != rec["sha256"] or rec["workload"] != workload:
        return None
    return rec["bytes_per_launch"]


def refresh_bytes(ctx, native, cfg, dev_states, warmup, idx_cap, ser_cap, intervals=(1, 2, 4, 8)):
    """Encoded bytes over the timed states when sender and receiver refresh
    their reference only every k-th iteration (Sec. 2.3), per k."""
    from paper_2509_24063_amd.exchange import Pipeline
    out = {}
    for k in intervals:
        pl = Pipeline(ctx, dev_states[0], cfg.w, cfg.ndirs, idx_cap, ser_cap, refresh=k)
        total = 0
        for t, ds in enumerate(dev_states):
            pl.step(ds)
            if t >= warmup:
                total += int(pl.outputs()[1][-1].item())
        ctx.check(f"refresh {k}")
        pl.close()
        del pl
        out[k] = total
    return out


def growth_pass(ctx, native, cfg, ds, idx_cap, ser_cap, warmup, steps, every=100, extra=2):
    """Growth of records used in place and compaction (Sec. 2.2.1
    "Mutability") on the messages of one state of the workload: every
    `every`-th record grows by `extra` words (a 16-byte behaviour), then the
    whole message set is compacted.  The messages are restored before each
    step, outside the timed region."""
    import numpy as np
    import torch
    dev = torch.device("cuda")
    idx, seg = ctx.select_aura(ds, cfg.w, cfg.ndirs, idx_cap=idx_cap)
    buf, moff = ctx.serialize(ds, idx, seg, idx_cap=idx_cap)
    ctx.check("growth setup")
    so, mo = seg.cpu().numpy(), moff.cpu().numpy()
    M, nrec = int(mo[-1]), int(so[-1])
    hb = buf[:M].cpu().numpy()
    g = np.arange(0, nrec, every, dtype=np.int64)
    s_of = np.searchsorted(so, g, side="right") - 1
    r_of = g - so[s_of]
    a = mo[s_of]
    n = hb[(a[:, None] + 8 + np.arange(4)).astype(np.int64)].view(np.uint32).ravel().astype(np.int64)
    off = hb[(a[:, None] + 32 + 4 * r_of[:, None] + np.arange(4)).astype(np.int64)].view(np.uint32).ravel()
    p = a + 32 + 8 * ((n + 1) // 2) + 8 * off.astype(np.int64)
    w = hb[(p[:, None] + 12 + np.arange(4)).astype(np.int64)].view(np.uint32).ravel().astype(np.int64)
    words = (w + extra).astype(np.uint32)
    arena = 8 * int(words.sum()) + 64
    work = torch.empty(M + arena, dtype=torch.uint8, device=dev)
    seg_t = torch.from_numpy(s_of.astype(np.int32)).to(dev)
    rec_t = torch.from_numpy(r_of.astype(np.uint32)).to(dev)
    words_t = torch.from_numpy(words).to(dev)
    used = torch.zeros(1, dtype=torch.int64, device=dev)
    out_cap = M + 8 * extra * len(g)
    out = torch.empty(out_cap, dtype=torch.uint8, device=dev)
    out_off = torch.empty(moff.numel(), dtype=torch.int64, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_grow = t_cmp = 0.0
    for k in range(warmup + steps):
        work[:M].copy_(buf[:M])
        used.zero_()
        ev[0].record()
        ctx.view_grow(work, moff, seg_t, rec_t, words_t, used)
        ev[1].record()
        ctx.view_compact(work, moff, out, out_off)
        ev[2].record()
        torch.cuda.synchronize()
        if k >= warmup:
            t_grow += ev[0].elapsed_time(ev[1])
            t_cmp += ev[1].elapsed_time(ev[2])
    ctx.check("growth steps")
    assert int(out_off[-1].item()) == out_cap, "compacted size"
    cmp_ms = t_cmp / steps
    cmp_bytes = M + out_cap  # read every message once, write its canonical copy
    return {"records": nrec, "grown": int(len(g)), "grow_ms": t_grow / steps, "compact_ms": cmp_ms,
            "compact_GBps": cmp_bytes / (cmp_ms / 1000.0) / 1e9,
            "compact_frac_hbm_peak": cmp_bytes / (cmp_ms / 1000.0) / 1e9 / HBM_PEAK_GBPS}


def migration_pass(native, synth, warmup, steps, agents=1e7):
    """Agent migration on one GPU's share of space: `agents` sphere agents in a
    2x2x2 grid of 500 um boxes (the 1000^3 um domain of the single-box
    workload), walls only at the domain boundary, one Gaussian walk step of
    sigma 0.1 um so that agents cross the inner faces.  A step selects the
    migrants, serializes them and builds the new store from the old one and
    the messages (each routed to the neighbouring box).  Every step takes the
    same input, so its outputs are identical from step to step."""
    import numpy as np
    import torch
    cfg = synth.config(2, grid=(2, 2, 2), side=500.0, median=agents / 8, walls="domain")
    world = synth.World(cfg)
    world.step()
    st = world.store
    ctx = native.Context(cfg.schema)
    ds = native.DeviceStore(st)
    F, I = st.f64.shape[0], st.i32.shape[0]
    nseg = st.P * 26
    dev = torch.device("cuda")
    dest = torch.from_numpy(synth.neighbour_table(cfg.grid)).to(dev)
    idx_cap = max(4096, st.n // 100)
    idx = torch.empty(idx_cap, dtype=torch.int32, device=dev)
    seg = torch.empty(nseg + 1, dtype=torch.int64, device=dev)
    ser_cap = ctx.serialize_bound(ds, nseg, idx_cap)
    buf = torch.empty(ser_cap, dtype=torch.uint8, device=dev)
    moff = torch.empty(nseg + 1, dtype=torch.int64, device=dev)
    out = native.DeviceStore.alloc(F, I, st.boxes, st.n + 4096, st.beh.size + (1 << 20))
    sizes = torch.empty(2, dtype=torch.int64, device=dev)

    def step():
        ctx.select_migrants(ds, idx_cap=idx_cap, out=(idx, seg))
        ctx.serialize(ds, idx, seg, idx_cap=idx_cap, out=(buf, moff))
        ctx.migrate_apply(ds, buf, moff, dest, out, sizes=sizes)

    for _ in range(warmup):
        step()
    ctx.check("migration warm-up")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(steps):
        step()
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / steps
    ctx.check("migration steps")
    ctx.time_kernel("migrate_keep")
    for _ in range(steps):
        step()
    launches, kernel_ms = ctx.kernel_time()
    ctx.time_kernel(None)
    ctx.check("migration instrumented steps")
    migrants = int(seg[-1].item())
    mi = idx[:migrants].cpu().numpy().astype(np.int64)
    beh_m = int((st.beh_off[mi + 1] - st.beh_off[mi]).sum())
    kept = st.n - migrants
    sz = sizes.cpu().numpy()
    assert int(sz[0]) == st.n and int(sz[1]) == st.beh.size, "migration lost or created agents"
    # k_mig_keep moves every column of each agent that stays (read + write) and
    # its behaviour bytes, reads two behaviour offsets and writes one
    col_bytes = 12 + 8 * F + 4 * I
    kb = 2 * (kept * col_bytes + (st.beh.size - beh_m)) + 24 * kept
    avg_ms = kernel_ms / max(launches, 1)
    achieved = kb / (avg_ms / 1000.0) / 1e9
    ctx.close()
    return {
        "workload": (f"{st.n} sphere agents in 8 boxes of 500^3 um (2x2x2, walls at the 1000^3 um domain only), "
                     "one walk step of sigma 0.1 um; select migrants + serialize + rebuild the store"),
        "ms_per_step": ms,
        "agents_per_s": st.n / (ms / 1000.0),
        "migrants_per_step": migrants,
        "roofline": {"kernel": "migrate_keep", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS, "traffic": None, "launches": launches,
                     "avg_ms": avg_ms, "algorithmic_bytes_per_launch": kb},
    }


def scale_pass(args, native, synth):
    """A large batched workload with its states advanced on the GPU
    (synth_device.DeviceWorld): every iteration (select, serialize, encode,
    decode over all partitions) is one graph replay, timed with events; the
    population moves on between iterations, outside the timed region.
    hetero: 80/20 spheres and cylinders with 14 fp64 fields, 0-4 behaviours
    of 1-7 words, the learned predictor (trained on the GPU on the 1e5-agent
    world); after each timed iteration the same messages are also encoded in
    plain mode for the bytes per record.  The receiver decodes against the
    sender's reference copy (byte-identical) and writes its C' over the
    consumed messages, so that 2e8 agents fit one GPU; tests/test_gpu_scale.py
    checks one sampled partition of the same runs against the oracle every
    iteration."""
    import numpy as np
    import torch

    from paper_2509_24063_amd.exchange import sized_pipeline
    from paper_2509_24063_amd.synth_device import DeviceWorld, partition_sizes

    hetero = args.workload == "hetero"
    over = {"median": args.agents} if args.agents else {}
    cfg = synth.config(5 if hetero else 3, **over)
    iterations = args.warmup + args.steps
    copy_gbps = copy_peak(args.copy_peak_mib)
    torch.cuda.empty_cache()
    t0 = time.time()
    cap, beh_cap = DeviceWorld.capacity(cfg, iterations + 1)
    counts, boxes = partition_sizes(cfg)
    ds = native.DeviceStore.alloc(max(cfg.n_f64), max(cfg.n_i32), boxes, cap, beh_cap)
    world = DeviceWorld(cfg, ds, log=log)
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    n0, P = world.n, world.P
    nseg = P * cfg.ndirs
    log(f"{cfg.name}: {n0} agents in {P} partitions (store for {cap}), {time.time() - t0:.0f}s")
    pred = None
    if hetero:
        blob = train_predictor(native, synth, log, which=("random_walk",))["random_walk"][0]
    ctx = native.Context(cfg.schema)
    if hetero:
        pred = native.Predictor(ctx, blob)
    pl = sized_pipeline(ctx, ds, cfg.ndirs, cfg.w, cap / n0, pred)
    pl.capture()
    torch.cuda.synchronize()
    log(f"buffers {pl.sizing}; {torch.cuda.memory_allocated() / 1e9:.1f} GB allocated by torch")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    acc = dict(records=0, msg=0, tad=0, plain=0, ms=0.0, agents=0, learned=0, mixed=0, sel=0, ser=0, match=0,
               enc=0, dec=0)
    prev_M, prev_S = 32 * nseg, 0
    for t in range(iterations):
        n_now = world.n
        ev[0].record()
        pl.step(graph=True)
        ev[1].record()
        torch.cuda.synchronize()
        ctx.check(f"iteration {t}")
        S = int(pl.seg_off[-1].item())
        M = int(pl.msg_off[-1].item())
        T = int(pl.enc_off[-1].item())
        if t >= args.warmup:
            acc["ms"] += ev[0].elapsed_time(ev[1])
            acc["records"] += S
            acc["agents"] += n_now
            acc["msg"] += M
            acc["tad"] += T
            modes = pl.modes[:nseg].cpu().numpy()
            acc["learned"] += int(np.count_nonzero(modes == 1))
            acc["mixed"] += int(np.count_nonzero(modes == 2))
            acc["sel"] += 24 * n_now + 4 * S
            acc["ser"] += 4 * S + 16 * S + 2 * M
            acc["match"] += 16 * (S + prev_S)
            acc["enc"] += M + prev_M + T + M
            acc["dec"] += T + prev_M + M
            if hetero:  # the same messages in plain mode (C' is the same either way)
                p = 1 - pl.r
                ctx.delta_encode(pl.msgs, pl.msg_off, pl.ref[p], pl.ref_off[p],
                                 out=(pl.enc, pl.enc_off, pl.ref[pl.last], pl.ref_off[pl.last], pl.modes))
                ctx.check(f"plain encoding {t}")
                acc["plain"] += int(pl.enc_off[-1].item())
        log(f"iteration {t}: {ev[0].elapsed_time(ev[1]):.2f} ms, {n_now} agents, {S} records, {T} encoded bytes")
        prev_M, prev_S = M, S
        world.step()
    K = args.steps
    # the dominant kernels in one more (eager) iteration, timed with events
    fams = "encode_groups,decode_unpack,serialize_pack,select_count,encode_join,predict"
    ctx.time_kernel(fams)
    pl.step()
    ktimes = {f: ctx.kernel_time(f) for f in fams.split(",")}
    ctx.time_kernel(None)
    ctx.check("instrumented iteration")
    at = pl.enc_off[:nseg, None] + torch.arange(64, device=pl.enc.device)
    heads = pl.enc[at.reshape(-1)].cpu().numpy().view(np.uint64).reshape(nseg, 8)
    one = dict(records=int(pl.seg_off[-1].item()), msg=int(pl.msg_off[-1].item()),
               W=int(heads[:, 5].sum()), var=int(heads[:, 7].sum()),
               matched=int((heads[:, 1] >> np.uint64(32)).sum()),
               groups=int(((heads[:, 5] + np.uint64(63)) // np.uint64(64)).sum()))
    one["sel"] = 24 * world.n + 4 * one["records"]
    one["match"] = 16 * (one["records"] + prev_S)
    rooflines = []
    for f, (launches, ms) in ktimes.items():
        key = f + "_learned" if (hetero and f == "encode_groups") else f
        b = kernel_bytes(key, one)
        if launches and b == b:
            rooflines.append(roofline_entry(f, launches, ms, b, copy_gbps, None))
    rooflines.sort(key=lambda r: -r["avg_ms"])
    single = [r for r in rooflines if r["kernel"] not in MULTI_KERNEL_FAMILIES]
    sd = acc["ser"] + acc["match"] + acc["enc"]
    step_bytes = acc["sel"] + sd + acc["dec"]
    out = {
        "metric": METRIC,
        "value": acc["records"] / (acc["ms"] / 1000.0),
        "unit": "aura records/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": acc["ms"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded, generated and advanced on the GPU; the paper's BioDynaMo models are not "
                "available)",
        "config": {
            "workload": (f"{P} partitions ({'x'.join(map(str, cfg.grid))} periodic, lognormal sizes, median "
                         f"{cfg.median:.3g}), {n0:.3g} agents at the start"
                         + (", 80/20 spheres/cylinders with 14 fp64 fields, 0-4 behaviours of 1-7 words, 2% "
                            "division, 1% death, learned predictor" if hetero else
                            ", spheres, 1% division, 0.5% death, plain delta")
                         + "; one graph replay per iteration (select + serialize + encode + decode)"),
            "agents_start": n0,
            "agents_mean_timed": acc["agents"] / K,
            "partitions": P,
            "segments": nseg,
            "records_per_step": acc["records"] / K,
        },
        "timed_mode": "graph",
        "copy_peak_GBps": copy_gbps,
        "step_algorithmic_GBps": step_bytes / (acc["ms"] / 1000.0) / 1e9,
        "bytes_per_agent": {"raw_record": acc["msg"] / acc["records"], "delta": acc["tad"] / acc["records"]},
        "roofline": single[0] if single else None,
        "rooflines": rooflines,
        "kernels_us_instrumented_step": {f: 1000.0 * ms for f, (n, ms) in ktimes.items() if n},
        "buffers": pl.sizing,
        "device_memory_GB": {"allocated_peak": torch.cuda.max_memory_allocated() / 1e9,
                             "reserved_peak": torch.cuda.max_memory_reserved() / 1e9},
    }
    if hetero:
        out["bytes_per_agent"]["plain_delta"] = acc["plain"] / acc["records"]
        out["bytes_per_agent"]["learned_delta"] = acc["tad"] / acc["records"]
        out["learned_segments"] = acc["learned"] / K
        out["mixed_segments"] = acc["mixed"] / K
    pl.close()
    ctx.close()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_exchange(oracle, store, cfg, ref, ref_off, pool, nthreads):
    """One exchange through the oracle (select, serialize, encode, decode).
    With a thread pool the oracle's one-message functions run concurrently
    over the segments (and the selection over agent ranges of the box, whose
    per-direction lists are concatenated in range order): the oracle's own
    code, called from several threads (ctypes releases the interpreter lock
    inside each call).  Returns (times per step, records, C', offsets)."""
    import ctypes as C
    import numpy as np
    L = oracle.lib()
    t = {}
    t0 = time.perf_counter()
    if pool is None or store.P != 1:
        idx, seg = oracle.select_aura(store, cfg.w, cfg.ndirs)
    else:
        f64 = np.ascontiguousarray(store.f64)
        n, stride = store.n, f64.shape[1]
        bounds = np.linspace(0, n, nthreads + 1).astype(np.int64)
        boxes = np.ascontiguousarray(store.boxes, np.float64)

        def sel(c):
            a, b = int(bounds[c]), int(bounds[c + 1])
            po = np.array([0, b - a], np.int64)
            so = np.zeros(cfg.ndirs + 1, np.int64)
            ix = np.zeros(max(1, 26 * (b - a)), np.int32)
            st = L.orc_select_aura(1, po.ctypes.data_as(C.c_void_p), C.c_void_p(f64.ctypes.data + 8 * a), stride,
                                   boxes.ctypes.data_as(C.c_void_p), float(cfg.w), cfg.ndirs,
                                   ix.ctypes.data_as(C.c_void_p), ix.size, so.ctypes.data_as(C.c_void_p))
            assert st == 0
            return [ix[so[d]:so[d + 1]] + a for d in range(cfg.ndirs)]
        parts = list(pool.map(sel, range(nthreads)))
        lists = [np.concatenate([parts[c][d] for c in range(nthreads)]) for d in range(cfg.ndirs)]
        seg = np.zeros(cfg.ndirs + 1, np.int64)
        np.cumsum([x.size for x in lists], out=seg[1:])
        idx = np.concatenate(lists).astype(np.int32)
    t1 = time.perf_counter()
    nseg = seg.shape[0] - 1
    if pool is None:
        buf, moff = oracle.serialize(store, cfg.schema, idx, seg)
        t2 = time.perf_counter()
        enc, eoff, nref, noff, _, _ = oracle.encode_all(buf, moff, ref, ref_off)
        t3 = time.perf_counter()
        dec, doff, _ = oracle.decode_all(enc, eoff, ref, ref_off)
    else:
        def ser(s):
            a, b = int(seg[s]), int(seg[s + 1])
            return oracle.serialize(store, cfg.schema, idx[a:b], np.array([0, b - a], np.int64))[0]
        msgs = list(pool.map(ser, range(nseg)))
        t2 = time.perf_counter()
        refs = oracle.split(ref, ref_off)

        def encode(s):
            st, e, nr, _, _ = oracle.delta_encode(msgs[s], refs[s])
            assert st == 0
            return e, nr
        er = list(pool.map(encode, range(nseg)))
        t3 = time.perf_counter()

        def decode(s):
            st, d, _ = oracle.delta_decode(er[s][0], refs[s])
            assert st == 0
            return d
        decs = list(pool.map(decode, range(nseg)))
        nref, noff = oracle.join([x[1] for x in er])
        dec, doff = oracle.join(decs)
    t4 = time.perf_counter()
    assert np.array_equal(dec, nref)
    t.update(select=t1 - t0, serialize=t2 - t1, encode=t3 - t2, decode=t4 - t3)
    return t, int(seg[-1]), nref, noff


def cpu_baseline(states, cfg, budget_s, bytes_per_record):
    """The oracle, as it stands, on the same workload's states: first on one
    host thread, then with its one-message calls spread over the host's
    threads (up to 16), each leg until its share of the time budget is used.
    Records per second over whole exchanges (select, serialize, encode,
    decode), and per step."""
    import concurrent.futures as cf

    import oracle

    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    legs = {}
    for name, nthreads, share in (("single_core", 1, 0.6), ("threads", threads, 0.4)):
        pool = cf.ThreadPoolExecutor(nthreads) if nthreads > 1 else None
        ref, ref_off = oracle.empty_messages(states[0].P * cfg.ndirs)
        # the first exchange against an empty reference is not representative: done untimed
        _, _, ref, ref_off = cpu_exchange(oracle, states[0], cfg, ref, ref_off, pool, nthreads)
        tot = dict(select=0.0, serialize=0.0, encode=0.0, decode=0.0)
        records, steps = 0, 0
        for st in states[1:]:
            t, S, ref, ref_off = cpu_exchange(oracle, st, cfg, ref, ref_off, pool, nthreads)
            for k in tot:
                tot[k] += t[k]
            records += S
            steps += 1
            if sum(tot.values()) > share * budget_s:
                break
        if pool is not None:
            pool.shutdown()
        spent = sum(tot.values())
        legs[name] = {"value": records / spent, "threads": nthreads, "exchanges": steps, "records": records,
                      "seconds": spent, "ms_per_step": {k: 1000.0 * v / steps for k, v in tot.items()},
                      "GBps_algorithmic": {k: bytes_per_record[k] * records / v / 1e9 for k, v in tot.items()}}
    best = legs["threads"] if legs["threads"]["value"] > legs["single_core"]["value"] else legs["single_core"]
    return {"value": best["value"], "unit": "aura records/s", "cores": best["threads"], "kind": "oracle",
            "sample": (f"{best['exchanges']} whole exchanges (select, serialize, encode, decode) of the same "
                       f"{states[0].n:.0e}-agent workload, {best['records']} records, {best['seconds']:.1f} s on "
                       f"{best['threads']} host thread(s); the oracle's one-message calls spread over the threads "
                       "by segment (the selection by agent range)"),
            "cpu_model": cpu_model(), "host_threads_available": len(os.sched_getaffinity(0)),
            "single_core": legs["single_core"], "threaded": legs["threads"]}


if __name__ == "__main__":
    main()
