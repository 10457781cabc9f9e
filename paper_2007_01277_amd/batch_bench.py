"""Batched N-way fusion of many small instances: workload and benchmark.

Workload: `count` instances; kind uniform over the six data kernels (the hash
kinds can be drawn too, see ``draw``); 2^k elements with k uniform in
[kmin, kmax]; image kinds shaped [1, 16, 16, 2^k / 256] (im2col 3x3/s1/p1,
upsample x2, maxpool 3x3/s2/p1 with indices), integer mixing with 32 rounds,
histogram bytes from the Zipf law; a hash instance counts as 64 elements.
Consecutive instances form groups of 2 to 4 (uniform).
Every instance has its own scratch region (so concurrent baselines cannot
race), zero-filled at allocation.

Modes timed (median of `reps` runs, events on the launch stream):
  back_to_back   every instance solo, one after the other, one stream
  streams4       round-robin over four streams, forked and joined with events
  graph_solo     a HIP graph of the back-to-back launches (launch cost removed,
                 no fusion)
  batch          the persistent N-way fused kernel, one launch, under the
                 schedule the schedule search picks (static groups or worker
                 intervals; workgroup size, split, item size)
  batch_graph    the same launch replayed from a captured HIP graph

    python -m paper_2007_01277_amd.batch_bench --count 1000 --out batch.json
    python -m paper_2007_01277_amd.batch_bench --schedule 512,4,64,0   (a fixed schedule)
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import hfuse as H
from . import inputs


DATA_KINDS = (H.HF_BN_STATS, H.HF_INT_MIX, H.HF_IM2COL, H.HF_LDS_HIST, H.HF_UPSAMPLE, H.HF_MAXPOOL)


def draw(count: int = 1000, seed: int = 3, kmin: int = 12, kmax: int = 18, kinds=DATA_KINDS):
    g = inputs.rng(seed)
    kinds = np.asarray(kinds)[g.integers(0, len(kinds), size=count)]
    logs = g.integers(kmin, kmax + 1, size=count)
    groups, gid, i = [], 0, 0
    while i < count:
        size = int(g.integers(2, 5))
        for _ in range(min(size, count - i)):
            groups.append(gid)
        i += size
        gid += 1
    return [int(k) for k in kinds], [int(v) for v in logs], groups[:count]


class Workload:
    """Device buffers and task descriptors of one drawn batch."""

    def __init__(self, kinds, logs, seed: int = 3):
        import torch
        self.kinds, self.logs = kinds, logs
        self.tasks, self.bufs, self.outs, self.ins = [], [], [], []
        self.meta = []  # per instance: (nonce0, table tensor) of hash kinds, else None
        for i, (kind, k) in enumerate(zip(kinds, logs)):
            n = 1 << k
            s = seed * 100000 + i
            if kind in (H.HF_BN_STATS, H.HF_IM2COL, H.HF_UPSAMPLE, H.HF_MAXPOOL):
                x = inputs.cuda_normal((1, 16, 16, n // 256), s)
                if kind == H.HF_BN_STATS:
                    o = [torch.empty(16, device="cuda"), torch.empty(16, device="cuda")]
                    t = H.task_bn_stats(x, *o)
                elif kind == H.HF_IM2COL:
                    o = [torch.empty((1, 16 * 9, 16 * (n // 256)), device="cuda")]
                    t = H.task_im2col(x, o[0], 3, 3, 1, 1)
                elif kind == H.HF_UPSAMPLE:
                    o = [torch.empty((1, 16, 32, 2 * (n // 256)), device="cuda")]
                    t = H.task_upsample(x, o[0], 2)
                else:
                    osh = H.maxpool_out_shape(tuple(x.shape), 3, 3, 2, 1)
                    o = [torch.empty(osh, device="cuda"), torch.empty(osh, dtype=torch.int32, device="cuda")]
                    t = H.task_maxpool(x, o[0], o[1], 3, 3, 2, 1)
            elif kind == H.HF_INT_MIX:
                x = inputs.cuda_uint32(n, s)
                o = [torch.empty_like(x)]
                t = H.task_int_mix(x, o[0], 32)
            elif kind in (H.HF_SHA256D, H.HF_BLAKE2B, H.HF_ETHASH):
                m = max(1, n >> 6)  # a hash counts as 64 elements of work
                x = torch.from_numpy(inputs.header80(s).view(np.int32)).cuda()
                o = [torch.empty((m, 8), dtype=torch.int32, device="cuda")]
                tab = None
                if kind == H.HF_ETHASH:
                    tab = inputs.cuda_eth_table(4099, s)
                    self.bufs.append(tab)
                    t = H.task_ethash(x, tab, o[0], inputs.nonce0(s), m)
                else:
                    t = (H.task_sha256d if kind == H.HF_SHA256D else H.task_blake2b)(x, o[0], inputs.nonce0(s), m)
                self.meta.append((inputs.nonce0(s), tab))
            else:
                x = inputs.cuda_zipf_u8(n, s)
                o = [torch.empty(256, dtype=torch.int32, device="cuda")]
                t = H.task_lds_hist(x, o[0])
            if len(self.meta) < len(self.tasks) + 1:
                self.meta.append(None)
            nb = H.hf_scratch_bytes(t)
            if nb > 0:
                scr = torch.zeros(nb // 4 + 64, dtype=torch.int32, device="cuda")
                t.scratch = scr.data_ptr()
                self.bufs.append(scr)
            self.ins.append(x)
            self.outs.append(o)
            self.tasks.append(t)
        torch.cuda.synchronize()

    def snapshot(self):
        return [[o.clone() for o in outs] for outs in self.outs]

    def clear(self):
        for outs in self.outs:
            for o in outs:
                o.fill_(7)

    def elements(self):
        return int(sum(x.numel() for x in self.ins))

    def bytes(self):
        b = 0
        for x, outs in zip(self.ins, self.outs):
            b += x.numel() * x.element_size() + sum(o.numel() * o.element_size() for o in outs)
        return b


def same(a, b):
    return all(all(bool((p == q).all()) for p, q in zip(x, y)) for x, y in zip(a, b))


def run_modes(w: Workload, groups, reps: int = 10, block=None, waves=None, log=sys.stderr, schedule=None):
    import torch
    st = torch.cuda.current_stream()
    side = [torch.cuda.Stream() for _ in range(3)]
    res = {}

    def timed(fn):
        ts = []
        for r in range(reps + 1):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(st)
            fn()
            b.record(st)
            torch.cuda.synchronize()
            if r > 0:
                ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    def back_to_back():
        for t in w.tasks:
            H.hf_run_solo(t, 256, 0, st)

    def streams4():
        ev = torch.cuda.Event()
        ev.record(st)
        for s in side:
            s.wait_event(ev)
        all_s = [st] + side
        for i, t in enumerate(w.tasks):
            H.hf_run_solo(t, 256, 0, all_s[i % 4])
        for s in side:
            e = torch.cuda.Event()
            e.record(s)
            st.wait_event(e)

    w.clear()
    res["back_to_back_ms"] = timed(back_to_back)
    ref = w.snapshot()
    print(f"back-to-back {res['back_to_back_ms']:.3f} ms", file=log, flush=True)
    w.clear()
    res["streams4_ms"] = timed(streams4)
    res["streams4_equal"] = same(ref, w.snapshot())
    # a HIP graph of the individual launches
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for t in w.tasks:
            H.hf_run_solo(t, 256, 0, None)
    w.clear()
    res["graph_solo_ms"] = timed(g.replay)
    res["graph_solo_equal"] = same(ref, w.snapshot())
    # the tuned schedule of the persistent fused kernel
    if schedule is not None:
        b = H.Batch(w.tasks, groups, schedule=schedule)
        res["schedule"] = {**schedule.as_dict(), **b.info()}
    elif block is None:
        t0 = time.time()
        sched, tms, nprof = H.hf_batch_tune_sched(w.tasks, groups, reps=5)
        res["tune_s"] = round(time.time() - t0, 3)
        res["schedules_profiled"] = nprof
        b = H.Batch(w.tasks, groups, schedule=sched)
        res["schedule"] = {**sched.as_dict(), **b.info()}
    else:
        b = H.Batch(w.tasks, groups, waves, block)
        res["schedule"] = {"block": block, **b.info()}
    w.clear()
    res["batch_ms"] = timed(lambda: b.run(False))
    res["batch_equal"] = same(ref, w.snapshot())
    w.clear()
    res["batch_graph_ms"] = timed(lambda: b.run(True))
    res["batch_graph_equal"] = same(ref, w.snapshot())
    b.close()
    for k in ("back_to_back", "streams4", "graph_solo"):
        res[f"speedup_vs_{k}"] = round(res[f"{k}_ms"] / res["batch_graph_ms"], 3)
    res["batch_graph_GBps"] = round(w.bytes() / (res["batch_graph_ms"] * 1e-3) / 1e9, 1)
    return res, ref


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=1000)
    ap.add_argument("--kmin", type=int, default=12)
    ap.add_argument("--kmax", type=int, default=18)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--out", default="")
    ap.add_argument("--schedule", default="",
                    help="block,interval_waves,item_kb,split_policy: a fixed schedule instead of the search")
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    H.hf_init()
    kinds, logs, groups = draw(a.count, kmin=a.kmin, kmax=a.kmax)
    w = Workload(kinds, logs)
    H.hf_warmup(300)
    sched = H.hf_batch_schedule(*[int(v) for v in a.schedule.split(",")]) if a.schedule else None
    res, _ = run_modes(w, groups, reps=a.reps, schedule=sched)
    res.update({"count": a.count, "groups": len(set(groups)), "elements": w.elements(), "bytes": w.bytes()})
    print(json.dumps(res), flush=True)
    if a.out:
        json.dump(res, open(a.out, "w"), indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
