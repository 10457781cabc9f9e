"""Benchmark of the horizontally fused kernel on one MI355X.

Workload (the memory + compute pair): batch-norm statistics of an fp32 NCHW
tensor [64, 256, 56, 56] (x = z*scale_c + shift_c) fused with 128 rounds of
integer mixing over 2^24 uint32 seeds.  A step is one fused launch of the pair
at the configuration the exhaustive tuner picks (split, workgroup size, VGPR
bound); the same inputs are also run back to back (each kernel at its best
solo workgroup size) and on two concurrent streams.  Inputs are resident in
HBM before any timing starts.

Prints one JSON line: metric = speedup of the fused launch over the back-to-back
launches in percent, plus absolute times, HBM GB/s, the ALU roofline of the
fused kernel and the CPU oracle's time for the same step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fused vs back-to-back time speedup (%) per pair at 1 MI355X; HBM GB/s + VALU busy"
SHAPE = (64, 256, 56, 56)
N_MIX, ROUNDS = 1 << 24, 128
# MI355X: 256 CUs x 64 lanes of 32-bit integer VALU x 2.4 GHz
INT_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
OPS_PER_ROUND = 8  # 3 shifts, 3 xors, 1 multiply, 1 add


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cfg", type=str, default="", help="split_waves,block,cap: skip the tuner")
    ap.add_argument("--blocks", type=str, default="", help="block_bn,block_mix: skip the solo block sweep")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--no-pairs", action="store_true", help="skip the memory + atomic pairs")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run the reference copy kernel over this many MiB (counter calibration)")
    return ap.parse_args()


def copy_calibration(mib):
    """Plain device copy of a known size: the reference for scaling HBM counters."""
    import torch

    from paper_2007_01277_amd import hfuse as H
    n = mib << 20
    src = torch.ones(n // 4, device="cuda")
    dst = torch.empty_like(src)
    ms = [H.hf_copy(dst, src, n, timed=True) for _ in range(5)]
    print(json.dumps({"copy_bytes": n, "launches": 5, "ms": ms,
                      "gbps": [round(2 * n / (m * 1e-3) / 1e9, 1) for m in ms]}), flush=True)
    return 0


def traffic_from_profiles(kernel_key, launches_per_step=1):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources; None otherwise."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        d = json.load(fh)
    from paper_2007_01277_amd.rocprof_summary import csrc_hash
    e = d.get(kernel_key)
    if not e or e.get("csrc_hash") != csrc_hash():
        return None
    return e["hbm_bytes_per_launch"] * launches_per_step


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the fused kernel's "
              "multi-GPU sharding is described in DESIGN.md and not run", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    from paper_2007_01277_amd import hfuse as H
    from paper_2007_01277_amd import inputs

    torch.cuda.set_device(0)
    H.hf_init()
    if a.copy_mib:
        return copy_calibration(a.copy_mib)
    print("generating inputs", file=sys.stderr, flush=True)
    x = inputs.bn_input(SHAPE, seed=0)
    seeds = inputs.uint32_seeds(N_MIX, seed=0)
    xd = torch.from_numpy(x).cuda()
    sd = torch.from_numpy(seeds.view(np.int32)).cuda()
    mean = torch.empty(SHAPE[1], device="cuda")
    var = torch.empty(SHAPE[1], device="cuda")
    out = torch.empty_like(sd)
    ta = H.task_bn_stats(xd, mean, var)
    tb = H.task_int_mix(sd, out, ROUNDS)
    pr = H.make_pair(ta, tb)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    H.hf_warmup(500)
    # best solo workgroup size of each kernel (the back-to-back baseline's blocks)
    if a.blocks:
        blk = [int(v) for v in a.blocks.split(",")]
    else:
        blk = []
        for t in (ta, tb):
            best = None
            for b in (256, 512, 1024):
                ts = sorted(H.hf_run_solo(t, b, timed=True) for _ in range(15))[7]
                if best is None or ts < best[1]:
                    best = (b, ts)
            blk.append(best[0])
    print(f"solo blocks {blk}", file=sys.stderr, flush=True)
    if a.cfg:
        w, b, c = (int(v) for v in a.cfg.split(","))
        cfg = H.hf_config(w, b, c, 0)
        tune = None
    else:
        cfg, tune = H.hf_tune(pr, H.HF_TUNE_EXHAUSTIVE)
        cfg = H.hf_config(cfg.split_waves, cfg.block, cfg.vgpr_cap, 0)
    print(f"fused config {cfg}", file=sys.stderr, flush=True)

    def run_fused():
        H.hf_run_fused_cfg(pr, cfg, stream)

    def run_serial():
        H.hf_run_unfused(pr, blk[0], blk[1], H.HF_SERIAL, stream)

    def run_streams():
        H.hf_run_unfused(pr, blk[0], blk[1], H.HF_STREAMS, stream)

    def timed(fn, steps):
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs[0].record(stream)
        for i in range(steps):
            fn()
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / steps
        per = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
        return wall, per

    for _ in range(a.warmup):
        run_fused()
    fused_ms, fused_per = timed(run_fused, a.steps)
    print(f"fused {fused_ms:.4f} ms/step", file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        run_serial()
    serial_ms, serial_per = timed(run_serial, a.steps)
    for _ in range(a.warmup):
        run_streams()
    streams_ms, _ = timed(run_streams, a.steps)
    solo_ms = []
    for t, b in zip((ta, tb), blk):
        solo_ms.append(float(np.median([H.hf_run_solo(t, b, timed=True) for _ in range(21)])))

    # parity of the timed configuration with the back-to-back result
    run_fused()
    torch.cuda.synchronize()
    f_out = [mean.clone(), var.clone(), out.clone()]
    run_serial()
    torch.cuda.synchronize()
    bit_exact = all(torch.equal(p, q) for p, q in zip(f_out, [mean, var, out]))

    kernel_ms = float(np.mean(fused_per))
    ops = OPS_PER_ROUND * ROUNDS * N_MIX
    bytes_alg = x.nbytes + 2 * seeds.nbytes + 2 * 4 * SHAPE[1]
    achieved = ops / (kernel_ms * 1e-3) / 1e12
    speedup = (serial_ms / fused_ms - 1.0) * 100.0
    res = {
        "metric": METRIC,
        "value": round(speedup, 3),
        "unit": "%",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(fused_ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+u32",
        "data": "synthetic",
        "config": {
            "workload": f"bn_stats fp32 {list(SHAPE)} + int_mix u32 2^24 x {ROUNDS} rounds",
            "split_waves": cfg.split_waves, "block": cfg.block, "vgpr_cap": cfg.vgpr_cap,
            "solo_blocks": blk, "cache": "warm (no scrub between steps)",
        },
        "fused_ms": round(fused_ms, 5),
        "serial_ms": round(serial_ms, 5),
        "streams_ms": round(streams_ms, 5),
        "speedup_vs_streams_pct": round((streams_ms / fused_ms - 1.0) * 100.0, 3),
        "solo_ms": {"bn_stats": round(solo_ms[0], 5), "int_mix": round(solo_ms[1], 5)},
        "ideal_speedup_pct": round((sum(solo_ms) / max(solo_ms) - 1.0) * 100.0, 3),
        "hbm_gbps": round(bytes_alg / (kernel_ms * 1e-3) / 1e9, 2),
        "valu_busy": None,
        "fused_bit_exact_vs_serial": bit_exact,
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": round(INT_PEAK_TOPS, 3),
            "unit": "Tlane-op/s",
            "frac": round(achieved / INT_PEAK_TOPS, 4),
            "traffic": traffic_from_profiles("fused_bn_stats_int_mix"),
            "kernel": "fused_nocap/fused_cap<BnStats,IntMix>",
            "kernel_ms": round(kernel_ms, 5),
        },
    }
    if tune:
        res["tune"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in tune.items()}
    if not a.no_pairs:
        del xd, sd, out
        torch.cuda.empty_cache()
        res["other_pairs"] = other_pairs(a.steps)
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline(x, seeds)
    print(json.dumps(res), flush=True)
    return 0


def other_pairs(steps):
    """The memory + atomic pairs: im2col [32,128,56,56] 3x3/s1/p1 and bilinear x2
    upsample [32,64,128,128], each fused with a 256-bin histogram of 2^26 Zipf
    bytes; exhaustive tune, then the fused step against the back-to-back one."""
    import numpy as np
    import torch

    from paper_2007_01277_amd import hfuse as H
    from paper_2007_01277_amd import inputs
    xh = torch.from_numpy(inputs.zipf_u8(1 << 26, seed=2)).cuda()
    counts = torch.empty(256, dtype=torch.int32, device="cuda")
    th = H.task_lds_hist(xh, counts)
    xi = torch.from_numpy(inputs.normal_image((32, 128, 56, 56), 1)).cuda()
    cols = torch.empty((32, 128 * 9, 56 * 56), device="cuda")
    ti = H.task_im2col(xi, cols, 3, 3, 1, 1)
    xu = torch.from_numpy(inputs.normal_image((32, 64, 128, 128), 3)).cuda()
    up = torch.empty((32, 64, 256, 256), device="cuda")
    tu = H.task_upsample(xu, up, 2)
    out = {}
    for name, ta, tb in (("im2col+lds_hist", ti, th), ("upsample+lds_hist", tu, th)):
        pr = H.make_pair(ta, tb)
        blk = []
        for t in (ta, tb):
            blk.append(min((256, 512, 1024), key=lambda b: float(np.median([H.hf_run_solo(t, b, timed=True)
                                                                             for _ in range(9)]))))
        cfg, st = H.hf_tune(pr, H.HF_TUNE_EXHAUSTIVE)
        cfg = H.hf_config(cfg.split_waves, cfg.block, cfg.vgpr_cap, 0)
        fused = float(np.median([H.hf_run_fused_cfg(pr, cfg, timed=True) for _ in range(steps)]))
        serial = float(np.median([H.hf_run_unfused(pr, blk[0], blk[1], H.HF_SERIAL, timed=True)
                                  for _ in range(steps)]))
        streams = float(np.median([H.hf_run_unfused(pr, blk[0], blk[1], H.HF_STREAMS, timed=True)
                                   for _ in range(steps)]))
        out[name] = {"fused_ms": round(fused, 5), "serial_ms": round(serial, 5), "streams_ms": round(streams, 5),
                     "speedup_pct": round((serial / fused - 1) * 100, 2),
                     "speedup_vs_streams_pct": round((streams / fused - 1) * 100, 2),
                     "config": [cfg.split_waves, cfg.block, cfg.vgpr_cap], "solo_blocks": blk}
    return out


def cpu_baseline(x, seeds):
    """The CPU oracle (plain C, double accumulation, one thread) on the same step."""
    import oracle
    t0 = time.perf_counter()
    oracle.bn_stats(x)
    t1 = time.perf_counter()
    oracle.int_mix(seeds, ROUNDS)
    t2 = time.perf_counter()
    ms = (t2 - t0) * 1e3
    return {"value": round(ms, 2), "unit": "ms/step", "cores": 1, "kind": "oracle",
            "sample": f"the full step: bn_stats {list(SHAPE)} ({(t1 - t0) * 1e3:.0f} ms) + "
                      f"int_mix 2^24 x {ROUNDS} ({(t2 - t1) * 1e3:.0f} ms), single thread"}


if __name__ == "__main__":
    sys.exit(main())
