"""Speedup against the execution-time ratio of the two kernels.

The evaluation varies the input size of one kernel of each pair (the kernel
marked "*") and reports every fusion method's speedup over the native
execution at each resulting ratio of solo times (Sec. IV-A "Run Different
Workload", Sec. IV-B).  This script does the same on one MI355X for eight pairs
of this library, each with one kernel fixed and the other varied:

  bn_stats [64,256,56,56]         + int_mix* 2^24 elements, R = 1 .. 128 rounds
  bn_stats* [N,256,56,56]          + lds_hist 2^26 Zipf bytes, N = 4 .. 128
  im2col [32,128,56,56] 3x3        + lds_hist* 2^22 .. 2^28 Zipf bytes
  upsample x2 [32,64,128,128]      + lds_hist* 2^22 .. 2^28 Zipf bytes
  maxpool* [N,64,112,112] 3x3/s2   + lds_hist 2^26 Zipf bytes, N = 4 .. 128
  ethash* 2^15 .. 2^20 hashes      + sha256d 2^22 hashes (1 GiB table)
  blake2b* 2^20 .. 2^24 hashes     + ethash 327,680 hashes
  sha256d 2^22 hashes              + blake2b* 2^20 .. 2^24 hashes
and (``--sets memmem``) the six pairs of two memory-bound data kernels, each
with the first kernel at its bench shape and the second's batch N varied:
  bn_stats [64,256,56,56]  + maxpool* / upsample* / im2col*
  im2col [32,128,56,56]    + maxpool* / upsample*
  maxpool [64,64,112,112]  + upsample*

Methods at each point: HFuse = the exhaustive tuner's fused configuration;
Naive = even split of a 1024-lane workgroup without a bound (Sec. IV-A); VFuse =
vertical fusion at its best block; Streams = the two kernels on two streams;
Serial = back to back.  Each kernel runs at its best workgroup size in the
serial and two-stream baselines, chosen over back-to-back launches (see
solo_best).  Speedup % = (T_serial / T_method - 1) * 100; the ratio is
t_star / t_other of the best solo times.

    python -m paper_2007_01277_amd.ratio_sweep --out ratio.json

``--sets`` picks the groups: ``data`` (the first five pairs), ``crypto`` (the
three hash pairs), ``paper`` (both) and ``memmem``.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import hfuse as H
from . import inputs


def med(f, n):
    return float(np.median([f() for _ in range(n)]))


def solo_best(t, reps):
    """The kernel's best workgroup size, with each candidate timed over `reps`
    back-to-back launches (after three untimed ones), as the serial baseline
    runs it, in two passes over the candidates, each candidate keeping its
    faster pass; isolated single launches would favour sizes that only win
    when the GPU is idle before them."""
    import torch
    st = torch.cuda.current_stream()

    def back_to_back(b):
        for _ in range(3):
            H.hf_run_solo(t, b, 0, st)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            H.hf_run_solo(t, b, 0, st)
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    times = {}
    for _ in range(2):
        for b in (256, 512, 1024):
            ms = back_to_back(b)
            times[b] = min(ms, times.get(b, ms))
    b = min(times, key=times.get)
    return b, times[b]


def point(pr, reps):
    ba, ta = solo_best(pr.a, reps)
    bb, tb = solo_best(pr.b, reps)
    cfg, _ = H.hf_tune(pr, H.HF_TUNE_EXHAUSTIVE)
    cfg = H.hf_config(cfg.split_waves, cfg.block, cfg.vgpr_cap, 0)
    hfuse = med(lambda: H.hf_run_fused_cfg(pr, cfg, timed=True), reps)
    naive = med(lambda: H.hf_run_fused_cfg(pr, H.hf_config(8, 1024, 0, 0), timed=True), reps)
    vf = min(med(lambda: H.hf_run_vfused(pr, b, timed=True), reps) for b in (256, 512, 1024))
    serial = med(lambda: H.hf_run_unfused(pr, ba, bb, H.HF_SERIAL, timed=True), reps)
    streams = med(lambda: H.hf_run_unfused(pr, ba, bb, H.HF_STREAMS, timed=True), reps)
    sp = lambda t: round((serial / t - 1) * 100, 2)
    return {"t_a_ms": round(ta, 5), "t_b_ms": round(tb, 5), "serial_ms": round(serial, 5),
            "streams_ms": round(streams, 5), "hfuse_ms": round(hfuse, 5), "naive_ms": round(naive, 5),
            "vfuse_ms": round(vf, 5), "hfuse_cfg": [cfg.split_waves, cfg.block, cfg.vgpr_cap],
            "speedup_pct": {"hfuse": sp(hfuse), "naive": sp(naive), "vfuse": sp(vf), "streams": sp(streams)},
            "hfuse_vs_streams_pct": round((streams / hfuse - 1) * 100, 2)}


def image_task(kind, N, seed, keep):
    """A task of an image kind at its bench shape with batch N; the tensors it
    uses are appended to `keep`."""
    import torch
    if kind == H.HF_BN_STATS:
        x = inputs.cuda_normal((N, 256, 56, 56), seed)
        m, v = torch.empty(256, device="cuda"), torch.empty(256, device="cuda")
        keep += [x, m, v]
        return H.task_bn_stats(x, m, v)
    if kind == H.HF_IM2COL:
        x = inputs.cuda_normal((N, 128, 56, 56), seed)
        o = torch.empty((N, 128 * 9, 56 * 56), device="cuda")
        keep += [x, o]
        return H.task_im2col(x, o, 3, 3, 1, 1)
    if kind == H.HF_UPSAMPLE:
        x = inputs.cuda_normal((N, 64, 128, 128), seed)
        o = torch.empty((N, 64, 256, 256), device="cuda")
        keep += [x, o]
        return H.task_upsample(x, o, 2)
    x = inputs.cuda_normal((N, 64, 112, 112), seed)
    osh = H.maxpool_out_shape((N, 64, 112, 112), 3, 3, 2, 1)
    o, oi = torch.empty(osh, device="cuda"), torch.empty(osh, dtype=torch.int32, device="cuda")
    keep += [x, o, oi]
    return H.task_maxpool(x, o, oi, 3, 3, 2, 1)


MEMMEM = [  # (fixed kind, its batch, varied kind, batches)
    (H.HF_BN_STATS, 64, H.HF_MAXPOOL, (8, 16, 32, 64, 128)),
    (H.HF_BN_STATS, 64, H.HF_UPSAMPLE, (4, 8, 16, 32)),
    (H.HF_BN_STATS, 64, H.HF_IM2COL, (4, 8, 16, 32)),
    (H.HF_IM2COL, 32, H.HF_MAXPOOL, (8, 16, 32, 64, 128)),
    (H.HF_IM2COL, 32, H.HF_UPSAMPLE, (4, 8, 16, 32)),
    (H.HF_MAXPOOL, 64, H.HF_UPSAMPLE, (4, 8, 16, 32)),
]


def memmem(res, reps):
    import torch
    for kf, nf, kv, batches in MEMMEM:
        keep = []
        fixed = image_task(kf, nf, 40 + kf, keep)
        name = f"{H.KIND_NAMES[kf]}+{H.KIND_NAMES[kv]}*"
        rows = []
        for N in batches:
            kv_keep = []
            var = image_task(kv, N, 50 + kv, kv_keep)
            p = point(H.make_pair(fixed, var), reps)
            p["batch"] = N
            p["ratio_star_over_other"] = round(p["t_b_ms"] / p["t_a_ms"], 3)
            rows.append(p)
            print(name, N, p["ratio_star_over_other"], p["speedup_pct"], flush=True)
            del kv_keep, var
            torch.cuda.empty_cache()
        res[name] = rows
        del keep, fixed
        torch.cuda.empty_cache()


def crypto(res, reps):
    import torch
    # the crypto pairs
    hdr = torch.from_numpy(inputs.header80(31).view(np.int32)).cuda()
    table = inputs.cuda_eth_table(1 << 23, 32)
    n0 = inputs.nonce0(31)

    def hashes(kind, n):
        o = torch.empty((n, 8), dtype=torch.int32, device="cuda")
        if kind == H.HF_ETHASH:
            return H.task_ethash(hdr, table, o, n0, n), o
        return (H.task_sha256d if kind == H.HF_SHA256D else H.task_blake2b)(hdr, o, n0, n), o

    sha, sha_o = hashes(H.HF_SHA256D, 1 << 22)
    rows = []
    for k in (15, 16, 17, 18, 19, 20):
        et, eo = hashes(H.HF_ETHASH, 1 << k)
        p = point(H.make_pair(et, sha), reps)
        p["log2_hashes"] = k
        p["ratio_star_over_other"] = round(p["t_a_ms"] / p["t_b_ms"], 3)
        rows.append(p)
        print("ethash* + sha256d", k, p["ratio_star_over_other"], p["speedup_pct"], flush=True)
    res["ethash*+sha256d"] = rows
    eth, eth_o = hashes(H.HF_ETHASH, 5 << 16)
    for name, other in (("blake2b*+ethash", eth), ("sha256d+blake2b*", sha)):
        rows = []
        for k in (20, 21, 22, 23, 24):
            bt, bo = hashes(H.HF_BLAKE2B, 1 << k)
            p = point(H.make_pair(bt, other), reps)
            p["log2_hashes"] = k
            p["ratio_star_over_other"] = round(p["t_a_ms"] / p["t_b_ms"], 3)
            rows.append(p)
            print(name, k, p["ratio_star_over_other"], p["speedup_pct"], flush=True)
        res[name] = rows


SETS = ("data", "crypto", "memmem")


def parse_sets(spec: str) -> set:
    """The groups named by ``--sets``: ``paper`` stands for data and crypto."""
    out = set()
    for s in (x.strip() for x in spec.split(",") if x.strip()):
        if s == "paper":
            out |= {"data", "crypto"}
        elif s in SETS:
            out.add(s)
        else:
            raise SystemExit(f"unknown set {s!r}: choose from paper, {', '.join(SETS)}")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=15)
    ap.add_argument("--out", default="")
    ap.add_argument("--sets", default="paper,memmem",
                    help="comma-separated: paper (= data,crypto), data, crypto, memmem")
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    H.hf_init()
    H.hf_warmup(300)
    res = {}
    sets = parse_sets(a.sets)
    if "memmem" in sets:
        memmem(res, a.reps)
    if "data" not in sets:
        if "crypto" in sets:
            crypto(res, a.reps)
        return finish(res, a.out)

    def zipf(n, seed):
        return inputs.cuda_zipf_u8(n, seed)

    # bn_stats fixed + int_mix* (rounds varied)
    x = inputs.cuda_normal((64, 256, 56, 56), 10)
    mean, var = torch.empty(256, device="cuda"), torch.empty(256, device="cuda")
    bn = H.task_bn_stats(x, mean, var)
    seeds = inputs.cuda_uint32(1 << 24, 11)
    out = torch.empty_like(seeds)
    rows = []
    for r in (1, 2, 4, 8, 16, 32, 64, 128):
        p = point(H.make_pair(bn, H.task_int_mix(seeds, out, r)), a.reps)
        p["rounds"] = r
        p["ratio_star_over_other"] = round(p["t_b_ms"] / p["t_a_ms"], 3)
        rows.append(p)
        print("bn_stats + int_mix*", r, p["ratio_star_over_other"], p["speedup_pct"], flush=True)
    res["bn_stats+int_mix*"] = rows
    del seeds, out

    # bn_stats* (batch varied) + lds_hist fixed
    h = zipf(1 << 26, 12)
    counts = torch.empty(256, dtype=torch.int32, device="cuda")
    hist = H.task_lds_hist(h, counts)
    rows = []
    for N in (4, 8, 16, 32, 64, 128):
        xb = inputs.cuda_normal((N, 256, 56, 56), 13)
        p = point(H.make_pair(H.task_bn_stats(xb, mean, var), hist), a.reps)
        p["batch"] = N
        p["ratio_star_over_other"] = round(p["t_a_ms"] / p["t_b_ms"], 3)
        rows.append(p)
        print("bn_stats* + lds_hist", N, p["ratio_star_over_other"], p["speedup_pct"], flush=True)
        del xb
    res["bn_stats*+lds_hist"] = rows
    del x

    # im2col / upsample fixed + lds_hist* (bytes varied)
    xi = inputs.cuda_normal((32, 128, 56, 56), 14)
    cols = torch.empty((32, 128 * 9, 56 * 56), device="cuda")
    im = H.task_im2col(xi, cols, 3, 3, 1, 1)
    xu = inputs.cuda_normal((32, 64, 128, 128), 15)
    up_out = torch.empty((32, 64, 256, 256), device="cuda")
    up = H.task_upsample(xu, up_out, 2)
    for name, t in (("im2col+lds_hist*", im), ("upsample+lds_hist*", up)):
        rows = []
        for k in (22, 23, 24, 25, 26, 27, 28):
            hk = zipf(1 << k, 16 + k)
            p = point(H.make_pair(t, H.task_lds_hist(hk, counts)), a.reps)
            p["log2_hist_bytes"] = k
            p["ratio_star_over_other"] = round(p["t_b_ms"] / p["t_a_ms"], 3)
            rows.append(p)
            print(name, k, p["ratio_star_over_other"], p["speedup_pct"], flush=True)
            del hk
        res[name] = rows
    # maxpool* (batch varied) + lds_hist fixed
    rows = []
    for N in (4, 8, 16, 32, 64, 128):
        xp = inputs.cuda_normal((N, 64, 112, 112), 30)
        osh = H.maxpool_out_shape((N, 64, 112, 112), 3, 3, 2, 1)
        po, pi = torch.empty(osh, device="cuda"), torch.empty(osh, dtype=torch.int32, device="cuda")
        p = point(H.make_pair(H.task_maxpool(xp, po, pi, 3, 3, 2, 1), hist), a.reps)
        p["batch"] = N
        p["ratio_star_over_other"] = round(p["t_a_ms"] / p["t_b_ms"], 3)
        rows.append(p)
        print("maxpool* + lds_hist", N, p["ratio_star_over_other"], p["speedup_pct"], flush=True)
        del xp, po, pi
    res["maxpool*+lds_hist"] = rows
    del h, xi, cols, xu, up_out
    torch.cuda.empty_cache()

    if "crypto" in sets:
        crypto(res, a.reps)
    return finish(res, a.out)


def finish(res, out):
    summary = {}
    for name, rows in list(res.items()):
        summary[name] = {m: round(float(np.mean([r["speedup_pct"][m] for r in rows])), 2)
                         for m in ("hfuse", "naive", "vfuse", "streams")}
    res["mean_speedup_pct"] = summary
    print(json.dumps(summary), flush=True)
    if out:
        json.dump(res, open(out, "w"), indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
