"""Learned tuner: sample collection, training and regret against the exhaustive search.

Workload: random pairs of two distinct kinds drawn from the nine kernels, each
of 2^k elements with k uniform in [16, 26] (image kinds as [2^k / 65536, 64, 32,
32], integer mixing with 32 rounds, histogram bytes from the Zipf law; the
hashes count a SHA-256d or BLAKE2b instance as 64 elements and an Ethash-like
instance, over a shared 1 GiB table, as 256).  For
every pair the tuner's own profiler times every candidate of the exhaustive
search (median of ``reps`` launches), and ``hf_featurize`` gives the model's
features.  Cross-validation is by pair: the model is trained on a random subset
of ``per_pair`` configurations of each training pair (600 pairs x 14 = about
6300 training samples per fold at the defaults: the sample budget is spread
over many pairs, which generalises far better than many configurations of few
pairs) and evaluated on the held-out pairs, where it ranks all candidates and
only the top k are "profiled" (their measured times are looked up).
Regret = T(choice) / T(exhaustive best) - 1.

Baselines without the network: the even split at block 1024 without a bound
("naive", Sec. IV-A), the even split with the register bound r0 of Sec. III-B
("r0"), and k candidates drawn at random.

    python -m paper_2007_01277_amd.learned_tuner --pairs 40 --out tuner.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import hfuse as H
from . import inputs

IMAGE = (64, 32, 32)  # C, H, W of the image kinds: 65536 elements per batch entry


DATA_KINDS = (H.HF_BN_STATS, H.HF_UPSAMPLE, H.HF_IM2COL, H.HF_LDS_HIST, H.HF_INT_MIX)  # the five of the C4 set


def draw_pairs(n_pairs: int, seed: int = 2, kmin: int = 16, kmax: int = 26, kinds=None):
    kinds = np.asarray(range(len(H.KIND_NAMES)) if kinds is None else kinds)
    g = inputs.rng(seed)
    out = []
    for _ in range(n_pairs):
        a, b = kinds[g.choice(len(kinds), size=2, replace=False)]
        ka, kb = g.integers(kmin, kmax + 1, size=2)
        out.append((int(a), int(b), int(ka), int(kb)))
    return out


class Instance:
    """Device buffers of one task of `kind` with 2^k elements (values only
    shape the timing; they are drawn on the GPU from a seeded generator)."""

    def __init__(self, kind: int, k: int, seed: int):
        import torch
        n = 1 << k
        self.bufs = []
        if kind in (H.HF_BN_STATS, H.HF_IM2COL, H.HF_UPSAMPLE, H.HF_MAXPOOL):
            N = n // 65536
            x = inputs.cuda_normal((N,) + IMAGE, seed)
            self.bufs.append(x)
            if kind == H.HF_BN_STATS:
                m, v = torch.empty(IMAGE[0], device="cuda"), torch.empty(IMAGE[0], device="cuda")
                self.bufs += [m, v]
                self.task = H.task_bn_stats(x, m, v)
            elif kind == H.HF_IM2COL:
                o = torch.empty((N, IMAGE[0] * 9, IMAGE[1] * IMAGE[2]), device="cuda")
                self.bufs.append(o)
                self.task = H.task_im2col(x, o, 3, 3, 1, 1)
            elif kind == H.HF_UPSAMPLE:
                o = torch.empty((N, IMAGE[0], 2 * IMAGE[1], 2 * IMAGE[2]), device="cuda")
                self.bufs.append(o)
                self.task = H.task_upsample(x, o, 2)
            else:
                osh = H.maxpool_out_shape((N,) + IMAGE, 3, 3, 2, 1)
                o, oi = torch.empty(osh, device="cuda"), torch.empty(osh, dtype=torch.int32, device="cuda")
                self.bufs += [o, oi]
                self.task = H.task_maxpool(x, o, oi, 3, 3, 2, 1)
        elif kind == H.HF_INT_MIX:
            s = inputs.cuda_uint32(n, seed)
            o = torch.empty_like(s)
            self.bufs += [s, o]
            self.task = H.task_int_mix(s, o, 32)
        elif kind in (H.HF_SHA256D, H.HF_BLAKE2B, H.HF_ETHASH):
            # a hash does the work of about 64 (256 for the table walk) elements
            hdr = torch.from_numpy(inputs.header80(seed).view(np.int32)).cuda()
            m = n >> (8 if kind == H.HF_ETHASH else 6)
            o = torch.empty((max(m, 1), 8), dtype=torch.int32, device="cuda")
            self.bufs += [hdr, o]
            if kind == H.HF_ETHASH:
                tab = eth_table()
                self.task = H.task_ethash(hdr, tab, o, inputs.nonce0(seed), m)
            elif kind == H.HF_SHA256D:
                self.task = H.task_sha256d(hdr, o, inputs.nonce0(seed), m)
            else:
                self.task = H.task_blake2b(hdr, o, inputs.nonce0(seed), m)
        else:
            x = inputs.cuda_zipf_u8(n, seed)
            o = torch.empty(256, dtype=torch.int32, device="cuda")
            self.bufs += [x, o]
            self.task = H.task_lds_hist(x, o)


_ETH = []


def eth_table():
    """The Ethash-like table shared by every instance: 1 GiB, past the 256 MB
    last-level cache, as a mining table is."""
    if not _ETH:
        _ETH.append(inputs.cuda_eth_table(1 << 23, 77))
    return _ETH[0]


def r0_config(kind_a: int, kind_b: int) -> H.hf_config:
    """Even split of a 1024-lane workgroup with the register bound r0."""
    va = H.hf_solo_info(kind_a, 1024)["vgprs"]
    vb = H.hf_solo_info(kind_b, 1024)["vgprs"]
    lds = H.hf_fused_info(kind_a, kind_b, 1024, 0)["lds_bytes"]
    r0 = H.hf_register_bound(512, 512, va, vb, lds)
    cap = max([c for c in (64, 80, 96, 128) if c <= r0] or [64])
    return H.hf_config(8, 1024, cap, 0)


def _store_key(p, pair, seed, reps):
    """Key of one pair's samples: position, kinds, sizes, seed, repetitions and
    the hash of the kernel sources they were measured on."""
    from .rocprof_summary import csrc_hash
    ka, kb, ea, eb = pair
    return f"{p}:{ka},{kb},{ea},{eb}:seed{seed}:reps{reps}:{csrc_hash()}"


def _load_store(path):
    done = {}
    if path and os.path.exists(path):
        with open(path) as fh:
            for ln in fh:
                try:
                    r = json.loads(ln)
                except ValueError:  # a line cut short by an interrupted run
                    continue
                done[r["key"]] = r
    return done


def _append(path, rec):
    """Appends one JSON line; a line left unterminated by an interrupted run is
    closed first, so the new record starts a line of its own."""
    lead = ""
    if os.path.exists(path) and os.path.getsize(path) > 0:
        with open(path, "rb") as fh:
            fh.seek(-1, os.SEEK_END)
            lead = "" if fh.read(1) == b"\n" else "\n"
    with open(path, "a") as fh:
        fh.write(lead + json.dumps(rec) + "\n")


def collect(pairs, reps: int = 10, seed: int = 2, log=sys.stderr, store: str = "", check: bool = False):
    """Profiles every exhaustive candidate of every pair; returns a dict of
    numpy arrays (features X, log2 times y, pair index, candidate index).
    With `check`, every candidate of a pair is profiled a second time after
    the first sweep over them (y_check): selections made on y are then judged
    on measurements they were not made on.
    With `store`, each pair's samples are appended to that JSON-lines file as
    soon as they are measured, and pairs already in it (same key, see
    _store_key) are read back instead of profiled again, so an interrupted
    sweep resumes where it stopped."""
    import torch
    cands = H.hf_tune_candidates(H.HF_TUNE_EXHAUSTIVE, 0)
    keys = [c.as_tuple() for c in cands]
    Xs, ys, y2s, pid, cid = [], [], [], [], []
    done = _load_store(store) if not check else {}
    t0 = time.time()
    for p, (ka, kb, ea, eb) in enumerate(pairs):
        key = _store_key(p, (ka, kb, ea, eb), seed, reps)
        if key in done:
            X = np.asarray(done[key]["X"], np.float32)
            y = np.asarray(done[key]["y"], np.float64)
            Xs.append(X)
            ys.append(y)
            pid += [p] * len(cands)
            cid += list(range(len(cands)))
            continue
        ia = Instance(ka, ea, seed * 1000 + 2 * p)
        ib = Instance(kb, eb, seed * 1000 + 2 * p + 1)
        pr = H.make_pair(ia.task, ib.task)
        X = H.hf_featurize(pr, cands)
        y = np.array([math.log2(H.hf_profile(pr, c, reps)) for c in cands])
        if check:
            y2s.append(np.array([math.log2(H.hf_profile(pr, c, reps)) for c in cands]))
        if store and not check:
            _append(store, {"key": key, "X": X.tolist(), "y": y.tolist()})
        Xs.append(X)
        ys.append(y)
        pid += [p] * len(cands)
        cid += list(range(len(cands)))
        print(f"pair {p} {H.KIND_NAMES[ka]}(2^{ea}) + {H.KIND_NAMES[kb]}(2^{eb}): best {2 ** y.min():.4f} ms "
              f"at {keys[int(np.argmin(y))]}  [{time.time() - t0:.1f}s]", file=log, flush=True)
        del ia, ib, pr
        torch.cuda.empty_cache()
    out = {"X": np.concatenate(Xs), "y": np.concatenate(ys), "pair": np.array(pid), "cand": np.array(cid),
           "cands": keys, "pairs": pairs}
    if check:
        out["y_check"] = np.concatenate(y2s)
    return out


SUM_SOLO = H.MLP_FEATURES - 1  # feature index of log2(sum of the best solo times)
MEMBERS = 5  # networks of the cost model's ensemble


def pick_topk(pred, cands, k):
    """Indices of the k best-predicted candidates with pairwise distinct
    (split, block), as hf_tune(MLP) picks them."""
    top, seen = [], set()
    for i in np.argsort(pred, kind="stable"):
        key = (cands[i][0], cands[i][1])
        if key not in seen:
            top.append(int(i))
            seen.add(key)
        if len(top) == k:
            break
    return np.array(top)
PER_KERNEL = len(H.KIND_NAMES) + 7  # features per kernel; the first kernel's come first
FEATURE_LAUNCHES = 2 * 3 * 6  # featurisation: each kernel alone at three block sizes, six launches each
TUNE_REPS = 20  # hf_tune's timed launches per candidate (after one untimed launch)


def featurisation_ms(x) -> float:
    """Time the featurisation's solo launches take, from one candidate's
    features: six launches of each kernel at each block size, whose median
    times are features (log2 ms) of the candidate."""
    t = 0.0
    for k in range(2):
        o = PER_KERNEL * k + len(H.KIND_NAMES)
        t += 6.0 * sum(2.0 ** float(x[o + b]) for b in range(3))
    return t


CLIP = 0.3  # training targets above a pair's best by more than this (log2) are clipped to it


def evaluate(data, folds: int = 4, per_pair: int = 14, topk: int = 3, epochs: int = 500,
             lr: float = 1e-3, seed: int = 7, ks=(1, 2, 3, 5, 8, 12), members: int = MEMBERS,
             clip: float = CLIP):
    """Regret of the learned tuner on held-out pairs.  The model (an ensemble
    of `members` networks) is trained on t_rel = log2(T_fused) - log2(t_a +
    t_b), which removes each pair's scale; per training pair the targets are
    clipped at the pair's best + `clip` (a configuration 2^0.3 = 1.23 times
    slower than the best, or more, is "bad" and its exact slowness is noise
    for the choice) and centred.  The order of the predictions within a pair
    is what the tuner uses, profiling the k best with distinct (split, block)
    (pick_topk).

    Regret = T(best of the k profiled) / T(exhaustive best) - 1 on the
    measurements the choices were made on.  With a second measurement of every
    candidate (data["y_check"]), the `*_checked` figures judge the same
    choices on it: the method's pick (the best of its k on the first
    measurement) against the exhaustive search's pick (the best of all on the
    first measurement).  The exhaustive best of one noisy measurement is the
    minimum of 85 noisy values and sits below what that configuration delivers
    on the next run; the checked regret compares what each method's choice
    delivers."""
    X, y, pair, cand = data["X"], data["y"], data["pair"], data["cand"]
    y2 = data.get("y_check")
    yrel = y - X[:, SUM_SOLO]
    keys = data["cands"]
    npairs = int(pair.max()) + 1
    g = inputs.rng(seed)
    order = g.permutation(npairs)
    naive = keys.index((8, 1024, 0, 0))
    res = {"per_pair": [], "folds": folds, "topk": topk, "per_pair_train": per_pair, "epochs": epochs,
           "n_candidates": len(keys)}
    train_loss = []
    for f in range(folds):
        test = set(order[f::folds].tolist())
        tr = [i for i in range(len(y)) if pair[i] not in test]
        # ~per_pair random configurations of each training pair
        keep = []
        for p in sorted(set(pair[tr].tolist())):
            idx = [i for i in tr if pair[i] == p]
            keep += g.choice(idx, size=min(per_pair, len(idx)), replace=False).tolist()
        keep = np.array(sorted(keep))
        # targets clipped and centred per training pair: only the order near
        # the top within a pair is used, and a pair's level is what the
        # features predict worst
        yt = yrel[keep].copy()
        for p in set(pair[keep].tolist()):
            m = pair[keep] == p
            if clip > 0:
                yt[m] = np.minimum(yt[m], yt[m].min() + clip)
            yt[m] -= yt[m].mean()
        H.hf_mlp_init(X.shape[1], 1000 * (seed + f), members=members)
        train_loss.append(H.hf_mlp_train(X[keep], yt, epochs=epochs, lr=lr))
        for p in sorted(test):
            idx = np.where(pair == p)[0]
            ty = y[idx]
            pred = H.hf_mlp_predict(X[idx])
            ck = [keys[c] for c in cand[idx]]
            top = pick_topk(pred, ck, topk)
            best = ty.min()
            ka, kb = data["pairs"][p][0], data["pairs"][p][1]
            r0 = r0_config(ka, kb).as_tuple()
            rnd = g.choice(len(idx), size=topk, replace=False)
            rperm = g.permutation(len(idx))
            rec = {"pair": p, "kinds": [H.KIND_NAMES[ka], H.KIND_NAMES[kb]],
                   "log2_sizes": list(data["pairs"][p][2:]),
                   "best_ms": float(2 ** best),
                   "regret_mlp_at_k": {int(k): float(2 ** (ty[pick_topk(pred, ck, k)].min() - best) - 1)
                                       for k in ks},
                   "regret_random_at_k": {int(k): float(2 ** (ty[rperm[:k]].min() - best) - 1) for k in ks},
                   "regret_mlp": float(2 ** (ty[top].min() - best) - 1),
                   "regret_naive": float(2 ** (ty[naive] - best) - 1),
                   "regret_r0": float(2 ** (ty[keys.index(r0)] - best) - 1),
                   "regret_random": float(2 ** (ty[rnd].min() - best) - 1),
                   "rank_corr": float(np.corrcoef(np.argsort(np.argsort(pred)), np.argsort(np.argsort(ty)))[0, 1]),
                   # profiling cost of the learned tuner (featurisation + its top k) over the exhaustive one
                   "cost_fraction": float((featurisation_ms(X[idx[0]]) + (TUNE_REPS + 1) * np.sum(2.0 ** ty[top]))
                                          / ((TUNE_REPS + 1) * np.sum(2.0 ** ty))),
                   # within-pair error: both sides centred (the targets were)
                   "pred_rmse_log2": float(np.sqrt(np.mean(((pred - pred.mean()) - (yrel[idx] - yrel[idx].mean()))
                                                           ** 2)))}
            if y2 is not None:
                cy = y2[idx]
                ex = int(np.argmin(ty))  # the exhaustive search's choice
                pick = int(top[np.argmin(ty[top])])  # the learned tuner's choice after profiling its k
                rpick = int(rnd[np.argmin(ty[rnd])])
                rec.update({"regret_mlp_checked": float(2 ** (cy[pick] - cy[ex]) - 1),
                            "regret_naive_checked": float(2 ** (cy[naive] - cy[ex]) - 1),
                            "regret_random_checked": float(2 ** (cy[rpick] - cy[ex]) - 1),
                            # the exhaustive choice on its second measurement against that measurement's best
                            "exhaustive_checked": float(2 ** (cy[ex] - cy.min()) - 1)})
            res["per_pair"].append(rec)
    pp = res["per_pair"]
    for k in ("regret_mlp", "regret_naive", "regret_r0", "regret_random", "rank_corr", "pred_rmse_log2",
              "cost_fraction"):
        v = np.array([r[k] for r in pp])
        res[k + "_mean"] = float(v.mean())
        res[k + "_max"] = float(v.max())
    if y2 is not None:
        for k in ("regret_mlp_checked", "regret_naive_checked", "regret_random_checked", "exhaustive_checked"):
            v = np.array([r[k] for r in pp])
            res[k + "_mean"] = float(v.mean())
            res[k + "_max"] = float(v.max())
        res["within_5pct_mlp_checked"] = float(np.mean([r["regret_mlp_checked"] <= 0.05 for r in pp]))
    res["within_5pct_mlp"] = float(np.mean([r["regret_mlp"] <= 0.05 for r in pp]))
    res["regret_mlp_mean_at_k"] = {int(k): float(np.mean([r["regret_mlp_at_k"][k] for r in pp])) for k in ks}
    res["regret_random_mean_at_k"] = {int(k): float(np.mean([r["regret_random_at_k"][k] for r in pp])) for k in ks}
    res["profiled_fraction"] = topk / len(keys)
    res["feature_launches"] = FEATURE_LAUNCHES
    res["train_loss"] = [float(v) for v in train_loss]
    res["n_samples"] = int(len(y))
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=600)
    ap.add_argument("--per-pair", type=int, default=14)
    ap.add_argument("--kmin", type=int, default=16)
    ap.add_argument("--kmax", type=int, default=26)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--folds", type=int, default=4)
    ap.add_argument("--topk", type=int, default=3)
    ap.add_argument("--epochs", type=int, default=500)
    ap.add_argument("--out", default="")
    ap.add_argument("--save-samples", default="")
    ap.add_argument("--store", default="", help="JSON-lines sample store: append as measured, resume from it")
    ap.add_argument("--collect-only", action="store_true")
    ap.add_argument("--check", action="store_true",
                    help="profile every candidate a second time and report the regret of the choices on it")
    ap.add_argument("--kinds", default="", help="comma-separated kind names to draw from (default: all nine)")
    a = ap.parse_args(argv)
    kinds = [H.KIND_NAMES.index(k) for k in a.kinds.split(",")] if a.kinds else None
    import torch
    torch.cuda.set_device(0)
    H.hf_init()
    H.hf_warmup(300)
    pairs = draw_pairs(a.pairs, kmin=a.kmin, kmax=a.kmax, kinds=kinds)
    data = collect(pairs, reps=a.reps, store=a.store, check=a.check)
    if a.save_samples:
        extra = {"y_check": data["y_check"]} if a.check else {}
        np.savez(a.save_samples, X=data["X"], y=data["y"], pair=data["pair"], cand=data["cand"],
                 cands=np.array(data["cands"]), pairs=np.array(pairs), **extra)
    if a.collect_only:
        return 0
    res = evaluate(data, folds=a.folds, per_pair=a.per_pair, topk=a.topk, epochs=a.epochs)
    summary = {k: v for k, v in res.items() if k != "per_pair"}
    print(json.dumps(summary), flush=True)
    if a.out:
        json.dump(res, open(a.out, "w"), indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
