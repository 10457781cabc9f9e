"""Seeded GPU test cases: device buffers for one task of each kind, plus the
check of its outputs against the CPU oracle.

Tolerances (written here, used by every GPU test):
  * integer and copy kernels (int_mix, lds_hist, im2col): bit-exact;
  * maxpool: bit-exact values (NaN where the oracle has NaN) and indices, since
    a maximum is one of its inputs;
  * hash kernels (sha256d, blake2b, ethash): bit-exact digests;
  * bn_stats: |d mean| <= 1e-5 * (|mean| + sigma) and |d var| <= 1e-5 * var
    (a relative bound on the mean alone is ill-posed when the mean is ~0);
  * upsample: |d out| <= 1e-5 * sum_k |w_k x_k| over the four taps.
"""
from __future__ import annotations

import contextlib
import functools
import hashlib

import numpy as np
import torch

import oracle
from oracle import hashes as OH
from paper_2007_01277_amd import hfuse as H
from paper_2007_01277_amd import inputs

DEV = "cuda"
TOL = 1e-5


@contextlib.contextmanager
def parallel_oracle():
    """Runs the oracle's OpenMP build inside the block (the same results as the
    sequential build, which a CPU test checks): full-size checks over every
    element then take seconds instead of minutes."""
    oracle.use_openmp(True)
    try:
        yield
    finally:
        oracle.use_openmp(False)


def dev(a: np.ndarray, offset: int = 0) -> torch.Tensor:
    """Device copy of `a`; with offset > 0 the tensor is a view that starts
    `offset` elements into a larger allocation (misaligned for vector loads)."""
    t = torch.from_numpy(np.ascontiguousarray(a))
    if offset == 0:
        return t.to(DEV)
    flat = t.reshape(-1)
    big = torch.zeros(flat.numel() + offset, dtype=flat.dtype, device=DEV)
    big[offset:] = flat.to(DEV)
    return big[offset:].view(a.shape)


class Case:
    """One task with its device buffers and host-side expected values."""

    def __init__(self, task, bufs, check, label):
        self.task, self.bufs, self.check, self.label = task, bufs, check, label

    def outputs(self):
        return [b.clone() for b in self.bufs["outs"]]

    def reset(self):
        for o in self.bufs["outs"]:
            o.fill_(0xCD if o.dtype == torch.uint8 else 7)


def bn_case(shape, seed=0, offset=0, x=None) -> Case:
    xh = inputs.bn_input(shape, seed) if x is None else x
    xd = dev(xh, offset)
    C = shape[1]
    mean = torch.full((C,), 7.0, device=DEV)
    var = torch.full((C,), 7.0, device=DEV)
    t = H.task_bn_stats(xd, mean, var)
    ref = None

    def check(outs, channels=None):
        nonlocal ref
        sel = np.arange(C) if channels is None else np.asarray(channels)
        if ref is None or channels is not None:
            m_ref, v_ref = oracle.bn_stats(xh[:, sel])
            if channels is None:
                ref = (m_ref, v_ref)
        else:
            m_ref, v_ref = ref
        m = outs[0].cpu().numpy().astype(np.float64)[sel]
        v = outs[1].cpu().numpy().astype(np.float64)[sel]
        sd = np.sqrt(v_ref)
        assert np.all(np.abs(m - m_ref) <= TOL * (np.abs(m_ref) + sd)), (m - m_ref, sd)
        assert np.all(np.abs(v - v_ref) <= TOL * v_ref), (v - v_ref) / np.maximum(v_ref, 1e-300)

    return Case(t, {"in": xd, "outs": [mean, var]}, check, f"bn_stats{tuple(shape)}+{offset}")


def mix_case(n, rounds, seed=0, offset=0, sample=None) -> Case:
    sh = inputs.uint32_seeds(n, seed)
    sd = dev(sh.view(np.int32), offset)
    out = dev(np.zeros(n, np.int32), offset)
    t = H.task_int_mix(sd, out, rounds)

    def check(outs):
        got = outs[0].cpu().numpy().view(np.uint32)
        if sample is None:
            assert np.array_equal(got, oracle.int_mix(sh, rounds))
        else:
            idx = np.unique(np.concatenate([np.arange(min(n, 64)), np.arange(max(0, n - 64), n),
                                            inputs.rng(seed + 7).integers(0, n, size=sample)]))
            assert np.array_equal(got[idx], oracle.int_mix(sh[idx], rounds))

    return Case(t, {"in": sd, "outs": [out]}, check, f"int_mix({n},{rounds})+{offset}")


def hist_case(n, seed=0, offset=0, zipf=True) -> Case:
    xh = inputs.zipf_u8(n, seed=seed) if zipf else inputs.uniform_u8(n, seed)
    xd = dev(xh, offset)
    counts = torch.full((256,), 12345, dtype=torch.int32, device=DEV)
    t = H.task_lds_hist(xd, counts)

    def check(outs):
        got = outs[0].cpu().numpy().view(np.uint32).astype(np.uint64)
        assert np.array_equal(got, oracle.hist256(xh))

    return Case(t, {"in": xd, "outs": [counts]}, check, f"lds_hist({n})+{offset}")


def im2col_case(shape, k=(3, 3), s=1, p=1, seed=0, check_images=None) -> Case:
    xh = inputs.normal_image(shape, seed)
    xd = dev(xh)
    oshape, Ho, Wo = oracle.im2col_shape(*shape, k[0], k[1], s, p)
    out = torch.full(oshape, 7.0, device=DEV)
    t = H.task_im2col(xd, out, k[0], k[1], s, p)

    def check(outs):
        imgs = range(shape[0]) if check_images is None else check_images
        for i in imgs:
            ref = oracle.im2col(xh[i:i + 1], k[0], k[1], s, p)
            assert np.array_equal(outs[0][i:i + 1].cpu().numpy(), ref), f"image {i}"

    return Case(t, {"in": xd, "outs": [out]}, check, f"im2col{tuple(shape)}k{k}s{s}p{p}")


def up_case(shape, scale=2, seed=0, check_slice=None) -> Case:
    xh = inputs.normal_image(shape, seed)
    xd = dev(xh)
    N, C, Hh, W = shape
    out = torch.full((N, C, Hh * scale, W * scale), 7.0, device=DEV)
    t = H.task_upsample(xd, out, scale)

    def check(outs):
        if check_slice is not None:
            slices = [check_slice]
        else:  # image by image, so the double-precision references stay small
            slices = [(slice(i, i + 1), slice(None)) for i in range(N)]
        for sl in slices:
            xs = np.ascontiguousarray(xh[sl])
            ref = oracle.upsample(xs, scale)
            mag = oracle.upsample_absmag(xs, scale)
            got = outs[0][sl].cpu().numpy().astype(np.float64)
            err = np.abs(got - ref)
            assert np.all(err <= TOL * mag), (sl, float(np.max(err / np.maximum(mag, 1e-300))))

    return Case(t, {"in": xd, "outs": [out]}, check, f"upsample{tuple(shape)}x{scale}")


def pool_case(shape, k=(3, 3), s=2, p=1, seed=0, offset=0, with_idx=True, x=None, check_images=None) -> Case:
    xh = inputs.normal_image(shape, seed) if x is None else x
    xd = dev(xh, offset)
    oshape = H.maxpool_out_shape(shape, k[0], k[1], s, p)
    out = torch.full(oshape, 7.0, device=DEV)
    idx = torch.full(oshape, 7, dtype=torch.int32, device=DEV) if with_idx else None
    t = H.task_maxpool(xd, out, idx, k[0], k[1], s, p)

    def check(outs):
        imgs = range(shape[0]) if check_images is None else check_images
        for i in imgs:
            v, ix = oracle.maxpool(xh[i:i + 1], k[0], k[1], s, p)
            got = outs[0][i:i + 1].cpu().numpy()
            assert np.array_equal(got, v, equal_nan=True), f"values of image {i}"
            if with_idx:
                assert np.array_equal(outs[1][i:i + 1].cpu().numpy(), ix), f"indices of image {i}"

    outs = [out] if idx is None else [out, idx]
    return Case(t, {"in": xd, "outs": outs}, check, f"maxpool{tuple(shape)}k{k}s{s}p{p}+{offset}")


@functools.lru_cache(maxsize=None)
def _hash_ref(kind, hdr_bytes, nonce0, i, table_key):
    if kind == H.HF_SHA256D:
        return OH.sha256d(hdr_bytes, nonce0, [i])[0]
    if kind == H.HF_BLAKE2B:
        return OH.blake2b_header(hdr_bytes, nonce0, [i])[0]
    rows, seed = table_key
    return OH.ethash_like_one(hdr_bytes, nonce0 + i, _eth_table(rows, seed))


@functools.lru_cache(maxsize=4)
def _eth_table(rows, seed):
    return inputs.eth_table(rows, seed)


def hash_case(kind, n, seed=0, nonce0=None, rows=4099, sample=None, header=None) -> Case:
    """n instances of a hash kind; the oracle checks every instance, or the first
    and last 64 plus `sample` drawn ones.  `header` (80 bytes) replaces the
    seeded header."""
    hdr = inputs.header80(seed) if header is None else np.frombuffer(bytes(header), np.uint8).copy()
    n0 = inputs.nonce0(seed) if nonce0 is None else nonce0 & 0xFFFFFFFF
    hd = dev(hdr.view(np.int32))
    out = torch.full((max(n, 1), 8), 7, dtype=torch.int32, device=DEV)[:n]
    tkey = None
    if kind == H.HF_ETHASH:
        tkey = (rows, seed + 5)
        td = dev(_eth_table(*tkey).view(np.int32))
        t = H.task_ethash(hd, td, out, n0, n)
        bufs = {"in": hd, "table": td, "outs": [out]}
    else:
        t = (H.task_sha256d if kind == H.HF_SHA256D else H.task_blake2b)(hd, out, n0, n)
        bufs = {"in": hd, "outs": [out]}

    def check(outs, full=False):
        """Every instance against the plain-integer oracle, or (sample set) the
        first and last 64 plus `sample` drawn ones; with full=True also every
        instance against the C transcription of the Ethash-like walk, or against
        hashlib's SHA-256 / BLAKE2b (the library routines the oracle is pinned
        to)."""
        got = outs[0].cpu().numpy().view(np.uint8).reshape(n, 32)
        if sample is None:
            idx = range(n)
        else:
            idx = np.unique(np.concatenate([np.arange(min(n, 64)), np.arange(max(0, n - 64), n),
                                            inputs.rng(seed + 9).integers(0, max(n, 1), size=sample)]))
        for i in idx:
            ref = _hash_ref(kind, hdr.tobytes(), n0, int(i), tkey)
            assert got[i].tobytes() == ref, (H.KIND_NAMES[kind], int(i))
        if not full:
            return
        if kind == H.HF_ETHASH:
            ref = oracle.ethash_like(hdr.tobytes(), n0, _eth_table(*tkey), n)
            bad = np.nonzero(np.any(got != ref, axis=1))[0]
            assert bad.size == 0, ("ethash", bad[:8])
            return
        head = hdr.tobytes()[:76]
        for i in range(n):
            m = head + ((n0 + i) & 0xFFFFFFFF).to_bytes(4, "little")
            if kind == H.HF_SHA256D:
                d = hashlib.sha256(hashlib.sha256(m).digest()).digest()
            else:
                d = hashlib.blake2b(m, digest_size=32).digest()
            assert got[i].tobytes() == d, (H.KIND_NAMES[kind], i)

    return Case(t, bufs, check, f"{H.KIND_NAMES[kind]}({n},nonce0={n0:#x})")


def small_cases(kind, seed=0):
    """Small cases of one kind covering several tiles and a ragged tail."""
    if kind == H.HF_BN_STATS:
        return [bn_case((8, 32, 16, 16), seed), bn_case((3, 5, 7, 9), seed), bn_case((2, 3, 40, 52), seed, offset=1)]
    if kind == H.HF_INT_MIX:
        return [mix_case(65536, 32, seed), mix_case(100_003, 7, seed), mix_case(1029, 5, seed, offset=1)]
    if kind == H.HF_LDS_HIST:
        return [hist_case(1 << 20, seed), hist_case(100_003, seed, offset=3), hist_case(50_000, seed, zipf=False)]
    if kind == H.HF_IM2COL:
        # the first and the last six take the 3x3/s1/p1 row path (64-column
        # chunks in 16-lane groups: a width of 64 fills a chunk, 4 is one
        # float4 column, 68 leaves a chunk of one column, 200 and 1024 span
        # several chunks per row, heights not a multiple of 4 leave a partial
        # unit)
        return [im2col_case((2, 8, 14, 16), seed=seed), im2col_case((2, 3, 9, 11), (3, 3), 2, 1, seed),
                im2col_case((1, 4, 6, 7), (2, 3), 1, 0, seed), im2col_case((1, 3, 5, 64), seed=seed),
                im2col_case((2, 2, 2, 4), seed=seed), im2col_case((1, 5, 1, 60), seed=seed),
                im2col_case((1, 2, 5, 68), seed=seed), im2col_case((2, 2, 3, 200), seed=seed),
                im2col_case((1, 3, 6, 1024), seed=seed)]
    if kind == H.HF_UPSAMPLE:
        # the first and the last four take the scale-2 row path (32 input
        # columns per 16-lane group: 34 leaves a chunk of one lane, 68, 200 and
        # 1024 span several chunks per row); 33 is odd
        return [up_case((2, 8, 16, 16), 2, seed), up_case((1, 3, 5, 7), 3, seed), up_case((2, 2, 9, 33), 2, seed),
                up_case((1, 2, 4, 34), 2, seed), up_case((1, 2, 5, 68), 2, seed), up_case((1, 3, 3, 200), 2, seed),
                up_case((1, 2, 2, 1024), 2, seed)]
    if kind == H.HF_MAXPOOL:
        # the last six take the 3x3/s2/p1 row path (128 input columns per
        # 16-lane group: 128 fills one, 8 is one float4 of outputs, 136 leaves a
        # chunk of one lane, 256 and 1024 span several chunks per row, odd
        # heights clamp)
        return [pool_case((2, 8, 24, 20), seed=seed), pool_case((1, 3, 9, 11), (2, 2), 2, 0, seed, offset=1),
                pool_case((2, 2, 7, 13), (3, 2), 1, 1, seed, with_idx=False), pool_case((2, 3, 10, 16), seed=seed),
                pool_case((1, 2, 7, 128), seed=seed), pool_case((1, 4, 16, 8), seed=seed, with_idx=False),
                pool_case((1, 3, 6, 136), seed=seed), pool_case((1, 2, 7, 256), seed=seed),
                pool_case((2, 2, 5, 1024), seed=seed, with_idx=False)]
    if kind in (H.HF_SHA256D, H.HF_BLAKE2B, H.HF_ETHASH):
        # several waves of work, a ragged tail, and a nonce range that wraps past 2^32
        return [hash_case(kind, 1000, seed), hash_case(kind, 333, seed + 1, nonce0=0xFFFFFF00, rows=37),
                hash_case(kind, 67, seed + 2, rows=1)]
    raise ValueError(kind)


def run_and_check(run, cases):
    for c in cases:
        c.reset()
    run()
    torch.cuda.synchronize()
    for c in cases:
        c.check(c.outputs())
