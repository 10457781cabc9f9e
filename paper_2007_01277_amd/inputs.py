"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers; it holds none of the kernels' arithmetic,
so the GPU path and the CPU oracle can both be fed the same bytes without
sharing any computation.  Every generator is numpy PCG64 with an explicit seed.

Distributions (the paper never states its input sizes or values, so these are
the synthetic stand-ins for its PyTorch and mining workloads):
  * batch-norm input: x[n,c,h,w] = z * scale_c + shift_c with z ~ N(0,1),
    scale_c ~ U[0.5, 2], shift_c ~ U[-1, 1]  (parameters from ``seed + 1``)
  * images for im2col and upsample: N(0, 1)
  * integer mixing seeds: uniform uint32
  * histogram input: uint8 values from a Zipf law with exponent 1.2 truncated to
    ranks 1..256 (value = rank - 1), drawn by inverse CDF
  * hash kernels: an 80-byte block header of uniform bytes and a first nonce
    of uniform uint32; the Ethash-like table: uniform uint32 rows of 32 words
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def bn_input(shape, seed: int = 0) -> np.ndarray:
    N, C, H, W = shape
    prm = rng(seed + 1)
    scale = prm.uniform(0.5, 2.0, size=C).astype(np.float32)
    shift = prm.uniform(-1.0, 1.0, size=C).astype(np.float32)
    g = rng(seed)
    x = np.empty(shape, np.float32)
    for n in range(N):  # plane by plane keeps the float64 temporaries small
        z = g.standard_normal(size=(C, H, W), dtype=np.float32)
        x[n] = z * scale[:, None, None] + shift[:, None, None]
    return x


def normal_image(shape, seed: int = 0) -> np.ndarray:
    g = rng(seed)
    x = np.empty(shape, np.float32)
    flat = x.reshape(shape[0], int(np.prod(shape[1:])))
    for n in range(shape[0]):
        flat[n] = g.standard_normal(size=flat.shape[1], dtype=np.float32)
    return x


def uint32_seeds(n: int, seed: int = 0) -> np.ndarray:
    return rng(seed).integers(0, 2**32, size=n, dtype=np.uint32)


def zipf_cdf(s: float = 1.2, ranks: int = 256) -> np.ndarray:
    w = 1.0 / np.arange(1, ranks + 1, dtype=np.float64) ** s
    c = np.cumsum(w)
    return c / c[-1]


def zipf_u8(n: int, s: float = 1.2, seed: int = 0, chunk: int = 1 << 22) -> np.ndarray:
    cdf = zipf_cdf(s)
    g = rng(seed)
    out = np.empty(n, np.uint8)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        u = g.random(hi - lo)
        r = np.searchsorted(cdf, u, side="right")
        out[lo:hi] = np.minimum(r, 255).astype(np.uint8)
    return out


def uniform_u8(n: int, seed: int = 0) -> np.ndarray:
    return rng(seed).integers(0, 256, size=n, dtype=np.uint8)


# ------------------------------------------------------------------ on-device generators
# Seeded draws made directly on the GPU (torch's Philox generator) for large
# timing workloads; the same distributions as above, different streams of
# numbers.  Tests copy the device values back to the host before checking them
# against the oracle.
def header80(seed: int = 0) -> np.ndarray:
    """An 80-byte block header (uint8)."""
    return rng(seed).integers(0, 256, size=80, dtype=np.uint8)


def nonce0(seed: int = 0) -> int:
    return int(rng(seed + 1).integers(0, 2 ** 32, dtype=np.uint64))


def eth_table(rows: int, seed: int = 0) -> np.ndarray:
    """The synthetic table of the Ethash-like kernel: uint32 [rows][32]."""
    return rng(seed).integers(0, 2 ** 32, size=(rows, 32), dtype=np.uint64).astype(np.uint32)


def cuda_generator(seed: int):
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return g


def cuda_normal(shape, seed: int):
    import torch
    return torch.randn(shape, generator=cuda_generator(seed), device="cuda")


def cuda_uint32(n: int, seed: int):
    import torch
    return torch.randint(-2**31, 2**31 - 1, (n,), generator=cuda_generator(seed), device="cuda", dtype=torch.int32)


def cuda_zipf_u8(n: int, seed: int, s: float = 1.2):
    import torch
    cdf = torch.from_numpy(zipf_cdf(s)).to("cuda")
    u = torch.rand(n, generator=cuda_generator(seed), device="cuda", dtype=torch.float64)
    return torch.clamp(torch.searchsorted(cdf, u, right=True), max=255).to(torch.uint8)


def cuda_eth_table(rows: int, seed: int):
    """A device table of uniform uint32 words [rows][32] (int32 storage)."""
    import torch
    return torch.randint(-2**31, 2**31 - 1, (rows, 32), generator=cuda_generator(seed), device="cuda",
                         dtype=torch.int32)
