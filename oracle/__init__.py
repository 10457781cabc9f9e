"""CPU oracle for horizontal fusion -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2007_01277_amd``) and never imports it.

The arithmetic lives in ``hf_oracle.c`` (plain loops, double accumulation);
this module only compiles it with gcc (a sequential and an OpenMP build of the
same source), loads it with ctypes and converts numpy arrays.  The
register-bound rule and the learned cost model's reference maths are in
``search.py`` and ``mlp.py`` of this package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_libs = {}
_use_omp = False


def build(force: bool = True) -> str:
    """Compile hf_oracle.c with gcc (-O2, no fast-math) twice: liboracle.so,
    sequential, and liboracle_omp.so, the same source with OpenMP."""
    for lib, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib):
            tmp = lib + ".tmp"
            subprocess.check_call(
                ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                 "-fvisibility=hidden"] + extra + [_SRC, "-o", tmp, "-lm"])
            os.replace(tmp, lib)
    return _LIB


def use_openmp(on: bool) -> None:
    """Route the oracle functions to the OpenMP build (True) or to the
    sequential build (False, the default)."""
    global _use_omp
    _use_omp = bool(on)


def threads() -> int:
    """Threads the current build's parallel loops use (1 when sequential)."""
    return int(_load().oracle_threads())


def _load():
    path = _LIB_OMP if _use_omp else _LIB
    lib = _libs.get(path)
    if lib is None:
        if not os.path.exists(path):
            build(force=False)
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int32
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_bn_stats.argtypes = [P, I64, I64, I64, I64, P, P]
        lib.oracle_bn_stats.restype = ctypes.c_int
        lib.oracle_int_mix.argtypes = [P, I64, I32, P]
        lib.oracle_int_mix.restype = None
        lib.oracle_hist256.argtypes = [P, I64, P]
        lib.oracle_hist256.restype = None
        lib.oracle_im2col.argtypes = [P, I64, I64, I64, I64, I32, I32, I32, I32, P]
        lib.oracle_im2col.restype = ctypes.c_int
        lib.oracle_upsample.argtypes = [P, I64, I64, I64, I64, I32, P]
        lib.oracle_upsample.restype = ctypes.c_int
        lib.oracle_upsample_absmag.argtypes = [P, I64, I64, I64, I64, I32, P]
        lib.oracle_upsample_absmag.restype = ctypes.c_int
        lib.oracle_maxpool.argtypes = [P, I64, I64, I64, I64, I32, I32, I32, I32, P, P]
        lib.oracle_maxpool.restype = ctypes.c_int
        lib.oracle_ethash_like.argtypes = [P, I64, P, I64, P]
        lib.oracle_ethash_like.restype = ctypes.c_int
        _libs[path] = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def bn_stats(x: np.ndarray):
    """Per-channel (mean, biased var) of float32 NCHW ``x`` in float64."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    N, C, H, W = x.shape
    mean = np.empty(C, np.float64)
    var = np.empty(C, np.float64)
    rc = _load().oracle_bn_stats(_ptr(x), N, C, H, W, _ptr(mean), _ptr(var))
    if rc != 0:
        raise ValueError("bn_stats of an empty channel is undefined")
    return mean, var


def int_mix(seed: np.ndarray, rounds: int) -> np.ndarray:
    seed = np.ascontiguousarray(seed, dtype=np.uint32)
    out = np.empty_like(seed)
    _load().oracle_int_mix(_ptr(seed), seed.size, int(rounds), _ptr(out))
    return out


def hist256(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.uint8)
    counts = np.empty(256, np.uint64)
    _load().oracle_hist256(_ptr(x), x.size, _ptr(counts))
    return counts


def im2col_shape(N, C, H, W, kh, kw, s, p):
    Ho = (H + 2 * p - kh) // s + 1
    Wo = (W + 2 * p - kw) // s + 1
    return (N, C * kh * kw, Ho * Wo), Ho, Wo


def im2col(x: np.ndarray, kh: int, kw: int, stride: int, pad: int) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    N, C, H, W = x.shape
    shape, Ho, Wo = im2col_shape(N, C, H, W, kh, kw, stride, pad)
    if Ho <= 0 or Wo <= 0:
        raise ValueError("empty im2col output")
    out = np.empty(shape, np.float32)
    rc = _load().oracle_im2col(_ptr(x), N, C, H, W, kh, kw, stride, pad, _ptr(out))
    if rc != 0:
        raise ValueError("bad im2col parameters")
    return out


def upsample(x: np.ndarray, scale: int) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    N, C, H, W = x.shape
    out = np.empty((N, C, H * scale, W * scale), np.float64)
    rc = _load().oracle_upsample(_ptr(x), N, C, H, W, int(scale), _ptr(out))
    if rc != 0:
        raise ValueError("bad upsample parameters")
    return out


def upsample_absmag(x: np.ndarray, scale: int) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    N, C, H, W = x.shape
    out = np.empty((N, C, H * scale, W * scale), np.float64)
    rc = _load().oracle_upsample_absmag(_ptr(x), N, C, H, W, int(scale), _ptr(out))
    if rc != 0:
        raise ValueError("bad upsample parameters")
    return out


def maxpool_shape(N, C, H, W, kh, kw, s, p):
    return (N, C, (H + 2 * p - kh) // s + 1, (W + 2 * p - kw) // s + 1)


def maxpool(x: np.ndarray, kh: int, kw: int, stride: int, pad: int):
    """(max, flat argmax index h*W + w as int32) of every pooling window."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    N, C, H, W = x.shape
    shape = maxpool_shape(N, C, H, W, kh, kw, stride, pad)
    if shape[2] <= 0 or shape[3] <= 0:
        raise ValueError("empty maxpool output")
    out = np.empty(shape, np.float32)
    idx = np.empty(shape, np.int32)
    rc = _load().oracle_maxpool(_ptr(x), N, C, H, W, kh, kw, stride, pad, _ptr(out), _ptr(idx))
    if rc != 0:
        raise ValueError("bad maxpool parameters")
    return out, idx


def ethash_like(header: bytes, nonce0: int, table: np.ndarray, n: int) -> np.ndarray:
    """Digests [n][32] (uint8) of the Ethash-like walk over `table` [rows][32]
    uint32: the seeds from hashes.ethash_seed (SHA-512 by hashlib), the walk
    and the fold by the C transcription of the definition in hashes.py."""
    from . import hashes
    assert len(header) == 80
    seeds = np.array([hashes.ethash_seed(hashes.message(bytes(header), nonce0 + i)) for i in range(n)],
                     np.uint32).reshape(n, 16)
    table = np.ascontiguousarray(table, dtype=np.uint32)
    out = np.empty((n, 32), np.uint8)
    rc = _load().oracle_ethash_like(_ptr(seeds), n, _ptr(table), table.shape[0], _ptr(out))
    if rc != 0:
        raise ValueError("bad Ethash-like parameters")
    return out
