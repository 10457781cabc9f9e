"""ctypes binding of libhfuse.so (the C ABI in include/hfuse.h).

Argument marshalling only: torch tensors become device pointers and shapes,
torch streams become hipStream_t handles.  Every step of the hot path runs in
the library's HIP kernels; there is no fallback.  If the library is not built,
``lib()`` raises instead of computing anything another way.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HFUSE_LIB") or os.path.join(PKG, "libhfuse.so")

HF_OK, HF_EINVAL, HF_EUNSUPPORTED, HF_EHIP, HF_ETIMEOUT, HF_ENOMEM, HF_ENOMODEL, HF_ESCRATCH = 0, -1, -2, -3, -4, -5, -6, -7
HF_NOALLOC_SCRATCH_BYTES = 4 << 20
(HF_BN_STATS, HF_INT_MIX, HF_IM2COL, HF_LDS_HIST, HF_UPSAMPLE, HF_MAXPOOL, HF_SHA256D, HF_BLAKE2B,
 HF_ETHASH) = range(9)
KIND_NAMES = ["bn_stats", "int_mix", "im2col", "lds_hist", "upsample", "maxpool", "sha256d", "blake2b", "ethash"]
HF_SERIAL, HF_STREAMS = 0, 1
HF_TUNE_EXHAUSTIVE, HF_TUNE_PAPER, HF_TUNE_NAIVE, HF_TUNE_MLP, HF_TUNE_EXHAUSTIVE_GRID = range(5)
CAPS = (0, 64, 80, 96, 128)


class HFError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status} ({_strerror(status)})")


class hf_task(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("p", ctypes.c_int32 * 4), ("reserved", ctypes.c_int32),
                ("in_", ctypes.c_void_p), ("out0", ctypes.c_void_p), ("out1", ctypes.c_void_p),
                ("scratch", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("c", ctypes.c_int64), ("h", ctypes.c_int64), ("w", ctypes.c_int64),
                ("in1", ctypes.c_void_p)]


class hf_pair(ctypes.Structure):
    _fields_ = [("a", hf_task), ("b", hf_task)]


class hf_config(ctypes.Structure):
    _fields_ = [("split_waves", ctypes.c_int32), ("block", ctypes.c_int32),
                ("vgpr_cap", ctypes.c_int32), ("grid", ctypes.c_int32)]

    def as_tuple(self):
        return (self.split_waves, self.block, self.vgpr_cap, self.grid)

    def __repr__(self):
        return f"hf_config(split_waves={self.split_waves}, block={self.block}, vgpr_cap={self.vgpr_cap}, grid={self.grid})"


class hf_batch_schedule(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("interval_waves", ctypes.c_int32), ("item_kb", ctypes.c_int32),
                ("split_policy", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class hf_kernel_info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "vgprs", "sgprs", "lds_bytes", "spill_bytes", "wg_per_cu", "waves_per_simd", "num_cus", "default_grid")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class hf_tune_stats(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int32), ("n_profiled", ctypes.c_int32),
                ("t_best_ms", ctypes.c_float), ("t_naive_ms", ctypes.c_float),
                ("wall_s", ctypes.c_float), ("reps", ctypes.c_int32),
                ("n_solo_launches", ctypes.c_int32), ("solo_ms", ctypes.c_float)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_P = ctypes.c_void_p
_I = ctypes.c_int
_F = ctypes.POINTER(ctypes.c_float)
_I32P = ctypes.POINTER(ctypes.c_int32)

# name -> (restype, argtypes); the exported surface of include/hfuse.h
SIGNATURES = {
    "hf_init": (_I, []),
    "hf_shutdown": (_I, []),
    "hf_strerror": (ctypes.c_char_p, [_I]),
    "hf_last_hip_error": (_I, []),
    "hf_version": (ctypes.c_char_p, []),
    "hf_validate_task": (_I, [ctypes.POINTER(hf_task)]),
    "hf_scratch_bytes": (ctypes.c_int64, [ctypes.POINTER(hf_task)]),
    "hf_validate_fused": (_I, [ctypes.POINTER(hf_pair), ctypes.POINTER(hf_config)]),
    "hf_run_solo": (_I, [ctypes.POINTER(hf_task), _I, _I, _P, _F]),
    "hf_run_unfused": (_I, [ctypes.POINTER(hf_pair), _I, _I, _I, _P, _P, _F]),
    "hf_run_fused": (_I, [ctypes.POINTER(hf_pair), _I, _I, _I, _I, _P, _F]),
    "hf_run_fused_cfg": (_I, [ctypes.POINTER(hf_pair), ctypes.POINTER(hf_config), _P, _F]),
    "hf_run_fused_noalloc": (_I, [ctypes.POINTER(hf_pair), ctypes.POINTER(hf_config), _P]),
    "hf_run_vfused": (_I, [ctypes.POINTER(hf_pair), _I, _I, _P, _F]),
    "hf_fused_info": (_I, [_I, _I, _I, _I, ctypes.POINTER(hf_kernel_info)]),
    "hf_solo_info": (_I, [_I, _I, ctypes.POINTER(hf_kernel_info)]),
    "hf_profile": (_I, [ctypes.POINTER(hf_pair), ctypes.POINTER(hf_config), _I, _P, _F]),
    "hf_tune_candidates": (_I, [_I, _I, _I, _I, _I, ctypes.POINTER(hf_config), _I]),
    "hf_tune": (_I, [ctypes.POINTER(hf_pair), _I, _I, _I, _P, ctypes.POINTER(hf_config),
                     ctypes.POINTER(hf_tune_stats)]),
    "hf_register_bound": (_I, [_I, _I, _I, _I, _I]),
    "hf_mlp_init": (_I, [_I, ctypes.c_uint64]),
    "hf_mlp_init_ensemble": (_I, [_I, ctypes.c_uint64, _I]),
    "hf_mlp_members": (_I, []),
    "hf_mlp_num_params": (_I, []),
    "hf_mlp_get_params": (_I, [_F, ctypes.c_int64]),
    "hf_mlp_set_params": (_I, [_F, ctypes.c_int64]),
    "hf_mlp_grad": (_I, [_F, _F, _I, _F, _F]),
    "hf_mlp_step": (_I, [_F, _F, _I, ctypes.c_float, _F]),
    "hf_mlp_adam_reset": (_I, []),
    "hf_mlp_train": (_I, [_F, _F, _I, _I, _I, ctypes.c_float, _F]),
    "hf_mlp_predict": (_I, [_F, _I, _F]),
    "hf_mlp_save": (_I, [ctypes.c_char_p]),
    "hf_mlp_load": (_I, [ctypes.c_char_p]),
    "hf_featurize": (_I, [ctypes.POINTER(hf_pair), ctypes.POINTER(hf_config), _I, _P, _F]),
    "hf_batch_create": (_I, [ctypes.POINTER(hf_task), _I, _I32P, _I32P, _I, ctypes.POINTER(_P)]),
    "hf_batch_create_sched": (_I, [ctypes.POINTER(hf_task), _I, _I32P, _I32P, ctypes.POINTER(hf_batch_schedule),
                                   ctypes.POINTER(_P)]),
    "hf_batch_tune_sched": (_I, [ctypes.POINTER(hf_task), _I, _I32P, _I, _P, ctypes.POINTER(hf_batch_schedule), _F,
                                 _I32P]),
    "hf_batch_run": (_I, [_P, _I, _P, _F]),
    "hf_batch_info": (_I, [_P, _I32P, _I32P, _I32P]),
    "hf_batch_destroy": (_I, [_P]),
    "hf_run_batch": (_I, [ctypes.POINTER(hf_task), _I, _I32P, _I32P, _I, _P, _F]),
    "hf_batch_tune": (_I, [ctypes.POINTER(hf_task), _I, _I32P, _I, _P, _I32P, _I32P, _F]),
    "hf_copy": (_I, [_P, _P, ctypes.c_int64, _P, _F]),
    "hf_read": (_I, [_P, ctypes.c_int64, _P, _F]),
    "hf_scrub": (_I, [_P]),
    "hf_warmup": (_I, [_I, _P]),
    "hf_int_peak": (_I, [_I, _I, _P, _F, ctypes.POINTER(ctypes.c_double)]),
    "hf_selftest_barrier": (_I, [_I, _I, _I, _I, ctypes.c_uint32, _I, _P, ctypes.POINTER(ctypes.c_uint32)]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _strerror(status: int) -> str:
    try:
        return lib().hf_strerror(status).decode()
    except Exception:  # library not loadable: still report the number
        return "?"


def _check(status: int, what: str) -> int:
    if status < 0:
        raise HFError(status, what)
    return status


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------------ descriptors
def _ptr(t):
    return None if t is None else t.data_ptr()


def task_bn_stats(x, mean, var) -> hf_task:
    t = hf_task()
    t.kind = HF_BN_STATS
    t.in_, t.out0, t.out1 = _ptr(x), _ptr(mean), _ptr(var)
    t.n, t.c, t.h, t.w = x.shape
    return t


def task_int_mix(seeds, out, rounds: int) -> hf_task:
    t = hf_task()
    t.kind = HF_INT_MIX
    t.p[0] = rounds
    t.in_, t.out0 = _ptr(seeds), _ptr(out)
    t.n = seeds.numel()
    return t


def task_im2col(x, out, kh: int, kw: int, stride: int, pad: int) -> hf_task:
    t = hf_task()
    t.kind = HF_IM2COL
    t.p[0], t.p[1], t.p[2], t.p[3] = kh, kw, stride, pad
    t.in_, t.out0 = _ptr(x), _ptr(out)
    t.n, t.c, t.h, t.w = x.shape
    return t


def task_lds_hist(x, counts) -> hf_task:
    t = hf_task()
    t.kind = HF_LDS_HIST
    t.p[0] = 256
    t.in_, t.out0 = _ptr(x), _ptr(counts)
    t.n = x.numel()
    return t


def task_upsample(x, out, scale: int) -> hf_task:
    t = hf_task()
    t.kind = HF_UPSAMPLE
    t.p[0] = scale
    t.in_, t.out0 = _ptr(x), _ptr(out)
    t.n, t.c, t.h, t.w = x.shape
    return t


def task_maxpool(x, out, idx=None, kh: int = 3, kw: int = 3, stride: int = 2, pad: int = 1) -> hf_task:
    """Max pooling of `x` into `out`; `idx` (int32, optional) receives each
    maximum's flat index h*W + w within its input plane."""
    t = hf_task()
    t.kind = HF_MAXPOOL
    t.p[0], t.p[1], t.p[2], t.p[3] = kh, kw, stride, pad
    t.in_, t.out0, t.out1 = _ptr(x), _ptr(out), _ptr(idx)
    t.n, t.c, t.h, t.w = x.shape
    return t


def _hash_task(kind, header, digests, nonce0: int, n: int) -> hf_task:
    t = hf_task()
    t.kind = kind
    t.p[0] = ctypes.c_int32(nonce0 & 0xFFFFFFFF).value
    t.in_, t.out0 = _ptr(header), _ptr(digests)
    t.n = n
    return t


def task_sha256d(header, digests, nonce0: int, n: int) -> hf_task:
    """SHA-256(SHA-256(header[0:76] || le32(nonce0 + i))) into digests[i] (32 bytes)."""
    return _hash_task(HF_SHA256D, header, digests, nonce0, n)


def task_blake2b(header, digests, nonce0: int, n: int) -> hf_task:
    """32-byte BLAKE2b (no key) of header[0:76] || le32(nonce0 + i) into digests[i]."""
    return _hash_task(HF_BLAKE2B, header, digests, nonce0, n)


def task_ethash(header, table, digests, nonce0: int, n: int) -> hf_task:
    """Ethash-like digests over `table` (uint32 [rows][32])."""
    t = _hash_task(HF_ETHASH, header, digests, nonce0, n)
    t.in1 = _ptr(table)
    t.h = table.shape[0]
    return t


def maxpool_out_shape(shape, kh=3, kw=3, stride=2, pad=1):
    n, c, h, w = shape
    return (n, c, (h + 2 * pad - kh) // stride + 1, (w + 2 * pad - kw) // stride + 1)


def make_pair(a: hf_task, b: hf_task) -> hf_pair:
    return hf_pair(a, b)


# ------------------------------------------------------------------ entry points
def hf_init():
    return _check(lib().hf_init(), "hf_init")


def hf_shutdown():
    return _check(lib().hf_shutdown(), "hf_shutdown")


def hf_validate_task(t: hf_task) -> int:
    return lib().hf_validate_task(ctypes.byref(t))


def hf_scratch_bytes(t: hf_task) -> int:
    return lib().hf_scratch_bytes(ctypes.byref(t))


def hf_validate_fused(pr: hf_pair, cfg: hf_config) -> int:
    return lib().hf_validate_fused(ctypes.byref(pr), ctypes.byref(cfg))


def _ms(timed):
    return ctypes.c_float(0.0) if timed else None


def hf_run_solo(t: hf_task, block: int = 256, grid: int = 0, stream=None, timed=False):
    ms = _ms(timed)
    _check(lib().hf_run_solo(ctypes.byref(t), block, grid, _stream(stream),
                             ctypes.byref(ms) if ms is not None else None), "hf_run_solo")
    return ms.value if ms is not None else None


def hf_run_unfused(pr: hf_pair, block_a: int = 256, block_b: int = 256, mode: int = HF_SERIAL,
                   stream0=None, stream1=None, timed=False):
    ms = _ms(timed)
    s1 = None if stream1 is None else _stream(stream1)
    _check(lib().hf_run_unfused(ctypes.byref(pr), block_a, block_b, mode, _stream(stream0), s1,
                                ctypes.byref(ms) if ms is not None else None), "hf_run_unfused")
    return ms.value if ms is not None else None


def hf_run_fused(pr: hf_pair, split_num: int = 1, split_den: int = 2, block: int = 256,
                 vgpr_cap: int = 0, stream=None, timed=False):
    ms = _ms(timed)
    _check(lib().hf_run_fused(ctypes.byref(pr), split_num, split_den, block, vgpr_cap, _stream(stream),
                              ctypes.byref(ms) if ms is not None else None), "hf_run_fused")
    return ms.value if ms is not None else None


def hf_run_fused_cfg(pr: hf_pair, cfg: hf_config, stream=None, timed=False):
    ms = _ms(timed)
    _check(lib().hf_run_fused_cfg(ctypes.byref(pr), ctypes.byref(cfg), _stream(stream),
                                  ctypes.byref(ms) if ms is not None else None), "hf_run_fused_cfg")
    return ms.value if ms is not None else None


def hf_run_fused_noalloc(pr: hf_pair, cfg: hf_config, stream=None):
    """The fused launch with the library's static scratch (no allocation)."""
    _check(lib().hf_run_fused_noalloc(ctypes.byref(pr), ctypes.byref(cfg), _stream(stream)),
           "hf_run_fused_noalloc")


def hf_run_vfused(pr: hf_pair, block: int = 256, grid: int = 0, stream=None, timed=False):
    ms = _ms(timed)
    _check(lib().hf_run_vfused(ctypes.byref(pr), block, grid, _stream(stream),
                               ctypes.byref(ms) if ms is not None else None), "hf_run_vfused")
    return ms.value if ms is not None else None


def hf_fused_info(kind_a: int, kind_b: int, block: int, vgpr_cap: int = 0) -> dict:
    info = hf_kernel_info()
    _check(lib().hf_fused_info(kind_a, kind_b, block, vgpr_cap, ctypes.byref(info)), "hf_fused_info")
    return info.as_dict()


def hf_solo_info(kind: int, block: int) -> dict:
    info = hf_kernel_info()
    _check(lib().hf_solo_info(kind, block, ctypes.byref(info)), "hf_solo_info")
    return info.as_dict()


def hf_profile(pr: hf_pair, cfg: hf_config, reps: int = 20, stream=None) -> float:
    ms = ctypes.c_float(0.0)
    _check(lib().hf_profile(ctypes.byref(pr), ctypes.byref(cfg), reps, _stream(stream), ctypes.byref(ms)),
           "hf_profile")
    return ms.value


def hf_tune_candidates(method: int, block: int = 0, vgpr_a: int = 32, vgpr_b: int = 32, lds_fused: int = 0):
    n = _check(lib().hf_tune_candidates(method, block, vgpr_a, vgpr_b, lds_fused, None, 0), "hf_tune_candidates")
    arr = (hf_config * max(n, 1))()
    lib().hf_tune_candidates(method, block, vgpr_a, vgpr_b, lds_fused, arr, n)
    return [arr[i] for i in range(n)]


def hf_tune(pr: hf_pair, method: int = HF_TUNE_EXHAUSTIVE, block: int = 0, topk: int = 3, stream=None):
    best = hf_config()
    stats = hf_tune_stats()
    _check(lib().hf_tune(ctypes.byref(pr), method, block, topk, _stream(stream), ctypes.byref(best),
                         ctypes.byref(stats)), "hf_tune")
    return best, stats.as_dict()


def hf_register_bound(d1: int, d2: int, vgpr_a: int, vgpr_b: int, lds_fused: int) -> int:
    return lib().hf_register_bound(d1, d2, vgpr_a, vgpr_b, lds_fused)


# ------------------------------------------------------------------ learned cost model
MLP_FEATURES = 2 * (len(KIND_NAMES) + 7) + 10  # HF_MLP_FEATURES


def _f32(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(_F)


def hf_mlp_init(d_in: int = MLP_FEATURES, seed: int = 0, members: int = 1):
    """A new model of `members` networks (an ensemble when members > 1)."""
    if members == 1:
        _check(lib().hf_mlp_init(d_in, seed), "hf_mlp_init")
    else:
        _check(lib().hf_mlp_init_ensemble(d_in, seed, members), "hf_mlp_init_ensemble")


def hf_mlp_members() -> int:
    return _check(lib().hf_mlp_members(), "hf_mlp_members")


def hf_mlp_num_params() -> int:
    return _check(lib().hf_mlp_num_params(), "hf_mlp_num_params")


def hf_mlp_get_params():
    import numpy as np
    p = np.empty(hf_mlp_num_params(), np.float32)
    _check(lib().hf_mlp_get_params(p.ctypes.data_as(_F), p.size), "hf_mlp_get_params")
    return p


def hf_mlp_set_params(p):
    a, ptr = _f32(p)
    _check(lib().hf_mlp_set_params(ptr, a.size), "hf_mlp_set_params")


def hf_mlp_grad(X, y):
    import numpy as np
    Xa, xp = _f32(X)
    ya, yp = _f32(y)
    loss = ctypes.c_float(0.0)
    g = np.empty(hf_mlp_num_params(), np.float32)
    _check(lib().hf_mlp_grad(xp, yp, ya.size, ctypes.byref(loss), g.ctypes.data_as(_F)), "hf_mlp_grad")
    return loss.value, g


def hf_mlp_step(X, y, lr: float):
    Xa, xp = _f32(X)
    ya, yp = _f32(y)
    loss = ctypes.c_float(0.0)
    _check(lib().hf_mlp_step(xp, yp, ya.size, lr, ctypes.byref(loss)), "hf_mlp_step")
    return loss.value


def hf_mlp_adam_reset():
    _check(lib().hf_mlp_adam_reset(), "hf_mlp_adam_reset")


def hf_mlp_train(X, y, epochs: int = 2000, lr: float = 1e-3) -> float:
    Xa, xp = _f32(X)
    ya, yp = _f32(y)
    loss = ctypes.c_float(0.0)
    _check(lib().hf_mlp_train(xp, yp, ya.size, Xa.shape[1], epochs, lr, ctypes.byref(loss)), "hf_mlp_train")
    return loss.value


def hf_mlp_predict(X):
    import numpy as np
    Xa, xp = _f32(X)
    y = np.empty(Xa.shape[0], np.float32)
    _check(lib().hf_mlp_predict(xp, Xa.shape[0], y.ctypes.data_as(_F)), "hf_mlp_predict")
    return y


def hf_mlp_save(path: str):
    _check(lib().hf_mlp_save(path.encode()), "hf_mlp_save")


def hf_mlp_load(path: str):
    _check(lib().hf_mlp_load(path.encode()), "hf_mlp_load")


def hf_featurize(pr: hf_pair, cfgs, stream=None):
    import numpy as np
    arr = (hf_config * len(cfgs))(*cfgs)
    X = np.empty((len(cfgs), MLP_FEATURES), np.float32)
    _check(lib().hf_featurize(ctypes.byref(pr), arr, len(cfgs), _stream(stream), X.ctypes.data_as(_F)),
           "hf_featurize")
    return X


# ------------------------------------------------------------------ batched N-way fusion
def _i32(a):
    if a is None:
        return None, None
    arr = (ctypes.c_int32 * len(a))(*[int(v) for v in a])
    return arr, ctypes.cast(arr, _I32P)


class Batch:
    """Owns an hf_batch handle; keep the tasks' tensors alive while it is used."""

    def __init__(self, tasks, groups, waves=None, block=256, schedule=None):
        """`schedule` (an hf_batch_schedule) replaces `block` when given."""
        self.ntask = len(tasks)
        self._tasks = (hf_task * len(tasks))(*tasks)
        g_arr, g_ptr = _i32(groups)
        w_arr, w_ptr = _i32(waves)
        h = _P()
        if schedule is None:
            _check(lib().hf_batch_create(self._tasks, len(tasks), g_ptr, w_ptr, block, ctypes.byref(h)),
                   "hf_batch_create")
        else:
            _check(lib().hf_batch_create_sched(self._tasks, len(tasks), g_ptr, w_ptr, ctypes.byref(schedule),
                                               ctypes.byref(h)), "hf_batch_create_sched")
        self.handle = h

    def run(self, use_graph=False, stream=None, timed=False):
        ms = _ms(timed)
        _check(lib().hf_batch_run(self.handle, int(bool(use_graph)), _stream(stream),
                                  ctypes.byref(ms) if ms is not None else None), "hf_batch_run")
        return ms.value if ms is not None else None

    def info(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().hf_batch_info(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "hf_batch_info")
        return {"items": a.value, "grid": b.value, "groups": c.value}

    def close(self):
        if self.handle:
            lib().hf_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hf_run_batch(tasks, groups, waves=None, block=256, stream=None, timed=False):
    arr = (hf_task * len(tasks))(*tasks)
    g_arr, g_ptr = _i32(groups)
    w_arr, w_ptr = _i32(waves)
    ms = _ms(timed)
    _check(lib().hf_run_batch(arr, len(tasks), g_ptr, w_ptr, block, _stream(stream),
                              ctypes.byref(ms) if ms is not None else None), "hf_run_batch")
    return ms.value if ms is not None else None


def hf_batch_tune(tasks, groups, reps=5, stream=None):
    arr = (hf_task * len(tasks))(*tasks)
    g_arr, g_ptr = _i32(groups)
    w_out = (ctypes.c_int32 * len(tasks))()
    b_out = ctypes.c_int32()
    ms = ctypes.c_float()
    _check(lib().hf_batch_tune(arr, len(tasks), g_ptr, reps, _stream(stream), ctypes.cast(w_out, _I32P),
                               ctypes.byref(b_out), ctypes.byref(ms)), "hf_batch_tune")
    return list(w_out), b_out.value, ms.value


def hf_copy(dst, src, nbytes: int, stream=None, timed=False):
    ms = _ms(timed)
    _check(lib().hf_copy(_ptr(dst), _ptr(src), nbytes, _stream(stream),
                         ctypes.byref(ms) if ms is not None else None), "hf_copy")
    return ms.value if ms is not None else None


def hf_read(src, nbytes: int, stream=None, timed=False):
    ms = _ms(timed)
    _check(lib().hf_read(_ptr(src), nbytes, _stream(stream), ctypes.byref(ms) if ms is not None else None),
           "hf_read")
    return ms.value if ms is not None else None


def hf_scrub(stream=None):
    _check(lib().hf_scrub(_stream(stream)), "hf_scrub")


def hf_selftest_barrier(block: int, split_waves: int, iters_a: int, iters_b: int, seed: int = 0, grid: int = 0,
                        stream=None) -> int:
    """Interval-barrier self-test; returns the number of mismatched reads."""
    m = ctypes.c_uint32(0)
    _check(lib().hf_selftest_barrier(block, split_waves, iters_a, iters_b, seed & 0xFFFFFFFF, grid,
                                     _stream(stream), ctypes.byref(m)), "hf_selftest_barrier")
    return m.value


def hf_warmup(ms: int = 500, stream=None):
    _check(lib().hf_warmup(ms, _stream(stream)), "hf_warmup")


def hf_int_peak(rounds: int = 16384, grid: int = 0, stream=None):
    """(ms, lane-ops) of one launch of the register-only int_mix round loop:
    the measured integer-issue ceiling."""
    ms = ctypes.c_float(0.0)
    ops = ctypes.c_double(0.0)
    _check(lib().hf_int_peak(rounds, grid, _stream(stream), ctypes.byref(ms), ctypes.byref(ops)), "hf_int_peak")
    return ms.value, ops.value


def hf_batch_tune_sched(tasks, groups, reps=5, stream=None):
    """(schedule, median ms, schedules profiled) of the batch schedule search."""
    arr = (hf_task * len(tasks))(*tasks)
    g_arr, g_ptr = _i32(groups)
    best = hf_batch_schedule()
    ms = ctypes.c_float(0.0)
    n = ctypes.c_int32(0)
    _check(lib().hf_batch_tune_sched(arr, len(tasks), g_ptr, reps, _stream(stream), ctypes.byref(best),
                                     ctypes.byref(ms), ctypes.byref(n)), "hf_batch_tune_sched")
    return best, ms.value, n.value
