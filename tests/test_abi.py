"""The C ABI without a GPU: the library loads, exports every function that
include/hfuse.h declares, and rejects bad arguments on the host before any HIP
call.  Host-side search logic is checked against the search reference."""
import ctypes
import os
import re

import pytest

from oracle import search
from paper_2007_01277_amd import hfuse as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "hfuse.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hf_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = H.lib()
    names = _declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(H.SIGNATURES), set(names) ^ set(H.SIGNATURES)


def test_strerror_and_version():
    L = H.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -99):
        assert L.hf_strerror(code)
    assert b"gfx950" in L.hf_version()


def _fake_ptr(off=0):
    return 0x10000000 + off  # never dereferenced: validation is host-only


def _bn(n=2, c=3, h=4, w=4):
    t = H.hf_task()
    t.kind = H.HF_BN_STATS
    t.in_, t.out0, t.out1 = _fake_ptr(), _fake_ptr(4096), _fake_ptr(8192)
    t.n, t.c, t.h, t.w = n, c, h, w
    return t


def _mix(n=100, rounds=4):
    t = H.hf_task()
    t.kind = H.HF_INT_MIX
    t.p[0] = rounds
    t.in_, t.out0 = _fake_ptr(), _fake_ptr(1 << 20)
    t.n = n
    return t


def _hist(n=100, bins=256):
    t = H.hf_task()
    t.kind = H.HF_LDS_HIST
    t.p[0] = bins
    t.in_, t.out0 = _fake_ptr(3), _fake_ptr(1 << 20)
    t.n = n
    return t


def _im2col(n=1, c=2, h=5, w=5, k=(3, 3, 1, 1)):
    t = H.hf_task()
    t.kind = H.HF_IM2COL
    for i, v in enumerate(k):
        t.p[i] = v
    t.in_, t.out0 = _fake_ptr(), _fake_ptr(1 << 20)
    t.n, t.c, t.h, t.w = n, c, h, w
    return t


def _up(n=1, c=2, h=5, w=5, s=2):
    t = H.hf_task()
    t.kind = H.HF_UPSAMPLE
    t.p[0] = s
    t.in_, t.out0 = _fake_ptr(), _fake_ptr(1 << 20)
    t.n, t.c, t.h, t.w = n, c, h, w
    return t


def _pool(n=1, c=2, h=6, w=6, k=(3, 3, 2, 1), idx=True):
    t = H.hf_task()
    t.kind = H.HF_MAXPOOL
    for i, v in enumerate(k):
        t.p[i] = v
    t.in_, t.out0 = _fake_ptr(), _fake_ptr(1 << 20)
    t.out1 = _fake_ptr(1 << 21) if idx else None
    t.n, t.c, t.h, t.w = n, c, h, w
    return t


def _hash(kind, n=100, rows=64):
    t = H.hf_task()
    t.kind = kind
    t.p[0] = -5  # any uint32 nonce
    t.in_, t.out0 = _fake_ptr(), _fake_ptr(1 << 20)
    if kind == H.HF_ETHASH:
        t.in1, t.h = _fake_ptr(1 << 22), rows
    t.n = n
    return t


def test_hash_tasks_validation():
    for k in (H.HF_SHA256D, H.HF_BLAKE2B, H.HF_ETHASH):
        assert H.hf_validate_task(_hash(k)) == H.HF_OK
        assert H.hf_validate_task(_hash(k, n=0)) == H.HF_OK
        assert H.hf_scratch_bytes(_hash(k)) == 0
        t = _hash(k)
        t.out0 = _fake_ptr((1 << 20) + 8)  # digests must be 16-byte aligned
        assert H.hf_validate_task(t) == H.HF_EINVAL
        t = _hash(k)
        t.in_ = None
        assert H.hf_validate_task(t) == H.HF_EINVAL
        assert H.hf_validate_task(_hash(k, n=1 << 28)) == H.HF_EINVAL  # 8 words per digest
    assert H.hf_validate_task(_hash(H.HF_ETHASH, rows=0)) == H.HF_EINVAL
    assert H.hf_validate_task(_hash(H.HF_ETHASH, rows=1 << 32)) == H.HF_EINVAL
    assert H.hf_validate_task(_hash(H.HF_ETHASH, rows=(1 << 32) - 1)) == H.HF_OK
    t = _hash(H.HF_ETHASH)
    t.in1 = None
    assert H.hf_validate_task(t) == H.HF_EINVAL


def test_valid_tasks_pass():
    for t in (_bn(), _mix(), _hist(), _im2col(), _up(), _pool(), _pool(idx=False), _mix(n=0), _hist(n=0),
              _im2col(n=0), _up(n=0), _pool(n=0)):
        assert H.hf_validate_task(t) == H.HF_OK


@pytest.mark.parametrize("make,change", [
    (_bn, dict(n=0)), (_bn, dict(c=0)), (_bn, dict(out1=None)), (_bn, dict(in_=None)),
    (_bn, dict(in_=_fake_ptr(2))),
    (_mix, dict(n=-1)), (_mix, dict(n=1 << 31)), (_mix, dict(out0=None)),
    (_hist, dict(out0=None)),
    (_im2col, dict(h=1, w=1)),  # 3x3 without enough padding... still legal with pad 1
    (_up, dict(c=0)),
    (_bn, dict(kind=len(H.KIND_NAMES))), (_bn, dict(kind=-1)),
])
def test_bad_tasks_rejected(make, change):
    t = make()
    for k, v in change.items():
        setattr(t, k, v)
    rc = H.hf_validate_task(t)
    if make is _im2col and change == dict(h=1, w=1):
        assert rc == H.HF_OK  # a 1x1 image padded by 1 still has one 3x3 window
    else:
        assert rc == H.HF_EINVAL


@pytest.mark.parametrize("p", [(0, 3, 1, 0), (3, 3, 0, 1), (3, 3, 1, -1), (5, 5, 1, 0)])
def test_bad_im2col_params(p):
    t = _im2col(h=4, w=4, k=p)
    assert H.hf_validate_task(t) == H.HF_EINVAL


@pytest.mark.parametrize("p", [(0, 3, 1, 0), (3, 3, 0, 1), (3, 3, 1, -1), (3, 3, 1, 3), (2, 3, 1, 2),
                               (65, 1, 1, 0), (3, 3, 65, 1)])
def test_bad_maxpool_params(p):
    # pad must stay below both window sizes, so that every window holds an element
    assert H.hf_validate_task(_pool(k=p)) == H.HF_EINVAL


def test_maxpool_shape_limits():
    assert H.hf_validate_task(_pool(h=1, w=1, k=(3, 3, 1, 1))) == H.HF_OK  # one clipped window
    assert H.hf_validate_task(_pool(h=1, w=1, k=(3, 3, 1, 0))) == H.HF_EINVAL  # no window fits
    t = _pool()
    t.out1 = _fake_ptr(2)  # misaligned index buffer
    assert H.hf_validate_task(t) == H.HF_EINVAL
    # stride 1 with padding has more outputs than inputs: both counts are bounded
    assert H.hf_validate_task(_pool(n=1 << 16, c=1, h=181, w=181, k=(3, 3, 1, 1))) == H.HF_OK
    assert H.hf_validate_task(_pool(n=1 << 16, c=1, h=181, w=181, k=(2, 2, 1, 1))) == H.HF_EINVAL
    assert H.hf_scratch_bytes(_pool()) == 0


def test_bad_hist_bins_and_upsample_scale():
    assert H.hf_validate_task(_hist(bins=128)) == H.HF_EINVAL
    assert H.hf_validate_task(_up(s=0)) == H.HF_EINVAL
    assert H.hf_validate_task(_up(s=17)) == H.HF_EINVAL


def test_scratch_bytes():
    assert H.hf_scratch_bytes(_mix()) == 0
    assert H.hf_scratch_bytes(_hist()) == 4 * 320
    # bn: C counters padded to 64 words, then (mean, M2) per 1024-element unit
    t = _bn(n=64, c=256, h=56, w=56)
    units = -(-64 * 56 * 56 // 1024)
    assert H.hf_scratch_bytes(t) == 4 * (256 + 2 * 256 * units)
    assert H.hf_scratch_bytes(_bn(n=0)) == H.HF_EINVAL


@pytest.mark.parametrize("cfg,rc", [
    ((2, 256, 0, 0), H.HF_OK), ((1, 256, 64, 0), H.HF_OK), ((15, 1024, 128, 0), H.HF_OK),
    ((0, 256, 0, 0), H.HF_EINVAL), ((4, 256, 0, 0), H.HF_EINVAL), ((2, 384, 0, 0), H.HF_EINVAL),
    ((2, 256, 72, 0), H.HF_EINVAL), ((2, 256, 0, -1), H.HF_EINVAL), ((16, 1024, 0, 0), H.HF_EINVAL),
])
def test_validate_fused(cfg, rc):
    pr = H.make_pair(_bn(), _mix())
    assert H.hf_validate_fused(pr, H.hf_config(*cfg)) == rc


def test_run_entry_points_reject_before_touching_the_gpu():
    pr = H.make_pair(_bn(), _mix())
    L = H.lib()
    assert L.hf_run_fused(ctypes.byref(pr), 1, 3, 256, 0, None, None) == H.HF_EINVAL  # 256/3 lanes
    assert L.hf_run_fused(ctypes.byref(pr), 1, 2, 300, 0, None, None) == H.HF_EINVAL
    assert L.hf_run_fused(ctypes.byref(pr), 1, 2, 256, 33, None, None) == H.HF_EINVAL
    assert L.hf_run_unfused(ctypes.byref(pr), 256, 256, 7, None, None, None) == H.HF_EINVAL
    assert L.hf_run_solo(ctypes.byref(_bn(n=0)), 256, 0, None, None) == H.HF_EINVAL
    assert L.hf_copy(None, None, 16, None, None) == H.HF_EINVAL
    assert L.hf_run_vfused(ctypes.byref(pr), 384, 0, None, None) == H.HF_EINVAL
    assert L.hf_run_vfused(None, 256, 0, None, None) == H.HF_EINVAL
    assert L.hf_tune(ctypes.byref(pr), 9, 0, 3, None, ctypes.byref(H.hf_config()), None) == H.HF_EINVAL
    assert L.hf_tune(ctypes.byref(pr), 5, 0, 3, None, ctypes.byref(H.hf_config()), None) == H.HF_EINVAL


@pytest.mark.parametrize("d1,d2,va,vb,lds", [(896, 128, 32, 32, 1024), (512, 512, 63, 11, 12),
                                              (128, 896, 100, 20, 4096), (256, 768, 256, 16, 0),
                                              (64, 192, 40, 40, 20000)])
def test_register_bound_matches_reference(d1, d2, va, vb, lds):
    ref = search.register_bound(d1 + d2, d1, va, vb, lds, hw=search.GFX950)
    assert H.hf_register_bound(d1, d2, va, vb, lds) == ref


def test_paper_candidates_follow_the_main_search():
    c = H.hf_tune_candidates(H.HF_TUNE_PAPER, 1024, 32, 32, 4096)
    ref = search.paper_candidates(1024)
    assert [(x.split_waves * 64, x.vgpr_cap != 0) for x in c] == ref
    # with light kernels the thread limit binds: r0 = 64 on gfx950
    assert all(x.vgpr_cap in (0, 64) for x in c) and all(x.block == 1024 for x in c)


def test_exhaustive_candidates_are_wave_aligned_eighths():
    c = H.hf_tune_candidates(H.HF_TUNE_EXHAUSTIVE, 0)
    pairs = sorted({(x.block, x.split_waves) for x in c})
    assert pairs == [(256, 1), (256, 2), (256, 3)] + [(512, k) for k in range(1, 8)] + \
        [(1024, 2 * k) for k in range(1, 8)]
    assert len(c) == 17 * len(H.CAPS)
    assert H.hf_tune_candidates(H.HF_TUNE_NAIVE, 0)[0].as_tuple() == (8, 1024, 0, 0)
    # the grid mode starts from the same space; its grid stage runs on the GPU
    g = H.hf_tune_candidates(H.HF_TUNE_EXHAUSTIVE_GRID, 0)
    assert [x.as_tuple() for x in g] == [x.as_tuple() for x in c]
    assert all(x.grid == 0 for x in g)


def test_batch_create_rejects_bad_groups_before_the_gpu():
    L = H.lib()
    tasks = (H.hf_task * 6)(*[_mix() for _ in range(6)])
    h = ctypes.c_void_p()

    def call(groups, waves, block=256):
        g = (ctypes.c_int32 * 6)(*groups)
        w = None if waves is None else ctypes.cast((ctypes.c_int32 * 6)(*waves), ctypes.POINTER(ctypes.c_int32))
        return L.hf_batch_create(tasks, 6, ctypes.cast(g, ctypes.POINTER(ctypes.c_int32)), w, block,
                                 ctypes.byref(h))

    assert call([0, 0, 0, 0, 0, 1], None) == H.HF_EINVAL         # five members
    assert call([0, 0, 1, 1, 0, 0], None) == H.HF_EINVAL         # ids go back
    assert call([0, 0, 1, 1, 2, 2], [2, 3, 1, 1, 1, 1]) == H.HF_EINVAL  # 5 waves > 4
    assert call([0, 0, 1, 1, 2, 2], [0, 1, 1, 1, 1, 1]) == H.HF_EINVAL  # a task without waves
    assert call([0, 0, 1, 1, 2, 2], None, block=384) == H.HF_EINVAL


def test_barrier_selftest_rejects_bad_arguments():
    # checked on the host before any HIP call
    m = ctypes.c_uint32(0)
    L = H.lib()
    for args in [(128, 1, 1, 1), (256, 0, 1, 1), (256, 4, 1, 1), (1024, 16, 1, 1), (512, 2, -1, 1),
                 (512, 2, 1, (1 << 20) + 1)]:
        assert L.hf_selftest_barrier(*args, 0, 0, None, ctypes.byref(m)) == H.HF_EINVAL, args
    assert L.hf_selftest_barrier(256, 1, 1, 1, 0, -1, None, ctypes.byref(m)) == H.HF_EINVAL
    assert L.hf_selftest_barrier(256, 1, 1, 1, 0, 0, None, None) == H.HF_EINVAL


def test_tuner_sample_store_skips_a_cut_line(tmp_path):
    from paper_2007_01277_amd import learned_tuner as LT
    p = tmp_path / "s.jsonl"
    p.write_text('{"key": "a", "X": [[1.0]], "y": [0.5]}\n{"key": "b", "X": [[')
    d = LT._load_store(str(p))
    assert list(d) == ["a"] and d["a"]["y"] == [0.5]
    assert LT._load_store(str(tmp_path / "missing.jsonl")) == {}
    LT._append(str(p), {"key": "c", "X": [[2.0]], "y": [1.5]})  # after the cut line, on a line of its own
    d = LT._load_store(str(p))
    assert sorted(d) == ["a", "c"] and len(p.read_text().splitlines()) == 3


def test_noalloc_rejects_before_touching_the_gpu():
    # bad configurations, and tasks whose scratch exceeds the static array
    # (bn_stats of 2^31 - 1 - 2^20 elements in one channel needs ~16 MiB)
    L = H.lib()
    pr = H.make_pair(_bn(), _mix())
    assert L.hf_run_fused_noalloc(ctypes.byref(pr), ctypes.byref(H.hf_config(4, 256, 0, 0)), None) == H.HF_EINVAL
    assert L.hf_run_fused_noalloc(None, ctypes.byref(H.hf_config(2, 256, 0, 0)), None) == H.HF_EINVAL
    big = _bn(n=1, c=1, h=1, w=(1 << 31) - 1 - (1 << 20))
    assert H.hf_scratch_bytes(big) > H.HF_NOALLOC_SCRATCH_BYTES
    pr = H.make_pair(big, _hist())
    assert L.hf_run_fused_noalloc(ctypes.byref(pr), ctypes.byref(H.hf_config(2, 256, 0, 0)), None) == H.HF_ESCRATCH
    # two tasks that each fit but not together
    half = H.HF_NOALLOC_SCRATCH_BYTES // 2
    w = 1024 * (half // 8)  # (mean, M2) per 1024-element unit: just over half the array
    a, b = _bn(n=1, c=1, h=1, w=w), _bn(n=1, c=1, h=1, w=w)
    b.in_, b.out0, b.out1 = _fake_ptr(1 << 24), _fake_ptr(1 << 25), _fake_ptr(1 << 26)
    assert H.hf_scratch_bytes(a) <= H.HF_NOALLOC_SCRATCH_BYTES
    pr = H.make_pair(a, b)
    assert L.hf_run_fused_noalloc(ctypes.byref(pr), ctypes.byref(H.hf_config(2, 256, 0, 0)), None) == H.HF_ESCRATCH
