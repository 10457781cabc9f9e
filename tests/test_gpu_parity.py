"""GPU parity: every kernel solo, every fused pair at every legal (split, block,
VGPR bound), the vertically fused comparator and the unfused baselines, against
the CPU oracle and against each other.  All calls go through the C ABI
(libhfuse.so)."""
import itertools

import numpy as np
import pytest
import torch

from paper_2007_01277_amd import hfuse as H
from paper_2007_01277_amd import inputs
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu

KINDS = range(len(H.KIND_NAMES))
BLOCKS = (256, 512, 1024)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available()
    H.hf_init()
    yield


@pytest.mark.parametrize("kind", KINDS, ids=H.KIND_NAMES)
@pytest.mark.parametrize("block", BLOCKS)
def test_solo_matches_oracle(kind, block):
    for c in G.small_cases(kind, seed=block):
        print(c.label, block, flush=True)
        G.run_and_check(lambda: H.hf_run_solo(c.task, block), [c])


@pytest.mark.parametrize("kind", KINDS, ids=H.KIND_NAMES)
def test_solo_grid_independent(kind):
    c = G.small_cases(kind, seed=3)[0]
    outs = []
    for grid in (1, 3, 64, 4096):
        c.reset()
        H.hf_run_solo(c.task, 256, grid)
        torch.cuda.synchronize()
        outs.append(c.outputs())
    c.check(outs[0])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert torch.equal(a, b)


PAIRS = [(a, b) for a in KINDS for b in KINDS]


@pytest.mark.parametrize("ka,kb", PAIRS, ids=[f"{H.KIND_NAMES[a]}+{H.KIND_NAMES[b]}" for a, b in PAIRS])
def test_fused_bit_exact_vs_solo_all_configs(ka, kb):
    """Fused output equals the solo output bit for bit for every split, block and
    VGPR bound, and the solo output matches the oracle."""
    ca = G.small_cases(ka, seed=11)[0]
    cb = G.small_cases(kb, seed=12)[1]  # a different shape than ca when ka == kb
    print(ca.label, cb.label, flush=True)
    G.run_and_check(lambda: (H.hf_run_solo(ca.task, 256), H.hf_run_solo(cb.task, 512)), [ca, cb])
    ref_a, ref_b = ca.outputs(), cb.outputs()
    pr = H.make_pair(ca.task, cb.task)
    for block in BLOCKS:
        W = block // 64
        for w1 in range(1, W):
            for cap in H.CAPS:
                ca.reset()
                cb.reset()
                H.hf_run_fused_cfg(pr, H.hf_config(w1, block, cap, 0))
                torch.cuda.synchronize()
                for r, o in zip(ref_a, ca.outputs()):
                    assert torch.equal(r, o), (ca.label, block, w1, cap)
                for r, o in zip(ref_b, cb.outputs()):
                    assert torch.equal(r, o), (cb.label, block, w1, cap)
        # the vertically fused comparator computes the same results
        ca.reset()
        cb.reset()
        H.hf_run_vfused(pr, block)
        torch.cuda.synchronize()
        for r, o in zip(ref_a + ref_b, ca.outputs() + cb.outputs()):
            assert torch.equal(r, o), ("vfused", block)


@pytest.mark.parametrize("mode", [H.HF_SERIAL, H.HF_STREAMS])
def test_unfused_modes_match_oracle(mode):
    for ka, kb in [(0, 1), (2, 3), (4, 3), (1, 0)]:
        ca = G.small_cases(ka, seed=21)[0]
        cb = G.small_cases(kb, seed=22)[0]
        pr = H.make_pair(ca.task, cb.task)
        side = torch.cuda.Stream()
        for s1 in (None, side):
            G.run_and_check(lambda: H.hf_run_unfused(pr, 256, 1024, mode, None, s1), [ca, cb])


def test_small_config_bn_stats_with_int_mix():
    """bn_stats [8,32,16,16] with int_mix 65536 x 32 rounds, split 1/2, block 256:
    fused, back-to-back and two-stream runs against the oracle."""
    ca = G.bn_case((8, 32, 16, 16), seed=0)
    cb = G.mix_case(65536, 32, seed=0)
    pr = H.make_pair(ca.task, cb.task)
    G.run_and_check(lambda: H.hf_run_fused(pr, 1, 2, 256), [ca, cb])
    f = [o.clone() for o in ca.outputs() + cb.outputs()]
    G.run_and_check(lambda: H.hf_run_unfused(pr, 256, 256, H.HF_SERIAL), [ca, cb])
    u = ca.outputs() + cb.outputs()
    for x, y in zip(f, u):
        assert torch.equal(x, y)
    G.run_and_check(lambda: H.hf_run_unfused(pr, 256, 256, H.HF_STREAMS), [ca, cb])


def test_repeated_launches_leave_scratch_clean():
    ca = G.bn_case((4, 16, 32, 32), seed=5)
    cb = G.hist_case(300_001, seed=5, offset=1)
    pr = H.make_pair(ca.task, cb.task)
    first = None
    for i in range(5):
        G.run_and_check(lambda: H.hf_run_fused(pr, 3, 4, 512), [ca, cb])
        outs = ca.outputs() + cb.outputs()
        if first is None:
            first = outs
        for x, y in zip(first, outs):
            assert torch.equal(x, y)


@pytest.mark.parametrize("method", [H.HF_TUNE_EXHAUSTIVE, H.HF_TUNE_PAPER, H.HF_TUNE_NAIVE,
                                    H.HF_TUNE_EXHAUSTIVE_GRID], ids=["exhaustive", "paper", "naive", "grid"])
def test_tuned_configuration_matches_oracle(method):
    """Every search returns a legal configuration whose fused run matches the
    oracle; the grid mode's grid is 0 or 2, 4 or 8 times the occupancy grid."""
    ca = G.bn_case((16, 64, 32, 32), seed=8)
    cb = G.mix_case(1 << 22, 8, seed=8, sample=4096)
    pr = H.make_pair(ca.task, cb.task)
    best, st = H.hf_tune(pr, method)
    print(method, best, st, flush=True)
    assert H.hf_validate_fused(pr, best) == H.HF_OK
    assert st["n_profiled"] >= 1 and st["t_best_ms"] > 0
    if method == H.HF_TUNE_EXHAUSTIVE_GRID:
        assert 85 <= st["n_candidates"] <= 85 + 9
        occ = H.hf_fused_info(ca.task.kind, cb.task.kind, best.block, best.vgpr_cap)["default_grid"]
        assert best.grid in (0, 2 * occ, 4 * occ, 8 * occ)
    else:
        assert best.grid == 0
    G.run_and_check(lambda: H.hf_run_fused_cfg(pr, best), [ca, cb])


def test_fused_grid_independent():
    ca = G.bn_case((4, 8, 30, 28), seed=6)
    cb = G.hist_case(777_777, seed=6)
    pr = H.make_pair(ca.task, cb.task)
    ref = None
    for grid in (1, 2, 13, 500, 3000):
        G.run_and_check(lambda: H.hf_run_fused_cfg(pr, H.hf_config(5, 1024, 0, grid)), [ca, cb])
        outs = ca.outputs() + cb.outputs()
        if ref is None:
            ref = outs
        for x, y in zip(ref, outs):
            assert torch.equal(x, y)


def test_caller_scratch_regions():
    ca = G.bn_case((2, 6, 20, 20), seed=8)
    cb = G.hist_case(65_537, seed=8)
    sa = torch.zeros(H.hf_scratch_bytes(ca.task) // 4 + 64, dtype=torch.int32, device="cuda")
    sb = torch.zeros(H.hf_scratch_bytes(cb.task) // 4 + 64, dtype=torch.int32, device="cuda")
    ca.task.scratch = sa.data_ptr()
    cb.task.scratch = sb.data_ptr()
    pr = H.make_pair(ca.task, cb.task)
    for _ in range(2):
        G.run_and_check(lambda: H.hf_run_fused(pr, 1, 4, 256), [ca, cb])
        assert int(sa.abs().sum()) == 0 and int(sb.abs().sum()) == 0  # left zero-filled


def test_edge_cases():
    # empty and tiny inputs, ragged tails, scalar paths
    cases = [G.mix_case(0, 3), G.mix_case(1, 3), G.mix_case(5, 2, offset=1), G.hist_case(0),
             G.hist_case(1, offset=5), G.hist_case(17, offset=15), G.bn_case((1, 1, 1, 1)),
             G.bn_case((1, 2, 1, 3)), G.im2col_case((1, 1, 1, 1)), G.im2col_case((1, 1, 2, 3), (1, 1), 1, 0),
             G.up_case((1, 1, 1, 1), 2), G.up_case((1, 1, 1, 5), 16), G.up_case((0, 3, 4, 4), 2)]
    for c in cases:
        print(c.label, flush=True)
        G.run_and_check(lambda: H.hf_run_solo(c.task, 256), [c])
    for ca, cb in itertools.combinations(cases[:8], 2):
        pr = H.make_pair(ca.task, cb.task)
        G.run_and_check(lambda: H.hf_run_fused(pr, 1, 2, 256), [ca, cb])


def test_edge_cases_pool_and_hashes():
    # empty and one-element pooling and hash tasks, a 1x1 window, a window
    # clipped to one element, solo and fused with each other and with a data kind
    cases = [G.pool_case((0, 3, 4, 4)), G.pool_case((1, 1, 1, 1), (1, 1), 1, 0),
             G.pool_case((1, 2, 1, 1), (3, 3), 2, 1, with_idx=False), G.pool_case((1, 1, 2, 3), (2, 2), 3, 1)]
    for k in (H.HF_SHA256D, H.HF_BLAKE2B, H.HF_ETHASH):
        cases += [G.hash_case(k, 0, seed=k), G.hash_case(k, 1, seed=k, rows=1)]
    for c in cases:
        print(c.label, flush=True)
        G.run_and_check(lambda: H.hf_run_solo(c.task, 256), [c])
    other = G.mix_case(5, 2, offset=1)
    for ca, cb in itertools.combinations(cases, 2):
        pr = H.make_pair(ca.task, cb.task)
        G.run_and_check(lambda: H.hf_run_fused(pr, 1, 2, 256), [ca, cb])
    for c in cases:
        pr = H.make_pair(c.task, other.task)
        G.run_and_check(lambda: H.hf_run_fused(pr, 3, 4, 256), [c, other])
        G.run_and_check(lambda: H.hf_run_vfused(pr, 512), [c, other])


def test_hashes_of_extreme_headers():
    # all-zero and all-0xFF headers: every 32-bit half of the 64-bit SHA-512 and
    # BLAKE2b words carries, and the uniform rounds run on extreme values; 96
    # instances end the Ethash-like walk after its first pass of an iteration,
    # and a nonce range wraps past 2^32
    for hdr in (bytes(80), b"\xff" * 80):
        for k in (H.HF_SHA256D, H.HF_BLAKE2B, H.HF_ETHASH):
            c = G.hash_case(k, 96, seed=k, nonce0=0xFFFFFFC0, header=hdr)
            print(c.label, hdr[:1].hex(), flush=True)
            G.run_and_check(lambda: H.hf_run_solo(c.task, 256), [c])


def test_maxpool_ties_nan_and_clamped_windows():
    """Ties keep the first element, NaN propagates, and windows clipped by the
    padding match the oracle's scan -- solo and fused, with and without indices.
    The width-16 image takes the 3x3/s2/p1 row path; its NaNs sit at the
    columns a lane takes from its left neighbour (8c - 1) and at column 0."""
    x = inputs.normal_image((2, 3, 13, 10), seed=17)
    x[0, 0] = np.round(x[0, 0])  # many ties
    x[0, 1] = 1.0                # one constant plane: every window ties
    x[1, 2, 4, 5] = np.nan
    x[1, 2, 12, 9] = np.nan      # in the bottom-right window, reached by clamping
    x[1, 0] = -np.inf
    y = inputs.normal_image((2, 3, 13, 16), seed=18)
    y[0, 0] = np.round(y[0, 0])
    y[0, 1] = 1.0
    y[1, 2, 4, 7] = np.nan
    y[1, 2, 0, 0] = np.nan
    y[1, 2, 12, 15] = np.nan
    y[1, 1, 6, 8] = np.nan
    y[1, 0] = -np.inf
    other = G.mix_case(4097, 3, seed=17)
    for img in (x, y):
        for k, s, p in [((3, 3), 2, 1), ((2, 2), 1, 1), ((3, 2), 3, 0), ((5, 4), 2, 2)]:
            for with_idx in (True, False):
                c = G.pool_case(img.shape, k, s, p, x=img, with_idx=with_idx)
                print(c.label, with_idx, flush=True)
                for block in BLOCKS:
                    G.run_and_check(lambda: H.hf_run_solo(c.task, block), [c])
                pr = H.make_pair(c.task, other.task)
                G.run_and_check(lambda: H.hf_run_fused(pr, 3, 4, 256), [c, other])


def test_bn_constant_input_exact():
    x = np.full((3, 4, 17, 12), 0.75, np.float32)
    c = G.bn_case(x.shape, x=x)
    for block in BLOCKS:
        c.reset()
        H.hf_run_solo(c.task, block)
        torch.cuda.synchronize()
        m, v = c.outputs()
        assert torch.all(m == 0.75) and torch.all(v == 0.0)


def test_hist_totals_equal_n():
    c = G.hist_case(3_000_017, seed=9, offset=7)
    other = G.mix_case(1 << 20, 16, seed=9)
    pr = H.make_pair(other.task, c.task)
    G.run_and_check(lambda: H.hf_run_fused(pr, 7, 8, 1024, 64), [c, other])
    assert int(c.outputs()[0].to(torch.int64).sum()) == 3_000_017


@pytest.mark.parametrize("block", BLOCKS)
def test_interval_barrier_stress(block):
    """Ring exchange through LDS in both intervals of every workgroup, with
    pseudo-random skew per wavefront and round, at every split; equal and
    unequal round counts (one interval finishes while the other still syncs)."""
    W = block // 64
    for w1 in range(1, W):
        for ia, ib, grid in [(64, 64, 0), (97, 13, 0), (5, 120, 1), (40, 40, 4096)]:
            bad = H.hf_selftest_barrier(block, w1, ia, ib, seed=block * 131 + w1, grid=grid)
            assert bad == 0, (block, w1, ia, ib, grid, bad)


def test_timeout_returns_etimeout_and_the_kernel_still_completes(monkeypatch):
    """The watchdog path: with HF_TIMEOUT_MS = 1 a timed launch of a ~14 ms
    kernel returns HF_ETIMEOUT instead of blocking; the kernel itself runs to
    completion (nothing is cancelled) and its output is correct."""
    c = G.mix_case(1 << 24, 4096, seed=3, sample=256)
    c.reset()
    torch.cuda.synchronize()
    monkeypatch.setenv("HF_TIMEOUT_MS", "1")
    with pytest.raises(H.HFError) as err:
        H.hf_run_solo(c.task, 256, timed=True)
    assert err.value.status == H.HF_ETIMEOUT
    monkeypatch.delenv("HF_TIMEOUT_MS")
    torch.cuda.synchronize()
    c.check(c.outputs())
    assert H.hf_run_solo(c.task, 256, timed=True) > 1.0  # the library is usable afterwards
