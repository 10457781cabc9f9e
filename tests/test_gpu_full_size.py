"""Parity at the full workload sizes, in the launch configurations the bench
uses: fused output bit-exact with the back-to-back output over every element,
and every output element against the CPU oracle (its OpenMP build, which gives
the sequential build's results); the hash digests against the oracle on a
sample and against the C transcription of the walk or hashlib on every digest."""
import numpy as np
import pytest
import torch

from paper_2007_01277_amd import hfuse as H
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bn_mix():
    ca = G.bn_case((64, 256, 56, 56), seed=0)
    cb = G.mix_case(1 << 24, 128, seed=0)
    return ca, cb


def _fused_vs_serial(ca, cb, cfg, blocks=(1024, 1024)):
    pr = H.make_pair(ca.task, cb.task)
    for c in (ca, cb):
        c.reset()
    H.hf_run_unfused(pr, blocks[0], blocks[1], H.HF_SERIAL)
    torch.cuda.synchronize()
    ref = ca.outputs() + cb.outputs()
    for c in (ca, cb):
        c.reset()
    H.hf_run_fused_cfg(pr, H.hf_config(*cfg, 0))
    torch.cuda.synchronize()
    got = ca.outputs() + cb.outputs()
    for r, g in zip(ref, got):
        assert torch.equal(r, g), cfg
    return got


@pytest.mark.parametrize("cfg", [(1, 512, 64), (4, 1024, 0), (2, 256, 0), (14, 1024, 128), (7, 512, 80)])
def test_bn_stats_int_mix_full_size(bn_mix, cfg):
    ca, cb = bn_mix
    print("bn_stats[64,256,56,56] + int_mix 2^24x128", cfg, flush=True)
    outs = _fused_vs_serial(ca, cb, cfg)
    with G.parallel_oracle():  # every channel and every word
        ca.check(outs[:2])
        cb.check(outs[2:])


def test_im2col_hist_full_size():
    ca = G.im2col_case((32, 128, 56, 56), seed=1)
    cb = G.hist_case(1 << 26, seed=2)
    for cfg in [(8, 1024, 128), (3, 512, 0), (2, 256, 64), (12, 1024, 0)]:
        print("im2col[32,128,56,56] + lds_hist 2^26", cfg, flush=True)
        outs = _fused_vs_serial(ca, cb, cfg)
    with G.parallel_oracle():  # all 32 images
        ca.check(outs[:1])
        cb.check(outs[1:])
    assert int(outs[1].to(torch.int64).sum()) == 1 << 26


def test_upsample_hist_full_size():
    ca = G.up_case((32, 64, 128, 128), 2, seed=3)
    cb = G.hist_case(1 << 26, seed=2)
    for cfg in [(4, 1024, 64), (5, 512, 0), (8, 1024, 0)]:
        print("upsample[32,64,128,128]x2 + lds_hist 2^26", cfg, flush=True)
        outs = _fused_vs_serial(ca, cb, cfg)
    with G.parallel_oracle():  # all 32 images, image by image
        ca.check(outs[:1])
        cb.check(outs[1:])


def test_maxpool_hist_full_size():
    """The ResNet-stem pooling shape [64,64,112,112] 3x3/s2/p1 with indices,
    fused with the 2^26-byte histogram: bit-exact vs back to back over every
    element, every image against the oracle."""
    ca = G.pool_case((64, 64, 112, 112), seed=4)
    cb = G.hist_case(1 << 26, seed=2)
    for cfg in [(8, 1024, 64), (12, 1024, 0), (2, 256, 80), (5, 512, 128)]:
        print("maxpool[64,64,112,112] + lds_hist 2^26", cfg, flush=True)
        outs = _fused_vs_serial(ca, cb, cfg)
    with G.parallel_oracle():
        ca.check(outs[:2])
        cb.check(outs[2:])


def test_ethash_sha256d_full_size():
    """The crypto pair at the bench's sizes (327,680 Ethash-like hashes over a
    1 GiB table, 2^22 SHA-256d hashes): fused bit-exact vs back to back over
    every digest, sampled digests against the plain-integer oracle, and every
    digest against the C transcription of the walk (Ethash-like) or hashlib's
    SHA-256 (SHA-256d)."""
    ca = G.hash_case(H.HF_ETHASH, 5 << 16, seed=21, rows=1 << 23, sample=48)
    cb = G.hash_case(H.HF_SHA256D, 1 << 22, seed=21, sample=96)
    for cfg in [(8, 1024, 0), (4, 512, 64), (1, 256, 128), (3, 256, 64)]:
        print("ethash 327680 + sha256d 2^22", cfg, flush=True)
        outs = _fused_vs_serial(ca, cb, cfg)
    with G.parallel_oracle():
        ca.check(outs[:1], full=True)
    cb.check(outs[1:], full=True)


def test_largest_element_counts_int_mix_and_hist():
    """The largest counts the ABI accepts (2^31 - 1 elements per buffer, odd, so
    both bodies take their ragged tails): int_mix over 2^31 - 1 words fused with
    a histogram of 2^31 - 1 bytes, against the oracle (sampled words, every
    count, every word in chunks) and against the back-to-back run."""
    from paper_2007_01277_amd import inputs
    import oracle
    n = (1 << 31) - 1
    seeds = inputs.cuda_uint32(n, 41)
    mixed = torch.empty_like(seeds)
    data = torch.empty(n, dtype=torch.uint8, device="cuda")
    chunk = 1 << 28
    for k, s in enumerate(range(0, n, chunk)):
        e = min(n, s + chunk)
        data[s:e] = inputs.cuda_zipf_u8(e - s, 42 + k)
    counts = torch.empty(256, dtype=torch.int32, device="cuda")
    ta, tb = H.task_int_mix(seeds, mixed, 2), H.task_lds_hist(data, counts)
    pr = H.make_pair(ta, tb)
    print("int_mix 2^31-1 x 2 rounds + lds_hist 2^31-1 bytes", flush=True)
    H.hf_run_unfused(pr, 1024, 1024, H.HF_SERIAL)
    torch.cuda.synchronize()
    ref_mixed, ref_counts = mixed.clone(), counts.clone()
    mixed.zero_()
    counts.zero_()
    H.hf_run_fused_cfg(pr, H.hf_config(8, 1024, 0, 0))
    torch.cuda.synchronize()
    assert torch.equal(mixed, ref_mixed) and torch.equal(counts, ref_counts)
    with G.parallel_oracle():
        for s in range(0, n, chunk):
            e = min(n, s + chunk)
            want = oracle.int_mix(seeds[s:e].cpu().numpy().view(np.uint32), 2)
            assert np.array_equal(mixed[s:e].cpu().numpy().view(np.uint32), want), s
        host = data.cpu().numpy()
        assert np.array_equal(counts.cpu().numpy().astype(np.uint64), oracle.hist256(host))


def test_largest_channel_bn_stats():
    """One channel of 2^31 - 1 - 2^20 elements (a ragged last unit; the ABI's
    limit is 2^31 - 1 per buffer), solo and fused with a small int_mix, against
    the oracle's two-pass double statistics."""
    from paper_2007_01277_amd import inputs
    import oracle
    from tests.gpu_cases import TOL
    shape = (1, 1, 1, (1 << 31) - 1 - (1 << 20))
    x = inputs.cuda_normal(shape, 44)
    x.mul_(2.0).add_(1.0)
    mean = torch.full((1,), 7.0, device="cuda")
    var = torch.full((1,), 7.0, device="cuda")
    ta = H.task_bn_stats(x, mean, var)
    cb = G.mix_case(100_003, 3, seed=44)
    print("bn_stats one channel of", shape[3], "elements", flush=True)
    m_ref, v_ref = oracle.bn_stats(x.cpu().numpy())
    for run in (lambda: H.hf_run_solo(ta, 1024), lambda: H.hf_run_fused_cfg(H.make_pair(ta, cb.task),
                                                                             H.hf_config(8, 1024, 0, 0))):
        mean.fill_(7.0)
        var.fill_(7.0)
        cb.reset()
        run()
        torch.cuda.synchronize()
        m, v = float(mean.item()), float(var.item())
        assert abs(m - m_ref[0]) <= TOL * (abs(m_ref[0]) + np.sqrt(v_ref[0])), (m, m_ref)
        assert abs(v - v_ref[0]) <= TOL * v_ref[0], (v, v_ref)
    cb.check(cb.outputs())
