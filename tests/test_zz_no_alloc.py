"""hf_run_fused_noalloc, the fused launch that allocates nothing (its tasks'
scratch lives in the library's static device array), against hf_run_fused_cfg,
the same launch with the library's allocated arena: bit-exact on two calls in a
row, the second with smaller inputs, and against the CPU oracle."""
import numpy as np
import pytest
import torch

from paper_2007_01277_amd import hfuse as H
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu


def _both_ways(ca, cb, cfg):
    pr = H.make_pair(ca.task, cb.task)
    for c in (ca, cb):
        c.reset()
    H.hf_run_fused_cfg(pr, cfg)
    torch.cuda.synchronize()
    ref = ca.outputs() + cb.outputs()
    for c in (ca, cb):
        c.reset()
    H.hf_run_fused_noalloc(pr, cfg)
    torch.cuda.synchronize()
    got = ca.outputs() + cb.outputs()
    for r, g in zip(ref, got):
        assert torch.equal(r, g), (ca.label, cb.label, cfg)
    return got


def test_noalloc_matches_the_arena_launch_twice_second_smaller():
    # bn_stats and the histogram both keep counters and partials in scratch
    big = (G.bn_case((16, 64, 28, 28), seed=51), G.hist_case(1 << 22, seed=52))
    small = (G.bn_case((2, 5, 7, 9), seed=53), G.hist_case(1001, seed=54, offset=3))
    for (ca, cb), cfg in ((big, H.hf_config(4, 512, 64, 0)), (small, H.hf_config(1, 256, 0, 0))):
        print("noalloc", ca.label, cb.label, cfg, flush=True)
        got = _both_ways(ca, cb, cfg)
        n = len(ca.bufs["outs"])
        ca.check(got[:n])
        cb.check(got[n:])


def test_noalloc_repeated_and_mirrored_pairs():
    # the same launch again (the array keeps the last call's contents, which
    # the call clears), the mirrored pair, and a pair with one scratch task
    ca, cb = G.bn_case((8, 32, 16, 16), seed=55), G.hist_case(1 << 20, seed=56)
    cm = G.mix_case(65536, 32, seed=57)
    for pair, cfg in (((ca, cb), H.hf_config(2, 256, 0, 0)), ((ca, cb), H.hf_config(2, 256, 0, 0)),
                      ((cb, ca), H.hf_config(6, 1024, 80, 0)), ((cm, ca), H.hf_config(1, 512, 0, 0))):
        print("noalloc", pair[0].label, pair[1].label, cfg, flush=True)
        got = _both_ways(pair[0], pair[1], cfg)
        n = len(pair[0].bufs["outs"])
        pair[0].check(got[:n])
        pair[1].check(got[n:])
    assert np.all(np.isfinite(ca.outputs()[0].cpu().numpy()))
