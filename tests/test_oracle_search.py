"""Pins of the search reference against the numbers the paper prints."""
from oracle import search


def test_occupancy_example_of_section_2a():
    # 24K shared memory, 512 threads, 64 registers -> 2 blocks per SM (registers bind);
    # 32 registers -> 4 blocks (Sec. II-A)
    assert search.blocks_per_core(512, 64, 24 * 1024) == 2
    assert search.blocks_per_core(512, 32, 24 * 1024) == 4


def test_register_bound_of_motivating_example():
    # 1024-thread fused kernel, 896 + 128 split: the search bounds registers to 32
    # per thread on the 1080 Ti (Sec. II-C).  With both kernels light enough to fit
    # two blocks, the thread limit 2048/1024 = 2 binds and r0 = 65536/(2*1024).
    assert search.register_bound(1024, 896, 32, 32, 16 * 1024) == 32
    assert search.register_bound(1024, 768, 32, 32, 16 * 1024) == 32


def test_register_bound_register_limited():
    # a heavy first kernel: b1 = 65536 // (512*64) = 2; d0 = 768 -> b0 = min(2, .., 2) = 2
    assert search.register_bound(768, 512, 64, 16, 0) == 65536 // (2 * 768)
    # heavier: b1 = 65536 // (512 * 128) = 1 -> r0 = 65536 // 768
    assert search.register_bound(768, 512, 128, 16, 0) == 65536 // 768


def test_paper_candidate_order():
    c = search.paper_candidates(1024)
    assert len(c) == 14
    assert c[:4] == [(128, False), (128, True), (256, False), (256, True)]
    assert c[-1] == (896, True)


def test_paper_search_strict_improvement_keeps_first():
    t = {(128, False): 5.0, (128, True): 5.0, (256, False): 4.0, (256, True): 4.0}
    best = search.paper_search(384, lambda d1, b: t[(d1, b)])
    assert best == (256, False, 4.0)


def test_gfx950_bound_is_full_occupancy_at_1024():
    # thread limit: 2 workgroups of 1024 per CU -> r0 = 131072 / 2048 = 64
    assert search.register_bound(1024, 512, 32, 32, 4096, hw=search.GFX950) == 64
