"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, a published value, library routines and brute force.

Each test is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign, index or divisor, a transposed operand) fails at least one of them.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
from paper_2007_01277_amd import inputs

M32 = 0xFFFFFFFF
K_MUL = 2654435761  # Knuth's multiplicative-hashing constant, 0x9E3779B1


# ------------------------------------------------------------------ bn_stats
def test_bn_constant_input_exact():
    # every partial sum of 0.75 is exact, so mean = 0.75 and var = 0 exactly
    x = np.full((3, 5, 7, 9), 0.75, np.float32)
    m, v = oracle.bn_stats(x)
    assert np.all(m == 0.75) and np.all(v == 0.0)


def test_bn_two_level_closed_form():
    # half of each channel at a_c - b_c, half at a_c + b_c: mean a_c, biased var b_c^2
    N, C, H, W = 4, 6, 3, 8
    a = np.linspace(-3, 5, C).astype(np.float32)
    b = np.linspace(0.25, 2.0, C).astype(np.float32)
    sign = np.where((np.arange(N * H * W) % 2) == 0, -1.0, 1.0).reshape(N, 1, H, W)
    x = (a[None, :, None, None] + sign * b[None, :, None, None]).astype(np.float32)
    m, v = oracle.bn_stats(x)
    # closed form from the two float32 levels actually stored: lo and hi
    lo = (a - b).astype(np.float64)
    hi = (a + b).astype(np.float64)
    np.testing.assert_allclose(m, (lo + hi) / 2, rtol=0, atol=1e-12)
    np.testing.assert_allclose(v, ((hi - lo) / 2) ** 2, rtol=1e-12, atol=0)


def test_bn_matches_numpy_population_stats():
    x = inputs.bn_input((3, 7, 5, 11), seed=5)
    m, v = oracle.bn_stats(x)
    xd = x.astype(np.float64).transpose(1, 0, 2, 3).reshape(7, -1)
    np.testing.assert_allclose(m, xd.mean(axis=1), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(v, xd.var(axis=1, ddof=0), rtol=1e-11, atol=0)


def test_bn_empty_channel_rejected():
    with pytest.raises(ValueError):
        oracle.bn_stats(np.zeros((0, 3, 4, 4), np.float32))


def test_bn_generator_statistics():
    # the synthetic input follows z*scale_c + shift_c: sample stats of each channel
    # lie within 5 sigma of their sampling distributions
    shape = (8, 4, 32, 32)
    x = inputs.bn_input(shape, seed=11)
    prm = inputs.rng(12)
    scale = prm.uniform(0.5, 2.0, size=4).astype(np.float32).astype(np.float64)
    shift = prm.uniform(-1.0, 1.0, size=4).astype(np.float32).astype(np.float64)
    m, v = oracle.bn_stats(x)
    M = 8 * 32 * 32
    assert np.all(np.abs(m - shift) <= 5 * scale / np.sqrt(M))
    assert np.all(np.abs(v - scale ** 2) <= 5 * scale ** 2 * np.sqrt(2.0 / M))


# ------------------------------------------------------------------ int_mix
def _unshift_left(y, k):
    # inverse of x ^= x << k on 32 bits
    x = y
    for _ in range(32 // k + 1):
        x = y ^ ((x << k) & M32)
    return x


def _unshift_right(y, k):
    x = y
    for _ in range(32 // k + 1):
        x = y ^ (x >> k)
    return x


def _int_mix_inverse(y, rounds):
    kinv = pow(K_MUL, -1, 2 ** 32)
    x = int(y)
    for r in reversed(range(rounds)):
        x = ((x - r) * kinv) & M32
        x = _unshift_left(x, 5)
        x = _unshift_right(x, 17)
        x = _unshift_left(x, 13)
    return x


def test_int_mix_zero_rounds_is_identity():
    s = inputs.uint32_seeds(1000, seed=3)
    assert np.array_equal(oracle.int_mix(s, 0), s)


def test_int_mix_xorshift_matches_marsaglia_published_value():
    # Marsaglia, "Xorshift RNGs" (J. Stat. Softw. 8(14), 2003): the 32-bit
    # generator with shifts (13, 17, 5) from y = 2463534242 first returns 723471715.
    # One round is that step followed by x*K + 0, so undo the multiply.
    y = oracle.int_mix(np.array([2463534242], np.uint32), 1)[0]
    kinv = pow(K_MUL, -1, 2 ** 32)
    assert (int(y) * kinv) & M32 == 723471715


@pytest.mark.parametrize("rounds", [1, 2, 7, 32, 128])
def test_int_mix_inverts_to_the_seeds(rounds):
    s = inputs.uint32_seeds(64, seed=rounds)
    y = oracle.int_mix(s, rounds)
    back = [_int_mix_inverse(v, rounds) for v in y]
    assert back == [int(v) for v in s]


def test_int_mix_round_index_matters():
    # 0 is a fixed point of xorshift and of the multiply; only the "+ r" term moves it
    z = np.zeros(1, np.uint32)
    assert oracle.int_mix(z, 1)[0] == 0
    assert oracle.int_mix(z, 2)[0] == 1


# ------------------------------------------------------------------ lds_hist
def test_hist_matches_bincount_and_total():
    x = inputs.zipf_u8(100_003, seed=4)
    c = oracle.hist256(x)
    assert int(c.sum()) == x.size
    assert np.array_equal(c, np.bincount(x, minlength=256).astype(np.uint64))


def test_hist_constant_and_ramp():
    c = oracle.hist256(np.full(777, 42, np.uint8))
    assert c[42] == 777 and c.sum() == 777
    ramp = (np.arange(256 * 13) % 256).astype(np.uint8)
    assert np.all(oracle.hist256(ramp) == 13)


def test_zipf_generator_head_mass():
    # truncated Zipf(1.2) over 256 ranks: P(rank 1) = 1/H, H = sum k^-1.2
    H = np.sum(1.0 / np.arange(1, 257) ** 1.2)
    x = inputs.zipf_u8(400_000, seed=9)
    p0 = np.mean(x == 0)
    assert abs(p0 - 1.0 / H) < 5 * np.sqrt((1 / H) * (1 - 1 / H) / x.size)


# ------------------------------------------------------------------ im2col
@pytest.mark.parametrize("shape,k,s,p", [
    ((2, 3, 7, 9), (3, 3), 1, 1),
    ((1, 2, 8, 8), (3, 3), 2, 1),
    ((2, 4, 5, 6), (1, 1), 1, 0),
    ((1, 3, 6, 5), (2, 3), 1, 0),
    ((1, 2, 9, 7), (5, 5), 2, 2),
])
def test_im2col_matches_torch_unfold(shape, k, s, p):
    x = inputs.normal_image(shape, seed=1)
    out = oracle.im2col(x, k[0], k[1], s, p)
    ref = F.unfold(torch.from_numpy(x), kernel_size=k, stride=s, padding=p).numpy()
    assert out.shape == ref.shape
    assert np.array_equal(out, ref)


def test_im2col_1x1_is_reshape():
    x = inputs.normal_image((2, 5, 4, 6), seed=2)
    out = oracle.im2col(x, 1, 1, 1, 0)
    assert np.array_equal(out, x.reshape(2, 5, 24))


def test_im2col_centre_row_is_input():
    x = inputs.normal_image((2, 3, 6, 7), seed=3)
    out = oracle.im2col(x, 3, 3, 1, 1).reshape(2, 3, 9, 42)
    assert np.array_equal(out[:, :, 4, :], x.reshape(2, 3, 42))


def test_im2col_overlap_counts():
    # folding the columns of an all-ones image back counts how many 3x3 windows
    # cover each pixel: 9 inside, 6 on an edge, 4 in a corner
    H, W = 6, 7
    cols = oracle.im2col(np.ones((1, 1, H, W), np.float32), 3, 3, 1, 1)
    cnt = F.fold(torch.from_numpy(cols), output_size=(H, W), kernel_size=3, padding=1)[0, 0]
    expect = np.full((H, W), 9.0)
    expect[0, :] = expect[-1, :] = expect[:, 0] = expect[:, -1] = 6.0
    expect[0, 0] = expect[0, -1] = expect[-1, 0] = expect[-1, -1] = 4.0
    assert np.array_equal(cnt.numpy(), expect)


def test_im2col_times_weights_is_direct_convolution():
    x = inputs.normal_image((2, 3, 6, 5), seed=4)
    w = inputs.normal_image((4, 3, 3, 3), seed=5)
    cols = oracle.im2col(x, 3, 3, 1, 1).astype(np.float64)
    y = np.einsum("ok,nkl->nol", w.reshape(4, 27).astype(np.float64), cols)
    # brute-force direct convolution, zero padding 1
    xp = np.zeros((2, 3, 8, 7))
    xp[:, :, 1:-1, 1:-1] = x
    ref = np.zeros((2, 4, 6, 5))
    for n in range(2):
        for o in range(4):
            for i in range(6):
                for j in range(5):
                    ref[n, o, i, j] = np.sum(xp[n, :, i:i + 3, j:j + 3] * w[o])
    np.testing.assert_allclose(y.reshape(2, 4, 6, 5), ref, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ upsample
@pytest.mark.parametrize("shape,s", [((2, 3, 5, 7), 2), ((1, 2, 4, 3), 3), ((1, 1, 1, 6), 2),
                                     ((1, 2, 6, 6), 1), ((1, 1, 3, 4), 4)])
def test_upsample_matches_torch_interpolate(shape, s):
    x = inputs.normal_image(shape, seed=6)
    out = oracle.upsample(x, s)
    ref = F.interpolate(torch.from_numpy(x).double(), scale_factor=s, mode="bilinear",
                        align_corners=False).numpy()
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12)


def test_upsample_constant_is_exact():
    out = oracle.upsample(np.full((1, 2, 5, 6), -1.375, np.float32), 2)
    assert np.all(out == -1.375)


def test_upsample_ramp_closed_form():
    # a ramp along w is reproduced at the clamped source coordinate:
    # out[ox] = min(max(ox/2 - 1/4, 0), W - 1)
    W = 9
    x = np.tile(np.arange(W, dtype=np.float32), (1, 1, 3, 1))
    out = oracle.upsample(x, 2)[0, 0, 1]
    ox = np.arange(2 * W)
    assert np.array_equal(out, np.clip(ox / 2 - 0.25, 0, W - 1))


def test_upsample_identity_scale():
    x = inputs.normal_image((1, 2, 4, 5), seed=7)
    assert np.array_equal(oracle.upsample(x, 1), x.astype(np.float64))


@pytest.mark.parametrize("shape,s", [((2, 3, 7, 9), 2), ((1, 2, 5, 4), 3), ((1, 1, 1, 6), 2), ((2, 2, 6, 1), 4)])
def test_upsample_absmag_is_the_interpolation_of_abs(shape, s):
    # The tolerance scale of every upsample check: sum_k |w_k x_k| over the
    # four taps.  Bilinear weights are non-negative, so it equals the
    # interpolation of |x|: against torch's bilinear interpolation of |x| in
    # double (a library routine), and against the oracle's own upsample of |x|.
    x = inputs.normal_image(shape, seed=31 + s)
    mag = oracle.upsample_absmag(x, s)
    ref = F.interpolate(torch.from_numpy(np.abs(x)).double(), scale_factor=s, mode="bilinear",
                        align_corners=False).numpy()
    np.testing.assert_allclose(mag, ref, rtol=1e-12, atol=0)
    np.testing.assert_allclose(mag, oracle.upsample(np.abs(x), s), rtol=1e-12, atol=0)
    # and it bounds the magnitude of the interpolated value itself
    assert np.all(np.abs(oracle.upsample(x, s)) <= mag * (1 + 1e-12))


def test_upsample_absmag_constant_and_sign():
    # a constant c gives |c| everywhere; flipping the sign of the input
    # changes nothing; a single non-zero input spreads exactly its weights
    for c in (-2.5, 0.0, 3.0):
        assert np.all(oracle.upsample_absmag(np.full((1, 1, 4, 5), c, np.float32), 2) == abs(c))
    x = inputs.normal_image((1, 2, 6, 7), seed=33)
    assert np.array_equal(oracle.upsample_absmag(x, 2), oracle.upsample_absmag(-x, 2))
    one = np.zeros((1, 1, 4, 4), np.float32)
    one[0, 0, 1, 2] = -1.0
    # output row 3: source 1.25 -> rows 1 (0.75) and 2 (0.25); output column 5:
    # source 2.25 -> columns 2 (0.75) and 3 (0.25): weight of x[1, 2] = 0.75 * 0.75
    assert oracle.upsample_absmag(one, 2)[0, 0, 3, 5] == 0.5625
    # output row 2 (source 0.75 -> rows 0 (0.25), 1 (0.75)), column 4 (source
    # 1.75 -> columns 1 (0.25), 2 (0.75)): weight 0.75 * 0.75 again; column 6
    # (source 2.75 -> columns 2 (0.25), 3 (0.75)): 0.75 * 0.25
    assert oracle.upsample_absmag(one, 2)[0, 0, 2, 4] == 0.5625
    assert oracle.upsample_absmag(one, 2)[0, 0, 2, 6] == 0.1875


# ------------------------------------------------------------------- maxpool
POOL_CASES = [((2, 3, 9, 11), (3, 3), 2, 1), ((1, 2, 8, 8), (2, 2), 2, 0), ((2, 1, 7, 5), (3, 2), 1, 1),
              ((1, 4, 12, 10), (3, 3), 3, 0), ((3, 2, 5, 6), (1, 1), 1, 0), ((1, 1, 4, 13), (2, 3), 1, 1)]


@pytest.mark.parametrize("shape,k,s,p", POOL_CASES)
def test_maxpool_matches_torch_max_pool2d(shape, k, s, p):
    # library routine: torch's CPU max pooling with indices (flat h*W + w)
    x = inputs.normal_image(shape, seed=sum(shape) + s)
    v, i = oracle.maxpool(x, k[0], k[1], s, p)
    tv, ti = F.max_pool2d(torch.from_numpy(x), k, s, p, return_indices=True)
    assert np.array_equal(v, tv.numpy()) and np.array_equal(i, ti.numpy().astype(np.int32))


@pytest.mark.parametrize("shape,k,s,p", POOL_CASES)
def test_maxpool_matches_sliding_window_max_and_first_argmax(shape, k, s, p):
    # library routine: numpy sliding windows over a -inf padded copy; argmax
    # returns the first maximum in row-major window order
    x = inputs.normal_image(shape, seed=7 * sum(shape))
    N, C, H, W = shape
    xp = np.full((N, C, H + 2 * p, W + 2 * p), -np.inf, np.float32)
    xp[:, :, p:p + H, p:p + W] = x
    win = np.lib.stride_tricks.sliding_window_view(xp, k, axis=(2, 3))[:, :, ::s, ::s]
    Ho, Wo = win.shape[2], win.shape[3]
    flat = win.reshape(N, C, Ho, Wo, k[0] * k[1])
    am = flat.argmax(-1)
    hh = np.arange(Ho)[:, None] * s - p + am // k[1]
    ww = np.arange(Wo)[None, :] * s - p + am % k[1]
    v, i = oracle.maxpool(x, k[0], k[1], s, p)
    assert np.array_equal(v, flat.max(-1)) and np.array_equal(i, (hh * W + ww).astype(np.int32))


def test_maxpool_increasing_ramp_picks_last_valid_element():
    # x = h*W + w grows along the scan, so each window's winner is its
    # bottom-right in-range element, and value == index
    N, C, H, W, k, s, p = 1, 1, 11, 9, 3, 2, 1
    x = np.arange(H * W, dtype=np.float32).reshape(N, C, H, W)
    v, i = oracle.maxpool(x, k, k, s, p)
    Ho, Wo = v.shape[2:]
    hb = np.minimum(np.arange(Ho) * s - p + k - 1, H - 1)[:, None]
    wb = np.minimum(np.arange(Wo) * s - p + k - 1, W - 1)[None, :]
    assert np.array_equal(i[0, 0], hb * W + wb) and np.array_equal(v[0, 0], (hb * W + wb).astype(np.float32))


def test_maxpool_ties_keep_first_and_constant_windows():
    # a constant image: every window ties, the winner is the top-left in-range element
    H, W, k, s, p = 7, 8, 3, 2, 1
    v, i = oracle.maxpool(np.full((1, 2, H, W), -1.5, np.float32), k, k, s, p)
    Ho, Wo = v.shape[2:]
    ht = np.maximum(np.arange(Ho) * s - p, 0)[:, None]
    wt = np.maximum(np.arange(Wo) * s - p, 0)[None, :]
    assert np.all(v == -1.5) and np.array_equal(i[0, 1], ht * W + wt)


def test_maxpool_non_overlapping_equals_block_reshape_max():
    x = inputs.normal_image((2, 3, 8, 12), seed=4)
    v, i = oracle.maxpool(x, 2, 2, 2, 0)
    blocks = x.reshape(2, 3, 4, 2, 6, 2)
    assert np.array_equal(v, blocks.max(axis=(3, 5)))
    np.testing.assert_array_equal(x.reshape(2, 3, -1)[np.arange(2)[:, None, None, None], np.arange(3)[None, :, None, None],
                                                      i.astype(np.int64)], v)


def test_maxpool_nan_propagates_and_minus_inf():
    x = np.zeros((1, 1, 4, 4), np.float32)
    x[0, 0, 1, 2] = np.nan
    x[0, 0, 2, 3] = 5.0
    x[0, 0, 3, 3] = np.nan
    v, i = oracle.maxpool(x, 2, 2, 2, 0)
    # window (0,1): NaN at (1,2) beats zeros; window (1,1): scan meets 5 then the NaN at (3,3)
    assert np.isnan(v[0, 0, 0, 1]) and i[0, 0, 0, 1] == 1 * 4 + 2
    assert np.isnan(v[0, 0, 1, 1]) and i[0, 0, 1, 1] == 3 * 4 + 3
    assert v[0, 0, 0, 0] == 0 and i[0, 0, 0, 0] == 0
    tv, ti = F.max_pool2d(torch.from_numpy(x), 2, 2, 0, return_indices=True)
    assert np.array_equal(np.isnan(v), np.isnan(tv.numpy())) and np.array_equal(i, ti.numpy())
    y = np.full((1, 1, 3, 3), -np.inf, np.float32)
    v, i = oracle.maxpool(y, 3, 3, 1, 1)
    assert np.all(v == -np.inf) and np.array_equal(i[0, 0], [[0, 0, 1], [0, 0, 1], [3, 3, 4]])


def test_maxpool_rejects_windows_with_no_input():
    with pytest.raises(ValueError):
        oracle.maxpool(np.zeros((1, 1, 4, 4), np.float32), 2, 2, 1, 2)


def test_openmp_build_gives_the_sequential_results():
    # the OpenMP build spreads independent units over threads; every result
    # must equal the sequential build's bit for bit
    x = inputs.bn_input((3, 7, 9, 11), seed=40)
    img = inputs.normal_image((2, 3, 9, 10), seed=41)
    seeds = inputs.uint32_seeds(10_007, seed=42)
    data = inputs.zipf_u8(100_003, seed=43)
    table = inputs.eth_table(61, seed=44)
    hdr = inputs.header80(45).tobytes()

    def run():
        return [*oracle.bn_stats(x), oracle.int_mix(seeds, 9), oracle.hist256(data),
                oracle.im2col(img, 3, 3, 1, 1), oracle.upsample(img, 2), oracle.upsample_absmag(img, 3),
                *oracle.maxpool(img, 3, 3, 2, 1), oracle.ethash_like(hdr, 5, table, 300)]

    seq = run()
    oracle.use_openmp(True)
    try:
        assert oracle.threads() >= 1
        par = run()
    finally:
        oracle.use_openmp(False)
    for a, b in zip(seq, par):
        assert np.array_equal(a, b)
