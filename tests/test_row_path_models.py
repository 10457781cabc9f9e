"""Per-lane models of the image kernels' row paths, on the CPU.

Each model follows its kernel's design: the unit -> (plane, chunk) mapping, one
chunk per 16-lane DPP row, a row shift by one lane whose out-of-row source
reads zero (row_shr:1 / row_shl:1 with bound control), the extra dword load at
a chunk's first or last lane, and buffer accesses whose out-of-range offsets
load zero and drop stores.  The models are checked against the oracle and
assert that every in-range offset stays inside its plane; they check the
index arithmetic of the design before any GPU run, the GPU parity tests check
the kernels themselves.
"""
import numpy as np
import pytest

import oracle

OOR = 0x80000000
U32 = 0xFFFFFFFF


def _load(buf, off, n, limit):
    if off == OOR:
        return np.zeros(n, buf.dtype)
    assert 0 <= off and off + 4 * n <= limit, (off, n, limit)
    return buf[off // 4: off // 4 + n]


def im2col_rows(x):
    """3x3 / stride 1 / pad 1: a unit is four 64-column chunks of one channel;
    each lane reads three input rows and writes one row of all nine planes."""
    N, C, H, W = x.shape
    HW = H * W
    xf = x.reshape(N * C, HW)
    out = np.full((N * C * 9, HW), 7.0, np.float32)
    nch = (W + 63) // 64
    nq = (H * nch + 3) // 4
    for u in range(N * C * nq):
        nc = u // nq
        for q in range(4):
            cid = 4 * (u - nc * nq) + q
            oh = cid // nch
            lanes = []
            for c4 in range(16):
                col = 64 * (cid - oh * nch) + 4 * c4
                ec = OOR
                if c4 == 0 and col > 0:
                    ec = col - 1
                if c4 == 15 and col + 4 < W:
                    ec = col + 4
                rows = []
                for i in range(3):
                    ih = (oh + i - 1) & U32
                    ok = oh < H and col < W and ih < H
                    v = _load(xf[nc], 4 * (ih * W + col) if ok else OOR, 4, 4 * HW)
                    e = _load(xf[nc], 4 * (ih * W + ec) if ok and ec != OOR else OOR, 1, 4 * HW)[0]
                    rows.append((v, e))
                lanes.append((rows, 4 * (oh * W + col) if (oh < H and col < W) else OOR))
            for c4 in range(16):
                rows, at = lanes[c4]
                for i in range(3):
                    v, e = rows[i]
                    left = e if c4 == 0 else lanes[c4 - 1][0][i][0][3]
                    right = e if c4 == 15 else lanes[c4 + 1][0][i][0][0]
                    for j, vals in enumerate(([left, v[0], v[1], v[2]], list(v), [v[1], v[2], v[3], right])):
                        if at != OOR:
                            assert at + 16 <= 4 * HW
                            out[nc * 9 + 3 * i + j, at // 4: at // 4 + 4] = vals
    return out.reshape(N, C * 9, HW)


def _lerp(a, b, l):
    f = np.float32
    return f(f(a) + f(f(l) * f(f(b) - f(a))))


def _coord(o, L):
    f = np.float32
    t = max(f(f(f(o) + f(0.5)) * f(0.5)) - f(0.5), f(0.0))
    a = min(int(t), L - 1)
    return a, min(a + 1, L - 1), f(t - f(a))


def upsample2_rows(x):
    """Scale 2: a unit is four 32-input-column chunks of one plane; each lane
    reads two input columns of the two source rows and writes four outputs."""
    N, C, H, W = x.shape
    Ho, Wo = 2 * H, 2 * W
    HW, OHW = H * W, Ho * Wo
    xf = x.reshape(N * C, HW)
    out = np.full((N * C, OHW), 7.0, np.float32)
    nch = (W + 31) // 32
    nq = (Ho * nch + 3) // 4
    for u in range(N * C * nq):
        pl = u // nq
        for q in range(4):
            cid = 4 * (u - pl * nq) + q
            oy = cid // nch
            lanes = []
            for c4 in range(16):
                col = 32 * (cid - oy * nch) + 2 * c4
                y0, y1, ly = _coord(min(oy, Ho - 1), H)
                ok = oy < Ho and col < W
                ec = OOR
                if c4 == 0 and col > 0:
                    ec = col - 1
                if c4 == 15 and col + 2 < W:
                    ec = col + 2
                r = []
                for y in (y0, y1):
                    v = _load(xf[pl], 4 * (y * W + col) if ok else OOR, 2, 4 * HW)
                    e = _load(xf[pl], 4 * (y * W + ec) if ok and ec != OOR else OOR, 1, 4 * HW)[0]
                    r.append((v, e))
                lanes.append((oy, col, ly, r))
            for c4 in range(16):
                oy, col, ly, r = lanes[c4]
                first, last = col == 0, col + 2 >= W
                h = []
                for k in range(2):
                    v, e = r[k]
                    sl = lanes[c4 - 1][3][k][0][1] if c4 > 0 else np.float32(0)
                    sr = lanes[c4 + 1][3][k][0][0] if c4 < 15 else np.float32(0)
                    p0 = v[0] if first else (e if c4 == 0 else sl)
                    p3 = v[1] if last else (e if c4 == 15 else sr)
                    h.append([_lerp(p0, v[0], .75), _lerp(v[0], v[1], .25), _lerp(v[0], v[1], .75),
                              _lerp(v[1], p3, .25)])
                if oy < Ho and col < W:
                    at = oy * Wo + 2 * col
                    assert 4 * (at + 4) <= 4 * OHW
                    out[pl, at:at + 4] = [_lerp(h[0][e], h[1][e], ly) for e in range(4)]
    return out.reshape(N, C, Ho, Wo)


def maxpool3s2_rows(x):
    """3x3 / stride 2 / pad 1: a unit is four 128-input-column chunks of one
    plane; each lane scans the windows of four outputs over three rows, the
    column left of its eight taken from the lane before or by one load."""
    N, C, H, W = x.shape
    Ho, Wo = (H - 1) // 2 + 1, W // 2
    HW, OHW = H * W, Ho * Wo
    xf = x.reshape(N * C, HW)
    val = np.full((N * C, OHW), 7.0, np.float32)
    idx = np.full((N * C, OHW), -7, np.int32)
    nch = (W + 127) // 128
    nq = (Ho * nch + 3) // 4
    for u in range(N * C * nq):
        pl = u // nq
        for q in range(4):
            cid = 4 * (u - pl * nq) + q
            oh = cid // nch
            lanes = []
            for c4 in range(16):
                col = 128 * (cid - oh * nch) + 8 * c4
                ok = oh < Ho and col < W
                ohc = min(oh, Ho - 1)
                rows = []
                for i in range(3):
                    h = min(max(2 * ohc + i - 1, 0), H - 1)
                    A = _load(xf[pl], 4 * (h * W + col) if ok else OOR, 4, 4 * HW)
                    B = _load(xf[pl], 4 * (h * W + col + 4) if ok else OOR, 4, 4 * HW)
                    E = _load(xf[pl], 4 * (h * W + col - 1) if ok and c4 == 0 and col > 0 else OOR, 1, 4 * HW)[0]
                    rows.append((h, A, B, E))
                lanes.append((oh, col, ok, rows))
            for c4 in range(16):
                oh, col, ok, rows = lanes[c4]
                best, at = [None] * 4, [None] * 4

                def take(k, v, e, first):
                    if first or v > best[k] or np.isnan(v):
                        best[k], at[k] = v, e
                for i, (h, A, B, E) in enumerate(rows):
                    lft = lanes[c4 - 1][3][i][2][3] if c4 > 0 else np.float32(0)
                    e0 = h * W + col
                    L = A[0] if col == 0 else (E if c4 == 0 else lft)
                    eL = e0 if col == 0 else e0 - 1
                    f = i == 0
                    take(0, L, eL, f), take(0, A[0], e0, False), take(0, A[1], e0 + 1, False)
                    take(1, A[1], e0 + 1, f), take(1, A[2], e0 + 2, False), take(1, A[3], e0 + 3, False)
                    take(2, A[3], e0 + 3, f), take(2, B[0], e0 + 4, False), take(2, B[1], e0 + 5, False)
                    take(3, B[1], e0 + 5, f), take(3, B[2], e0 + 6, False), take(3, B[3], e0 + 7, False)
                if ok:
                    o = oh * Wo + col // 2
                    assert 4 * (o + 4) <= 4 * OHW
                    val[pl, o:o + 4] = best
                    idx[pl, o:o + 4] = at
    return val.reshape(N, C, Ho, Wo), idx.reshape(N, C, Ho, Wo)


SHAPES4 = [(1, 1, 3, 4), (1, 2, 5, 64), (1, 1, 4, 68), (2, 1, 3, 128), (1, 1, 2, 200), (1, 1, 2, 1024),
           (1, 2, 7, 60)]


@pytest.mark.parametrize("shape", SHAPES4)
def test_im2col_row_model_equals_the_oracle(shape):
    x = np.random.default_rng(1).standard_normal(shape).astype(np.float32)
    assert np.array_equal(im2col_rows(x), oracle.im2col(x, 3, 3, 1, 1))


@pytest.mark.parametrize("shape", [(1, 1, 1, 2), (1, 2, 3, 64), (1, 1, 2, 34), (2, 1, 3, 128), (1, 1, 2, 200),
                                   (1, 1, 1, 1024), (1, 2, 5, 56), (1, 1, 3, 6)])
def test_upsample2_row_model_is_within_the_oracle_tolerance(shape):
    x = np.random.default_rng(2).standard_normal(shape).astype(np.float32)
    got = upsample2_rows(x)
    assert np.all(np.abs(got - oracle.upsample(x, 2)) <= 1e-5 * oracle.upsample_absmag(x, 2) + 1e-30)


@pytest.mark.parametrize("shape", [(1, 1, 5, 8), (1, 2, 7, 128), (1, 1, 6, 136), (1, 1, 5, 256), (2, 1, 3, 1024)])
@pytest.mark.parametrize("mode", ["normal", "ties", "nan"])
def test_maxpool_row_model_equals_the_oracle(shape, mode):
    g = np.random.default_rng(3)
    x = g.standard_normal(shape).astype(np.float32)
    if mode == "ties":
        x = np.round(x)
    elif mode == "nan":
        x[g.random(shape) < 0.1] = np.nan
        x[g.random(shape) < 0.1] = -np.inf
    v, i = maxpool3s2_rows(x)
    rv, ri = oracle.maxpool(x, 3, 3, 2, 1)
    assert np.array_equal(v, rv, equal_nan=True)
    assert np.array_equal(i, ri)
