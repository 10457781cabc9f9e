/*
 * hf_oracle.c -- plain, sequential CPU oracle for the kernels that horizontal
 * fusion combines.  TEST INFRASTRUCTURE ONLY: it is linked by the test suite,
 * by the smoke check and by the CPU-baseline leg of the benchmark, never by the
 * library.  It shares no code, header or constant table with the GPU path.
 *
 * Floating point is accumulated in double.  Every function is the plain
 * definition of what the kernel computes, written out loop by loop:
 *
 *   - A horizontally fused kernel is functionally equivalent to running its two
 *     original kernels (Sec. I-A; Sec. III-A "Replace Synchronization Barriers"),
 *     so the oracle of a fused launch is the pair of oracles of its kernels.
 *   - bn_stats : the statistics kernel of the normalisation example (Sec. II-C;
 *     "Batchnorm" in Sec. IV-A): per-channel mean and variance.  Reading taken:
 *     the biased variance (divided by the element count), as normalisation uses.
 *   - lds_hist : the histogram kernel of Sec. II-C ("Hist", Sec. IV-A).  Reading
 *     taken for uint8 input and 256 bins: the bin of a value is the value.
 *   - im2col   : "Im2Col rearranges the input image blocks into columns"
 *     (Sec. IV-A).  Reading taken: the unfold layout [N][C*kh*kw][Ho*Wo], row
 *     index (c*kh + i)*kw + j, zero padding.
 *   - upsample : 2-D bilinear upsampling (Sec. IV-A).  Reading taken: half-pixel
 *     centres (align_corners = false), source coordinate clamped at 0, upper
 *     neighbour clamped at the last row/column, linear interpolation written as
 *     a + l*(b - a), first along x then along y.
 *   - maxpool  : "Maxpool applies a 2D maxpooling over an input matrix" (Sec.
 *     IV-A; the kernel is PyTorch's).  Readings taken: square-or-rectangular
 *     window kh x kw, one stride, one zero-count padding (padded positions never
 *     win), floor output size, no dilation; outputs the maximum and the flat
 *     index h*W + w of the element it came from.  The scan order is row-major
 *     over the window; an element replaces the running maximum when it is
 *     greater or is NaN, and the first valid element starts the scan, so ties
 *     keep the first occurrence and a NaN propagates (the last NaN's index).
 *   - int_mix  : stands in for the compute-bound hash kernels of Sec. IV-A.  It
 *     is not defined by the paper; the definition fixed here is R rounds of
 *       x ^= x << 13;  x ^= x >> 17;  x ^= x << 5;    (Marsaglia's xorshift32)
 *       x = x * 2654435761 + r                         (mod 2^32, r = round index)
 *
 * Parity pins (closed forms, published values, library routines, brute force)
 * live in the oracle tests; none of them calls back into this file's formulas.
 *
 * The file is compiled twice: sequentially (the oracle the tests use) and with
 * OpenMP (-fopenmp), where the `omp` pragmas below spread independent units
 * over the host's cores -- channels, elements, (image, channel) planes, and
 * thread-private histograms summed at the end.  The arithmetic of every unit
 * is the same in both builds, so both give the same results (bn_stats sums
 * each channel in one thread, in the same order).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_EXPORT __attribute__((visibility("default")))

/* Threads the parallel loops use (1 in the sequential build). */
OR_EXPORT int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ bn_stats */
/* mean[c] = (1/M) sum_{n,h,w} x[n,c,h,w];  var[c] = (1/M) sum (x - mean[c])^2,
 * M = N*H*W, two passes in double.  Returns 0, or -1 when M == 0. */
OR_EXPORT int oracle_bn_stats(const float* x, int64_t N, int64_t C, int64_t H,
                              int64_t W, double* mean, double* var) {
  const int64_t HW = H * W;
  const int64_t M = N * HW;
  if (M <= 0) return -1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t c = 0; c < C; ++c) {
    double s = 0.0;
    for (int64_t n = 0; n < N; ++n) {
      const float* plane = x + (n * C + c) * HW;
      for (int64_t k = 0; k < HW; ++k) s += (double)plane[k];
    }
    const double mu = s / (double)M;
    double ss = 0.0;
    for (int64_t n = 0; n < N; ++n) {
      const float* plane = x + (n * C + c) * HW;
      for (int64_t k = 0; k < HW; ++k) {
        const double d = (double)plane[k] - mu;
        ss += d * d;
      }
    }
    mean[c] = mu;
    var[c] = ss / (double)M;
  }
  return 0;
}

/* ------------------------------------------------------------------ int_mix */
OR_EXPORT void oracle_int_mix(const uint32_t* seed, int64_t n, int32_t rounds,
                              uint32_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    uint32_t x = seed[i];
    for (int32_t r = 0; r < rounds; ++r) {
      x ^= x << 13;
      x ^= x >> 17;
      x ^= x << 5;
      x = x * 2654435761u + (uint32_t)r;
    }
    out[i] = x;
  }
}

/* ------------------------------------------------------------------ lds_hist */
/* counts[b] = number of i with in[i] == b, b in [0, 256). */
OR_EXPORT void oracle_hist256(const uint8_t* in, int64_t n, uint64_t* counts) {
  for (int b = 0; b < 256; ++b) counts[b] = 0;
#pragma omp parallel for schedule(static) reduction(+ : counts[:256])
  for (int64_t i = 0; i < n; ++i) counts[in[i]] += 1;
}

/* ------------------------------------------------------------------ im2col */
/* out[n][(c*kh + i)*kw + j][oh*Wo + ow] = x[n][c][oh*s - p + i][ow*s - p + j]
 * when the source row and column are inside the image, else 0. */
OR_EXPORT int oracle_im2col(const float* x, int64_t N, int64_t C, int64_t H,
                            int64_t W, int32_t kh, int32_t kw, int32_t s,
                            int32_t p, float* out) {
  if (kh <= 0 || kw <= 0 || s <= 0 || p < 0) return -1;
  const int64_t Ho = (H + 2 * p - kh) / s + 1;
  const int64_t Wo = (W + 2 * p - kw) / s + 1;
  if (Ho <= 0 || Wo <= 0) return -1;
  const int64_t rows = C * kh * kw;
#pragma omp parallel for collapse(2) schedule(static)
  for (int64_t n = 0; n < N; ++n)
    for (int64_t c = 0; c < C; ++c)
      for (int32_t i = 0; i < kh; ++i)
        for (int32_t j = 0; j < kw; ++j) {
          const int64_t row = (c * kh + i) * kw + j;
          float* dst = out + (n * rows + row) * (Ho * Wo);
          for (int64_t oh = 0; oh < Ho; ++oh)
            for (int64_t ow = 0; ow < Wo; ++ow) {
              const int64_t ih = oh * s - p + i;
              const int64_t iw = ow * s - p + j;
              float v = 0.0f;
              if (ih >= 0 && ih < H && iw >= 0 && iw < W)
                v = x[((n * C + c) * H + ih) * W + iw];
              dst[oh * Wo + ow] = v;
            }
        }
  return 0;
}

/* ------------------------------------------------------------------ upsample */
/* Source coordinate of output index o for an integer factor s along an axis of
 * length L: t = max(0, (o + 0.5)/s - 0.5), i0 = floor(t), i1 = min(i0 + 1, L - 1),
 * weight l = t - i0. */
static void src_coord(int64_t o, int32_t s, int64_t L, int64_t* i0, int64_t* i1,
                      double* l) {
  double t = ((double)o + 0.5) / (double)s - 0.5;
  if (t < 0.0) t = 0.0;
  int64_t a = (int64_t)floor(t);
  if (a > L - 1) a = L - 1;
  *i0 = a;
  *i1 = (a + 1 < L) ? a + 1 : L - 1;
  *l = t - (double)a;
}

OR_EXPORT int oracle_upsample(const float* x, int64_t N, int64_t C, int64_t H,
                              int64_t W, int32_t s, double* out) {
  if (s <= 0 || H <= 0 || W <= 0) return -1;
  const int64_t Ho = H * s, Wo = W * s;
#pragma omp parallel for collapse(2) schedule(static)
  for (int64_t n = 0; n < N; ++n)
    for (int64_t c = 0; c < C; ++c) {
      const float* img = x + (n * C + c) * H * W;
      double* dst = out + (n * C + c) * Ho * Wo;
      for (int64_t oy = 0; oy < Ho; ++oy) {
        int64_t y0, y1;
        double ly;
        src_coord(oy, s, H, &y0, &y1, &ly);
        for (int64_t ox = 0; ox < Wo; ++ox) {
          int64_t x0, x1;
          double lx;
          src_coord(ox, s, W, &x0, &x1, &lx);
          const double a = img[y0 * W + x0], b = img[y0 * W + x1];
          const double c2 = img[y1 * W + x0], d = img[y1 * W + x1];
          const double top = a + lx * (b - a);
          const double bot = c2 + lx * (d - c2);
          dst[oy * Wo + ox] = top + ly * (bot - top);
        }
      }
    }
  return 0;
}

/* Condition-aware error scale of upsample output o: sum_k |w_k * x_k| over the
 * four interpolation taps, in double.  Tolerances are stated relative to it,
 * because a plain relative error is ill-posed where the taps cancel. */
OR_EXPORT int oracle_upsample_absmag(const float* x, int64_t N, int64_t C,
                                     int64_t H, int64_t W, int32_t s,
                                     double* out) {
  if (s <= 0 || H <= 0 || W <= 0) return -1;
  const int64_t Ho = H * s, Wo = W * s;
#pragma omp parallel for collapse(2) schedule(static)
  for (int64_t n = 0; n < N; ++n)
    for (int64_t c = 0; c < C; ++c) {
      const float* img = x + (n * C + c) * H * W;
      double* dst = out + (n * C + c) * Ho * Wo;
      for (int64_t oy = 0; oy < Ho; ++oy) {
        int64_t y0, y1;
        double ly;
        src_coord(oy, s, H, &y0, &y1, &ly);
        for (int64_t ox = 0; ox < Wo; ++ox) {
          int64_t x0, x1;
          double lx;
          src_coord(ox, s, W, &x0, &x1, &lx);
          dst[oy * Wo + ox] = fabs((1 - ly) * (1 - lx) * img[y0 * W + x0]) +
                              fabs((1 - ly) * lx * img[y0 * W + x1]) +
                              fabs(ly * (1 - lx) * img[y1 * W + x0]) +
                              fabs(ly * lx * img[y1 * W + x1]);
        }
      }
    }
  return 0;
}

/* ------------------------------------------------------------------- maxpool */
/* out[n][c][oh][ow] = max over the window's in-range elements of
 * x[n][c][oh*s - p + i][ow*s - p + j], idx = the winner's h*W + w (see the
 * scan rule above).  Ho = (H + 2p - kh)/s + 1, Wo likewise.  Returns -1 when a
 * window can hold no in-range element (p >= kh or p >= kw) or sizes are bad. */
OR_EXPORT int oracle_maxpool(const float* x, int64_t N, int64_t C, int64_t H, int64_t W, int32_t kh,
                             int32_t kw, int32_t s, int32_t p, float* out, int32_t* idx) {
  if (kh < 1 || kw < 1 || s < 1 || p < 0 || p >= kh || p >= kw) return -1;
  if (H + 2 * p < kh || W + 2 * p < kw) return -1;
  const int64_t Ho = (H + 2 * p - kh) / s + 1, Wo = (W + 2 * p - kw) / s + 1;
  int bad = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(| : bad)
  for (int64_t n = 0; n < N; ++n)
    for (int64_t c = 0; c < C; ++c) {
      const float* img = x + (n * C + c) * H * W;
      float* dst = out + (n * C + c) * Ho * Wo;
      int32_t* dix = idx + (n * C + c) * Ho * Wo;
      for (int64_t oh = 0; oh < Ho; ++oh)
        for (int64_t ow = 0; ow < Wo; ++ow) {
          int have = 0;
          float best = 0.0f;
          int64_t at = -1;
          for (int32_t i = 0; i < kh; ++i) {
            const int64_t h = oh * s - p + i;
            if (h < 0 || h >= H) continue;
            for (int32_t j = 0; j < kw; ++j) {
              const int64_t w = ow * s - p + j;
              if (w < 0 || w >= W) continue;
              const float v = img[h * W + w];
              if (!have || v > best || isnan(v)) {
                best = v;
                at = h * W + w;
                have = 1;
              }
            }
          }
          if (!have) bad = 1; /* a window with no in-range element */
          dst[oh * Wo + ow] = best;
          dix[oh * Wo + ow] = (int32_t)at;
        }
    }
  return bad ? -1 : 0;
}

/* --------------------------------------------------------------- Ethash-like */
/* The Ethash-like walk written out in C for the full-size checks; the same
 * definition as oracle/hashes.py (the tests check the two against each other).
 * The seeds come in from the caller: seeds[16 i .. 16 i + 15] are the sixteen
 * little-endian words of SHA-512 of instance i's message.  mix_j = s_(j mod 16);
 * for a = 0..63: p = fnv(a ^ s0, mix_(a mod 32)) mod rows,
 * mix_j = fnv(mix_j, T[p][j]);  out_k = fnv(fnv(fnv(mix_4k, mix_4k+1),
 * mix_4k+2), mix_4k+3), as 8 little-endian words per instance. */
static uint32_t fnv32(uint32_t a, uint32_t b) { return (a * 16777619u) ^ b; }

OR_EXPORT int oracle_ethash_like(const uint32_t* seeds, int64_t n, const uint32_t* table, int64_t rows,
                                 uint8_t* out) {
  if (rows < 1 || n < 0) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t* s = seeds + 16 * i;
    uint32_t mix[32];
    for (int j = 0; j < 32; ++j) mix[j] = s[j % 16];
    for (uint32_t a = 0; a < 64; ++a) {
      const uint64_t p = (uint64_t)fnv32(a ^ s[0], mix[a % 32]) % (uint64_t)rows;
      const uint32_t* row = table + p * 32;
      for (int j = 0; j < 32; ++j) mix[j] = fnv32(mix[j], row[j]);
    }
    for (int k = 0; k < 8; ++k) {
      const uint32_t v = fnv32(fnv32(fnv32(mix[4 * k], mix[4 * k + 1]), mix[4 * k + 2]), mix[4 * k + 3]);
      for (int b = 0; b < 4; ++b) out[32 * i + 4 * k + b] = (uint8_t)(v >> (8 * b));
    }
  }
  return 0;
}
