// hf_mlp.hip -- learned cost model of the fused-kernel tuner.
//
// A multilayer perceptron (three hidden layers of 64 ReLU units, linear output)
// predicts log2 of a fused launch's time from features of the two solo kernels
// and of the configuration (split, workgroup size, VGPR bound).  It is trained
// on the GPU by the kernels below (forward, mean-squared-error gradient, the
// two backward products, Adam), all deterministic: every output element is
// written by one lane that reduces in a fixed order, with no atomics.  The
// tuner ranks every candidate with it and profiles only the best k; the
// exhaustive search remains the fallback and the reference for its regret.
//
// Parameter layout (one flat fp32 vector): W1[d][64] b1[64] W2[64][64] b2[64]
// W3[64][64] b3[64] W4[64][1] b4[1], row-major W[in][out].
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "hf_runtime.hpp"

namespace hf {

constexpr int kHid = 64;
constexpr int kFeat = HF_MLP_FEATURES;

// ------------------------------------------------------------------ kernels
// Z[i][j] = b[j] + sum_k X[i][k] W[k][j];  H = relu(Z) when H != nullptr.
__global__ void __launch_bounds__(256) k_lin_fwd(const float* __restrict__ X, int n, int din,
                                                 const float* __restrict__ W, const float* __restrict__ b,
                                                 int dout, float* __restrict__ Z, float* __restrict__ H) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * dout) return;
  const int i = t / dout, j = t - (t / dout) * dout;
  float acc = b[j];
  const float* x = X + (size_t)i * din;
  for (int k = 0; k < din; ++k) acc = __builtin_fmaf(x[k], W[k * dout + j], acc);
  Z[t] = acc;
  if (H) H[t] = fmaxf(acc, 0.f);
}

// dz[i] = (2/n)(yhat[i] - y[i]);  loss[0] = (1/n) sum (yhat - y)^2.  One
// workgroup of 1024 lanes: strided partial sums, then a fixed LDS tree.
__global__ void __launch_bounds__(1024) k_mse(const float* __restrict__ yhat, const float* __restrict__ y,
                                              int n, float* __restrict__ dz, float* __restrict__ loss) {
  __shared__ float red[1024];
  float s = 0.f;
  const float inv = 1.0f / (float)n;
  for (int i = threadIdx.x; i < n; i += 1024) {
    const float e = yhat[i] - y[i];
    dz[i] = 2.0f * e * inv;
    s = __builtin_fmaf(e, e, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] * inv;
}

// dW[k][j] = sum_i A[i][k] dZ[i][j] (lanes t < din*dout);  db[j] = sum_i dZ[i][j]
// (lanes din*dout + j).  Sequential over i in row order.
__global__ void __launch_bounds__(256) k_lin_bwd_w(const float* __restrict__ A, const float* __restrict__ dZ,
                                                   int n, int din, int dout, float* __restrict__ dW,
                                                   float* __restrict__ db) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < din * dout) {
    const int k = t / dout, j = t - (t / dout) * dout;
    float acc = 0.f;
    for (int i = 0; i < n; ++i) acc = __builtin_fmaf(A[(size_t)i * din + k], dZ[(size_t)i * dout + j], acc);
    dW[t] = acc;
  } else if (t < din * dout + dout) {
    const int j = t - din * dout;
    float acc = 0.f;
    for (int i = 0; i < n; ++i) acc += dZ[(size_t)i * dout + j];
    db[j] = acc;
  }
}

// dZp[i][k] = (sum_j dZ[i][j] W[k][j]) * (Zp[i][k] > 0): the gradient through
// the layer below and its ReLU.
__global__ void __launch_bounds__(256) k_lin_bwd_x(const float* __restrict__ dZ, const float* __restrict__ W,
                                                   const float* __restrict__ Zp, int n, int din, int dout,
                                                   float* __restrict__ dZp) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * din) return;
  const int i = t / din, k = t - (t / din) * din;
  float acc = 0.f;
  const float* dz = dZ + (size_t)i * dout;
  const float* w = W + (size_t)k * dout;
  for (int j = 0; j < dout; ++j) acc = __builtin_fmaf(dz[j], w[j], acc);
  dZp[t] = Zp[t] > 0.f ? acc : 0.f;
}

// Adam with bias corrections bc1 = 1 - b1^t, bc2 = 1 - b2^t.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int np, float lr,
                                              float b1, float b2, float eps, float bc1, float bc2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np) return;
  const float gi = g[t];
  const float mi = b1 * m[t] + (1.f - b1) * gi;
  const float vi = b2 * v[t] + (1.f - b2) * gi * gi;
  m[t] = mi;
  v[t] = vi;
  p[t] = p[t] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ------------------------------------------------------------------ model state
// An ensemble of `members` networks of the same shape, trained one after the
// other on the same standardised data from different initial weights; the
// prediction is the mean of the members' predictions.  p/m/v point at the
// active member's slice of pall/mall/vall (use_member).
struct MlpModel {
  int d = 0, np = 0, cap_n = 0, t = 0, members = 1;
  bool trained = false;
  float *pall = nullptr, *mall = nullptr, *vall = nullptr;
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  // workspace
  float *X = nullptr, *y = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr;
  float *Z3 = nullptr, *H3 = nullptr, *yh = nullptr, *d4 = nullptr, *d3 = nullptr, *d2 = nullptr,
        *d1 = nullptr, *loss = nullptr;
  std::vector<float> mu, sd;
  float ymu = 0.f, ysd = 1.f;
};

static MlpModel* g_model = nullptr;  // one model per process, on the device that created it
static int g_model_dev = -1;

static void mlp_free_ws(MlpModel* M) {
  float** ws[] = {&M->X, &M->y, &M->Z1, &M->H1, &M->Z2, &M->H2, &M->Z3, &M->H3,
                  &M->yh, &M->d4, &M->d3, &M->d2, &M->d1, &M->loss};
  for (float** q : ws)
    if (*q) {
      (void)hipFree(*q);
      *q = nullptr;
    }
  M->cap_n = 0;
}

static void use_member(MlpModel* M, int k) {
  M->p = M->pall + (size_t)k * M->np;
  M->m = M->mall + (size_t)k * M->np;
  M->v = M->vall + (size_t)k * M->np;
}

void mlp_free() {
  if (!g_model) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(g_model_dev);
  mlp_free_ws(g_model);
  float** ps[] = {&g_model->pall, &g_model->mall, &g_model->vall, &g_model->g};
  for (float** q : ps)
    if (*q) (void)hipFree(*q);
  delete g_model;
  g_model = nullptr;
  (void)hipSetDevice(cur);
}

static int nparams(int d) { return d * kHid + kHid + 2 * (kHid * kHid + kHid) + kHid + 1; }

static int alloc_f(float** q, size_t n) {
  hipError_t e = hipMalloc(q, std::max<size_t>(n, 1) * sizeof(float));
  if (e != hipSuccess) {
    record_hip(e);
    return HF_ENOMEM;
  }
  return HF_OK;
}

static int ensure_ws(MlpModel* M, int n) {
  if (n <= M->cap_n) return HF_OK;
  mlp_free_ws(M);
  const int c = std::max(n, 1024);
  int rc;
  if ((rc = alloc_f(&M->X, (size_t)c * M->d)) || (rc = alloc_f(&M->y, c)) || (rc = alloc_f(&M->Z1, (size_t)c * kHid)) ||
      (rc = alloc_f(&M->H1, (size_t)c * kHid)) || (rc = alloc_f(&M->Z2, (size_t)c * kHid)) ||
      (rc = alloc_f(&M->H2, (size_t)c * kHid)) || (rc = alloc_f(&M->Z3, (size_t)c * kHid)) ||
      (rc = alloc_f(&M->H3, (size_t)c * kHid)) || (rc = alloc_f(&M->yh, c)) || (rc = alloc_f(&M->d4, c)) ||
      (rc = alloc_f(&M->d3, (size_t)c * kHid)) || (rc = alloc_f(&M->d2, (size_t)c * kHid)) ||
      (rc = alloc_f(&M->d1, (size_t)c * kHid)) || (rc = alloc_f(&M->loss, 1)))
    return rc;
  M->cap_n = c;
  return HF_OK;
}

static int model(MlpModel** out) {
  if (!g_model) return HF_ENOMODEL;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return record_hip(e);
  if (dev != g_model_dev) return HF_EINVAL;  // the model lives on another device
  *out = g_model;
  return HF_OK;
}

static int blocks_for(int n) { return std::max(1, (n + 255) / 256); }

#define HF_LAUNCH(...)                                  \
  do {                                                  \
    hipLaunchKernelGGL(__VA_ARGS__);                    \
    hipError_t e_ = hipGetLastError();                  \
    if (e_ != hipSuccess) return record_hip(e_);        \
  } while (0)

// Forward on M->X[n][d] (standardised); fills Z*, H*, yh.
static int forward(MlpModel* M, int n, hipStream_t st) {
  const float* W1 = M->p;
  const float* b1 = W1 + M->d * kHid;
  const float* W2 = b1 + kHid;
  const float* b2 = W2 + kHid * kHid;
  const float* W3 = b2 + kHid;
  const float* b3 = W3 + kHid * kHid;
  const float* W4 = b3 + kHid;
  const float* b4 = W4 + kHid;
  HF_LAUNCH(k_lin_fwd, dim3(blocks_for(n * kHid)), dim3(256), 0, st, M->X, n, M->d, W1, b1, kHid, M->Z1, M->H1);
  HF_LAUNCH(k_lin_fwd, dim3(blocks_for(n * kHid)), dim3(256), 0, st, M->H1, n, kHid, W2, b2, kHid, M->Z2, M->H2);
  HF_LAUNCH(k_lin_fwd, dim3(blocks_for(n * kHid)), dim3(256), 0, st, M->H2, n, kHid, W3, b3, kHid, M->Z3, M->H3);
  HF_LAUNCH(k_lin_fwd, dim3(blocks_for(n)), dim3(256), 0, st, M->H3, n, kHid, W4, b4, 1, M->yh, (float*)nullptr);
  return HF_OK;
}

// Loss and full gradient into M->g (forward must have run on the same X).
static int backward(MlpModel* M, int n, hipStream_t st) {
  const int d = M->d;
  float* gW1 = M->g;
  float* gb1 = gW1 + d * kHid;
  float* gW2 = gb1 + kHid;
  float* gb2 = gW2 + kHid * kHid;
  float* gW3 = gb2 + kHid;
  float* gb3 = gW3 + kHid * kHid;
  float* gW4 = gb3 + kHid;
  float* gb4 = gW4 + kHid;
  const float* W2 = M->p + d * kHid + kHid;
  const float* W3 = W2 + kHid * kHid + kHid;
  const float* W4 = W3 + kHid * kHid + kHid;
  HF_LAUNCH(k_mse, dim3(1), dim3(1024), 0, st, M->yh, M->y, n, M->d4, M->loss);
  HF_LAUNCH(k_lin_bwd_w, dim3(blocks_for(kHid + 1)), dim3(256), 0, st, M->H3, M->d4, n, kHid, 1, gW4, gb4);
  HF_LAUNCH(k_lin_bwd_x, dim3(blocks_for(n * kHid)), dim3(256), 0, st, M->d4, W4, M->Z3, n, kHid, 1, M->d3);
  HF_LAUNCH(k_lin_bwd_w, dim3(blocks_for(kHid * kHid + kHid)), dim3(256), 0, st, M->H2, M->d3, n, kHid, kHid, gW3, gb3);
  HF_LAUNCH(k_lin_bwd_x, dim3(blocks_for(n * kHid)), dim3(256), 0, st, M->d3, W3, M->Z2, n, kHid, kHid, M->d2);
  HF_LAUNCH(k_lin_bwd_w, dim3(blocks_for(kHid * kHid + kHid)), dim3(256), 0, st, M->H1, M->d2, n, kHid, kHid, gW2, gb2);
  HF_LAUNCH(k_lin_bwd_x, dim3(blocks_for(n * kHid)), dim3(256), 0, st, M->d2, W2, M->Z1, n, kHid, kHid, M->d1);
  HF_LAUNCH(k_lin_bwd_w, dim3(blocks_for(d * kHid + kHid)), dim3(256), 0, st, M->X, M->d1, n, d, kHid, gW1, gb1);
  return HF_OK;
}

static int adam(MlpModel* M, float lr, hipStream_t st) {
  M->t += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float bc1 = (float)(1.0 - std::pow(b1, M->t)), bc2 = (float)(1.0 - std::pow(b2, M->t));
  HF_LAUNCH(k_adam, dim3(blocks_for(M->np)), dim3(256), 0, st, M->p, M->g, M->m, M->v, M->np, lr, (float)b1,
            (float)b2, 1e-8f, bc1, bc2);
  return HF_OK;
}

static int upload(float* dst, const float* src, size_t n, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(dst, src, n * sizeof(float), hipMemcpyHostToDevice, st);
  return e == hipSuccess ? HF_OK : record_hip(e);
}
static int download(float* dst, const float* src, size_t n, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(dst, src, n * sizeof(float), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return record_hip(e);
  e = hipStreamSynchronize(st);
  return e == hipSuccess ? HF_OK : record_hip(e);
}

// splitmix64 (Steele, Lea & Flood, OOPSLA 2014): seeded uniform doubles for the
// He-uniform initialisation.
static uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ------------------------------------------------------------------ features
struct SoloFeat {
  double t_ms = 0, bytes = 0, ops = 0;
  double t_blk[3] = {0, 0, 0};  // solo time at blocks 256, 512, 1024
  int kind = 0, vgprs = 0;
};

static void alg_work(const hf_task* t, double* bytes, double* ops) {
  const double n = (double)t->n, c = (double)t->c, h = (double)t->h, w = (double)t->w;
  switch (t->kind) {
    case HF_BN_STATS:
      *bytes = 4.0 * n * c * h * w + 8.0 * c;
      *ops = 4.0 * n * c * h * w;
      break;
    case HF_INT_MIX:
      *bytes = 8.0 * n;
      *ops = 8.0 * n * (double)t->p[0];
      break;
    case HF_IM2COL: {
      const double kh = t->p[0], kw = t->p[1], s = t->p[2], p = t->p[3];
      const double Ho = std::floor((h + 2 * p - kh) / s) + 1, Wo = std::floor((w + 2 * p - kw) / s) + 1;
      const double out = n * c * kh * kw * Ho * Wo;
      *bytes = 4.0 * n * c * h * w + 4.0 * out;
      *ops = 10.0 * out;
      break;
    }
    case HF_LDS_HIST:
      *bytes = n + 1024.0;
      *ops = 3.0 * n;
      break;
    case HF_UPSAMPLE: {
      const double s = t->p[0];
      const double out = n * c * h * w * s * s;
      *bytes = 4.0 * n * c * h * w + 4.0 * out;
      *ops = 20.0 * out;
      break;
    }
    case HF_MAXPOOL: {
      const double kh = t->p[0], kw = t->p[1], s = t->p[2], p = t->p[3];
      const double out = n * c * (std::floor((h + 2 * p - kh) / s) + 1) * (std::floor((w + 2 * p - kw) / s) + 1);
      *bytes = 4.0 * n * c * h * w + (t->out1 ? 8.0 : 4.0) * out;
      *ops = 4.0 * kh * kw * out;
      break;
    }
    case HF_SHA256D:
      *bytes = 32.0 * n;
      *ops = 3.0 * 64 * 24 * n;
      break;
    case HF_BLAKE2B:
      *bytes = 32.0 * n;
      *ops = 12.0 * 8 * 28 * n;
      break;
    case HF_ETHASH:
      *bytes = (64.0 * 128 + 32) * n;
      *ops = (64.0 * 40 / 8 + 80 * 55) * n;  // the walk, then the 80 SHA-512 rounds of the seed
      break;
  }
}

// Times the task alone at each block size (6 launches each, the first a warm
// up; the median of the other five).  `cost`, if given, accumulates the
// launches made and their summed time in milliseconds.
static int solo_feat(DeviceState* s, const hf_task* t, hipStream_t st, SoloFeat* f, FeatCost* cost) {
  f->kind = t->kind;
  alg_work(t, &f->bytes, &f->ops);
  double best = 1e30;
  const int blocks[] = {256, 512, 1024};
  for (int bi = 0; bi < 3; ++bi) {
    std::vector<float> ts;
    for (int r = 0; r < 6; ++r) {
      hipError_t e = hipEventRecord(s->ev_start, st);
      if (e != hipSuccess) return record_hip(e);
      int rc = launch_solo(s, t, blocks[bi], 0, 0, st);
      if (rc != HF_OK) return rc;
      if ((e = hipEventRecord(s->ev_stop, st)) != hipSuccess) return record_hip(e);
      if ((rc = wait_event(s->ev_stop)) != HF_OK) return rc;
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, s->ev_start, s->ev_stop)) != hipSuccess) return record_hip(e);
      if (cost) {
        cost->launches += 1;
        cost->ms += ms;
      }
      if (r > 0) ts.push_back(ms);  // the first launch warms up
    }
    std::sort(ts.begin(), ts.end());
    f->t_blk[bi] = std::max((double)ts[ts.size() / 2], 1e-4);
    best = std::min(best, f->t_blk[bi]);
  }
  f->t_ms = best;
  hf_kernel_info info;
  int rc = kernel_info(s, find_kernel(t->kind, -1, 1024, 0)->fn, 1024, &info);
  if (rc != HF_OK) return rc;
  f->vgprs = info.vgprs;
  return HF_OK;
}

// Features of one candidate (kFeat values), kernels in canonical order (the
// smaller kind first; the split fraction refers to that kernel):
//   per kernel (kPerKernel each): one-hot kind (HF_NUM_KINDS); log2 solo time
//   at blocks 256, 512, 1024; log2 algorithmic MB and mega-lane-ops; fractions
//   of the HBM and integer-ALU peaks the best solo run reached;
//   configuration (10): split fraction s = 64*split_waves/block; log2(block/512);
//   VGPR bound / 128 (1 when unbounded); resident waves per SIMD / 8;
//   log2(t_a(block)/s), log2(t_b(block)/(1-s)) and the log2 of their maximum,
//   with t_k(block) the solo time at the candidate's block size; the fused
//   instantiation's spill bytes per lane (log2(1 + bytes) / 8) and VGPRs / 128;
//   log2 of the sum of the best solo times (the last feature).
constexpr int kPerKernel = HF_NUM_KINDS + 7;
constexpr int kCfg = 2 * kPerKernel;
static_assert(kCfg + 10 == kFeat, "feature layout and HF_MLP_FEATURES disagree");

static void fill_features(const SoloFeat& fa0, const SoloFeat& fb0, const hf_config& c,
                          const hf_kernel_info& fused, float* x) {
  const int waves_per_simd = fused.waves_per_simd;
  auto l2 = [](double v) { return (float)std::log2(std::max(v, 1e-30)); };
  // canonical order: the kernel of the smaller kind first, with the split
  // fraction mirrored, so (a, b, s) and (b, a, 1 - s) -- the same fused kernel
  // -- get the same features
  const bool swap = fa0.kind > fb0.kind;
  const SoloFeat& fa = swap ? fb0 : fa0;
  const SoloFeat& fb = swap ? fa0 : fb0;
  const SoloFeat* f[2] = {&fa, &fb};
  for (int k = 0; k < 2; ++k) {
    float* o = x + kPerKernel * k;
    for (int i = 0; i < HF_NUM_KINDS; ++i) o[i] = (f[k]->kind == i) ? 1.f : 0.f;
    float* q = o + HF_NUM_KINDS;
    q[0] = l2(f[k]->t_blk[0]);
    q[1] = l2(f[k]->t_blk[1]);
    q[2] = l2(f[k]->t_blk[2]);
    q[3] = l2(f[k]->bytes / 1e6 + 1e-3);
    q[4] = l2(f[k]->ops / 1e6 + 1e-3);
    q[5] = (float)(f[k]->bytes / (f[k]->t_ms * 1e-3) / 8e12);
    q[6] = (float)(f[k]->ops / (f[k]->t_ms * 1e-3) / 39.3216e12);
  }
  const int bi = c.block == 256 ? 0 : (c.block == 512 ? 1 : 2);
  const double W = c.block / 64.0;
  const double s = swap ? 1.0 - c.split_waves / W : c.split_waves / W;
  float* g = x + kCfg;
  g[0] = (float)s;
  g[1] = l2(c.block / 512.0);
  g[2] = c.vgpr_cap == 0 ? 1.f : c.vgpr_cap / 128.f;
  g[3] = waves_per_simd / 8.f;
  const double ta = fa.t_blk[bi] / s, tb = fb.t_blk[bi] / (1.0 - s);
  g[4] = l2(ta);
  g[5] = l2(tb);
  g[6] = l2(std::max(ta, tb));
  g[7] = (float)(std::log2(1.0 + std::max(0, fused.spill_bytes)) / 8.0);
  g[8] = fused.vgprs / 128.f;
  g[9] = l2(fa.t_ms + fb.t_ms);
}

int featurize(DeviceState* s, const hf_pair* pr, const hf_config* cfg, int n, hipStream_t st, float* X,
              FeatCost* cost) {
  SoloFeat fa, fb;
  int rc;
  if ((rc = solo_feat(s, &pr->a, st, &fa, cost)) != HF_OK) return rc;
  if ((rc = solo_feat(s, &pr->b, st, &fb, cost)) != HF_OK) return rc;
  for (int i = 0; i < n; ++i) {
    hf_kernel_info info;
    if ((rc = hf_fused_info(pr->a.kind, pr->b.kind, cfg[i].block, cfg[i].vgpr_cap, &info)) != HF_OK) return rc;
    fill_features(fa, fb, cfg[i], info, X + (size_t)i * kFeat);
  }
  return HF_OK;
}

// Standardise raw features / predictions with the model's statistics.
static void standardise(const MlpModel* M, const float* X, int n, std::vector<float>* out) {
  out->resize((size_t)n * M->d);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < M->d; ++k)
      (*out)[(size_t)i * M->d + k] = (X[(size_t)i * M->d + k] - M->mu[k]) / M->sd[k];
}

// Mean of the members' predictions, in the units of the training targets.
static int predict(MlpModel* M, const float* X, int n, float* y, hipStream_t st) {
  int rc;
  if ((rc = ensure_ws(M, n)) != HF_OK) return rc;
  std::vector<float> xs, yk(n);
  standardise(M, X, n, &xs);
  if ((rc = upload(M->X, xs.data(), xs.size(), st)) != HF_OK) return rc;
  std::vector<double> acc(n, 0.0);
  for (int k = 0; k < M->members; ++k) {
    use_member(M, k);
    if ((rc = forward(M, n, st)) != HF_OK) break;
    if ((rc = download(yk.data(), M->yh, n, st)) != HF_OK) break;
    for (int i = 0; i < n; ++i) acc[i] += yk[i];
  }
  use_member(M, 0);
  if (rc != HF_OK) return rc;
  for (int i = 0; i < n; ++i) y[i] = (float)(acc[i] / M->members) * M->ysd + M->ymu;
  return HF_OK;
}

int mlp_rank(DeviceState* s, const hf_pair* pr, const std::vector<hf_config>& cands, hipStream_t st,
             std::vector<int>* order, FeatCost* cost) {
  MlpModel* M = nullptr;
  int rc = model(&M);
  if (rc != HF_OK) return rc;
  if (!M->trained || M->d != kFeat) return HF_ENOMODEL;
  const int n = (int)cands.size();
  std::vector<float> X((size_t)n * kFeat), y(n);
  if ((rc = featurize(s, pr, cands.data(), n, st, X.data(), cost)) != HF_OK) return rc;
  if ((rc = predict(M, X.data(), n, y.data(), st)) != HF_OK) return rc;
  order->resize(n);
  std::iota(order->begin(), order->end(), 0);
  std::stable_sort(order->begin(), order->end(), [&](int a, int b) { return y[a] < y[b]; });
  return HF_OK;
}

}  // namespace hf

using namespace hf;

extern "C" {

int hf_mlp_init_ensemble(int d_in, uint64_t seed, int members) {
  if (d_in < 1 || d_in > 4096 || members < 1 || members > HF_MLP_MAX_MEMBERS) return HF_EINVAL;
  int rc;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  mlp_free();
  MlpModel* M = new MlpModel();
  M->d = d_in;
  M->np = nparams(d_in);
  M->members = members;
  const size_t all = (size_t)members * M->np;
  if ((rc = alloc_f(&M->pall, all)) || (rc = alloc_f(&M->mall, all)) || (rc = alloc_f(&M->vall, all)) ||
      (rc = alloc_f(&M->g, M->np))) {
    float** ps[] = {&M->pall, &M->mall, &M->vall, &M->g};
    for (float** q : ps)
      if (*q) (void)hipFree(*q);
    delete M;
    return rc;
  }
  use_member(M, 0);
  // He-uniform weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)), zero biases;
  // member k draws from the splitmix64 stream seeded with seed + k
  std::vector<float> host(all, 0.f);
  const int dims[5] = {d_in, kHid, kHid, kHid, 1};
  for (int k = 0; k < members; ++k) {
    uint64_t st = seed + (uint64_t)k;
    size_t o = (size_t)k * M->np;
    for (int l = 0; l < 4; ++l) {
      const double lim = std::sqrt(6.0 / dims[l]);
      for (int i = 0; i < dims[l] * dims[l + 1]; ++i) {
        const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
        host[o++] = (float)((2.0 * u - 1.0) * lim);
      }
      o += dims[l + 1];
    }
  }
  M->mu.assign(d_in, 0.f);
  M->sd.assign(d_in, 1.f);
  g_model = M;
  g_model_dev = s->device;
  hipError_t e = hipMemcpy(M->pall, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return record_hip(e);
  if ((e = hipMemset(M->mall, 0, all * sizeof(float))) != hipSuccess) return record_hip(e);
  if ((e = hipMemset(M->vall, 0, all * sizeof(float))) != hipSuccess) return record_hip(e);
  return HF_OK;
}

int hf_mlp_init(int d_in, uint64_t seed) { return hf_mlp_init_ensemble(d_in, seed, 1); }

int hf_mlp_members(void) {
  MlpModel* M = nullptr;
  int rc = model(&M);
  return rc != HF_OK ? rc : M->members;
}

int hf_mlp_num_params(void) {
  MlpModel* M = nullptr;
  int rc = model(&M);
  return rc != HF_OK ? rc : M->np;
}

int hf_mlp_get_params(float* host, int64_t n) {
  MlpModel* M = nullptr;
  int rc = model(&M);
  if (rc != HF_OK) return rc;
  if (!host || n != M->np) return HF_EINVAL;
  return download(host, M->p, M->np, nullptr);
}

int hf_mlp_set_params(const float* host, int64_t n) {
  MlpModel* M = nullptr;
  int rc = model(&M);
  if (rc != HF_OK) return rc;
  if (!host || n != M->np) return HF_EINVAL;
  if ((rc = upload(M->p, host, M->np, nullptr)) != HF_OK) return rc;
  hipError_t e = hipStreamSynchronize(nullptr);
  return e == hipSuccess ? HF_OK : record_hip(e);
}

int hf_mlp_grad(const float* X, const float* y, int n, float* loss_out, float* grad_out) {
  if (!X || !y || n < 1 || !loss_out || !grad_out) return HF_EINVAL;
  MlpModel* M = nullptr;
  int rc = model(&M);
  if (rc != HF_OK) return rc;
  if ((rc = ensure_ws(M, n)) != HF_OK) return rc;
  if ((rc = upload(M->X, X, (size_t)n * M->d, nullptr)) || (rc = upload(M->y, y, n, nullptr)) ||
      (rc = forward(M, n, nullptr)) || (rc = backward(M, n, nullptr)))
    return rc;
  if ((rc = download(loss_out, M->loss, 1, nullptr)) != HF_OK) return rc;
  return download(grad_out, M->g, M->np, nullptr);
}

int hf_mlp_step(const float* X, const float* y, int n, float lr, float* loss_out) {
  if (!X || !y || n < 1 || lr <= 0.f) return HF_EINVAL;
  MlpModel* M = nullptr;
  int rc = model(&M);
  if (rc != HF_OK) return rc;
  if ((rc = ensure_ws(M, n)) != HF_OK) return rc;
  if ((rc = upload(M->X, X, (size_t)n * M->d, nullptr)) || (rc = upload(M->y, y, n, nullptr)) ||
      (rc = forward(M, n, nullptr)) || (rc = backward(M, n, nullptr)) || (rc = adam(M, lr, nullptr)))
    return rc;
  return loss_out ? download(loss_out, M->loss, 1, nullptr) : HF_OK;
}

int hf_mlp_adam_reset(void) {
  MlpModel* M = nullptr;
  int rc = model(&M);
  if (rc != HF_OK) return rc;
  M->t = 0;
  hipError_t e;
  if ((e = hipMemset(M->m, 0, M->np * sizeof(float))) != hipSuccess) return record_hip(e);
  if ((e = hipMemset(M->v, 0, M->np * sizeof(float))) != hipSuccess) return record_hip(e);
  return HF_OK;
}

int hf_mlp_train(const float* X, const float* y, int n, int d, int epochs, float lr, float* loss_out) {
  if (!X || !y || n < 2 || epochs < 1 || lr <= 0.f) return HF_EINVAL;
  MlpModel* M = nullptr;
  int rc = model(&M);
  if (rc != HF_OK) return rc;
  if (d != M->d) return HF_EINVAL;
  // feature and target standardisation from the training set (double sums)
  for (int k = 0; k < d; ++k) {
    double s = 0, q = 0;
    for (int i = 0; i < n; ++i) s += X[(size_t)i * d + k];
    const double mu = s / n;
    for (int i = 0; i < n; ++i) q += (X[(size_t)i * d + k] - mu) * (X[(size_t)i * d + k] - mu);
    const double sd = std::sqrt(q / n);
    M->mu[k] = (float)mu;
    M->sd[k] = sd > 1e-6 ? (float)sd : 1.f;
  }
  {
    double s = 0, q = 0;
    for (int i = 0; i < n; ++i) s += y[i];
    const double mu = s / n;
    for (int i = 0; i < n; ++i) q += (y[i] - mu) * (y[i] - mu);
    M->ymu = (float)mu;
    M->ysd = std::sqrt(q / n) > 1e-6 ? (float)std::sqrt(q / n) : 1.f;
  }
  std::vector<float> xs, ys(n);
  standardise(M, X, n, &xs);
  for (int i = 0; i < n; ++i) ys[i] = (y[i] - M->ymu) / M->ysd;
  if ((rc = ensure_ws(M, n)) != HF_OK) return rc;
  if ((rc = upload(M->X, xs.data(), xs.size(), nullptr)) || (rc = upload(M->y, ys.data(), n, nullptr))) return rc;
  // every member from its own initial weights, on the same data
  double lsum = 0.0;
  for (int k = 0; k < M->members; ++k) {
    use_member(M, k);
    M->t = 0;
    hipError_t e;
    if ((e = hipMemset(M->m, 0, M->np * sizeof(float))) != hipSuccess ||
        (e = hipMemset(M->v, 0, M->np * sizeof(float))) != hipSuccess) {
      use_member(M, 0);
      return record_hip(e);
    }
    for (int ep = 0; ep < epochs && rc == HF_OK; ++ep)
      if ((rc = forward(M, n, nullptr)) || (rc = backward(M, n, nullptr)) || (rc = adam(M, lr, nullptr))) break;
    // loss of the member's final parameters
    if (rc == HF_OK && ((rc = forward(M, n, nullptr)) == HF_OK) && ((rc = backward(M, n, nullptr)) == HF_OK)) {
      float l = 0.f;
      rc = download(&l, M->loss, 1, nullptr);
      lsum += l;
    }
    if (rc != HF_OK) break;
  }
  use_member(M, 0);
  if (rc != HF_OK) return rc;
  if (loss_out) *loss_out = (float)(lsum / M->members);
  M->trained = true;
  return HF_OK;
}

int hf_mlp_predict(const float* X, int n, float* y_out) {
  if (!X || n < 1 || !y_out) return HF_EINVAL;
  MlpModel* M = nullptr;
  int rc = model(&M);
  if (rc != HF_OK) return rc;
  return predict(M, X, n, y_out, nullptr);
}

int hf_mlp_save(const char* path) {
  MlpModel* M = nullptr;
  int rc = model(&M);
  if (rc != HF_OK) return rc;
  if (!path) return HF_EINVAL;
  const size_t all = (size_t)M->members * M->np;
  std::vector<float> p(all);
  if ((rc = download(p.data(), M->pall, all, nullptr)) != HF_OK) return rc;
  FILE* f = std::fopen(path, "wb");
  if (!f) return HF_EINVAL;
  const char magic[8] = {'H', 'F', 'M', 'L', 'P', '2', 0, 0};
  const int32_t hdr[4] = {M->d, M->np, M->trained ? 1 : 0, M->members};
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 4, f) == 4 &&
            std::fwrite(&M->ymu, 4, 1, f) == 1 && std::fwrite(&M->ysd, 4, 1, f) == 1 &&
            std::fwrite(M->mu.data(), 4, M->d, f) == (size_t)M->d &&
            std::fwrite(M->sd.data(), 4, M->d, f) == (size_t)M->d &&
            std::fwrite(p.data(), 4, all, f) == all;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? HF_OK : HF_EINVAL;
}

int hf_mlp_load(const char* path) {
  if (!path) return HF_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) return HF_EINVAL;
  char magic[8];
  int32_t hdr[4];
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "HFMLP2", 6) == 0 &&
            std::fread(hdr, 4, 4, f) == 4 && hdr[0] >= 1 && hdr[0] <= 4096 && hdr[1] == nparams(hdr[0]) &&
            hdr[3] >= 1 && hdr[3] <= HF_MLP_MAX_MEMBERS;
  if (!ok) {
    std::fclose(f);
    return HF_EINVAL;
  }
  float ymu = 0, ysd = 1;
  const size_t all = (size_t)hdr[3] * hdr[1];
  std::vector<float> mu(hdr[0]), sd(hdr[0]), p(all);
  ok = std::fread(&ymu, 4, 1, f) == 1 && std::fread(&ysd, 4, 1, f) == 1 &&
       std::fread(mu.data(), 4, hdr[0], f) == (size_t)hdr[0] && std::fread(sd.data(), 4, hdr[0], f) == (size_t)hdr[0] &&
       std::fread(p.data(), 4, all, f) == all;
  std::fclose(f);
  if (!ok) return HF_EINVAL;
  int rc = hf_mlp_init_ensemble(hdr[0], 0, hdr[3]);
  if (rc != HF_OK) return rc;
  if ((rc = upload(g_model->pall, p.data(), all, nullptr)) != HF_OK) return rc;
  hipError_t e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return record_hip(e);
  g_model->mu = mu;
  g_model->sd = sd;
  g_model->ymu = ymu;
  g_model->ysd = ysd;
  g_model->trained = hdr[2] != 0;
  return HF_OK;
}

int hf_featurize(const hf_pair* pr, const hf_config* cfg, int n, void* stream, float* X_out) {
  if (!pr || !cfg || n < 1 || !X_out) return HF_EINVAL;
  int rc;
  for (int i = 0; i < n; ++i)
    if ((rc = hf_validate_fused(pr, &cfg[i])) != HF_OK) return rc;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  return featurize(s, pr, cfg, n, static_cast<hipStream_t>(stream), X_out, nullptr);
}

}  // extern "C"
