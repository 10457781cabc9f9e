// hf_runtime.hip -- host side of the C ABI declared in include/hfuse.h.
//
// Validation and argument marshalling (host only, no HIP call), the kernel
// registry, grid sizing from occupancy, scratch arenas, stream/event plumbing
// for the solo, unfused (back-to-back or two-stream) and fused launches, and
// the microbenchmark kernels.  The tuner lives in hf_tune.hip.
#include "hf_runtime.hpp"

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <thread>

namespace hf {

// ------------------------------------------------------------------ errors
static thread_local int g_last_hip = 0;
int record_hip(hipError_t e) {
  g_last_hip = (int)e;
  return HF_EHIP;
}

// ------------------------------------------------------------------ registry
#define HF_DECLARE_TABLE(KA, KB) const KernelEntry* hf_table_##KA##_##KB(int* count);
HF_DECLARE_TABLE(0, 0) HF_DECLARE_TABLE(0, 1) HF_DECLARE_TABLE(0, 2) HF_DECLARE_TABLE(0, 3)
HF_DECLARE_TABLE(0, 4) HF_DECLARE_TABLE(0, 5) HF_DECLARE_TABLE(0, 6) HF_DECLARE_TABLE(0, 7)
HF_DECLARE_TABLE(0, 8) HF_DECLARE_TABLE(1, 1) HF_DECLARE_TABLE(1, 2) HF_DECLARE_TABLE(1, 3)
HF_DECLARE_TABLE(1, 4) HF_DECLARE_TABLE(1, 5) HF_DECLARE_TABLE(1, 6) HF_DECLARE_TABLE(1, 7)
HF_DECLARE_TABLE(1, 8) HF_DECLARE_TABLE(2, 2) HF_DECLARE_TABLE(2, 3) HF_DECLARE_TABLE(2, 4)
HF_DECLARE_TABLE(2, 5) HF_DECLARE_TABLE(2, 6) HF_DECLARE_TABLE(2, 7) HF_DECLARE_TABLE(2, 8)
HF_DECLARE_TABLE(3, 3) HF_DECLARE_TABLE(3, 4) HF_DECLARE_TABLE(3, 5) HF_DECLARE_TABLE(3, 6)
HF_DECLARE_TABLE(3, 7) HF_DECLARE_TABLE(3, 8) HF_DECLARE_TABLE(4, 4) HF_DECLARE_TABLE(4, 5)
HF_DECLARE_TABLE(4, 6) HF_DECLARE_TABLE(4, 7) HF_DECLARE_TABLE(4, 8) HF_DECLARE_TABLE(5, 5)
HF_DECLARE_TABLE(5, 6) HF_DECLARE_TABLE(5, 7) HF_DECLARE_TABLE(5, 8) HF_DECLARE_TABLE(6, 6)
HF_DECLARE_TABLE(6, 7) HF_DECLARE_TABLE(6, 8) HF_DECLARE_TABLE(7, 7) HF_DECLARE_TABLE(7, 8)
HF_DECLARE_TABLE(8, 8)
const KernelEntry* hf_table_solo(int* count);

static std::vector<KernelEntry>& registry() {
  static std::vector<KernelEntry> all;
  static std::once_flag once;
  std::call_once(once, [] {
    const KernelEntry* (*tabs[])(int*) = {
        hf_table_0_0, hf_table_0_1, hf_table_0_2, hf_table_0_3, hf_table_0_4, hf_table_0_5, hf_table_0_6,
        hf_table_0_7, hf_table_0_8, hf_table_1_1, hf_table_1_2, hf_table_1_3, hf_table_1_4, hf_table_1_5,
        hf_table_1_6, hf_table_1_7, hf_table_1_8, hf_table_2_2, hf_table_2_3, hf_table_2_4, hf_table_2_5,
        hf_table_2_6, hf_table_2_7, hf_table_2_8, hf_table_3_3, hf_table_3_4, hf_table_3_5, hf_table_3_6,
        hf_table_3_7, hf_table_3_8, hf_table_4_4, hf_table_4_5, hf_table_4_6, hf_table_4_7, hf_table_4_8,
        hf_table_5_5, hf_table_5_6, hf_table_5_7, hf_table_5_8, hf_table_6_6, hf_table_6_7, hf_table_6_8,
        hf_table_7_7, hf_table_7_8, hf_table_8_8, hf_table_solo};
    for (auto f : tabs) {
      int n = 0;
      const KernelEntry* e = f(&n);
      all.insert(all.end(), e, e + n);
    }
  });
  return all;
}

const KernelEntry* find_kernel(int ka, int kb, int block, int cap) {
  for (const KernelEntry& e : registry())
    if (e.kind_a == ka && e.kind_b == kb && e.block == block && e.cap == cap) return &e;
  return nullptr;
}

bool cap_in_menu(int cap) {
  return cap == 0 || cap == 64 || cap == 80 || cap == 96 || cap == 128;
}

// ------------------------------------------------------------------ static scratch
// Scratch of hf_run_fused_noalloc: a fixed array in the code object, one copy
// per device, held until the process ends.  In host code `scratch` is only a
// stand-in for the symbol, never an address: the device address is looked up
// once per device (hipGetSymbolAddress, with that device current) when the
// device's state is set up, and host code uses that address only.
static __device__ __align__(256) uint8_t scratch[HF_NOALLOC_SCRATCH_BYTES];

// ------------------------------------------------------------------ device state
static std::mutex g_mu;
static std::vector<DeviceState*> g_devs;

DeviceState* device_state(int* status) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *status = record_hip(e);
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_devs.size() <= dev) g_devs.resize(dev + 1, nullptr);
  if (!g_devs[dev]) {
    DeviceState* s = new DeviceState();
    s->device = dev;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess) {
      delete s;
      *status = record_hip(e);
      return nullptr;
    }
    s->num_cus = prop.multiProcessorCount;
    hipEvent_t* evs[] = {&s->ev_start, &s->ev_stop};
    for (hipEvent_t* ev : evs)
      if ((e = hipEventCreate(ev)) != hipSuccess) {
        *status = record_hip(e);
        return nullptr;
      }
    if ((e = hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming)) != hipSuccess) {
      *status = record_hip(e);
      return nullptr;
    }
    if ((e = hipGetSymbolAddress(&s->static_scratch, HIP_SYMBOL(scratch))) != hipSuccess) {
      *status = record_hip(e);
      return nullptr;
    }
    g_devs[dev] = s;
  }
  *status = HF_OK;
  return g_devs[dev];
}

void shutdown_all() {
  mlp_free();
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (DeviceState* s : g_devs) {
    if (!s) continue;
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
    for (Slot& sl : s->slots)
      if (sl.ptr) (void)hipFree(sl.ptr);
    if (s->scrub) (void)hipFree(s->scrub);
    if (s->warm) (void)hipFree(s->warm);
    if (s->side) (void)hipStreamDestroy(s->side);
    (void)hipEventDestroy(s->ev_start);
    (void)hipEventDestroy(s->ev_stop);
    (void)hipEventDestroy(s->ev_fork);
    (void)hipEventDestroy(s->ev_join);
    delete s;
  }
  g_devs.clear();
  (void)hipSetDevice(cur);
}

// Zero-filled library scratch for slot `i` of at least `bytes` bytes.
int arena_slot(DeviceState* s, int i, size_t bytes, void** out) {
  if ((int)s->slots.size() <= i) s->slots.resize(i + 1);
  Slot& sl = s->slots[i];
  if (sl.bytes < bytes) {
    hipError_t e = hipDeviceSynchronize();  // the old region may still be in use
    if (e != hipSuccess) return record_hip(e);
    if (sl.ptr) (void)hipFree(sl.ptr);
    sl.ptr = nullptr;
    sl.bytes = 0;
    const size_t want = std::max<size_t>((bytes + (1u << 20) - 1) & ~size_t((1u << 20) - 1), 1u << 20);
    if ((e = hipMalloc(&sl.ptr, want)) != hipSuccess) {
      record_hip(e);
      return HF_ENOMEM;
    }
    if ((e = hipMemset(sl.ptr, 0, want)) != hipSuccess) return record_hip(e);
    if ((e = hipDeviceSynchronize()) != hipSuccess) return record_hip(e);
    sl.bytes = want;
  }
  *out = sl.ptr;
  return HF_OK;
}

// ------------------------------------------------------------------ validation
static constexpr int64_t kMaxElems = (int64_t(1) << 31) - 1;

static bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int validate_task(const hf_task* t) {
  if (!t) return HF_EINVAL;
  if (t->kind < 0 || t->kind >= HF_NUM_KINDS) return HF_EINVAL;
  if (t->n < 0 || t->c < 0 || t->h < 0 || t->w < 0) return HF_EINVAL;
  switch (t->kind) {
    case HF_BN_STATS: {
      if (!t->in || !t->out0 || !t->out1) return HF_EINVAL;
      if (t->n < 1 || t->c < 1 || t->h < 1 || t->w < 1) return HF_EINVAL;  // empty channel
      if (t->n > kMaxElems / t->c / t->h / t->w) return HF_EINVAL;
      if (!aligned(t->in, 4) || !aligned(t->out0, 4) || !aligned(t->out1, 4)) return HF_EINVAL;
      return HF_OK;
    }
    case HF_INT_MIX: {
      if (t->p[0] < 0 || t->n > kMaxElems) return HF_EINVAL;
      if (t->n > 0 && (!t->in || !t->out0)) return HF_EINVAL;
      if (!aligned(t->in, 4) || !aligned(t->out0, 4)) return HF_EINVAL;
      return HF_OK;
    }
    case HF_LDS_HIST: {
      if (t->p[0] != 256 || t->n > kMaxElems) return HF_EINVAL;
      if (!t->out0 || (t->n > 0 && !t->in)) return HF_EINVAL;
      if (!aligned(t->out0, 4)) return HF_EINVAL;
      return HF_OK;
    }
    case HF_IM2COL: {
      const int kh = t->p[0], kw = t->p[1], s = t->p[2], p = t->p[3];
      if (kh < 1 || kw < 1 || s < 1 || p < 0 || kh > 64 || kw > 64 || s > 64 || p > 64)
        return HF_EINVAL;
      if (t->c < 1 || t->h < 1 || t->w < 1) return HF_EINVAL;
      const int64_t Ho = (t->h + 2 * p - kh) / s + 1, Wo = (t->w + 2 * p - kw) / s + 1;
      if (t->h + 2 * p < kh || t->w + 2 * p < kw || Ho < 1 || Wo < 1) return HF_EINVAL;
      if (t->n > 0) {
        if (!t->in || !t->out0) return HF_EINVAL;
        if (t->n > kMaxElems / t->c / t->h / t->w) return HF_EINVAL;
        if (t->n > kMaxElems / (t->c * kh * kw) / (Ho * Wo)) return HF_EINVAL;
      }
      if (!aligned(t->in, 4) || !aligned(t->out0, 4)) return HF_EINVAL;
      return HF_OK;
    }
    case HF_UPSAMPLE: {
      const int s = t->p[0];
      if (s < 1 || s > 16) return HF_EINVAL;
      if (t->c < 1 || t->h < 1 || t->w < 1) return HF_EINVAL;
      if (t->n > 0) {
        if (!t->in || !t->out0) return HF_EINVAL;
        if (t->n > kMaxElems / t->c / (t->h * s) / (t->w * s)) return HF_EINVAL;
      }
      if (!aligned(t->in, 4) || !aligned(t->out0, 4)) return HF_EINVAL;
      return HF_OK;
    }
    case HF_MAXPOOL: {
      const int kh = t->p[0], kw = t->p[1], s = t->p[2], p = t->p[3];
      if (kh < 1 || kw < 1 || s < 1 || kh > 64 || kw > 64 || s > 64) return HF_EINVAL;
      if (p < 0 || p >= kh || p >= kw) return HF_EINVAL;  // every window holds an input element
      if (t->c < 1 || t->h < 1 || t->w < 1) return HF_EINVAL;
      if (t->h + 2 * p < kh || t->w + 2 * p < kw) return HF_EINVAL;
      const int64_t Ho = (t->h + 2 * p - kh) / s + 1, Wo = (t->w + 2 * p - kw) / s + 1;
      if (t->n > 0) {
        if (!t->in || !t->out0) return HF_EINVAL;
        if (t->n > kMaxElems / t->c / t->h / t->w) return HF_EINVAL;
        if (t->n > kMaxElems / t->c / Ho / Wo) return HF_EINVAL;
      }
      if (!aligned(t->in, 4) || !aligned(t->out0, 4) || !aligned(t->out1, 4)) return HF_EINVAL;
      return HF_OK;
    }
    case HF_SHA256D:
    case HF_BLAKE2B:
    case HF_ETHASH: {
      if (t->n > kMaxElems / 8) return HF_EINVAL;  // 8 digest words per instance
      if (t->n > 0) {
        if (!t->in || !t->out0) return HF_EINVAL;
        if (!aligned(t->in, 4) || !aligned(t->out0, 16)) return HF_EINVAL;
      }
      if (t->kind == HF_ETHASH) {
        if (t->h < 1 || t->h > (int64_t)UINT32_MAX) return HF_EINVAL;  // table rows
        if (t->n > 0 && (!t->in1 || !aligned(t->in1, 16))) return HF_EINVAL;
      }
      return HF_OK;
    }
  }
  return HF_EINVAL;
}

static uint32_t bn_units(const hf_task* t) {
  const int64_t M = t->n * t->h * t->w;
  return (uint32_t)((M + BnStats::kUnit - 1) / BnStats::kUnit);
}

int64_t scratch_bytes(const hf_task* t) {
  const int v = validate_task(t);
  if (v != HF_OK) return v;
  switch (t->kind) {
    case HF_BN_STATS: {
      const int64_t ctr = (t->c + 63) / 64 * 64;  // counters, padded to 256 B
      return 4 * (ctr + 2 * t->c * (int64_t)bn_units(t));
    }
    case HF_LDS_HIST:
      return 4 * (256 + 64);
    default:
      return 0;
  }
}

// ------------------------------------------------------------------ marshalling
int prepare(const hf_task* t, void* scratch, DevTask* dt) {
  std::memset(dt, 0, sizeof(*dt));
  switch (t->kind) {
    case HF_BN_STATS: {
      BnArgs& a = dt->bn;
      a.x = static_cast<const float*>(t->in);
      a.mean = static_cast<float*>(t->out0);
      a.var = static_cast<float*>(t->out1);
      const uint32_t ctrw = (uint32_t)((t->c + 63) / 64 * 64);
      a.ctr = static_cast<uint32_t*>(scratch);
      a.part = static_cast<uint32_t*>(scratch) + ctrw;
      a.C = (uint32_t)t->c;
      a.HW = (uint32_t)(t->h * t->w);
      a.M = (uint32_t)(t->n * t->h * t->w);
      a.CHWm = (a.C - 1u) * a.HW;
      a.upc = bn_units(t);
      a.total = a.C * a.upc;
      a.vec = (a.HW % 4u == 0u) && aligned(t->in, 16);
      a.div_hw = make_fastdiv(a.HW);
      a.div_upc = make_fastdiv(a.upc);
      return HF_OK;
    }
    case HF_INT_MIX: {
      MixArgs& a = dt->mix;
      a.in = static_cast<const uint32_t*>(t->in);
      a.out = static_cast<uint32_t*>(t->out0);
      a.n = (uint32_t)t->n;
      a.n4 = (aligned(t->in, 16) && aligned(t->out0, 16)) ? a.n / 4u : 0u;
      a.rounds = t->p[0];
      return HF_OK;
    }
    case HF_LDS_HIST: {
      HistArgs& a = dt->hist;
      a.in = static_cast<const uint8_t*>(t->in);
      a.out = static_cast<uint32_t*>(t->out0);
      a.acc = static_cast<uint32_t*>(scratch);
      a.ctr = static_cast<uint32_t*>(scratch) + 256;
      a.n = (uint32_t)t->n;
      const uint32_t mis = (uint32_t)(reinterpret_cast<uintptr_t>(t->in) % 16u);
      a.head = std::min<uint32_t>(a.n, (16u - mis) % 16u);
      a.n16 = (a.n - a.head) / 16u;
      a.tail_start = a.head + 16u * a.n16;
      return HF_OK;
    }
    case HF_IM2COL: {
      Im2colArgs& a = dt->im2col;
      const uint32_t kh = t->p[0], kw = t->p[1], s = t->p[2], p = t->p[3];
      a.x = static_cast<const float*>(t->in);
      a.out = static_cast<float*>(t->out0);
      a.C = (uint32_t)t->c;
      a.H = (uint32_t)t->h;
      a.W = (uint32_t)t->w;
      a.kw = kw;
      a.s = s;
      a.p = p;
      a.Ho = (a.H + 2 * p - kh) / s + 1;
      a.Wo = (a.W + 2 * p - kw) / s + 1;
      a.KK = kh * kw;
      a.units = (uint32_t)t->n * a.C * a.KK;
      a.vec = (a.Wo % 4u == 0u) && aligned(t->out0, 16);
      const uint32_t rowlen = a.vec ? a.Wo / 4u : a.Wo;
      a.lanes_per_unit = a.Ho * rowlen;
      a.div_kk = make_fastdiv(a.KK);
      a.div_row = make_fastdiv(rowlen);
      a.div_kw = make_fastdiv(kw);
      // the row path addresses one plane through a buffer resource of < 2^31 bytes
      a.row3 = kh == 3 && kw == 3 && s == 1 && p == 1 && a.W % 4u == 0u &&
               (uint64_t)a.H * a.W * 4u < (1ull << 31) && aligned(t->in, 16) && aligned(t->out0, 16);
      a.nch = (a.W + 63u) / 64u;
      a.nq = (uint32_t)(((uint64_t)a.H * a.nch + 3u) / 4u);
      a.row_units = (uint32_t)t->n * a.C * a.nq;
      a.div_nq = make_fastdiv(a.nq);
      a.div_nch = make_fastdiv(a.nch);
      return HF_OK;
    }
    case HF_UPSAMPLE: {
      UpArgs& a = dt->up;
      const uint32_t s = t->p[0];
      a.x = static_cast<const float*>(t->in);
      a.out = static_cast<float*>(t->out0);
      a.H = (uint32_t)t->h;
      a.W = (uint32_t)t->w;
      a.Ho = a.H * s;
      a.Wo = a.W * s;
      a.inv_s = 1.0f / (float)s;
      a.rows = (uint32_t)t->n * (uint32_t)t->c * a.Ho;
      a.vec = (a.Wo % 4u == 0u) && aligned(t->out0, 16);
      const uint32_t rowlen = a.vec ? a.Wo / 4u : a.Wo;
      a.rows_per_unit = rowlen >= 64u ? 1u : 64u / rowlen;
      a.units = (a.rows + a.rows_per_unit - 1u) / a.rows_per_unit;
      a.lanes_per_unit = a.rows_per_unit * rowlen;
      a.div_ho = make_fastdiv(a.Ho);
      a.div_row = make_fastdiv(rowlen);
      // the row path addresses one input and one output plane through buffer
      // resources of < 2^31 bytes
      a.row2 = s == 2u && a.W % 2u == 0u && (uint64_t)a.Ho * a.Wo * 4u < (1ull << 31) && aligned(t->in, 8) &&
               aligned(t->out0, 16);
      a.nch = (a.W + 31u) / 32u;
      a.nq = (uint32_t)(((uint64_t)a.Ho * a.nch + 3u) / 4u);
      a.row_units = (uint32_t)t->n * (uint32_t)t->c * a.nq;
      a.div_nq = make_fastdiv(a.nq);
      a.div_nch = make_fastdiv(a.nch);
      return HF_OK;
    }
    case HF_MAXPOOL: {
      PoolArgs& a = dt->pool;
      a.x = static_cast<const float*>(t->in);
      a.out = static_cast<float*>(t->out0);
      a.idx = static_cast<int32_t*>(t->out1);
      a.H = (uint32_t)t->h;
      a.W = (uint32_t)t->w;
      a.kh = (uint32_t)t->p[0];
      a.kw = (uint32_t)t->p[1];
      a.s = (uint32_t)t->p[2];
      a.p = (uint32_t)t->p[3];
      a.Ho = (a.H + 2 * a.p - a.kh) / a.s + 1;
      a.Wo = (a.W + 2 * a.p - a.kw) / a.s + 1;
      a.total = (uint32_t)t->n * (uint32_t)t->c * a.Ho * a.Wo;
      a.units = (a.total + Maxpool::kUnit - 1u) / Maxpool::kUnit;
      a.div_plane = make_fastdiv(a.Ho * a.Wo);
      a.div_wo = make_fastdiv(a.Wo);
      // the row path addresses one plane through buffer resources of < 2^31 bytes
      a.row3 = a.kh == 3u && a.kw == 3u && a.s == 2u && a.p == 1u && a.W % 8u == 0u &&
               (uint64_t)a.H * a.W * 4u < (1ull << 31) && aligned(t->in, 16) && aligned(t->out0, 16) &&
               aligned(t->out1, 16);
      a.nch = (a.W + 127u) / 128u;
      a.nq = (uint32_t)(((uint64_t)a.Ho * a.nch + 3u) / 4u);
      a.row_units = (uint32_t)t->n * (uint32_t)t->c * a.nq;
      a.div_nq = make_fastdiv(a.nq);
      a.div_nch = make_fastdiv(a.nch);
      return HF_OK;
    }
    case HF_SHA256D:
    case HF_BLAKE2B: {
      ShaArgs& a = dt->sha;
      a.hdr = static_cast<const uint32_t*>(t->in);
      a.out = static_cast<uint32_t*>(t->out0);
      a.nonce0 = (uint32_t)t->p[0];
      a.n = (uint32_t)t->n;
      return HF_OK;
    }
    case HF_ETHASH: {
      EthArgs& a = dt->eth;
      a.hdr = static_cast<const uint32_t*>(t->in);
      a.table = static_cast<const uint4*>(t->in1);
      a.out = static_cast<uint32_t*>(t->out0);
      a.nonce0 = (uint32_t)t->p[0];
      a.n = (uint32_t)t->n;
      a.rows = make_fastmod((uint32_t)t->h);
      return HF_OK;
    }
  }
  return HF_EINVAL;
}

// Workgroups that still find work when the task runs on `waves` wavefronts per
// workgroup (1 for an empty task).
int64_t useful_wgs(const hf_task* t, const DevTask& d, int waves) {
  auto cdiv = [](int64_t a, int64_t b) { return (a + b - 1) / b; };
  int64_t units = 1;
  switch (t->kind) {
    case HF_BN_STATS: units = cdiv(d.bn.total, waves); break;
    case HF_INT_MIX: units = cdiv(d.mix.n4 ? d.mix.n4 : d.mix.n, 64 * waves); break;
    case HF_LDS_HIST: units = cdiv(std::max<uint32_t>(d.hist.n16, 1), 64 * waves); break;
    case HF_IM2COL: units = cdiv(d.im2col.row3 ? d.im2col.row_units : d.im2col.units, waves); break;
    case HF_UPSAMPLE: units = cdiv(d.up.row2 ? d.up.row_units : d.up.units, waves); break;
    case HF_MAXPOOL: units = cdiv(d.pool.row3 ? d.pool.row_units : d.pool.units, waves); break;
    case HF_SHA256D:
    case HF_BLAKE2B: units = cdiv(d.sha.n, 64 * waves); break;
    case HF_ETHASH: units = cdiv(d.eth.n, EthashLike::kPerIter * waves); break;
  }
  return std::max<int64_t>(units, 1);
}

int occupancy_grid(DeviceState* s, const void* fn, int block, int* wg_per_cu) {
  int occ = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, block, 0);
  if (e != hipSuccess) return record_hip(e);
  if (occ < 1) occ = 1;
  if (wg_per_cu) *wg_per_cu = occ;
  return occ * s->num_cus;
}

// Scratch of a task: caller-provided or arena slot `slot`.
int task_scratch(DeviceState* s, const hf_task* t, int slot, void** out) {
  const int64_t need = scratch_bytes(t);
  if (need < 0) return (int)need;
  *out = nullptr;
  if (need == 0) return HF_OK;
  if (t->scratch) {
    if (!aligned(t->scratch, 16)) return HF_EINVAL;
    *out = t->scratch;
    return HF_OK;
  }
  return arena_slot(s, slot, (size_t)need, out);
}

// ------------------------------------------------------------------ timing
int wait_event(hipEvent_t ev) {
  const char* env = std::getenv("HF_TIMEOUT_MS");
  const long limit = env ? std::atol(env) : 0;
  if (limit <= 0) {
    hipError_t e = hipEventSynchronize(ev);
    return e == hipSuccess ? HF_OK : record_hip(e);
  }
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    hipError_t e = hipEventQuery(ev);
    if (e == hipSuccess) return HF_OK;
    if (e != hipErrorNotReady) return record_hip(e);
    const auto dt = std::chrono::steady_clock::now() - t0;
    if (std::chrono::duration_cast<std::chrono::milliseconds>(dt).count() > limit) return HF_ETIMEOUT;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

int timed_begin(DeviceState* s, hipStream_t st, float* ms) {
  if (!ms) return HF_OK;
  hipError_t e = hipEventRecord(s->ev_start, st);
  return e == hipSuccess ? HF_OK : record_hip(e);
}

int timed_end(DeviceState* s, hipStream_t st, float* ms) {
  if (!ms) return HF_OK;
  hipError_t e = hipEventRecord(s->ev_stop, st);
  if (e != hipSuccess) return record_hip(e);
  int rc = wait_event(s->ev_stop);
  if (rc != HF_OK) return rc;
  if ((e = hipEventElapsedTime(ms, s->ev_start, s->ev_stop)) != hipSuccess) return record_hip(e);
  return HF_OK;
}

// ------------------------------------------------------------------ launches
int launch_solo(DeviceState* s, const hf_task* t, int block, int grid, int slot, hipStream_t st) {
  const KernelEntry* k = find_kernel(t->kind, -1, block, 0);
  if (!k) return HF_EUNSUPPORTED;
  void* scr = nullptr;
  int rc = task_scratch(s, t, slot, &scr);
  if (rc != HF_OK) return rc;
  DevTask d;
  if ((rc = prepare(t, scr, &d)) != HF_OK) return rc;
  if (grid <= 0) {
    const int g = occupancy_grid(s, k->fn, block, nullptr);
    if (g < 0) return g;
    grid = (int)std::min<int64_t>(g, useful_wgs(t, d, block / 64));
  }
  void* args[] = {&d};
  hipError_t e = hipLaunchKernel(k->fn, dim3(grid), dim3(block), args, 0, st);
  return e == hipSuccess ? HF_OK : record_hip(e);
}

int check_block(int block) { return (block == 256 || block == 512 || block == 1024) ? HF_OK : HF_EINVAL; }

int validate_fused(const hf_pair* pr, const hf_config* cfg) {
  if (!pr || !cfg) return HF_EINVAL;
  int rc;
  if ((rc = validate_task(&pr->a)) != HF_OK || (rc = validate_task(&pr->b)) != HF_OK) return rc;
  if (check_block(cfg->block) != HF_OK) return HF_EINVAL;
  const int W = cfg->block / 64;
  if (cfg->split_waves < 1 || cfg->split_waves >= W) return HF_EINVAL;
  if (!cap_in_menu(cfg->vgpr_cap)) return HF_EINVAL;
  if (cfg->grid < 0) return HF_EINVAL;
  if (pr->a.scratch && pr->a.scratch == pr->b.scratch && scratch_bytes(&pr->a) > 0 &&
      scratch_bytes(&pr->b) > 0)
    return HF_EINVAL;  // the two tasks would race on one region
  return HF_OK;
}

int launch_fused(DeviceState* s, const hf_pair* pr, const hf_config* cfg, hipStream_t st,
                 int* grid_used) {
  int rc = validate_fused(pr, cfg);
  if (rc != HF_OK) return rc;
  // instantiations exist for kind_a <= kind_b; the mirrored pair swaps the intervals
  const hf_task* ta = &pr->a;
  const hf_task* tb = &pr->b;
  int w1 = cfg->split_waves;
  const int W = cfg->block / 64;
  if (ta->kind > tb->kind) {
    std::swap(ta, tb);
    w1 = W - w1;
  }
  const KernelEntry* k = find_kernel(ta->kind, tb->kind, cfg->block, cfg->vgpr_cap);
  if (!k) return HF_EUNSUPPORTED;
  void *sa = nullptr, *sb = nullptr;
  if ((rc = task_scratch(s, ta, 0, &sa)) != HF_OK) return rc;
  if ((rc = task_scratch(s, tb, 1, &sb)) != HF_OK) return rc;
  DevTask da, db;
  if ((rc = prepare(ta, sa, &da)) != HF_OK || (rc = prepare(tb, sb, &db)) != HF_OK) return rc;
  int grid = cfg->grid;
  if (grid <= 0) {
    const int g = occupancy_grid(s, k->fn, cfg->block, nullptr);
    if (g < 0) return g;
    const int64_t need = std::max(useful_wgs(ta, da, w1), useful_wgs(tb, db, W - w1));
    grid = (int)std::min<int64_t>(g, need);
  }
  if (grid_used) *grid_used = grid;
  uint32_t uw1 = (uint32_t)w1;
  void* args[] = {&da, &db, &uw1};
  hipError_t e = hipLaunchKernel(k->fn, dim3(grid), dim3(cfg->block), args, 0, st);
  return e == hipSuccess ? HF_OK : record_hip(e);
}

int launch_unfused(DeviceState* s, const hf_pair* pr, int block_a, int block_b, int mode,
                   hipStream_t s0, hipStream_t s1) {
  int rc;
  if (mode == HF_SERIAL) {
    if ((rc = launch_solo(s, &pr->a, block_a, 0, 0, s0)) != HF_OK) return rc;
    return launch_solo(s, &pr->b, block_b, 0, 1, s0);
  }
  if (!s1) {
    if (!s->side) {
      hipError_t e = hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking);
      if (e != hipSuccess) return record_hip(e);
    }
    s1 = s->side;
  }
  hipError_t e;
  if ((e = hipEventRecord(s->ev_fork, s0)) != hipSuccess) return record_hip(e);
  if ((e = hipStreamWaitEvent(s1, s->ev_fork, 0)) != hipSuccess) return record_hip(e);
  if ((rc = launch_solo(s, &pr->a, block_a, 0, 0, s0)) != HF_OK) return rc;
  if ((rc = launch_solo(s, &pr->b, block_b, 0, 1, s1)) != HF_OK) return rc;
  if ((e = hipEventRecord(s->ev_join, s1)) != hipSuccess) return record_hip(e);
  if ((e = hipStreamWaitEvent(s0, s->ev_join, 0)) != hipSuccess) return record_hip(e);
  return HF_OK;
}

int kernel_info(DeviceState* s, const void* fn, int block, hf_kernel_info* out) {
  hipFuncAttributes attr;
  hipError_t e = hipFuncGetAttributes(&attr, fn);
  if (e != hipSuccess) return record_hip(e);
  int wg = 0;
  const int g = occupancy_grid(s, fn, block, &wg);
  if (g < 0) return g;
  std::memset(out, 0, sizeof(*out));
  out->vgprs = attr.numRegs;
  out->sgprs = 0;
  out->lds_bytes = (int)attr.sharedSizeBytes;
  out->spill_bytes = (int)attr.localSizeBytes;
  out->wg_per_cu = wg;
  out->waves_per_simd = wg * (block / 64) / 4;
  out->num_cus = s->num_cus;
  out->default_grid = g;
  return HF_OK;
}

// ------------------------------------------------------------------ microbenchmarks
// Copies n float4.  Launched with one element per lane: a lane that loops over
// several elements waits, at each load, for its previous store as well (the
// vector-memory counter retires in order), which costs about a fifth of the
// copy rate; a lane that exits after its store does not wait for it.
__global__ void __launch_bounds__(256) k_copy(float4* __restrict__ dst, const float4* __restrict__ src,
                                              uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Reads n float4 and writes one word per workgroup (a read-bandwidth ceiling).
__global__ void __launch_bounds__(256) k_read(const float4* __restrict__ src, uint64_t n, float* __restrict__ sink) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  float acc = 0.f;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float4 v = src[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  if (acc == 1234.5f) sink[blockIdx.x] = acc;  // keeps the loads alive
}

__global__ void __launch_bounds__(256) k_fill(float4* __restrict__ dst, uint64_t n, float v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = make_float4(v, v, v, v);
}

// The library's 64 KiB `warm` buffer: words [0, kSinkWords) are the sinks the
// measurement kernels write (one per workgroup, practically never), the last
// word is the barrier self-test's error counter.
constexpr int kSinkWords = (1 << 14) - 1;

// Interval-barrier self-test: both intervals of each workgroup run a ring
// exchange through LDS.  In round r every wavefront sleeps a pseudo-random
// 0..7 short intervals (so the wavefronts arrive skewed), writes a tag for
// (r, its index) into its slot, syncs, reads its neighbour's slot, checks the
// neighbour's tag, and syncs again before the next round's write.  The two
// intervals run different round counts, so one finishes while the other still
// synchronises.  Every wavefront of an interval calls sync() equally often.
__device__ __forceinline__ uint32_t selftest_mix(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}

template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_barrier_selftest(uint32_t w1, uint32_t iters1, uint32_t iters2,
                                                            uint32_t seed, uint32_t* errors) {
  constexpr uint32_t W = BLOCK / 64;
  __shared__ uint32_t ctr[2];
  __shared__ uint32_t slots[W];
  if (threadIdx.x == 0) {
    ctr[0] = 0u;
    ctr[1] = 0u;
  }
  __syncthreads();
  const uint32_t wave = uniform(threadIdx.x >> 6);
  const bool first = wave < w1;
  const uint32_t nw = first ? w1 : W - w1;
  const uint32_t k = first ? wave : wave - w1;
  uint32_t* slot = first ? slots : slots + w1;
  PartBarrier bar(first ? &ctr[0] : &ctr[1], nw);
  const uint32_t iters = first ? iters1 : iters2;
  const uint32_t nb = (k + 1u) % nw;
  uint32_t bad = 0;
  for (uint32_t r = 0; r < iters; ++r) {
    const uint32_t skew = selftest_mix(seed ^ (blockIdx.x * 0x9E3779B1u) ^ (wave << 24) ^ r) & 7u;
    for (uint32_t n = 0; n < skew; ++n) __builtin_amdgcn_s_sleep(1);
    if (lane_id() == 0) slot[k] = selftest_mix(r * 0x01000193u ^ (k << 20) ^ blockIdx.x);
    bar.sync();
    if (slot[nb] != selftest_mix(r * 0x01000193u ^ (nb << 20) ^ blockIdx.x)) ++bad;
    bar.sync();
  }
  if (bad) __hip_atomic_fetch_add(errors, bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Zeroes n words (the static scratch before an allocation-free launch; a
// kernel rather than a memset, so that a captured graph holds no memset node).
__global__ void __launch_bounds__(256) k_zero_words(uint32_t* __restrict__ p, uint32_t n) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

// The integer-issue ceiling: the int_mix round on four independent chains per
// lane, as the int_mix body runs it, from registers only (no memory traffic
// in the loop), so its rate is what the VALU sustains for this instruction mix.
__global__ void __launch_bounds__(256) k_int_peak(uint32_t* sink, uint32_t rounds) {
  // every chain starts from a per-lane value, so all four stay vector
  // registers (a wave-uniform start would let the compiler run a chain on the
  // scalar unit)
  uint32_t a = threadIdx.x, b = threadIdx.x * 977u + blockIdx.x, c = threadIdx.x ^ 0x5555u,
           d = (threadIdx.x << 8) ^ blockIdx.x;
  for (uint32_t r = 0; r < rounds; ++r) {
    a = IntMix::round1(a, r);
    b = IntMix::round1(b, r);
    c = IntMix::round1(c, r);
    d = IntMix::round1(d, r);
  }
  if ((a ^ b ^ c ^ d) == 0x12345678u) sink[blockIdx.x % kSinkWords] = a;  // keeps the loop alive
}

__global__ void __launch_bounds__(256) k_spin(uint32_t* sink, uint32_t iters) {
  uint32_t x = threadIdx.x ^ (blockIdx.x << 10);
  for (uint32_t i = 0; i < iters; ++i) x = IntMix::round1(x, i);
  if (x == 0x12345678u) sink[0] = x;  // keeps the loop alive
}

}  // namespace hf

using namespace hf;

// =================================================================== C ABI
extern "C" {

int hf_init(void) {
  int st;
  return device_state(&st) ? HF_OK : st;
}

int hf_shutdown(void) {
  shutdown_all();
  return HF_OK;
}

const char* hf_strerror(int status) {
  switch (status) {
    case HF_OK: return "ok";
    case HF_EINVAL: return "invalid argument";
    case HF_EUNSUPPORTED: return "no compiled kernel for this pair, block and cap";
    case HF_EHIP: return "HIP runtime error";
    case HF_ETIMEOUT: return "timed out waiting for the GPU";
    case HF_ENOMEM: return "device allocation failed";
    case HF_ENOMODEL: return "no learned cost model trained or loaded";
    case HF_ESCRATCH: return "the tasks need more scratch than the allocation-free entry point's static buffer holds";
  }
  return "unknown status";
}

int hf_last_hip_error(void) { return g_last_hip; }

const char* hf_version(void) { return "hfuse-gfx950 0.1"; }

int hf_validate_task(const hf_task* t) { return validate_task(t); }

int64_t hf_scratch_bytes(const hf_task* t) { return scratch_bytes(t); }

int hf_validate_fused(const hf_pair* pr, const hf_config* cfg) {
  int rc = validate_fused(pr, cfg);
  if (rc != HF_OK) return rc;
  const int ka = std::min(pr->a.kind, pr->b.kind), kb = std::max(pr->a.kind, pr->b.kind);
  return find_kernel(ka, kb, cfg->block, cfg->vgpr_cap) ? HF_OK : HF_EUNSUPPORTED;
}

int hf_run_solo(const hf_task* t, int block, int grid, void* stream, float* ms_out) {
  int rc = validate_task(t);
  if (rc != HF_OK) return rc;
  if (check_block(block) != HF_OK || grid < 0) return HF_EINVAL;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = timed_begin(s, st, ms_out)) != HF_OK) return rc;
  if ((rc = launch_solo(s, t, block, grid, 0, st)) != HF_OK) return rc;
  return timed_end(s, st, ms_out);
}

int hf_run_unfused(const hf_pair* pr, int block_a, int block_b, int mode, void* stream0,
                   void* stream1, float* ms_out) {
  if (!pr) return HF_EINVAL;
  int rc;
  if ((rc = validate_task(&pr->a)) != HF_OK || (rc = validate_task(&pr->b)) != HF_OK) return rc;
  if (check_block(block_a) != HF_OK || check_block(block_b) != HF_OK) return HF_EINVAL;
  if (mode != HF_SERIAL && mode != HF_STREAMS) return HF_EINVAL;
  if (pr->a.scratch && pr->a.scratch == pr->b.scratch && scratch_bytes(&pr->a) > 0 &&
      scratch_bytes(&pr->b) > 0)
    return HF_EINVAL;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  hipStream_t s0 = static_cast<hipStream_t>(stream0), s1 = static_cast<hipStream_t>(stream1);
  if ((rc = timed_begin(s, s0, ms_out)) != HF_OK) return rc;
  if ((rc = launch_unfused(s, pr, block_a, block_b, mode, s0, s1)) != HF_OK) return rc;
  return timed_end(s, s0, ms_out);
}

int hf_run_fused_cfg(const hf_pair* pr, const hf_config* cfg, void* stream, float* ms_out) {
  int rc = hf_validate_fused(pr, cfg);
  if (rc != HF_OK) return rc;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = timed_begin(s, st, ms_out)) != HF_OK) return rc;
  if ((rc = launch_fused(s, pr, cfg, st, nullptr)) != HF_OK) return rc;
  return timed_end(s, st, ms_out);
}

int hf_run_fused_noalloc(const hf_pair* pr, const hf_config* cfg, void* stream) {
  int rc = hf_validate_fused(pr, cfg);
  if (rc != HF_OK) return rc;
  // host only: where each task without caller scratch gets its region
  hf_pair p = *pr;
  hf_task* ts[2] = {&p.a, &p.b};
  size_t off[2] = {0, 0}, total = 0;
  bool mine[2] = {false, false};
  for (int i = 0; i < 2; ++i) {
    const int64_t need = scratch_bytes(ts[i]);
    if (need > 0 && !ts[i]->scratch) {
      mine[i] = true;
      off[i] = total;
      total += ((size_t)need + 255) & ~size_t(255);
    }
  }
  if (total > (size_t)HF_NOALLOC_SCRATCH_BYTES) return HF_ESCRATCH;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (total > 0) {
    uint8_t* base = static_cast<uint8_t*>(s->static_scratch);
    for (int i = 0; i < 2; ++i)
      if (mine[i]) ts[i]->scratch = base + off[i];
    // the regions must start zero-filled; the array keeps whatever the last
    // call on this device left in it
    const uint32_t words = (uint32_t)(total / 4);
    const int grid = (int)std::min<uint32_t>((words + 255u) / 256u, 1024u);
    hipLaunchKernelGGL(k_zero_words, dim3(grid), dim3(256), 0, st, reinterpret_cast<uint32_t*>(base), words);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return record_hip(e);
  }
  return launch_fused(s, &p, cfg, st, nullptr);
}

int hf_run_fused(const hf_pair* pr, int split_num, int split_den, int block, int vgpr_cap,
                 void* stream, float* ms_out) {
  if (split_den <= 0 || split_num <= 0 || split_num >= split_den) return HF_EINVAL;
  if (check_block(block) != HF_OK) return HF_EINVAL;
  const int64_t d1 = (int64_t)block * split_num;
  if (d1 % split_den != 0 || (d1 / split_den) % 64 != 0) return HF_EINVAL;
  hf_config cfg{(int32_t)(d1 / split_den / 64), block, vgpr_cap, 0};
  return hf_run_fused_cfg(pr, &cfg, stream, ms_out);
}

int hf_run_vfused(const hf_pair* pr, int block, int grid, void* stream, float* ms_out) {
  if (!pr) return HF_EINVAL;
  int rc;
  if ((rc = validate_task(&pr->a)) != HF_OK || (rc = validate_task(&pr->b)) != HF_OK) return rc;
  if (check_block(block) != HF_OK || grid < 0) return HF_EINVAL;
  if (pr->a.scratch && pr->a.scratch == pr->b.scratch && scratch_bytes(&pr->a) > 0 &&
      scratch_bytes(&pr->b) > 0)
    return HF_EINVAL;
  const hf_task* ta = &pr->a;
  const hf_task* tb = &pr->b;
  if (ta->kind > tb->kind) std::swap(ta, tb);  // same work, canonical instantiation
  const KernelEntry* k = find_kernel(ta->kind, tb->kind, block, -1);
  if (!k) return HF_EUNSUPPORTED;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  void *sa = nullptr, *sb = nullptr;
  if ((rc = task_scratch(s, ta, 0, &sa)) != HF_OK || (rc = task_scratch(s, tb, 1, &sb)) != HF_OK) return rc;
  DevTask da, db;
  if ((rc = prepare(ta, sa, &da)) != HF_OK || (rc = prepare(tb, sb, &db)) != HF_OK) return rc;
  if (grid <= 0) {
    const int g = occupancy_grid(s, k->fn, block, nullptr);
    if (g < 0) return g;
    const int64_t need = std::max(useful_wgs(ta, da, block / 64), useful_wgs(tb, db, block / 64));
    grid = (int)std::min<int64_t>(g, need);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = timed_begin(s, st, ms_out)) != HF_OK) return rc;
  void* args[] = {&da, &db};
  hipError_t e = hipLaunchKernel(k->fn, dim3(grid), dim3(block), args, 0, st);
  if (e != hipSuccess) return record_hip(e);
  return timed_end(s, st, ms_out);
}

int hf_fused_info(int kind_a, int kind_b, int block, int vgpr_cap, hf_kernel_info* out) {
  if (!out || kind_a < 0 || kind_a >= HF_NUM_KINDS || kind_b < 0 || kind_b >= HF_NUM_KINDS)
    return HF_EINVAL;
  if (check_block(block) != HF_OK || !cap_in_menu(vgpr_cap)) return HF_EINVAL;
  const KernelEntry* k = find_kernel(std::min(kind_a, kind_b), std::max(kind_a, kind_b), block, vgpr_cap);
  if (!k) return HF_EUNSUPPORTED;
  int rc;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  return kernel_info(s, k->fn, block, out);
}

int hf_solo_info(int kind, int block, hf_kernel_info* out) {
  if (!out || kind < 0 || kind >= HF_NUM_KINDS || check_block(block) != HF_OK) return HF_EINVAL;
  const KernelEntry* k = find_kernel(kind, -1, block, 0);
  if (!k) return HF_EUNSUPPORTED;
  int rc;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  return kernel_info(s, k->fn, block, out);
}

int hf_copy(void* dst, const void* src, int64_t bytes, void* stream, float* ms_out) {
  if (!dst || !src || bytes < 0 || bytes % 16 != 0 || !aligned(dst, 16) || !aligned(src, 16))
    return HF_EINVAL;
  int rc;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = timed_begin(s, st, ms_out)) != HF_OK) return rc;
  const uint64_t n = (uint64_t)bytes / 16;
  const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, uint64_t(1) << 30));
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, st, static_cast<float4*>(dst),
                     static_cast<const float4*>(src), n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return record_hip(e);
  return timed_end(s, st, ms_out);
}

int hf_read(const void* src, int64_t bytes, void* stream, float* ms_out) {
  if (!src || bytes < 0 || bytes % 16 != 0 || !aligned(src, 16)) return HF_EINVAL;
  int rc;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  if (!s->warm) {
    hipError_t e = hipMalloc(&s->warm, 1 << 16);
    if (e != hipSuccess) {
      record_hip(e);
      return HF_ENOMEM;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = timed_begin(s, st, ms_out)) != HF_OK) return rc;
  const uint64_t n = (uint64_t)bytes / 16;
  const int grid = std::max(1, std::min<int>((int)((n + 255) / 256), std::min(s->num_cus * 8, kSinkWords)));
  hipLaunchKernelGGL(k_read, dim3(grid), dim3(256), 0, st, static_cast<const float4*>(src), n,
                     static_cast<float*>(s->warm));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return record_hip(e);
  return timed_end(s, st, ms_out);
}

int hf_scrub(void* stream) {
  int rc;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  const size_t bytes = size_t(1) << 30;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!s->warm) {
    hipError_t e = hipMalloc(&s->warm, 1 << 16);
    if (e != hipSuccess) {
      record_hip(e);
      return HF_ENOMEM;
    }
  }
  if (!s->scrub) {
    hipError_t e = hipMalloc(&s->scrub, bytes);
    if (e != hipSuccess) {
      record_hip(e);
      return HF_ENOMEM;
    }
    // written once; every scrub afterwards only reads it, so the lines it
    // leaves in the caches are clean and the next kernel pays no write-back
    hipLaunchKernelGGL(k_fill, dim3(s->num_cus * 8), dim3(256), 0, st, static_cast<float4*>(s->scrub),
                       (uint64_t)(bytes / 16), 1.0f);
  }
  // one word per workgroup of sink: num_cus * 8 <= 16384 words of `warm`
  hipLaunchKernelGGL(k_read, dim3(std::min(s->num_cus * 8, kSinkWords)), dim3(256), 0, st,
                     static_cast<const float4*>(s->scrub), (uint64_t)(bytes / 16), static_cast<float*>(s->warm));
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? HF_OK : record_hip(e);
}

int hf_selftest_barrier(int block, int split_waves, int iters_a, int iters_b, uint32_t seed, int grid,
                        void* stream, uint32_t* mismatches) {
  if (!mismatches || check_block(block) != HF_OK) return HF_EINVAL;
  if (split_waves < 1 || split_waves >= block / 64) return HF_EINVAL;
  if (iters_a < 0 || iters_b < 0 || iters_a > (1 << 20) || iters_b > (1 << 20)) return HF_EINVAL;
  if (grid < 0 || grid > 65536) return HF_EINVAL;
  int rc;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  if (!s->warm) {
    hipError_t e = hipMalloc(&s->warm, 1 << 16);
    if (e != hipSuccess) {
      record_hip(e);
      return HF_ENOMEM;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the error counter: the word after the sinks of the 64 KiB buffer
  uint32_t* errors = static_cast<uint32_t*>(s->warm) + kSinkWords;
  hipError_t e = hipMemsetAsync(errors, 0, 4, st);
  if (e != hipSuccess) return record_hip(e);
  const void* fn = block == 256   ? reinterpret_cast<const void*>(&k_barrier_selftest<256>)
                   : block == 512 ? reinterpret_cast<const void*>(&k_barrier_selftest<512>)
                                  : reinterpret_cast<const void*>(&k_barrier_selftest<1024>);
  if (grid == 0) {
    if ((rc = occupancy_grid(s, fn, block, nullptr)) < 0) return rc;
    grid = rc;
  }
  uint32_t w1 = (uint32_t)split_waves, ia = (uint32_t)iters_a, ib = (uint32_t)iters_b;
  void* args[] = {&w1, &ia, &ib, &seed, &errors};
  if ((e = hipLaunchKernel(fn, dim3(grid), dim3(block), args, 0, st)) != hipSuccess) return record_hip(e);
  if ((e = hipMemcpyAsync(mismatches, errors, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return record_hip(e);
  if ((e = hipEventRecord(s->ev_stop, st)) != hipSuccess) return record_hip(e);
  return wait_event(s->ev_stop);
}

int hf_int_peak(int rounds, int grid, void* stream, float* ms_out, double* lane_ops_out) {
  if (rounds < 1 || grid < 0 || grid > (1 << 20)) return HF_EINVAL;
  int rc;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  if (!s->warm) {
    hipError_t e = hipMalloc(&s->warm, 1 << 16);
    if (e != hipSuccess) {
      record_hip(e);
      return HF_ENOMEM;
    }
  }
  if (grid == 0) grid = s->num_cus * 8;  // 2048 lanes per CU: eight wavefronts per SIMD
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = timed_begin(s, st, ms_out)) != HF_OK) return rc;
  hipLaunchKernelGGL(k_int_peak, dim3(grid), dim3(256), 0, st, static_cast<uint32_t*>(s->warm), (uint32_t)rounds);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return record_hip(e);
  if (lane_ops_out) *lane_ops_out = 8.0 * 4.0 * 256.0 * (double)grid * (double)rounds;
  return timed_end(s, st, ms_out);
}

int hf_warmup(int ms, void* stream) {
  if (ms < 0) return HF_EINVAL;
  int rc;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  if (!s->warm) {
    hipError_t e = hipMalloc(&s->warm, 1 << 16);
    if (e != hipSuccess) {
      record_hip(e);
      return HF_ENOMEM;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    hipLaunchKernelGGL(k_spin, dim3(s->num_cus * 8), dim3(256), 0, st, static_cast<uint32_t*>(s->warm),
                       (uint32_t)20000);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return record_hip(e);
    const auto dt = std::chrono::steady_clock::now() - t0;
    if (std::chrono::duration_cast<std::chrono::milliseconds>(dt).count() >= ms) break;
  }
  return HF_OK;
}

}  // extern "C"
