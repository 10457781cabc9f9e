// hf_batch.hip -- many small kernel instances fused into one persistent launch.
//
// The paper fuses two kernels per launch; with many small, uneven instances the
// launch overhead itself dominates (Sec. I, footnote on tiny kernels).  Here the
// instances are cut into groups of two to four, and each group is executed as
// an N-way horizontally fused "virtual launch": a workgroup's wavefronts are
// split into one interval per member (the Generate algorithm with N bodies),
// each member runs its own body on its own interval, with its own interval
// barrier.  One persistent kernel executes every group: each resident
// workgroup repeatedly pulls the next (group, virtual workgroup) item from a
// device queue, so the items of one group run concurrently on many CUs and the
// whole batch costs one launch, which can be captured in a HIP graph.
//
// Item boundaries are the only whole-workgroup barriers; every cross-workgroup
// counter (queue, bn_stats units, histogram arrivals) is left at zero when the
// launch ends, so the captured graph can be replayed without a memset.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hf_runtime.hpp"

namespace hf {

constexpr int kMaxMembers = 4;

struct BatchTables {
  const DevTask* tasks;        // [ntask]
  const int32_t* kinds;        // [ntask]
  const int32_t* wave0;        // [ntask] first wavefront of the task's interval
  const int32_t* wave1;        // [ntask] one past its last wavefront
  const int32_t* lds_slot;     // [ntask] histogram LDS slot of the task (-1: none)
  const int32_t* grp_first;    // [ngroup + 1] first task of each group
  const uint32_t* item_start;  // [ngroup + 1] first item of each group
  const uint32_t* grp_nwg;     // [ngroup] virtual workgroups of each group
  uint32_t* queue;             // [1] pull counter, zero between launches
  uint32_t ngroup;
  uint32_t total_items;
};

// HASH: the variant that also runs the hash kinds.  The hash bodies need more
// registers than the others, so batches without them use the variant that
// leaves them out and keeps five waves per SIMD without spilling.
template <bool HASH, class Bar>
__device__ __forceinline__ void run_body(int kind, const DevTask& t, const Part& p, Bar& bar, uint32_t* lds) {
  switch (kind) {
    case HF_BN_STATS: BnStats::run(t, p, bar, lds); break;
    case HF_INT_MIX: IntMix::run(t, p, bar, lds); break;
    case HF_IM2COL: Im2col::run(t, p, bar, lds); break;
    case HF_LDS_HIST: LdsHist::run(t, p, bar, lds); break;
    case HF_UPSAMPLE: Upsample::run(t, p, bar, lds); break;
    case HF_MAXPOOL: Maxpool::run(t, p, bar, lds); break;
    default:
      if constexpr (HASH) {
        switch (kind) {
          case HF_SHA256D: Sha256d::run(t, p, bar, lds); break;
          case HF_BLAKE2B: Blake2b::run(t, p, bar, lds); break;
          case HF_ETHASH: EthashLike::run(t, p, bar, lds); break;
          default: break;
        }
      }
      break;
  }
}

constexpr bool is_hash_kind(int kind) { return kind == HF_SHA256D || kind == HF_BLAKE2B || kind == HF_ETHASH; }

// LDS: kMaxMembers interval-barrier counters, then (dynamic) one histogram
// region per histogram member of the largest group's histogram count.
extern __shared__ uint32_t hf_batch_hist_lds[];

template <int BLOCK, bool HASH, int WPE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) k_batch(BatchTables T) {
  __shared__ uint32_t smem[kMaxMembers];
  __shared__ uint32_t item_sh[2];
  const uint32_t wave = uniform(threadIdx.x >> 6);
  if (threadIdx.x == 0)
    item_sh[0] = __hip_atomic_fetch_add(T.queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (uint32_t it = 0;; it ^= 1u) {
    if (threadIdx.x == 0)
      for (int m = 0; m < kMaxMembers; ++m) smem[m] = 0u;
    __syncthreads();
    const uint32_t item = uniform(item_sh[it]);
    if (item >= T.total_items) {
      // the last pull of the launch resets the queue for the next launch
      if (threadIdx.x == 0 && item == T.total_items + gridDim.x - 1u)
        __hip_atomic_store(T.queue, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    // the next item is pulled now; its latency hides behind this item's work
    if (threadIdx.x == 0)
      item_sh[it ^ 1u] = __hip_atomic_fetch_add(T.queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // group of the item: last g with item_start[g] <= item
    uint32_t lo = 0, hi = T.ngroup;
    while (hi - lo > 1u) {
      const uint32_t mid = (lo + hi) >> 1;
      if (T.item_start[mid] <= item) lo = mid;
      else hi = mid;
    }
    const uint32_t g = lo;
    const uint32_t b = item - T.item_start[g];
    const int32_t t0 = T.grp_first[g], t1 = T.grp_first[g + 1];
    int32_t mine = -1;
    for (int32_t m = t0; m < t1; ++m)
      if (wave >= (uint32_t)T.wave0[m] && wave < (uint32_t)T.wave1[m]) mine = m;
    mine = (int32_t)uniform((uint32_t)mine);
    if (mine >= 0) {
      const uint32_t w0 = uniform((uint32_t)T.wave0[mine]), w1 = uniform((uint32_t)T.wave1[mine]);
      const uint32_t nw = w1 - w0;
      const Part p{threadIdx.x - 64u * w0, 64u * nw, wave - w0, nw, b, uniform(T.grp_nwg[g])};
      PartBarrier bar(&smem[mine - t0], nw);
      // the task's arguments are wave-uniform: keep them in scalar registers
      DevTask dt;
      const uint32_t* src = reinterpret_cast<const uint32_t*>(&T.tasks[mine]);
      uint32_t* dst = reinterpret_cast<uint32_t*>(&dt);
#pragma unroll
      for (int i = 0; i < (int)(sizeof(DevTask) / 4); ++i) dst[i] = uniform(src[i]);
      const int32_t slot = (int32_t)uniform((uint32_t)T.lds_slot[mine]);
      uint32_t* lds = slot >= 0 ? hf_batch_hist_lds + (uint32_t)slot * LdsHist::lds_words(BLOCK) : nullptr;
      run_body<HASH>((int)uniform((uint32_t)T.kinds[mine]), dt, p, bar, lds);
    }
    __syncthreads();  // item boundary: every interval has finished
  }
}

// ------------------------------------------------------------------ worker intervals
// The second schedule: every workgroup is cut into `nint` intervals of `iw`
// wavefronts, and each interval is a worker of its own: it pulls a (task,
// virtual workgroup) item from the device queue, runs that task's body on
// its interval with its own interval barrier and LDS region, and pulls the
// next, with no whole-workgroup barrier between items.  The intervals of one
// workgroup run different kernels side by side whenever consecutive queue
// entries belong to different tasks -- the queue interleaves the members of
// each group item by item -- which is horizontal fusion with the pairing of
// intervals and kernels decided at run time instead of per group.  Every
// item of a task uses the same interval size, so the bodies' decomposition
// of the task's work is the same whichever interval runs which item.
struct BatchDynTables {
  const DevTask* tasks;        // [ntask]
  const int32_t* kinds;        // [ntask]
  const uint32_t* nvwg;        // [ntask] virtual workgroups of each task
  const uint32_t* item_task;   // [total_items] task of each queue entry
  const uint32_t* item_vwg;    // [total_items] its virtual workgroup
  uint32_t* queue;             // [1] pull counter, zero between launches
  uint32_t total_items;
  uint32_t iw;                 // wavefronts per interval
  uint32_t hist_words;         // LDS words of each interval's histogram region (0: none)
};

template <int BLOCK, bool HASH, int WPE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) k_batch_dyn(BatchDynTables T) {
  constexpr uint32_t W = BLOCK / 64;
  __shared__ uint32_t ctr[W];       // one interval-barrier counter per interval
  __shared__ uint32_t item_sh[W][2];
  const uint32_t wave = uniform(threadIdx.x >> 6);
  const uint32_t iw = T.iw;
  const uint32_t k = wave / iw, wv = wave - k * iw;
  const uint32_t pullers = gridDim.x * (W / iw);
  if (threadIdx.x < W) ctr[threadIdx.x] = 0u;
  if (wv == 0u && lane_id() == 0u)
    item_sh[k][0] = __hip_atomic_fetch_add(T.queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();  // the only whole-workgroup barrier: counters zero, first items visible
  PartBarrier bar(&ctr[k], iw);
  uint32_t* lds = T.hist_words ? hf_batch_hist_lds + k * T.hist_words : nullptr;
  for (uint32_t it = 0;; it ^= 1u) {
    const uint32_t item = uniform(item_sh[k][it]);
    if (item >= T.total_items) {
      // the last of the launch's past-the-end pulls resets the queue
      if (wv == 0u && lane_id() == 0u && item == T.total_items + pullers - 1u)
        __hip_atomic_store(T.queue, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    // the next item is pulled now; its latency hides behind this item's work
    if (wv == 0u && lane_id() == 0u)
      item_sh[k][it ^ 1u] = __hip_atomic_fetch_add(T.queue, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t t = uniform(T.item_task[item]);
    const Part p{threadIdx.x - 64u * iw * k, 64u * iw, wv, iw, uniform(T.item_vwg[item]), uniform(T.nvwg[t])};
    DevTask dt;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&T.tasks[t]);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&dt);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(DevTask) / 4); ++i) dst[i] = uniform(src[i]);
    run_body<HASH>((int)uniform((uint32_t)T.kinds[t]), dt, p, bar, lds);
    bar.sync();  // every wavefront of the interval is done with this item and read the next one
  }
}

// ------------------------------------------------------------------ host side
struct Batch {
  int device = 0, block = 256, ntask = 0, ngroup = 0;
  bool hash = false;  // some task is a hash kind: the hash-capable kernel variant
  uint32_t total_items = 0;
  std::vector<hf_task> tasks;
  void* dmem = nullptr;     // tables + queue
  void* scratch = nullptr;  // per-task scratch regions
  BatchTables tab{};
  BatchDynTables dyn{};
  int interval_waves = 0;  // 0: one interval per group member; else worker intervals of this many waves
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  int grid = 0;
  size_t lds_bytes = 0;  // dynamic LDS per workgroup
};

static const void* batch_kernel(int block, bool hash) {
  switch (block) {
    case 256: return hash ? reinterpret_cast<const void*>(&k_batch<256, true, 4>)
                          : reinterpret_cast<const void*>(&k_batch<256, false, 5>);
    case 512: return hash ? reinterpret_cast<const void*>(&k_batch<512, true, 4>)
                          : reinterpret_cast<const void*>(&k_batch<512, false, 5>);
    case 1024: return hash ? reinterpret_cast<const void*>(&k_batch<1024, true, 4>)
                           : reinterpret_cast<const void*>(&k_batch<1024, false, 5>);
  }
  return nullptr;
}

static const void* batch_dyn_kernel(int block, bool hash) {
  switch (block) {
    case 256: return hash ? reinterpret_cast<const void*>(&k_batch_dyn<256, true, 4>)
                          : reinterpret_cast<const void*>(&k_batch_dyn<256, false, 5>);
    case 512: return hash ? reinterpret_cast<const void*>(&k_batch_dyn<512, true, 4>)
                          : reinterpret_cast<const void*>(&k_batch_dyn<512, false, 5>);
    case 1024: return hash ? reinterpret_cast<const void*>(&k_batch_dyn<1024, true, 4>)
                           : reinterpret_cast<const void*>(&k_batch_dyn<1024, false, 5>);
  }
  return nullptr;
}

static double est_cost_us(const hf_task* t) {
  const double n = (double)t->n, c = (double)t->c, h = (double)t->h, w = (double)t->w;
  double bytes = 0, ops = 0;
  switch (t->kind) {
    case HF_BN_STATS: bytes = 4 * n * c * h * w; ops = 4 * n * c * h * w; break;
    case HF_INT_MIX: bytes = 8 * n; ops = 8.0 * n * t->p[0]; break;
    case HF_IM2COL: {
      const double kk = (double)t->p[0] * t->p[1];
      bytes = 4 * n * c * h * w * (1 + kk);
      ops = 10 * n * c * h * w * kk;
      break;
    }
    case HF_LDS_HIST: bytes = n; ops = 16 * n; break;  // LDS atomics, not HBM, bound this kernel
    case HF_UPSAMPLE: {
      const double s2 = (double)t->p[0] * t->p[0];
      bytes = 4 * n * c * h * w * (1 + s2);
      ops = 20 * n * c * h * w * s2;
      break;
    }
    case HF_MAXPOOL: {
      const double kh = t->p[0], kw = t->p[1], s = t->p[2], p = t->p[3];
      const double out = n * c * (std::floor((h + 2 * p - kh) / s) + 1) * (std::floor((w + 2 * p - kw) / s) + 1);
      bytes = 4 * n * c * h * w + (t->out1 ? 8 : 4) * out;
      ops = 4 * kh * kw * out;
      break;
    }
    case HF_SHA256D: bytes = 32 * n; ops = 3 * 64 * 24.0 * n; break;  // 3 compressions of ~24 ops/round
    case HF_BLAKE2B: bytes = 32 * n; ops = 12 * 8 * 28.0 * n; break;  // 12 rounds of 8 G of ~28 ops
    case HF_ETHASH: bytes = (64 * 128.0 + 32) * n; ops = (64 * 40.0 / 8 + 80 * 55.0) * n; break;  // rows + SHA-512
  }
  return std::max(bytes / 5.0e6, ops / 38.0e6);  // us at ~5 TB/s and ~38 T lane-op/s
}

// Waves of each task of a group: proportional to the estimated cost, at
// least one each, summing to W.
static void proportional_waves(const hf_task* t, int n, int W, int32_t* out) {
  std::vector<double> c(n);
  double tot = 0;
  for (int i = 0; i < n; ++i) tot += (c[i] = std::max(est_cost_us(&t[i]), 1e-3));
  int left = W;
  for (int i = 0; i < n; ++i) {
    out[i] = 1;
    --left;
  }
  while (left > 0) {  // give each next wave to the member with the largest cost per wave
    int best = 0;
    for (int i = 1; i < n; ++i)
      if (c[i] / out[i] > c[best] / out[best]) best = i;
    ++out[best];
    --left;
  }
  (void)tot;
}

static int batch_free(Batch* B) {
  if (!B) return HF_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(B->device);
  (void)hipDeviceSynchronize();
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  if (B->dmem) (void)hipFree(B->dmem);
  if (B->scratch) (void)hipFree(B->scratch);
  delete B;
  (void)hipSetDevice(cur);
  return HF_OK;
}

static int batch_launch(Batch* B, hipStream_t st) {
  hipError_t e;
  if (B->interval_waves) {
    void* args[] = {&B->dyn};
    e = hipLaunchKernel(batch_dyn_kernel(B->block, B->hash), dim3(B->grid), dim3(B->block), args, B->lds_bytes, st);
  } else {
    void* args[] = {&B->tab};
    e = hipLaunchKernel(batch_kernel(B->block, B->hash), dim3(B->grid), dim3(B->block), args, B->lds_bytes, st);
  }
  return e == hipSuccess ? HF_OK : record_hip(e);
}

// Host-side checks and tables of a batch under `sc`; nothing is launched.
static int batch_create(const hf_task* tasks, int ntask, const int32_t* group_of_task,
                        const int32_t* waves_of_task, const hf_batch_schedule& sc, Batch** out) {
  if (!tasks || ntask < 1 || !group_of_task || !out) return HF_EINVAL;
  const int block = sc.block;
  if (check_block(block) != HF_OK) return HF_EINVAL;
  const int W = block / 64;
  const int iw = sc.interval_waves;
  if (iw < 0 || (iw > 0 && (iw > W || W % iw != 0))) return HF_EINVAL;
  if (sc.item_kb < 0 || sc.item_kb > (1 << 20)) return HF_EINVAL;
  if (iw > 0 && waves_of_task) return HF_EINVAL;  // worker intervals have one size for every task
  int rc;
  // groups: consecutive runs of equal ids, ids nondecreasing, 1..4 members
  std::vector<int32_t> first{0};
  bool any_hist = false;
  for (int i = 0; i < ntask; ++i) {
    if ((rc = validate_task(&tasks[i])) != HF_OK) return rc;
    any_hist = any_hist || tasks[i].kind == HF_LDS_HIST;
    if (i > 0 && group_of_task[i] != group_of_task[i - 1]) {
      if (group_of_task[i] < group_of_task[i - 1]) return HF_EINVAL;
      first.push_back(i);
    }
  }
  first.push_back(ntask);
  const int ngroup = (int)first.size() - 1;
  std::vector<int32_t> waves(ntask), w0(ntask), w1(ntask), slot(ntask, -1);
  int max_hist = 0;
  for (int g = 0; g < ngroup; ++g) {
    const int n = first[g + 1] - first[g];
    if (n > kMaxMembers) return HF_EINVAL;
    if (iw > 0) continue;
    int nh = 0;
    for (int i = first[g]; i < first[g + 1]; ++i)
      if (tasks[i].kind == HF_LDS_HIST) slot[i] = nh++;
    max_hist = std::max(max_hist, nh);
    if (n > W) return HF_EINVAL;
    if (waves_of_task) {
      int sum = 0;
      for (int i = first[g]; i < first[g + 1]; ++i) {
        if (waves_of_task[i] < 1) return HF_EINVAL;
        sum += waves_of_task[i];
        waves[i] = waves_of_task[i];
      }
      if (sum > W) return HF_EINVAL;
    } else {
      proportional_waves(&tasks[first[g]], n, W, &waves[first[g]]);
    }
    int w = 0;
    for (int i = first[g]; i < first[g + 1]; ++i) {
      w0[i] = w;
      w += waves[i];
      w1[i] = w;
    }
  }
  const size_t hist_words = LdsHist::lds_words(block);
  const size_t lds_bytes = iw > 0 ? (any_hist ? (size_t)(W / iw) * hist_words * 4u : 0u)
                                  : (size_t)max_hist * hist_words * 4u;
  if (lds_bytes > 160u * 1024u - 1024u) return HF_EUNSUPPORTED;  // with the static LDS, past the CU's 160 KiB
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  Batch* B = new Batch();
  B->device = s->device;
  B->block = block;
  B->ntask = ntask;
  B->ngroup = ngroup;
  B->interval_waves = iw;
  B->tasks.assign(tasks, tasks + ntask);
  // scratch: one 256-byte aligned region per task that needs it
  std::vector<size_t> soff(ntask, 0);
  size_t sbytes = 0;
  for (int i = 0; i < ntask; ++i) {
    const int64_t nb = scratch_bytes(&tasks[i]);
    if (nb > 0 && !tasks[i].scratch) {
      soff[i] = sbytes;
      sbytes += ((size_t)nb + 255) & ~size_t(255);
    }
  }
  hipError_t e;
  if (sbytes > 0) {
    if ((e = hipMalloc(&B->scratch, sbytes)) != hipSuccess) {
      batch_free(B);
      record_hip(e);
      return HF_ENOMEM;
    }
    if ((e = hipMemset(B->scratch, 0, sbytes)) != hipSuccess) {
      batch_free(B);
      return record_hip(e);
    }
  }
  // device task arguments; virtual workgroups: enough for every member's
  // units, but items of about item_bytes of traffic, so that the per-item
  // synchronisation stays cheap
  const double item_bytes = 1024.0 * (sc.item_kb > 0 ? sc.item_kb : 256);
  std::vector<DevTask> dts(ntask);
  std::vector<int32_t> kinds(ntask);
  for (int i = 0; i < ntask; ++i) {
    void* scr = tasks[i].scratch ? tasks[i].scratch
                                 : (scratch_bytes(&tasks[i]) > 0 ? (char*)B->scratch + soff[i] : nullptr);
    if ((rc = prepare(&tasks[i], scr, &dts[i])) != HF_OK) {
      batch_free(B);
      return rc;
    }
    kinds[i] = tasks[i].kind;
    B->hash = B->hash || is_hash_kind(tasks[i].kind);
  }
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  std::vector<char> host;
  char* d = nullptr;
  if (iw == 0) {
    std::vector<uint32_t> nwg(ngroup), istart(ngroup + 1, 0);
    for (int g = 0; g < ngroup; ++g) {
      int64_t need = 1;
      double bytes = 0;
      for (int i = first[g]; i < first[g + 1]; ++i) {
        need = std::max(need, useful_wgs(&tasks[i], dts[i], waves[i]));
        bytes += est_cost_us(&tasks[i]) * 5.0e6;
      }
      const int64_t by_bytes = std::max<int64_t>(1, (int64_t)(bytes / item_bytes));
      nwg[g] = (uint32_t)std::max<int64_t>(1, std::min<int64_t>(need, by_bytes));
      istart[g + 1] = istart[g] + nwg[g];
    }
    B->total_items = istart[ngroup];
    const size_t o_tasks = 0, o_kinds = al(o_tasks + sizeof(DevTask) * ntask),
                 o_w0 = al(o_kinds + 4 * ntask), o_w1 = al(o_w0 + 4 * ntask), o_slot = al(o_w1 + 4 * ntask),
                 o_first = al(o_slot + 4 * ntask), o_istart = al(o_first + 4 * (ngroup + 1)),
                 o_nwg = al(o_istart + 4 * (ngroup + 1)), o_queue = al(o_nwg + 4 * ngroup), total = al(o_queue + 4);
    host.assign(total, 0);
    std::memcpy(host.data() + o_tasks, dts.data(), sizeof(DevTask) * ntask);
    std::memcpy(host.data() + o_kinds, kinds.data(), 4 * ntask);
    std::memcpy(host.data() + o_w0, w0.data(), 4 * ntask);
    std::memcpy(host.data() + o_w1, w1.data(), 4 * ntask);
    std::memcpy(host.data() + o_slot, slot.data(), 4 * ntask);
    std::memcpy(host.data() + o_first, first.data(), 4 * (ngroup + 1));
    std::memcpy(host.data() + o_istart, istart.data(), 4 * (ngroup + 1));
    std::memcpy(host.data() + o_nwg, nwg.data(), 4 * ngroup);
    if ((e = hipMalloc(&B->dmem, total)) != hipSuccess) {
      batch_free(B);
      record_hip(e);
      return HF_ENOMEM;
    }
    d = static_cast<char*>(B->dmem);
    B->tab.tasks = reinterpret_cast<const DevTask*>(d + o_tasks);
    B->tab.kinds = reinterpret_cast<const int32_t*>(d + o_kinds);
    B->tab.wave0 = reinterpret_cast<const int32_t*>(d + o_w0);
    B->tab.wave1 = reinterpret_cast<const int32_t*>(d + o_w1);
    B->tab.lds_slot = reinterpret_cast<const int32_t*>(d + o_slot);
    B->tab.grp_first = reinterpret_cast<const int32_t*>(d + o_first);
    B->tab.item_start = reinterpret_cast<const uint32_t*>(d + o_istart);
    B->tab.grp_nwg = reinterpret_cast<const uint32_t*>(d + o_nwg);
    B->tab.queue = reinterpret_cast<uint32_t*>(d + o_queue);
    B->tab.ngroup = (uint32_t)ngroup;
    B->tab.total_items = B->total_items;
  } else {
    // per-task virtual workgroups, then the queue: the members of each group
    // interleaved item by item
    std::vector<uint32_t> nvwg(ntask), itask, ivwg;
    for (int i = 0; i < ntask; ++i) {
      const int64_t by_bytes = std::max<int64_t>(1, (int64_t)(est_cost_us(&tasks[i]) * 5.0e6 / item_bytes));
      nvwg[i] = (uint32_t)std::max<int64_t>(1, std::min<int64_t>(useful_wgs(&tasks[i], dts[i], iw), by_bytes));
    }
    // groups in order of decreasing work, so that the launch ends on short items
    std::vector<int> gorder(ngroup);
    std::vector<double> gcost(ngroup, 0.0);
    for (int g = 0; g < ngroup; ++g) {
      gorder[g] = g;
      for (int i = first[g]; i < first[g + 1]; ++i) gcost[g] += est_cost_us(&tasks[i]);
    }
    std::stable_sort(gorder.begin(), gorder.end(), [&](int x, int y) { return gcost[x] > gcost[y]; });
    for (int g : gorder) {
      uint32_t most = 0;
      for (int i = first[g]; i < first[g + 1]; ++i) most = std::max(most, nvwg[i]);
      for (uint32_t b = 0; b < most; ++b)
        for (int i = first[g]; i < first[g + 1]; ++i)
          if (b < nvwg[i]) {
            itask.push_back((uint32_t)i);
            ivwg.push_back(b);
          }
    }
    B->total_items = (uint32_t)itask.size();
    const size_t o_tasks = 0, o_kinds = al(o_tasks + sizeof(DevTask) * ntask), o_nvwg = al(o_kinds + 4 * ntask),
                 o_it = al(o_nvwg + 4 * ntask), o_iv = al(o_it + 4 * (size_t)B->total_items),
                 o_queue = al(o_iv + 4 * (size_t)B->total_items), total = al(o_queue + 4);
    host.assign(total, 0);
    std::memcpy(host.data() + o_tasks, dts.data(), sizeof(DevTask) * ntask);
    std::memcpy(host.data() + o_kinds, kinds.data(), 4 * ntask);
    std::memcpy(host.data() + o_nvwg, nvwg.data(), 4 * ntask);
    std::memcpy(host.data() + o_it, itask.data(), 4 * itask.size());
    std::memcpy(host.data() + o_iv, ivwg.data(), 4 * ivwg.size());
    if ((e = hipMalloc(&B->dmem, total)) != hipSuccess) {
      batch_free(B);
      record_hip(e);
      return HF_ENOMEM;
    }
    d = static_cast<char*>(B->dmem);
    B->dyn.tasks = reinterpret_cast<const DevTask*>(d + o_tasks);
    B->dyn.kinds = reinterpret_cast<const int32_t*>(d + o_kinds);
    B->dyn.nvwg = reinterpret_cast<const uint32_t*>(d + o_nvwg);
    B->dyn.item_task = reinterpret_cast<const uint32_t*>(d + o_it);
    B->dyn.item_vwg = reinterpret_cast<const uint32_t*>(d + o_iv);
    B->dyn.queue = reinterpret_cast<uint32_t*>(d + o_queue);
    B->dyn.total_items = B->total_items;
    B->dyn.iw = (uint32_t)iw;
    B->dyn.hist_words = any_hist ? (uint32_t)hist_words : 0u;
  }
  if ((e = hipMemcpy(B->dmem, host.data(), host.size(), hipMemcpyHostToDevice)) != hipSuccess) {
    batch_free(B);
    return record_hip(e);
  }
  B->lds_bytes = lds_bytes;
  const void* fn = iw > 0 ? batch_dyn_kernel(block, B->hash) : batch_kernel(block, B->hash);
  int occ = 0;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, block, B->lds_bytes)) != hipSuccess) {
    batch_free(B);
    return record_hip(e);
  }
  if (occ < 1) {
    batch_free(B);
    return HF_EUNSUPPORTED;
  }
  const int64_t per_wg = iw > 0 ? W / iw : 1;  // workers per workgroup
  const int64_t want = ((int64_t)B->total_items + per_wg - 1) / per_wg;
  B->grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)occ * s->num_cus, want));
  *out = B;
  return HF_OK;
}

static int batch_run(Batch* B, int use_graph, hipStream_t st) {
  if (!use_graph) return batch_launch(B, st);
  hipError_t e;
  if (!B->exec) {
    if (!B->cap && (e = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking)) != hipSuccess)
      return record_hip(e);
    if ((e = hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) return record_hip(e);
    int rc = batch_launch(B, B->cap);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(B->cap, &gr);
    if (rc != HF_OK) return rc;
    if (e != hipSuccess) return record_hip(e);
    B->graph = gr;
    if ((e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0)) != hipSuccess) return record_hip(e);
  }
  e = hipGraphLaunch(B->exec, st);
  return e == hipSuccess ? HF_OK : record_hip(e);
}

static int batch_time(Batch* B, int use_graph, hipStream_t st, float* ms) {
  int rc;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  if (ms) {
    hipError_t e = hipEventRecord(s->ev_start, st);
    if (e != hipSuccess) return record_hip(e);
  }
  if ((rc = batch_run(B, use_graph, st)) != HF_OK) return rc;
  if (!ms) return HF_OK;
  hipError_t e = hipEventRecord(s->ev_stop, st);
  if (e != hipSuccess) return record_hip(e);
  if ((rc = wait_event(s->ev_stop)) != HF_OK) return rc;
  e = hipEventElapsedTime(ms, s->ev_start, s->ev_stop);
  return e == hipSuccess ? HF_OK : record_hip(e);
}

static int check_batch(void* b, Batch** out) {
  if (!b) return HF_EINVAL;
  Batch* B = static_cast<Batch*>(b);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return record_hip(e);
  if (dev != B->device) return HF_EINVAL;
  *out = B;
  return HF_OK;
}

}  // namespace hf

using namespace hf;

extern "C" {

int hf_batch_create_sched(const hf_task* tasks, int ntask, const int32_t* group_of_task,
                          const int32_t* waves_of_task, const hf_batch_schedule* sched, void** batch_out) {
  if (!batch_out || !sched) return HF_EINVAL;
  *batch_out = nullptr;
  if (sched->split_policy < 0 || sched->split_policy > 1) return HF_EINVAL;
  std::vector<int32_t> even;
  if (!waves_of_task && sched->interval_waves == 0 && sched->split_policy == 1 && tasks && group_of_task &&
      ntask > 0 && check_block(sched->block) == HF_OK) {
    // the even split: every member of a group gets W / n wavefronts (the
    // first W % n one more)
    const int W = sched->block / 64;
    even.assign(ntask, 1);
    for (int i = 0; i < ntask;) {
      int j = i;
      while (j < ntask && group_of_task[j] == group_of_task[i]) ++j;
      const int n = j - i;
      for (int k = 0; k < n; ++k) even[i + k] = std::max(1, W / n + (k < W % n ? 1 : 0));
      i = j;
    }
    waves_of_task = even.data();
  }
  Batch* B = nullptr;
  int rc = batch_create(tasks, ntask, group_of_task, waves_of_task, *sched, &B);
  if (rc == HF_OK) *batch_out = B;
  return rc;
}

int hf_batch_create(const hf_task* tasks, int ntask, const int32_t* group_of_task,
                    const int32_t* waves_of_task, int block, void** batch_out) {
  const hf_batch_schedule sc{block, 0, 0, 0};
  return hf_batch_create_sched(tasks, ntask, group_of_task, waves_of_task, &sc, batch_out);
}

int hf_batch_run(void* batch, int use_graph, void* stream, float* ms_out) {
  Batch* B = nullptr;
  int rc = check_batch(batch, &B);
  if (rc != HF_OK) return rc;
  return batch_time(B, use_graph, static_cast<hipStream_t>(stream), ms_out);
}

int hf_batch_info(void* batch, int32_t* total_items, int32_t* grid, int32_t* ngroup) {
  Batch* B = nullptr;
  int rc = check_batch(batch, &B);
  if (rc != HF_OK) return rc;
  if (total_items) *total_items = (int32_t)B->total_items;
  if (grid) *grid = B->grid;
  if (ngroup) *ngroup = B->ngroup;
  return HF_OK;
}

int hf_batch_destroy(void* batch) { return batch_free(static_cast<Batch*>(batch)); }

int hf_run_batch(const hf_task* tasks, int ntask, const int32_t* group_of_task,
                 const int32_t* waves_of_task, int block, void* stream, float* ms_out) {
  void* b = nullptr;
  int rc = hf_batch_create(tasks, ntask, group_of_task, waves_of_task, block, &b);
  if (rc != HF_OK) return rc;
  rc = hf_batch_run(b, 0, stream, ms_out);
  if (rc == HF_OK && !ms_out) {
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));  // before freeing the tables
    if (e != hipSuccess) rc = record_hip(e);
  }
  hf_batch_destroy(b);
  return rc;
}

// Median time (ms) of `reps` timed launches of the batch under `sc` (after
// one untimed launch); HF_EUNSUPPORTED / HF_EINVAL from creation pass through.
static int profile_schedule(const hf_task* tasks, int ntask, const int32_t* group_of_task,
                            const hf_batch_schedule& sc, int reps, hipStream_t st, float* med) {
  void* b = nullptr;
  int rc = hf_batch_create_sched(tasks, ntask, group_of_task, nullptr, &sc, &b);
  if (rc != HF_OK) return rc;
  std::vector<float> ts;
  for (int r = 0; r <= reps && rc == HF_OK; ++r) {
    float ms = 0.f;
    rc = hf_batch_run(b, 0, st, &ms);
    if (r > 0) ts.push_back(ms);
  }
  hf_batch_destroy(b);
  if (rc != HF_OK) return rc;
  std::sort(ts.begin(), ts.end());
  *med = ts[ts.size() / 2];
  return HF_OK;
}

// The schedule tuner: every static schedule (workgroup size 256, 512 or 1024;
// wavefronts split in proportion to the estimated cost or evenly; items of
// 128, 256 or 512 KiB) and every worker-interval schedule (workgroup size x
// interval of 1, 2, 4 or 8 wavefronts x items of 64, 128, 256 or 512 KiB) that
// the batch admits, each profiled as the median of `reps` launches; writes the
// fastest.
int hf_batch_tune_sched(const hf_task* tasks, int ntask, const int32_t* group_of_task, int reps, void* stream,
                        hf_batch_schedule* best_out, float* ms_out, int32_t* n_profiled) {
  if (!tasks || ntask < 1 || !group_of_task || !best_out || reps < 1) return HF_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<hf_batch_schedule> cands;
  for (int block : {256, 512, 1024}) {
    for (int pol = 0; pol < 2; ++pol)
      for (int kb : {128, 256, 512}) cands.push_back({block, 0, kb, pol});
    for (int iw : {1, 2, 4, 8})
      if (iw <= block / 64)
        for (int kb : {64, 128, 256, 512}) cands.push_back({block, iw, kb, 0});
  }
  float best = 1e30f;
  int nprof = 0;
  for (const hf_batch_schedule& sc : cands) {
    float med = 0.f;
    const int rc = profile_schedule(tasks, ntask, group_of_task, sc, reps, st, &med);
    if (rc == HF_EINVAL || rc == HF_EUNSUPPORTED) continue;  // this batch does not admit the schedule
    if (rc != HF_OK) return rc;
    ++nprof;
    if (med < best) {
      best = med;
      *best_out = sc;
    }
  }
  if (best >= 1e30f) return HF_EINVAL;
  if (ms_out) *ms_out = best;
  if (n_profiled) *n_profiled = nprof;
  return HF_OK;
}

// The static-schedule tuner of the earlier interface: both split policies at
// workgroup sizes 256, 512 and 1024 (items of 256 KiB); writes the fastest
// schedule's per-task waves and block.
int hf_batch_tune(const hf_task* tasks, int ntask, const int32_t* group_of_task, int reps, void* stream,
                  int32_t* waves_out, int32_t* block_out, float* ms_out) {
  if (!tasks || ntask < 1 || !group_of_task || !waves_out || !block_out || reps < 1) return HF_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float best = 1e30f;
  for (int block : {256, 512, 1024}) {
    const int W = block / 64;
    for (int policy = 0; policy < 2; ++policy) {
      std::vector<int32_t> waves(ntask);
      int i = 0;
      bool ok = true;
      while (i < ntask) {
        int j = i;
        while (j < ntask && group_of_task[j] == group_of_task[i]) ++j;
        const int n = j - i;
        if (n > W || n > kMaxMembers) {
          ok = false;
          break;
        }
        if (policy == 0) proportional_waves(&tasks[i], n, W, &waves[i]);
        else
          for (int k = 0; k < n; ++k) waves[i + k] = W / n + (k < W % n ? 1 : 0);
        i = j;
      }
      if (!ok) continue;
      const hf_batch_schedule sc{block, 0, 256, policy};
      float med = 0.f;
      const int rc = profile_schedule(tasks, ntask, group_of_task, sc, reps, st, &med);
      if (rc == HF_EINVAL || rc == HF_EUNSUPPORTED) continue;
      if (rc != HF_OK) return rc;
      if (med < best) {
        best = med;
        std::copy(waves.begin(), waves.end(), waves_out);
        *block_out = block;
      }
    }
  }
  if (best >= 1e30f) return HF_EINVAL;
  if (ms_out) *ms_out = best;
  return HF_OK;
}

}  // extern "C"
