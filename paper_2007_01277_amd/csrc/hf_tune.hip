// hf_tune.hip -- configuration search for a fused pair (Sec. III-B).
//
// The paper's Main search profiles, for d0 = 1024 and d1 = 128, 256, ..., 896,
// the fused kernel once without a register bound and once with the bound r0,
// and keeps a candidate only when it is strictly faster.  The exhaustive mode
// widens the space to workgroup sizes 256/512/1024, splits in eighths of the
// workgroup (wavefront aligned) and every compiled VGPR bound.  The learned
// mode ranks that space with the cost model and profiles only the top k.  The
// grid mode adds the launch grid, a free parameter here because every body is a
// grid-stride loop: the three best configurations of the exhaustive space are
// profiled again at 2, 4 and 8 times the occupancy grid, which lets workgroups
// whose partitions finish early leave the CU to new ones.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>

#include "hf_runtime.hpp"

namespace hf {

static const int kCaps[] = {0, 64, 80, 96, 128};

// Largest compiled VGPR bound not above r0 (the smallest bound if r0 is below
// every compiled one: occupancy cannot exceed 8 wavefronts per SIMD anyway).
static int cap_for_bound(int r0) {
  int best = 64;
  for (int c : kCaps)
    if (c > 0 && c <= r0) best = c;
  return best;
}

int register_bound(int d1, int d2, int va, int vb, int lds) {
  const int R = 4 * 512 * 64, LDS = 160 * 1024, T = 2048;
  if (d1 <= 0 || d2 <= 0 || va <= 0 || vb <= 0 || lds < 0) return HF_EINVAL;
  const int d0 = d1 + d2;
  int b0 = std::min(R / (d1 * va), R / (d2 * vb));
  b0 = std::min(b0, T / d0);
  if (lds > 0) b0 = std::min(b0, LDS / lds);
  if (b0 <= 0) return HF_EINVAL;
  return R / (b0 * d0);
}

int candidates(int method, int block, int va, int vb, int lds, std::vector<hf_config>* out) {
  out->clear();
  if (block != 0 && check_block(block) != HF_OK) return HF_EINVAL;
  switch (method) {
    case HF_TUNE_NAIVE: {
      const int b = block ? block : 1024;
      out->push_back(hf_config{b / 128, b, 0, 0});
      return HF_OK;
    }
    case HF_TUNE_PAPER: {
      const int d0 = block ? block : 1024;
      for (int d1 = 128; d1 < d0; d1 += 128) {
        out->push_back(hf_config{d1 / 64, d0, 0, 0});
        const int r0 = register_bound(d1, d0 - d1, va, vb, lds);
        if (r0 < 0) return r0;
        out->push_back(hf_config{d1 / 64, d0, cap_for_bound(r0), 0});
      }
      return HF_OK;
    }
    case HF_TUNE_EXHAUSTIVE:
    case HF_TUNE_EXHAUSTIVE_GRID:
    case HF_TUNE_MLP: {
      const int blocks[] = {256, 512, 1024};
      for (int b : blocks) {
        if (block && b != block) continue;
        for (int k = 1; k < 8; ++k) {
          if ((b * k) % 8 != 0 || ((b * k) / 8) % 64 != 0) continue;
          for (int cap : kCaps) out->push_back(hf_config{(b * k) / 8 / 64, b, cap, 0});
        }
      }
      return HF_OK;
    }
  }
  return HF_EINVAL;
}

static int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

// Median time of `reps` launches after one untimed launch.
int profile(DeviceState* s, const hf_pair* pr, const hf_config& cfg, int reps, hipStream_t st,
            float* median) {
  int rc = launch_fused(s, pr, &cfg, st, nullptr);
  if (rc != HF_OK) return rc;
  const bool scrub = env_int("HF_TUNE_SCRUB", 0) != 0;
  std::vector<float> t(reps);
  for (int r = 0; r < reps; ++r) {
    if (scrub && (rc = hf_scrub(st)) != HF_OK) return rc;
    hipError_t e = hipEventRecord(s->ev_start, st);
    if (e != hipSuccess) return record_hip(e);
    if ((rc = launch_fused(s, pr, &cfg, st, nullptr)) != HF_OK) return rc;
    if ((e = hipEventRecord(s->ev_stop, st)) != hipSuccess) return record_hip(e);
    if ((rc = wait_event(s->ev_stop)) != HF_OK) return rc;
    if ((e = hipEventElapsedTime(&t[r], s->ev_start, s->ev_stop)) != hipSuccess) return record_hip(e);
  }
  std::sort(t.begin(), t.end());
  *median = t[reps / 2];
  return HF_OK;
}

int solo_vgprs(DeviceState* s, int kind, int* v) {
  hf_kernel_info info;
  const KernelEntry* k = find_kernel(kind, -1, 1024, 0);
  if (!k) return HF_EUNSUPPORTED;
  int rc = kernel_info(s, k->fn, 1024, &info);
  if (rc != HF_OK) return rc;
  *v = std::max(1, info.vgprs);
  return HF_OK;
}

// Ranks candidates with the learned model; defined in hf_mlp.hip.
int mlp_rank(DeviceState* s, const hf_pair* pr, const std::vector<hf_config>& cands, hipStream_t st,
             std::vector<int>* order, FeatCost* cost);

}  // namespace hf

using namespace hf;

extern "C" {

int hf_register_bound(int d1, int d2, int vgpr_a, int vgpr_b, int lds_fused) {
  return register_bound(d1, d2, vgpr_a, vgpr_b, lds_fused);
}

int hf_tune_candidates(int method, int block, int vgpr_a, int vgpr_b, int lds_fused,
                       hf_config* out, int max) {
  std::vector<hf_config> c;
  int rc = candidates(method, block, vgpr_a, vgpr_b, lds_fused, &c);
  if (rc != HF_OK) return rc;
  if (out) std::memcpy(out, c.data(), sizeof(hf_config) * std::min<size_t>(c.size(), std::max(max, 0)));
  return (int)c.size();
}

int hf_profile(const hf_pair* pr, const hf_config* cfg, int reps, void* stream, float* median_ms) {
  if (!median_ms || reps < 1) return HF_EINVAL;
  int rc = hf_validate_fused(pr, cfg);
  if (rc != HF_OK) return rc;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  return profile(s, pr, *cfg, reps, static_cast<hipStream_t>(stream), median_ms);
}

int hf_tune(const hf_pair* pr, int method, int block, int topk, void* stream, hf_config* best,
            hf_tune_stats* stats) {
  if (!pr || !best) return HF_EINVAL;
  if (method < HF_TUNE_EXHAUSTIVE || method > HF_TUNE_EXHAUSTIVE_GRID) return HF_EINVAL;
  int rc;
  if ((rc = validate_task(&pr->a)) != HF_OK || (rc = validate_task(&pr->b)) != HF_OK) return rc;
  if (block != 0 && check_block(block) != HF_OK) return HF_EINVAL;
  if (method == HF_TUNE_MLP && topk < 1) return HF_EINVAL;
  DeviceState* s = device_state(&rc);
  if (!s) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  const int reps = std::max(1, env_int("HF_TUNE_REPS", 20));

  int va = 1, vb = 1, lds = 0;
  if (method == HF_TUNE_PAPER) {
    if ((rc = solo_vgprs(s, pr->a.kind, &va)) != HF_OK) return rc;
    if ((rc = solo_vgprs(s, pr->b.kind, &vb)) != HF_OK) return rc;
    hf_kernel_info fi;
    if ((rc = hf_fused_info(pr->a.kind, pr->b.kind, block ? block : 1024, 0, &fi)) != HF_OK) return rc;
    lds = fi.lds_bytes;
  }
  std::vector<hf_config> cands;
  if ((rc = candidates(method, block, va, vb, lds, &cands)) != HF_OK) return rc;

  std::vector<int> order(cands.size());
  for (size_t i = 0; i < cands.size(); ++i) order[i] = (int)i;
  FeatCost fcost;
  if (method == HF_TUNE_MLP) {
    if ((rc = mlp_rank(s, pr, cands, st, &order, &fcost)) != HF_OK) return rc;
    // the k best-ranked candidates with pairwise distinct (split, block): the
    // VGPR bounds of one (split, block) often time alike, and a profile spent
    // on a second bound of the same split hedges less than another split
    std::vector<int> top;
    for (int i : order) {
      if ((int)top.size() >= topk) break;
      bool seen = false;
      for (int j : top) seen = seen || (cands[j].split_waves == cands[i].split_waves && cands[j].block == cands[i].block);
      if (!seen) top.push_back(i);
    }
    order.swap(top);
  }

  float tbest = 0.f;
  int ibest = -1, nprof = 0;
  std::vector<float> times(cands.size(), 0.f);
  for (int i : order) {
    float t = 0.f;
    if ((rc = profile(s, pr, cands[i], reps, st, &t)) != HF_OK) return rc;
    times[i] = t;
    ++nprof;
    if (ibest < 0 || t < tbest) {  // strict: the first-found candidate keeps ties
      tbest = t;
      ibest = i;
    }
  }
  *best = cands[ibest];
  int ncand = (int)cands.size();
  if (method == HF_TUNE_EXHAUSTIVE_GRID) {
    std::vector<int> top(order);
    std::stable_sort(top.begin(), top.end(), [&](int x, int y) { return times[x] < times[y]; });
    if (top.size() > 3) top.resize(3);
    for (int i : top) {
      hf_config c = cands[i];
      hf_kernel_info fi;
      if ((rc = hf_fused_info(pr->a.kind, pr->b.kind, c.block, c.vgpr_cap, &fi)) != HF_OK) return rc;
      int used = 0;
      if ((rc = launch_fused(s, pr, &c, st, &used)) != HF_OK) return rc;
      if (used < fi.default_grid) continue;  // too little work to fill even the occupancy grid
      for (int m : {2, 4, 8}) {
        c.grid = fi.default_grid * m;
        float t = 0.f;
        if ((rc = profile(s, pr, c, reps, st, &t)) != HF_OK) return rc;
        ++nprof;
        ++ncand;
        if (t < tbest) {
          tbest = t;
          *best = c;
        }
      }
    }
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->n_candidates = ncand;
    stats->n_profiled = nprof;
    stats->t_best_ms = tbest;
    stats->reps = reps;
    const hf_config naive{8, 1024, 0, 0};
    float tn = 0.f;
    if ((rc = profile(s, pr, naive, reps, st, &tn)) != HF_OK) return rc;
    stats->t_naive_ms = tn;
    stats->n_solo_launches = fcost.launches;
    stats->solo_ms = (float)fcost.ms;
    stats->wall_s = std::chrono::duration<float>(std::chrono::steady_clock::now() - t0).count();
  }
  return HF_OK;
}

}  // extern "C"
