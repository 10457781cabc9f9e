// Host-side checks of the C ABI under AddressSanitizer: the validation,
// scratch sizing, candidate generation, register bound, batch-table checks
// and error strings, driven with well-formed and malformed descriptors.  Every
// call here returns before any HIP call, so it runs without a GPU.  The
// library's host translation units are compiled with -fsanitize=address for
// the host side only; an out-of-bounds access or use of freed memory in them
// aborts the run with a report.  Prints "host checks ok" and exits 0 on success.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/hfuse.h"

static int failures = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint64_t next() {  // xorshift64 (Marsaglia)
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return rng;
}
static int64_t pick(const int64_t* v, int n) { return v[next() % n]; }

static void* fake(uintptr_t off) { return reinterpret_cast<void*>(uintptr_t(0x10000000) + off); }

static hf_task random_task() {
  static const int64_t dims[] = {-1, 0, 1, 2, 3, 7, 16, 56, 1000, 1 << 20, int64_t(1) << 31, int64_t(1) << 40};
  static const int64_t ps[] = {-3, -1, 0, 1, 2, 3, 5, 16, 64, 65, 256, 1 << 30};
  hf_task t;
  std::memset(&t, 0, sizeof(t));
  t.kind = (int32_t)(next() % (HF_NUM_KINDS + 2)) - 1;
  for (int i = 0; i < 4; ++i) t.p[i] = (int32_t)pick(ps, 12);
  t.in = (next() % 5) ? fake(16 * (next() % 64) + (next() % 3 == 0 ? 1 : 0)) : nullptr;
  t.out0 = (next() % 5) ? fake(1 << 20) : nullptr;
  t.out1 = (next() % 3) ? fake(1 << 21) : nullptr;
  t.in1 = (next() % 3) ? fake(1 << 22) : nullptr;
  t.n = pick(dims, 12);
  t.c = pick(dims, 12);
  t.h = pick(dims, 12);
  t.w = pick(dims, 12);
  return t;
}

int main() {
  // error strings for every status and a few that do not exist
  for (int s = -10; s <= 1; ++s) EXPECT(hf_strerror(s) != nullptr && std::strlen(hf_strerror(s)) > 0);
  EXPECT(std::strstr(hf_version(), "gfx950") != nullptr);

  // malformed and well-formed descriptors: validation, scratch size, pairs
  int valid = 0;
  for (int it = 0; it < 200000; ++it) {
    hf_task a = random_task(), b = random_task();
    const int va = hf_validate_task(&a);
    EXPECT(va == HF_OK || va == HF_EINVAL);
    const int64_t sb = hf_scratch_bytes(&a);
    EXPECT((va == HF_OK) == (sb >= 0));
    valid += va == HF_OK;
    hf_pair pr{a, b};
    hf_config cfg{(int32_t)(next() % 18) - 1, (int32_t)(128 << (next() % 5)), (int32_t)((next() % 6) * 16),
                  (int32_t)(next() % 4) - 1};
    const int vf = hf_validate_fused(&pr, &cfg);
    EXPECT(vf == HF_OK || vf == HF_EINVAL || vf == HF_EUNSUPPORTED);
  }
  EXPECT(valid > 100);  // the generator reaches valid descriptors too
  EXPECT(hf_validate_task(nullptr) == HF_EINVAL);
  EXPECT(hf_validate_fused(nullptr, nullptr) == HF_EINVAL);

  // candidate lists of every method, with an exact-size and a short buffer
  for (int m = -1; m <= 5; ++m)
    for (int blk : {0, 256, 384, 512, 1024}) {
      const int n = hf_tune_candidates(m, blk, 40, 90, 16384, nullptr, 0);
      if (n < 0) continue;
      std::vector<hf_config> all(n);
      EXPECT(hf_tune_candidates(m, blk, 40, 90, 16384, all.data(), n) == n);
      std::vector<hf_config> few(1);
      EXPECT(hf_tune_candidates(m, blk, 40, 90, 16384, few.data(), 1) == n);
    }

  // the register bound over a range of partitions and register counts
  for (int it = 0; it < 100000; ++it) {
    const int d1 = 64 * (int)(next() % 17), d2 = 64 * (int)(next() % 17);
    const int r = hf_register_bound(d1, d2, (int)(next() % 300) - 5, (int)(next() % 300) - 5,
                                    (int)(next() % 200000) - 100);
    EXPECT(r >= 1 || r == HF_EINVAL);
  }

  // batch tables rejected on the host: bad groups, blocks, waves
  std::vector<hf_task> tasks(6);
  for (auto& t : tasks) {
    std::memset(&t, 0, sizeof(t));
    t.kind = HF_INT_MIX;
    t.p[0] = 3;
    t.in = fake(0);
    t.out0 = fake(1 << 20);
    t.n = 1000;
  }
  const int32_t dec[6] = {0, 1, 1, 0, 2, 2};       // decreasing ids
  const int32_t five[6] = {0, 0, 0, 0, 0, 1};      // a group of five
  const int32_t ok[6] = {0, 0, 1, 1, 2, 2};
  const int32_t zero_waves[6] = {1, 0, 1, 1, 1, 1};
  const int32_t too_many[6] = {3, 2, 1, 1, 1, 1};  // 5 waves in a 256-lane group
  void* handle = nullptr;
  EXPECT(hf_batch_create(tasks.data(), 6, dec, nullptr, 256, &handle) == HF_EINVAL);
  EXPECT(hf_batch_create(tasks.data(), 6, five, nullptr, 256, &handle) == HF_EINVAL);
  EXPECT(hf_batch_create(tasks.data(), 6, ok, nullptr, 384, &handle) == HF_EINVAL);
  EXPECT(hf_batch_create(tasks.data(), 6, ok, zero_waves, 256, &handle) == HF_EINVAL);
  EXPECT(hf_batch_create(tasks.data(), 6, ok, too_many, 256, &handle) == HF_EINVAL);
  EXPECT(hf_batch_create(tasks.data(), 0, ok, nullptr, 256, &handle) == HF_EINVAL);
  EXPECT(hf_batch_create(nullptr, 6, ok, nullptr, 256, &handle) == HF_EINVAL);
  EXPECT(handle == nullptr);

  // the allocation-free launch rejects before the GPU
  hf_task big;
  std::memset(&big, 0, sizeof(big));
  big.kind = HF_BN_STATS;
  big.in = fake(0);
  big.out0 = fake(1 << 20);
  big.out1 = fake(1 << 21);
  big.n = big.c = big.h = 1;
  big.w = (int64_t(1) << 31) - 1 - (1 << 20);
  hf_pair bp{big, tasks[0]};
  hf_config c2{2, 256, 0, 0};
  EXPECT(hf_run_fused_noalloc(&bp, &c2, nullptr) == HF_ESCRATCH);

  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host checks ok (%d valid descriptors)\n", valid);
  return 0;
}
