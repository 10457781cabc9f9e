// hf_bodies.hpp -- the kernel bodies that horizontal fusion combines.
//
// Each body is written once, as a __device__ function of an interval (Part) and
// a barrier type.  The solo kernel instantiates it with the whole workgroup and
// the native workgroup barrier; the fused kernel instantiates it with one
// wavefront-aligned interval and the interval's LDS barrier (Sec. III-A,
// Generate algorithm: the built-ins threadIdx.x / blockDim.x become the interval
// variables tid_i / size_i, and __syncthreads becomes the interval barrier).
//
// Every body is grid-stride over work units, so it is correct for any grid and
// any interval size; units whose result is floating point are owned by one
// wavefront and reduced in a fixed order, so a fused launch reproduces the solo
// launch bit for bit whatever the split.
#pragma once
#include "hf_device.hpp"

namespace hf {

// ======================================================================= args
// Per-kind kernel arguments, filled on the host from an hf_task.

struct BnArgs {  // per-channel mean / biased variance of NCHW fp32
  const float* x;
  float* mean;
  float* var;
  uint32_t* ctr;   // [C] unit arrival counters (zero between launches)
  uint32_t* part;  // [C][upc][2] per-unit (mean, M2) as float bits
  uint32_t C, HW, M, CHWm;  // M = N*HW elements per channel, CHWm = (C-1)*HW
  uint32_t upc;             // units per channel
  uint32_t total;           // C * upc
  uint32_t vec;             // float4 path: HW % 4 == 0 and x 16-byte aligned
  FastDiv div_hw, div_upc;
};

struct MixArgs {  // R rounds of xorshift32 + multiply-add per uint32
  const uint32_t* in;
  uint32_t* out;
  uint32_t n, n4;  // elements, and uint4 vectors in the vector path (0 otherwise)
  int32_t rounds;
};

struct HistArgs {  // 256-bin histogram of bytes
  const uint8_t* in;
  uint32_t* out;
  uint32_t* acc;  // [256] merged counts (zero between launches)
  uint32_t* ctr;  // [1] workgroup arrival counter (zero between launches)
  uint32_t n;
  uint32_t head;        // bytes before the first 16-byte aligned address
  uint32_t n16;         // aligned 16-byte vectors after the head
  uint32_t tail_start;  // head + 16 * n16
};

struct Im2colArgs {  // patches -> columns, [N][C*kh*kw][Ho*Wo]
  const float* x;
  float* out;
  uint32_t C, H, W, kw, s, p, Ho, Wo, KK;
  uint32_t units;           // N * C * kh*kw output planes
  uint32_t lanes_per_unit;  // Ho * Wo4 (vector) or Ho * Wo (scalar)
  uint32_t vec;             // Wo % 4 == 0 and out 16-byte aligned
  FastDiv div_kk, div_row, div_kw;  // div_row: by Wo4 (vector) or Wo
  uint32_t row3;            // the 3x3 / stride 1 / pad 1 row path (see Im2col)
  uint32_t nch;             // row path: chunks of 64 columns per row, ceil(W / 64)
  uint32_t nq;              // row path: units per channel, ceil(H * nch / 4)
  uint32_t row_units;       // row path: N * C * nq
  FastDiv div_nq, div_nch;
};

struct UpArgs {  // bilinear upsampling by integer factor s, half-pixel centres
  const float* x;
  float* out;
  uint32_t H, W, Ho, Wo;
  float inv_s;
  uint32_t rows;            // N*C*Ho output rows
  uint32_t rows_per_unit;   // rows handled together when rows are short
  uint32_t units;           // ceil(rows / rows_per_unit)
  uint32_t lanes_per_unit;  // rows_per_unit * Wo4 (vector) or * Wo
  uint32_t vec;             // Wo % 4 == 0 and out 16-byte aligned
  FastDiv div_ho, div_row;  // div_row: by Wo4 (vector) or Wo
  uint32_t row2;            // the scale-2 row path (see Upsample)
  uint32_t nch;             // row path: chunks of 32 input columns per row, ceil(W / 32)
  uint32_t nq;              // row path: units per plane, ceil(Ho * nch / 4)
  uint32_t row_units;       // row path: N * C * nq
  FastDiv div_nq, div_nch;
};

struct PoolArgs {  // max pooling with the winner's flat index
  const float* x;
  float* out;
  int32_t* idx;  // null: values only
  uint32_t H, W, Ho, Wo, kh, kw, s, p;
  uint32_t total;  // N*C*Ho*Wo outputs
  uint32_t units;  // ceil(total / Maxpool::kUnit)
  FastDiv div_plane, div_wo;  // by Ho*Wo and by Wo
  uint32_t row3;       // the 3x3 / stride 2 / pad 1 row path (see Maxpool)
  uint32_t nch;        // row path: chunks of 128 input columns per row, ceil(W / 128)
  uint32_t nq;         // row path: units per plane, ceil(Ho * nch / 4)
  uint32_t row_units;  // row path: planes * nq
  FastDiv div_nq, div_nch;
};

struct ShaArgs {  // SHA-256d and BLAKE2b over header || nonce
  const uint32_t* hdr;  // 20 words: the 80-byte header
  uint32_t* out;        // [n][8] words: 32-byte digests
  uint32_t nonce0, n;
};

struct EthArgs {  // Ethash-like folds of table rows
  const uint32_t* hdr;  // 20 words: the 80-byte header
  const uint4* table;   // [rows][8] uint4: rows of 128 bytes
  uint32_t* out;        // [n][8] words
  uint32_t nonce0, n;
  FastMod rows;         // rows.d: the table's row count
};

union DevTask {
  BnArgs bn;
  MixArgs mix;
  HistArgs hist;
  Im2colArgs im2col;
  UpArgs up;
  PoolArgs pool;
  ShaArgs sha;
  EthArgs eth;
};

// Agent-scope helpers for partial results exchanged between workgroups.
__device__ __forceinline__ void store_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_agent(uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until every vector-memory operation this wave issued has completed
// (s_waitcnt vmcnt(0); expcnt and lgkmcnt left at their maxima, GFX9 encoding).
// For a store or an atomic, completion means the device-coherent level has
// acknowledged it.
__device__ __forceinline__ void wait_vmem() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // keeps prior accesses above
  __builtin_amdgcn_s_waitcnt(0x0F70);
}

// Arrival on a cross-workgroup counter after publishing results.  Everything a
// wave publishes for other workgroups goes through device-coherent accesses
// (agent-scope atomic stores and RMWs, read back with agent-scope atomic loads
// or RMWs), so no L2 writeback or invalidate is needed: it is enough that those
// accesses have completed before the arrival is counted.  An agent-scope
// release would add an L2 writeback, and an acquire an L2 invalidate, to every
// arrival, which on a multi-XCD part stalls every wave of the die.  The wave
// that sees itself as the last arrival reads the published data only with
// agent-scope atomic loads or RMWs issued after its counter RMW returned.
__device__ __forceinline__ uint32_t arrive_after_coherent_stores(uint32_t* ctr, uint32_t n = 1u) {
  wait_vmem();
  return __hip_atomic_fetch_add(ctr, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ================================================================== bn_stats
// Statistics kernel of the normalisation example (Sec. II-C): per-channel mean
// and variance of x[N][C][H][W].
//
// Work decomposition (fixed by the shape, independent of grid and interval):
//   unit = 1024 consecutive elements of one channel's N*H*W sequence.  One
//          wavefront loads it (16 values per lane; the next unit is already in
//          flight in its own register slot), computes the unit's mean and M2
//          by two passes over registers with fixed-order wave sums, and
//          publishes (mean, M2).
//   Each wavefront of the launch owns a contiguous, balanced range of units;
//   at the end of each channel segment of its range it adds the segment's unit
//   count to the channel's arrival counter.  The wavefront that completes a
//   channel merges its units' (count, mean, M2) in double, in unit order, with
//   Chan's pairwise update, and writes mean[c] and var[c] = M2 / M.
// The unit results and their merge order do not depend on which wavefront
// computed a unit, so every grid and split gives the same bits.
struct BnStats {
#ifndef HF_BN_VEC
#define HF_BN_VEC 4
#endif
#ifndef HF_BN_DEPTH
#define HF_BN_DEPTH 2
#endif
  static constexpr uint32_t kVec = HF_BN_VEC;      // float4 per lane per unit
  static constexpr uint32_t kVals = 4 * kVec;      // values per lane per unit
  static constexpr uint32_t kUnit = 64 * kVals;    // 1024 elements by default
  static constexpr uint32_t kDepth = HF_BN_DEPTH;  // units in flight per wavefront
  static constexpr uint32_t lds_words(int) { return 0; }

  struct Regs {
    float v[kVals];  // lane-major: every load instruction is coalesced
  };

  // Loads every lane unconditionally (lanes past the channel's end read the
  // channel's first element, which unit_stats masks out), so the loads of a
  // unit are straight-line code and no value is consumed before its reduction.
  template <bool VEC>
  __device__ static __forceinline__ void load_unit(const BnArgs& a, uint32_t c, uint32_t ubase,
                                                   uint32_t lane, Regs& r) {
    const float* xc = a.x + (size_t)c * a.HW;
    if constexpr (VEC) {
#pragma unroll
      for (uint32_t t = 0; t < kVec; ++t) {
        const uint32_t j = ubase + 4u * (lane + 64u * t);
        const bool ok = j < a.M;
        const uint32_t jj = ok ? j : 0u;
        const uint32_t n = fdiv(jj, a.div_hw);
        const float4 q = *reinterpret_cast<const float4*>(xc + ((size_t)jj + (size_t)n * a.CHWm));
        r.v[4 * t + 0] = q.x;
        r.v[4 * t + 1] = q.y;
        r.v[4 * t + 2] = q.z;
        r.v[4 * t + 3] = q.w;
      }
    } else {
#pragma unroll
      for (uint32_t t = 0; t < kVals; ++t) {
        const uint32_t j = ubase + lane + 64u * t;
        const bool ok = j < a.M;
        const uint32_t jj = ok ? j : 0u;
        const uint32_t n = fdiv(jj, a.div_hw);
        r.v[t] = xc[(size_t)jj + (size_t)n * a.CHWm];
      }
    }
  }

  template <bool VEC>
  __device__ static __forceinline__ bool valid(const BnArgs& a, uint32_t ubase, uint32_t lane,
                                               uint32_t t) {
    const uint32_t j = VEC ? ubase + 4u * (lane + 64u * (t >> 2)) + (t & 3u) : ubase + lane + 64u * t;
    return j < a.M;
  }

  // mean and M2 of one unit held in registers: two passes, fixed-order wave
  // sums.  FULL: the unit has kUnit elements (every unit but a channel's last).
  template <bool VEC, bool FULL>
  __device__ static __forceinline__ void unit_stats(const BnArgs& a, const Regs& r, uint32_t ub,
                                                    uint32_t lane, float& mu, float& m2) {
    const uint32_t cnt = FULL ? kUnit : min(kUnit, a.M - ub);
    float s = 0.f, q = 0.f;
    // lanes past the channel's end hold a copy of another element: masked out
#pragma unroll
    for (uint32_t t = 0; t < kVals; ++t) s += (FULL || valid<VEC>(a, ub, lane, t)) ? r.v[t] : 0.f;
    mu = wave_sum(s) / (float)cnt;
#pragma unroll
    for (uint32_t t = 0; t < kVals; ++t) {
      const float d = (FULL || valid<VEC>(a, ub, lane, t)) ? r.v[t] - mu : 0.f;
      q += d * d;
    }
    m2 = wave_sum(q);
  }

  // Reduces the unit held in `r` (unit k of channel c, global unit index u)
  // and publishes its (mean, M2) with one 8-byte store.
  template <bool VEC, bool FULL>
  __device__ static __forceinline__ void consume(const BnArgs& a, const Regs& r, uint32_t u,
                                                 uint32_t k, uint32_t lane) {
    float mu, m2;
    unit_stats<VEC, FULL>(a, r, k * kUnit, lane, mu, m2);
    if (lane == 0) {
      const uint64_t v = (uint64_t)__builtin_bit_cast(uint32_t, mu) |
                         ((uint64_t)__builtin_bit_cast(uint32_t, m2) << 32);
      __hip_atomic_store(reinterpret_cast<uint64_t*>(a.part) + u, v, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
  }

  // Units [k0, k0 + n) of channel c (global index u0 = c * upc + k0).  kDepth
  // register slots; slot s always holds unit i + s of the current stride, so a
  // unit is requested kDepth - 1 reductions before it is reduced.  The steady
  // loop has no branch: every unit in it is full and every reload exists, which
  // keeps the compiler's count of outstanding loads exact.
  template <bool VEC>
  __device__ static __forceinline__ void segment(const BnArgs& a, uint32_t c, uint32_t k0,
                                                 uint32_t u0, uint32_t n, uint32_t lane) {
    Regs buf[kDepth];
    // unconditional, so that the loop is entered with every slot outstanding in
    // slot order (a segment shorter than kDepth loads its last unit again)
#pragma unroll
    for (uint32_t s = 0; s < kDepth; ++s) load_unit<VEC>(a, c, (k0 + min(s, n - 1u)) * kUnit, lane, buf[s]);
    uint32_t i = 0;
    for (; i + 2u * kDepth <= n; i += kDepth) {
#pragma unroll
      for (uint32_t s = 0; s < kDepth; ++s) {
        consume<VEC, true>(a, buf[s], u0 + i + s, k0 + i + s, lane);
        load_unit<VEC>(a, c, (k0 + i + s + kDepth) * kUnit, lane, buf[s]);
      }
    }
#pragma unroll
    for (uint32_t s = 0; s < kDepth; ++s) {
      if (i + s < n) {
        consume<VEC, false>(a, buf[s], u0 + i + s, k0 + i + s, lane);
        if (i + s + kDepth < n) load_unit<VEC>(a, c, (k0 + i + s + kDepth) * kUnit, lane, buf[s]);
      }
    }
#pragma unroll
    for (uint32_t s = 0; s < kDepth; ++s)
      if (i + kDepth + s < n) consume<VEC, false>(a, buf[s], u0 + i + kDepth + s, k0 + i + kDepth + s, lane);
  }

  // The wavefront's contiguous unit range, one channel segment at a time; at
  // the end of each segment it arrives on the channel's counter, and the last
  // arriver merges the channel.
  template <bool VEC>
  __device__ static void run_range(const BnArgs& a, uint32_t ubeg, uint32_t uend, uint32_t lane) {
    uint32_t c = fdiv(ubeg, a.div_upc);
    uint32_t k0 = ubeg - c * a.upc;
    for (uint32_t u = ubeg; u < uend; ++c, k0 = 0) {
      const uint32_t n = min(uend - u, a.upc - k0);
      segment<VEC>(a, c, k0, u, n, lane);
      uint32_t old = 0;
      if (lane == 0) old = arrive_after_coherent_stores(a.ctr + c, n);
      old = uniform(old);
      if (old + n == a.upc) finish_channel(a, c, lane);
      u += n;
    }
  }

  template <class Bar>
  __device__ static void run(const DevTask& dt, const Part& p, Bar&, uint32_t*) {
    const BnArgs& a = dt.bn;
    const uint32_t lane = lane_id();
    const uint32_t nw = p.nwg * p.nwaves;
    const uint32_t gw = p.wg * p.nwaves + p.wave;
    const uint32_t q = a.total / nw, r = a.total - q * nw;
    const uint32_t ubeg = gw * q + min(gw, r);
    const uint32_t uend = ubeg + q + (gw < r ? 1u : 0u);
    if (ubeg >= uend) return;
    if (a.vec)
      run_range<true>(a, ubeg, uend, lane);
    else
      run_range<false>(a, ubeg, uend, lane);
  }

  // Chan et al. pairwise update of (n, mean, M2) with (nb, mb, m2b), in double.
  __device__ static __forceinline__ void chan(double& n, double& m, double& m2, double nb, double mb,
                                              double m2b) {
    const double nab = n + nb;
    const double d = mb - m;
    m = m + d * (nb / nab);
    m2 = m2 + m2b + d * d * (n * nb / nab);
    n = nab;
  }

  // Merge the units of channel c: each lane merges units lane, lane+64, ... in
  // order, then the 64 lane results are merged by a fixed butterfly.
  __device__ static void finish_channel(const BnArgs& a, uint32_t c, uint32_t lane) {
    const uint32_t base = 2u * c * a.upc;
    double n = 0.0, m = 0.0, m2 = 0.0;
    for (uint32_t k = lane; k < a.upc; k += 64u) {
      const double nk = (double)min(kUnit, a.M - k * kUnit);
      const double mk = (double)__builtin_bit_cast(float, load_agent(a.part + base + 2u * k));
      const double m2k = (double)__builtin_bit_cast(float, load_agent(a.part + base + 2u * k + 1u));
      chan(n, m, m2, nk, mk, m2k);
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double nb = __shfl_xor(n, off, kWave);
      const double mb = __shfl_xor(m, off, kWave);
      const double m2b = __shfl_xor(m2, off, kWave);
      if (nb > 0.0) {
        if (n > 0.0) {
          // the lower lane of the pair is always the left operand
          if ((lane & (uint32_t)off) == 0u) {
            chan(n, m, m2, nb, mb, m2b);
          } else {
            double nl = nb, ml = mb, m2l = m2b;
            chan(nl, ml, m2l, n, m, m2);
            n = nl;
            m = ml;
            m2 = m2l;
          }
        } else {
          n = nb;
          m = mb;
          m2 = m2b;
        }
      }
    }
    // leave the scratch zero-filled, as every kernel of the library does
    for (uint32_t k = lane; k < a.upc; k += 64u) {
      store_agent(a.part + base + 2u * k, 0u);
      store_agent(a.part + base + 2u * k + 1u, 0u);
    }
    if (lane == 0) {
      a.mean[c] = (float)m;
      a.var[c] = (float)(m2 / (double)a.M);
      store_agent(a.ctr + c, 0u);  // leave the counter zero for the next launch
    }
  }
};

// ================================================================== int_mix
// Integer mixing loop standing in for the compute-bound hash kernels: per element
// R rounds of  x ^= x<<13; x ^= x>>17; x ^= x<<5; x = x*2654435761 + r  (mod 2^32).
//
// A lane's grid-stride walk goes in steps of up to four uint4 vectors (sixteen
// independent chains): four while at least four remain, then one step of the
// remaining one to three.  The vector-memory counter retires in order, so the
// wait for a step's loads also waits for the previous step's stores: each step
// exposes one load and one store latency, and four vectors per step divide the
// number of steps, and of exposed latencies, by four without computing any
// vector twice.
struct IntMix {
  static constexpr uint32_t lds_words(int) { return 0; }

  __device__ static __forceinline__ uint32_t round1(uint32_t x, uint32_t r) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x * 2654435761u + r;
  }

  // vectors i, i + stride, ..., i + (K-1)*stride, all in range
  template <uint32_t K>
  __device__ static __forceinline__ void step(const uint4* in4, uint4* out4, uint32_t i, uint32_t stride,
                                              uint32_t R) {
    uint4 v[K];
#pragma unroll
    for (uint32_t k = 0; k < K; ++k) v[k] = in4[i + k * stride];
    for (uint32_t r = 0; r < R; ++r) {
#pragma unroll
      for (uint32_t k = 0; k < K; ++k) {
        v[k].x = round1(v[k].x, r);
        v[k].y = round1(v[k].y, r);
        v[k].z = round1(v[k].z, r);
        v[k].w = round1(v[k].w, r);
      }
    }
#pragma unroll
    for (uint32_t k = 0; k < K; ++k) out4[i + k * stride] = v[k];
  }

  template <class Bar>
  __device__ static void run(const DevTask& dt, const Part& p, Bar&, uint32_t*) {
    const MixArgs& a = dt.mix;
    const uint32_t gl = p.wg * p.nlanes + p.lane;
    const uint32_t stride = p.nwg * p.nlanes;
    const uint32_t R = (uint32_t)a.rounds;
    const uint4* in4 = reinterpret_cast<const uint4*>(a.in);
    uint4* out4 = reinterpret_cast<uint4*>(a.out);
    if (gl < a.n4) {
      // vectors left for this lane, i = gl, gl + stride, ...
      uint32_t left = (a.n4 - gl + stride - 1u) / stride;
      uint32_t i = gl;
      for (; left >= 4u; left -= 4u, i += 4u * stride) step<4>(in4, out4, i, stride, R);
      if (left == 3u) step<3>(in4, out4, i, stride, R);
      else if (left == 2u) step<2>(in4, out4, i, stride, R);
      else if (left == 1u) step<1>(in4, out4, i, stride, R);
    }
    for (uint32_t i = 4u * a.n4 + gl; i < a.n; i += stride) {
      uint32_t x = a.in[i];
      for (uint32_t r = 0; r < R; ++r) x = round1(x, r);
      a.out[i] = x;
    }
  }
};

// ================================================================== lds_hist
// Histogram kernel of Sec. II-C: clear shared-memory bins, count with shared-
// memory atomics, merge the bins into the global counts.  The interval keeps
// kCopies copies of the 256 bins in LDS, interleaved so that bin b of copy k is
// word b*kCopies + k, and lane l counts into copy l % kCopies: lanes of one
// instruction that see the same (frequent) value hit different words in
// different banks instead of serialising on one address.  The interval's
// barriers separate clearing, counting and merging.  Workgroups add their bins
// into an agent-scope accumulator; the last workgroup to arrive moves the
// totals to the output with atomic exchanges, which also re-zero it.
#ifndef HF_HIST_COPIES
#define HF_HIST_COPIES 16
#endif
struct LdsHist {
  static constexpr uint32_t kCopies = HF_HIST_COPIES;
  static constexpr uint32_t lds_words(int) { return 256u * kCopies; }

  __device__ static __forceinline__ void count_byte(uint32_t* mine, uint32_t b) {
    __hip_atomic_fetch_add(mine + b * kCopies, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __device__ static __forceinline__ void count_word(uint32_t* mine, uint32_t w) {
    count_byte(mine, w & 0xFFu);
    count_byte(mine, (w >> 8) & 0xFFu);
    count_byte(mine, (w >> 16) & 0xFFu);
    count_byte(mine, w >> 24);
  }
  __device__ static __forceinline__ void count_vec(uint32_t* mine, const uint4& q) {
    count_word(mine, q.x);
    count_word(mine, q.y);
    count_word(mine, q.z);
    count_word(mine, q.w);
  }

  template <class Bar>
  __device__ static void run(const DevTask& dt, const Part& p, Bar& bar, uint32_t* lds) {
    const HistArgs& a = dt.hist;
    const uint32_t lane = lane_id();
    for (uint32_t i = p.lane; i < 256u * kCopies; i += p.nlanes) lds[i] = 0u;
    bar.sync();

    uint32_t* mine = lds + (lane % kCopies);
    const uint32_t gl = p.wg * p.nlanes + p.lane;
    const uint32_t stride = p.nwg * p.nlanes;
    const uint4* v16 = reinterpret_cast<const uint4*>(a.in + a.head);
    // Two vectors per step, and the next step's two requested before this
    // step's atomics, so up to four 16-byte loads per lane are in flight:
    // inside a fused kernel the interval may have only a few wavefronts per
    // CU, and their loads alone must keep the input streaming.  The loop has
    // no stores, so each wait covers only the loads it needs.
    if (gl < a.n16) {
      const uint32_t last = a.n16 - 1u;
      uint4 q0 = v16[gl], q1 = v16[min(gl + stride, last)];
      uint32_t i = gl;
      for (; i + stride < a.n16; i += 2u * stride) {
        const uint4 p0 = v16[min(i + 2u * stride, last)], p1 = v16[min(i + 3u * stride, last)];
        count_vec(mine, q0);
        count_vec(mine, q1);
        q0 = p0;
        q1 = p1;
      }
      if (i < a.n16) count_vec(mine, q0);  // the last vector of an odd count
    }
    if (gl < a.head) count_byte(mine, a.in[gl]);
    for (uint32_t i = a.tail_start + gl; i < a.n; i += stride) count_byte(mine, a.in[i]);
    bar.sync();

    for (uint32_t b = p.lane; b < 256u; b += p.nlanes) {
      uint32_t s = 0;
#pragma unroll
      for (uint32_t k = 0; k < kCopies; ++k) s += lds[b * kCopies + k];
      if (s) __hip_atomic_fetch_add(a.acc + b, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    wait_vmem();  // this wave's merge atomics have completed ...
    bar.sync();   // ... before wave 0 of the interval counts the workgroup in

    if (p.wave == 0) {
      uint32_t old = 0;
      if (lane == 0) old = arrive_after_coherent_stores(a.ctr);
      old = uniform(old);
      if (old == p.nwg - 1u) {
        for (uint32_t b = lane; b < 256u; b += 64u)
          a.out[b] = __hip_atomic_exchange(a.acc + b, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (lane == 0) store_agent(a.ctr, 0u);
      }
    }
  }
};

// ================================================================== im2col
// Im2Col (Sec. IV-A): out[n][(c*kh + i)*kw + j][oh*Wo + ow] = x[n][c][oh*s-p+i][ow*s-p+j],
// zero outside the image.  A unit is one output plane (n, c*kh*kw + kk): Ho*Wo
// contiguous floats, written front to back (float4 when Wo % 4 == 0), so every
// store instruction covers whole aligned cache lines.  Kernel offsets kk are the
// fastest-varying unit index, so the kh*kw planes that read one input plane run
// next to each other and find it in cache.
//
// Row path (3x3 kernel, stride 1, pad 1, W % 4 == 0, 16-byte aligned input and
// output): with stride 1, output plane (i, j) of a channel is the channel
// shifted by i - 1 rows and j - 1 columns with zero fill, so one output row of
// all nine planes is made from three input rows.  Each row is cut into chunks
// of 64 columns; a unit is four consecutive chunks of one channel (four rows
// when W <= 64), one chunk per 16-lane DPP row of the wavefront.  Lane 16q + c
// loads columns 4c..4c+3 of input rows oh-1, oh, oh+1 (one aligned float4 each)
// and writes columns 4c..4c+3 of row oh of all nine planes: a column shift
// takes the neighbouring lane's edge element with a DPP row shift, and the
// first and last lane of a chunk take the element beyond it with one extra
// dword load per row (zero at the image's edge).  Every input element is thus
// loaded by one unit only (plus the rows shared with the neighbouring quads,
// which the same wavefront reads next), instead of once per plane.  All
// accesses go through buffer resources over one plane: rows and columns
// outside the image load zero, which is exactly the zero padding, and lanes
// past the plane's end store nothing, so the loop has no branch around a
// memory access.  Each store instruction writes four chunks of one plane.
// kStep units per step: their loads are issued together, so the wait for them
// comes once per kStep units.
struct Im2col {
  static constexpr uint32_t lds_words(int) { return 0; }
  static constexpr uint32_t kStep = 3;

  __device__ static void run_rows(const Im2colArgs& a, const Part& p, uint32_t lane) {
    const uint32_t nw = p.nwg * p.nwaves;
    const uint32_t gw = p.wg * p.nwaves + p.wave;
    const uint32_t q = a.row_units / nw, r = a.row_units - q * nw;
    const uint32_t ubeg = gw * q + min(gw, r);
    const uint32_t uend = ubeg + q + (gw < r ? 1u : 0u);
    const uint32_t W = a.W, H = a.H, HW = H * W, pbytes = 4u * HW;
    const uint32_t qrow = lane >> 4, c4 = lane & 15u;
    // The channel and output position of unit u in this lane (shared by both
    // phases; the store phase recomputes it rather than keep registers live).
    auto where = [&](uint32_t u, uint32_t& nc, uint32_t& oh, uint32_t& col) {
      nc = fdiv(u, a.div_nq);
      const uint32_t cid = 4u * (u - nc * a.nq) + qrow;  // chunk of this DPP row
      oh = fdiv(cid, a.div_nch);
      col = 64u * (cid - oh * a.nch) + 4u * c4;
    };
    for (uint32_t u0 = ubeg; u0 < uend; u0 += kStep) {
      float4 x[kStep][3];
      float edge[kStep][3];
#pragma unroll
      for (uint32_t k = 0; k < kStep; ++k) {
        uint32_t nc, oh, col;
        where(min(u0 + k, uend - 1u), nc, oh, col);  // a unit past the range repeats the last one
        const __amdgpu_buffer_rsrc_t src = buffer_rsrc(a.x + (size_t)nc * HW, pbytes);
        uint32_t ec = kOutOfRange;  // the column left or right of the lane's four, if another lane's
        if (c4 == 0u && col > 0u) ec = col - 1u;
        if (c4 == 15u && col + 4u < W) ec = col + 4u;
#pragma unroll
        for (uint32_t i = 0; i < 3u; ++i) {
          const uint32_t ih = oh + i - 1u;  // wraps past H above the image
          const bool rowok = oh < H && col < W && ih < H;
          x[k][i] = buffer_load4(src, rowok ? 4u * (ih * W + col) : kOutOfRange);
          edge[k][i] = buffer_load1(src, rowok && ec != kOutOfRange ? 4u * (ih * W + ec) : kOutOfRange);
        }
      }
#pragma unroll
      for (uint32_t k = 0; k < kStep; ++k) {
        uint32_t nc, oh, col;
        where(min(u0 + k, uend - 1u), nc, oh, col);
        const uint32_t at = (oh < H && col < W && u0 + k < uend) ? 4u * (oh * W + col) : kOutOfRange;
#pragma unroll
        for (uint32_t i = 0; i < 3u; ++i) {
          const float4 v = x[k][i];
          // every lane takes part in the shifts (row_shr:1 / row_shl:1)
          const float sl = dpp_f32<0x111>(v.w), sr = dpp_f32<0x101>(v.x);
          const float lft = c4 == 0u ? edge[k][i] : sl;
          const float rgt = c4 == 15u ? edge[k][i] : sr;
          const float* base = a.out + ((size_t)nc * 9u + 3u * i) * HW;  // plane (i, 0) of channel nc
          buffer_store4_nt(buffer_rsrc(base, pbytes), at, lft, v.x, v.y, v.z);
          buffer_store4_nt(buffer_rsrc(base + HW, pbytes), at, v.x, v.y, v.z, v.w);
          buffer_store4_nt(buffer_rsrc(base + 2u * (size_t)HW, pbytes), at, v.y, v.z, v.w, rgt);
        }
      }
    }
  }

  template <class Bar>
  __device__ static void run(const DevTask& dt, const Part& p, Bar&, uint32_t*) {
    const Im2colArgs& a = dt.im2col;
    const uint32_t lane = lane_id();
    if (a.row3) {
      run_rows(a, p, lane);
      return;
    }
    const uint32_t nw = p.nwg * p.nwaves;
    const uint32_t HW = a.H * a.W;
    const uint32_t plane = a.Ho * a.Wo;
    for (uint32_t u = p.wg * p.nwaves + p.wave; u < a.units; u += nw) {
      const uint32_t nc = fdiv(u, a.div_kk);  // n*C + c
      const uint32_t kk = u - nc * a.KK;
      const uint32_t i = fdiv(kk, a.div_kw);
      const uint32_t j = kk - i * a.kw;
      const float* img = a.x + nc * HW;
      float* dst = a.out + u * plane;  // plane u = (n, c*KK + kk)
      for (uint32_t t = lane; t < a.lanes_per_unit; t += 64u) {
        const uint32_t oh = fdiv(t, a.div_row);
        const uint32_t col = t - oh * a.div_row.d;  // ow4 (vector) or ow (scalar)
        const int ih = (int)(oh * a.s + i) - (int)a.p;
        const bool rowok = ih >= 0 && ih < (int)a.H;
        const float* src = img + (rowok ? ih : 0) * (int)a.W;
        if (a.vec) {
          float v[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int iw = (int)((4u * col + e) * a.s + j) - (int)a.p;
            v[e] = (rowok && iw >= 0 && iw < (int)a.W) ? src[iw] : 0.f;
          }
          store_nt4(dst + oh * a.Wo + 4u * col, v[0], v[1], v[2], v[3]);
        } else {
          const int iw = (int)(col * a.s + j) - (int)a.p;
          __builtin_nontemporal_store((rowok && iw >= 0 && iw < (int)a.W) ? src[iw] : 0.f,
                                      dst + oh * a.Wo + col);
        }
      }
    }
  }
};

// ================================================================== upsample
// Bilinear upsampling (Sec. IV-A) by an integer factor s with half-pixel
// centres: t = max(0, (o + 0.5)/s - 0.5), i0 = floor(t), i1 = min(i0+1, L-1),
// l = t - i0; lerp along x on rows y0 and y1, then along y, as a + l*(b - a).
// Units are output rows (several short rows per unit), written front to back.
// For s = 2 the four outputs 4c..4c+3 of a float4 read the four consecutive
// inputs 2c-1..2c+2 (clamped) with weights 0.75, 0.25, 0.75, 0.25, which are
// exactly the values the general formula produces, so both paths give the same
// bits; the fast path just skips the per-output coordinate arithmetic.
struct Upsample {
  static constexpr uint32_t lds_words(int) { return 0; }

  __device__ static __forceinline__ void coord(uint32_t o, float inv_s, uint32_t L, uint32_t& i0,
                                               uint32_t& i1, float& l) {
    const float t = fmaxf(((float)o + 0.5f) * inv_s - 0.5f, 0.f);
    uint32_t a = (uint32_t)t;
    a = min(a, L - 1u);
    i0 = a;
    i1 = min(a + 1u, L - 1u);
    l = t - (float)a;
  }

  __device__ static __forceinline__ float lerp(float a, float b, float l) { return a + l * (b - a); }

  // Row path (scale 2, W even, 8-byte aligned input, 16-byte aligned output).
  // Each output row is cut into chunks that read 32 input columns and write 64
  // output columns; a unit is four consecutive chunks of one plane (four output
  // rows when W <= 32), one chunk per 16-lane DPP row.  Lane 16q + c reads input
  // columns 2c, 2c+1 of the output row's two source rows (one float2 each) and
  // writes output columns 4c..4c+3 (one float4), so every store instruction
  // covers whole contiguous lines.  Column 2c-1 comes from the lane before and
  // column 2c+2 from the lane after by DPP row shifts, from one extra dword load
  // at a chunk's first and last lane, and from the lane itself at the image's
  // edges (the coordinate clamp).  The four outputs are the general scale-2
  // path's expressions of the same inputs, so both paths give the same bits.
  // Buffer accesses keep the loop free of branches around memory instructions;
  // kStep units per step.
  static constexpr uint32_t kStep = 4;

  __device__ static void run_rows(const UpArgs& a, const Part& p, uint32_t lane) {
    const uint32_t nw = p.nwg * p.nwaves;
    const uint32_t gw = p.wg * p.nwaves + p.wave;
    const uint32_t q = a.row_units / nw, r = a.row_units - q * nw;
    const uint32_t ubeg = gw * q + min(gw, r);
    const uint32_t uend = ubeg + q + (gw < r ? 1u : 0u);
    const uint32_t W = a.W, HW = a.H * a.W, OHW = a.Ho * a.Wo;
    const uint32_t qrow = lane >> 4, c4 = lane & 15u;
    auto where = [&](uint32_t u, uint32_t& plane, uint32_t& oy, uint32_t& col) {
      plane = fdiv(u, a.div_nq);
      const uint32_t cid = 4u * (u - plane * a.nq) + qrow;  // chunk of this DPP row
      oy = fdiv(cid, a.div_nch);
      col = 32u * (cid - oy * a.nch) + 2u * c4;  // first input column of this lane
    };
    for (uint32_t u0 = ubeg; u0 < uend; u0 += kStep) {
      float2 x0[kStep], x1[kStep];
      float e0[kStep], e1[kStep];
#pragma unroll
      for (uint32_t k = 0; k < kStep; ++k) {
        uint32_t plane, oy, col;
        where(min(u0 + k, uend - 1u), plane, oy, col);  // a unit past the range repeats the last one
        uint32_t y0, y1;
        float ly;
        coord(min(oy, a.Ho - 1u), a.inv_s, a.H, y0, y1, ly);
        const bool ok = oy < a.Ho && col < W;
        const __amdgpu_buffer_rsrc_t src = buffer_rsrc(a.x + (size_t)plane * HW, 4u * HW);
        uint32_t eo = kOutOfRange;  // the column left or right of the lane's two, if another lane's
        if (c4 == 0u && col > 0u) eo = col - 1u;
        if (c4 == 15u && col + 2u < W) eo = col + 2u;
        x0[k] = buffer_load2(src, ok ? 4u * (y0 * W + col) : kOutOfRange);
        x1[k] = buffer_load2(src, ok ? 4u * (y1 * W + col) : kOutOfRange);
        e0[k] = buffer_load1(src, ok && eo != kOutOfRange ? 4u * (y0 * W + eo) : kOutOfRange);
        e1[k] = buffer_load1(src, ok && eo != kOutOfRange ? 4u * (y1 * W + eo) : kOutOfRange);
      }
#pragma unroll
      for (uint32_t k = 0; k < kStep; ++k) {
        uint32_t plane, oy, col;
        where(min(u0 + k, uend - 1u), plane, oy, col);
        uint32_t y0, y1;
        float ly;
        coord(min(oy, a.Ho - 1u), a.inv_s, a.H, y0, y1, ly);
        // every lane takes part in the shifts (row_shr:1 / row_shl:1)
        const float l0 = dpp_f32<0x111>(x0[k].y), r0 = dpp_f32<0x101>(x0[k].x);
        const float l1 = dpp_f32<0x111>(x1[k].y), r1 = dpp_f32<0x101>(x1[k].x);
        const bool first = col == 0u, last = col + 2u >= W;
        const float p0 = first ? x0[k].x : (c4 == 0u ? e0[k] : l0), p1 = x0[k].x, p2 = x0[k].y;
        const float p3 = last ? x0[k].y : (c4 == 15u ? e0[k] : r0);
        const float q0 = first ? x1[k].x : (c4 == 0u ? e1[k] : l1), q1 = x1[k].x, q2 = x1[k].y;
        const float q3 = last ? x1[k].y : (c4 == 15u ? e1[k] : r1);
        const uint32_t at = (oy < a.Ho && col < W && u0 + k < uend) ? 4u * (oy * a.Wo + 2u * col) : kOutOfRange;
        buffer_store4_nt(buffer_rsrc(a.out + (size_t)plane * OHW, 4u * OHW), at,
                         lerp(lerp(p0, p1, 0.75f), lerp(q0, q1, 0.75f), ly),
                         lerp(lerp(p1, p2, 0.25f), lerp(q1, q2, 0.25f), ly),
                         lerp(lerp(p1, p2, 0.75f), lerp(q1, q2, 0.75f), ly),
                         lerp(lerp(p2, p3, 0.25f), lerp(q2, q3, 0.25f), ly));
      }
    }
  }

  __device__ static __forceinline__ float sample(const float* r0, const float* r1, float ly, uint32_t W,
                                                 uint32_t ox, float inv_s) {
    uint32_t x0, x1;
    float lx;
    coord(ox, inv_s, W, x0, x1, lx);
    const float top = lerp(r0[x0], r0[x1], lx);
    const float bot = lerp(r1[x0], r1[x1], lx);
    return lerp(top, bot, ly);
  }

  template <class Bar>
  __device__ static void run(const DevTask& dt, const Part& p, Bar&, uint32_t*) {
    const UpArgs& a = dt.up;
    const uint32_t lane = lane_id();
    if (a.row2) {
      run_rows(a, p, lane);
      return;
    }
    const uint32_t nw = p.nwg * p.nwaves;
    const uint32_t HW = a.H * a.W;
    const bool x2 = a.vec && a.Wo == 2u * a.W;  // scale 2 with float4 stores
    for (uint32_t u = p.wg * p.nwaves + p.wave; u < a.units; u += nw) {
      const uint32_t row0 = u * a.rows_per_unit;
      for (uint32_t t = lane; t < a.lanes_per_unit; t += 64u) {
        const uint32_t rr = fdiv(t, a.div_row);
        const uint32_t col = t - rr * a.div_row.d;
        const uint32_t row = row0 + rr;
        if (row >= a.rows) continue;
        const uint32_t plane = fdiv(row, a.div_ho);
        const uint32_t oy = row - plane * a.Ho;
        uint32_t y0, y1;
        float ly;
        coord(oy, a.inv_s, a.H, y0, y1, ly);
        const float* img = a.x + plane * HW;
        const float* r0 = img + y0 * a.W;
        const float* r1 = img + y1 * a.W;
        float* dst = a.out + row * a.Wo;
        if (x2) {
          const uint32_t xm = col > 0u ? 2u * col - 1u : 0u;
          const uint32_t xp = min(2u * col + 2u, a.W - 1u);
          const float p0 = r0[xm], p1 = r0[2u * col], p2 = r0[2u * col + 1u], p3 = r0[xp];
          const float q0 = r1[xm], q1 = r1[2u * col], q2 = r1[2u * col + 1u], q3 = r1[xp];
          store_nt4(dst + 4u * col, lerp(lerp(p0, p1, 0.75f), lerp(q0, q1, 0.75f), ly),
                    lerp(lerp(p1, p2, 0.25f), lerp(q1, q2, 0.25f), ly),
                    lerp(lerp(p1, p2, 0.75f), lerp(q1, q2, 0.75f), ly),
                    lerp(lerp(p2, p3, 0.25f), lerp(q2, q3, 0.25f), ly));
        } else if (a.vec) {
          float v[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = sample(r0, r1, ly, a.W, 4u * col + e, a.inv_s);
          store_nt4(dst + 4u * col, v[0], v[1], v[2], v[3]);
        } else {
          __builtin_nontemporal_store(sample(r0, r1, ly, a.W, col, a.inv_s), dst + col);
        }
      }
    }
  }
};

// =================================================================== maxpool
// 2-D max pooling (Sec. IV-A "Maxpool").  A unit is kUnit consecutive outputs
// of the flattened [N][C][Ho][Wo] output, kPer per lane (lane l takes outputs
// l, l + 64, ...).  Each wavefront owns a contiguous, balanced range of units,
// so the input rows shared by vertically adjacent windows are re-read from the
// caches of the same CU.
//
// Window coordinates are clamped into the image instead of being skipped: with
// pad < kh, kw a clamped row or column is always inside the window, and it is
// met in the scan before (low side) or after (high side) the real copy of the
// same element, never between two other elements, so under the scan rule (a
// later element wins only if greater or NaN) the winner and its index are
// exactly those of the unclamped scan.  All loads are therefore unconditional.
//
// Row path (3x3 window, stride 2, pad 1, W % 8 == 0, 16-byte aligned
// buffers): each output row is cut into chunks that read 128 input columns
// and write 64 outputs; a unit is four consecutive chunks of one plane (four
// output rows when W <= 128), one per 16-lane DPP row of the wavefront.  Lane
// 16q + c computes outputs 4c..4c+3 of its chunk, whose windows span input
// columns 8c-1 .. 8c+7 (chunk-relative) of three input rows: columns 8c..8c+7
// are two aligned float4 per row, and column 8c-1 is the left neighbour lane's
// last element, taken with a DPP row shift, or, at a chunk's first lane, one
// extra dword load (at the image's first column the column clamps to 0, as in
// the general path).  Rows clamp the same way.  Each window is scanned in the
// general path's order, and values and indices are stored as float4 / int4
// through buffer resources (lanes past the plane's end store nothing), four
// chunks per store instruction.
struct Maxpool {
  static constexpr int kSoloWaves = 8;  // 45 VGPRs, but 106 SGPRs would allow only 7
  static constexpr uint32_t kPer = 2;
  static constexpr uint32_t kUnit = 64 * kPer;
  static constexpr uint32_t lds_words(int) { return 0; }

  __device__ static __forceinline__ void take(float v, int32_t e, bool first, float& best, int32_t& at) {
    if (first || v > best || __builtin_isnan(v)) {
      best = v;
      at = e;
    }
  }

  __device__ static void run_rows(const PoolArgs& a, const Part& p, uint32_t lane) {
    const uint32_t nw = p.nwg * p.nwaves;
    const uint32_t gw = p.wg * p.nwaves + p.wave;
    const uint32_t q = a.row_units / nw, r = a.row_units - q * nw;
    const uint32_t ubeg = gw * q + min(gw, r);
    const uint32_t uend = ubeg + q + (gw < r ? 1u : 0u);
    const uint32_t W = a.W, HW = a.H * a.W, OHW = a.Ho * a.Wo;
    const uint32_t qrow = lane >> 4, c4 = lane & 15u;
    for (uint32_t u = ubeg; u < uend; ++u) {
      const uint32_t plane = fdiv(u, a.div_nq);
      const uint32_t cid = 4u * (u - plane * a.nq) + qrow;  // chunk of this DPP row
      const uint32_t oh = fdiv(cid, a.div_nch);
      const uint32_t col = 128u * (cid - oh * a.nch) + 8u * c4;  // first input column of this lane
      const bool ok = oh < a.Ho && col < W;
      const uint32_t ohc = min(oh, a.Ho - 1u);
      const __amdgpu_buffer_rsrc_t src = buffer_rsrc(a.x + (size_t)plane * HW, 4u * HW);
      float4 A[3], B[3];
      float E[3];
#pragma unroll
      for (uint32_t i = 0; i < 3; ++i) {
        const uint32_t h = (uint32_t)clampi((int32_t)(2u * ohc + i) - 1, (int32_t)a.H - 1);
        A[i] = buffer_load4(src, ok ? 4u * (h * W + col) : kOutOfRange);
        B[i] = buffer_load4(src, ok ? 4u * (h * W + col + 4u) : kOutOfRange);
        // column col - 1 of the first lane of a chunk that is not the image's first
        E[i] = buffer_load1(src, ok && c4 == 0u && col > 0u ? 4u * (h * W + col - 1u) : kOutOfRange);
      }
      float best[4];
      int32_t at[4];
#pragma unroll
      for (uint32_t i = 0; i < 3; ++i) {
        const int32_t h = clampi((int32_t)(2u * ohc + i) - 1, (int32_t)a.H - 1);
        const float lft = dpp_f32<0x111>(B[i].w);  // column col - 1 from the lane before
        const int32_t e0 = h * (int32_t)W + (int32_t)col;
        // at the image's first column the window's clamped column is column 0
        const float L = col == 0u ? A[i].x : (c4 == 0u ? E[i] : lft);
        const int32_t eL = col == 0u ? e0 : e0 - 1;
        const bool f = i == 0;
        take(L, eL, f, best[0], at[0]);
        take(A[i].x, e0, false, best[0], at[0]);
        take(A[i].y, e0 + 1, false, best[0], at[0]);
        take(A[i].y, e0 + 1, f, best[1], at[1]);
        take(A[i].z, e0 + 2, false, best[1], at[1]);
        take(A[i].w, e0 + 3, false, best[1], at[1]);
        take(A[i].w, e0 + 3, f, best[2], at[2]);
        take(B[i].x, e0 + 4, false, best[2], at[2]);
        take(B[i].y, e0 + 5, false, best[2], at[2]);
        take(B[i].y, e0 + 5, f, best[3], at[3]);
        take(B[i].z, e0 + 6, false, best[3], at[3]);
        take(B[i].w, e0 + 7, false, best[3], at[3]);
      }
      const uint32_t o = ok ? 4u * (oh * a.Wo + col / 2u) : kOutOfRange;
      buffer_store4_nt(buffer_rsrc(a.out + (size_t)plane * OHW, 4u * OHW), o, best[0], best[1], best[2], best[3]);
      if (a.idx)
        buffer_store4_nt(buffer_rsrc(a.idx + (size_t)plane * OHW, 4u * OHW), o, __builtin_bit_cast(float, at[0]),
                         __builtin_bit_cast(float, at[1]), __builtin_bit_cast(float, at[2]),
                         __builtin_bit_cast(float, at[3]));
    }
  }

  __device__ static __forceinline__ int32_t clampi(int32_t v, int32_t hi) { return min(max(v, 0), hi); }

  template <int KH, int KW>
  __device__ static __forceinline__ void window(const PoolArgs& a, const float* img, int32_t h0, int32_t w0,
                                                uint32_t kh, uint32_t kw, float& best, int32_t& at) {
    const int32_t Hm = (int32_t)a.H - 1, Wm = (int32_t)a.W - 1, W = (int32_t)a.W;
    const uint32_t nh = KH > 0 ? (uint32_t)KH : kh, nw = KW > 0 ? (uint32_t)KW : kw;
    best = 0.f;
    at = -1;
#pragma unroll
    for (uint32_t i = 0; i < nh; ++i) {
      const int32_t h = clampi(h0 + (int32_t)i, Hm);
#pragma unroll
      for (uint32_t j = 0; j < nw; ++j) {
        const int32_t e = h * W + clampi(w0 + (int32_t)j, Wm);
        const float v = img[e];
        if ((i == 0 && j == 0) || v > best || __builtin_isnan(v)) {
          best = v;
          at = e;
        }
      }
    }
  }

  template <int KH, int KW>
  __device__ static __forceinline__ void units(const PoolArgs& a, uint32_t ubeg, uint32_t uend, uint32_t lane) {
    const uint32_t plane_sz = a.H * a.W;
    for (uint32_t u = ubeg; u < uend; ++u) {
#pragma unroll
      for (uint32_t t = 0; t < kPer; ++t) {
        const uint32_t o = u * kUnit + lane + 64u * t;
        const uint32_t oc = min(o, a.total - 1u);  // lanes past the end redo the last output
        const uint32_t plane = fdiv(oc, a.div_plane);
        const uint32_t r = oc - plane * a.div_plane.d;
        const uint32_t oh = fdiv(r, a.div_wo);
        const uint32_t ow = r - oh * a.Wo;
        const float* img = a.x + (size_t)plane * plane_sz;
        float best;
        int32_t at;
        window<KH, KW>(a, img, (int32_t)(oh * a.s) - (int32_t)a.p, (int32_t)(ow * a.s) - (int32_t)a.p, a.kh,
                       a.kw, best, at);
        if (o < a.total) {
          __builtin_nontemporal_store(best, a.out + o);
          if (a.idx) __builtin_nontemporal_store(at, a.idx + o);
        }
      }
    }
  }

  template <class Bar>
  __device__ static void run(const DevTask& dt, const Part& p, Bar&, uint32_t*) {
    const PoolArgs& a = dt.pool;
    const uint32_t lane = lane_id();
    if (a.row3) {
      run_rows(a, p, lane);
      return;
    }
    const uint32_t nw = p.nwg * p.nwaves;
    const uint32_t gw = p.wg * p.nwaves + p.wave;
    const uint32_t q = a.units / nw, r = a.units - q * nw;
    const uint32_t ubeg = gw * q + min(gw, r);
    const uint32_t uend = ubeg + q + (gw < r ? 1u : 0u);
    if (ubeg >= uend) return;
    if (a.kh == 3 && a.kw == 3)
      units<3, 3>(a, ubeg, uend, lane);
    else if (a.kh == 2 && a.kw == 2)
      units<2, 2>(a, ubeg, uend, lane);
    else
      units<0, 0>(a, ubeg, uend, lane);
  }
};

}  // namespace hf

#include "hf_hash.hpp"
