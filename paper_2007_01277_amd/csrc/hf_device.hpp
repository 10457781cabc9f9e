// hf_device.hpp -- device-side building blocks of the fused kernels (gfx950).
//
//  * Part         : the prologue variables of a fused kernel (Sec. III-A, Generate
//                   algorithm): the thread id and size of the interval a lane
//                   belongs to, here at wavefront granularity.
//  * WGBarrier    : the original kernels' workgroup barrier (s_barrier).
//  * PartBarrier  : the partition-scoped barrier that replaces it inside a fused
//                   kernel (Sec. III-A "Replace Synchronization Barriers").  CDNA
//                   has no counted named barriers, so arrivals are counted in LDS:
//                   one arrival per wavefront, waiters sleep between polls.
//  * wave_sum     : a fixed-order wavefront reduction built from DPP row moves
//                   and lane reads, so the same inputs give the same bits in a
//                   solo and in a fused kernel, whatever the partition size.
//  * FastDiv      : division by a run-time constant as multiply-high + shift.
//  * FastMod      : remainder by a run-time constant for any 32-bit numerator.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hf {

constexpr int kWave = 64;

// Interval of the fused workgroup that the calling lane belongs to.
struct Part {
  uint32_t lane;    // lane index inside the interval, 0 .. nlanes-1
  uint32_t nlanes;  // lanes in the interval (multiple of 64)
  uint32_t wave;    // wavefront index inside the interval (wave-uniform)
  uint32_t nwaves;  // wavefronts in the interval
  uint32_t wg;      // workgroup index
  uint32_t nwg;     // workgroups in the launch
};

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// ----------------------------------------------------------------- streaming stores
typedef float f32x4 __attribute__((ext_vector_type(4)));

// 16-byte store with the non-temporal hint: output that is written once and
// not read back by the kernel should not displace inputs from the caches.
__device__ __forceinline__ void store_nt4(float* p, float a, float b, float c, float d) {
  f32x4 v = {a, b, c, d};
  __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(p));
}

// ----------------------------------------------------------------- buffer accesses
// A raw buffer resource (stride 0) over `bytes` bytes from `base`: every access
// through it is range-checked by the hardware, a load whose offset is out of
// range returns zero and a store whose offset is out of range is dropped.
// Zero padding and ragged edges then need no branch around a memory
// instruction: an invalid lane gets the offset kOutOfRange.  With no branches,
// the compiler counts outstanding loads exactly and waits only for the one a
// use needs (a load under a branch makes it wait for every older access).
// `bytes` must be below 2^31 and the resource must lie inside the allocation.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr uint32_t kOutOfRange = 0x80000000u;
constexpr int kAuxNT = 2;  // cache policy bits of a non-temporal access

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
// (whole vectors are bit-cast: a bit cast of one element of a vector value
// reads element 0 in this compiler)
__device__ __forceinline__ float4 buffer_load4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  const f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 buffer_load2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const f32x2 v = __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ float buffer_load1(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buffer_store4_nt(__amdgpu_buffer_rsrc_t r, uint32_t off, float a, float b,
                                                 float c, float d) {
  const f32x4 v = {a, b, c, d};
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, (int)off, 0, kAuxNT);
}

// ----------------------------------------------------------------- barriers
struct WGBarrier {
  __device__ __forceinline__ void sync() { __syncthreads(); }
};

// Arrival counter in LDS, monotonically increasing during one launch.  The k-th
// barrier of an interval of W wavefronts completes when the counter reaches k*W.
// Every wavefront of the interval must call sync() the same number of times, in
// wave-uniform control flow.  The counter must be zeroed, and the zero made
// visible with a whole-workgroup barrier, before the intervals branch apart.
struct PartBarrier {
  uint32_t* ctr;
  uint32_t nwaves;
  uint32_t target;
  __device__ __forceinline__ PartBarrier(uint32_t* c, uint32_t w) : ctr(c), nwaves(w), target(0) {}
  __device__ __forceinline__ void sync() {
    target += nwaves;
    // make this wave's LDS and global writes visible inside the workgroup
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane_id() == 0) {
      __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      while ((int32_t)(__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) -
                       target) < 0)
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
};

// ----------------------------------------------------------------- reductions
// DPP controls (GFX9 encoding): quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E,
// row_half_mirror = 0x141, row_mirror = 0x140.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ float readlane_f32(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Sum over the 64 lanes; every lane must be active.  After the four DPP steps
// each 16-lane row holds its row sum in every lane; the four row sums are then
// added in a fixed order.  Commutativity makes every lane's value identical.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f32<0xB1>(v);
  v += dpp_f32<0x4E>(v);
  v += dpp_f32<0x141>(v);
  v += dpp_f32<0x140>(v);
  const float r0 = readlane_f32(v, 0), r1 = readlane_f32(v, 16);
  const float r2 = readlane_f32(v, 32), r3 = readlane_f32(v, 48);
  return (r0 + r1) + (r2 + r3);
}

// Butterfly sum in double through ds_bpermute; identical result in every lane.
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

// ----------------------------------------------------------------- division
// q = n / d for 0 <= n < 2^31: with l = ceil(log2 d) and m = ceil(2^(31+l) / d),
// floor(n*m / 2^(31+l)) = floor(n/d) (Granlund & Montgomery, PLDI 1994), and m
// fits in 32 bits.  For d >= 2 the shift is >= 32, so only the high word of the
// product is needed.  d == 1 has m = 0 and an all-ones `id` mask that adds n
// back, so the quotient is one multiply-high, an and-or and a shift with no
// branch (a branch per division would split the kernels' loops into blocks).
struct FastDiv {
  uint32_t d;
  uint32_t m;
  uint32_t sh;  // 31 + l - 32
  uint32_t id;  // 0xFFFFFFFF when d == 1, else 0
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  if (d <= 1) {
    f.m = 0;
    f.sh = 0;
    f.id = 0xFFFFFFFFu;
    return f;
  }
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  const uint64_t num = 1ull << (31 + l);  // l <= 31, so this fits
  f.m = (uint32_t)((num + d - 1) / d);
  f.sh = 31 + l - 32;
  f.id = 0u;
  return f;
}

__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return ((uint32_t)(((uint64_t)n * f.m) >> 32) | (n & f.id)) >> f.sh;
}

// Remainder by a run-time constant d >= 1 for every 32-bit numerator.  With
// m = floor((2^32 - 1) / d) >= 2^32/d - 1, the estimate q = mulhi(n, m) lies
// in (n/d - 1 - n/2^32, n/d), so it is floor(n/d) or one less and r = n - q*d
// lies in [0, 2d); one conditional subtraction finishes it, written as the
// unsigned minimum of r and r - d (which wraps above r when r < d): five
// VALU instructions against nine for the compiler's reciprocal sequence.
struct FastMod {
  uint32_t d;
  uint32_t m;
};

inline FastMod make_fastmod(uint32_t d) { return FastMod{d, d ? 0xFFFFFFFFu / d : 0u}; }

__host__ __device__ __forceinline__ uint32_t fmod32(uint32_t n, const FastMod& f) {
  const uint32_t r = n - (uint32_t)(((uint64_t)n * f.m) >> 32) * f.d;
  const uint32_t s = r - f.d;
  return s < r ? s : r;
}

}  // namespace hf
