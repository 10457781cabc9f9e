// hf_kernels.hpp -- solo and horizontally fused global kernels.
//
// fused<K1, K2, BLOCK, WPE> is the fused kernel F of the Generate algorithm
// (Sec. III-A) for workgroup size d0 = BLOCK:
//   prologue  : the interval barriers' counters are cleared once, behind the only
//               whole-workgroup barrier of the kernel;
//   dispatch  : wavefronts [0, w1) run K1 with tid_1 = threadIdx.x, size_1 = 64*w1;
//               wavefronts [w1, BLOCK/64) run K2 with tid_2 = threadIdx.x - 64*w1,
//               size_2 = BLOCK - 64*w1.  The test is on a wave-uniform value, so it
//               compiles to a scalar branch, never to divergent lanes;
//   barriers  : each body gets its own interval barrier (PartBarrier).
// WPE > 0 asks the compiler for at least WPE resident wavefronts per SIMD, which
// bounds the VGPRs per lane to 512/WPE: the register bound of Sec. III-B.
#pragma once
#include <type_traits>
#include "hf_bodies.hpp"

namespace hf {

template <int KIND>
struct BodyOf;
template <> struct BodyOf<0> { using T = BnStats; };
template <> struct BodyOf<1> { using T = IntMix; };
template <> struct BodyOf<2> { using T = Im2col; };
template <> struct BodyOf<3> { using T = LdsHist; };
template <> struct BodyOf<4> { using T = Upsample; };
template <> struct BodyOf<5> { using T = Maxpool; };
template <> struct BodyOf<6> { using T = Sha256d; };
template <> struct BodyOf<7> { using T = Blake2b; };
template <> struct BodyOf<8> { using T = EthashLike; };

constexpr uint32_t max1(uint32_t v) { return v ? v : 1u; }

template <class K1, class K2, int BLOCK>
__device__ __forceinline__ void fused_body(const DevTask& ta, const DevTask& tb, uint32_t w1) {
  constexpr uint32_t L1 = K1::lds_words(BLOCK);
  constexpr uint32_t L2 = K2::lds_words(BLOCK);
  __shared__ uint32_t smem[2 + max1(L1 + L2)];
  if (threadIdx.x == 0) {
    smem[0] = 0u;
    smem[1] = 0u;
  }
  __syncthreads();  // the one whole-workgroup barrier: counters are zero
  const uint32_t wave = uniform(threadIdx.x >> 6);
  constexpr uint32_t W = BLOCK / 64;
  if (wave < w1) {
    const Part p{threadIdx.x, 64u * w1, wave, w1, blockIdx.x, gridDim.x};
    PartBarrier bar(&smem[0], w1);
    K1::run(ta, p, bar, &smem[2]);
  } else {
    const uint32_t w2 = W - w1;
    const Part p{threadIdx.x - 64u * w1, 64u * w2, wave - w1, w2, blockIdx.x, gridDim.x};
    PartBarrier bar(&smem[1], w2);
    K2::run(tb, p, bar, &smem[2 + L1]);
  }
}

template <class K1, class K2, int BLOCK>
__global__ void __launch_bounds__(BLOCK) fused_nocap(DevTask ta, DevTask tb, uint32_t w1) {
  fused_body<K1, K2, BLOCK>(ta, tb, w1);
}

template <class K1, class K2, int BLOCK, int WPE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE)))
fused_cap(DevTask ta, DevTask tb, uint32_t w1) {
  fused_body<K1, K2, BLOCK>(ta, tb, w1);
}

// Vertical fusion, the comparator of the paper (Sec. II-B "Vertical Kernel
// Fusion", Sec. IV-A): one launch in which every thread executes the first
// kernel's statements and then the second's, so both bodies see the whole
// workgroup and keep the native workgroup barrier.
template <class K1, class K2, int BLOCK>
__global__ void __launch_bounds__(BLOCK) vfused(DevTask ta, DevTask tb) {
  constexpr uint32_t L1 = K1::lds_words(BLOCK);
  constexpr uint32_t L2 = K2::lds_words(BLOCK);
  __shared__ uint32_t smem[max1(L1 > L2 ? L1 : L2)];
  const Part p{threadIdx.x, (uint32_t)BLOCK, uniform(threadIdx.x >> 6), (uint32_t)(BLOCK / 64),
               blockIdx.x, gridDim.x};
  WGBarrier bar;
  K1::run(ta, p, bar, smem);
  __syncthreads();  // the second body may reuse the LDS of the first
  K2::run(tb, p, bar, smem);
}

// Waves per SIMD the solo kernel of body K asks the compiler to fit (its
// kSoloWaves, else no request): a body whose scalar registers would otherwise
// cost it a wavefront per SIMD sets 8.
template <class K, class = void>
struct SoloWaves {
  static constexpr int v = 1;
};
template <class K>
struct SoloWaves<K, std::void_t<decltype(K::kSoloWaves)>> {
  static constexpr int v = K::kSoloWaves;
};

// The original kernel: the whole workgroup is one interval and its barrier is
// the native s_barrier.
template <class K, int BLOCK>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(SoloWaves<K>::v))) solo(DevTask t) {
  __shared__ uint32_t smem[max1(K::lds_words(BLOCK))];
  const Part p{threadIdx.x, (uint32_t)BLOCK, uniform(threadIdx.x >> 6), (uint32_t)(BLOCK / 64),
               blockIdx.x, gridDim.x};
  WGBarrier bar;
  K::run(t, p, bar, smem);
}

// ----------------------------------------------------------------- registry
struct KernelEntry {
  int kind_a, kind_b;  // kind_b < 0: solo kernel of kind_a
  int block;
  int cap;             // VGPR bound (0 = none); -1: vertically fused comparator
  const void* fn;
};

// caps offered and the waves-per-SIMD floor that realises each one
#define HF_CAP_LIST(X, KA, KB, B) X(KA, KB, B, 64, 8) X(KA, KB, B, 80, 6) X(KA, KB, B, 96, 5) X(KA, KB, B, 128, 4)

#define HF_FUSED_CAP_ENTRY(KA, KB, B, CAP, WPE)                                                  \
  {KA, KB, B, CAP,                                                                              \
   reinterpret_cast<const void*>(                                                               \
       &::hf::fused_cap<::hf::BodyOf<KA>::T, ::hf::BodyOf<KB>::T, B, WPE>)},

#define HF_FUSED_BLOCK_ENTRIES(KA, KB, B)                                                        \
  {KA, KB, B, 0,                                                                                \
   reinterpret_cast<const void*>(&::hf::fused_nocap<::hf::BodyOf<KA>::T, ::hf::BodyOf<KB>::T, B>)}, \
      HF_CAP_LIST(HF_FUSED_CAP_ENTRY, KA, KB, B)

// vertically fused kernels are registered with cap = -1
#define HF_VFUSED_ENTRY(KA, KB, B)                                                               \
  {KA, KB, B, -1, reinterpret_cast<const void*>(&::hf::vfused<::hf::BodyOf<KA>::T, ::hf::BodyOf<KB>::T, B>)},

// Defines `const KernelEntry* NAME(int* count)` listing every fused
// instantiation of the ordered pair (KA, KB) for blocks 256, 512, 1024, and the
// vertically fused comparator.
#define HF_DEFINE_PAIR_TABLE(KA, KB, NAME)                                                       \
  const ::hf::KernelEntry* NAME(int* count) {                                                   \
    static const ::hf::KernelEntry tab[] = {HF_FUSED_BLOCK_ENTRIES(KA, KB, 256)                  \
                                                HF_FUSED_BLOCK_ENTRIES(KA, KB, 512)              \
                                                    HF_FUSED_BLOCK_ENTRIES(KA, KB, 1024)         \
                                                        HF_VFUSED_ENTRY(KA, KB, 256)             \
                                                            HF_VFUSED_ENTRY(KA, KB, 512)         \
                                                                HF_VFUSED_ENTRY(KA, KB, 1024)};  \
    *count = (int)(sizeof(tab) / sizeof(tab[0]));                                               \
    return tab;                                                                                 \
  }

}  // namespace hf
