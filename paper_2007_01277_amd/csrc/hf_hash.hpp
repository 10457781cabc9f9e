// hf_hash.hpp -- the hash kernels of the evaluation's cryptography pairs
// (Sec. IV-A "Benchmark Kernels": SHA256 and Blake2B, compute-bound; Ethash,
// memory-bound).  Instance i hashes the 80-byte header with its last four bytes
// replaced by the little-endian nonce nonce0 + i and writes a 32-byte digest.
//
// The bodies follow the work-unit rule of every other body: the result of an
// instance depends only on the instance, so any grid, split or block size gives
// the same bytes.
#pragma once
#include "hf_device.hpp"

namespace hf {

// 64-bit rotate and shift right by a compile-time amount (SHA-512).  A value
// that differs between lanes (uni false) takes one funnel shift
// (v_alignbit_b32) per 32-bit half, where the compiler's own lowering of a
// 64-bit rotate takes two 64-bit shifts and two ORs.  A wave-uniform value (uni
// true) keeps the plain form, which the scalar unit executes: the alignbit form
// exists only as a vector instruction and would move uniform work, and the
// registers that hold its results across the loop, to the vector unit.
__device__ __forceinline__ uint64_t rotr64(uint64_t x, uint32_t n, bool uni = false) {
  if (uni) return __builtin_rotateright64(x, n);
  const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  uint32_t rl, rh;
  if (n < 32) {
    rl = __builtin_amdgcn_alignbit(hi, lo, n);
    rh = __builtin_amdgcn_alignbit(lo, hi, n);
  } else {
    rl = __builtin_amdgcn_alignbit(lo, hi, n - 32);
    rh = __builtin_amdgcn_alignbit(hi, lo, n - 32);
  }
  return ((uint64_t)rh << 32) | rl;
}
__device__ __forceinline__ uint64_t shr64(uint64_t x, uint32_t n, bool uni = false) {  // 0 < n < 32
  if (uni) return x >> n;
  const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  return ((uint64_t)(hi >> n) << 32) | __builtin_amdgcn_alignbit(hi, lo, n);
}

// ============================================================ SHA-256d
// FIPS 180-4.  The first 64 header bytes are the same for every nonce, so their
// compression (the midstate) is computed once per wavefront from uniform
// values; each lane then compresses the second block of its message and hashes
// the 32-byte digest again.
struct Sha256d {
  static constexpr uint32_t lds_words(int) { return 0; }

  // Sec. 4.2.2: round constants
  static constexpr uint32_t kK[64] = {
      0x428a2f98u, 0x71374491u, 0xb5c0fbcfu, 0xe9b5dba5u, 0x3956c25bu, 0x59f111f1u, 0x923f82a4u, 0xab1c5ed5u,
      0xd807aa98u, 0x12835b01u, 0x243185beu, 0x550c7dc3u, 0x72be5d74u, 0x80deb1feu, 0x9bdc06a7u, 0xc19bf174u,
      0xe49b69c1u, 0xefbe4786u, 0x0fc19dc6u, 0x240ca1ccu, 0x2de92c6fu, 0x4a7484aau, 0x5cb0a9dcu, 0x76f988dau,
      0x983e5152u, 0xa831c66du, 0xb00327c8u, 0xbf597fc7u, 0xc6e00bf3u, 0xd5a79147u, 0x06ca6351u, 0x14292967u,
      0x27b70a85u, 0x2e1b2138u, 0x4d2c6dfcu, 0x53380d13u, 0x650a7354u, 0x766a0abbu, 0x81c2c92eu, 0x92722c85u,
      0xa2bfe8a1u, 0xa81a664bu, 0xc24b8b70u, 0xc76c51a3u, 0xd192e819u, 0xd6990624u, 0xf40e3585u, 0x106aa070u,
      0x19a4c116u, 0x1e376c08u, 0x2748774cu, 0x34b0bcb5u, 0x391c0cb3u, 0x4ed8aa4au, 0x5b9cca4fu, 0x682e6ff3u,
      0x748f82eeu, 0x78a5636fu, 0x84c87814u, 0x8cc70208u, 0x90befffau, 0xa4506cebu, 0xbef9a3f7u, 0xc67178f2u};
  // Sec. 5.3.3: initial hash value
  static constexpr uint32_t kH0[8] = {0x6a09e667u, 0xbb67ae85u, 0x3c6ef372u, 0xa54ff53au,
                                      0x510e527fu, 0x9b05688cu, 0x1f83d9abu, 0x5be0cd19u};

  __device__ static __forceinline__ uint32_t rotr(uint32_t x, uint32_t n) { return __builtin_rotateright32(x, n); }

  // Sec. 6.2.2, rounds t0 .. t0+15 on the working variables; w is the rolling
  // 16-word message schedule (FIRST: rounds 0..15 read the block itself).
  // Within a chunk every schedule index is a compile-time constant.
  template <bool FIRST>
  __device__ static __forceinline__ void chunk(uint32_t (&v)[8], uint32_t (&w)[16], int t0) {
    uint32_t a = v[0], b = v[1], c = v[2], d = v[3], e = v[4], f = v[5], g = v[6], h = v[7];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      uint32_t wt;
      if (FIRST) {
        wt = w[i];
      } else {
        const uint32_t x = w[(i + 1) & 15], y = w[(i + 14) & 15];
        const uint32_t s0 = rotr(x, 7) ^ rotr(x, 18) ^ (x >> 3);
        const uint32_t s1 = rotr(y, 17) ^ rotr(y, 19) ^ (y >> 10);
        wt = s1 + w[(i + 9) & 15] + s0 + w[i];
        w[i] = wt;
      }
      const uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
      const uint32_t ch = (e & f) ^ (~e & g);
      const uint32_t T1 = h + S1 + ch + kK[t0 + i] + wt;
      const uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
      const uint32_t maj = (a & b) ^ (a & c) ^ (b & c);
      const uint32_t T2 = S0 + maj;
      h = g;
      g = f;
      f = e;
      e = d + T1;
      d = c;
      c = b;
      b = a;
      a = T1 + T2;
    }
    v[0] = a;
    v[1] = b;
    v[2] = c;
    v[3] = d;
    v[4] = e;
    v[5] = f;
    v[6] = g;
    v[7] = h;
  }

  // one block into the state st (Sec. 6.2.2): four unrolled 16-round chunks.
  // The constant words of a padded block fold into the schedule, and writing
  // the rounds as chunks over one 16-word schedule array (rather than as one
  // 64-round loop) keeps the compiler's live ranges short: the same 3139
  // instructions per nonce in 51 VGPRs instead of 79, so a fused kernel can
  // hold 8 waves per SIMD without spilling.
  __device__ static __forceinline__ void compress(uint32_t (&st)[8], uint32_t (&w)[16]) {
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = st[k];
    chunk<true>(v, w, 0);
    chunk<false>(v, w, 16);
    chunk<false>(v, w, 32);
    chunk<false>(v, w, 48);
#pragma unroll
    for (int k = 0; k < 8; ++k) st[k] += v[k];
  }

  template <class Bar>
  __device__ static void run(const DevTask& dt, const Part& p, Bar&, uint32_t*) {
    const ShaArgs& a = dt.sha;
    if (a.n == 0) return;
    // midstate of the first 64 bytes (big-endian words, Sec. 5.2.1); the
    // compiler also hoists the rounds of the second block that do not read the
    // nonce out of the loop
    uint32_t mid[8], w[16];
#pragma unroll
    for (int k = 0; k < 8; ++k) mid[k] = kH0[k];
#pragma unroll
    for (int k = 0; k < 16; ++k) w[k] = __builtin_bswap32(a.hdr[k]);
    compress(mid, w);
    // uniform across the wavefront: scalar registers, not VGPRs
#pragma unroll
    for (int k = 0; k < 8; ++k) mid[k] = uniform(mid[k]);
    const uint32_t t16 = __builtin_bswap32(a.hdr[16]), t17 = __builtin_bswap32(a.hdr[17]),
                   t18 = __builtin_bswap32(a.hdr[18]);
    const uint32_t stride = 64u * p.nwg * p.nwaves;
    for (uint32_t i = 64u * (p.wg * p.nwaves + p.wave) + lane_id(); i < a.n; i += stride) {
      // second block: bytes 64..79, then the padding of an 80-byte message (Sec. 5.1.1)
      uint32_t st[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) st[k] = mid[k];
      uint32_t m[16] = {t16, t17, t18, __builtin_bswap32(a.nonce0 + i), 0x80000000u, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0,
                        640u};
      compress(st, m);
      // second hash: the 32-byte digest, padded
      uint32_t s2[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) s2[k] = kH0[k];
      uint32_t m2[16] = {st[0], st[1], st[2], st[3], st[4], st[5], st[6], st[7], 0x80000000u, 0, 0, 0, 0, 0, 0,
                         256u};
      compress(s2, m2);
      uint4* o = reinterpret_cast<uint4*>(a.out + 8u * i);
      o[0] = make_uint4(__builtin_bswap32(s2[0]), __builtin_bswap32(s2[1]), __builtin_bswap32(s2[2]),
                        __builtin_bswap32(s2[3]));
      o[1] = make_uint4(__builtin_bswap32(s2[4]), __builtin_bswap32(s2[5]), __builtin_bswap32(s2[6]),
                        __builtin_bswap32(s2[7]));
    }
  }
};

// ============================================================ BLAKE2b
// RFC 7693, 32-byte digest, no key: the 80-byte message is one padded block.
// Message words 0..8 are the same for every nonce; word 9 carries the nonce.
struct Blake2b {
  static constexpr uint32_t lds_words(int) { return 0; }

  // Sec. 2.6
  static constexpr uint64_t kIV[8] = {0x6a09e667f3bcc908ull, 0xbb67ae8584caa73bull, 0x3c6ef372fe94f82bull,
                                      0xa54ff53a5f1d36f1ull, 0x510e527fade682d1ull, 0x9b05688c2b3e6c1full,
                                      0x1f83d9abfb41bd6bull, 0x5be0cd19137e2179ull};
  // Sec. 2.7, rounds 10 and 11 repeating rows 0 and 1
  static constexpr uint8_t kSigma[12][16] = {
      {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15}, {14, 10, 4, 8, 9, 15, 13, 6, 1, 12, 0, 2, 11, 7, 5, 3},
      {11, 8, 12, 0, 5, 2, 15, 13, 10, 14, 3, 6, 7, 1, 9, 4}, {7, 9, 3, 1, 13, 12, 11, 14, 2, 6, 5, 10, 4, 0, 15, 8},
      {9, 0, 5, 7, 2, 4, 10, 15, 14, 1, 11, 12, 6, 8, 3, 13}, {2, 12, 6, 10, 0, 11, 8, 3, 4, 13, 7, 5, 15, 14, 1, 9},
      {12, 5, 1, 15, 14, 13, 4, 10, 0, 7, 6, 3, 9, 2, 8, 11}, {13, 11, 7, 14, 12, 1, 3, 9, 5, 0, 15, 4, 8, 6, 2, 10},
      {6, 15, 14, 9, 11, 3, 0, 8, 12, 2, 13, 7, 1, 4, 10, 5}, {10, 2, 8, 4, 7, 6, 1, 5, 15, 11, 9, 14, 3, 12, 13, 0},
      {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15}, {14, 10, 4, 8, 9, 15, 13, 6, 1, 12, 0, 2, 11, 7, 5, 3}};

  __device__ static __forceinline__ uint64_t rotr(uint64_t x, uint32_t n) { return __builtin_rotateright64(x, n); }

  // Sec. 3.1
  __device__ static __forceinline__ void G(uint64_t (&v)[16], int a, int b, int c, int d, uint64_t x, uint64_t y) {
    v[a] = v[a] + v[b] + x;
    v[d] = rotr(v[d] ^ v[a], 32);
    v[c] = v[c] + v[d];
    v[b] = rotr(v[b] ^ v[c], 24);
    v[a] = v[a] + v[b] + y;
    v[d] = rotr(v[d] ^ v[a], 16);
    v[c] = v[c] + v[d];
    v[b] = rotr(v[b] ^ v[c], 63);
  }

  template <class Bar>
  __device__ static void run(const DevTask& dt, const Part& p, Bar&, uint32_t*) {
    const ShaArgs& a = dt.sha;
    if (a.n == 0) return;
    uint64_t m[16];
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = (uint64_t)a.hdr[2 * k] | ((uint64_t)a.hdr[2 * k + 1] << 32);
    const uint64_t m9lo = a.hdr[18];
#pragma unroll
    for (int k = 10; k < 16; ++k) m[k] = 0;
    const uint32_t stride = 64u * p.nwg * p.nwaves;
    for (uint32_t i = 64u * (p.wg * p.nwaves + p.wave) + lane_id(); i < a.n; i += stride) {
      m[9] = m9lo | ((uint64_t)(a.nonce0 + i) << 32);
      // Sec. 3.2 with the parameter block of Sec. 2.5 (digest 32 bytes, fanout
      // and depth 1) and the byte count t = 80 of the final block
      uint64_t v[16];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = kIV[k];
      v[0] ^= 0x01010020ull;
#pragma unroll
      for (int k = 0; k < 8; ++k) v[8 + k] = kIV[k];
      v[12] ^= 80ull;
      v[14] = ~v[14];
#pragma unroll
      for (int r = 0; r < 12; ++r) {
        G(v, 0, 4, 8, 12, m[kSigma[r][0]], m[kSigma[r][1]]);
        G(v, 1, 5, 9, 13, m[kSigma[r][2]], m[kSigma[r][3]]);
        G(v, 2, 6, 10, 14, m[kSigma[r][4]], m[kSigma[r][5]]);
        G(v, 3, 7, 11, 15, m[kSigma[r][6]], m[kSigma[r][7]]);
        G(v, 0, 5, 10, 15, m[kSigma[r][8]], m[kSigma[r][9]]);
        G(v, 1, 6, 11, 12, m[kSigma[r][10]], m[kSigma[r][11]]);
        G(v, 2, 7, 8, 13, m[kSigma[r][12]], m[kSigma[r][13]]);
        G(v, 3, 4, 9, 14, m[kSigma[r][14]], m[kSigma[r][15]]);
      }
      uint64_t h[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) h[k] = kIV[k] ^ (k == 0 ? 0x01010020ull : 0ull) ^ v[k] ^ v[k + 8];
      uint4* o = reinterpret_cast<uint4*>(a.out + 8u * i);
      o[0] = make_uint4((uint32_t)h[0], (uint32_t)(h[0] >> 32), (uint32_t)h[1], (uint32_t)(h[1] >> 32));
      o[1] = make_uint4((uint32_t)h[2], (uint32_t)(h[2] >> 32), (uint32_t)h[3], (uint32_t)(h[3] >> 32));
    }
  }
};

// ============================================================ SHA-512
// FIPS 180-4, the seed hash of the Ethash-like walk.  An 80-byte message is one
// padded 128-byte block (Sec. 5.1.2): message words 0..9, then 2^63, four zero
// words and the bit length 640.  Words 0..8 do not depend on the nonce, so the
// caller runs rounds 0..8 once per wavefront on uniform values.
struct Sha512 {
  // Sec. 4.2.3: round constants
  static constexpr uint64_t kK[80] = {
      0x428a2f98d728ae22ull, 0x7137449123ef65cdull, 0xb5c0fbcfec4d3b2full, 0xe9b5dba58189dbbcull,
      0x3956c25bf348b538ull, 0x59f111f1b605d019ull, 0x923f82a4af194f9bull, 0xab1c5ed5da6d8118ull,
      0xd807aa98a3030242ull, 0x12835b0145706fbeull, 0x243185be4ee4b28cull, 0x550c7dc3d5ffb4e2ull,
      0x72be5d74f27b896full, 0x80deb1fe3b1696b1ull, 0x9bdc06a725c71235ull, 0xc19bf174cf692694ull,
      0xe49b69c19ef14ad2ull, 0xefbe4786384f25e3ull, 0x0fc19dc68b8cd5b5ull, 0x240ca1cc77ac9c65ull,
      0x2de92c6f592b0275ull, 0x4a7484aa6ea6e483ull, 0x5cb0a9dcbd41fbd4ull, 0x76f988da831153b5ull,
      0x983e5152ee66dfabull, 0xa831c66d2db43210ull, 0xb00327c898fb213full, 0xbf597fc7beef0ee4ull,
      0xc6e00bf33da88fc2ull, 0xd5a79147930aa725ull, 0x06ca6351e003826full, 0x142929670a0e6e70ull,
      0x27b70a8546d22ffcull, 0x2e1b21385c26c926ull, 0x4d2c6dfc5ac42aedull, 0x53380d139d95b3dfull,
      0x650a73548baf63deull, 0x766a0abb3c77b2a8ull, 0x81c2c92e47edaee6ull, 0x92722c851482353bull,
      0xa2bfe8a14cf10364ull, 0xa81a664bbc423001ull, 0xc24b8b70d0f89791ull, 0xc76c51a30654be30ull,
      0xd192e819d6ef5218ull, 0xd69906245565a910ull, 0xf40e35855771202aull, 0x106aa07032bbd1b8ull,
      0x19a4c116b8d2d0c8ull, 0x1e376c085141ab53ull, 0x2748774cdf8eeb99ull, 0x34b0bcb5e19b48a8ull,
      0x391c0cb3c5c95a63ull, 0x4ed8aa4ae3418acbull, 0x5b9cca4f7763e373ull, 0x682e6ff3d6b2b8a3ull,
      0x748f82ee5defb2fcull, 0x78a5636f43172f60ull, 0x84c87814a1f0ab72ull, 0x8cc702081a6439ecull,
      0x90befffa23631e28ull, 0xa4506cebde82bde9ull, 0xbef9a3f7b2c67915ull, 0xc67178f2e372532bull,
      0xca273eceea26619cull, 0xd186b8c721c0c207ull, 0xeada7dd6cde0eb1eull, 0xf57d4f7fee6ed178ull,
      0x06f067aa72176fbaull, 0x0a637dc5a2c898a6ull, 0x113f9804bef90daeull, 0x1b710b35131c471bull,
      0x28db77f523047d84ull, 0x32caab7b40c72493ull, 0x3c9ebe0a15c9bebcull, 0x431d67c49c100d4cull,
      0x4cc5d4becb3e42b6ull, 0x597f299cfc657e2aull, 0x5fcb6fab3ad6faecull, 0x6c44198c4a475817ull};
  // Sec. 5.3.5: the initial hash value, which BLAKE2b takes as its IV
  __device__ static __forceinline__ uint64_t h0(int k) { return Blake2b::kIV[k]; }

  // Which words of the schedule of an 80-byte message with a varying word 9
  // are the same in every lane: the header words 0..8, the padding words
  // 10..15, and the schedule words 17, 19 and 21, whose four inputs all are.
  // It only picks the instruction form of a rotate (above), never the value.
  __device__ static constexpr bool uni(int j) {
    return j <= 8 || (j >= 10 && j <= 15) || j == 17 || j == 19 || j == 21;
  }

  // Sec. 6.4.2, rounds T0 .. T1-1 on the working variables v; w is the rolling
  // 16-word schedule (rounds below 16 read the block itself).  Every index is a
  // compile-time constant once the loop is unrolled.  Rounds below 9 see only
  // uniform values (the caller runs them once per wavefront).  The uniform
  // terms of a schedule word are summed first and with the round constant, so
  // that they form one loop-invariant value.
  template <int T0, int T1>
  __device__ static __forceinline__ void rounds(uint64_t (&v)[8], uint64_t (&w)[16]) {
    uint64_t a = v[0], b = v[1], c = v[2], d = v[3], e = v[4], f = v[5], g = v[6], h = v[7];
#pragma unroll
    for (int t = T0; t < T1; ++t) {
      const bool us = t < 9;  // the state is uniform
      uint64_t ku, wv;        // round constant plus the uniform part of W_t; the rest
      if (t < 16) {
        ku = uni(t) ? kK[t] + w[t] : kK[t];
        wv = uni(t) ? 0 : w[t];
      } else {
        const int i = t & 15;
        const uint64_t x = w[(i + 1) & 15], y = w[(i + 14) & 15];
        const bool ux = uni(t - 15), uy = uni(t - 2);
        const uint64_t s0 = rotr64(x, 1, ux) ^ rotr64(x, 8, ux) ^ shr64(x, 7, ux);
        const uint64_t s1 = rotr64(y, 19, uy) ^ rotr64(y, 61, uy) ^ shr64(y, 6, uy);
        const uint64_t q = w[(i + 9) & 15], r = w[i];
        const bool uq = uni(t - 7), ur = uni(t - 16);
        const uint64_t wu = (uy ? s1 : 0) + (uq ? q : 0) + (ux ? s0 : 0) + (ur ? r : 0);
        wv = (uy ? 0 : s1) + (uq ? 0 : q) + (ux ? 0 : s0) + (ur ? 0 : r);
        ku = kK[t] + wu;
        w[i] = wu + wv;
      }
      const uint64_t S1 = rotr64(e, 14, us) ^ rotr64(e, 18, us) ^ rotr64(e, 41, us);
      const uint64_t ch = (e & f) ^ (~e & g);
      const uint64_t T1v = ku + h + S1 + ch + wv;
      const uint64_t S0 = rotr64(a, 28, us) ^ rotr64(a, 34, us) ^ rotr64(a, 39, us);
      const uint64_t ab = a ^ b, maj = (ab & c) | (~ab & a);  // a where a == b, else c
      h = g;
      g = f;
      f = e;
      e = d + T1v;
      d = c;
      c = b;
      b = a;
      a = T1v + S0 + maj;
    }
    v[0] = a;
    v[1] = b;
    v[2] = c;
    v[3] = d;
    v[4] = e;
    v[5] = f;
    v[6] = g;
    v[7] = h;
  }
};

// ============================================================ Ethash-like
// Ethash's hashimoto loop over a synthetic table, with SHA-512 of the message
// as the 512-bit seed: a 32-word mix (the seed words twice) folded with 64
// table rows of 128 bytes, each row chosen from the mix.  Every lane first
// hashes the message of one instance (64 instances per wavefront and
// iteration, rounds 0..8 hoisted as uniform work).  The walks then run in two
// passes of 32 instances: eight lanes carry one walk, lane g of the group
// holding mix words 4g..4g+3, so a row is read as one contiguous 128-byte
// segment (a 16-byte load per lane), and the word that picks the next row is
// broadcast within the group with a lane permute.  Each group carries kChains
// walks whose row reads are issued back to back, so every wavefront keeps
// 8 * kChains reads in flight per step.  Lanes past the last instance redo
// the last instance and store nothing, so every lane takes part in every
// permute.
struct EthashLike {
  static constexpr uint32_t lds_words(int) { return 0; }
  static constexpr uint32_t kPrime = 16777619u;
  static constexpr uint32_t kChains = 4;
  static constexpr uint32_t kPerPass = 8 * kChains;  // walks per wavefront per pass
  static constexpr uint32_t kPerIter = 64;            // seeds per wavefront per iteration

  __device__ static __forceinline__ uint32_t fnv(uint32_t x, uint32_t y) { return (x * kPrime) ^ y; }

  // the big-endian 64-bit message word k of the header (bytes 8k .. 8k+7)
  __device__ static __forceinline__ uint64_t hdr64(const uint32_t* hdr, int k) {
    return ((uint64_t)__builtin_bswap32(hdr[2 * k]) << 32) | __builtin_bswap32(hdr[2 * k + 1]);
  }

  template <class Bar>
  __device__ static void run(const DevTask& dt, const Part& p, Bar&, uint32_t*) {
    const EthArgs& a = dt.eth;
    if (a.n == 0) return;
    // rounds 0..8 read header words only: uniform, so scalar registers
    uint64_t w0[16], mid[8];
#pragma unroll
    for (int k = 0; k < 16; ++k) w0[k] = k < 9 ? hdr64(a.hdr, k) : 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) mid[k] = Sha512::h0(k);
    Sha512::rounds<0, 9>(mid, w0);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      mid[k] = ((uint64_t)uniform((uint32_t)(mid[k] >> 32)) << 32) | uniform((uint32_t)mid[k]);
    const uint64_t w9hi = (uint64_t)__builtin_bswap32(a.hdr[18]) << 32;
    const uint32_t lane = lane_id();
    const uint32_t grp = lane >> 3, gl = lane & 7u, q = gl & 3u;
    const uint32_t gbase = lane & ~7u;
    const uint32_t stride = kPerIter * p.nwg * p.nwaves;
    for (uint32_t base = kPerIter * (p.wg * p.nwaves + p.wave); base < a.n; base += stride) {  // wave-uniform
      // this lane's seed: SHA-512 of instance base + lane, as 16 little-endian words
      uint32_t sd[16];
      {
        uint64_t v[8], w[16];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = mid[k];
#pragma unroll
        for (int k = 0; k < 9; ++k) w[k] = w0[k];
        w[9] = w9hi | __builtin_bswap32(a.nonce0 + min(base + lane, a.n - 1u));
        w[10] = 0x8000000000000000ull;
#pragma unroll
        for (int k = 11; k < 15; ++k) w[k] = 0;
        w[15] = 640;
        Sha512::rounds<9, 16>(v, w);
        Sha512::rounds<16, 32>(v, w);
        Sha512::rounds<32, 48>(v, w);
        Sha512::rounds<48, 64>(v, w);
        Sha512::rounds<64, 80>(v, w);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint64_t hk = Sha512::h0(k) + v[k];
          sd[2 * k] = __builtin_bswap32((uint32_t)(hk >> 32));
          sd[2 * k + 1] = __builtin_bswap32((uint32_t)hk);
        }
      }
#pragma unroll 1
      for (uint32_t pass = 0; pass < kPerIter / kPerPass; ++pass) {
        const uint32_t pbase = base + kPerPass * pass;
        if (pbase >= a.n) break;  // wave-uniform
        // walk h of group grp is instance pbase + 8h + grp, whose seed lane
        // kPerPass*pass + 8h + grp holds; lane g of the group takes mix words
        // 4g..4g+3 = seed words 4(g % 4)..4(g % 4)+3, and every lane seed word 0
        uint32_t s0[kChains], mx[kChains][4];
#pragma unroll
        for (uint32_t h = 0; h < kChains; ++h) {
          const int src = (int)((kPerPass * pass + 8u * h + grp) << 2);
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            uint32_t v = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const uint32_t t = (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)sd[4 * r + c]);
              if (r == 0 && c == 0) s0[h] = t;
              v = q == (uint32_t)r ? t : v;
            }
            mx[h][c] = v;
          }
        }
#pragma unroll 4
        for (uint32_t j = 0; j < 64; ++j) {
          // mix word j % 32 is component j % 4 of lane (j % 32) / 4 of the group
          const uint32_t cj = j & 3u;
          const uint32_t src = (gbase + ((j & 31u) >> 2)) << 2;
          uint4 d[kChains];
#pragma unroll
          for (uint32_t h = 0; h < kChains; ++h) {
            const uint32_t comp = cj == 0 ? mx[h][0] : (cj == 1 ? mx[h][1] : (cj == 2 ? mx[h][2] : mx[h][3]));
            const uint32_t mw = (uint32_t)__builtin_amdgcn_ds_bpermute((int)src, (int)comp);
            const uint32_t row = fmod32(fnv(j ^ s0[h], mw), a.rows);
            d[h] = a.table[(size_t)row * 8u + gl];
          }
#pragma unroll
          for (uint32_t h = 0; h < kChains; ++h) {
            mx[h][0] = fnv(mx[h][0], d[h].x);
            mx[h][1] = fnv(mx[h][1], d[h].y);
            mx[h][2] = fnv(mx[h][2], d[h].z);
            mx[h][3] = fnv(mx[h][3], d[h].w);
          }
        }
#pragma unroll
        for (uint32_t h = 0; h < kChains; ++h) {
          const uint32_t i = pbase + 8u * h + grp;
          const uint32_t outw = fnv(fnv(fnv(mx[h][0], mx[h][1]), mx[h][2]), mx[h][3]);
          if (i < a.n) a.out[8u * i + gl] = outw;
        }
      }
    }
  }
};

}  // namespace hf
