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

// ============================================================ Ethash-like
// The inner loop of Ethash over a synthetic table: a 32-word mix folded with
// 64 table rows of 128 bytes, each row chosen from the mix.  Eight lanes carry
// one hash: lane g of the group holds mix words 4g..4g+3, so a row is read as
// one contiguous 128-byte segment (a 16-byte load per lane) and the word that
// picks the next row is broadcast within the group with a lane permute.  Each
// group carries kChains independent hashes whose row reads are issued back to
// back, so every wavefront keeps 8 * kChains reads in flight per step.  Lanes
// of a group past the last instance redo the last instance and store nothing,
// so every lane takes part in every permute.
struct EthashLike {
  static constexpr uint32_t lds_words(int) { return 0; }
  static constexpr uint32_t kPrime = 16777619u;
  static constexpr uint32_t kOffset = 2166136261u;
  static constexpr uint32_t kChains = 4;
  static constexpr uint32_t kPerWave = 8 * kChains;  // hashes per wavefront per step

  __device__ static __forceinline__ uint32_t fnv(uint32_t x, uint32_t y) { return (x * kPrime) ^ y; }

  template <class Bar>
  __device__ static void run(const DevTask& dt, const Part& p, Bar&, uint32_t*) {
    const EthArgs& a = dt.eth;
    if (a.n == 0) return;
    // FNV-1 over the 76 header bytes that every instance shares: uniform
    uint32_t h76 = kOffset;
#pragma unroll
    for (int k = 0; k < 19; ++k) {
      const uint32_t w = a.hdr[k];
#pragma unroll
      for (int b = 0; b < 4; ++b) h76 = fnv(h76, (w >> (8 * b)) & 0xFFu);
    }
    h76 = uniform(h76);
    const uint32_t lane = lane_id();
    const uint32_t grp = lane >> 3, gl = lane & 7u, q = gl & 3u;
    const uint32_t gbase = lane & ~7u;
    const uint32_t stride = kPerWave * p.nwg * p.nwaves;
    for (uint32_t base = kPerWave * (p.wg * p.nwaves + p.wave); base < a.n; base += stride) {  // wave-uniform
      uint32_t s0[kChains], mx[kChains][4];
#pragma unroll
      for (uint32_t h = 0; h < kChains; ++h) {
        const uint32_t ic = min(base + 8u * h + grp, a.n - 1u);
        const uint32_t nonce = a.nonce0 + ic;  // its four bytes, little-endian
        s0[h] = fnv(fnv(fnv(fnv(h76, nonce & 0xFFu), (nonce >> 8) & 0xFFu), (nonce >> 16) & 0xFFu), nonce >> 24);
        uint32_t s[16];
        s[0] = s0[h];
#pragma unroll
        for (int k = 1; k < 16; ++k) s[k] = fnv(s[k - 1], (uint32_t)k);
        // mix words 4*gl .. 4*gl+3 are s[(4*gl + c) % 16] = s[4*(gl % 4) + c]
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          uint32_t v = s[c];
#pragma unroll
          for (int r = 1; r < 4; ++r) v = (q == (uint32_t)r) ? s[4 * r + c] : v;
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
          const uint32_t row = fnv(j ^ s0[h], mw) % a.rows;
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
        const uint32_t i = base + 8u * h + grp;
        const uint32_t outw = fnv(fnv(fnv(mx[h][0], mx[h][1]), mx[h][2]), mx[h][3]);
        if (i < a.n) a.out[8u * i + gl] = outw;
      }
    }
  }
};

}  // namespace hf
