"""CPU oracle of the hash kernels -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It shares no code, table or constant with
the GPU library and never imports it.  Plain Python integers, one hash at a
time, every step in the order of its standard.

The evaluation's cryptography kernels (Sec. IV-A "Benchmark Kernels": SHA256,
Blake2B, and the memory-bound Ethash) each compute many hashes of a block
header that differ only in a nonce.  Readings taken (the paper names the
kernels, not their inputs): the message of instance i is an 80-byte header
whose last four bytes are replaced by the little-endian 32-bit nonce
nonce0 + i (mod 2^32); each instance outputs a 32-byte digest.

  * sha256d : SHA-256(SHA-256(message)) per FIPS 180-4 (padding 5.1.1, parsing
    5.2.1, functions 4.1.2, computation 6.2.2).  The round constants and the
    initial hash value are derived here from their definitions (4.2.2: the first
    32 bits of the fractional parts of the cube roots of the first 64 primes;
    5.3.3: of the square roots of the first 8 primes) with exact integer roots.
  * blake2b : BLAKE2b with a 32-byte digest and no key, per RFC 7693 (G 3.1,
    F 3.2, parameter block and padding 3.3).  The IV is derived from its
    definition (2.6: the SHA-512 initial value, i.e. the first 64 fractional
    bits of the square roots of the first 8 primes).  The message schedule
    SIGMA (2.7) is a table of the RFC, typed here.
  * ethash_like : not Ethash itself (synthetic table, SHA-512 in place of
    Keccak-512), but the shape of its hashimoto loop: a 512-bit seed hash of
    the message, repeated into a 32-word mix that is folded with 64
    pseudo-random 128-byte table rows, the row of access i chosen from the
    mix, by the FNV step fnv(a, b) = (a * 16777619) ^ b (mod 2^32).
    Definition used here:
      msg = the 80-byte message of the instance (header[0:76] || le32(nonce));
      s[0..15] = SHA-512(msg) (FIPS 180-4, the library's) read as sixteen
                 little-endian 32-bit words, where Ethash reads its Keccak-512
                 seed the same way;  mix[j] = s[j mod 16];
      for i in 0..63: p = fnv(i ^ s[0], mix[i mod 32]) mod R;
                      mix[j] = fnv(mix[j], T[p][j]) for j in 0..31;
      out[k] = fnv(fnv(fnv(mix[4k], mix[4k+1]), mix[4k+2]), mix[4k+3]), k < 8;
      digest = out[0..7] as little-endian bytes.
    The row of access i is Ethash's own access formula (its hashimoto loop)
    with the table's row count in place of the dataset's page count; Ethash
    hashes the seed and the folded mix once more with Keccak-256, which is
    left out here (the fold is the digest).
    Pins: the seed is hashlib's SHA-512; the FNV step against the published
    FNV-1 test values; the all-zero-table closed form of the 64 folds and of
    the final 4-to-1 fold; the nonce's little-endian placement; which rows
    the computation depends on.  The access formula itself is a stated
    reading (Ethash's), checked only through those dependence tests.
"""
from __future__ import annotations

import hashlib

M32 = 0xFFFFFFFF
M64 = 0xFFFFFFFFFFFFFFFF


# ------------------------------------------------------------------ constants
def first_primes(k: int):
    out, n = [], 2
    while len(out) < k:
        if all(n % p for p in out if p * p <= n):
            out.append(n)
        n += 1
    return out


def _iroot(x: int, e: int) -> int:
    """floor(x ** (1/e)) for a non-negative integer x, exactly."""
    if x < 2:
        return x
    r = 1 << ((x.bit_length() + e - 1) // e)  # an upper bound
    while True:
        y = ((e - 1) * r + x // r ** (e - 1)) // e
        if y >= r:
            break
        r = y
    while r ** e > x:
        r -= 1
    while (r + 1) ** e <= x:
        r += 1
    return r


def sha256_constants():
    """(K[64], H0[8]) of FIPS 180-4, from the cube / square roots of primes."""
    ps = first_primes(64)
    K = [_iroot(p << 96, 3) & M32 for p in ps]
    H0 = [_iroot(p << 64, 2) & M32 for p in ps[:8]]
    return K, H0


def blake2b_iv():
    """The 8 64-bit IV words of RFC 7693 (the SHA-512 initial value)."""
    return [_iroot(p << 128, 2) & M64 for p in first_primes(8)]


# RFC 7693, 2.7: message word permutations of the ten rounds (rounds 10 and 11
# reuse rows 0 and 1)
SIGMA = [
    [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15],
    [14, 10, 4, 8, 9, 15, 13, 6, 1, 12, 0, 2, 11, 7, 5, 3],
    [11, 8, 12, 0, 5, 2, 15, 13, 10, 14, 3, 6, 7, 1, 9, 4],
    [7, 9, 3, 1, 13, 12, 11, 14, 2, 6, 5, 10, 4, 0, 15, 8],
    [9, 0, 5, 7, 2, 4, 10, 15, 14, 1, 11, 12, 6, 8, 3, 13],
    [2, 12, 6, 10, 0, 11, 8, 3, 4, 13, 7, 5, 15, 14, 1, 9],
    [12, 5, 1, 15, 14, 13, 4, 10, 0, 7, 6, 3, 9, 2, 8, 11],
    [13, 11, 7, 14, 12, 1, 3, 9, 5, 0, 15, 4, 8, 6, 2, 10],
    [6, 15, 14, 9, 11, 3, 0, 8, 12, 2, 13, 7, 1, 4, 10, 5],
    [10, 2, 8, 4, 7, 6, 1, 5, 15, 11, 9, 14, 3, 12, 13, 0],
]


# ------------------------------------------------------------------ messages
def message(header: bytes, nonce: int) -> bytes:
    """The 80-byte message of one instance: header[0:76] || le32(nonce)."""
    assert len(header) == 80
    return bytes(header[:76]) + (nonce & M32).to_bytes(4, "little")


# ------------------------------------------------------------------ SHA-256
def _rotr32(x, n):
    return ((x >> n) | (x << (32 - n))) & M32


def sha256(msg: bytes, _c=[]) -> bytes:
    """SHA-256 of a byte string (FIPS 180-4, 6.2)."""
    if not _c:
        _c.append(sha256_constants())
    K, H0 = _c[0]
    # 5.1.1 padding: a 1 bit, zeros, then the 64-bit big-endian bit length
    bitlen = 8 * len(msg)
    data = msg + b"\x80" + b"\x00" * ((55 - len(msg)) % 64) + bitlen.to_bytes(8, "big")
    H = list(H0)
    for off in range(0, len(data), 64):
        # 6.2.2 step 1: message schedule
        W = [int.from_bytes(data[off + 4 * t: off + 4 * t + 4], "big") for t in range(16)]
        for t in range(16, 64):
            s0 = _rotr32(W[t - 15], 7) ^ _rotr32(W[t - 15], 18) ^ (W[t - 15] >> 3)
            s1 = _rotr32(W[t - 2], 17) ^ _rotr32(W[t - 2], 19) ^ (W[t - 2] >> 10)
            W.append((s1 + W[t - 7] + s0 + W[t - 16]) & M32)
        # steps 2-3: working variables and the 64 rounds
        a, b, c, d, e, f, g, h = H
        for t in range(64):
            S1 = _rotr32(e, 6) ^ _rotr32(e, 11) ^ _rotr32(e, 25)
            ch = (e & f) ^ (~e & g)
            T1 = (h + S1 + ch + K[t] + W[t]) & M32
            S0 = _rotr32(a, 2) ^ _rotr32(a, 13) ^ _rotr32(a, 22)
            maj = (a & b) ^ (a & c) ^ (b & c)
            T2 = (S0 + maj) & M32
            h, g, f, e, d, c, b, a = g, f, e, (d + T1) & M32, c, b, a, (T1 + T2) & M32
        # step 4: intermediate hash value
        H = [(x + y) & M32 for x, y in zip(H, (a, b, c, d, e, f, g, h))]
    return b"".join(x.to_bytes(4, "big") for x in H)


def sha256d(header: bytes, nonce0: int, indices) -> list:
    """Digests SHA-256(SHA-256(message_i)) for the instances i in `indices`."""
    return [sha256(sha256(message(header, nonce0 + i))) for i in indices]


# ------------------------------------------------------------------ BLAKE2b
def _rotr64(x, n):
    return ((x >> n) | (x << (64 - n))) & M64


def _g(v, a, b, c, d, x, y):
    """RFC 7693, 3.1: the mixing function G."""
    v[a] = (v[a] + v[b] + x) & M64
    v[d] = _rotr64(v[d] ^ v[a], 32)
    v[c] = (v[c] + v[d]) & M64
    v[b] = _rotr64(v[b] ^ v[c], 24)
    v[a] = (v[a] + v[b] + y) & M64
    v[d] = _rotr64(v[d] ^ v[a], 16)
    v[c] = (v[c] + v[d]) & M64
    v[b] = _rotr64(v[b] ^ v[c], 63)


def _f(h, m, t, last, iv):
    """RFC 7693, 3.2: the compression function F (12 rounds)."""
    v = list(h) + list(iv)
    v[12] ^= t & M64
    v[13] ^= (t >> 64) & M64
    if last:
        v[14] ^= M64
    for r in range(12):
        s = SIGMA[r % 10]
        _g(v, 0, 4, 8, 12, m[s[0]], m[s[1]])
        _g(v, 1, 5, 9, 13, m[s[2]], m[s[3]])
        _g(v, 2, 6, 10, 14, m[s[4]], m[s[5]])
        _g(v, 3, 7, 11, 15, m[s[6]], m[s[7]])
        _g(v, 0, 5, 10, 15, m[s[8]], m[s[9]])
        _g(v, 1, 6, 11, 12, m[s[10]], m[s[11]])
        _g(v, 2, 7, 8, 13, m[s[12]], m[s[13]])
        _g(v, 3, 4, 9, 14, m[s[14]], m[s[15]])
    return [h[i] ^ v[i] ^ v[i + 8] for i in range(8)]


def blake2b(msg: bytes, outlen: int = 32, _iv=[]) -> bytes:
    """Unkeyed BLAKE2b of a byte string with an outlen-byte digest (RFC 7693, 3.3)."""
    if not _iv:
        _iv.append(blake2b_iv())
    iv = _iv[0]
    h = list(iv)
    h[0] ^= 0x01010000 ^ outlen  # parameter block: depth 1, fanout 1, no key
    blocks = [msg[i:i + 128] for i in range(0, len(msg), 128)] or [b""]
    for k, blk in enumerate(blocks):
        last = k == len(blocks) - 1
        t = len(msg) if last else 128 * (k + 1)
        blk = blk + b"\x00" * (128 - len(blk))
        m = [int.from_bytes(blk[8 * i: 8 * i + 8], "little") for i in range(16)]
        h = _f(h, m, t, last, iv)
    return b"".join(x.to_bytes(8, "little") for x in h)[:outlen]


def blake2b_header(header: bytes, nonce0: int, indices) -> list:
    """32-byte BLAKE2b digests of message_i for the instances i in `indices`."""
    return [blake2b(message(header, nonce0 + i), 32) for i in indices]


# ------------------------------------------------------------------ Ethash-like
FNV_PRIME = 16777619
FNV_OFFSET = 2166136261


def fnv(a: int, b: int) -> int:
    """The FNV-1 step: multiply by the 32-bit FNV prime, then xor."""
    return ((a * FNV_PRIME) & M32) ^ b


def fnv1_32(data: bytes) -> int:
    """FNV-1 hash (32 bits) of a byte string, built from the same step."""
    h = FNV_OFFSET
    for byte in data:
        h = fnv(h, byte)
    return h


def ethash_seed(msg: bytes) -> list:
    """The 16 seed words of a message: its SHA-512 digest (FIPS 180-4, computed
    by hashlib) read as little-endian 32-bit words."""
    d = hashlib.sha512(msg).digest()
    return [int.from_bytes(d[4 * k: 4 * k + 4], "little") for k in range(16)]


def ethash_like_one(header: bytes, nonce: int, table, rows_accessed=None) -> bytes:
    """One instance of the definition in this module's docstring.  `table` is a
    sequence of R rows of 32 uint32 words; `rows_accessed`, if a list, receives
    the 64 row indices in access order."""
    R = len(table)
    s = ethash_seed(message(header, nonce))
    mix = [s[j % 16] for j in range(32)]
    for i in range(64):
        p = fnv(i ^ s[0], mix[i % 32]) % R
        if rows_accessed is not None:
            rows_accessed.append(p)
        row = table[p]
        mix = [fnv(mix[j], int(row[j])) for j in range(32)]
    out = [fnv(fnv(fnv(mix[4 * k], mix[4 * k + 1]), mix[4 * k + 2]), mix[4 * k + 3]) for k in range(8)]
    return b"".join(x.to_bytes(4, "little") for x in out)


def ethash_like(header: bytes, nonce0: int, table, indices) -> list:
    return [ethash_like_one(header, nonce0 + i, table) for i in indices]
