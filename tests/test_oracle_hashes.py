"""Pins of the hash oracles (oracle/hashes.py) against what does not come from
them: the worked examples and constants printed in FIPS 180-4 and RFC 7693,
the published FNV-1 test values, an independent implementation (hashlib), and
closed forms and dependence checks of the Ethash-like loop (whose seed is
hashlib's SHA-512 of the message)."""
import hashlib
import os

import numpy as np
import pytest

from oracle import hashes as O
from paper_2007_01277_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


def test_sha256_published_example():
    for msg, dig in _rows("sha256_fips180_4_abc.txt"):
        assert O.sha256(msg.encode()).hex() == dig


def test_sha256_constants_published_values():
    K, H0 = O.sha256_constants()
    for name, i, v in _rows("sha256_fips180_4_constants.txt"):
        assert (K if name == "K" else H0)[int(i)] == int(v, 16), (name, i)
    assert len(set(K)) == 64 and len(H0) == 8


@pytest.mark.parametrize("length", [0, 1, 3, 55, 56, 63, 64, 65, 80, 119, 120, 128, 191, 300])
def test_sha256_matches_hashlib_at_padding_boundaries(length):
    msg = bytes(inputs.rng(length).integers(0, 256, size=length, dtype=np.uint8))
    assert O.sha256(msg) == hashlib.sha256(msg).digest()


def test_sha256d_of_headers_matches_hashlib():
    hdr = bytes(inputs.rng(5).integers(0, 256, size=80, dtype=np.uint8))
    idx = [0, 1, 2, 1000, 65535]
    got = O.sha256d(hdr, 0xFFFFFFF0, idx)
    for i, d in zip(idx, got):
        m = hdr[:76] + ((0xFFFFFFF0 + i) & 0xFFFFFFFF).to_bytes(4, "little")  # wraps past 2^32
        assert d == hashlib.sha256(hashlib.sha256(m).digest()).digest()


def test_blake2b_published_example():
    for msg, n, dig in _rows("blake2b_rfc7693_abc.txt"):
        assert O.blake2b(msg.encode(), int(n)).hex() == dig


def test_blake2b_iv_is_the_sha512_initial_value():
    # RFC 7693 2.6: IV[0] = 0x6A09E667F3BCC908, whose high half is SHA-256's H0[0]
    iv = O.blake2b_iv()
    _, H0 = O.sha256_constants()
    assert [v >> 32 for v in iv] == H0
    assert iv[0] == 0x6A09E667F3BCC908


@pytest.mark.parametrize("length", [0, 1, 80, 127, 128, 129, 256, 300])
@pytest.mark.parametrize("outlen", [32, 64, 20])
def test_blake2b_matches_hashlib(length, outlen):
    msg = bytes(inputs.rng(length + outlen).integers(0, 256, size=length, dtype=np.uint8))
    assert O.blake2b(msg, outlen) == hashlib.blake2b(msg, digest_size=outlen).digest()


def test_blake2b_sigma_rows_are_permutations():
    for row in O.SIGMA:
        assert sorted(row) == list(range(16))


def test_blake2b_of_headers_matches_hashlib():
    hdr = bytes(inputs.rng(6).integers(0, 256, size=80, dtype=np.uint8))
    idx = [0, 7, 123456]
    for i, d in zip(idx, O.blake2b_header(hdr, 17, idx)):
        assert d == hashlib.blake2b(hdr[:76] + (17 + i).to_bytes(4, "little"), digest_size=32).digest()


def test_fnv1_published_values():
    for msg, v in _rows("fnv1_32_test_values.txt"):
        assert O.fnv1_32(b"" if msg == "-" else msg.encode()) == int(v, 16)


def _table(R, seed):
    return inputs.rng(seed).integers(0, 2 ** 32, size=(R, 32), dtype=np.uint64).astype(np.uint32)


def _fold8(mix):
    out = []
    for k in range(8):
        a = mix[4 * k]
        for t in range(1, 4):
            a = ((a * 16777619) % 2 ** 32) ^ mix[4 * k + t]
        out.append(a)
    return out


def test_ethash_like_zero_table_closed_form():
    # With an all-zero table every access multiplies each mix word by the FNV
    # prime, whatever rows are read: mix_j = s_(j mod 16) * P^64, then the
    # 4-to-1 fold.  The seed words are SHA-512 of the instance's 80-byte
    # message, read here as little-endian words by numpy.
    hdr = bytes(inputs.rng(8).integers(0, 256, size=80, dtype=np.uint8))
    p64 = pow(16777619, 64, 2 ** 32)
    for nonce in (99, 0xFFFFFFFF, 0x01020304):
        msg = hdr[:76] + nonce.to_bytes(4, "little")
        s = np.frombuffer(hashlib.sha512(msg).digest(), "<u4").astype(int)
        mix = [(int(s[j % 16]) * p64) % 2 ** 32 for j in range(32)]
        want = np.array(_fold8(mix), "<u4").tobytes()
        assert O.ethash_like_one(hdr, nonce, np.zeros((37, 32), np.uint32)) == want


def test_ethash_like_seed_takes_every_nonce_byte_little_endian():
    # Nonces on both sides of each byte carry: under the zero-table closed form
    # the digest is a function of SHA-512 of the message with the nonce's four
    # bytes in little-endian order, and of nothing else.
    hdr = bytes(range(80))
    p64 = pow(16777619, 64, 2 ** 32)
    for nonce in (0xFF, 0x100, 0xFFFF, 0x10000, 0xFFFFFF, 0x1000000):
        msg = hdr[:76] + bytes([nonce & 0xFF, (nonce >> 8) & 0xFF, (nonce >> 16) & 0xFF, nonce >> 24])
        s = np.frombuffer(hashlib.sha512(msg).digest(), "<u4").astype(int)
        mix = [(int(s[j % 16]) * p64) % 2 ** 32 for j in range(32)]
        got = O.ethash_like_one(hdr, nonce, np.zeros((1, 32), np.uint32))
        assert got == np.array(_fold8(mix), "<u4").tobytes(), hex(nonce)


def test_ethash_like_uses_all_sixteen_seed_words():
    # A one-row table whose words all equal c: every access reads that row and
    # maps each mix word x to x*P ^ c, so mix_j = g(s_(j mod 16)) with g those
    # 64 maps composed, whatever the access rule; then the 4-to-1 fold.  Two
    # nonces give seeds that differ in all 16 words, and digests that differ.
    hdr = bytes(inputs.rng(14).integers(0, 256, size=80, dtype=np.uint8))
    T = np.full((1, 32), 0x9E3779B9, np.uint32)
    a = np.frombuffer(O.ethash_like_one(hdr, 1, T), "<u4")
    b = np.frombuffer(O.ethash_like_one(hdr, 2, T), "<u4")
    sa = np.frombuffer(hashlib.sha512(hdr[:76] + (1).to_bytes(4, "little")).digest(), "<u4")
    sb = np.frombuffer(hashlib.sha512(hdr[:76] + (2).to_bytes(4, "little")).digest(), "<u4")
    assert np.all(sa != sb) and np.all(a != b)
    def g(x):
        for _ in range(64):
            x = ((x * 16777619) % 2 ** 32) ^ 0x9E3779B9
        return x
    for s, d in ((sa, a), (sb, b)):
        mix = [g(int(s[j % 16])) for j in range(32)]
        assert list(d) == _fold8(mix)


def test_ethash_like_depends_exactly_on_the_rows_it_reads():
    # flipping a word of a row changes the digest iff the row is read
    hdr = bytes(inputs.rng(9).integers(0, 256, size=80, dtype=np.uint8))
    R = 96
    T = _table(R, 10)
    seen = []
    base = O.ethash_like_one(hdr, 5, T, seen)
    assert len(seen) == 64 and all(0 <= p < R for p in seen)
    for r in range(R):
        T2 = T.copy()
        T2[r, 3] ^= 0x10000
        assert (O.ethash_like_one(hdr, 5, T2) != base) == (r in seen), r


def test_ethash_like_rows_spread_over_the_table():
    # 64 accesses x 200 nonces over 1024 rows: the accessed rows cover the table
    hdr = bytes(range(80))
    T = _table(1024, 11)
    rows = []
    for n in range(200):
        O.ethash_like_one(hdr, n, T, rows)
    counts = np.bincount(rows, minlength=1024)
    assert counts.min() > 0 and counts.max() < 40


def test_ethash_like_c_transcription_matches_the_python_definition():
    # the C walk (used for the full-size checks) against the plain-integer one,
    # with a nonce range that wraps past 2^32 and tables of 1, 37 and 4099 rows
    import oracle
    hdr = bytes(inputs.rng(12).integers(0, 256, size=80, dtype=np.uint8))
    for rows, n0, n in ((4099, 12345, 40), (37, 0xFFFFFFF0, 33), (1, 7, 5)):
        T = _table(rows, 13 + rows)
        got = oracle.ethash_like(hdr, n0, T, n)
        for i in range(n):
            assert got[i].tobytes() == O.ethash_like_one(hdr, (n0 + i) & 0xFFFFFFFF, T), (rows, i)
