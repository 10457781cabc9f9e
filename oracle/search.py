"""Reference for the configuration search of horizontal fusion -- TEST INFRASTRUCTURE.

Follows Sec. II-A ("Stream Multiprocessor and Occupancy") and the Main search
algorithm of Sec. III-B in the paper's notation:

  occupancy  : blocks per core = min(ShMemPerCore / ShMem(block),
                                     RegsPerCore / (threads * regs per thread),
                                     ThreadsPerCore / threads)
  bound r0   : b1 = SMNRegs / (d1 * NRegs(S1));  b2 = SMNRegs / (d2 * NRegs(S2));
               b0 = min(b1, b2, SMShMem / ShMem(F), SMNThreads / d0);
               r0 = SMNRegs / (b0 * d0)
  search     : d1 = 128, 256, ... while d1 < d0; profile F(d1) without a bound,
               then with r0; keep a candidate only if strictly faster than the
               best so far.

Readings (the paper gives the formulas without rounding and never defines d2 in
the search): every division is a floor, d2 = d0 - d1, and a core with no shared
memory use is not limited by shared memory.
"""
from __future__ import annotations

PASCAL = dict(regs=65536, shmem=96 * 1024, threads=2048)       # Sec. II-A / III-B
GFX950 = dict(regs=4 * 512 * 64, shmem=160 * 1024, threads=2048)  # per compute unit


def blocks_per_core(threads: int, regs_per_thread: int, shmem_bytes: int, hw=PASCAL) -> int:
    lim = [hw["regs"] // (threads * regs_per_thread), hw["threads"] // threads]
    if shmem_bytes > 0:
        lim.append(hw["shmem"] // shmem_bytes)
    return min(lim)


def register_bound(d0: int, d1: int, nregs1: int, nregs2: int, shmem_fused: int, hw=PASCAL) -> int:
    d2 = d0 - d1
    b1 = hw["regs"] // (d1 * nregs1)
    b2 = hw["regs"] // (d2 * nregs2)
    lim = [b1, b2, hw["threads"] // d0]
    if shmem_fused > 0:
        lim.append(hw["shmem"] // shmem_fused)
    b0 = min(lim)
    if b0 <= 0:
        return -1
    return hw["regs"] // (b0 * d0)


def paper_candidates(d0: int, step: int = 128):
    """The (d1, bounded) pairs in the order the Main search profiles them."""
    out = []
    d1 = step
    while d1 < d0:
        out.append((d1, False))
        out.append((d1, True))
        d1 += step
    return out


def paper_search(d0: int, profile, step: int = 128):
    """Returns (d1*, bounded*, t*) with the strict-improvement rule."""
    best = (None, None, float("inf"))
    for d1, bounded in paper_candidates(d0, step):
        t = profile(d1, bounded)
        if t < best[2]:
            best = (d1, bounded, t)
    return best
