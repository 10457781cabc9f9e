"""Builds libhfuse.so (gfx950) in-tree with hipcc.

Every translation unit under ``csrc/`` is compiled to an object in ``_build/``
in parallel, then linked into ``paper_2007_01277_amd/libhfuse.so``.  The fused
instantiations are split into one object per pair of kernel kinds.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libhfuse.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    # packed fp32 instructions stay off: only scalar fp32 VALU forms are emitted
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]

NUM_KINDS = 9
PAIRS = [(a, b) for a in range(NUM_KINDS) for b in range(a, NUM_KINDS)]


def _units():
    units = []
    for a, b in PAIRS:
        units.append((os.path.join(CSRC, "hf_pairs.hip"), f"pair_{a}_{b}.o", [f"-DHF_KA={a}", f"-DHF_KB={b}"]))
    for name in ("hf_solo", "hf_runtime", "hf_tune", "hf_mlp", "hf_batch"):
        units.append((os.path.join(CSRC, name + ".hip"), name + ".o", []))
    return units


def _compile(src, obj, defs, remarks):
    cmd = [HIPCC] + FLAGS + defs + ["-c", src, "-o", os.path.join(BUILD, obj)]
    if remarks:
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {obj}:\n{r.stderr[-4000:]}")
    return obj, r.stderr


def _stale(src, obj):
    """True unless `obj` is newer than its source and every header it may include."""
    path = os.path.join(BUILD, obj)
    if not os.path.exists(path):
        return True
    deps = [src, os.path.join(PKG, os.pardir, "include", "hfuse.h")] + \
        [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    return os.path.getmtime(path) < max(os.path.getmtime(d) for d in deps)


def build(jobs: int | None = None, remarks: bool = False, verbose: bool = True,
          incremental: bool = False) -> str:
    """Compiles every HIP translation unit (with incremental=True only those
    older than their sources or any header) and links libhfuse.so; returns
    its path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    units = _units()
    todo = [u for u in units if not incremental or remarks or _stale(u[0], u[1])]
    logs = {}
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, s, o, d, remarks) for s, o, d in todo]
        for f in cf.as_completed(futs):
            obj, err = f.result()
            logs[obj] = err
    if remarks:
        with open(os.path.join(BUILD, "resource_usage.txt"), "w") as fh:
            for obj in sorted(logs):
                fh.write(logs[obj])
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
        [os.path.join(BUILD, o) for _, o, _ in units]
    subprocess.check_call(cmd)
    shutil.move(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


ASAN_DIR = os.path.join(BUILD, "asan")
ASAN_EXE = os.path.join(ASAN_DIR, "host_checks")
HOST_UNITS = ("hf_runtime", "hf_tune", "hf_mlp", "hf_batch")


def build_asan(jobs: int | None = None) -> str:
    """Builds tests/asan/host_checks.cpp against the library with the host side
    of its host translation units compiled under AddressSanitizer (the device
    code is unchanged; the kernel-table objects of the regular build are
    reused).  Returns the executable's path; it runs without a GPU."""
    needed = [os.path.join(BUILD, o) for _, o, _ in _units()]
    if not os.path.exists(LIB) or not all(os.path.exists(o) for o in needed):
        build(jobs=jobs)
    os.makedirs(ASAN_DIR, exist_ok=True)
    asan = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
    jobs = jobs or min(16, os.cpu_count() or 4)
    units = [(os.path.join(CSRC, u + ".hip"), os.path.join(ASAN_DIR, u + ".o")) for u in HOST_UNITS]

    def comp(src, obj):
        r = subprocess.run([HIPCC] + FLAGS + asan + ["-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {obj}:\n{r.stderr[-4000:]}")

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda u: comp(*u), units))
    others = [os.path.join(BUILD, o) for _, o, _ in _units() if o[:-2] not in HOST_UNITS]
    # the driver is host code only: compiled by the ROCm clang as plain C++
    drv = os.path.join(PKG, os.pardir, "tests", "asan", "host_checks.cpp")
    drv_o = os.path.join(ASAN_DIR, "host_checks.o")
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), os.pardir, "lib", "llvm", "bin", "clang++")
    r = subprocess.run([clang, "-O1", "-g", "-std=c++17", "-fsanitize=address", "-fno-omit-frame-pointer", "-c",
                        drv, "-o", drv_o], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling the host checks failed:\n{r.stderr[-4000:]}")
    cmd = [HIPCC, f"--offload-arch={ARCH}"] + asan + [drv_o] + [o for _, o in units] + others + ["-o", ASAN_EXE]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking the host checks failed:\n{r.stderr[-4000:]}")
    return ASAN_EXE


if __name__ == "__main__":
    import sys
    if "--asan" in sys.argv:
        print(build_asan())
    else:
        build(remarks="--remarks" in sys.argv, incremental="--incremental" in sys.argv)
