"""CPU oracle — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU reference for everything the HIP library
computes, written from Li, Narayana & El-Ghazawi (2015) and from the readings
of it that the library documents.  Only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it.  It shares no code with
``paper_1511_07983_amd`` (neither imports the other); the only common module
is ``synth``, which draws inputs and holds none of the method's arithmetic.

Parts:
  * ``ko_oracle.c``  discrete-event dispatch model, one block at a time
                      (Section 2 and Table 1), lexicographic unranking, many
                      orders over threads, and the round-synchronous reading
                      of Section 2's execution rounds, and a third model in
                      which resident blocks share the chip's memory
                      throughput (Section 4).  Loaded here through ctypes.
  * ``heuristic``    Algorithm 1 (ScoreGen, ProfileCombine, execution rounds)
                      in binary64 Python floats.
  * ``tick``         a second formulation of the dispatch model that advances
                      one cycle at a time, for brute-force cross-checks.
  * ``stats``        per-set statistics, rank counts, percentiles, histogram,
                      and the Table 3 report formulas.
  * ``sampling``     counter-based sampled ranks (SplitMix64 + multiply-shift).
  * ``features``, ``mlp``  the surrogate's per-kernel features, area lower
                      bound and network in float64.
  * ``beam``         the bookkeeping of one beam-search step (expansion,
                      diversity rules, gather).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libko_oracle.so")
_lib = None

GPU_FIELDS = ("n_cu", "wave_size", "wave_cu", "blk_cu", "reg_cu", "lds_cu", "rb_milli")
KERNEL_FIELDS = ("n_tblk", "n_inst", "lds_blk", "waves_blk", "regs_thr", "r_milli")


def build(force: bool = True) -> str:
    """Compile ko_oracle.c with plain -O2 (no SIMD intrinsics) into libko_oracle.so."""
    global _lib
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-pthread", os.path.join(_HERE, "ko_oracle.c"), "-o", tmp])
        os.replace(tmp, _LIB_PATH)
        _lib = None
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.oc_derive.argtypes = [i64p, ctypes.c_int32, i64p, i64p, i64p]
        L.oc_derive.restype = ctypes.c_int
        L.oc_makespan.argtypes = [i64p, ctypes.c_int32, i64p, i32p]
        L.oc_makespan.restype = ctypes.c_int64
        L.oc_unrank.argtypes = [ctypes.c_int32, ctypes.c_uint64, i32p]
        L.oc_unrank.restype = None
        L.oc_rank.argtypes = [ctypes.c_int32, i32p]
        L.oc_rank.restype = ctypes.c_uint64
        L.oc_makespans_range.argtypes = [i64p, ctypes.c_int32, i64p, ctypes.c_uint64,
                                         ctypes.c_int64, i64p, ctypes.c_int32]
        L.oc_makespans_range.restype = ctypes.c_int
        L.oc_makespans_ranks.argtypes = [i64p, ctypes.c_int32, i64p, u64p,
                                         ctypes.c_int64, i64p, ctypes.c_int32]
        L.oc_makespans_ranks.restype = ctypes.c_int
        L.oc_makespans_orders.argtypes = [i64p, ctypes.c_int32, i64p, i32p,
                                          ctypes.c_int64, i64p, ctypes.c_int32]
        L.oc_makespans_orders.restype = ctypes.c_int
        L.oc_rounds_makespans.argtypes = [i64p, ctypes.c_int32, i64p, i32p, ctypes.c_int64, i64p]
        L.oc_rounds_makespans.restype = ctypes.c_int
        L.oc_contended_makespans.argtypes = [i64p, ctypes.c_int64, ctypes.c_int32, i64p, i32p,
                                             ctypes.c_uint64, ctypes.c_int64, i64p]
        L.oc_contended_makespans.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def gpu_array(gpu) -> np.ndarray:
    """GPU model (mapping or object with the GPU_FIELDS attributes) as int64[7]."""
    get = gpu.get if isinstance(gpu, dict) else (lambda f: getattr(gpu, f))
    return np.array([int(get(f)) for f in GPU_FIELDS], dtype=np.int64)


def kernel_array(kernels) -> np.ndarray:
    """Kernel descriptors (structured array or list of dicts) as int64[n, 6]."""
    if isinstance(kernels, np.ndarray) and kernels.dtype.names:
        return np.ascontiguousarray(
            np.stack([kernels[f].astype(np.int64) for f in KERNEL_FIELDS], axis=1))
    return np.array([[int(k[f]) for f in KERNEL_FIELDS] for k in kernels], dtype=np.int64)


def derive(gpu, kernels):
    """(use[n,4] = reg, lds, wave, blk per block;  dur[n] cycles per block)."""
    g, k = gpu_array(gpu), kernel_array(kernels)
    n = k.shape[0]
    use = np.zeros((n, 4), dtype=np.int64)
    dur = np.zeros(n, dtype=np.int64)
    rc = lib().oc_derive(_ptr(g, ctypes.c_int64), n, _ptr(k, ctypes.c_int64),
                         _ptr(use, ctypes.c_int64), _ptr(dur, ctypes.c_int64))
    if rc:
        raise ValueError("invalid GPU model or kernel descriptor")
    return use, dur


def makespan(gpu, kernels, order) -> int:
    """Makespan (int64 cycles) of one launch order; order[j] = kernel at position j."""
    g, k = gpu_array(gpu), kernel_array(kernels)
    o = np.ascontiguousarray(order, dtype=np.int32)
    if o.shape != (k.shape[0],):
        raise ValueError("order length must equal the number of kernels")
    m = lib().oc_makespan(_ptr(g, ctypes.c_int64), k.shape[0], _ptr(k, ctypes.c_int64),
                          _ptr(o, ctypes.c_int32))
    if m < 0:
        raise ValueError("invalid input (bad descriptor or order is not a permutation)")
    return int(m)


def unrank(n: int, rank: int) -> list:
    perm = np.zeros(n, dtype=np.int32)
    lib().oc_unrank(n, rank, _ptr(perm, ctypes.c_int32))
    return perm.tolist()


def rank(perm) -> int:
    p = np.ascontiguousarray(perm, dtype=np.int32)
    return int(lib().oc_rank(len(p), _ptr(p, ctypes.c_int32)))


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


def makespans_range(gpu, kernels, lo: int, count: int, threads: int | None = None) -> np.ndarray:
    """Makespans of the orders with lexicographic ranks lo .. lo+count-1."""
    g, k = gpu_array(gpu), kernel_array(kernels)
    out = np.zeros(count, dtype=np.int64)
    rc = lib().oc_makespans_range(_ptr(g, ctypes.c_int64), k.shape[0], _ptr(k, ctypes.c_int64),
                                  lo, count, _ptr(out, ctypes.c_int64),
                                  threads or default_threads())
    if rc:
        raise ValueError("invalid input")
    return out


def makespans_all(gpu, kernels, threads: int | None = None) -> np.ndarray:
    n = kernel_array(kernels).shape[0]
    import math
    return makespans_range(gpu, kernels, 0, math.factorial(n), threads)


def makespans_ranks(gpu, kernels, ranks, threads: int | None = None) -> np.ndarray:
    g, k = gpu_array(gpu), kernel_array(kernels)
    r = np.ascontiguousarray(ranks, dtype=np.uint64)
    out = np.zeros(len(r), dtype=np.int64)
    rc = lib().oc_makespans_ranks(_ptr(g, ctypes.c_int64), k.shape[0], _ptr(k, ctypes.c_int64),
                                  _ptr(r, ctypes.c_uint64), len(r), _ptr(out, ctypes.c_int64),
                                  threads or default_threads())
    if rc:
        raise ValueError("invalid input")
    return out


def makespans_orders(gpu, kernels, orders, threads: int | None = None) -> np.ndarray:
    g, k = gpu_array(gpu), kernel_array(kernels)
    o = np.ascontiguousarray(orders, dtype=np.int32)
    out = np.zeros(o.shape[0], dtype=np.int64)
    rc = lib().oc_makespans_orders(_ptr(g, ctypes.c_int64), k.shape[0], _ptr(k, ctypes.c_int64),
                                   _ptr(o, ctypes.c_int32), o.shape[0], _ptr(out, ctypes.c_int64),
                                   threads or default_threads())
    if rc:
        raise ValueError("invalid input")
    return out


def rounds_makespans(gpu, kernels, orders) -> np.ndarray:
    """Makespans under the round-synchronous reading of Section 2's execution
    rounds: a round closes when the head block fits on no CU and lasts as long
    as its longest block; the makespan is the sum of the rounds.  orders is an
    int array [count, n] of permutations."""
    g, k = gpu_array(gpu), kernel_array(kernels)
    o = np.ascontiguousarray(orders, dtype=np.int32)
    if o.ndim != 2 or o.shape[1] != k.shape[0]:
        raise ValueError("orders must be [count, n]")
    out = np.zeros(o.shape[0], dtype=np.int64)
    rc = lib().oc_rounds_makespans(_ptr(g, ctypes.c_int64), k.shape[0], _ptr(k, ctypes.c_int64),
                                   _ptr(o, ctypes.c_int32), o.shape[0], _ptr(out, ctypes.c_int64))
    if rc:
        raise ValueError("invalid input (bad descriptor or an order is not a permutation)")
    return out


def contended_makespans(gpu, kernels, mem_blocks: int, orders=None, *, first: int = 0,
                        count: int | None = None) -> np.ndarray:
    """Makespans when the resident blocks share the chip's memory throughput
    (Section 4's balance of instructions and memory accesses): mem_blocks
    memory-bound blocks run at full speed at once, more slow every resident
    block down by the same factor.  orders: int array [count, n] of
    permutations, or None for lexicographic ranks first .. first+count-1."""
    g, k = gpu_array(gpu), kernel_array(kernels)
    n = k.shape[0]
    if orders is not None:
        o = np.ascontiguousarray(orders, dtype=np.int32)
        if o.ndim != 2 or o.shape[1] != n:
            raise ValueError("orders must be [count, n]")
        count = o.shape[0]
        optr = _ptr(o, ctypes.c_int32)
    else:
        optr = None
    out = np.zeros(count, dtype=np.int64)
    rc = lib().oc_contended_makespans(_ptr(g, ctypes.c_int64), int(mem_blocks), n, _ptr(k, ctypes.c_int64),
                                      optr, int(first), int(count), _ptr(out, ctypes.c_int64))
    if rc:
        raise ValueError("invalid input (bad descriptor, mem_blocks or order)")
    return out
