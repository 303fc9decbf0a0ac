"""Seeded synthetic kernel sets and GPU models.

This module only draws inputs: integer kernel descriptors (the per-kernel
parameters of Table 1) and the constant GPU models they run on.  It holds no
part of the dispatch model, the ordering rule or any statistic; both the CPU
oracle and the HIP library read what it produces.

Every set is drawn from its own generator,
``numpy.random.Generator(PCG64(SeedSequence([20151123, config, set])))``, so a
set can be regenerated alone.  Per kernel the draws are, in this order:

1. ``n_tblk``   uniform integer in ``[tblk_lo, tblk_hi]``
2. ``waves_blk`` uniform choice of {2, 4, 8}
3. ``regs_thr`` uniform integer in [16, 64]
4. ``lds_blk``  4096 times a uniform integer in [0, 12]   (0 .. 48 KiB)
5. ``n_inst``   round(10 ** U(4, 6))                       (log-uniform 1e4 .. 1e6)
6. ``r_milli``  round(1000 * 10 ** U(log10 0.5, log10 50)) (R log-uniform 0.5 .. 50)

For the batched workload the set size ``n`` is drawn first, uniform in
``[n_lo, n_hi]``.  Real-valued R is stored in thousandths (``r_milli``) so
that every descriptor is an integer.
"""

from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass

import numpy as np

ROOT_SEED = 20151123

KERNEL_FIELDS = ("n_tblk", "n_inst", "lds_blk", "waves_blk", "regs_thr", "r_milli")
KERNEL_DTYPE = np.dtype([(f, np.int64) for f in KERNEL_FIELDS])

GPU_FIELDS = ("n_cu", "wave_size", "wave_cu", "blk_cu", "reg_cu", "lds_cu", "rb_milli")


@dataclass(frozen=True)
class GpuModel:
    """Per-CU limits of Table 1 (first three rows) for one modelled GPU.

    ``reg_cu`` counts lane registers (4-byte VGPR slots) per CU, ``lds_cu`` is
    bytes of shared memory / LDS per CU, ``wave_cu`` and ``blk_cu`` are the
    resident wave and block limits, ``rb_milli`` is the balanced
    instruction/memory ratio R_B in thousandths.
    """

    n_cu: int
    wave_size: int
    wave_cu: int
    blk_cu: int
    reg_cu: int
    lds_cu: int
    rb_milli: int

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f in GPU_FIELDS}


# The 16-SM model of the tiny workload: 64 K registers, 64 KiB shared memory,
# 64 warps and 16 blocks per SM, 32-wide warps, R_B = 8.
SMALL_MODEL = GpuModel(n_cu=16, wave_size=32, wave_cu=64, blk_cu=16,
                       reg_cu=65536, lds_cu=65536, rb_milli=8000)

# MI355X-shaped model: 256 CUs, 512 KiB VGPR file per CU (131072 four-byte
# lane registers), 160 KiB LDS, 32 waves and 32 blocks per CU, wave64, R_B = 10.
MI355X_MODEL = GpuModel(n_cu=256, wave_size=64, wave_cu=32, blk_cu=32,
                        reg_cu=131072, lds_cu=163840, rb_milli=10000)

# The platform of the paper's experiments (Section "Experimental Results"):
# 16 SMs, 32 K registers, 48 warps, 48 KiB shared memory, 8 blocks per SM,
# R_B = 4.11.  Used only for paper-shaped examples.
GTX580_MODEL = GpuModel(n_cu=16, wave_size=32, wave_cu=48, blk_cu=8,
                        reg_cu=32768, lds_cu=49152, rb_milli=4110)


@dataclass(frozen=True)
class Workload:
    """One named synthetic workload: how many sets, of what size, on which model."""

    index: int
    name: str
    model: GpuModel
    n_sets: int
    n_lo: int
    n_hi: int
    tblk_lo: int
    tblk_hi: int
    set_base: int = 0  # first set index (seed component) of this workload


WORKLOADS = {
    0: Workload(0, "tiny-n6-16cu", SMALL_MODEL, 1, 6, 6, 8, 128),
    1: Workload(1, "full-enum-n10-mi355x", MI355X_MODEL, 1, 10, 10, 64, 2048),
    2: Workload(2, "batch-4096-n4to9-mi355x", MI355X_MODEL, 4096, 4, 9, 64, 2048),
    3: Workload(3, "surrogate-train-n12-mi355x", MI355X_MODEL, 512, 12, 12, 64, 2048),
    # held-out sets of the n=12 workload use set indices disjoint from training
    13: Workload(3, "surrogate-heldout-n12-mi355x", MI355X_MODEL, 16, 12, 12, 64, 2048,
                 set_base=100000),
    4: Workload(4, "search-n16-mi355x", MI355X_MODEL, 1024, 16, 16, 256, 8192),
    14: Workload(4, "search-train-n16-mi355x", MI355X_MODEL, 512, 16, 16, 256, 8192,
                 set_base=100000),
    # a small surrogate workload (n=8, 40,320 orders per set: exact quantiles
    # by full enumeration are cheap), for tests of the learned search
    5: Workload(5, "surrogate-train-n8-mi355x", MI355X_MODEL, 256, 8, 8, 64, 2048),
    15: Workload(5, "surrogate-heldout-n8-mi355x", MI355X_MODEL, 16, 8, 8, 64, 2048,
                 set_base=100000),
}


def rng_for(config: int, set_index: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence([ROOT_SEED, int(config), int(set_index)])))


def draw_kernels(rng: np.random.Generator, n: int, tblk_lo: int, tblk_hi: int) -> np.ndarray:
    """Draw ``n`` kernel descriptors from ``rng`` in the documented order."""
    out = np.zeros(n, dtype=KERNEL_DTYPE)
    lo_r, hi_r = math.log10(0.5), math.log10(50.0)
    for i in range(n):
        out["n_tblk"][i] = rng.integers(tblk_lo, tblk_hi + 1)
        out["waves_blk"][i] = (2, 4, 8)[int(rng.integers(0, 3))]
        out["regs_thr"][i] = rng.integers(16, 65)
        out["lds_blk"][i] = 4096 * int(rng.integers(0, 13))
        out["n_inst"][i] = int(round(10.0 ** rng.uniform(4.0, 6.0)))
        out["r_milli"][i] = int(round(1000.0 * 10.0 ** rng.uniform(lo_r, hi_r)))
    return out


def draw_set(workload: int, set_index: int) -> np.ndarray:
    """The ``set_index``-th kernel set of a workload (0-based, before ``set_base``)."""
    w = WORKLOADS[workload]
    rng = rng_for(w.index, w.set_base + set_index)
    n = w.n_lo if w.n_lo == w.n_hi else int(rng.integers(w.n_lo, w.n_hi + 1))
    return draw_kernels(rng, n, w.tblk_lo, w.tblk_hi)


def draw_sets(workload: int, first: int = 0, count: int | None = None):
    """Concatenated kernels and CSR offsets for sets ``first .. first+count-1``.

    Returns ``(kernels, offsets)`` with ``kernels`` a KERNEL_DTYPE array and
    ``offsets`` an int32 array of length count+1.
    """
    w = WORKLOADS[workload]
    if count is None:
        count = w.n_sets - first
    sets = [draw_set(workload, first + s) for s in range(count)]
    offsets = np.zeros(count + 1, dtype=np.int32)
    offsets[1:] = np.cumsum([len(s) for s in sets])
    kernels = np.concatenate(sets) if sets else np.zeros(0, dtype=KERNEL_DTYPE)
    return kernels, offsets


def digest(kernels: np.ndarray, offsets: np.ndarray) -> str:
    """SHA-256 of the canonical little-endian bytes of a batch of sets."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(offsets, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(kernels).astype(KERNEL_DTYPE.newbyteorder("<")).tobytes())
    return h.hexdigest()


def random_tiny_set(rng: np.random.Generator, n: int, model: GpuModel,
                    tblk_hi: int = 6, inst_hi: int = 12, equal_d: bool = False) -> np.ndarray:
    """A small random set whose blocks always fit an empty CU of ``model``.

    Used for brute-force cross-checks: block counts, instruction counts and
    hence durations are kept small so that tick-by-tick simulation stays cheap.
    """
    out = np.zeros(n, dtype=KERNEL_DTYPE)
    for i in range(n):
        waves = int(rng.integers(1, max(2, model.wave_cu // 2) + 1))
        waves = min(waves, model.wave_cu)
        max_regs = max(1, model.reg_cu // (waves * model.wave_size))
        out["n_tblk"][i] = rng.integers(1, tblk_hi + 1)
        out["waves_blk"][i] = waves
        out["regs_thr"][i] = rng.integers(1, min(max_regs, 64) + 1)
        out["lds_blk"][i] = int(rng.integers(0, model.lds_cu + 1))
        out["n_inst"][i] = 5 if equal_d else int(rng.integers(1, inst_hi + 1))
        out["r_milli"][i] = model.rb_milli if equal_d else int(rng.integers(200, 3 * model.rb_milli))
    return out
