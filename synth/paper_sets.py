"""Kernel sets shaped like the paper's experiments (Table 2), on the GTX580 model.

Input data only, like the rest of this package: integer Table 1 descriptors for
the six experiments of Table 2, to be run on ``GTX580_MODEL`` (16 SMs, 32 K
registers, 48 warps, 48 KiB shared memory and 8 blocks per SM, R_B = 4.11).

What Table 2 fixes is copied: grid and block sizes, shared memory per block and
the instruction/memory ratios R (EP 3.11, BS 11.1).  What it leaves out is an
assumption, stated here once and used everywhere:

* registers per thread: EP 24, BS 20, ES 28, SW 32;
* instructions per block (N_inst, per block, independent of grid and block
  size within a kernel type): EP 200,000, BS 150,000, ES 400,000, SW 100,000;
* the ES (electrostatics) and SW (Smith-Waterman) kernels of EpBsEsSw-8, which
  Table 2 does not describe: ES R = 20 (compute bound), 64 blocks of 256
  threads, no shared memory; SW R = 1.8 (memory bound), 32 blocks of 128
  threads, 16 KiB of shared memory;
* EpBs-6 and EpBs-6-shm: "4 warps" and "12 warps" are per-SM shares (grid / 16
  SMs x warps per block), as in EP-6-grid, where grid 16..96 with 128-thread
  blocks gives the printed 4..24: EP kernels are 16 blocks of 128 threads, BS
  kernels 32 blocks of 192 threads.

The makespans these sets give are model cycles, not the GTX580 milliseconds of
Table 3, which were measured on the paper's real kernels.
"""

from __future__ import annotations

import numpy as np

from . import GTX580_MODEL, KERNEL_DTYPE

MODEL = GTX580_MODEL

# per kernel type: R in thousandths, registers per thread, instructions per block
EP = (3110, 24, 200_000)
BS = (11100, 20, 150_000)
ES = (20000, 28, 400_000)
SW = (1800, 32, 100_000)


def _kernel(kind, grid: int, block: int, shm_bytes: int):
    r_milli, regs, n_inst = kind
    return (grid, n_inst, shm_bytes, block // 32, regs, r_milli)


def _set(rows) -> np.ndarray:
    out = np.zeros(len(rows), dtype=KERNEL_DTYPE)
    for i, (n_tblk, n_inst, lds, waves, regs, r_milli) in enumerate(rows):
        out[i] = (n_tblk, n_inst, lds, waves, regs, r_milli)
    return out


K = 1024
EXPERIMENTS = {
    "EP-6-shm": _set([_kernel(EP, 16, 128, s * K) for s in (8, 16, 24, 32, 40, 48)]),
    "EP-6-grid": _set([_kernel(EP, g, 128, 0) for g in (16, 32, 48, 64, 80, 96)]),
    "BS-6-blk": _set([_kernel(BS, 32, b, 0) for b in (64, 128, 256, 512, 768, 1024)]),
    "EpBs-6": _set([_kernel(EP, 16, 128, 0)] * 3 + [_kernel(BS, 32, 192, 0)] * 3),
    "EpBs-6-shm": _set([_kernel(EP, 16, 128, s * K) for s in (16, 24, 48)]
                       + [_kernel(BS, 32, 192, s * K) for s in (16, 24, 48)]),
    "EpBsEsSw-8": _set([_kernel(EP, 16, 128, 0)] * 2 + [_kernel(BS, 32, 192, 0)] * 2
                       + [_kernel(ES, 64, 256, 0)] * 2 + [_kernel(SW, 32, 128, 16 * K)] * 2),
}
