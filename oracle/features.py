"""Oracle: the surrogate's per-kernel features and the set's area lower bound.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Per kernel (Table 1 quantities; d = block cycles as in the dispatch model,
occ = how many blocks of the kernel alone fit one CU):
  log2(N_tblk)/16, waves/wave_cu, lane registers/reg_cu, LDS/lds_cu (per block),
  log2(d)/32, log2(R/R_B)/8, occ/blk_cu, log2(1 + N_tblk/(occ N_CU))/8.
Lower bound of any order's makespan: the longest block, and for each resource
the total block-time x use divided by what all CUs hold at once (rounded up).
"""

from __future__ import annotations

import math


def _block(gpu, k):
    waves = int(k["waves_blk"])
    use = (int(k["regs_thr"]) * waves * int(gpu["wave_size"]), int(k["lds_blk"]), waves, 1)
    r, rb = int(k["r_milli"]), int(gpu["rb_milli"])
    d = -(-(int(k["n_inst"]) * max(r, rb)) // r)
    return use, d


def features(gpu, kernels):
    caps = (int(gpu["reg_cu"]), int(gpu["lds_cu"]), int(gpu["wave_cu"]), int(gpu["blk_cu"]))
    out = []
    for k in kernels:
        use, d = _block(gpu, k)
        occ = min(c // u for c, u in zip(caps, use) if u > 0)
        n_tblk = int(k["n_tblk"])
        out.append([
            math.log2(n_tblk) / 16.0,
            use[2] / caps[2],
            use[0] / caps[0],
            use[1] / caps[1],
            math.log2(d) / 32.0,
            math.log2(int(k["r_milli"]) / int(gpu["rb_milli"])) / 8.0,
            occ / caps[3],
            math.log2(1.0 + n_tblk / (occ * int(gpu["n_cu"]))) / 8.0,
        ])
    return out


def lower_bound(gpu, kernels) -> int:
    caps = (int(gpu["reg_cu"]), int(gpu["lds_cu"]), int(gpu["wave_cu"]), int(gpu["blk_cu"]))
    lb = 0
    area = [0, 0, 0, 0]
    for k in kernels:
        use, d = _block(gpu, k)
        lb = max(lb, d)
        for x in range(4):
            area[x] += int(k["n_tblk"]) * d * use[x]
    for x in range(4):
        lb = max(lb, -(-area[x] // (int(gpu["n_cu"]) * caps[x])))
    return lb
