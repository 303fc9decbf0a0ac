"""Oracle: the dispatch model advanced one cycle at a time.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A second, independent formulation of the block-dispatch model of Section 2
(and the per-SM limits of Table 1), for brute-force cross-checks of the
event-driven oracle on tiny sets.  Instead of jumping from one finish time to
the next, it visits every cycle t = 0, 1, 2, ...: first every block whose
finish cycle is t gives its resources back, then blocks are taken from the
front of the launch-ordered block stream and placed round-robin (the first CU
at or after the cyclic pointer that has room in all four resources) until the
front block fits nowhere.  The makespan is the first cycle at which nothing is
left to place and nothing runs.  Durations must be small: the cost is linear
in the makespan.
"""

from __future__ import annotations


def _per_block(gpu, k):
    waves = int(k["waves_blk"])
    use = (int(k["regs_thr"]) * waves * int(gpu["wave_size"]), int(k["lds_blk"]), waves, 1)
    r, rb = int(k["r_milli"]), int(gpu["rb_milli"])
    dur = -(-(int(k["n_inst"]) * max(r, rb)) // r)
    return use, dur


def tick_makespan(gpu, kernels, order, max_cycles: int = 10_000_000) -> int:
    n_cu = int(gpu["n_cu"])
    caps = (int(gpu["reg_cu"]), int(gpu["lds_cu"]), int(gpu["wave_cu"]), int(gpu["blk_cu"]))
    info = [_per_block(gpu, k) for k in kernels]
    stream = [k for k in order for _ in range(int(kernels[k]["n_tblk"]))]
    free = [list(caps) for _ in range(n_cu)]
    resident = []  # (finish cycle, cu, kernel)
    head, ptr = 0, 0
    for t in range(max_cycles):
        still = []
        for fin, cu, k in resident:
            if fin == t:
                for x in range(4):
                    free[cu][x] += info[k][0][x]
            else:
                still.append((fin, cu, k))
        resident = still
        while head < len(stream):
            k = stream[head]
            use = info[k][0]
            target = None
            for i in range(n_cu):
                c = (ptr + i) % n_cu
                if all(free[c][x] >= use[x] for x in range(4)):
                    target = c
                    break
            if target is None:
                break
            for x in range(4):
                free[target][x] -= use[x]
            resident.append((t + info[k][1], target, k))
            ptr = (target + 1) % n_cu
            head += 1
        if head == len(stream) and not resident:
            return t
    raise RuntimeError("tick simulation did not finish")


def tick_contended_makespan(gpu, kernels, order, mem_blocks: int, max_cycles: int = 10_000_000) -> int:
    """The memory-contention model (Section 4; see ``contended_makespans``)
    advanced one cycle at a time: each cycle every resident block gains
    floor(65536 * 1024 * B / U) units of progress (65536 when U <= 1024 * B),
    U being the sum of the resident blocks' memory shares
    ceil(1024 * min(R_i, R_B) / R_i); a block ends at the first cycle at which
    its progress reaches 65536 times its duration; releases come before
    placement."""
    n_cu = int(gpu["n_cu"])
    caps = (int(gpu["reg_cu"]), int(gpu["lds_cu"]), int(gpu["wave_cu"]), int(gpu["blk_cu"]))
    info = [_per_block(gpu, k) for k in kernels]
    rb = int(gpu["rb_milli"])
    share = [-(-1024 * min(int(k["r_milli"]), rb) // int(k["r_milli"])) for k in kernels]
    stream = [k for k in order for _ in range(int(kernels[k]["n_tblk"]))]
    free = [list(caps) for _ in range(n_cu)]
    resident = []  # [progress so far, progress needed, cu, kernel]
    head, ptr = 0, 0
    rate = 65536
    for t in range(max_cycles):
        if t > 0:
            for b in resident:
                b[0] += rate
        still = []
        for b in resident:
            if b[0] >= b[1]:
                for x in range(4):
                    free[b[2]][x] += info[b[3]][0][x]
            else:
                still.append(b)
        resident = still
        while head < len(stream):
            k = stream[head]
            use = info[k][0]
            target = None
            for i in range(n_cu):
                c = (ptr + i) % n_cu
                if all(free[c][x] >= use[x] for x in range(4)):
                    target = c
                    break
            if target is None:
                break
            for x in range(4):
                free[target][x] -= use[x]
            resident.append([0, info[k][1] * 65536, target, k])
            ptr = (target + 1) % n_cu
            head += 1
        if head == len(stream) and not resident:
            return t
        used = sum(share[b[3]] for b in resident)
        rate = 65536 if used <= 1024 * mem_blocks else (65536 * 1024 * mem_blocks) // used
    raise RuntimeError("tick simulation did not finish")
