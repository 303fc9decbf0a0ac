"""Table 1 parameters of real HIP kernels from a profile, and their check.

Section 6 takes every kernel's block count, registers, shared memory, warps
and instruction/memory ratio from the vendor profiler, and Section 4 defines
the ratio from profiler counts: instructions over four times the global
stores plus the L1 global load misses.  This module is that front-end for
MI355X: it reads the CSV files rocprofv3 writes and turns each dispatch into
the `ko_kernel` record the model takes.

Inputs (one row per dispatch, matched by dispatch id):
  * a kernel trace (`rocprofv3 --kernel-trace`): grid and workgroup sizes, LDS
    bytes per workgroup, the kernel's VGPR and accumulation-VGPR counts;
  * counter collections (`rocprofv3 --pmc`, one pass each):
      SQ_WAVES, SQ_INSTS_VALU, SQ_INSTS_SALU       (wave instructions),
      TCP_TCC_READ_REQ_sum, TCP_TCC_WRITE_REQ_sum  (requests from the vector
                                                    L1 to L2: L1 read misses
                                                    and stores).

Readings (the paper's are for a GTX580 and its profiler):
  * n_tblk = grid / workgroup size; waves_blk = ceil(workgroup / wave size);
  * lds_blk = the trace's LDS bytes per workgroup plus the dynamic LDS bytes of
    the launch, which the caller supplies: rocprofv3's LDS_Block_Size is the
    code object's static LDS only (0 for a kernel whose LDS is all dynamic);
  * regs_thr = the registers a lane holds: VGPRs plus accumulation VGPRs from
    the trace, which on gfx950 reports them in units of two (measured: every
    kernel of this library reads half its allocated count, e.g. 20 for a
    kernel compiled to 40 VGPRs), so times `vgpr_unit` = 2;
  * R = (VALU + SALU instructions) / (4 x (L1 read misses + stores)), the
    Section 4 formula with wave instructions and 64-byte L1-L2 requests;
  * n_inst = cycles a block needs when compute bound: a wave issues one VALU
    instruction per 4 cycles (64 lanes on a 16-lane SIMD), so
    4 x (VALU + SALU) / SQ_WAVES; the model stretches it by R_B / R when
    R < R_B.
The CU placement order is not a parameter: the model's cyclic pointer over
identical CUs gives the same makespans under any relabelling of the CUs, so
MI355X's dispatch of consecutive workgroups to different XCDs (and within an
XCD to its CUs) is the same placement up to a relabelling.

    python -m paper_1511_07983_amd.profiling launch --workload 4 --set 0 --scale 4096
        runs each synthetic kernel of a set once, in index order (to be
        profiled);
    python -m paper_1511_07983_amd.profiling derive --trace T.csv --counters C1.csv [C2.csv ...]
        [--workload 4 --set 0]
        prints the derived records, and with a set the comparison with the
        parameters the synthetic kernels were built from.
"""

from __future__ import annotations

import csv
import json
import math
from collections import defaultdict

import numpy as np

INSTRUCTION_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_SALU")
MEMORY_COUNTERS = ("TCP_TCC_READ_REQ_sum", "TCP_TCC_WRITE_REQ_sum")


def _int(row, *names, default=0):
    for n in names:
        if n in row and row[n] not in ("", None):
            return int(float(row[n]))
    return default


def read_trace(path: str) -> dict:
    """Kernel-trace rows by dispatch id: name, grid, workgroup, LDS bytes,
    VGPRs, accumulation VGPRs, start and end timestamps (ns)."""
    out = {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            grid = _int(r, "Grid_Size_X", "Grid_Size") * max(1, _int(r, "Grid_Size_Y", default=1)) * \
                max(1, _int(r, "Grid_Size_Z", default=1))
            wg = _int(r, "Workgroup_Size_X", "Workgroup_Size") * max(1, _int(r, "Workgroup_Size_Y", default=1)) * \
                max(1, _int(r, "Workgroup_Size_Z", default=1))
            out[d] = {"name": r["Kernel_Name"], "grid": grid, "workgroup": wg,
                      "lds": _int(r, "LDS_Block_Size"), "vgpr": _int(r, "VGPR_Count"),
                      "agpr": _int(r, "Accum_VGPR_Count"),
                      "start": _int(r, "Start_Timestamp"), "end": _int(r, "End_Timestamp")}
    return out


def read_counters(path: str) -> list:
    """One counter pass: [(dispatch id, kernel name, {counter: value})] in
    dispatch order, each counter summed over its rows."""
    vals = defaultdict(lambda: defaultdict(float))
    names = {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            vals[d][r["Counter_Name"]] += float(r["Counter_Value"])
            names[d] = r["Kernel_Name"]
    return [(d, names[d], dict(vals[d])) for d in sorted(vals)]


def table1(trace_row: dict, counters: dict, *, wave_size: int = 64, vgpr_unit: int = 2,
           dynamic_lds: int = 0) -> dict:
    """The ko_kernel fields of one dispatch (see the module docstring)."""
    wg = trace_row["workgroup"]
    rec = {"n_tblk": trace_row["grid"] // wg, "waves_blk": -(-wg // wave_size),
           "lds_blk": trace_row["lds"] + dynamic_lds,
           "regs_thr": vgpr_unit * (trace_row["vgpr"] + trace_row["agpr"])}
    inst = sum(counters.get(c, 0.0) for c in INSTRUCTION_COUNTERS)
    mem = sum(counters.get(c, 0.0) for c in MEMORY_COUNTERS)
    waves = counters.get("SQ_WAVES", 0.0)
    rec["r"] = inst / (4.0 * mem) if mem > 0 else math.inf
    rec["r_milli"] = max(1, int(round(1000 * rec["r"]))) if math.isfinite(rec["r"]) else 1 << 30
    rec["n_inst"] = max(1, int(round(4.0 * inst / waves))) if waves > 0 else 1
    rec["duration_ns"] = trace_row["end"] - trace_row["start"]
    return rec


def derive(trace_path: str, counter_paths, *, name_filter: str | None = None, wave_size: int = 64,
           vgpr_unit: int = 2, dynamic_lds=None) -> list:
    """Derived records of the trace's dispatches (in dispatch order),
    optionally only of kernels whose name contains `name_filter`.  Each
    counter pass is its own run of the same program, so its dispatches are
    matched to the trace's by their order among the selected kernels (the
    k-th selected dispatch of the trace with the k-th of each pass).
    dynamic_lds: the dynamic LDS bytes of each selected dispatch, or None."""
    def keep(name):
        return not name_filter or name_filter in name
    trace = read_trace(trace_path)
    tsel = [d for d in sorted(trace) if keep(trace[d]["name"])]
    merged = [dict() for _ in tsel]
    for p in counter_paths:
        sel = [(d, nm, c) for d, nm, c in read_counters(p) if keep(nm)]
        if len(sel) != len(tsel):
            raise ValueError(f"{p}: {len(sel)} selected dispatches, the trace has {len(tsel)}")
        for k, (_, nm, c) in enumerate(sel):
            if nm != trace[tsel[k]]["name"]:
                raise ValueError(f"{p}: dispatch {k} is {nm}, the trace's is {trace[tsel[k]]['name']}")
            merged[k].update(c)
    if dynamic_lds is not None and len(dynamic_lds) != len(tsel):
        raise ValueError(f"{len(dynamic_lds)} dynamic LDS sizes for {len(tsel)} dispatches")
    rows = []
    for k, (d, c) in enumerate(zip(tsel, merged)):
        missing = [m for m in (*INSTRUCTION_COUNTERS, *MEMORY_COUNTERS, "SQ_WAVES") if m not in c]
        if missing:
            raise ValueError(f"dispatch {d}: counters {missing} missing")
        dyn = int(dynamic_lds[k]) if dynamic_lds is not None else 0
        rows.append({"dispatch": d, "name": trace[d]["name"],
                     **table1(trace[d], c, wave_size=wave_size, vgpr_unit=vgpr_unit, dynamic_lds=dyn)})
    return rows


def compare(derived: list, kernels, vgprs: list, scale: int, loads: list) -> dict:
    """Derived records of a synthetic set (dispatch i = kernel i) against the
    parameters the synthetic kernels were built from: the exact fields, the
    compiled register counts (rounded up to gfx950's allocation granule of 8),
    and the agreement of the derived ratio and cycle count with the drawn R
    and the drawn work F = n_inst / scale (rank correlation; log-log slope).
    Kernels with no streaming load (`loads` = 0: their F * 1000 / r_milli
    rounds to 0) must come out with R = inf and are left out of the R figures."""
    from .hw import spearman
    n = len(kernels)
    if len(derived) != n:
        raise ValueError(f"{len(derived)} profiled dispatches for {n} kernels")
    exact = {f: all(int(d[f]) == int(kernels[f][i]) for i, d in enumerate(derived))
             for f in ("n_tblk", "waves_blk", "lds_blk")}
    alloc = [-(-int(v) // 8) * 8 for v in vgprs]
    r_drawn = np.asarray(kernels["r_milli"], dtype=np.float64) / 1000.0
    r_got = np.array([d["r"] for d in derived])
    mem = np.asarray(loads) > 0
    f_drawn = np.maximum(1, np.asarray(kernels["n_inst"], dtype=np.int64) // scale).astype(np.float64)
    n_got = np.array([d["n_inst"] for d in derived], dtype=np.float64)
    out = {"kernels": n, **{f"{f}_exact": v for f, v in exact.items()},
           "regs_equal_compiled": bool(all(int(d["regs_thr"]) == a for d, a in zip(derived, alloc))),
           "no_load_kernels": int((~mem).sum()),
           "no_load_kernels_have_infinite_r": bool(np.all(np.isinf(r_got[~mem]))),
           "n_inst_spearman": spearman(n_got, f_drawn),
           "n_inst_log_slope": float(np.polyfit(np.log(f_drawn), np.log(n_got), 1)[0]),
           "n_inst_cycles_per_drawn_fma_median": float(np.median(n_got / f_drawn))}
    if mem.sum() >= 3:
        out.update({"r_spearman": spearman(r_got[mem], r_drawn[mem]),
                    "r_log_slope": float(np.polyfit(np.log(r_drawn[mem]), np.log(r_got[mem]), 1)[0]),
                    "r_over_drawn_median": float(np.median(r_got[mem] / r_drawn[mem]))})
    return out


def _launch(workload: int, set_index: int, scale: int) -> None:
    import synth
    from . import ko_hw_time_orders
    ks = synth.draw_set(workload, set_index)
    ms = ko_hw_time_orders(ks, [list(range(len(ks)))], scale, 1)
    print(json.dumps({"workload": workload, "set": set_index, "scale": scale, "kernels": len(ks),
                      "makespan_ms": float(ms[0])}), flush=True)


def main(argv=None) -> int:
    import argparse
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    la = sub.add_parser("launch")
    la.add_argument("--workload", type=int, default=4)
    la.add_argument("--set", type=int, default=0)
    la.add_argument("--scale", type=int, default=4096)
    de = sub.add_parser("derive")
    de.add_argument("--trace", required=True)
    de.add_argument("--counters", nargs="+", required=True)
    de.add_argument("--name", default=None, help="only kernels whose name contains this")
    de.add_argument("--workload", type=int, default=None)
    de.add_argument("--set", type=int, default=0)
    de.add_argument("--scale", type=int, default=4096)
    a = ap.parse_args(argv)
    if a.cmd == "launch":
        import torch
        torch.cuda.set_device(0)
        _launch(a.workload, a.set, a.scale)
        return 0
    dyn = None
    if a.workload is not None:
        import synth
        ks = synth.draw_set(a.workload, a.set)
        dyn = [int(v) for v in ks["lds_blk"]]  # the launcher's dynamic LDS, kernel i = dispatch i
    rows = derive(a.trace, a.counters, name_filter=a.name, dynamic_lds=dyn)
    for r in rows:
        print(json.dumps(r), flush=True)
    if a.workload is not None:
        import torch
        from . import ko_hw_vgprs
        torch.cuda.set_device(0)
        vgprs = [ko_hw_vgprs(int(r)) for r in ks["regs_thr"]]
        f = np.maximum(1, ks["n_inst"].astype(np.int64) // a.scale)
        loads = (f * 1000 // ks["r_milli"].astype(np.int64)).tolist()
        print(json.dumps({"comparison": True, "scale": a.scale, **compare(rows, ks, vgprs, a.scale, loads)}),
              flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
