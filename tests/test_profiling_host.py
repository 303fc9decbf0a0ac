"""The profiling front-end on hand-made rocprofv3 CSV files (no GPU): Table 1
fields from the kernel trace, R and n_inst from the counters by the formulas
of the module docstring, dispatch matching across counter passes.

Hand-worked case: a kernel with grid 65,536 and workgroup 256 (256 blocks of
4 waves), 8,192 static LDS bytes, a trace count of 40 VGPRs + 8 accumulation
VGPRs (in units of two: 96 registers per lane); its counters are
1,000 VALU + 200 SALU wave instructions over 1,024 waves, and 100 L1 read
misses + 50 stores.  So R = 1,200 / (4 x 150) = 2.0 (r_milli 2,000) and
n_inst = 4 x 1,200 / 1,024 = 4.69 -> 5 cycles."""

import csv

import pytest

pytest.importorskip("torch")
from paper_1511_07983_amd import profiling  # noqa: E402

TRACE_FIELDS = ["Kind", "Dispatch_Id", "Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z",
                "Workgroup_Size_X", "Workgroup_Size_Y", "Workgroup_Size_Z", "LDS_Block_Size", "VGPR_Count",
                "Accum_VGPR_Count", "Start_Timestamp", "End_Timestamp"]


def _write(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _trace(path):
    _write(path, TRACE_FIELDS, [
        dict(Kind="KERNEL_DISPATCH", Dispatch_Id=1, Kernel_Name="fill", Grid_Size_X=1024, Grid_Size_Y=1,
             Grid_Size_Z=1, Workgroup_Size_X=256, Workgroup_Size_Y=1, Workgroup_Size_Z=1, LDS_Block_Size=0,
             VGPR_Count=8, Accum_VGPR_Count=0, Start_Timestamp=100, End_Timestamp=200),
        dict(Kind="KERNEL_DISPATCH", Dispatch_Id=2, Kernel_Name="work_kernel<4>", Grid_Size_X=65536,
             Grid_Size_Y=1, Grid_Size_Z=1, Workgroup_Size_X=256, Workgroup_Size_Y=1, Workgroup_Size_Z=1,
             LDS_Block_Size=8192, VGPR_Count=40, Accum_VGPR_Count=8, Start_Timestamp=1000, End_Timestamp=5000),
    ])


def _pass(path, values, first_id=7):
    rows = []
    for k, (name, counters) in enumerate(values):
        for c, v in counters.items():
            rows.append(dict(Dispatch_Id=first_id + k, Kernel_Name=name, Counter_Name=c, Counter_Value=v))
    _write(path, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], rows)


def test_table1_from_trace_and_counters(tmp_path):
    _trace(tmp_path / "trace.csv")
    # two passes of their own runs (dispatch ids differ from the trace's); the
    # TCP counter comes as two rows that add up
    _pass(tmp_path / "sq.csv", [("fill", {"SQ_WAVES": 4, "SQ_INSTS_VALU": 9, "SQ_INSTS_SALU": 1}),
                                ("work_kernel<4>", {"SQ_WAVES": 1024, "SQ_INSTS_VALU": 1000, "SQ_INSTS_SALU": 200})])
    with open(tmp_path / "tcp.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writerow([30, "fill", "TCP_TCC_READ_REQ_sum", 3])
        w.writerow([30, "fill", "TCP_TCC_WRITE_REQ_sum", 1])
        w.writerow([31, "work_kernel<4>", "TCP_TCC_READ_REQ_sum", 60])
        w.writerow([31, "work_kernel<4>", "TCP_TCC_READ_REQ_sum", 40])
        w.writerow([31, "work_kernel<4>", "TCP_TCC_WRITE_REQ_sum", 50])
    rows = profiling.derive(str(tmp_path / "trace.csv"), [str(tmp_path / "sq.csv"), str(tmp_path / "tcp.csv")],
                            name_filter="work_kernel")
    assert len(rows) == 1
    r = rows[0]
    assert (r["n_tblk"], r["waves_blk"], r["lds_blk"], r["regs_thr"]) == (256, 4, 8192, 96)
    assert r["r"] == 2.0 and r["r_milli"] == 2000
    assert r["n_inst"] == 5
    assert r["duration_ns"] == 4000
    # the launch's dynamic LDS adds to the trace's static bytes
    rows = profiling.derive(str(tmp_path / "trace.csv"), [str(tmp_path / "sq.csv"), str(tmp_path / "tcp.csv")],
                            name_filter="work_kernel", dynamic_lds=[4096])
    assert rows[0]["lds_blk"] == 8192 + 4096
    # both kernels, in dispatch order
    rows = profiling.derive(str(tmp_path / "trace.csv"), [str(tmp_path / "sq.csv"), str(tmp_path / "tcp.csv")])
    assert [x["name"] for x in rows] == ["fill", "work_kernel<4>"]
    assert rows[0]["n_tblk"] == 4 and rows[0]["r"] == 10 / 16


def test_mismatched_passes_are_refused(tmp_path):
    _trace(tmp_path / "trace.csv")
    _pass(tmp_path / "sq.csv", [("work_kernel<4>", {"SQ_WAVES": 1, "SQ_INSTS_VALU": 1, "SQ_INSTS_SALU": 1})])
    with pytest.raises(ValueError):
        profiling.derive(str(tmp_path / "trace.csv"), [str(tmp_path / "sq.csv")])
