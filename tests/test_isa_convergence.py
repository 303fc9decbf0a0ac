"""Compiled gfx950 assembly: wave collectives run with every lane active.

The simulate, lane-simulate, reduce and surrogate kernels exchange values
between the lanes of a wave (readlane, readfirstlane, shuffles).  These tests compile the
library sources to assembly with the build's own flags (CPU only, nothing is
launched) and check, with the dataflow analysis of tests/isa_convergence.py,
that no cross-lane instruction of those kernels can execute while some lanes
are masked off, and that the simulate kernels contain no lane-divergent loop
at all (every loop of theirs is uniform by construction).

A compile-only snippet with a lane-0 fetch at the top of a persistent loop and
a lane-0 store at its bottom shows that the analysis reports that shape: the
compiler threads the store's branch around the fetch, and the other lanes go
round the loop without lane 0.
"""

import importlib.util
import os
import shutil
import subprocess

import pytest

import isa_convergence as ic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1511_07983_amd", "csrc")

pytestmark = pytest.mark.skipif(
    shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
    reason="hipcc is needed to compile the kernels to assembly")


def _build_module():
    spec = importlib.util.spec_from_file_location(
        "ko_build", os.path.join(ROOT, "paper_1511_07983_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _asm(src, out, extra_inc=()):
    b = _build_module()
    cmd = [b.HIPCC, *b.COMMON, *b.DEVICE, *b.EXTRA.get(os.path.basename(src), []),
           *[f"-I{d}" for d in extra_inc], "--cuda-device-only", "-S", src, "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    with open(out) as f:
        return f.read()


@pytest.fixture(scope="module")
def sim_report(tmp_path_factory):
    d = tmp_path_factory.mktemp("isa")
    return ic.check(_asm(os.path.join(CSRC, "ko_sim.hip"), str(d / "ko_sim.s")))


@pytest.fixture(scope="module")
def lanes_report(tmp_path_factory):
    d = tmp_path_factory.mktemp("isa")
    return ic.check(_asm(os.path.join(CSRC, "ko_lanes.hip"), str(d / "ko_lanes.s")))


@pytest.fixture(scope="module")
def rounds_report(tmp_path_factory):
    d = tmp_path_factory.mktemp("isa")
    return ic.check(_asm(os.path.join(CSRC, "ko_rounds.hip"), str(d / "ko_rounds.s")))


@pytest.fixture(scope="module")
def nn_report(tmp_path_factory):
    d = tmp_path_factory.mktemp("isa")
    return ic.check(_asm(os.path.join(CSRC, "ko_nn.hip"), str(d / "ko_nn.s")))


@pytest.fixture(scope="module")
def select_report(tmp_path_factory):
    d = tmp_path_factory.mktemp("isa")
    return ic.check(_asm(os.path.join(CSRC, "ko_select.hip"), str(d / "ko_select.s")))


def _pick(report, needle):
    names = [n for n in report if needle in n]
    assert names, f"no kernel matching {needle} in {sorted(report)}"
    return names


@pytest.mark.parametrize("needle", ["simulate_kernelILi1E", "simulate_kernelILi2E", "simulate_kernelILi4E"])
def test_simulate_collectives_full_exec(sim_report, needle):
    for name in _pick(sim_report, needle):
        bad, div_loops = sim_report[name]
        assert bad == [], (name, bad[:5])
        assert div_loops == 0, (name, div_loops)


@pytest.mark.parametrize("needle", ["simulate_lanes_kernelILi12ELi8E", "simulate_lanes_kernelILi12ELi10E",
                                    "simulate_lanes_kernelILi16ELi12E", "simulate_lanes_kernelILi20ELi16E"])
def test_lane_kernels_collectives_full_exec(lanes_report, needle):
    """The lane kernels diverge by design (each lane runs its own order), so
    their loops may be lane-divergent; every wave operation (item fetch,
    statistics shuffles, overflow ballot) must still see all lanes."""
    for name in _pick(lanes_report, needle):
        bad, _ = lanes_report[name]
        assert bad == [], (name, bad[:5])


@pytest.mark.parametrize("needle", ["rounds_kernelILi1E", "rounds_kernelILi2E", "rounds_kernelILi3E",
                                    "rounds_kernelILi4E"])
def test_rounds_collectives_full_exec(rounds_report, needle):
    """The round-synchronous kernel branches on wave-uniform values only: no
    collective under a partial exec mask and no lane-divergent loop."""
    for name in _pick(rounds_report, needle):
        bad, div_loops = rounds_report[name]
        assert bad == [], (name, bad[:5])
        assert div_loops == 0, (name, div_loops)


def test_spill_kernel_collectives_full_exec(sim_report):
    for name in _pick(sim_report, "spill_kernel"):
        bad, div_loops = sim_report[name]
        assert bad == [], (name, bad[:5])


@pytest.mark.parametrize("needle", ["reduce_kernel", "reduce_wide_kernel"])
def test_reduce_collectives_full_exec(sim_report, needle):
    for name in _pick(sim_report, needle):
        bad, _ = sim_report[name]
        assert bad == [], (name, bad[:5])


def test_sort_scatter_collectives_full_exec(select_report):
    """The radix sort's scatter ranks lanes by digit with ballots: every lane
    of the wavefront must take part in them, also past the end of the data."""
    for name in _pick(select_report, "sort_scatter_kernel"):
        bad, _ = select_report[name]
        assert bad == [], (name, bad[:5])



@pytest.mark.parametrize("needle", ["out_forward_kernel", "head_kernel", "colsum_multi_kernel", "finish_kernel",
                                    "dz1_kernel", "pool_kernel", "gather_pool_kernel", "within_set_rank_kernel",
                                    "gemm_bf16_kernel", "gemm_nt_kernel", "panel_gemm_kernel", "score_kernel",
                                    "score_split_kernel", "split_table_kernel"])
def test_surrogate_collectives_full_exec(nn_report, needle):
    for name in _pick(nn_report, needle):
        bad, _ = nn_report[name]
        assert bad == [], (name, bad[:5])


THREADED_LOOP = r"""
#include <hip/hip_runtime.h>
#include <stdint.h>
__global__ __launch_bounds__(64) void threaded_loop(unsigned long long *counter, uint64_t n_items,
                                                     const uint32_t *table, uint64_t *out)
{
    const uint32_t lane = __lane_id();
    for (;;) {
        uint64_t item = 0;
        if (lane == 0)
            item = atomicAdd(counter, 1ull);
        item = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(item >> 32)) << 32) |
               __builtin_amdgcn_readfirstlane((uint32_t)item);
        if (item >= n_items)
            break;
        uint32_t v = table[(item * 64 + lane) % 4096];
        uint32_t first = __builtin_amdgcn_readlane(v, 0);
        uint64_t acc = 0;
        for (uint32_t j = 0; j < 4; j++)
            acc += __builtin_amdgcn_readlane(v + first, j);
        if (lane == 0)
            out[item] = acc;
    }
}
"""


def test_analysis_reports_threaded_lane0_loop(tmp_path):
    src = tmp_path / "threaded.hip"
    src.write_text(THREADED_LOOP)
    report = ic.check(_asm(str(src), str(tmp_path / "threaded.s")))
    (name,) = _pick(report, "threaded_loop")
    bad, div_loops = report[name]
    assert div_loops > 0 and bad, "the lane-0 fetch/store loop should compile to a divergent cycle"


def test_analysis_accepts_branch_free_fetch(tmp_path):
    src = tmp_path / "fixed.hip"
    src.write_text(THREADED_LOOP.replace(
        """        uint64_t item = 0;
        if (lane == 0)
            item = atomicAdd(counter, 1ull);
""", """        uint64_t item = atomicAdd(counter, lane == 0 ? 1ull : 0ull);
"""))
    report = ic.check(_asm(str(src), str(tmp_path / "fixed.s")))
    (name,) = _pick(report, "threaded_loop")
    bad, div_loops = report[name]
    assert bad == [] and div_loops == 0, (bad[:5], div_loops)


SCALAR_SOURCE_ASM = """
kern:
	s_and_saveexec_b64 s[4:5], vcc
	v_sub_co_u32_e64 v0, s[6:7], s2, 1
	v_readfirstlane_b32 s1, v0
	s_or_b64 exec, exec, s[4:5]
	s_endpgm
.Lfunc_end0:
"""


def test_readfirstlane_of_a_scalar_computed_value_is_accepted():
    """Under a partial exec mask, a readfirstlane of n - 1 computed from an SGPR
    reads the same value in every active lane."""
    (bad, _), = ic.check(SCALAR_SOURCE_ASM).values()
    assert bad == []


@pytest.mark.parametrize("define", ["v_mbcnt_lo_u32_b32 v0, -1, 0",
                                    "v_add_u32_e32 v0, s2, v7",
                                    "v_cndmask_b32_e64 v0, 0, 1, s[6:7]"])
def test_readfirstlane_of_a_lane_varying_value_is_reported(define):
    asm = SCALAR_SOURCE_ASM.replace("v_sub_co_u32_e64 v0, s[6:7], s2, 1", define)
    (bad, _), = ic.check(asm).values()
    assert [t for _, t in bad] == ["v_readfirstlane_b32 s1, v0"]


IF_ELSE_ASM = """
kern:
	v_cmp_lt_u32_e32 vcc, s4, v0
	s_and_saveexec_b64 s[4:5], vcc
	s_xor_b64 s[4:5], exec, s[4:5]
	v_lshrrev_b32_e32 v18, 2, v0
	s_or_saveexec_b64 s[14:15], s[4:5]
	s_xor_b64 exec, exec, s[14:15]
	s_cbranch_execz .LBB0_2
	v_mov_b32_e32 v1, 1
	ds_bpermute_b32 v2, v3, v1
.LBB0_2:
	s_or_b64 exec, exec, s[14:15]
	ds_bpermute_b32 v2, v3, v1
	s_endpgm
.Lfunc_end0:
"""


def test_if_else_restores_exec():
    """The if/else idiom (then-lanes saved, the complement taken with xor, the
    else entered with or_saveexec, exec restored with or): a cross-lane
    instruction inside the else-block runs with lanes masked off, the one
    after the construct with all lanes."""
    (bad, _), = ic.check(IF_ELSE_ASM).values()
    assert [i for i, _ in bad] == [bad[0][0]] and len(bad) == 1, bad
    lines = IF_ELSE_ASM.strip().splitlines()
    inside = next(k for k, l in enumerate(lines) if "ds_bpermute" in l)
    assert "ds_bpermute" in lines[inside] and bad[0][1] == lines[inside].strip()
