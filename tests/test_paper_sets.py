"""The paper-shaped kernel sets (synth/paper_sets.py) reproduce what Table 2
fixes and fit the GTX580 model of the experimental section."""

import numpy as np

import oracle
from synth import paper_sets

M = paper_sets.MODEL


def _col(name, field):
    return [int(x) for x in paper_sets.EXPERIMENTS[name][field]]


def test_table2_constants():
    # EP-6-shm: 16 x 128 threads, R = 3.11, shared memory 8K..48K
    assert _col("EP-6-shm", "n_tblk") == [16] * 6 and _col("EP-6-shm", "waves_blk") == [4] * 6
    assert _col("EP-6-shm", "lds_blk") == [k * 1024 for k in (8, 16, 24, 32, 40, 48)]
    assert set(_col("EP-6-shm", "r_milli")) == {3110}
    # EP-6-grid: grids 16..96 of 128 threads, no shared memory
    assert _col("EP-6-grid", "n_tblk") == [16, 32, 48, 64, 80, 96]
    assert set(_col("EP-6-grid", "lds_blk")) == {0}
    # BS-6-blk: 32 blocks of 64..1024 threads, R = 11.1
    assert _col("BS-6-blk", "waves_blk") == [b // 32 for b in (64, 128, 256, 512, 768, 1024)]
    assert set(_col("BS-6-blk", "n_tblk")) == {32} and set(_col("BS-6-blk", "r_milli")) == {11100}
    # EpBs-6-shm: shared memory 16K, 24K, 48K for each kind
    assert _col("EpBs-6-shm", "lds_blk") == [k * 1024 for k in (16, 24, 48, 16, 24, 48)]
    assert len(paper_sets.EXPERIMENTS["EpBsEsSw-8"]) == 8


def test_per_sm_warp_shares_match_the_printed_columns():
    """Table 2 prints EP-6-grid's warps as 4..24 and EpBs-6's as 4 and 12: the
    per-SM share ceil(grid / 16) x warps per block."""
    def share(name):
        ks = paper_sets.EXPERIMENTS[name]
        return [int(-(-t // M.n_cu) * w) for t, w in zip(ks["n_tblk"], ks["waves_blk"])]
    assert share("EP-6-grid") == [4, 8, 12, 16, 20, 24]
    assert share("EpBs-6") == [4, 4, 4, 12, 12, 12]


def test_every_block_fits_an_empty_sm():
    g = M.as_dict()
    for name, ks in paper_sets.EXPERIMENTS.items():
        use, dur = oracle.derive(g, ks)
        for u in use:
            assert u[0] <= M.reg_cu and u[1] <= M.lds_cu and u[2] <= M.wave_cu, name
        assert (np.asarray(dur) > 0).all()
