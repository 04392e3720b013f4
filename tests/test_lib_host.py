"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol the header declares, plans calls, and rejects bad arguments
before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_1508_03167_amd as M

    return M, M.lib()


def test_exports_every_declared_symbol():
    M, L = _lib()
    hdr = open(os.path.join(ROOT, "include", "mergeshuffle.h")).read()
    names = set(re.findall(r"^\s*(?:int|uint64_t|uint32_t|const char\*)\s+(ms_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 14
    for nm in names:
        assert hasattr(L, nm), nm
    from paper_1508_03167_amd._lib import SYMBOLS

    assert set(SYMBOLS) == names


def test_plan_matches_the_driver_partition():
    M, _ = _lib()
    p = M.plan(1 << 20)
    assert (p["levels"], p["leaves"], p["leaf_B"]) == (8, 256, 4096)
    assert p["lds_levels"] + p["hbm_levels"] == 8
    p = M.plan(1 << 30)
    # a 64 KiB super-block holds four leaves of 4096 u32: two merge levels in LDS
    assert p["levels"] == 18 and p["lds_levels"] == 2 and p["hbm_levels"] == 16
    assert p["scratch_bytes"] >= 4 << 30
    p = M.plan(1 << 27, 16)
    assert p["levels"] == 15
    p = M.plan(4096)
    assert p["levels"] == 0 and p["hbm_levels"] == 0 and p["scratch_bytes"] == 0
    p = M.plan(8193)
    assert p["levels"] == 1
    p = M.plan(100000, 4, leaf_B=16, hbm_only=True)
    assert p["lds_levels"] == 0 and p["levels"] == p["hbm_levels"]


def test_leaves_of_cutoff_plus_one_plan_for_every_element_size():
    # the partition [n*i/q, n*(i+1)/q) makes leaves of cutoff + 1 elements for
    # most n that are not powers of two (Appendix A.2); every element size
    # must accept them
    M, _ = _lib()
    for n in (8193, (1 << 20) + 7, (1 << 27) + 5, 4096 * 2**9 + 300, (1 << 32) - (1 << 16)):
        for eb in (4, 8, 16):
            p = M.plan(n, eb)
            assert -(-n // p["leaves"]) <= 4097


def test_levels_per_pass_default_and_knob():
    # default: 3 levels per pass, 4 from 13 HBM levels on (for 4-byte
    # elements only when 3 does not divide them); the passes split the
    # levels as evenly as possible
    M, _ = _lib()
    for k in range(17, 33):
        n = min(1 << k, (1 << 32) - (1 << 17))
        for eb in (4, 8, 16):
            p = M.plan(n, eb)
            h = p["hbm_levels"]
            lpp = 4 if h >= 13 and (eb != 4 or h % 3) else 3
            passes = -(-h // lpp)
            assert p["hbm_passes"] == passes, (k, eb, p)
            assert p["max_levels_per_pass"] == (-(-h // passes) if h else 0), (k, eb, p)
    p = M.plan(1 << 30)
    assert (p["hbm_levels"], p["hbm_passes"], p["max_levels_per_pass"]) == (16, 4, 4)
    p = M.plan(1 << 26)
    assert (p["hbm_levels"], p["hbm_passes"], p["max_levels_per_pass"]) == (12, 4, 3)
    for lpp in (1, 2, 3, 4, 9):
        p = M.plan(1 << 30, levels_per_pass=lpp)
        assert p["hbm_passes"] == -(-16 // min(lpp, 4))
    p = M.plan(1 << 30, one_level_passes=True)
    assert p["hbm_passes"] == 16 and p["max_levels_per_pass"] == 1


def test_rejects_bad_arguments_without_a_device():
    M, L = _lib()
    assert L.ms_shuffle(None, 10, 4, 1, None) == -1          # null pointer, n > 0
    assert L.ms_shuffle(ctypes.c_void_p(16), 10, 12, 1, None) == -2   # element size
    assert L.ms_shuffle(ctypes.c_void_p(16), 1 << 33, 4, 1, None) == -2  # n too large
    assert L.ms_shuffle(ctypes.c_void_p(18), 10, 4, 1, None) == -1    # misaligned
    cfg = M._lib.MSConfig(5000, 0, 0, 0)
    assert L.ms_shuffle_ex(ctypes.c_void_p(16), 10, 4, 1, None, ctypes.byref(cfg), None) == -2
    assert b"cutoff" in L.ms_last_error()
    assert L.ms_shuffle_batched(None, None, 3, 1, None) == -1
    assert L.ms_shuffle_batched(None, None, 0, 1, None) == 0
    # batched: every array is checked before anything runs, and the message names it
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    ptrs = (vp * 3)(16, None, 32)
    sizes = (u64 * 3)(10, 5, 7)
    assert L.ms_shuffle_batched(ptrs, sizes, 3, 1, None) == -1
    assert b"array 1" in L.ms_last_error()
    ptrs = (vp * 3)(16, 32, 36)
    ebs = (u32 * 3)(4, 8, 8)
    assert L.ms_shuffle_batched_ex(ptrs, sizes, ebs, 3, 1, None, None, None) == -1   # 36 not 8-aligned
    assert b"array 2" in L.ms_last_error()
    ebs = (u32 * 3)(4, 8, 12)
    assert L.ms_shuffle_batched_ex(ptrs, sizes, ebs, 3, 1, None, None, None) == -2   # element size
    sizes = (u64 * 3)(10, 1 << 33, 7)
    assert L.ms_shuffle_batched(ptrs, sizes, 3, 1, None) == -2                       # n too large
    info = M._lib.MSPlanInfo()
    assert L.ms_plan(10, 3, None, ctypes.byref(info)) == -2
    assert L.ms_scratch_bytes(1 << 20, 4) > 4 << 20
    assert L.ms_leaf_B_for(1 << 20, 4) == 4096


def test_listing_placement_plans_every_level_as_one_level_pass():
    # the listing's in-place placement (R1) runs every merge level as a
    # one-level HBM pass: the leaf kernel's LDS merges use the stable interleave
    M, _ = _lib()
    for n in (1 << 20, (1 << 24) + 12345, 4097):
        p2 = M.plan(n)
        p1 = M.plan(n, placement="R1")
        assert p1["levels"] == p2["levels"]
        assert p1["lds_levels"] == 0
        assert p1["hbm_levels"] == p1["levels"]
    with pytest.raises(ValueError):
        M.plan(1000, placement="R3")


def test_tuning_table_sets_the_cutoff_and_is_validated():
    M, L = _lib()
    try:
        assert M.leaf_B_for(5000) == 4096
        M.tune_set([{"elem_bytes": 4, "log2_n": 12, "leaf_B": 1000, "levels_per_pass": 2, "leaf_big": True},
                    {"elem_bytes": 8, "log2_n": 20, "leaf_B": 2048, "levels_per_pass": 0}])
        assert M.leaf_B_for(4096) == 1000 and M.leaf_B_for(8191) == 1000
        assert M.leaf_B_for(8192) == 4096 and M.leaf_B_for(4095) == 4096
        assert M.leaf_B_for(4096, 8) == 4096 and M.leaf_B_for((1 << 20) + 5, 8) == 2048
        # a tuned call plans with the entry's knobs; an untuned one does not
        assert M.plan(5000, leaf_B=0)["leaf_B"] == 4096
        from paper_1508_03167_amd._lib import MS_CFG_TUNED, MSConfig, MSPlanInfo

        info = MSPlanInfo()
        assert L.ms_plan(5000, 4, ctypes.byref(MSConfig(0, 0, 0, MS_CFG_TUNED)), ctypes.byref(info)) == 0
        assert info.leaf_B == 1000 and info.levels == 3
        assert L.ms_plan((1 << 20) + 5, 8, ctypes.byref(MSConfig(0, 0, 0, MS_CFG_TUNED)), ctypes.byref(info)) == 0
        assert info.leaf_B == 2048
        # bad entries are refused and the table is kept
        for bad in ({"elem_bytes": 5, "log2_n": 3, "leaf_B": 10, "levels_per_pass": 0},
                    {"elem_bytes": 4, "log2_n": 40, "leaf_B": 10, "levels_per_pass": 0},
                    {"elem_bytes": 4, "log2_n": 3, "leaf_B": 0, "levels_per_pass": 0},
                    {"elem_bytes": 4, "log2_n": 3, "leaf_B": 5000, "levels_per_pass": 0},
                    {"elem_bytes": 4, "log2_n": 3, "leaf_B": 10, "levels_per_pass": 5}):
            with pytest.raises(M.MSError):
                M.tune_set([bad])
        assert M.leaf_B_for(5000) == 1000
    finally:
        M.tune_set([])
    assert M.leaf_B_for(5000) == 4096
