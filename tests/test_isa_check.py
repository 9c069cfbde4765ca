"""The build's check of the device assembly for half-spilled register pairs
(paper_2312_02898_amd/isa_check.py).

The device compiler of this toolchain was caught spilling a 64-bit value as
one 32-bit half and reloading only that half before 64-bit use (one part
kernel of g g > t t~ g g g, FP64 schedule with budget 320: wrong results on
the GPU, exact C++ on the host, exact with scratch-only spills).  The fixtures
are excerpts of that kernel's assembly as built here, with the shipped flags
and with scratch-only spills.
"""
import glob
import os

import pytest

from paper_2312_02898_amd import isa_check

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


def _read(name):
    with open(os.path.join(GOLD, name)) as f:
        return f.read()


def test_flags_the_half_reloads_of_the_miscompiled_part():
    found = isa_check.half_reloads(_read("half_reload_part4.s"))
    assert len(found) == 2
    assert "scratch_load_dword v122" in found[0] and "v[122:123]" in found[0]
    assert "scratch_load_dword v36" in found[1] and "v[36:37]" in found[1]


def test_whole_pair_spills_pass():
    assert isa_check.half_reloads(_read("half_reload_part4_scratch_only.s")) == []


FN = "_Zkernel:\n"


@pytest.mark.parametrize("body,n", [
    # reload of the low half, pair read: flagged
    ("\tscratch_load_dword v10, off, off offset:8\n\tv_add_f64 v[0:1], v[10:11], v[2:3]\n", 1),
    # reload of the high half, pair read: flagged
    ("\tscratch_load_dword v11, off, off offset:8\n\tv_mul_f64 v[0:1], v[2:3], v[10:11]\n", 1),
    # the mate written first: the pair is defined
    ("\tscratch_load_dword v10, off, off offset:8\n\tv_mov_b32_e32 v11, v5\n\tv_add_f64 v[0:1], v[10:11], v[2:3]\n", 0),
    # the reloaded register overwritten first: dead
    ("\tscratch_load_dword v10, off, off offset:8\n\tv_mov_b32_e32 v10, v5\n\tv_add_f64 v[0:1], v[10:11], v[2:3]\n", 0),
    # a 32-bit use only (FP32 code spills single registers legitimately)
    ("\tscratch_load_dword v10, off, off offset:8\n\tv_add_f32_e32 v0, v10, v2\n\tv_mov_b32_e32 v10, v1\n", 0),
    # stored as part of a pair: a read of the pair
    ("\tscratch_load_dword v10, off, off offset:8\n\tglobal_store_dwordx2 v[4:5], v[10:11], off\n", 1),
    # a pair saved half to scratch and half to a spare register, restored by
    # adjacent instructions (what the compiler does right)
    ("\tv_accvgpr_read_b32 v11, a207\n\tscratch_load_dword v10, off, off offset:84\n"
     "\tv_lshl_add_u64 v[66:67], v[10:11], 3, s[0:1]\n", 0),
])
def test_synthetic_cases(body, n):
    assert len(isa_check.half_reloads(FN + body)) == n


def test_every_built_unit_was_checked():
    """Each object of the in-tree build carries the stamp of a passed check."""
    objs = glob.glob(os.path.join(HERE, "..", "paper_2312_02898_amd", "_build", "*.o"))
    if not objs:
        pytest.skip("no in-tree build")
    missing = [o for o in objs if not os.path.exists(o + ".isa-ok")]
    assert not missing, missing[:5]
