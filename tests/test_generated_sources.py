"""The committed generated kernels are exactly what the process compiler emits.

The build regenerates ``csrc/gen`` from ``procgen`` before compiling, and the
GPU parity tests validate the kernels of the committed schedules.  These CPU
tests make a change to the compiler that would alter any generated source
(and so ship a schedule the GPU tests have not seen) fail until the sources
are regenerated and committed together with it; the schedule parameters of
the shipped configurations are pinned by value as well.
"""
import os
import tempfile

import pytest

from paper_2312_02898_amd.procgen import codegen, program

HERE = os.path.dirname(os.path.abspath(__file__))
GEN = os.path.join(os.path.dirname(HERE), "paper_2312_02898_amd", "csrc", "gen")


@pytest.mark.slow
def test_regenerated_sources_equal_committed():
    with tempfile.TemporaryDirectory() as d:
        codegen.generate(d)
        fresh = sorted(os.listdir(d))
        committed = sorted(f for f in os.listdir(GEN) if f.endswith((".hip", ".inc")))
        assert fresh == committed
        for f in fresh:
            with open(os.path.join(d, f)) as a, open(os.path.join(GEN, f)) as b:
                assert a.read() == b.read(), f"csrc/gen/{f} differs from the compiler's output"


def test_shipped_schedule_parameters():
    """(budget, greedy passes) per process and form, and the split form's
    (budget, jamp accumulators, parts[, accumulators in LDS]): the
    configurations whose kernels the GPU parity tests validate."""
    assert program.DEFAULT_SCHEDULE_F64 == {"eemumu": (512, 4), "ggtt": (512, 4), "ggttg": (512, 4),
                                            "ggttgg": (250, 4)}
    assert program.DEFAULT_SCHEDULE_F32 == {"eemumu": (1024, 4), "ggtt": (1024, 4), "ggttg": (1024, 1),
                                            "ggttgg": (1024, 2), "ugttug": (512, 4), "guttug": (512, 4),
                                            "uxgttuxg": (512, 4), "guxttuxg": (512, 4)}
    assert program.SCHEDULE_F64_OTHERS == (512, 4) and program.SCHEDULE_F32_OTHERS == (1024, 4)
    assert program.SPLIT == {"ggttggg": {"f64": (288, 36, 12, True), "f32": (384, 56, 8)}}
    assert program.SHARE_HALF == {"ggttg": False, "ggttgg": True, "ggttggg": True}
    assert program.FP64_LDS_JAMPS == set()
    assert "ggttgg" in program.DEN_CACHE_F64
    assert program.MOM_CACHE_F32 == program.DEN_CACHE_F32 - {"ugttug", "guttug", "uxgttuxg", "guxttuxg", "ggttuux"}
    assert program.F32_KC_WAVES == 2
    assert program.MOM_CACHE_F64 == program.DEN_CACHE_F64 and program.F64_KCW_WAVES == 4
