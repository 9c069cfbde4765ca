"""The C ABI library loads on a host without a GPU and exports every
function include/me.h declares (no compute calls here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "me.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(me_[a-z_]+)\s*\(", txt)))


def test_library_exports_header_symbols():
    from paper_2312_02898_amd import binding
    L = binding.lib()
    names = declared()
    assert "me_compute" in names and "me_server_submit" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(binding.EXPORTS) == names


def test_defaults_and_errors_without_gpu():
    from paper_2312_02898_amd import binding as B
    p = B.me_default_params()
    assert abs(p.alpha_em - 1 / 132.507) < 1e-15 and p.tchannel_zero_width == 1
    assert p.filter_nevt == 1024 and p.precision == B.ME_FP64
    h = ctypes.c_void_p()
    assert B.lib().me_create(None, ctypes.byref(p), ctypes.byref(h)) == B.ME_EINVAL
    assert B.lib().me_compute(None, None, 0, None, None) == B.ME_EINVAL
    assert B.lib().me_info(None, None) == B.ME_EINVAL
    assert B.lib().me_destroy(None) == B.ME_EINVAL
    assert isinstance(B.me_last_error(), str)
