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


def _header_enum(body_of):
    txt = open(os.path.join(ROOT, "include", "me.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    m = re.search(r"typedef enum \{([^}]*)\}\s*" + body_of + ";", txt)
    return {k: int(v) for k, v in re.findall(r"(ME_\w+)\s*=\s*(-?\d+)", m.group(1))}


def test_binding_constants_match_header():
    """The binding's precision and status values are the header's."""
    from paper_2312_02898_amd import binding as B
    prec = _header_enum("me_precision")
    assert prec and all(getattr(B, k) == v for k, v in prec.items()), prec
    txt = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "me.h")).read(), flags=re.S)
    status = {k: int(v) for k, v in re.findall(r"(ME_E\w+|ME_OK)\s*=\s*(-?\d+)", txt)}
    assert len(status) == 7 and all(getattr(B, k) == v for k, v in status.items()), status


def test_bf16_colour_matrices_exact():
    """The BF16 MFMA colour sum takes the integer colour matrix as BF16
    operands (8 significant bits): exact for every process with 6..32 colour
    flows."""
    import glob
    n = 0
    for f in glob.glob(os.path.join(ROOT, "paper_2312_02898_amd", "csrc", "gen", "*_proc.inc")):
        t = open(f).read()
        m = re.search(r"kCmat_\w+\[[^\]]*\]\s*=\s*\{([^}]*)\}", t)
        vals = [int(x) for x in m.group(1).split(",") if x.strip()]
        nc = int(round(len(vals) ** 0.5))
        if not 6 <= nc <= 32:
            continue
        n += 1
        for v in vals:
            a = abs(v)
            while a and a % 2 == 0:
                a //= 2
            assert a < 256, (f, v)
    assert n >= 10
