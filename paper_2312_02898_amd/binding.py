"""ctypes binding of the C ABI in include/me.h (argument marshalling only).

Every function keeps the name of the C entry point it wraps.  Device buffers
are passed as integers (device addresses, e.g. ``tensor.data_ptr()``) and
streams as ``hipStream_t`` integers (``torch.cuda.current_stream().cuda_stream``);
PyTorch is only used by callers for device memory and streams.  Loading fails
loudly when the built library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libme_mi355x.so")

ME_OK, ME_EINVAL, ME_EPROCESS, ME_ENOMEM, ME_EHIP, ME_ENOTSUP, ME_EBUSY = 0, -1, -2, -3, -4, -5, -6
ME_FP64, ME_MIXED, ME_MIXED_VALU, ME_MIXED_MFMA32, ME_MIXED_MFMA16, ME_MIXED_MFMABF16 = 0, 1, 2, 3, 4, 5


class MeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class me_sm_params(ctypes.Structure):
    _fields_ = [
        ("alpha_em", ctypes.c_double),
        ("sin2_thetaw", ctypes.c_double),
        ("mz", ctypes.c_double),
        ("wz", ctypes.c_double),
        ("mt", ctypes.c_double),
        ("wt", ctypes.c_double),
        ("alpha_s", ctypes.c_double),
        ("tchannel_zero_width", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("filter_sqrt_s", ctypes.c_double),
        ("filter_seed", ctypes.c_uint64),
        ("filter_nevt", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class me_info_t(ctypes.Structure):
    _fields_ = [
        ("npar", ctypes.c_int32),
        ("nhel", ctypes.c_int32),
        ("nhel_good", ctypes.c_int32),
        ("ndiagrams", ctypes.c_int32),
        ("ncolor", ctypes.c_int32),
        ("iden", ctypes.c_int32),
        ("flops_per_event", ctypes.c_int64),
        ("bytes_per_event", ctypes.c_int64),
        ("precision", ctypes.c_int32),
        ("filtered", ctypes.c_int32),
    ]


class me_server_stats_t(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("failed", ctypes.c_int64),
        ("rejected", ctypes.c_int64),
        ("events_completed", ctypes.c_int64),
        ("bytes_in_use", ctypes.c_int64),
        ("peak_bytes_in_use", ctypes.c_int64),
        ("active_slots", ctypes.c_int32),
        ("queued", ctypes.c_int32),
        ("bypassed", ctypes.c_int64),
        ("passed_large", ctypes.c_int64),
    ]


# every symbol declared in include/me.h
EXPORTS = [
    "me_default_params", "me_create", "me_helicity_filter", "me_compute", "me_compute_helicities",
    "me_good_helicities", "me_info", "me_destroy", "me_last_error",
    "me_server_create", "me_server_submit", "me_server_poll", "me_server_wait", "me_server_stats",
    "me_server_destroy", "me_max_weight", "me_rambo", "me_compute_channels", "me_server_times",
    "me_workspace_bytes", "me_compute_channels_noalloc", "me_sample", "me_compute_weighted",
]

# fixed device workspace of me_compute_channels_noalloc (ME_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2312_02898_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, vp, i32, i64, d = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.me_default_params.argtypes = [P(me_sm_params)]
        L.me_default_params.restype = None
        L.me_create.argtypes = [ctypes.c_char_p, P(me_sm_params), P(vp)]
        L.me_helicity_filter.argtypes = [vp]
        L.me_compute.argtypes = [vp, vp, i64, vp, vp]
        L.me_compute_weighted.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
        L.me_compute_helicities.argtypes = [vp, vp, i64, vp, vp]
        L.me_good_helicities.argtypes = [vp, P(i32), i32, P(i32)]
        L.me_info.argtypes = [vp, P(me_info_t)]
        L.me_destroy.argtypes = [vp]
        L.me_last_error.argtypes = []
        L.me_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("me_default_params", "me_last_error") and hasattr(L, name):
                getattr(L, name).restype = i32
        L.me_max_weight.argtypes = [vp, vp, i64, vp, vp, vp]
        L.me_rambo.argtypes = [i64, i32, P(d), d, ctypes.c_uint64, vp, vp]
        L.me_sample.argtypes = [i64, i32, P(d), d, ctypes.c_uint64, vp, vp, vp]
        L.me_compute_channels.argtypes = [P(vp), i32, vp, vp, vp, i64, vp, vp]
        L.me_compute_channels_noalloc.argtypes = [P(vp), i32, vp, vp, vp, i64, vp, vp]
        L.me_workspace_bytes.argtypes = [vp, i64, P(i64)]
        if hasattr(L, "me_server_create"):
            L.me_server_create.argtypes = [i64, i32, P(vp)]
            L.me_server_submit.argtypes = [vp, vp, vp, i64, vp, P(i64)]
            L.me_server_poll.argtypes = [vp, i64, P(i32), P(i32), P(d)]
            L.me_server_wait.argtypes = [vp, i64, d, P(i32), P(d)]
            L.me_server_stats.argtypes = [vp, P(me_server_stats_t)]
            L.me_server_times.argtypes = [vp, i64, P(d), P(d)]
            L.me_server_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _check(status, what):
    if status != ME_OK:
        raise MeError(status, f"{what}: {lib().me_last_error().decode(errors='replace')}")


def me_default_params(**overrides) -> me_sm_params:
    p = me_sm_params()
    lib().me_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def me_create(process: str, params: me_sm_params | None = None) -> int:
    h = ctypes.c_void_p()
    p = params if params is not None else me_default_params()
    _check(lib().me_create(process.encode(), ctypes.byref(p), ctypes.byref(h)), "me_create")
    return h.value


def me_helicity_filter(handle: int) -> None:
    _check(lib().me_helicity_filter(handle), "me_helicity_filter")


def me_compute(handle: int, d_momenta: int, nevt: int, d_me: int, stream: int = 0) -> None:
    _check(lib().me_compute(handle, d_momenta, nevt, d_me, stream or None), "me_compute")


def me_compute_helicities(handle: int, d_momenta: int, nevt: int, d_me_hel: int, stream: int = 0) -> None:
    _check(lib().me_compute_helicities(handle, d_momenta, nevt, d_me_hel, stream or None),
           "me_compute_helicities")


def me_good_helicities(handle: int) -> list:
    n = ctypes.c_int32()
    buf = (ctypes.c_int32 * 128)()
    _check(lib().me_good_helicities(handle, buf, 128, ctypes.byref(n)), "me_good_helicities")
    return list(buf[: n.value])


def me_info(handle: int) -> dict:
    info = me_info_t()
    _check(lib().me_info(handle, ctypes.byref(info)), "me_info")
    return {f: getattr(info, f) for f, _ in me_info_t._fields_}


def me_destroy(handle: int) -> None:
    _check(lib().me_destroy(handle), "me_destroy")


def me_compute_weighted(h, d_momenta: int, nevt: int, d_factor: int, d_me: int, d_w: int, d_max: int,
                        stream: int = 0) -> None:
    """me_compute with the weights d_w = max(d_me * d_factor, 0) (d_w may be
    0) and their maximum *d_max formed in the same kernel (device pointers)."""
    _check(lib().me_compute_weighted(h, d_momenta or None, int(nevt), d_factor or None, d_me or None, d_w or None,
                                     d_max or None, stream or None), "me_compute_weighted")


def me_max_weight(d_me: int, d_factor: int, nevt: int, d_w: int, d_max: int, stream: int = 0) -> None:
    """Device pointers in; *d_max receives max_i(me_i * factor_i)."""
    _check(lib().me_max_weight(d_me or None, d_factor or None, nevt, d_w or None, d_max or None, stream or None),
           "me_max_weight")


def me_rambo(nevt: int, masses, sqrt_s: float, seed: int, d_momenta: int, stream: int = 0) -> None:
    """Device RAMBO: nevt events with final-state masses `masses` into the
    device buffer d_momenta [nevt][len(masses)+2][4]."""
    m = (ctypes.c_double * len(masses))(*[float(x) for x in masses])
    _check(lib().me_rambo(int(nevt), len(masses), m, float(sqrt_s), int(seed), d_momenta or None, stream or None),
           "me_rambo")


def me_sample(nevt: int, masses, sqrt_s: float, seed: int, d_momenta: int, d_weight: int, stream: int = 0) -> None:
    """Device importance-sampled phase space: momenta into d_momenta
    [nevt][len(masses)+2][4] and phase-space weights into d_weight [nevt]."""
    m = (ctypes.c_double * len(masses))(*[float(x) for x in masses])
    _check(lib().me_sample(int(nevt), len(masses), m, float(sqrt_s), int(seed), d_momenta or None,
                           d_weight or None, stream or None), "me_sample")


def me_compute_channels(handles, d_momenta: int, d_channel: int, d_alphas: int, nevt: int, d_out: int,
                        stream: int = 0) -> None:
    """Multi-subprocess batch: event e evaluated by handles[channel[e]],
    optionally rescaled to a per-event alpha_s (device pointers; d_alphas may
    be 0)."""
    arr = (ctypes.c_void_p * len(handles))(*handles)
    _check(lib().me_compute_channels(arr, len(handles), d_momenta or None, d_channel or None, d_alphas or None,
                                     int(nevt), d_out or None, stream or None), "me_compute_channels")


def me_compute_channels_noalloc(handles, d_momenta: int, d_channel: int, d_alphas: int, nevt: int, d_out: int,
                                stream: int = 0) -> None:
    """me_compute_channels with its workspace in the library's fixed device
    array (nothing is allocated; calls that overlap on one device race)."""
    arr = (ctypes.c_void_p * len(handles))(*handles)
    _check(lib().me_compute_channels_noalloc(arr, len(handles), d_momenta or None, d_channel or None,
                                             d_alphas or None, int(nevt), d_out or None, stream or None),
           "me_compute_channels_noalloc")


def me_workspace_bytes(handle: int, nevt: int) -> int:
    """Device workspace me_compute allocates for nevt events of this handle."""
    b = ctypes.c_int64()
    _check(lib().me_workspace_bytes(handle, int(nevt), ctypes.byref(b)), "me_workspace_bytes")
    return b.value


def me_last_error() -> str:
    return lib().me_last_error().decode(errors="replace")


# ----------------------------------------------------------------- serving
def me_server_create(budget_bytes: int, n_slots: int) -> int:
    s = ctypes.c_void_p()
    _check(lib().me_server_create(int(budget_bytes), int(n_slots), ctypes.byref(s)), "me_server_create")
    return s.value


def me_server_submit(server: int, handle: int, h_momenta: np.ndarray, h_out: np.ndarray) -> int:
    """h_momenta float64 [nevt][npar][4] and h_out float64 [nevt], both
    C-contiguous host arrays that must stay alive until the ticket completes."""
    if h_momenta.dtype != np.float64 or not h_momenta.flags.c_contiguous:
        raise ValueError("h_momenta must be C-contiguous float64")
    if h_out.dtype != np.float64 or not h_out.flags.c_contiguous:
        raise ValueError("h_out must be C-contiguous float64")
    npar = me_info(handle)["npar"]
    if h_momenta.ndim != 3 or h_momenta.shape[1] != npar or h_momenta.shape[2] != 4:
        raise ValueError(f"h_momenta must have shape [nevt][{npar}][4]")
    if h_out.ndim != 1 or h_out.shape[0] < h_momenta.shape[0]:
        raise ValueError("h_out must hold nevt elements")
    t = ctypes.c_int64()
    _check(lib().me_server_submit(server, handle, h_momenta.ctypes.data, h_momenta.shape[0], h_out.ctypes.data,
                                  ctypes.byref(t)), "me_server_submit")
    return t.value


def me_server_poll(server: int, ticket: int):
    done, res, lat = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(lib().me_server_poll(server, ticket, ctypes.byref(done), ctypes.byref(res), ctypes.byref(lat)),
           "me_server_poll")
    return bool(done.value), res.value, lat.value


def me_server_wait(server: int, ticket: int, timeout_s: float = 60.0):
    res, lat = ctypes.c_int32(), ctypes.c_double()
    st = lib().me_server_wait(server, ticket, float(timeout_s), ctypes.byref(res), ctypes.byref(lat))
    _check(st, "me_server_wait")
    return res.value, lat.value


def me_server_times(server: int, ticket: int):
    """(queue_s, service_s) of a finished ticket."""
    q, sv = ctypes.c_double(), ctypes.c_double()
    _check(lib().me_server_times(server, ticket, ctypes.byref(q), ctypes.byref(sv)), "me_server_times")
    return q.value, sv.value


def me_server_stats(server: int) -> dict:
    s = me_server_stats_t()
    _check(lib().me_server_stats(server, ctypes.byref(s)), "me_server_stats")
    return {f: getattr(s, f) for f, _ in me_server_stats_t._fields_}


def me_server_destroy(server: int) -> None:
    _check(lib().me_server_destroy(server), "me_server_destroy")
