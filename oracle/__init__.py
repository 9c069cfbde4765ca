"""CPU oracle for leading-order |M|^2 -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It never imports the GPU package and
the GPU package never imports it.

Python side: ctypes marshalling of ``oracle.cpp`` (built with g++ -fopenmp),
plus the process table of the oracle (legs, masses, IDEN).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

PROCESSES = {
    "e+ e- > mu+ mu-": 0,
    "g g > t t~": 1,
    "g g > t t~ g": 2,
    "g g > t t~ g g": 3,
    "g g > t t~ g g g": 4,
    "u u~ > t t~": 5,
    "u~ u > t t~": 6,
    "u u~ > t t~ g": 7,
    "u~ u > t t~ g": 8,
    "u g > t t~ u": 9,
    "g u > t t~ u": 10,
    "u~ g > t t~ u~": 11,
    "g u~ > t t~ u~": 12,
}


class Params(ctypes.Structure):
    _fields_ = [
        ("alpha_em", ctypes.c_double),
        ("sin2w", ctypes.c_double),
        ("mz", ctypes.c_double),
        ("wz", ctypes.c_double),
        ("mt", ctypes.c_double),
        ("wt", ctypes.c_double),
        ("alpha_s", ctypes.c_double),
        ("tchan_zero_width", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


def default_params(tchan_zero_width: int = 1, **kw) -> Params:
    """SM inputs of the benchmark configurations (alpha = 1/132.507,
    MZ = 91.188, GZ = 2.441, sin^2 theta_W = 0.2222, mt = 173, Gt = 1.49,
    alpha_s = 0.118)."""
    vals = dict(alpha_em=1.0 / 132.507, sin2w=0.2222, mz=91.188, wz=2.441,
                mt=173.0, wt=1.49, alpha_s=0.118)
    vals.update(kw)
    return Params(tchan_zero_width=tchan_zero_width, reserved=0, **vals)


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (OpenMP).  Building the checker is not
    using it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
                               "-Wall", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d = ctypes.c_double
        i = ctypes.c_int
        L.oracle_npar.argtypes = [i]
        L.oracle_ncolor.argtypes = [i]
        L.oracle_iden.argtypes = [i]
        L.oracle_iden.restype = d
        L.oracle_me.argtypes = [i, P(Params), P(d), ctypes.c_int64, P(d), i, i]
        L.oracle_me_hel.argtypes = [i, P(Params), P(d), ctypes.c_int64, P(d), i]
        L.oracle_partial_amps.argtypes = [i, P(Params), P(d), i, i, P(d)]
        L.oracle_dressed_amp.argtypes = [i, P(Params), P(d), i, P(i), P(d)]
        L.oracle_colour_basis.argtypes = [i, P(i), P(d)]
        L.oracle_colour_matrix.argtypes = [i, P(d)]
        L.oracle_me_gauge.argtypes = [i, P(Params), P(d), ctypes.c_int64, P(d)]
        L.oracle_uniforms.argtypes = [ctypes.c_int64, i, ctypes.c_uint64, P(d)]
        L.oracle_rambo.argtypes = [ctypes.c_int64, i, P(d), d, ctypes.c_uint64, P(d)]
        L.oracle_sample.argtypes = [ctypes.c_int64, i, P(d), d, ctypes.c_uint64, P(d), P(d)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def proc_id(process) -> int:
    return PROCESSES[process] if isinstance(process, str) else int(process)


def npar(process) -> int:
    if _general(process):
        from . import feyn
        return feyn.process(process).n
    return lib().oracle_npar(proc_id(process))


def ncolor(process) -> int:
    return lib().oracle_ncolor(proc_id(process))


def iden(process) -> float:
    if _general(process):
        from . import feyn
        return float(feyn.process(process).iden)
    return lib().oracle_iden(proc_id(process))


def _general(process) -> bool:
    """Processes of the diagram-by-diagram evaluation (feyn.py): every QCD
    process the C++ oracle does not cover."""
    return isinstance(process, str) and process not in PROCESSES


def me(process, mom, params: Params | None = None, long_double=False, nthreads=0):
    """Averaged |M|^2 per event; mom is float64 [nevt][npar][4]."""
    p = params or default_params()
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    if _general(process):
        from . import feyn
        return feyn.me(process, mom, p, long_double=long_double)
    out = np.empty(mom.shape[0], dtype=np.float64)
    rc = lib().oracle_me(proc_id(process), ctypes.byref(p), _dp(mom), mom.shape[0], _dp(out),
                         int(long_double), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_me failed ({rc})")
    return out


def me_hel(process, mom, params: Params | None = None, nthreads=0):
    """Colour-summed (not averaged) |M_h|^2, shape [nevt][2^npar]."""
    p = params or default_params()
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    if _general(process):
        from . import feyn
        return feyn.me(process, mom, p, per_helicity=True)
    n = npar(process)
    out = np.empty((mom.shape[0], 1 << n), dtype=np.float64)
    rc = lib().oracle_me_hel(proc_id(process), ctypes.byref(p), _dp(mom), mom.shape[0], _dp(out),
                             int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_me_hel failed ({rc})")
    return out


def me_gauge(process, mom, params: Params | None = None):
    """Processes with one light-quark line and one gluon: |M|^2 with the
    gluon polarisation replaced by k/k^0 (gauge invariance: zero)."""
    p = params or default_params()
    mom = np.ascontiguousarray(mom, dtype=np.float64)
    out = np.empty(mom.shape[0], dtype=np.float64)
    if lib().oracle_me_gauge(proc_id(process), ctypes.byref(p), _dp(mom), mom.shape[0], _dp(out)) != 0:
        raise ValueError("oracle_me_gauge failed")
    return out


def partial_amps(process, mom1, hel, gauge_leg=-1, params: Params | None = None):
    p = params or default_params()
    mom1 = np.ascontiguousarray(mom1, dtype=np.float64)
    nc = ncolor(process)
    out = np.empty((nc, 2), dtype=np.float64)
    rc = lib().oracle_partial_amps(proc_id(process), ctypes.byref(p), _dp(mom1), int(hel),
                                   int(gauge_leg), _dp(out))
    if rc != 0:
        raise ValueError(f"oracle_partial_amps failed ({rc})")
    return out[:, 0] + 1j * out[:, 1]


def dressed_amp(process, mom1, hel, colours, params: Params | None = None):
    p = params or default_params()
    mom1 = np.ascontiguousarray(mom1, dtype=np.float64)
    col = np.ascontiguousarray(colours, dtype=np.int32)
    out = np.empty(2, dtype=np.float64)
    rc = lib().oracle_dressed_amp(proc_id(process), ctypes.byref(p), _dp(mom1), int(hel), _ip(col),
                                  _dp(out))
    if rc != 0:
        raise ValueError(f"oracle_dressed_amp failed ({rc})")
    return out[0] + 1j * out[1]


def colour_basis(ngluons, colours):
    col = np.ascontiguousarray(colours, dtype=np.int32)
    nf = int(np.prod(np.arange(1, ngluons + 1)))
    out = np.empty((nf, 2), dtype=np.float64)
    if lib().oracle_colour_basis(int(ngluons), _ip(col), _dp(out)) != 0:
        raise ValueError("oracle_colour_basis failed")
    return out[:, 0] + 1j * out[:, 1]


def colour_matrix(ngluons):
    nf = int(np.prod(np.arange(1, ngluons + 1)))
    out = np.empty((nf, nf), dtype=np.float64)
    if lib().oracle_colour_matrix(int(ngluons), _dp(out)) != 0:
        raise ValueError("oracle_colour_matrix failed")
    return out


def max_weight(me_values, factors):
    """Batch unweighting step (paper, Sec. 3): weights w_i = |M|^2_i f_i
    (negative or NaN products count as 0) and their maximum."""
    w = np.asarray(me_values, dtype=np.float64) * np.asarray(factors, dtype=np.float64)
    w = np.where(w > 0, w, 0.0)
    return w, (float(w.max()) if w.size else 0.0)


def uniforms(nevt, nfinal, seed):
    """Philox4x32-10 uniforms of the device phase-space generator, [nevt][nfinal][4]."""
    out = np.empty((nevt, nfinal, 4), dtype=np.float64)
    if lib().oracle_uniforms(int(nevt), int(nfinal), int(seed), _dp(out)) != 0:
        raise ValueError("oracle_uniforms failed")
    return out


def rambo(nevt, masses, sqrt_s, seed):
    """RAMBO momenta from the Philox stream, [nevt][nfinal+2][4]."""
    m = np.ascontiguousarray(masses, dtype=np.float64)
    out = np.empty((nevt, m.size + 2, 4), dtype=np.float64)
    if lib().oracle_rambo(int(nevt), int(m.size), _dp(m), float(sqrt_s), int(seed), _dp(out)) != 0:
        raise ValueError("oracle_rambo failed")
    return out


def sample(nevt, masses, sqrt_s, seed):
    """Importance-sampled momenta [nevt][nfinal+2][4] and phase-space
    weights [nevt] from the Philox stream."""
    m = np.ascontiguousarray(masses, dtype=np.float64)
    out = np.empty((nevt, m.size + 2, 4), dtype=np.float64)
    w = np.empty(nevt, dtype=np.float64)
    if lib().oracle_sample(int(nevt), int(m.size), _dp(m), float(sqrt_s), int(seed), _dp(out), _dp(w)) != 0:
        raise ValueError("oracle_sample failed")
    return out, w
