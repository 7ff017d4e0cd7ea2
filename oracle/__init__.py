"""Serial-EMD CPU oracle -- TEST INFRASTRUCTURE ONLY.

ctypes wrappers around ``semd_oracle.c``: a plain scalar FP64 implementation
of Serial-EMD (arXiv 2106.15319, Sec. 2.1, 2.2, 3.2 and 3.3).  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark may import this
module; the product path (the HIP library and its binding) never does.

Every function takes and returns numpy float64 arrays on the host.  X is an
M x N matrix whose columns are the signals (Sec. 3.2); it is passed as a
column-major buffer, i.e. ``X.ravel(order="F")``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_DIR, "semd_oracle.c")
_LIB = os.path.join(_DIR, "libsemd_oracle.so")

_d = C.POINTER(C.c_double)
_i64 = C.POINTER(C.c_int64)
_int = C.POINTER(C.c_int)


class Stats(C.Structure):
    _fields_ = [("min_gap", C.c_double), ("n_sifts", C.c_int64), ("n_equal", C.c_int64),
                ("sd_margin", C.c_double)]


def compile_source(src: str, out: str) -> str:
    """Compile an oracle source with gcc: scalar FP64, no contraction, no fast-math."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-I", _DIR, "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle into the package directory."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = bind(C.CDLL(_LIB))
    return _lib


def bind(L):
    """Declare the C signatures on a loaded oracle library and return it."""
    L.semd_ref_serial_length.restype = C.c_int64
    L.semd_ref_serial_length.argtypes = [C.c_int64] * 3
    L.semd_ref_serialize.argtypes = [_d, C.c_int64, C.c_int64, C.c_int64, _d]
    L.semd_ref_deserialize.argtypes = [_d, C.c_int64, C.c_int64, C.c_int64, _d]
    L.semd_ref_extrema.argtypes = [_d, C.c_int64, _i64, _i64, _i64, _i64]
    L.semd_ref_spline_solve.argtypes = [_d, _d, C.c_int64, _d]
    L.semd_ref_spline_eval.argtypes = [_d, _d, _d, C.c_int64, C.c_int64, _d]
    L.semd_ref_envelope.argtypes = [_d, C.c_int64, _i64, C.c_int64, _d]
    L.semd_ref_emd.argtypes = [_d, C.c_int64, C.c_int, C.c_int, _d, _int, C.POINTER(Stats)]
    L.semd_ref_emd_sd.argtypes = [_d, C.c_int64, C.c_int, C.c_int, C.c_double, _d, _int,
                                  C.POINTER(Stats)]
    L.semd_ref_decompose_sd.argtypes = [_d, C.c_int64, C.c_int64, C.c_int64, C.c_int,
                                        C.c_int, C.c_double, _d, _int, C.POINTER(Stats)]
    L.semd_ref_decompose.argtypes = [_d, C.c_int64, C.c_int64, C.c_int64, C.c_int, C.c_int,
                                     _d, _int, C.POINTER(Stats)]
    L.semd_ref_decompose_slices.argtypes = [_d, C.c_int64, C.c_int64, C.c_int, C.c_int,
                                            _d, _int]
    L.semd_ref_decompose_slices_sd.argtypes = [_d, C.c_int64, C.c_int64, C.c_int, C.c_int,
                                               C.c_double, _d, _int]
    L.semd_ref_emd_trace.argtypes = [_d, C.c_int64, C.c_int, C.c_int, C.c_double, _d, _int,
                                     _i64, C.c_int64, _i64, _int, C.c_int, C.c_int, _d, _int]
    L.semd_ref_splitmix64.restype = C.c_uint64
    L.semd_ref_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    L.semd_ref_noise.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_int64, _d]
    L.semd_ref_eemd.argtypes = [_d, C.c_int64, C.c_int64, C.c_int64, C.c_int, C.c_int,
                                C.c_int, C.c_double, C.c_uint64, C.c_uint64, _d]
    L.semd_ref_eemd_sd.argtypes = [_d, C.c_int64, C.c_int64, C.c_int64, C.c_int, C.c_int,
                                   C.c_int, C.c_double, C.c_uint64, C.c_uint64, C.c_double,
                                   _d]
    L.semd_ref_ceemdan.argtypes = [_d, C.c_int64, C.c_int64, C.c_int64, C.c_int, C.c_int,
                                   C.c_int, C.c_double, C.c_uint64, C.c_uint64, C.c_double,
                                   _d, _int]
    for name in ("semd_ref_ceemdan", "semd_ref_serialize", "semd_ref_deserialize", "semd_ref_extrema",
                 "semd_ref_spline_solve", "semd_ref_spline_eval", "semd_ref_envelope",
                 "semd_ref_emd", "semd_ref_decompose", "semd_ref_decompose_slices",
                 "semd_ref_emd_sd", "semd_ref_decompose_sd",
                 "semd_ref_decompose_slices_sd", "semd_ref_noise", "semd_ref_eemd",
                 "semd_ref_eemd_sd", "semd_ref_emd_trace"):
        getattr(L, name).restype = C.c_int
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(_d)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def serial_length(M: int, N: int, D: int) -> int:
    return int(lib().semd_ref_serial_length(M, N, D))


def serialize(Xcol: np.ndarray, M: int, N: int, D: int) -> np.ndarray:
    """Sec. 3.2: column-major X (M*N) -> serialized x (M*N + D*N - D)."""
    X = _f64(Xcol)
    x = np.empty(serial_length(M, N, D))
    _check(lib().semd_ref_serialize(_p(X), M, N, D, _p(x)), "serialize")
    return x


def deserialize(y: np.ndarray, M: int, N: int, D: int) -> np.ndarray:
    """Sec. 3.3: serialized y -> column-major M*N (transition samples dropped)."""
    y = _f64(y)
    out = np.empty(M * N)
    _check(lib().semd_ref_deserialize(_p(y), M, N, D, _p(out)), "deserialize")
    return out


def extrema(h: np.ndarray):
    """Sec. 2.1 Step 1: sorted maxima and minima index arrays."""
    h = _f64(h)
    L = h.size
    imax = np.empty(L // 2 + 2, dtype=np.int64)
    imin = np.empty(L // 2 + 2, dtype=np.int64)
    na, ni = C.c_int64(), C.c_int64()
    _check(lib().semd_ref_extrema(_p(h), L, imax.ctypes.data_as(_i64), C.byref(na),
                                  imin.ctypes.data_as(_i64), C.byref(ni)), "extrema")
    return imax[: na.value].copy(), imin[: ni.value].copy()


def spline_solve(t, y) -> np.ndarray:
    t, y = _f64(t), _f64(y)
    Mpp = np.empty(t.size)
    _check(lib().semd_ref_spline_solve(_p(t), _p(y), t.size, _p(Mpp)), "spline_solve")
    return Mpp


def spline_eval(t, y, Mpp, L: int) -> np.ndarray:
    t, y, Mpp = _f64(t), _f64(y), _f64(Mpp)
    out = np.empty(L)
    _check(lib().semd_ref_spline_eval(_p(t), _p(y), _p(Mpp), t.size, L, _p(out)), "spline_eval")
    return out


def envelope(h, idx) -> np.ndarray:
    """Sec. 2.1 Step 2: mirrored natural-spline envelope through h[idx]."""
    h = _f64(h)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    env = np.empty(h.size)
    _check(lib().semd_ref_envelope(_p(h), h.size, idx.ctypes.data_as(_i64), idx.size, _p(env)),
           "envelope")
    return env


def _stats(st) -> dict:
    return {"min_gap": st.min_gap, "n_sifts": st.n_sifts, "n_equal": st.n_equal,
            "sd_margin": st.sd_margin}


def emd(x, K: int, S: int, with_stats: bool = False, sd: float = 0.0):
    """Sec. 2.1: (K+1, L) slots (IMFs, zero fill, residue in slot K) and n_imfs.
    sd > 0: an IMF also ends once a sift's SD falls below sd (at most S sifts)."""
    x = _f64(x)
    L = x.size
    out = np.empty((K + 1) * L)
    n = C.c_int()
    st = Stats()
    _check(lib().semd_ref_emd_sd(_p(x), L, K, S, float(sd), _p(out), C.byref(n), C.byref(st)),
           "emd")
    res = (out.reshape(K + 1, L), n.value)
    if with_stats:
        return res + (_stats(st),)
    return res


def parse_trace(buf) -> list[tuple[int, int, np.ndarray, np.ndarray]]:
    """Records (imf, sift, maxima, minima) of a flat extremum-decision trace."""
    buf = np.asarray(buf, dtype=np.int64)
    recs, o = [], 0
    while o + 4 <= buf.size:
        imf, sift, na, ni = (int(v) for v in buf[o:o + 4])
        if na < 0 or ni < 0 or o + 4 + na + ni > buf.size:
            raise ValueError(f"malformed trace record at {o}")
        recs.append((imf, sift, buf[o + 4:o + 4 + na].copy(),
                     buf[o + 4 + na:o + 4 + na + ni].copy()))
        o += 4 + na + ni
    return recs


def emd_trace(x, K: int, S: int, sd: float = 0.0, cap: int | None = None):
    """Sec. 2.1 with every extremum detection recorded: ((K+1, L) slots,
    n_imfs, records [(imf, sift, maxima, minima)], complete)."""
    x = _f64(x)
    L = x.size
    cap = cap if cap is not None else (K * S) * (L + 8) + 64
    buf = np.empty(max(cap, 1), dtype=np.int64)
    out = np.empty((K + 1) * L)
    n = C.c_int()
    used, complete = C.c_int64(), C.c_int()
    _check(lib().semd_ref_emd_trace(_p(x), L, K, S, float(sd), _p(out), C.byref(n),
                                    buf.ctypes.data_as(_i64), cap, C.byref(used),
                                    C.byref(complete), -1, -1, None, None), "emd_trace")
    return out.reshape(K + 1, L), n.value, parse_trace(buf[: used.value]), bool(complete.value)


def emd_tested(x, K: int, S: int, imf: int, sift: int, sd: float = 0.0):
    """The array that detection (imf, sift) of the EMD of x tests (the
    residue for sift 0, else the candidate before that sift), or None if the
    decomposition makes no such detection."""
    x = _f64(x)
    L = x.size
    out = np.empty((K + 1) * L)
    h = np.empty(L)
    n = C.c_int()
    used, complete, found = C.c_int64(), C.c_int(), C.c_int()
    _check(lib().semd_ref_emd_trace(_p(x), L, K, S, float(sd), _p(out), C.byref(n), None, 0,
                                    C.byref(used), C.byref(complete), int(imf), int(sift),
                                    _p(h), C.byref(found)), "emd_tested")
    return h if found.value else None


def decompose(Xcol, M: int, N: int, D: int, K: int, S: int, with_stats: bool = False,
              sd: float = 0.0):
    """Serial-EMD (Sec. 3): (K+1, M*N) column-major slots and n_imfs (sd as in emd)."""
    X = _f64(Xcol)
    out = np.empty((K + 1) * M * N)
    n = C.c_int()
    st = Stats()
    _check(lib().semd_ref_decompose_sd(_p(X), M, N, D, K, S, float(sd), _p(out), C.byref(n),
                                       C.byref(st)), "decompose")
    res = (out.reshape(K + 1, M * N), n.value)
    if with_stats:
        return res + (_stats(st),)
    return res


def decompose_slices(Xcol, M: int, N: int, K: int, S: int, sd: float = 0.0):
    """Standard-version EMD: each column on its own.  ((K+1, M*N), n_imfs[N])."""
    X = _f64(Xcol)
    out = np.empty((K + 1) * M * N)
    n = np.empty(N, dtype=np.int32)
    _check(lib().semd_ref_decompose_slices_sd(_p(X), M, N, K, S, float(sd), _p(out),
                                              n.ctypes.data_as(_int)), "decompose_slices")
    return out.reshape(K + 1, M * N), n


def splitmix64(state: int, n: int) -> int:
    return int(lib().semd_ref_splitmix64(state & (2**64 - 1), n & (2**64 - 1)))


def noise(seed: int, item: int, m: int, L: int) -> np.ndarray:
    w = np.empty(L)
    _check(lib().semd_ref_noise(seed, item, m, L, _p(w)), "noise")
    return w


def eemd(Xcol, M: int, N: int, D: int, K: int, S: int, NR: int, beta: float, seed: int,
         item: int = 0, sd: float = 0.0) -> np.ndarray:
    """Sec. 2.2 EEMD of the serialized signal: (K+1, M*N) mean slots."""
    X = _f64(Xcol)
    out = np.empty((K + 1) * M * N)
    _check(lib().semd_ref_eemd_sd(_p(X), M, N, D, K, S, NR, float(beta), seed, item, float(sd),
                                  _p(out)), "eemd")
    return out.reshape(K + 1, M * N)


def ceemdan(Xcol, M: int, N: int, D: int, K: int, S: int, NR: int, eps: float, seed: int,
            item: int = 0, sd: float = 0.0):
    """Sec. 2.2 CEEMDAN of the serialized signal: ((K+1, M*N) slots, n_modes)."""
    X = _f64(Xcol)
    out = np.empty((K + 1) * M * N)
    n = C.c_int()
    _check(lib().semd_ref_ceemdan(_p(X), M, N, D, K, S, NR, float(eps), seed, item, float(sd),
                                  _p(out), C.byref(n)), "ceemdan")
    return out.reshape(K + 1, M * N), n.value
