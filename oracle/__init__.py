"""CPU oracle for Range-Tiled CDF sort (RT-CDF) -- test infrastructure only.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may import this package.  The product library never does, and the oracle
shares no code with the HIP path.  The arithmetic lives in plain C
(``rtcdf_oracle.c``, built with gcc into ``liboracle.so``) and in
``mlp_ref.py`` / ``tune_ref.py``; this module is argument marshalling.

``parallel_sort`` is not an oracle: it wraps ``cpu_parallel.cc``, the
multi-threaded CPU counting sort that the benchmark times beside the oracle
and that the tests check against it.

Each wrapper names the passage of the paper it follows (sections of
"Shared-Memory Range-Tiled CDF Sort for Small-Range Integer Keys on GPUs").
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RTCDF_ORACLE_LIB lets the mutation test load a deliberately broken copy.
_SO = os.environ.get("RTCDF_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "rtcdf_oracle.c")
# The multi-threaded CPU counting sort timed beside the oracle (not an oracle).
_PAR_SO = os.path.join(_HERE, "libcpu_parallel.so")
_PAR_SRC = os.path.join(_HERE, "cpu_parallel.cc")

ORC_OK = 0
ORC_INVALID_ARGUMENT = 1
ORC_KEY_OUT_OF_RANGE = 2
ORC_MISMATCH = 3


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle returned {code}")
        self.code = code


def _stale(so: str, src: str) -> bool:
    return not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, -O2, no vectorisation tricks), and
    the multi-threaded CPU baseline with g++."""
    if force or _stale(_SO, _SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    if force or _stale(_PAR_SO, _PAR_SRC):
        tmp = _PAR_SO + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-Wall", "-Wextra", "-pthread", "-shared",
                               "-fPIC", "-o", tmp, _PAR_SRC])
        os.replace(tmp, _PAR_SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u64, i64 = ctypes.c_uint64, ctypes.c_int64
        lib.oracle_counts.argtypes = [i32p, u64, i64, i64, u64p]
        lib.oracle_sort.argtypes = [i32p, u64, i64, i64, i32p]
        lib.oracle_tile_intermediates.argtypes = [i32p, u64, i64, i64, u64, u64p, u64p, u64p]
        lib.oracle_output_from_local_cdfs.argtypes = [u64p, u64p, i64, i64, u64, u64, i32p]
        lib.oracle_prefix_max_output.argtypes = [u64p, i64, i64, u64, i32p]
        lib.oracle_verify_begin.argtypes = [ctypes.c_void_p, u64p, u64, i64]
        lib.oracle_verify_chunk.argtypes = [ctypes.c_void_p, i32p, u64, u64p]
        lib.oracle_verify_end.argtypes = [ctypes.c_void_p, u64]
        for f in ("oracle_counts", "oracle_sort", "oracle_tile_intermediates",
                  "oracle_output_from_local_cdfs", "oracle_prefix_max_output",
                  "oracle_verify_chunk", "oracle_verify_end"):
            getattr(lib, f).restype = ctypes.c_int
        lib.oracle_verify_begin.restype = None
        _lib = lib
    return _lib


_par_lib = None


def _load_parallel():
    global _par_lib
    if _par_lib is None:
        if not os.path.exists(_PAR_SO):
            build()
        lib = ctypes.CDLL(_PAR_SO)
        lib.cpu_parallel_sort.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_uint64,
                                          ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int)]
        lib.cpu_parallel_sort.restype = ctypes.c_int
        _par_lib = lib
    return _par_lib


def _i32(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _check(rc: int, what: str):
    if rc != ORC_OK:
        raise OracleError(rc, what)


def counts(A, minVal: int, maxVal: int) -> np.ndarray:
    """Sec. 2.1: c_v for v in [0, R), as uint64."""
    A = _i32(A)
    R = int(maxVal) - int(minVal)
    cnt = np.zeros(max(R, 1), dtype=np.uint64)
    rc = _load().oracle_counts(_p(A, ctypes.c_int32), A.size, int(minVal), int(maxVal),
                               _p(cnt, ctypes.c_uint64))
    _check(rc, "oracle_counts")
    return cnt[:R]


def sort(A, minVal: int, maxVal: int) -> np.ndarray:
    """Sec. 2.1 / Theorem 1: the keys in nondecreasing order (plain counting sort)."""
    A = _i32(A)
    B = np.empty(A.size, dtype=np.int32)
    rc = _load().oracle_sort(_p(A, ctypes.c_int32), A.size, int(minVal), int(maxVal),
                             _p(B, ctypes.c_int32))
    _check(rc, "oracle_sort")
    return B


def parallel_sort(A, minVal: int, maxVal: int, threads: int, out=None):
    """Measurement baseline, not an oracle: the counting sort of Sec. 2.1 on
    `threads` host threads (per-thread histograms, parallel merge, parallel
    fill by output position).  Returns (B, threads actually used)."""
    A = _i32(A)
    B = np.empty(A.size, dtype=np.int32) if out is None else out
    if B.dtype != np.int32 or B.size != A.size or not B.flags.c_contiguous:
        raise OracleError(ORC_INVALID_ARGUMENT, "parallel_sort: out")
    used = ctypes.c_int(0)
    rc = _load_parallel().cpu_parallel_sort(_p(A, ctypes.c_int32), A.size, int(minVal),
                                            int(maxVal), int(threads), _p(B, ctypes.c_int32),
                                            ctypes.byref(used))
    _check(rc, "cpu_parallel_sort")
    return B, used.value


def tile_intermediates(A, minVal: int, maxVal: int, T: int):
    """Alg. 4-6: (tile histograms, local CDFs, tile offsets O) for tile width T."""
    A = _i32(A)
    R = int(maxVal) - int(minVal)
    if T <= 0:
        raise OracleError(ORC_INVALID_ARGUMENT, "tile_intermediates")
    m = -(-R // int(T)) if R > 0 else 1
    hist = np.zeros(max(R, 1), dtype=np.uint64)
    cdf = np.zeros(max(R, 1), dtype=np.uint64)
    O = np.zeros(max(m, 1), dtype=np.uint64)
    rc = _load().oracle_tile_intermediates(_p(A, ctypes.c_int32), A.size, int(minVal),
                                           int(maxVal), int(T), _p(hist, ctypes.c_uint64),
                                           _p(cdf, ctypes.c_uint64), _p(O, ctypes.c_uint64))
    _check(rc, "oracle_tile_intermediates")
    return hist[:R], cdf[:R], O[:m]


def output_from_local_cdfs(cdf, O, minVal: int, maxVal: int, T: int, n: int) -> np.ndarray:
    """Alg. 7 over all tiles: B[O[t] + p] = b_t + min{j : C_t[j] >= p + 1}."""
    cdf = np.ascontiguousarray(cdf, dtype=np.uint64)
    O = np.ascontiguousarray(O, dtype=np.uint64)
    B = np.empty(int(n), dtype=np.int32)
    rc = _load().oracle_output_from_local_cdfs(_p(cdf, ctypes.c_uint64), _p(O, ctypes.c_uint64),
                                               int(minVal), int(maxVal), int(T), int(n),
                                               _p(B, ctypes.c_int32))
    _check(rc, "oracle_output_from_local_cdfs")
    return B


def prefix_max_output(P1, minVal: int, maxVal: int, n: int) -> np.ndarray:
    """Alg. 3 (RefHP): step writes at P1[d-1] for every step d, then a prefix maximum."""
    P1 = np.ascontiguousarray(P1, dtype=np.uint64)
    B = np.empty(int(n), dtype=np.int32)
    rc = _load().oracle_prefix_max_output(_p(P1, ctypes.c_uint64), int(minVal), int(maxVal),
                                          int(n), _p(B, ctypes.c_int32))
    _check(rc, "oracle_prefix_max_output")
    return B


class _Cursor(ctypes.Structure):
    _fields_ = [("cnt", ctypes.c_void_p), ("R", ctypes.c_uint64), ("minVal", ctypes.c_int64),
                ("v", ctypes.c_uint64), ("left", ctypes.c_uint64), ("pos", ctypes.c_uint64)]


class StreamingVerifier:
    """Compare a sorted candidate chunk by chunk with the expansion of the counts
    in value order (Sec. 2.1 output intervals), in O(R) memory plus one chunk."""

    def __init__(self, cnt: np.ndarray, minVal: int):
        self._cnt = np.ascontiguousarray(cnt, dtype=np.uint64)
        self._cur = _Cursor()
        _load().oracle_verify_begin(ctypes.byref(self._cur), _p(self._cnt, ctypes.c_uint64),
                                    self._cnt.size, int(minVal))

    def chunk(self, Bchunk) -> None:
        Bchunk = _i32(Bchunk)
        bad = ctypes.c_uint64(0)
        rc = _load().oracle_verify_chunk(ctypes.byref(self._cur), _p(Bchunk, ctypes.c_int32),
                                         Bchunk.size, ctypes.byref(bad))
        if rc != ORC_OK:
            raise OracleError(rc, f"sorted output differs from the oracle at position {bad.value}")

    def end(self, n: int) -> None:
        rc = _load().oracle_verify_end(ctypes.byref(self._cur), int(n))
        _check(rc, "streaming verifier: length")

    @property
    def position(self) -> int:
        return int(self._cur.pos)
