"""Thin Python binding of librtcdf.so (the C ABI in include/rtcdf.h).

Argument marshalling only: every step of the sort runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  The library
is loaded when this module is imported; if it has not been built the import
fails (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtcdf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2609_00843_amd.build`")

# torch ships its own HIP runtime (libamdhip64.so) next to its libraries; the
# library's own dependency is the system libamdhip64.so.7.  Importing torch
# first puts torch's runtime in the global symbol scope, so the library's HIP
# calls bind to the same runtime that owns torch's streams and allocations.
# Loaded the other way round, the process would hold two HIP runtimes and
# torch's stream handles would reach the wrong one.
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)

STATUS = {
    0: "RTCDF_SUCCESS",
    1: "RTCDF_ERROR_INVALID_VALUE",
    2: "RTCDF_ERROR_SIZE_TOO_LARGE",
    3: "RTCDF_ERROR_RANGE_TOO_LARGE",
    4: "RTCDF_ERROR_OVERLAP",
    5: "RTCDF_ERROR_OUT_OF_MEMORY",
    6: "RTCDF_ERROR_HIP",
    7: "RTCDF_ERROR_WORKSPACE_TOO_SMALL",
    8: "RTCDF_ERROR_NOT_SUPPORTED",
    9: "RTCDF_ERROR_NO_MODEL",
    10: "RTCDF_ERROR_KEY_OUT_OF_RANGE",
    11: "RTCDF_ERROR_CAPTURE_NEEDS_WORKSPACE",
}
SUCCESS, INVALID_VALUE, SIZE_TOO_LARGE, RANGE_TOO_LARGE, OVERLAP = 0, 1, 2, 3, 4
OUT_OF_MEMORY, HIP_ERROR, WORKSPACE_TOO_SMALL, NOT_SUPPORTED, NO_MODEL = 5, 6, 7, 8, 9
KEY_OUT_OF_RANGE, CAPTURE_NEEDS_WORKSPACE = 10, 11
MAX_RANGE = 1 << 28
BATCH_MAX_RANGE = 1 << 16
CONFIG_DEFAULT, CONFIG_TUNED, CONFIG_LEARNED = 0, 1, 2


class RtcdfError(RuntimeError):
    def __init__(self, status: int, what: str):
        name = STATUS.get(status, str(status))
        extra = ""
        if status == HIP_ERROR:
            extra = f" (hipError {lib.rtcdf_last_hip_error()})"
        super().__init__(f"{what}: {name}{extra}")
        self.status = status


class Config(ctypes.Structure):
    """rtcdf_config_t: tile width T, items per thread, blocks per tile, flags."""
    _fields_ = [("tile_width", ctypes.c_uint32), ("items_per_thread", ctypes.c_uint32),
                ("blocks_per_tile", ctypes.c_uint32), ("flags", ctypes.c_uint32)]

    def as_tuple(self):
        """(T, items, blocks, flags): the form of the grid points."""
        return (self.tile_width, self.items_per_thread, self.blocks_per_tile, self.flags)

    def __repr__(self):
        extra = f", flags={self.flags}" if self.flags else ""
        return (f"Config(T={self.tile_width}, items={self.items_per_thread}, "
                f"bpt={self.blocks_per_tile}{extra})")


class Segment(ctypes.Structure):
    """rtcdf_segment_t (32 bytes, lives in device memory for the batched call)."""
    _fields_ = [("keys_in", ctypes.c_uint64), ("keys_out", ctypes.c_uint64),
                ("n", ctypes.c_uint32), ("minVal", ctypes.c_int32),
                ("range", ctypes.c_uint32), ("config", ctypes.c_uint32)]


class BatchBounds(ctypes.Structure):
    _fields_ = [("total_keys", ctypes.c_uint64), ("max_n", ctypes.c_uint32),
                ("max_range", ctypes.c_uint32)]


class StageStats(ctypes.Structure):
    _fields_ = [("sorts", ctypes.c_uint64), ("ms", ctypes.c_double * 4)]


STAGES = ("hist", "reduce", "tilescan", "fill")

_vp, _sz, _i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64
_cfgp = ctypes.POINTER(Config)
_u32p = ctypes.c_void_p

_SIGS = {
    "rtcdf_sort": [_vp, _vp, _sz, _i64, _i64, _vp],
    "rtcdf_sort_with_config": [_vp, _vp, _sz, _i64, _i64, _cfgp, _vp],
    "rtcdf_workspace_bytes": [_sz, _i64, _i64, _cfgp, _vp, ctypes.POINTER(ctypes.c_size_t)],
    "rtcdf_sort_ws": [_vp, _vp, _sz, _i64, _i64, _cfgp, _vp, _sz, _vp],
    "rtcdf_sort_noalloc": [_vp, _vp, _sz, _i64, _i64, _cfgp, _vp],
    "rtcdf_debug_intermediates": [_vp, _sz, _i64, _i64, _cfgp, _u32p, _u32p, _u32p, _vp],
    "rtcdf_batched_workspace_bytes": [ctypes.c_uint32, ctypes.POINTER(BatchBounds),
                                      ctypes.POINTER(ctypes.c_size_t)],
    "rtcdf_sort_batched": [_vp, ctypes.c_uint32, ctypes.POINTER(BatchBounds), _vp, _sz, _vp],
    "rtcdf_set_config_mode": [ctypes.c_int],
    "rtcdf_get_config_mode": [],
    "rtcdf_pick_config": [_vp, _sz, _i64, _i64, _vp, _cfgp],
    "rtcdf_status_string": [ctypes.c_int],
    "rtcdf_last_hip_error": [],
    "rtcdf_version": [],
    "rtcdf_release_workspaces": [],
    "rtcdf_profile_enable": [ctypes.c_int],
    "rtcdf_profile_collect": [ctypes.POINTER(StageStats)],
    "rtcdf_stream_copy": [_vp, _vp, _sz, _vp],
    "rtcdf_count_out_of_range": [_vp, _sz, _i64, _i64, _vp, _vp],
    "rtcdf_sort_checked": [_vp, _vp, _sz, _i64, _i64, _cfgp, _vp],
    "rtcdf_sort_keys": [_vp, _vp, _sz, ctypes.c_int, _i64, _i64, _cfgp, _vp],
}
for _name, _args in _SIGS.items():
    if hasattr(lib, _name):
        _f = getattr(lib, _name)
        _f.argtypes = _args
        _f.restype = ctypes.c_int
lib.rtcdf_status_string.restype = ctypes.c_char_p


def _check(st: int, what: str):
    if st != SUCCESS:
        raise RtcdfError(st, what)


# rtcdf_config_t.flags: output by step writes and a prefix maximum (Alg. 3);
# the histogram's counter width; wave-level aggregation of duplicates; output
# chunk size
FLAG_OUTPUT_PREFIX_MAX = 0x01
FLAG_COUNTERS_16 = 0x04
FLAG_COUNTERS_32 = 0x08
FLAG_COUNTERS_4 = 0x40
FLAG_WAVE_DEDUPE = 0x10
FLAG_CHUNK_4096 = 0x20
# how a configuration was chosen (rtcdf_last_pick_source)
PICK_STATIC, PICK_NETWORK, PICK_NETWORK_KEPT_STATIC, PICK_AUTOTUNED, PICK_CACHED, PICK_PENDING = 0, 1, 2, 3, 4, 5


def make_config(tile_width: int, items_per_thread: int = 16, blocks_per_tile: int = 1,
                flags: int = 0) -> Config:
    return Config(int(tile_width), int(items_per_thread), int(blocks_per_tile), int(flags))


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _check_keys(t, what):
    import torch
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous int32 CUDA tensor")


def sort(keys_in, minVal: int, maxVal: int, keys_out=None, config: Config | None = None,
         stream=None):
    """Sort keys_in (int32 in [minVal, maxVal)) into keys_out (allocated if None).
    Asynchronous on `stream` (default: torch's current stream).  int64, int16,
    uint16, int8 and uint8 tensors go to sort_keys."""
    import torch
    if getattr(keys_in, "dtype", None) in (torch.int64, torch.int16, torch.int8, torch.uint8,
                                           getattr(torch, "uint16", None)):
        return sort_keys(keys_in, minVal, maxVal, keys_out=keys_out, config=config, stream=stream)
    _check_keys(keys_in, "keys_in")
    if keys_out is None:
        keys_out = torch.empty_like(keys_in)
    _check_keys(keys_out, "keys_out")
    if keys_out.numel() != keys_in.numel():
        raise ValueError("keys_out must have as many elements as keys_in")
    s = _stream_ptr(stream)
    if config is None:
        st = lib.rtcdf_sort(_ptr(keys_in), _ptr(keys_out), keys_in.numel(), int(minVal),
                            int(maxVal), s)
    else:
        st = lib.rtcdf_sort_with_config(_ptr(keys_in), _ptr(keys_out), keys_in.numel(),
                                        int(minVal), int(maxVal), ctypes.byref(config), s)
    _check(st, "rtcdf_sort")
    return keys_out


# rtcdf_key_type_t
KEY_INT32, KEY_INT16, KEY_UINT16, KEY_INT8, KEY_UINT8, KEY_INT64 = 0, 1, 2, 3, 4, 5


def _key_type(t):
    import torch
    types = {torch.int32: KEY_INT32, torch.int16: KEY_INT16, torch.int8: KEY_INT8, torch.uint8: KEY_UINT8,
             torch.int64: KEY_INT64}
    if hasattr(torch, "uint16"):
        types[torch.uint16] = KEY_UINT16
    if t.dtype not in types or not t.is_cuda or not t.is_contiguous():
        raise TypeError("keys must be a contiguous CUDA tensor of int32, int64, int16, uint16, int8 or uint8")
    return types[t.dtype]


def sort_keys(keys_in, minVal: int, maxVal: int, keys_out=None, config: Config | None = None,
              stream=None):
    """Sort int32, int64, int16, uint16, int8 or uint8 keys in [minVal, maxVal)
    into keys_out (same dtype; allocated if None).  Asynchronous on `stream`."""
    import torch
    kt = _key_type(keys_in)
    if keys_out is None:
        keys_out = torch.empty_like(keys_in)
    if keys_out.dtype != keys_in.dtype or keys_out.numel() != keys_in.numel():
        raise ValueError("keys_out must match keys_in in dtype and size")
    _key_type(keys_out)
    st = lib.rtcdf_sort_keys(_ptr(keys_in), _ptr(keys_out), keys_in.numel(), kt, int(minVal), int(maxVal),
                             ctypes.byref(config) if config is not None else None, _stream_ptr(stream))
    _check(st, "rtcdf_sort_keys")
    return keys_out


def count_out_of_range(keys, minVal: int, maxVal: int, out=None, stream=None):
    """Number of keys outside [minVal, maxVal), as a one-element int64 CUDA
    tensor filled asynchronously on `stream` (checked mode)."""
    import torch
    _check_keys(keys, "keys")
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=keys.device)
    st = lib.rtcdf_count_out_of_range(_ptr(keys), keys.numel(), int(minVal), int(maxVal), _ptr(out),
                                      _stream_ptr(stream))
    _check(st, "rtcdf_count_out_of_range")
    return out


def sort_checked(keys_in, minVal: int, maxVal: int, keys_out=None, config: Config | None = None,
                 stream=None):
    """sort() that first verifies every key lies in [minVal, maxVal) (waits for
    that count); raises RtcdfError with status KEY_OUT_OF_RANGE otherwise,
    leaving keys_out unchanged."""
    import torch
    _check_keys(keys_in, "keys_in")
    if keys_out is None:
        keys_out = torch.empty_like(keys_in)
    _check_keys(keys_out, "keys_out")
    if keys_out.numel() != keys_in.numel():
        raise ValueError("keys_out must have as many elements as keys_in")
    st = lib.rtcdf_sort_checked(_ptr(keys_in), _ptr(keys_out), keys_in.numel(), int(minVal), int(maxVal),
                                ctypes.byref(config) if config is not None else None, _stream_ptr(stream))
    _check(st, "rtcdf_sort_checked")
    return keys_out


def workspace_bytes(n: int, minVal: int, maxVal: int, config: Config | None = None,
                    keys_out=None) -> int:
    out = ctypes.c_size_t(0)
    st = lib.rtcdf_workspace_bytes(int(n), int(minVal), int(maxVal),
                                   ctypes.byref(config) if config is not None else None,
                                   _ptr(keys_out) if keys_out is not None else None,
                                   ctypes.byref(out))
    _check(st, "rtcdf_workspace_bytes")
    return int(out.value)


def sort_ws(keys_in, keys_out, minVal: int, maxVal: int, workspace, config: Config | None = None,
            stream=None):
    """Sort with a caller-owned device workspace (a uint8 CUDA tensor)."""
    _check_keys(keys_in, "keys_in")
    _check_keys(keys_out, "keys_out")
    st = lib.rtcdf_sort_ws(_ptr(keys_in), _ptr(keys_out), keys_in.numel(), int(minVal),
                           int(maxVal), ctypes.byref(config) if config is not None else None,
                           _ptr(workspace), workspace.numel() * workspace.element_size(),
                           _stream_ptr(stream))
    _check(st, "rtcdf_sort_ws")
    return keys_out


NOALLOC_MAX_WORKSPACE = 64 << 20


def sort_noalloc(keys_in, keys_out, minVal: int, maxVal: int, config: Config | None = None,
                 stream=None):
    """Sort with the library's fixed device workspace (no allocation); calls
    on one GPU must not overlap in time."""
    _check_keys(keys_in, "keys_in")
    _check_keys(keys_out, "keys_out")
    st = lib.rtcdf_sort_noalloc(_ptr(keys_in), _ptr(keys_out), keys_in.numel(), int(minVal), int(maxVal),
                                ctypes.byref(config) if config is not None else None, _stream_ptr(stream))
    _check(st, "rtcdf_sort_noalloc")
    return keys_out


def debug_intermediates(keys_in, minVal: int, maxVal: int, config: Config, stream=None):
    """(tile histograms, local CDFs, tile offsets) as int32 CUDA tensors holding
    uint32 values (Alg. 5, Alg. 4, Alg. 6)."""
    import torch
    _check_keys(keys_in, "keys_in")
    R = int(maxVal) - int(minVal)
    T = min(config.tile_width, (R + 127) // 128 * 128)
    m = -(-R // T)
    dev = keys_in.device
    hist = torch.empty(R, dtype=torch.int32, device=dev)
    cdf = torch.empty(R, dtype=torch.int32, device=dev)
    O = torch.empty(m, dtype=torch.int32, device=dev)
    st = lib.rtcdf_debug_intermediates(_ptr(keys_in), keys_in.numel(), int(minVal), int(maxVal),
                                       ctypes.byref(config), _ptr(hist), _ptr(cdf), _ptr(O),
                                       _stream_ptr(stream))
    _check(st, "rtcdf_debug_intermediates")
    return hist, cdf, O


def set_config_mode(mode: int):
    _check(lib.rtcdf_set_config_mode(int(mode)), "rtcdf_set_config_mode")


def get_config_mode() -> int:
    return int(lib.rtcdf_get_config_mode())


def pick_config(n: int, minVal: int, maxVal: int, keys_in=None, stream=None) -> Config:
    cfg = Config()
    st = lib.rtcdf_pick_config(_ptr(keys_in) if keys_in is not None else None, int(n), int(minVal),
                               int(maxVal), _stream_ptr(stream) if keys_in is not None else None,
                               ctypes.byref(cfg))
    _check(st, "rtcdf_pick_config")
    return cfg


def status_string(status: int) -> str:
    return lib.rtcdf_status_string(int(status)).decode()


def release_workspaces():
    _check(lib.rtcdf_release_workspaces(), "rtcdf_release_workspaces")


def profile_enable(on: bool = True):
    _check(lib.rtcdf_profile_enable(1 if on else 0), "rtcdf_profile_enable")


def profile_collect() -> dict:
    """{'sorts': k, 'hist': ms, 'reduce': ms, 'tilescan': ms, 'fill': ms} summed
    over the sorts recorded since the last collect."""
    st = StageStats()
    _check(lib.rtcdf_profile_collect(ctypes.byref(st)), "rtcdf_profile_collect")
    d = {"sorts": int(st.sorts)}
    for i, k in enumerate(STAGES):
        d[k] = float(st.ms[i])
    return d


def stream_copy(src, dst, stream=None):
    """Copy src into dst (same byte size, multiple of 16) with the library's
    plain streaming kernel (the attainable-bandwidth reference)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("size mismatch")
    _check(lib.rtcdf_stream_copy(_ptr(src), _ptr(dst), nb, _stream_ptr(stream)), "rtcdf_stream_copy")


# ---- batched sort

def make_segments(pairs, device="cuda", configs=None):
    """Device descriptor array and host bounds for rtcdf_sort_batched.

    pairs: iterable of (keys_in, keys_out, minVal, maxVal) with int32 CUDA
    tensors.  configs: None (every segment's config 0), a list with one
    config word per segment (keys per thread per load step: 4, 8 or 16), or
    "auto": the items_per_thread of the configuration the current config mode
    chooses for each segment's (n, range).  Returns (descriptors as a uint8
    CUDA tensor, BatchBounds, count)."""
    import torch
    pairs = list(pairs)
    if isinstance(configs, str) and configs == "auto":
        configs = [pick_config(max(a.numel(), 1), lo, hi).items_per_thread for a, _, lo, hi in pairs]
    elif configs is not None and len(configs) != len(pairs):
        raise ValueError("one config per segment")
    arr = (Segment * max(len(pairs), 1))()
    total, max_n, max_r = 0, 0, 0
    for i, (a, b, lo, hi) in enumerate(pairs):
        R = int(hi) - int(lo)
        if R < 1 or R > BATCH_MAX_RANGE or lo < -(2 ** 31) or hi > 2 ** 31:
            raise ValueError(f"segment {i}: range [{lo}, {hi}) not supported by the batched sort")
        n = a.numel()
        arr[i] = Segment(a.data_ptr() if n else 0, b.data_ptr() if n else 0, n, int(lo), R,
                         int(configs[i]) if configs is not None else 0)
        total += n
        max_n = max(max_n, n)
        max_r = max(max_r, R)
    raw = bytes(arr)[: ctypes.sizeof(Segment) * len(pairs)]
    host = torch.frombuffer(bytearray(raw), dtype=torch.uint8) if raw else torch.zeros(0, dtype=torch.uint8)
    return host.to(device), BatchBounds(total, max_n, max_r), len(pairs)


def batched_workspace_bytes(num_segments: int, bounds: BatchBounds) -> int:
    out = ctypes.c_size_t(0)
    _check(lib.rtcdf_batched_workspace_bytes(int(num_segments), ctypes.byref(bounds), ctypes.byref(out)),
           "rtcdf_batched_workspace_bytes")
    return int(out.value)


def sort_batched(d_segments, num_segments: int, bounds: BatchBounds, workspace, stream=None):
    """rtcdf_sort_batched on a device descriptor array (uint8 CUDA tensor)."""
    st = lib.rtcdf_sort_batched(_ptr(d_segments), int(num_segments), ctypes.byref(bounds),
                                _ptr(workspace), workspace.numel() * workspace.element_size(),
                                _stream_ptr(stream))
    _check(st, "rtcdf_sort_batched")


# ---- configuration grid, autotuner, learned picker

GRID_SIZE = 62
MLP_INPUTS, MLP_HIDDEN, MLP_OUTPUTS, MLP_PARAMS = 34, 64, 62, 10430
SKETCH_BINS, SKETCH_SAMPLES = 32, 4096

_fp = ctypes.c_void_p
for _name, _args in {
    "rtcdf_config_grid": [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_uint8)],
    "rtcdf_autotune": [_vp, _vp, _sz, _i64, _i64, ctypes.c_uint32, ctypes.c_uint32,
                       ctypes.POINTER(ctypes.c_float), _cfgp, _vp],
    "rtcdf_load_tuned_table": [ctypes.c_char_p],
    "rtcdf_load_model": [ctypes.c_char_p],
    "rtcdf_unload_model": [],
    "rtcdf_set_learned_fallback": [ctypes.c_int],
    "rtcdf_clear_pick_cache": [],
    "rtcdf_last_pick_source": [],
    "rtcdf_last_pick_index": [],
    "rtcdf_sketch": [_vp, _sz, _i64, _i64, _fp, _vp],
    "rtcdf_mlp_forward": [_fp, _fp, ctypes.c_uint32, _fp, _vp],
    "rtcdf_mlp_workspace_bytes": [ctypes.c_uint32, ctypes.POINTER(ctypes.c_size_t)],
    "rtcdf_mlp_gradient": [_fp, _fp, _fp, _fp, ctypes.c_uint32, _fp, _fp, _vp, _sz, _vp],
    "rtcdf_mlp_adam_step": [_fp, _fp, _fp, _fp, ctypes.c_uint32, ctypes.c_float, ctypes.c_float,
                            ctypes.c_float, ctypes.c_float, _vp],
    "rtcdf_mlp_train": [_fp, _fp, _fp, ctypes.c_uint32, _fp, _fp, _fp, ctypes.c_uint32,
                        ctypes.c_uint32, ctypes.c_float, _vp, _sz, _fp, _vp],
    "rtcdf_mlp_pick": [_vp, _sz, _i64, _i64, _fp, _fp, _vp, _vp, _fp, _vp],
}.items():
    if hasattr(lib, _name):
        getattr(lib, _name).argtypes = _args
        getattr(lib, _name).restype = ctypes.c_int


def config_grid():
    """[(T, items, blocks, flags)] * GRID_SIZE (option points as (0, 0, 0,
    flags)) and the validity mask."""
    cfgs = (Config * GRID_SIZE)()
    valid = (ctypes.c_uint8 * GRID_SIZE)()
    _check(lib.rtcdf_config_grid(cfgs, valid), "rtcdf_config_grid")
    return [c.as_tuple() for c in cfgs], [bool(v) for v in valid]


def autotune(keys_in, minVal: int, maxVal: int, keys_out=None, warmup: int = 2, reps: int = 5,
             stream=None):
    """Median ms of every grid configuration (-1 for invalid ones) and the best config."""
    import torch
    if keys_out is None:
        keys_out = torch.empty_like(keys_in)
    times = (ctypes.c_float * GRID_SIZE)()
    best = Config()
    _check(lib.rtcdf_autotune(_ptr(keys_in), _ptr(keys_out), keys_in.numel(), int(minVal), int(maxVal),
                              int(warmup), int(reps), times, ctypes.byref(best), _stream_ptr(stream)),
           "rtcdf_autotune")
    return [float(t) for t in times], best


def load_tuned_table(path: str):
    _check(lib.rtcdf_load_tuned_table(os.fsencode(path)), "rtcdf_load_tuned_table")


def load_model(path: str):
    _check(lib.rtcdf_load_model(os.fsencode(path)), "rtcdf_load_model")


def unload_model():
    _check(lib.rtcdf_unload_model(), "rtcdf_unload_model")


def set_learned_fallback(on: bool):
    _check(lib.rtcdf_set_learned_fallback(1 if on else 0), "rtcdf_set_learned_fallback")


def clear_pick_cache():
    _check(lib.rtcdf_clear_pick_cache(), "rtcdf_clear_pick_cache")


def last_pick() -> tuple:
    """(grid index or -1, PICK_* source) of the last choice on this thread."""
    return int(lib.rtcdf_last_pick_index()), int(lib.rtcdf_last_pick_source())


def sketch(keys_in, minVal: int, maxVal: int, out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty(MLP_INPUTS, dtype=torch.float32, device=keys_in.device)
    _check(lib.rtcdf_sketch(_ptr(keys_in), keys_in.numel(), int(minVal), int(maxVal), _ptr(out),
                            _stream_ptr(stream)), "rtcdf_sketch")
    return out


def _check_mlp(params=None, X=None, rows=None, what="mlp"):
    """Shape checks of the picker's device arrays (the kernels index them by
    the network's fixed sizes)."""
    if params is not None and params.numel() != MLP_PARAMS:
        raise ValueError(f"{what}: params must hold {MLP_PARAMS} floats")
    if X is not None and (X.dim() != 2 or X.shape[1] != MLP_INPUTS):
        raise ValueError(f"{what}: X must be batch x {MLP_INPUTS}")
    for t in rows or ():
        if X is not None and t.numel() != X.shape[0] * MLP_OUTPUTS:
            raise ValueError(f"{what}: targets and mask must be batch x {MLP_OUTPUTS}")


def mlp_forward(params, X, stream=None):
    import torch
    _check_mlp(params, X, what="mlp_forward")
    B = X.shape[0]
    Y = torch.empty((B, MLP_OUTPUTS), dtype=torch.float32, device=X.device)
    _check(lib.rtcdf_mlp_forward(_ptr(params), _ptr(X), B, _ptr(Y), _stream_ptr(stream)),
           "rtcdf_mlp_forward")
    return Y


def mlp_workspace(batch: int, device="cuda"):
    import torch
    nb = ctypes.c_size_t(0)
    _check(lib.rtcdf_mlp_workspace_bytes(int(batch), ctypes.byref(nb)), "rtcdf_mlp_workspace_bytes")
    return torch.empty(int(nb.value), dtype=torch.uint8, device=device)


def mlp_gradient(params, X, T, M, ws=None, stream=None):
    """(gradient, loss) of the masked MSE at params."""
    import torch
    _check_mlp(params, X, (T, M), what="mlp_gradient")
    B = X.shape[0]
    if ws is None:
        ws = mlp_workspace(B, X.device)
    G = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
    L = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(lib.rtcdf_mlp_gradient(_ptr(params), _ptr(X), _ptr(T), _ptr(M), B, _ptr(G), _ptr(L), _ptr(ws),
                                  ws.numel(), _stream_ptr(stream)), "rtcdf_mlp_gradient")
    return G, L


def mlp_adam_step(params, grad, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    for a in (params, grad, m, v):
        _check_mlp(a, what="mlp_adam_step")
    _check(lib.rtcdf_mlp_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(t), lr, beta1, beta2,
                                   eps, _stream_ptr(stream)), "rtcdf_mlp_adam_step")


def mlp_train(params, m, v, t0: int, X, T, M, steps: int, lr: float, ws=None, loss_history=None,
              stream=None):
    for a in (params, m, v):
        _check_mlp(a, what="mlp_train")
    _check_mlp(None, X, (T, M), what="mlp_train")
    if loss_history is not None and loss_history.numel() < steps:
        raise ValueError("mlp_train: loss_history must hold one float per step")
    B = X.shape[0]
    if ws is None:
        ws = mlp_workspace(B, X.device)
    _check(lib.rtcdf_mlp_train(_ptr(params), _ptr(m), _ptr(v), int(t0), _ptr(X), _ptr(T), _ptr(M), B,
                               int(steps), float(lr), _ptr(ws), ws.numel(),
                               _ptr(loss_history) if loss_history is not None else None,
                               _stream_ptr(stream)), "rtcdf_mlp_train")


def mlp_pick(keys_in, minVal: int, maxVal: int, params, norm, valid, stream=None):
    """(index tensor[1], predictions tensor[MLP_OUTPUTS]) on the device."""
    import torch
    _check_mlp(params, what="mlp_pick")
    if norm.numel() != 2 * MLP_INPUTS or valid.numel() != MLP_OUTPUTS:
        raise ValueError("mlp_pick: norm must hold 2 x 34 floats and valid one byte per grid point")
    idx = torch.empty(1, dtype=torch.int32, device=keys_in.device)
    pred = torch.empty(MLP_OUTPUTS, dtype=torch.float32, device=keys_in.device)
    _check(lib.rtcdf_mlp_pick(_ptr(keys_in), keys_in.numel(), int(minVal), int(maxVal), _ptr(params),
                              _ptr(norm), _ptr(valid), _ptr(idx), _ptr(pred), _stream_ptr(stream)),
           "rtcdf_mlp_pick")
    return idx, pred


class PlanInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint32) for k in (
        "tile_width", "tiles", "counter_bits", "passes", "pass_bins", "hist_workgroups",
        "hist_threads", "items_per_thread", "scan_workgroups", "out_chunk", "out_chunks",
        "fill_workgroups")] + [("workspace_bytes", ctypes.c_uint64), ("output_flags", ctypes.c_uint32),
                                ("partition_buckets", ctypes.c_uint32), ("hist_dedupe", ctypes.c_uint32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


if hasattr(lib, "rtcdf_plan_info"):
    lib.rtcdf_plan_info.argtypes = [_sz, _i64, _i64, _cfgp, _vp, _vp, ctypes.POINTER(PlanInfo)]
    lib.rtcdf_plan_info.restype = ctypes.c_int


def plan_info(n: int, minVal: int, maxVal: int, config: Config | None = None, keys_in=None,
              keys_out=None) -> dict:
    out = PlanInfo()
    _check(lib.rtcdf_plan_info(int(n), int(minVal), int(maxVal),
                               ctypes.byref(config) if config is not None else None,
                               _ptr(keys_in) if keys_in is not None else None,
                               _ptr(keys_out) if keys_out is not None else None, ctypes.byref(out)),
           "rtcdf_plan_info")
    return out.as_dict()
