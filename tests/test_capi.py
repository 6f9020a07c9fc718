"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point include/rtcdf.h declares, and rejects bad arguments before any GPU
work.  The calls made here never reach a HIP API."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rtcdf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rtcdf_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def r():
    from paper_2609_00843_amd import rtcdf
    return rtcdf


def test_every_declared_symbol_is_exported(r):
    names = _declared()
    assert "rtcdf_sort" in names and "rtcdf_sort_batched" in names
    missing = [n for n in names if not hasattr(r.lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_version_and_strings(r):
    assert r.lib.rtcdf_version() >= 100
    for code, name in r.STATUS.items():
        assert r.status_string(code) and r.status_string(code) != "unknown status"
    assert r.status_string(99) == "unknown status"


P_IN, P_OUT = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30)   # never dereferenced


def test_argument_errors_before_gpu(r):
    L = r.lib
    sort = L.rtcdf_sort
    assert sort(P_IN, P_OUT, 0, 0, 10, None) == r.SUCCESS                 # n = 0 is a no-op
    assert sort(P_IN, P_OUT, 10, 5, 5, None) == r.INVALID_VALUE           # empty range
    assert sort(P_IN, P_OUT, 10, 6, 5, None) == r.INVALID_VALUE
    assert sort(P_IN, P_OUT, 10, -(2 ** 31) - 1, 0, None) == r.INVALID_VALUE
    assert sort(P_IN, P_OUT, 10, 0, 2 ** 31 + 1, None) == r.INVALID_VALUE
    assert sort(P_IN, P_OUT, 10, 0, (1 << 28) + 1, None) == r.RANGE_TOO_LARGE
    assert sort(P_IN, P_OUT, (1 << 40) + 1, 0, 10, None) == r.SIZE_TOO_LARGE   # n >= 2^32 is taken up to 2^40
    assert sort(None, P_OUT, 10, 0, 10, None) == r.INVALID_VALUE
    assert sort(P_IN, None, 10, 0, 10, None) == r.INVALID_VALUE
    assert sort(ctypes.c_void_p((1 << 20) + 2), P_OUT, 10, 0, 10, None) == r.INVALID_VALUE  # not 4-byte aligned
    # partial overlap is rejected, exact aliasing is not an argument error
    assert sort(P_IN, ctypes.c_void_p((1 << 20) + 8), 10, 0, 10, None) == r.OVERLAP
    assert sort(P_IN, ctypes.c_void_p((1 << 20) - 8), 10, 0, 10, None) == r.OVERLAP


def test_checked_mode_argument_errors(r):
    L = r.lib
    cnt = ctypes.c_void_p(1 << 24)                                        # never dereferenced
    assert L.rtcdf_count_out_of_range(P_IN, 10, 0, 10, None, None) == r.INVALID_VALUE
    assert L.rtcdf_count_out_of_range(P_IN, 10, 0, 10, ctypes.c_void_p((1 << 24) + 4), None) == r.INVALID_VALUE
    assert L.rtcdf_count_out_of_range(P_IN, 10, 5, 5, cnt, None) == r.INVALID_VALUE
    assert L.rtcdf_count_out_of_range(None, 10, 0, 10, cnt, None) == r.INVALID_VALUE
    assert L.rtcdf_count_out_of_range(P_IN, (1 << 40) + 1, 0, 10, cnt, None) == r.SIZE_TOO_LARGE
    sc = L.rtcdf_sort_checked
    assert sc(P_IN, P_OUT, 0, 0, 10, None, None) == r.SUCCESS                # n = 0 is a no-op
    assert sc(P_IN, P_OUT, 10, 0, (1 << 28) + 1, None, None) == r.RANGE_TOO_LARGE
    assert sc(P_IN, ctypes.c_void_p((1 << 20) + 8), 10, 0, 10, None, None) == r.OVERLAP
    bad = r.Config(100, 16, 1, 0)
    assert sc(P_IN, P_OUT, 10, 0, 10, ctypes.byref(bad), None) == r.INVALID_VALUE
    assert r.status_string(r.KEY_OUT_OF_RANGE) == "a key lies outside [minVal, maxVal)"


@pytest.mark.parametrize("cfg", [(100, 16, 1), (0, 16, 1), (1024, 5, 1), (1024, 16, 3),
                                 (32768, 16, 2), (16384, 16, 4), (32896, 16, 1), (1024, 0, 1),
                                 (1024, 16, 1, 2), (1024, 16, 1, 3), (1024, 16, 1, 1 << 31),
                                 (100, 16, 1, 1)])
def test_invalid_configs(r, cfg):
    c = r.make_config(*cfg)
    assert r.lib.rtcdf_sort_with_config(P_IN, P_OUT, 10, 0, 10, ctypes.byref(c), None) == r.INVALID_VALUE


def test_config_mode_api(r):
    assert r.lib.rtcdf_set_config_mode(7) == r.INVALID_VALUE
    old = r.get_config_mode()
    r.set_config_mode(r.CONFIG_DEFAULT)
    assert r.get_config_mode() == r.CONFIG_DEFAULT
    r.set_config_mode(old)


def test_load_fails_loudly_without_library(tmp_path):
    """The binding has no fallback: without the built library the import fails."""
    import subprocess
    import sys
    code = ("import sys, os; sys.path.insert(0, %r); import paper_2609_00843_amd.rtcdf as m" % str(tmp_path))
    pkg = tmp_path / "paper_2609_00843_amd"
    pkg.mkdir()
    (pkg / "__init__.py").write_text("")
    (pkg / "rtcdf.py").write_text(open(os.path.join(ROOT, "paper_2609_00843_amd", "rtcdf.py")).read())
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert res.returncode != 0 and "not built" in res.stderr


def test_batched_argument_errors(r):
    L = r.lib
    b = r.BatchBounds(10, 10, 100)
    out = ctypes.c_size_t(0)
    assert L.rtcdf_batched_workspace_bytes(4, None, ctypes.byref(out)) == r.INVALID_VALUE
    assert L.rtcdf_batched_workspace_bytes(4, ctypes.byref(b), None) == r.INVALID_VALUE
    big = r.BatchBounds(10, 10, (1 << 16) + 1)
    assert L.rtcdf_batched_workspace_bytes(4, ctypes.byref(big), ctypes.byref(out)) == r.RANGE_TOO_LARGE
    ws = ctypes.c_void_p(1 << 20)
    assert L.rtcdf_sort_batched(P_IN, 0, ctypes.byref(b), ws, 1 << 20, None) == r.SUCCESS     # empty batch
    assert L.rtcdf_sort_batched(None, 4, ctypes.byref(b), ws, 1 << 20, None) == r.INVALID_VALUE
    assert L.rtcdf_sort_batched(P_IN, 4, None, ws, 1 << 20, None) == r.INVALID_VALUE
    assert L.rtcdf_sort_batched(P_IN, 4, ctypes.byref(b), None, 1 << 20, None) == r.INVALID_VALUE
    assert L.rtcdf_sort_batched(P_IN, 4, ctypes.byref(b), ctypes.c_void_p((1 << 20) + 64), 1 << 20,
                                None) == r.INVALID_VALUE                                       # ws not 256-aligned
    assert L.rtcdf_sort_batched(P_IN, 4, ctypes.byref(big), ws, 1 << 20, None) == r.RANGE_TOO_LARGE


def test_segment_layout(r):
    assert ctypes.sizeof(r.Segment) == 32
    assert ctypes.sizeof(r.BatchBounds) == 16
    assert ctypes.sizeof(r.Config) == 16
    # 12 uint32, uint64 workspace_bytes, output_flags, partition_buckets,
    # hist_dedupe, padded to 8 bytes
    assert ctypes.sizeof(r.PlanInfo) == 72
    assert ctypes.sizeof(r.StageStats) == 40


def test_flags_and_sizes_match_header(r):
    txt = open(os.path.join(ROOT, "include", "rtcdf.h")).read()
    for name in ("OUTPUT_PREFIX_MAX", "COUNTERS_16", "COUNTERS_32", "COUNTERS_4", "WAVE_DEDUPE", "CHUNK_4096"):
        m = re.search(r"#define\s+RTCDF_FLAG_%s\s+(0x[0-9a-f]+|\d+)u" % name, txt)
        assert m and int(m.group(1), 0) == getattr(r, "FLAG_" + name), name
    for name, val in (("GRID_SIZE", r.GRID_SIZE), ("MLP_OUTPUTS", r.MLP_OUTPUTS), ("MLP_PARAMS", r.MLP_PARAMS),
                      ("NOALLOC_MAX_WORKSPACE", r.NOALLOC_MAX_WORKSPACE)):
        m = re.search(r"#define\s+RTCDF_%s\s+\(?(\d+)u?( << (\d+))?" % name, txt)
        assert m, name
        got = int(m.group(1)) << (int(m.group(3)) if m.group(3) else 0)
        assert got == val, name


def test_config_validation(r):
    """Option flags: known bits only, at most one counter width; a config
    with zero knobs and some flags is valid (the static knobs with those
    flags)."""
    L = r.lib
    c_in, c_out = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30)
    def st(cfg):
        return L.rtcdf_sort_with_config(c_in, c_out, 10, 0, 100, ctypes.byref(cfg), None)
    assert st(r.make_config(1024, 16, 1, flags=0x80)) == r.INVALID_VALUE          # unknown bit
    for two in (0x0c, 0x44, 0x48, 0x4c):                                          # two widths
        assert st(r.make_config(1024, 16, 1, flags=two)) == r.INVALID_VALUE
        assert st(r.make_config(0, 0, 0, flags=two)) == r.INVALID_VALUE
    assert st(r.make_config(0, 16, 1, flags=0x04)) == r.INVALID_VALUE             # partly zero


def test_sort_keys_argument_errors(r):
    """rtcdf_sort_keys rejects bad key types, ranges outside the type, bad
    pointers and configurations before any GPU work."""
    L, c_in, c_out = r.lib, ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30)
    sk = lambda kt, lo, hi, n=10, a=c_in, b=c_out, cfg=None: L.rtcdf_sort_keys(a, b, n, kt, lo, hi, cfg, None)
    assert sk(7, 0, 10) == r.INVALID_VALUE
    assert sk(-1, 0, 10) == r.INVALID_VALUE
    assert sk(r.KEY_INT16, -32769, 0) == r.INVALID_VALUE
    assert sk(r.KEY_INT16, 0, 32769) == r.INVALID_VALUE
    assert sk(r.KEY_UINT16, -1, 5) == r.INVALID_VALUE
    assert sk(r.KEY_UINT16, 0, 65537) == r.INVALID_VALUE
    assert sk(r.KEY_INT8, -129, 0) == r.INVALID_VALUE
    assert sk(r.KEY_UINT8, 0, 257) == r.INVALID_VALUE
    assert sk(r.KEY_UINT8, 5, 5) == r.INVALID_VALUE
    assert sk(r.KEY_INT16, -32768, 32768, n=(1 << 40) + 1) == r.SIZE_TOO_LARGE
    assert sk(r.KEY_INT16, -32768, 32768, n=0) == r.SUCCESS                  # no-op
    assert sk(r.KEY_INT16, 0, 10, a=None) == r.INVALID_VALUE
    assert sk(r.KEY_INT16, 0, 10, a=ctypes.c_void_p((1 << 20) + 1)) == r.INVALID_VALUE   # odd address
    assert sk(r.KEY_UINT8, 0, 10, b=ctypes.c_void_p((1 << 20) + 5)) == r.OVERLAP
    assert sk(r.KEY_INT16, 0, 10, b=ctypes.c_void_p((1 << 20) - 4)) == r.OVERLAP
    pm = r.make_config(1024, 16, 1, flags=r.FLAG_OUTPUT_PREFIX_MAX)
    assert sk(r.KEY_INT16, 0, 10, cfg=ctypes.byref(pm)) == r.INVALID_VALUE
    bad = r.Config(100, 16, 1, 0)
    assert sk(r.KEY_UINT8, 0, 10, cfg=ctypes.byref(bad)) == r.INVALID_VALUE
    assert sk(r.KEY_INT32, 0, 10, n=(1 << 40) + 1) == r.SIZE_TOO_LARGE       # the int32 entry's checks
    # int64 keys: any window of at most RTCDF_MAX_RANGE values below INT64_MAX
    i64min, i64max = -(1 << 63), (1 << 63) - 1
    assert sk(r.KEY_INT64, i64min, i64min + (1 << 28) + 1) == r.RANGE_TOO_LARGE
    assert sk(r.KEY_INT64, i64min, i64max) == r.RANGE_TOO_LARGE
    assert sk(r.KEY_INT64, 5, 5) == r.INVALID_VALUE
    assert sk(r.KEY_INT64, 0, 10, n=(1 << 40) + 1) == r.SIZE_TOO_LARGE
    assert sk(r.KEY_INT64, 0, 10, a=ctypes.c_void_p((1 << 20) + 4)) == r.INVALID_VALUE   # 8-byte alignment
    assert sk(r.KEY_INT64, 0, 10, b=ctypes.c_void_p((1 << 20) + 72)) == r.OVERLAP        # 80 bytes from 2^20
    assert sk(r.KEY_INT64, 0, 10, cfg=ctypes.byref(pm)) == r.INVALID_VALUE


def test_wide_sorts_limits(r):
    """n >= 2^32 is sorted (64-bit counts) up to 2^40 keys; the calls that
    describe one plain plan (plan info, intermediates) stay below 2^32."""
    L = r.lib
    info = r.PlanInfo()
    assert L.rtcdf_plan_info(1 << 32, 0, 10, None, None, None, ctypes.byref(info)) == r.SIZE_TOO_LARGE
    assert L.rtcdf_debug_intermediates(P_IN, 1 << 32, 0, 10, None, None, None, None, None) == r.SIZE_TOO_LARGE
    size = ctypes.c_size_t(0)
    assert L.rtcdf_workspace_bytes((1 << 40) + 1, 0, 10, None, None, ctypes.byref(size)) == r.SIZE_TOO_LARGE
    assert L.rtcdf_sort_ws(P_IN, P_IN, (1 << 40) + 1, 0, 10, None, ctypes.c_void_p(1 << 24), 1 << 20,
                           None) == r.SIZE_TOO_LARGE
    # above 2^32 the argument checks still come first: overlap, alignment
    assert L.rtcdf_sort(P_IN, P_OUT, 1 << 32, 0, 10, None) == r.OVERLAP
    assert L.rtcdf_sort(ctypes.c_void_p((1 << 20) + 2), ctypes.c_void_p(1 << 40), 1 << 32, 0, 10,
                        None) == r.INVALID_VALUE
