"""Host logic of the tuning tables and the model file (no GPU): the product's
static-table selection agrees with the reference rule, the tables and the
model file load into the library, and DEFAULT / TUNED picks follow them."""
import math
import os

import numpy as np
import pytest

from oracle import tune_ref
from paper_2609_00843_amd import learn, tune


def _rows(seed):
    rng = np.random.default_rng(seed)
    _, valid = tune.grid()
    rows = []
    for i in range(60):
        R = int(2 ** rng.uniform(7, 18))
        n = int(10 ** rng.uniform(6, 9))
        t = rng.uniform(0.5, 2.0, size=54) * (n / 1e7)
        t = [float(x) if v else -1.0 for x, v in zip(t, valid)]
        rows.append({"key": f"k{i}", "n": n, "minVal": 0, "R": R, "dist": "uniform", "sd_div": 6.0,
                     "features": list(rng.random(34)), "times_ms": t})
    return rows


def test_grid_matches_library():
    from paper_2609_00843_amd import rtcdf
    pts, valid = tune.grid()
    lp, lv = rtcdf.config_grid()
    assert pts == lp and valid == lv and sum(valid) == 45


def test_static_selection_matches_reference():
    rows = _rows(1)
    _, valid = tune.grid()
    ref_rows = [(tune.range_class(r["R"]), r["key"], j, r["times_ms"][j])
                for r in rows for j in range(54) if valid[j]]
    assert tune.select_static(rows) == tune_ref.select_per_range(ref_rows)


def test_default_and_tuned_tables_drive_the_pick(tmp_path):
    from paper_2609_00843_amd import rtcdf
    rows = _rows(2)
    tuned = tmp_path / "tuned.txt"
    tune.write_tuned_table(rows, str(tuned))
    rtcdf.load_tuned_table(str(tuned))
    pts, valid = tune.grid()
    old = rtcdf.get_config_mode()
    try:
        rtcdf.set_config_mode(rtcdf.CONFIG_TUNED)
        for r in rows[:10]:
            best = min((t, j) for j, t in enumerate(r["times_ms"]) if valid[j])[1]
            got = rtcdf.pick_config(r["n"], 0, r["R"]).as_tuple()
            assert got == pts[best]
    finally:
        rtcdf.set_config_mode(old)
    bad = tmp_path / "bad.txt"
    bad.write_text("10 7 1000 16 1\n")        # T not a multiple of 128
    with pytest.raises(rtcdf.RtcdfError):
        rtcdf.load_tuned_table(str(bad))


def test_model_file_round_trip(tmp_path):
    from paper_2609_00843_amd import rtcdf
    p = learn.init_params(5)
    mu, sd = np.zeros(34), np.ones(34)
    path = str(tmp_path / "m.bin")
    learn.save_model(path, p, mu, sd, (20.0, 30.0, 7.0, 18.0))
    rtcdf.load_model(path)
    p2, mu2, sd2, ranges = learn.load_model_file(path)
    assert np.array_equal(p2, p) and ranges == (20.0, 30.0, 7.0, 18.0)
    rtcdf.unload_model()
    raw = bytearray(open(path, "rb").read())
    raw[8] = 7                                  # unknown version
    (tmp_path / "v.bin").write_bytes(bytes(raw))
    with pytest.raises(rtcdf.RtcdfError):
        rtcdf.load_model(str(tmp_path / "v.bin"))
    (tmp_path / "short.bin").write_bytes(bytes(raw[:100]))
    with pytest.raises(rtcdf.RtcdfError):
        rtcdf.load_model(str(tmp_path / "short.bin"))


def test_dataset_targets_are_centred():
    rows = _rows(3)
    X, T, M = learn.dataset(rows)
    assert X.shape == (60, 34) and T.shape == (60, 54)
    assert np.allclose((T * M).sum(axis=1), 0.0, atol=1e-9)
    assert M.sum(axis=1).tolist() == [45.0] * 60
