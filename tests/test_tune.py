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
        t = rng.uniform(0.5, 2.0, size=len(valid)) * (n / 1e7)
        t = [float(x) if v else -1.0 for x, v in zip(t, valid)]
        rows.append({"key": f"k{i}", "n": n, "minVal": 0, "R": R, "dist": "uniform", "sd_div": 6.0,
                     "features": list(rng.random(34)), "times_ms": t})
    return rows


def test_grid_matches_library():
    from paper_2609_00843_amd import rtcdf
    pts, valid = tune.grid()
    lp, lv = rtcdf.config_grid()
    assert pts == lp and valid == lv and sum(valid) == 53
    assert sum(valid[:tune.PLAIN_POINTS]) == 45 and all(p[:3] == (0, 0, 0) for p in pts[tune.PLAIN_POINTS:])


def test_static_selection_matches_reference():
    rows = _rows(1)
    _, valid = tune.grid()
    ref_rows = [(tune.range_class(r["R"]), r["key"], j, r["times_ms"][j])
                for r in rows for j in range(tune.PLAIN_POINTS) if valid[j]]
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
        for r in rows[:30]:
            best = min((t, j) for j, t in enumerate(r["times_ms"]) if valid[j])[1]
            got = rtcdf.pick_config(r["n"], 0, r["R"]).as_tuple()
            assert rtcdf.last_pick()[0] == best
            if best < tune.PLAIN_POINTS:
                assert got == pts[best]
            else:     # an option point: the static table's knobs with its flags
                assert got[3] == pts[best][3] and got[:3] != (0, 0, 0)
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
    learn.save_model(path, p, mu, sd, (20.0, 30.0, 7.0, 18.0), margin=0.025, zmax=5.5)
    rtcdf.load_model(path)
    p2, mu2, sd2, ranges, margin, zmax = learn.load_model_file(path)
    assert np.array_equal(p2, p) and ranges == (20.0, 30.0, 7.0, 18.0)
    assert margin == pytest.approx(0.025) and zmax == pytest.approx(5.5)
    rtcdf.unload_model()
    raw = bytearray(open(path, "rb").read())
    # version 1: no margin and zmax fields
    v1 = bytearray(raw[:44]) + raw[52:]
    v1[8] = 1
    (tmp_path / "v1.bin").write_bytes(bytes(v1))
    rtcdf.load_model(str(tmp_path / "v1.bin"))
    assert learn.load_model_file(str(tmp_path / "v1.bin"))[4:] == (0.0, 0.0)
    rtcdf.unload_model()
    neg = bytearray(raw)
    neg[44:48] = np.float32(-0.1).tobytes()      # a negative margin is refused
    (tmp_path / "neg.bin").write_bytes(bytes(neg))
    with pytest.raises(rtcdf.RtcdfError):
        rtcdf.load_model(str(tmp_path / "neg.bin"))
    raw[8] = 7                                  # unknown version
    (tmp_path / "v.bin").write_bytes(bytes(raw))
    with pytest.raises(rtcdf.RtcdfError):
        rtcdf.load_model(str(tmp_path / "v.bin"))
    (tmp_path / "short.bin").write_bytes(bytes(raw[:100]))
    with pytest.raises(rtcdf.RtcdfError):
        rtcdf.load_model(str(tmp_path / "short.bin"))


def test_decision_margin():
    """The network's choice replaces the static one only with at least the
    margin of predicted gain; the margin is chosen on measured times."""
    _, valid = tune.grid()
    ok = np.array(valid)
    y = np.zeros(learn.NOUT)
    y[5] = -0.03                                  # predicted 3% faster than everything else
    assert learn.decide(y, ok, 0, 0.02) == 5
    assert learn.decide(y, ok, 0, 0.05) == 0
    assert learn.decide(y, ok, 5, 0.0) == 5
    assert learn.decide(y, ok, 0, 0.0, trusted=False) == 0
    rows = []
    for g in (1.10, 0.90, 1.02):                # static / picked time ratio per row
        t = np.ones(learn.NOUT)
        t[5] = 1.0 / g
        t[~ok] = -1.0
        rows.append({"times_ms": t.tolist()})
    Y = np.zeros((3, learn.NOUT))
    Y[:, 5] = [-0.2, -0.01, -0.05]               # the network is confident where it is right
    mg, gain = learn.choose_margin(Y, rows, [0, 0, 0])
    # margins in (0.01, 0.05] keep rows 0 and 2 and drop row 1; the largest wins the tie
    assert mg == pytest.approx(0.05) and gain == pytest.approx((1.10 * 1.02) ** (1 / 3))


def test_dataset_targets_are_centred():
    rows = _rows(3)
    X, T, M = learn.dataset(rows)
    assert X.shape == (60, 34) and T.shape == (60, learn.NOUT) == (60, 62)
    assert np.allclose((T * M).sum(axis=1), 0.0, atol=1e-9)
    assert M.sum(axis=1).tolist() == [53.0] * 60
