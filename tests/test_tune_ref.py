"""Pins for the static-table reference (no GPU): hand-computed geometric means,
a dominating configuration, and the gain ratio."""
import math

import pytest

from oracle import tune_ref


def test_hand_example():
    # R = 128: conditions c1, c2; configs A, B, C
    # c1: A=1, B=2, C=4  -> r = 1, 2, 4
    # c2: A=8, B=2, C=2  -> r = 4, 1, 1
    # geomeans: A=2, B=sqrt(2), C=2  -> B
    rows = [(128, "c1", "A", 1), (128, "c1", "B", 2), (128, "c1", "C", 4),
            (128, "c2", "A", 8), (128, "c2", "B", 2), (128, "c2", "C", 2)]
    assert tune_ref.select_per_range(rows) == {128: "B"}


def test_dominating_config_and_ties():
    rows = []
    for c in range(5):
        for cfg, t in (("x", 3.0 + c), ("y", 1.0 + c), ("z", 2.0 + c)):
            rows.append((1024, c, cfg, t))
    assert tune_ref.select_per_range(rows) == {1024: "y"}
    rows = [(7, 0, "b", 1.0), (7, 0, "a", 1.0)]
    assert tune_ref.select_per_range(rows) == {7: "a"}


def test_gain_ratio():
    assert tune_ref.geomean_ratio([2, 8], [1, 2]) == pytest.approx(math.sqrt(8))
    assert tune_ref.geomean_ratio([1, 1], [1, 1]) == 1.0
