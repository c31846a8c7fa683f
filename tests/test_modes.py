"""Observing-mode presets against the instrument's mode table (the paper's
Table 1, stored as printed in tests/golden/table1_modes.txt): every preset
lies inside its row, its spectral resolution is bandwidth / channels within
the table's printed rounding, its dump interval covers the minimum
integration time, and its real-time requirement counts both polarisations of
every sub-band."""
import os

import pytest

from paper_1411_0436_amd.modes import MODES, real_time_factor

HERE = os.path.dirname(os.path.abspath(__file__))


def _rows():
    rows = []
    with open(os.path.join(HERE, "golden", "table1_modes.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = line.split()
                rows.append(dict(sub=int(v[0]), bw=(float(v[1]), float(v[2])), ch=(int(v[3]), int(v[4])),
                                 res=(float(v[5]), float(v[6])), tint=(float(v[7]), float(v[8]))))
    return rows


def _row_of(m):
    for r in _rows():
        if (r["sub"] == m.subbands and r["bw"][0] - 0.01 <= m.bw_hz / 1e6 <= r["bw"][1] + 0.01
                and r["ch"][0] <= m.N <= r["ch"][1]):
            return r
    return None


def test_table_has_three_rows():
    assert [r["sub"] for r in _rows()] == [1, 1, 8]


@pytest.mark.parametrize("name", sorted(MODES))
def test_preset_inside_its_table_row(name):
    m = MODES[name]
    r = _row_of(m)
    assert r is not None, name
    # resolution: the table prints one or two significant digits
    res_khz = m.resolution_hz / 1e3
    lo, hi = r["res"]
    assert lo * 0.85 <= res_khz <= hi * 1.05, (name, res_khz, r["res"])
    assert r["tint"][0] <= m.min_int_s * 1e3 <= r["tint"][1]
    assert m.N & (m.N - 1) == 0


@pytest.mark.parametrize("name", sorted(MODES))
def test_dump_interval_covers_minimum_integration(name):
    m = MODES[name]
    assert m.dump_interval_s >= m.min_int_s - 1e-12
    assert (m.n_int - 1) * m.N / m.bw_hz < m.min_int_s  # the smallest such n_int


def test_each_table_row_has_both_ends():
    rows = _rows()
    for r in rows:
        ms = [m for m in MODES.values() if _row_of(m) == r]
        assert {m.N for m in ms} == set(r["ch"]), r


def test_real_time_requirement():
    m = MODES["wide-32k"]
    assert m.required_samples_per_s == 2 * 187.5e6
    assert MODES["eight-4k"].required_samples_per_s == 2 * 8 * 23.4375e6
    assert real_time_factor(m, 3.75e8) == 1.0
