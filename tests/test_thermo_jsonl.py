"""Thermo rows written as JSON lines (host logic, no GPU): column names per
ensemble, integers where the row holds counts, floats that read back equal
to the row bit for bit, and a row of the wrong width refused."""
import io
import json

import numpy as np
import pytest

from paper_1009_4330_amd.system import (THERMO_COLUMNS, THERMO_NPT, THERMO_NVT, thermo_records,
                                        write_thermo_jsonl)


def rows_of(width, n=5, seed=3):
    rng = np.random.default_rng(seed)
    r = rng.standard_normal((n, width)) * 10.0 ** rng.integers(-12, 12, (n, width))
    r[:, 0] = np.arange(n) * 10          # step
    r[:, 6] = np.arange(n) // 2          # builds so far
    r[:, 7] = 70 + np.arange(n)          # largest neighbour count
    return r


@pytest.mark.parametrize("columns", [THERMO_COLUMNS, THERMO_NVT, THERMO_NPT])
def test_round_trip(columns):
    rows = rows_of(len(columns))
    fh = io.StringIO()
    write_thermo_jsonl(fh, rows, columns)
    lines = fh.getvalue().splitlines()
    assert len(lines) == len(rows)
    for line, row in zip(lines, rows):
        rec = json.loads(line)
        assert list(rec) == list(columns)
        for c in ("step", "builds", "maxneigh"):
            assert isinstance(rec[c], int)
        back = np.array([rec[c] for c in columns], dtype=np.float64)
        assert np.array_equal(back, row)


def test_columns():
    assert THERMO_COLUMNS == ("step", "pe", "ke", "etotal", "temp", "press", "builds", "maxneigh")
    assert THERMO_NVT[-1] == "conserved" and len(THERMO_NVT) == 9
    assert THERMO_NPT[-2:] == ("conserved", "volume") and len(THERMO_NPT) == 10


def test_wrong_width_refused():
    with pytest.raises(ValueError):
        thermo_records(rows_of(8), THERMO_NVT)
    with pytest.raises(ValueError):
        thermo_records(np.zeros(8), THERMO_COLUMNS)
