"""MDSystem's thermo log: the JSON lines written during setup and run hold
exactly the rows the calls returned (NVE and NPT), steps numbered across
calls."""
import json
import os
import tempfile

import numpy as np
import pytest

from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd.system import THERMO_COLUMNS, THERMO_NPT, MDSystem

pytestmark = pytest.mark.gpu

W = I.scaled(I.LJ_4K, 6)


@pytest.mark.parametrize("ens", ["nve", "npt"])
def test_log_matches_rows(ens):
    x, v, _ = I.initial_state(W)
    kw = {"npt": (1.5, 0.5, 3, 2.0, 0.25)} if ens == "npt" else {}
    cols = THERMO_NPT if ens == "npt" else THERMO_COLUMNS
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "thermo.jsonl")
        s = MDSystem(W, x, v, "fp64", "auto", thermo_jsonl=path, **kw)
        rows = np.concatenate([s.setup(True), s.run(20, 5), s.run(10, 5)])
        with open(path) as fh:
            recs = [json.loads(line) for line in fh]
    assert len(recs) == len(rows)
    back = np.array([[r[c] for c in cols] for r in recs], dtype=np.float64)
    assert np.array_equal(back, rows)
    assert [r["step"] for r in recs] == [0, 5, 10, 15, 20, 25, 30]
