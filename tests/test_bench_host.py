"""Host-side pieces of bench.py: the drift summary for any number of thermo
rows (a short timed run yields one row or none) and the byte model."""
import importlib.util
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def rows_of(steps, energies):
    r = np.zeros((len(steps), 8))
    r[:, 0] = steps
    r[:, 3] = energies
    return r


def test_drift_needs_two_rows(bench):
    assert bench.nve_drift(np.zeros((0, 8)), 100, 0.005) is None
    assert bench.nve_drift(rows_of([20], [-5.0]), 100, 0.005) is None


def test_drift_values(bench):
    d = bench.nve_drift(rows_of([100, 200, 300], [-10.0, -10.1, -10.2]), 10, 0.005)
    assert d["rows"] == 3
    assert d["max_rel"] == pytest.approx(0.02)
    # E/N falls by 0.01 per 100 steps = 0.5 time units
    assert d["slope_per_tau"] == pytest.approx(-0.02)


def test_headline_never_shorter_than_the_workload(bench):
    assert bench.HEADLINE_STEPS == 1000
    assert max(20, bench.HEADLINE_STEPS) == 1000


def test_step_bytes(bench):
    nn = 75.7
    f = bench.force_bytes_per_atom(nn)
    assert f == pytest.approx(196 + 4 * nn)
    assert bench.step_bytes_per_atom(nn, 0, 1000) == pytest.approx(f)
    b = bench.step_bytes_per_atom(nn, 200, 1000)
    assert b == pytest.approx(f + 0.2 * bench.rebuild_bytes_per_atom(nn))


def test_guarded_reports_errors(bench):
    def boom():
        raise IndexError("no rows")
    r = bench.guarded("x", boom)
    assert r == {"error": "IndexError: no rows"}
    assert bench.guarded("y", lambda: 3.0) == 3.0
