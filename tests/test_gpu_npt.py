"""md_step_npt against the oracle's NPT run (isotropic barostat of Martyna,
Tobias and Klein with Nose-Hoover chains on the particles and the barostat):
thermo rows (energies, temperature, pressure, the conserved extended energy,
the volume), rebuild steps, final positions, velocities and box; the
frozen-barostat limit against the library's own NVT run bit for bit; the
trajectory independent of the thermo interval; a run split over two calls;
FP32-mixed against the FP64 oracle."""
import numpy as np
import pytest

from gpu_helpers import assert_fp64, rel
from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd.system import MDSystem

pytestmark = pytest.mark.gpu

W = I.scaled(I.LJ_4K, 10, temp=1.5)     # 4000 atoms
NPT = (1.5, 0.5, 3, 2.0, 0.25)          # t_target, t_damp, chain, p_target, p_damp


def oracle_npt(orc, w, steps, every, npt=NPT):
    x, v, box = I.initial_state(w)
    t, td, M, p, pd = npt
    return orc.md_run_npt(orc.params_for(w), x, v, box, steps, t, td, p, pd, M,
                          thermo_every=every)


def box_diff(a, b, L):
    L = np.asarray(L)[:, None]
    d = a - b
    return d - L * np.round(d / L)


@pytest.mark.parametrize("kernel", ["k4", "tpa"])
def test_npt_fp64_against_oracle(orc, kernel):
    w = W
    x, v, box = I.initial_state(w)
    s = MDSystem(w, x, v, "fp64", kernel, npt=NPT)
    rows = np.concatenate([s.setup(True), s.run(100, 10)])
    ref, ch, L = oracle_npt(orc, w, 100, 10)
    assert np.array_equal(rows[:, 6].astype(int), ref.thermo[:, 6].astype(int))
    assert rows[-1, 6] > 3                               # the box moved and lists were rebuilt
    for c in (1, 2, 3, 4, 5, 8, 9):
        assert rel(rows[:, c], ref.thermo[:, c]) < 1e-10, c
    assert abs(ref.thermo[-1, 9] / ref.thermo[0, 9] - 1.0) > 1e-3   # the volume did change
    assert np.abs(np.array(s.box.L) / L - 1.0).max() < 1e-12
    gx, gv, gf = s.host_state()
    assert np.abs(box_diff(gx, ref.x, L)).max() < 1e-9
    assert np.abs(gv - ref.v).max() < 1e-9
    assert_fp64(gf, ref.f, 1e-9)


def test_npt_frozen_barostat_equals_nvt(orc):
    """A barostat period of 1e150 leaves every barostat factor exactly 1: the
    NPT run is the library's NVT run bit for bit (positions, velocities,
    forces, the first eight thermo columns) and the box never moves."""
    w = W
    x, v, box = I.initial_state(w)
    a = MDSystem(w, x, v, "fp64", "k4", npt=(1.5, 0.5, 3, 3.0, 1e150))
    ra = np.concatenate([a.setup(True), a.run(60, 10)])
    b = MDSystem(w, x, v, "fp64", "k4", nvt=(1.5, 0.5, 3))
    rb = np.concatenate([b.setup(True), b.run(60, 10)])
    assert tuple(a.box.L) == tuple(box)
    assert np.array_equal(ra[:, :8], rb[:, :8])
    for ta, tb in zip(a.host_state(), b.host_state()):
        assert np.array_equal(ta, tb)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_npt_thermo_interval_leaves_trajectory(orc, prec):
    """Steps with a thermo row evaluate energy and virial, the others the
    virial's trace alone; the barostat sums the same per-atom trace column
    either way, so thermo rows every 7 steps or only at the end leave the
    trajectory and the box the same bit for bit."""
    w = W
    x, v, box = I.initial_state(w)
    a = MDSystem(w, x, v, prec, "k4", npt=NPT)
    a.setup(False)
    ra = a.run(60, 7)
    b = MDSystem(w, x, v, prec, "k4", npt=NPT)
    b.setup(False)
    b.run(60, 60)
    assert len(ra) == 8 and tuple(a.box.L) == tuple(b.box.L)
    assert tuple(a.box.L) != tuple(box)
    for ta, tb in zip(a.host_state(), b.host_state()):
        assert np.array_equal(ta, tb)


def test_npt_run_split_over_calls(orc):
    """Two calls of 50 steps continue the barostat and thermostat state (the
    second call re-sums the kinetic energy from v, a rounding-level change)."""
    w = W
    x, v, box = I.initial_state(w)
    a = MDSystem(w, x, v, "fp64", "k4", npt=NPT)
    a.setup(False)
    a.run(100, 100)
    b = MDSystem(w, x, v, "fp64", "k4", npt=NPT)
    b.setup(False)
    b.run(50, 50)
    b.run(50, 50)
    assert np.abs(np.array(a.box.L) / np.array(b.box.L) - 1.0).max() < 1e-12
    xa, va, _ = a.host_state()
    xb, vb, _ = b.host_state()
    assert np.abs(box_diff(xa, xb, a.box.L)).max() < 1e-9
    assert np.abs(va - vb).max() < 1e-9


def test_npt_mixed_against_oracle(orc):
    """FP32-mixed pair forces under the barostat: after 100 steps the volume,
    temperature, pressure and conserved energy stay within the divergence
    that 1e-7-level force differences allow of the FP64 oracle's run."""
    w = W
    x, v, box = I.initial_state(w)
    s = MDSystem(w, x, v, "mixed", "auto", npt=NPT)
    rows = np.concatenate([s.setup(True), s.run(100, 10)])
    ref, _, L = oracle_npt(orc, w, 100, 10)
    # measured 3.4e-9, 1.4e-8, 4.4e-8 and 9.0e-8
    for c, tol in ((9, 5e-8), (4, 2e-7), (5, 5e-7), (8, 1e-6)):
        err = np.abs(rows[:, c] - ref.thermo[:, c]).max() / np.abs(ref.thermo[:, c]).max()
        print(f"[npt mixed] column {c}: {err:.3e}")
        assert err < tol, c
