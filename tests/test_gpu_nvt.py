"""md_step_nvt (Nose-Hoover chain NVT, all on the device) against the
oracle's NVT run from the same seeded state."""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_helpers import assert_fp64, rel
from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd import md
from paper_1009_4330_amd.system import MDSystem

pytestmark = pytest.mark.gpu


def min_image_diff(a, b, box):
    L = np.array(box)[:, None]
    d = a - b
    return d - L * np.round(d / L)


@pytest.mark.parametrize("kernel,M", [("tpa", 3), ("k4", 1), ("wpa", 3)])
def test_nvt_fp64_trajectory(orc, kernel, M):
    """4000-atom melt from T = 3 to a 1.5 target: same rebuild steps, thermo
    rows (including the conserved energy), final state and chain."""
    w = I.LJ_4K
    x, v, box = I.initial_state(w)
    ref, ch = orc.md_run_nvt(orc.params_for(w), x, v, box, w.steps, 1.5, 0.5, M,
                             thermo_every=5)
    sysm = MDSystem(w, x, v, "fp64", kernel, nvt=(1.5, 0.5, M))
    rows = np.concatenate([sysm.setup(True), sysm.run(w.steps, 5)])
    assert rows.shape == ref.thermo.shape
    assert np.array_equal(rows[:, 0], ref.thermo[:, 0])
    assert np.array_equal(rows[:, 6].astype(int), ref.thermo[:, 6].astype(int))
    assert np.array_equal(rows[:, 7].astype(int), ref.thermo[:, 7].astype(int))
    for c in (1, 2, 3, 4, 5, 8):
        assert rel(rows[:, c], ref.thermo[:, c]) < 1e-10, c
    gx, gv, gf = sysm.host_state()
    assert np.abs(min_image_diff(gx, ref.x, box)).max() < 1e-9
    assert np.abs(gv - ref.v).max() < 1e-9
    st = sysm.nhc.state.cpu().numpy()
    got_chain = np.concatenate([st[:M], st[md.MD_NHC_MAX:md.MD_NHC_MAX + M]])
    assert rel(got_chain, ch) < 1e-10
    # the thermostat took the melt from T = 3 toward the target
    assert rows[-1, 4] < 2.0


def test_nvt_decoupled_is_nve_bit_for_bit():
    """A thermostat period of 1e9 leaves every scale factor at exactly 1, so
    md_step_nvt reproduces md_step's trajectory bit for bit."""
    w = dataclasses.replace(I.LJ_4K, steps=60)
    x, v, box = I.initial_state(w)
    a = MDSystem(w, x, v, "fp64", "k4")
    ra = np.concatenate([a.setup(True), a.run(60, 10)])
    b = MDSystem(w, x, v, "fp64", "k4", nvt=(1.5, 1e9, 3))
    rb = np.concatenate([b.setup(True), b.run(60, 10)])
    assert np.array_equal(ra, rb[:, :8])
    for ta, tb in zip(a.host_state(), b.host_state()):
        assert np.array_equal(ta, tb)


def test_nvt_chunked_run_matches_single_call():
    """Two calls of 50 steps continue the chain state of one call of 100."""
    w = I.LJ_4K
    x, v, box = I.initial_state(w)
    a = MDSystem(w, x, v, "fp64", "tpa", nvt=(1.5, 0.5, 3))
    a.setup(False)
    ra = a.run(100, 10)
    b = MDSystem(w, x, v, "fp64", "tpa", nvt=(1.5, 0.5, 3))
    b.setup(False)
    rb = b.run(100, 10, chunk=50)
    for c in (1, 2, 3, 4, 5, 8):
        assert rel(rb[:, c], ra[:, c]) < 1e-12, c
    assert rel(b.nhc.state.cpu().numpy(), a.nhc.state.cpu().numpy()) < 1e-12


def test_nvt_mixed_conserved_energy():
    """MIXED: the conserved energy drifts no more than a few times the FP64 run's."""
    w = dataclasses.replace(I.LJ_4K, steps=200)
    x, v, box = I.initial_state(w)
    drift = {}
    for prec in ("fp64", "mixed"):
        s = MDSystem(w, x, v, prec, "tpa", nvt=(1.5, 0.5, 3))
        rows = np.concatenate([s.setup(True), s.run(200, 1)])
        h = rows[:, 8]
        drift[prec] = np.abs(h - h[0]).max() / abs(h[0])
    print(f"NVT conserved-energy drift over 200 steps: fp64 {drift['fp64']:.3e} "
          f"mixed {drift['mixed']:.3e}")
    assert drift["mixed"] < 2.0 * drift["fp64"] + 1e-6


def test_nvt_rejects_bad_thermostat():
    w = I.LJ_4K
    x, v, box = I.initial_state(w)
    for bad in ((1.5, 0.5, 0), (1.5, 0.5, 9), (-1.0, 0.5, 3), (1.5, 0.0, 3)):
        s = MDSystem(w, x, v, "fp64", "tpa", nvt=bad)
        with pytest.raises(md.MDError):
            s.setup(False)


@pytest.mark.parametrize("which", ["sc", "buck"])
def test_nvt_other_potentials_fp64(orc, which):
    """The thermostat is independent of the potential: Sutton-Chen (metal
    units) and Buckingham + Coulomb (two species permuted by the sorts) NVT
    runs against the oracle's."""
    if which == "sc":
        w = I.scaled(I.SC_500K, 6, steps=40)
        t_target, cap = 300.0, None
    else:
        w = dataclasses.replace(I.scaled(I.BUCK_141K, 8, steps=40), skin=0.3)
        t_target, cap = 300.0, 2300
    x, v, box = I.initial_state(w)
    ref, ch = orc.md_run_nvt(orc.params_for(w), x, v, box, w.steps, t_target, 0.1, 3,
                             thermo_every=5)
    sysm = MDSystem(w, x, v, "fp64", "k4", capacity=cap, nvt=(t_target, 0.1, 3))
    rows = np.concatenate([sysm.setup(True), sysm.run(w.steps, 5)])
    assert np.array_equal(rows[:, 6].astype(int), ref.thermo[:, 6].astype(int))
    for c in (1, 2, 3, 4, 5, 8):
        assert rel(rows[:, c], ref.thermo[:, c]) < 1e-10, c
    gx, gv, gf = sysm.host_state()
    assert np.abs(min_image_diff(gx, ref.x, box)).max() < 1e-9
    assert_fp64(gf, ref.f, 1e-9)
