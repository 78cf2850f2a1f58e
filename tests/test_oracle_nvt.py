"""Pins of the oracle's Nose-Hoover chain NVT integrator, each against
something other than the integrator's own formulas: the conserved extended
energy (second order in dt), the decoupled limit (a huge thermostat period
gives the NVE trajectory bit for bit), time reversibility of the splitting,
and relaxation to the target temperature."""
import dataclasses

import numpy as np
import pytest

from paper_1009_4330_amd import inputs as I

W = I.LJ_4K


def run(orc, w, steps, t_target=1.5, t_damp=0.5, M=3, chain=None, x=None, v=None, every=1):
    x0, v0, box = I.initial_state(w)
    x = x0 if x is None else x
    v = v0 if v is None else v
    return orc.md_run_nvt(orc.params_for(w), x, v, box, steps, t_target, t_damp, M, chain,
                          thermo_every=every)


@pytest.mark.parametrize("M", [1, 3])
def test_nvt_conserved_energy_is_second_order(orc, M):
    """max |H' - H'_0| over a fixed time shrinks four-fold when dt halves."""
    errs = []
    for dt in (0.004, 0.002):
        w = dataclasses.replace(W, dt=dt)
        r, _ = run(orc, w, int(round(0.4 / dt)), M=M)
        h = r.thermo[:, 8]
        errs.append(np.abs(h - h[0]).max())
        # the thermostat does work: plain pe + ke is not conserved
        e = r.thermo[:, 3]
        assert np.abs(e - e[0]).max() > 20.0 * errs[-1]
    ratio = errs[0] / errs[1]
    assert 3.5 < ratio < 4.5, (errs, ratio)


def test_nvt_decoupled_limit_is_nve(orc):
    """With a thermostat period of 1e9 the chain never moves the velocities
    (the scale factor rounds to exactly 1), so the run is the NVE run."""
    w = dataclasses.replace(W, steps=60)
    x, v, box = I.initial_state(w)
    r, ch = run(orc, w, 60, t_damp=1e9)
    ref = orc.md_run(orc.params_for(w), x, v, box, 60, 1)
    assert np.array_equal(r.x, ref.x) and np.array_equal(r.v, ref.v)
    assert np.array_equal(r.thermo[:, :8], ref.thermo)


def test_nvt_time_reversible(orc):
    """N steps forward, then negate particle and chain velocities and run N
    more: the start comes back (up to rounding amplified by the dynamics)."""
    w = dataclasses.replace(W, steps=40)
    x0, v0, box = I.initial_state(w)
    # start from a thermostatted state with nonzero chain velocities
    r1, ch1 = run(orc, w, 40)
    x1, v1 = r1.x, r1.v
    r2, ch2 = run(orc, w, 40, chain=ch1, x=x1, v=v1)
    back_chain = ch2.copy()
    back_chain[3:] = -back_chain[3:]
    r3, ch3 = run(orc, w, 40, chain=back_chain, x=r2.x, v=-r2.v)
    L = np.array(box)[:, None]
    d = r3.x - x1
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-8
    assert np.abs(r3.v + v1).max() < 1e-8
    assert np.abs(ch3[3:] + ch1[3:]).max() < 1e-8


def test_nvt_relaxes_to_target_temperature(orc):
    """From T = 3 the chain brings the melt to the target; the mean over the
    second half of 1200 steps sits within 3 % of it (4000 atoms)."""
    r, _ = run(orc, W, 1200, t_target=1.2, t_damp=0.25, every=10)
    t = r.thermo[:, 4]
    mean = t[len(t) // 2:].mean()
    assert abs(mean / 1.2 - 1.0) < 0.03, mean
