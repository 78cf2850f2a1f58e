"""Pins of the oracle's isotropic NPT integrator (barostat of Martyna, Tobias
and Klein with Nose-Hoover chains on the particles and on the barostat), each
against something other than the integrator's own formulas: the conserved
extended energy (its error second order in dt), the frozen-barostat limit (a
huge barostat period gives the NVT run bit for bit), time reversibility of
the splitting, and relaxation to the target pressure and temperature from
either side."""
import dataclasses

import numpy as np
import pytest

from paper_1009_4330_amd import inputs as I

W = I.scaled(I.LJ_4K, 6, temp=1.5)      # 864 atoms, box 10.08 sigma


def run(orc, w, steps, p_target=1.0, p_damp=0.5, t_target=1.5, t_damp=0.5, M=3, chain=None,
        x=None, v=None, box=None, every=1):
    x0, v0, box0 = I.initial_state(w)
    return orc.md_run_npt(orc.params_for(w), x0 if x is None else x, v0 if v is None else v,
                          box0 if box is None else box, steps, t_target, t_damp, p_target,
                          p_damp, M, chain, thermo_every=every)


def test_npt_conserved_energy_is_second_order(orc):
    """max |H - H_0| over a fixed time shrinks four-fold each time dt halves
    (dt = 0.004, 0.002, 0.001), while the volume and pe + ke change at first
    order (the barostat does work).  A term left out of H or G_eps leaves an
    error that does not shrink with dt and breaks the ratios."""
    errs = []
    for dt in (0.004, 0.002, 0.001):
        w = dataclasses.replace(W, dt=dt)
        r, _, _ = run(orc, w, int(round(0.4 / dt)), p_target=2.0, p_damp=0.25)
        h = r.thermo[:, 8]
        errs.append(np.abs(h - h[0]).max())
        vol = r.thermo[:, 9]
        assert np.abs(vol - vol[0]).max() > 1e-3 * vol[0]
        e = r.thermo[:, 3]
        assert np.abs(e - e[0]).max() > 20.0 * errs[-1]
    for k in range(2):
        ratio = errs[k] / errs[k + 1]
        assert 3.5 < ratio < 4.5, (errs, ratio)


def test_npt_frozen_barostat_is_nvt(orc):
    """With a barostat period of 1e150 the barostat velocity rounds every
    factor it enters to exactly 1 (and the box never moves), so positions,
    velocities, thermo columns 0..7 and the particle chain equal the NVT
    run's bit for bit."""
    w = dataclasses.replace(W, steps=60)
    x, v, box = I.initial_state(w)
    r, ch, L = run(orc, w, 60, p_target=3.0, p_damp=1e150)
    ref, ch_ref = orc.md_run_nvt(orc.params_for(w), x, v, box, 60, 1.5, 0.5, 3,
                                 thermo_every=1)
    assert np.array_equal(L, np.array(box))
    assert np.array_equal(r.x, ref.x) and np.array_equal(r.v, ref.v)
    assert np.array_equal(r.thermo[:, :8], ref.thermo[:, :8])
    assert np.array_equal(ch[:6], ch_ref)


def test_npt_time_reversible(orc):
    """N steps forward, then negate the particle velocities, both chains'
    velocities and the barostat momentum and run N more: positions, box and
    velocities come back."""
    w = W
    r1, ch1, L1 = run(orc, w, 40, p_target=2.0, p_damp=0.25)
    r2, ch2, L2 = run(orc, w, 40, p_target=2.0, p_damp=0.25, chain=ch1, x=r1.x, v=r1.v, box=L1)
    back = ch2.copy()
    back[3:6] = -back[3:6]      # particle chain velocities
    back[9:12] = -back[9:12]    # barostat chain velocities
    back[12] = -back[12]        # barostat momentum
    r3, ch3, L3 = run(orc, w, 40, p_target=2.0, p_damp=0.25, chain=back, x=r2.x, v=-r2.v,
                      box=L2)
    assert np.abs(L3 / L1 - 1.0).max() < 1e-10
    Lc = L3[:, None]
    d = r3.x - r1.x * (L3 / L1)[:, None]
    d -= Lc * np.round(d / Lc)
    assert np.abs(d).max() < 1e-8
    assert np.abs(r3.v + r1.v).max() < 1e-8
    # p_eps integrates G_eps, a difference of terms of order 1e3 to 1e4 here
    assert abs(ch3[12] + ch1[12]) < 1e-6 * max(1.0, abs(ch1[12]))


def test_npt_relaxes_to_target_pressure(orc):
    """From the fcc lattice at density 0.8442 and T = 1.5, the mean pressure
    and temperature over the second half of 4000 steps sit at the targets
    (864 atoms; the pressure fluctuates by about 0.1 per sample), and the
    lower target pressure ends in the larger box."""
    edge = {}
    for p_target in (0.5, 2.0):
        r, _, L = run(orc, W, 4000, p_target=p_target, p_damp=2.5, every=10)
        th = r.thermo[len(r.thermo) // 2:]
        assert abs(th[:, 5].mean() - p_target) < 0.1, (p_target, th[:, 5].mean())
        assert abs(th[:, 4].mean() / 1.5 - 1.0) < 0.03, (p_target, th[:, 4].mean())
        assert np.allclose(th[:, 9], L.prod(), rtol=0.2)
        edge[p_target] = L[0]
    assert edge[0.5] > edge[2.0]
