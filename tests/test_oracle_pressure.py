"""Pins of the oracle's thermo pressure column, P = (2 KE + tr W) / (3 V),
each by a route other than that formula:

* configurational part: at zero velocity the pressure is minus the derivative
  of the potential energy with respect to volume under a uniform scaling of
  box and positions (thermodynamic route), here by central differences of the
  oracle's own energies, for LJ, Sutton-Chen (many-body virial) and
  Buckingham + Coulomb;
* kinetic part: with the interactions switched off the oracle's columns must
  obey the ideal-gas law P V = (N - 1) k_B T (N - 1 because the temperature
  counts 3N - 3 degrees of freedom after the net momentum is removed), in LJ
  and in metal units;
* the two parts add on a lattice that carries thermal velocities."""
import dataclasses

import numpy as np
import pytest

from paper_1009_4330_amd import inputs as I

LJ = I.scaled(I.LJ_4K, 5)
SC = dataclasses.replace(I.scaled(I.SC_500K, 5), a=3.55)   # shells clear of rc = 7.22 A
BUCK = I.scaled(I.BUCK_141K, 8)


def row0(orc, w, x, v, box, **over):
    """The oracle's thermo row at step 0 (setup only)."""
    return orc.md_run(orc.params_for(w, **over), x, v, box, 0, 1).thermo[0]


def minus_dE_dV(orc, w, x, box, h=1e-6):
    """-dE/dV by central differences of the potential energy under a uniform
    scaling of positions and box by (1 +- h)."""
    zero = np.zeros_like(x)
    e, vol = [], []
    for s in (1.0 + h, 1.0 - h):
        bs = tuple(s * L for L in box)
        e.append(row0(orc, w, s * x, zero, bs)[1])
        vol.append(bs[0] * bs[1] * bs[2])
    return -(e[0] - e[1]) / (vol[0] - vol[1])


def min_pair_gap_to_rc(orc, x, box, rc):
    """Smallest |r - rc| over the listed pairs (the FD must not move a pair
    across the cutoff, where the unshifted energies jump)."""
    nl, c = orc.build_nlist(x, box, rc + 0.5)
    L = np.array(box)[:, None]
    p = nl.pairs()
    d = c.x[:, p[:, 0]] - c.x[:, p[:, 1]]
    d -= L * np.rint(d / L)
    return float(np.abs(np.sqrt((d * d).sum(0)) - rc).min())


CASES = {
    "lj_lattice": (LJ, lambda w: I.fcc_positions(w.ncell, w.a)),
    "lj_jittered": (LJ, lambda w: I.jitter(I.fcc_positions(w.ncell, w.a), 0.2, 3)),
    "sc_lattice": (SC, lambda w: I.fcc_positions(w.ncell, w.a)),
    "sc_jittered": (SC, lambda w: I.jitter(I.fcc_positions(w.ncell, w.a), 0.1, 4)),
    "buck_lattice": (BUCK, lambda w: I.rocksalt_positions(w.ncell, w.a)),
    "buck_jittered": (BUCK, lambda w: I.jitter(I.rocksalt_positions(w.ncell, w.a), 0.05, 5)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_pressure_is_minus_energy_volume_derivative(orc, case):
    w, make = CASES[case]
    x = make(w)
    box = w.box
    h = 1e-6
    assert min_pair_gap_to_rc(orc, x, box, w.rc) > 4 * h * w.rc, "a pair sits at the cutoff"
    p = row0(orc, w, x, np.zeros_like(x), box)[5]
    ref = minus_dE_dV(orc, w, x, box, h)
    # FD error: h^2 curvature plus rounding of E (|E| eps / (h dV/dh))
    assert abs(p - ref) <= 1e-6 * abs(ref) + 1e-9, (p, ref)


@pytest.mark.parametrize("w,off", [(LJ, dict(lj_eps=0.0)), (SC, dict(sc_eps=0.0))])
def test_ideal_gas_law(orc, w, off):
    x, v, box = I.initial_state(w)
    x = I.jitter(x, 0.3, 9)
    r = row0(orc, w, x, v, box, **off)
    n = x.shape[1]
    vol = box[0] * box[1] * box[2]
    assert r[1] == 0.0
    assert r[5] * vol == pytest.approx((n - 1) * w.units.boltz * r[4], rel=1e-13)
    # and T is the workload's target (scaled by the input generator)
    assert r[4] == pytest.approx(w.temp, rel=1e-13)


def test_kinetic_and_configurational_parts_add(orc):
    w = LJ
    x, v, box = I.initial_state(w)
    n = x.shape[1]
    vol = box[0] * box[1] * box[2]
    r = row0(orc, w, x, v, box)
    expect = (n - 1) * w.units.boltz * w.temp / vol + minus_dE_dV(orc, w, x, box)
    assert r[5] == pytest.approx(expect, rel=1e-6)
