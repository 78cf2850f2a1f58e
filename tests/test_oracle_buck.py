"""Pins of the oracle's Buckingham + cut Coulomb forces (the potential of the
paper's silicate system, Appendix A), each against something other than the
oracle itself: lattice symmetry, independent brute-force pair sums of each
term, finite differences of the energy, and the textbook simple-cubic
lattice sum of r^-6."""
import dataclasses
import math

import numpy as np
import pytest

from paper_1009_4330_amd import inputs as I

W8 = dataclasses.replace(I.scaled(I.BUCK_141K, 8, steps=20))   # 4096 atoms, L = 35.0 A
QS = np.array([2.0, -2.0, 0.0, 0.0])


def tables(w, A=None, rho=None, C=None):
    t = lambda name: I.pair_table(w, name)
    return (t("buck_A") if A is None else A, t("buck_rho") if rho is None else rho,
            t("buck_C") if C is None else C)


def oracle_buck(orc, x, box, w, A, rho, C, q=QS, qqr2e=None):
    nl, cells = orc.build_nlist(x, box, w.rc + w.skin)
    r = orc.buck_forces(cells.x, box, nl, w.rc, w.species(), A, rho, C, q,
                        w.qqr2e if qqr2e is None else qqr2e)
    return r, cells.x


def brute(x, box, types, rc, pair):
    """Energy per atom and forces from all pairs (minimum image, r < rc):
    pair(r, ti, tj) -> (phi, -dphi/dr)."""
    n = x.shape[1]
    L = np.array(box)[:, None]
    e = np.zeros(n)
    f = np.zeros((3, n))
    for i in range(n):
        d = x[:, i:i + 1] - x
        d -= L * np.rint(d / L)
        s = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
        m = (s < rc * rc) & (np.arange(n) != i)
        r = np.sqrt(s[m])
        phi, fr = pair(r, types[i], types[m])
        e[i] = 0.5 * phi.sum()
        f[:, i] = (d[:, m] * (fr / r)).sum(axis=1)
    return e, f


@pytest.fixture(scope="module")
def jittered():
    x, _, box = I.initial_state(W8)
    return I.jitter(x, 0.08, 11), box


def test_perfect_crystal_forces_vanish(orc):
    """Every ion of a perfect rocksalt crystal sits on an inversion centre of
    the (truncated) pair sum, so its force is zero up to rounding."""
    x, _, box = I.initial_state(W8)
    r, _ = oracle_buck(orc, x, box, W8, *tables(W8))
    assert np.abs(r.f).max() < 1e-10
    assert abs(r.f.sum()) < 1e-9


@pytest.mark.parametrize("term", ["born_mayer", "dispersion", "coulomb"])
def test_each_term_against_brute_force(orc, jittered, term):
    """Each term on its own (others zeroed) against an all-pairs numpy sum
    that shares no code with the oracle's cells and lists."""
    x, box = jittered
    w = W8
    A, rho, C = tables(w)
    types = w.species()
    if term == "born_mayer":
        C = np.zeros(16)
        q = np.zeros(4)
        pair = lambda r, a, b: (A[a * 4 + b] * np.exp(-r / rho[a * 4 + b]),
                                A[a * 4 + b] / rho[a * 4 + b] * np.exp(-r / rho[a * 4 + b]))
    elif term == "dispersion":
        A = np.zeros(16)
        C = np.full(16, 1.0)
        q = np.zeros(4)
        pair = lambda r, a, b: (-1.0 / r ** 6, -6.0 / r ** 7)
    else:
        A = np.zeros(16)
        C = np.zeros(16)
        q = QS
        pair = lambda r, a, b: (w.qqr2e * q[a] * q[b] / r, w.qqr2e * q[a] * q[b] / r ** 2)
    rho_safe = np.where(rho == 0.0, 1.0, rho)
    if term == "born_mayer":
        pair = lambda r, a, b: (A[a * 4 + b] * np.exp(-r / rho_safe[a * 4 + b]),
                                A[a * 4 + b] / rho_safe[a * 4 + b]
                                * np.exp(-r / rho_safe[a * 4 + b]))
    r, xw = oracle_buck(orc, x, box, w, A, rho_safe, C, q)
    e_ref, f_ref = brute(xw, box, types, w.rc, pair)
    assert abs(r.energy - e_ref.sum()) <= 1e-11 * np.abs(e_ref).sum()
    assert np.abs(r.eatom - e_ref).max() <= 1e-11 * np.abs(e_ref).max()
    assert np.linalg.norm(r.f - f_ref) <= 1e-11 * np.linalg.norm(f_ref)
    assert abs(r.f.sum()) <= 1e-9 * np.abs(r.f).max()   # Newton's third law


def test_forces_are_minus_energy_gradient(orc, jittered):
    """Central differences of the energy for atoms none of whose pairs lies
    within 1e-3 A of the cutoff (the cut Coulomb energy jumps there).  Moving
    atom i alone changes the total energy by twice the change of its own
    share e_i, which is differenced instead of the large total."""
    x, box = jittered
    w = W8
    A, rho, C = tables(w)
    rho = np.where(rho == 0.0, 1.0, rho)
    r0, xw = oracle_buck(orc, x, box, w, A, rho, C)
    L = np.array(box)[:, None]
    rng = np.random.default_rng(5)
    h = 1e-5
    checked = 0
    for i in rng.permutation(w.natoms)[:60]:
        d = xw[:, i:i + 1] - xw
        d -= L * np.rint(d / L)
        dist = np.sqrt((d * d).sum(axis=0))
        if np.any(np.abs(dist - w.rc) < 1e-3):
            continue
        for c in range(3):
            xp = xw.copy()
            xm = xw.copy()
            xp[c, i] += h
            xm[c, i] -= h
            ep = 2.0 * oracle_buck(orc, xp, box, w, A, rho, C)[0].eatom[i]
            em = 2.0 * oracle_buck(orc, xm, box, w, A, rho, C)[0].eatom[i]
            fd = -(ep - em) / (2 * h)
            assert abs(fd - r0.f[c, i]) <= 1e-6 * max(1.0, abs(r0.f[c, i])), (i, c)
            checked += 1
        if checked >= 12:
            break
    assert checked >= 12


def test_dispersion_lattice_sum(orc):
    """All ions of rocksalt form a simple-cubic lattice of spacing a/2.  With
    only -1/r^6 between every pair, the energy per atom is -1/2 (a/2)^-6
    times the truncated lattice sum S(R), R = rc / (a/2); the full sum is
    8.40192 (simple cubic), and the part beyond R is close to 4 pi / (3 R^3)."""
    w = W8
    x, _, box = I.initial_state(w)
    r, _ = oracle_buck(orc, x, box, w, np.zeros(16), np.ones(16), np.full(16, 1.0), np.zeros(4))
    d0 = w.a / 2
    R = w.rc / d0
    s_trunc = -2.0 * r.energy / w.natoms * d0 ** 6
    assert abs(s_trunc - (8.40192 - 4.0 * math.pi / (3.0 * R ** 3))) < 3e-3
    assert s_trunc < 8.40192
