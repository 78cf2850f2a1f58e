"""Pins of the CPU oracle against what the mathematics fixes.

Each test checks the oracle against something other than itself: explicit
all-image brute force (tests/brute.py), closed-form lattice sums from an
enumeration of fcc lattice vectors, textbook two-atom values (tests/golden),
invariants (Newton's third law, momentum, translation invariance, Hessian
symmetry), finite differences, and the convergence order and time
reversibility of velocity Verlet.
"""
import math
import os

import numpy as np
import pytest

import brute
from paper_1009_4330_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SC = dict(eps=1.2382e-2, a=3.61, c=39.432, nexp=9, mexp=6)


def _load(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append([float(t) for t in line.split()])
    return np.array(rows)


def lj_system(ncell, amp, seed, outside=0.0):
    """Jittered fcc LJ liquid-like configuration; optionally pushes a few atoms
    up to `outside` beyond the box faces (as between rebuilds)."""
    x = I.jitter(I.fcc_positions(ncell, I.A_LJ), amp, seed)
    box = (ncell * I.A_LJ,) * 3
    if outside:
        rng = np.random.default_rng(seed + 1)
        for d in range(3):
            k = rng.choice(x.shape[1], 8, replace=False)
            x[d, k[:4]] = -rng.uniform(0, outside, 4)
            x[d, k[4:]] = box[d] + rng.uniform(0, outside, 4)
    return x, box


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


# ------------------------------------------------------------ binning --


def test_cell_dims_and_box_guard(orc):
    assert list(orc.cell_dims((16.795961913825073,) * 3, 2.8)) == [5, 5, 5]
    assert list(orc.cell_dims((67.18384765530029,) * 3, 2.8)) == [23, 23, 23]
    with pytest.raises(orc.OracleError):
        orc.cell_dims((5.6, 10.0, 10.0), 2.8)


@pytest.mark.parametrize("ncell,seed", [(4, 1), (6, 2)])
def test_bin_is_stable_counting_sort(orc, ncell, seed):
    x, box = lj_system(ncell, 0.4, seed, outside=0.15)
    c = orc.bin_cells(x, box, 2.8)
    n = x.shape[1]
    L = np.array(box)
    assert np.all(c.x >= 0) and np.all(c.x < L[:, None])
    # wrapped positions are congruent to the inputs modulo L
    k = (x - c.x) / L[:, None]
    assert np.allclose(k, np.round(k), atol=1e-12)
    assert sorted(c.perm.tolist()) == list(range(n))
    cells_in_order = c.atom_cell[c.perm]
    assert np.all(np.diff(cells_in_order) >= 0)
    same = np.diff(cells_in_order) == 0
    assert np.all(np.diff(c.perm)[same] > 0), "not stable inside a cell"
    ncell_tot = int(np.prod(c.nc))
    assert np.array_equal(np.diff(c.cell_start), np.bincount(c.atom_cell, minlength=ncell_tot))
    # each atom lies inside (or within rounding of) the cell it was put in
    edge = L / c.nc
    cx = np.stack([c.atom_cell % c.nc[0], (c.atom_cell // c.nc[0]) % c.nc[1],
                   c.atom_cell // (c.nc[0] * c.nc[1])])
    lo = cx * edge[:, None] - 1e-9
    hi = (cx + 1) * edge[:, None] + 1e-9
    assert np.all((c.x >= lo) & (c.x <= hi))


# ----------------------------------------------------- neighbour list --


@pytest.mark.parametrize("ncell,amp,seed,outside", [(4, 0.3, 11, 0.0), (5, 0.5, 12, 0.15),
                                                     (6, 0.25, 13, 0.15)])
def test_nlist_equals_all_image_brute_force(orc, ncell, amp, seed, outside):
    x, box = lj_system(ncell, amp, seed, outside)
    nl, cells = orc.build_nlist(x, box, 2.8)
    want = brute.pairs_within(x, box, 2.8)
    got = nl.pairs()
    assert got.shape == want.shape
    assert np.array_equal(got, want)
    # a full list: (i, j) listed iff (j, i) listed
    flip = got[:, ::-1]
    flip = flip[np.lexsort((flip[:, 1], flip[:, 0]))]
    assert np.array_equal(flip, got)


def test_nlist_atoms_on_cell_faces(orc):
    """Atoms placed exactly on cell boundaries and on the box faces."""
    L = 4 * I.A_LJ
    nc = int(L // 2.8)
    edge = L / nc
    rng = np.random.default_rng(5)
    x = rng.uniform(0, L, (3, 200))
    x[0, :40] = edge * rng.integers(0, nc, 40)
    x[1, 40:80] = edge * rng.integers(0, nc + 1, 40)
    x[2, 80:90] = L
    x[2, 90:100] = 0.0
    nl, _ = orc.build_nlist(x, (L,) * 3, 2.8)
    assert np.array_equal(nl.pairs(), brute.pairs_within(x, (L,) * 3, 2.8))


def test_nlist_overflow_reports_true_count(orc):
    x, box = lj_system(4, 0.3, 3)
    with pytest.raises(orc.OracleError) as ei:
        orc.build_nlist(x, box, 2.8, cap=10)
    assert ei.value.code == 3
    full, _ = orc.build_nlist(x, box, 2.8)
    assert ei.value.max_count == full.max_count > 10


# ------------------------------------------------------- Lennard-Jones --


def test_lj_two_atom_golden(orc):
    """Two atoms along a body diagonal, in a box large enough that only the
    pair itself interacts."""
    for r, phi, fr in _load("lj_pair.txt"):
        L = 20.0
        u = np.array([1.0, 2.0, 2.0]) / 3.0
        x = np.array([[5.0, 5.0 + r * u[0]], [5.0, 5.0 + r * u[1]], [5.0, 5.0 + r * u[2]]])
        rc = 2.5 + 1e-9 if r >= 2.5 else 2.5
        nl, cells = orc.build_nlist(x, (L,) * 3, 3.0)
        res = orc.lj_forces(cells.x, (L,) * 3, nl, rc)
        assert res.energy == pytest.approx(phi, abs=1e-13)
        # force on atom 1 points along +u when repulsive (F_r > 0)
        assert np.allclose(res.f[:, 1], fr * u, atol=1e-12)
        assert np.allclose(res.f[:, 0], -fr * u, atol=1e-12)
        w = res.virial
        assert w[0] + w[1] + w[2] == pytest.approx(r * fr, abs=1e-12)


@pytest.mark.parametrize("rc", [2.5, 5.0])
def test_lj_perfect_lattice_closed_form(orc, rc):
    """E/N = 1/2 sum_shells m phi(r), tr W / N = 1/2 sum_shells m r F_r(r)."""
    ncell = 6 if rc < 3 else 8
    x = I.fcc_positions(ncell, I.A_LJ)
    box = (ncell * I.A_LJ,) * 3
    r, m, _ = brute.fcc_shells(rc, I.A_LJ)
    phi = 4.0 * (r ** -12 - r ** -6)
    fr = 24.0 * (2.0 * r ** -13 - r ** -7)
    e_n = 0.5 * np.sum(m * phi)
    w_n = 0.5 * np.sum(m * r * fr)
    nl, cells = orc.build_nlist(x, box, rc + 0.3)
    res = orc.lj_forces(cells.x, box, nl, rc)
    n = x.shape[1]
    assert res.energy / n == pytest.approx(e_n, rel=1e-13)
    assert res.virial[:3].sum() / n == pytest.approx(w_n, rel=1e-13)
    assert np.max(np.abs(res.f)) < 1e-11
    # shifted energy: subtract phi(rc) once per unordered interacting pair
    sh = orc.lj_forces(cells.x, box, nl, rc, shift=1)
    phic = 4.0 * (rc ** -12 - rc ** -6)
    assert sh.energy / n == pytest.approx(e_n - 0.5 * np.sum(m) * phic, rel=1e-13)


def test_fcc_shell_multiplicities_golden():
    g = _load("fcc_shells.txt")
    r, m, v = brute.fcc_shells(2.01, 1.0)
    assert np.allclose(v / 4.0, g[:, 0])
    assert np.array_equal(m, g[:, 1].astype(int))


@pytest.mark.parametrize("ncell,amp,seed", [(4, 0.3, 21), (5, 0.6, 22)])
def test_lj_equals_all_image_brute_force(orc, ncell, amp, seed):
    x, box = lj_system(ncell, amp, seed, outside=0.1)
    nl, cells = orc.build_nlist(x, box, 2.8)
    res = orc.lj_forces(x, box, nl, 2.5, eps=1.3, sigma=0.95)
    f, e, w = brute.lj(x, box, 2.5, eps=1.3, sigma=0.95)
    assert rel(res.f, f) < 1e-12
    assert res.energy == pytest.approx(e, rel=1e-12)
    assert np.allclose(res.virial, w, rtol=1e-12, atol=1e-12 * np.abs(w).max())
    # Newton's third law: pair forces cancel
    assert np.abs(res.f.sum(axis=1)).max() < 1e-12 * np.sqrt(x.shape[1]) * np.abs(f).max()
    assert res.eatom.sum() == pytest.approx(res.energy, rel=1e-14)


def _frozen_ok(x, box, atom, rc, tol):
    """True when no pair of `atom` lies within tol of the cutoff."""
    L = np.array(box)
    d = x[:, atom:atom + 1] - x
    d -= L[:, None] * np.round(d / L[:, None])
    r = np.sqrt((d * d).sum(axis=0))
    r[atom] = 1e9
    return np.min(np.abs(r - rc)) > tol


def test_lj_forces_are_minus_energy_gradient(orc):
    x, box = lj_system(4, 0.35, 31)
    nl, cells = orc.build_nlist(x, box, 2.8)
    h = 1e-5
    base = orc.lj_forces(x, box, nl, 2.5)
    checked = 0
    for atom in range(0, x.shape[1], 17):
        if not _frozen_ok(x, box, atom, 2.5, 1e-3):
            continue
        for d in range(3):
            xp = x.copy(); xp[d, atom] += h
            xm = x.copy(); xm[d, atom] -= h
            ep = orc.lj_forces(xp, box, nl, 2.5).energy
            em = orc.lj_forces(xm, box, nl, 2.5).energy
            fd = -(ep - em) / (2 * h)
            assert fd == pytest.approx(base.f[d, atom], rel=1e-6, abs=1e-7)
            checked += 1
    assert checked >= 30


# --------------------------------------------------------- Sutton-Chen --


def sc_system(ncell, amp, seed):
    x = I.jitter(I.fcc_positions(ncell, 3.61), amp, seed)
    return x, (ncell * 3.61,) * 3


def test_sc_perfect_lattice_closed_form(orc):
    """rho = sum_shells m (a/r)^m, E/N = eps (1/2 sum m (a/r)^n - c sqrt(rho))
    with a cutoff strictly between shells (7.0 A: shells 1..7, since the
    8th shell sits at 2a = 7.22 A) and strictly beyond the 8th shell."""
    x = I.fcc_positions(5, 3.61)
    box = (5 * 3.61,) * 3
    n = x.shape[1]
    for rc in (7.0, 7.3):
        r, m, _ = brute.fcc_shells(rc, 3.61)
        rho = np.sum(m * (3.61 / r) ** 6)
        e_n = SC["eps"] * (0.5 * np.sum(m * (3.61 / r) ** 9) - SC["c"] * np.sqrt(rho))
        nl, cells = orc.build_nlist(x, box, rc + 1.0)
        res = orc.sc_forces(cells.x, box, nl, rc, **SC)
        assert np.allclose(res.rho, rho, rtol=1e-13)
        assert res.energy / n == pytest.approx(e_n, rel=1e-13)
        assert np.max(np.abs(res.f)) < 1e-11


def test_sc_lattice_tie_at_cutoff_is_rounding_decided(orc):
    """At rc = 7.22 = 2a the 8th shell is exactly at the cutoff; each atom's
    density is one of the two shell sums, depending on FP64 rounding of the
    separations.  Both sums bracket every per-atom density."""
    x = I.fcc_positions(5, 3.61)
    box = (5 * 3.61,) * 3
    lo_r, lo_m, _ = brute.fcc_shells(7.0, 3.61)
    rho_lo = np.sum(lo_m * (3.61 / lo_r) ** 6)
    rho_hi = rho_lo + 6 * (0.5) ** 6
    nl, cells = orc.build_nlist(x, box, 8.22)
    res = orc.sc_forces(cells.x, box, nl, 7.22, **SC)
    assert np.all(res.rho >= rho_lo * (1 - 1e-13))
    assert np.all(res.rho <= rho_hi * (1 + 1e-13))


def test_sc_equals_all_image_brute_force(orc):
    x, box = sc_system(5, 0.2, 41)
    nl, cells = orc.build_nlist(x, box, 8.22)
    res = orc.sc_forces(x, box, nl, 7.22, **SC)
    f, e, rho = brute.sutton_chen(x, box, 7.22, **SC)
    assert np.allclose(res.rho, rho, rtol=1e-12)
    assert res.energy == pytest.approx(e, rel=1e-12)
    assert rel(res.f, f) < 1e-11
    assert np.abs(res.f.sum(axis=1)).max() < 1e-10


def test_sc_forces_are_minus_energy_gradient(orc):
    x, box = sc_system(5, 0.2, 42)
    nl, _ = orc.build_nlist(x, box, 8.22)
    base = orc.sc_forces(x, box, nl, 7.22, **SC)
    h = 1e-5
    checked = 0
    for atom in range(0, x.shape[1], 37):
        if not _frozen_ok(x, box, atom, 7.22, 1e-3):
            continue
        for d in range(3):
            xp = x.copy(); xp[d, atom] += h
            xm = x.copy(); xm[d, atom] -= h
            fd = -(orc.sc_forces(xp, box, nl, 7.22, **SC).energy
                   - orc.sc_forces(xm, box, nl, 7.22, **SC).energy) / (2 * h)
            assert fd == pytest.approx(base.f[d, atom], rel=1e-6, abs=1e-9)
            checked += 1
    assert checked >= 20


# --------------------------------------------------- velocity Verlet --


def small_lj_run(orc, ncell=5, temp=1.5, dt=0.005, steps=40, seed=7, skin=0.3, every=1):
    w = I.scaled(I.LJ_4K, ncell, temp=temp, dt=dt, steps=steps, skin=skin)
    x, v, box = I.initial_state(w, seed)
    x = I.jitter(x, 0.05, seed)
    return orc.md_run(orc.params_for(w), x, v, box, steps, every), x, v, box, w


def test_initial_temperature_and_momentum(orc):
    res, x, v, box, w = small_lj_run(orc, steps=0)
    assert res.thermo[0, 4] == pytest.approx(1.5, rel=1e-13)
    assert np.abs(v.sum(axis=1)).max() < 1e-12


def test_nve_momentum_conserved(orc):
    res, x, v, box, w = small_lj_run(orc, steps=60)
    p = res.v.sum(axis=1)
    assert np.abs(p).max() < 1e-10 * x.shape[1]


def test_nve_energy_error_is_second_order_in_dt(orc):
    """Velocity Verlet: the energy fluctuation over a fixed time scales as dt^2.
    (Shifted LJ energy is continuous at the cutoff.)"""
    devs = []
    for dt in (0.004, 0.002, 0.001):
        steps = int(round(0.2 / dt))
        res, *_ = small_lj_run(orc, dt=dt, steps=steps, temp=1.0, seed=9)
        et = res.thermo[:, 3]
        devs.append(np.max(np.abs(et - et[0])))
    r1, r2 = devs[0] / devs[1], devs[1] / devs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, devs


def test_nve_time_reversible(orc):
    res, x0, v0, box, w = small_lj_run(orc, steps=50, temp=1.0, seed=10)
    back = orc.md_run(orc.params_for(w), res.x, -res.v, box, 50, 50)
    L = np.array(box)[:, None]
    d = back.x - x0
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-9
    assert np.abs(back.v + v0).max() < 1e-9


def test_rebuild_trigger_keeps_list_valid(orc):
    """After a run with rebuilds, the forces the run ends with equal a fresh
    all-image brute-force sum at the final positions, so the list was never
    stale; a vanishing skin makes every step rebuild."""
    res, x, v, box, w = small_lj_run(orc, ncell=4, steps=80, temp=2.0, seed=12)
    f, e, _ = brute.lj(res.x, box, 2.5)
    assert rel(res.f, f) < 1e-11
    assert res.rebuilt.sum() >= 3
    tiny = orc.md_run(orc.params_for(w, skin=0.0001), x, v, box, 20, 20)
    assert tiny.rebuilt[1:].all()


def test_rebuild_schedule_follows_half_skin(orc):
    """Rebuild happens exactly at the steps where some atom has moved more than
    skin/2 since the last build: re-run step by step and check the criterion
    from the trajectory itself."""
    w = I.scaled(I.LJ_4K, 4, temp=3.0, steps=30)
    x, v, box = I.initial_state(w, 3)
    p = orc.params_for(w)
    xs, last_build = [], None
    cur_x, cur_v = x, v
    flags = []
    first = orc.md_run(p, cur_x, cur_v, box, 0, 1)
    xref = first.x.copy()
    cur_x, cur_v = first.x, first.v
    for s in range(30):
        nxt = orc.md_run(p, cur_x, cur_v, box, 1, 1)
        # one-step runs always rebuild at their own setup, so compare the
        # displacement of the unwrapped drift against xref directly
        dx = nxt.x - xref
        L = np.array(box)[:, None]
        dx -= L * np.round(dx / L)
        moved = np.max(np.sum(dx * dx, axis=0))
        flags.append(moved > 0.15 ** 2)
        if flags[-1]:
            xref = nxt.x.copy()
        cur_x, cur_v = nxt.x, nxt.v
    whole = orc.md_run(p, x, v, box, 30, 1)
    assert whole.rebuilt[1:].astype(bool).tolist() == flags


# ------------------------------------------------------------- LJ VJP --


def lj_u_dot_f(orc, x, box, nl, u, eps=1.0, sigma=1.0):
    return float(np.sum(u * orc.lj_forces(x, box, nl, 2.5, eps=eps, sigma=sigma).f))


def test_vjp_matches_central_differences(orc):
    x, box = lj_system(4, 0.3, 51)
    nl, _ = orc.build_nlist(x, box, 2.8)
    u = I.random_unit_vectors(x.shape[1], 52)
    gx, gp = orc.lj_vjp(x, box, nl, 2.5, 1.1, 1.05, u)
    h = 1e-5
    checked = 0
    for atom in range(0, x.shape[1], 11):
        if not _frozen_ok(x, box, atom, 2.5, 1e-3):
            continue
        for d in range(3):
            xp = x.copy(); xp[d, atom] += h
            xm = x.copy(); xm[d, atom] -= h
            fd = (lj_u_dot_f(orc, xp, box, nl, u, 1.1, 1.05)
                  - lj_u_dot_f(orc, xm, box, nl, u, 1.1, 1.05)) / (2 * h)
            assert fd == pytest.approx(gx[d, atom], rel=1e-6, abs=1e-6)
            checked += 1
    assert checked >= 30
    for k, (e1, s1, e2, s2) in enumerate([(1.1 + h, 1.05, 1.1 - h, 1.05),
                                          (1.1, 1.05 + h, 1.1, 1.05 - h)]):
        fd = (lj_u_dot_f(orc, x, box, nl, u, e1, s1) - lj_u_dot_f(orc, x, box, nl, u, e2, s2)) / (2 * h)
        assert fd == pytest.approx(gp[k], rel=1e-7)


def test_vjp_symmetry_translation_and_linearity(orc):
    x, box = lj_system(5, 0.3, 61)
    nl, _ = orc.build_nlist(x, box, 2.8)
    n = x.shape[1]
    u = I.random_unit_vectors(n, 62)
    w = I.random_unit_vectors(n, 63)
    gu, _ = orc.lj_vjp(x, box, nl, 2.5, 1.0, 1.0, u)
    gw, _ = orc.lj_vjp(x, box, nl, 2.5, 1.0, 1.0, w)
    # the force Jacobian (-Hessian) is symmetric
    assert np.sum(w * gu) == pytest.approx(np.sum(u * gw), rel=1e-11)
    # a uniform translation does not change forces: J c = 0 and, by symmetry, J^T c = 0
    c = np.zeros_like(u); c[0] = 0.3; c[1] = -1.2; c[2] = 0.7
    gc, gpc = orc.lj_vjp(x, box, nl, 2.5, 1.0, 1.0, c)
    assert np.abs(gc).max() < 1e-12 * np.abs(gu).max()
    # linear in the cotangent
    g2, _ = orc.lj_vjp(x, box, nl, 2.5, 1.0, 1.0, 2.0 * u - 0.5 * w)
    assert rel(g2, 2.0 * gu - 0.5 * gw) < 1e-12


def test_force_matching_gradient_vanishes_at_target(orc):
    """L(eps, sigma) = mean |F(eps, sigma) - F(1.1, 1.05)|^2 has L = 0 and zero
    gradient at the target, and its VJP gradient matches FD elsewhere."""
    x, box = lj_system(4, 0.3, 71)
    nl, _ = orc.build_nlist(x, box, 2.8)
    ft = orc.lj_forces(x, box, nl, 2.5, eps=1.1, sigma=1.05).f
    n3 = ft.size

    def loss(e, s):
        return float(np.sum((orc.lj_forces(x, box, nl, 2.5, eps=e, sigma=s).f - ft) ** 2) / n3)

    for e, s in ((1.1, 1.05), (1.0, 1.0)):
        f = orc.lj_forces(x, box, nl, 2.5, eps=e, sigma=s).f
        u = 2.0 * (f - ft) / n3
        _, gp = orc.lj_vjp(x, box, nl, 2.5, e, s, u)
        if (e, s) == (1.1, 1.05):
            assert loss(e, s) == 0.0 and np.all(gp == 0.0)
        else:
            h = 1e-6
            fde = (loss(e + h, s) - loss(e - h, s)) / (2 * h)
            fds = (loss(e, s + h) - loss(e, s - h)) / (2 * h)
            assert gp[0] == pytest.approx(fde, rel=1e-6)
            assert gp[1] == pytest.approx(fds, rel=1e-6)
