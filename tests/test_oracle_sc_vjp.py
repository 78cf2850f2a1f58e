"""Pins of the oracle's Sutton-Chen force adjoint (vector-Jacobian product of
F(x; eps, a, c) with a cotangent u), each against something other than the
adjoint's own formulas: central differences of L = sum u . F computed from the
oracle's forces, the symmetry of the force Jacobian (minus the Hessian), its
null space (uniform translations), linearity in u, and the c = 0 limit."""
import numpy as np
import pytest

from paper_1009_4330_amd import inputs as I
from test_oracle import _frozen_ok, rel

RC = 7.22
PAR = dict(eps=1.2382e-2, a=3.61, c=39.432, nexp=9, mexp=6)


def sc_system(ncell, amp, seed):
    x = I.jitter(I.fcc_positions(ncell, 3.61), amp, seed)
    return x, (ncell * 3.61,) * 3


def u_dot_f(orc, x, box, nl, u, **kw):
    p = dict(PAR, **kw)
    return float(np.sum(u * orc.sc_forces(x, box, nl, RC, **p).f))


def vjp(orc, x, box, nl, u, **kw):
    p = dict(PAR, **kw)
    return orc.sc_vjp(x, box, nl, RC, p["eps"], p["a"], p["c"], p["nexp"], p["mexp"], u)


@pytest.fixture(scope="module")
def system(orc):
    x, box = sc_system(5, 0.25, 81)
    nl, _ = orc.build_nlist(x, box, RC + 1.0)
    return x, box, nl


def test_sc_vjp_matches_central_differences_in_x(orc, system):
    x, box, nl = system
    u = I.random_unit_vectors(x.shape[1], 82)
    gx, _ = vjp(orc, x, box, nl, u)
    h = 1e-5
    checked = 0
    for atom in range(0, x.shape[1], 13):
        if not _frozen_ok(x, box, atom, RC, 1e-3):
            continue
        for d in range(3):
            xp = x.copy(); xp[d, atom] += h
            xm = x.copy(); xm[d, atom] -= h
            fd = (u_dot_f(orc, xp, box, nl, u) - u_dot_f(orc, xm, box, nl, u)) / (2 * h)
            assert fd == pytest.approx(gx[d, atom], rel=1e-6, abs=1e-9)
            checked += 1
    assert checked >= 30


@pytest.mark.parametrize("k,name", [(0, "eps"), (1, "a"), (2, "c")])
def test_sc_vjp_parameter_gradients(orc, system, k, name):
    x, box, nl = system
    u = I.random_unit_vectors(x.shape[1], 83)
    _, gp = vjp(orc, x, box, nl, u)
    v = PAR[name]
    h = 1e-6 * v
    fd = (u_dot_f(orc, x, box, nl, u, **{name: v + h})
          - u_dot_f(orc, x, box, nl, u, **{name: v - h})) / (2 * h)
    assert gp[k] == pytest.approx(fd, rel=1e-7)


def test_sc_vjp_symmetry_translation_and_linearity(orc, system):
    x, box, nl = system
    n = x.shape[1]
    u = I.random_unit_vectors(n, 84)
    w = I.random_unit_vectors(n, 85)
    gu, _ = vjp(orc, x, box, nl, u)
    gw, _ = vjp(orc, x, box, nl, w)
    # -H is symmetric, including the many-body (embedding) part
    assert np.sum(w * gu) == pytest.approx(np.sum(u * gw), rel=1e-11)
    c = np.zeros_like(u); c[0] = 0.3; c[1] = -1.2; c[2] = 0.7
    gc, _ = vjp(orc, x, box, nl, c)
    assert np.abs(gc).max() < 1e-12 * np.abs(gu).max()
    g2, _ = vjp(orc, x, box, nl, 2.0 * u - 0.5 * w)
    assert rel(g2, 2.0 * gu - 0.5 * gw) < 1e-12


def test_sc_vjp_without_embedding(orc, system):
    """c = 0 leaves the pair repulsion alone: dL/dc is still the FD slope at
    c = 0, and the position adjoint matches FD of that pair potential."""
    x, box, nl = system
    u = I.random_unit_vectors(x.shape[1], 86)
    gx, gp = vjp(orc, x, box, nl, u, c=0.0)
    h = 1e-4
    fd = (u_dot_f(orc, x, box, nl, u, c=h) - u_dot_f(orc, x, box, nl, u, c=-h)) / (2 * h)
    # L is linear in c only through the embedding term's prefactor, but
    # rho^(1/2) is c-independent: FD is exact up to rounding
    assert gp[2] == pytest.approx(fd, rel=1e-8)
    atom = next(a for a in range(x.shape[1]) if _frozen_ok(x, box, a, RC, 1e-3))
    hx = 1e-5
    for d in range(3):
        xp = x.copy(); xp[d, atom] += hx
        xm = x.copy(); xm[d, atom] -= hx
        fdx = (u_dot_f(orc, xp, box, nl, u, c=0.0) - u_dot_f(orc, xm, box, nl, u, c=0.0)) / (2 * hx)
        assert fdx == pytest.approx(gx[d, atom], rel=1e-6, abs=1e-9)


def test_sc_fit_gradient_vanishes_at_target(orc, system):
    """Force matching on (eps, a, c): zero loss and zero gradient at the target."""
    x, box, nl = system
    ft = orc.sc_forces(x, box, nl, RC, **PAR).f
    u = 2.0 * (ft - ft) / ft.size
    _, gp = vjp(orc, x, box, nl, u)
    assert np.all(gp == 0.0)
