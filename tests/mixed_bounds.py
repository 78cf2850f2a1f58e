"""Rounding-error bounds for MIXED-precision totals (test-side numpy).

In MIXED the scalar pair function is evaluated in FP32: every pair term is a
difference of two positive parts (LJ: repulsion - attraction; Sutton-Chen:
pair repulsion - embedding attraction), each carrying a relative FP32
rounding of a few units of u32 = 2^-24.  The error of any sum of such terms is
therefore bounded by K u32 times the sum of the *magnitudes* of the parts, not
by the size of the (often heavily cancelled) total.  These helpers form those
magnitude sums per pair from the oracle's neighbour list, so a test can assert
|GPU - oracle| <= K u32 M.

Worst case per pair (K_WORST = 32): the FP32 separation s carries one
rounding and the hardware reciprocal up to one ulp (2 u), and the powers
amplify that relative error by their exponent: the LJ repulsion
sigma^12 / s^7 by 7, so about 21 u, plus the roundings of the products and
of the difference of the two parts -- about 25 u in all.  Sums of many pair
terms have independent-signed rounding errors, so each tested quantity is
held to a tighter factor (K_BY_QUANTITY), about ten times the largest ratio
error / (u M) measured over the GPU parity suite (forces at rc = 5 sigma 4.2,
virial components 1.1, position adjoint 1.2, energy 0.4, parameter
gradients 0.07), and never above the worst case.
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53
K_WORST = 32.0
K = K_WORST
K_BY_QUANTITY = {"force": 32.0, "energy": 4.0, "virial": 12.0, "gx": 12.0,
                 "dL/deps": 1.0, "dL/dsigma": 1.0, "geps": 1.0, "ga": 1.0, "gc": 1.0}


def k_for(what: str) -> float:
    """The bar factor of a quantity ('virial 3' uses the virial's)."""
    return K_BY_QUANTITY.get(what.rstrip("0123456789 "), K_WORST)
VPAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def pair_geometry(x, box, onl, rc):
    """Ordered pairs (i, j) of the oracle list with s < rc^2, their d and s."""
    p = onl.pairs()
    i, j = p[:, 0], p[:, 1]
    L = np.asarray(box, dtype=np.float64)[:, None]
    d = x[:, i] - x[:, j]
    d = d - L * np.rint(d / L)
    s = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    m = s < rc * rc
    return i[m], j[m], d[:, m], s[m]


def _per_atom(n, i, vals):
    out = np.zeros(n)
    np.add.at(out, i, vals)
    return out


def lj_magnitudes(x, box, onl, rc, eps, sigma, u=None):
    """Magnitude sums for LJ: 'f' [n] per-atom force-term sums, 'e' energy,
    'w' [6] virial, and with a cotangent u: 'gx' [n], 'geps', 'gsig'."""
    n = x.shape[1]
    i, j, d, s = pair_geometry(x, box, onl, rc)
    sr6 = (sigma * sigma / s) ** 3
    mag_g = (48.0 * eps * sr6 * sr6 + 24.0 * eps * sr6) / s
    dn = np.sqrt(s)
    out = {"f": _per_atom(n, i, mag_g * dn),
           "e": 0.5 * np.sum(4.0 * eps * (sr6 * sr6 + sr6)),
           "w": np.array([0.5 * np.sum(np.abs(d[a] * d[b]) * mag_g) for a, b in VPAIRS])}
    if u is not None:
        du = u[:, i] - u[:, j]
        dun = np.sqrt(np.sum(du * du, axis=0))
        mag_gp = (336.0 * eps * sr6 * sr6 + 96.0 * eps * sr6) / (s * s)
        out["gx"] = _per_atom(n, i, mag_g * dun + 2.0 * mag_gp * dun * s)
        un = np.sqrt(np.sum(u[:, i] ** 2, axis=0))
        out["geps"] = np.sum(un * mag_g * dn) / eps
        mag_dg = 24.0 * eps / sigma * (24.0 * sr6 * sr6 + 6.0 * sr6) / s
        out["gsig"] = np.sum(mag_dg * un * dn)
    return out


def sc_magnitudes(x, box, onl, rc, eps, a, c, nexp, mexp, rho):
    """Magnitude sums for Sutton-Chen, given the oracle's densities rho [n]."""
    n = x.shape[1]
    i, j, d, s = pair_geometry(x, box, onl, rc)
    t = a * a / s
    pn = t ** (0.5 * nexp)
    pm = t ** (0.5 * mexp)
    e = np.where(rho > 0, 1.0 / np.sqrt(np.where(rho > 0, rho, 1.0)), 0.0)
    mag_h = (nexp * eps * pn + 0.5 * mexp * eps * c * (e[i] + e[j]) * pm) / s
    dn = np.sqrt(s)
    return {"f": _per_atom(n, i, mag_h * dn),
            "e": 0.5 * eps * np.sum(pn) + eps * c * np.sum(np.sqrt(rho)),
            "w": np.array([0.5 * np.sum(np.abs(d[a_] * d[b_]) * mag_h) for a_, b_ in VPAIRS])}


def assert_total(got, want, mag, u=U32, what=""):
    k = k_for(what)
    err = abs(got - want)
    bound = k * u * mag
    print(f"[bound] {what}: error {err:.3e} = {err / bound:.3g} of the bound (K = {k:g})")
    assert err <= bound, f"{what}: |{got} - {want}| = {err:.3e} > {bound:.3e}"


def assert_vector(got, want, mag_per_atom, u=U32, what=""):
    """Norm-wise: ||got - want|| <= K u ||per-atom magnitude||."""
    k = k_for(what)
    err = float(np.linalg.norm((np.asarray(got) - np.asarray(want)).ravel()))
    bound = k * u * float(np.linalg.norm(mag_per_atom))
    print(f"[bound] {what}: error {err:.3e} = {err / bound:.3g} of the bound (K = {k:g})")
    assert err <= bound, f"{what}: error {err:.3e} > bound {bound:.3e}"


def buck_magnitudes(x, box, onl, rc, types, A, rho, C, q, qqr2e):
    """Magnitude sums for Buckingham + cut Coulomb.  The FP32 exponential of
    -r / rho carries the relative error of its argument times |r / rho|, so
    the Born-Mayer parts are weighted by (1 + r / rho)."""
    n = x.shape[1]
    i, j, d, s = pair_geometry(x, box, onl, rc)
    ab = 4 * np.asarray(types)[i] + np.asarray(types)[j]
    r = np.sqrt(s)
    a_, c_ = np.asarray(A)[ab], np.asarray(C)[ab]
    rh = np.where(a_ > 0, np.asarray(rho)[ab], 1.0)
    qq = np.abs(qqr2e * np.asarray(q)[np.asarray(types)[i]] * np.asarray(q)[np.asarray(types)[j]])
    ex = a_ * np.exp(-r / rh) * (1.0 + r / rh)
    mag_g = (ex / rh + 6.0 * c_ / s ** 3.5 + qq / s) / r
    return {"f": _per_atom(n, i, mag_g * r),
            "e": 0.5 * np.sum(ex + c_ / s ** 3 + qq / r),
            "w": np.array([0.5 * np.sum(np.abs(d[a] * d[b]) * mag_g) for a, b in VPAIRS])}


def sc_vjp_magnitudes(x, box, onl, rc, eps, a, c, nexp, mexp, rho, u):
    """Magnitude sums for the Sutton-Chen adjoint: 'gx' [n] per atom, and the
    parameter gradients 'geps', 'ga', 'gc'.  The error of dL/drho_i (lam_i)
    from its own sum enters the position pass through 2 (lam_i + lam_j) psi',
    so the lam magnitudes are carried into 'gx'."""
    n = x.shape[1]
    i, j, d, s = pair_geometry(x, box, onl, rc)
    t = a * a / s
    phi, psi = t ** (0.5 * nexp), t ** (0.5 * mexp)
    e = np.where(rho > 0, 1.0 / np.sqrt(np.where(rho > 0, rho, 1.0)), 0.0)
    A = nexp * eps * phi / s
    Bc = 0.5 * mexp * eps * psi / s                    # |B| / c
    du = u[:, i] - u[:, j]
    dun = np.sqrt(np.sum(du * du, axis=0))
    r = np.sqrt(s)
    wmag = dun * r                                     # bound on |w|
    lam = 0.5 * e ** 3 * c * _per_atom(n, i, Bc * wmag)
    eij = e[i] + e[j]
    h = A + c * Bc * eij
    hp = ((0.5 * nexp + 1.0) * A + (0.5 * mexp + 1.0) * c * Bc * eij) / s
    psip = 0.5 * mexp * psi / s
    gx = _per_atom(n, i, h * dun + 2.0 * hp * wmag * r + 2.0 * (lam[i] + lam[j]) * psip * r)
    la = 0.5 * np.sum(A * wmag)
    lb = np.sum(e[i] * Bc * wmag)
    return {"gx": gx, "geps": (la + c * lb) / eps, "ga": (nexp * la + 0.5 * mexp * c * lb) / a,
            "gc": lb}
