"""Independent O(N^2) checks for tiny periodic boxes (numpy, FP64).

Nothing here shares code with the oracle: no cells, no minimum-image rule.
Every image of every atom within range is enumerated explicitly, for shifts
-2..2 of the box in each dimension, and pair sums are formed from the
textbook potentials written out again.
"""
from __future__ import annotations

import itertools

import numpy as np

SHIFTS = np.array(list(itertools.product(range(-2, 3), repeat=3)), dtype=np.float64)


def _images(x, box, i0, i1):
    """d[i, j, s, :] = x_i - (x_j + shift_s * L) for i in [i0, i1)."""
    L = np.asarray(box, dtype=np.float64)
    xi = x.T[i0:i1, None, None, :]
    xj = x.T[None, :, None, :] + (SHIFTS * L)[None, None, :, :]
    return xi - xj


def pairs_within(x, box, r, chunk=16):
    """Sorted ordered pairs (i, j), i != j, with some image of j within r of i."""
    n = x.shape[1]
    out = []
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        d = _images(x, box, i0, i1)
        s = np.einsum("ijsk,ijsk->ijs", d, d)
        hit = (s < r * r).any(axis=2)
        ii, jj = np.nonzero(hit)
        ii = ii + i0
        keep = ii != jj
        out.append(np.stack([ii[keep], jj[keep]], axis=1))
    p = np.concatenate(out).astype(np.int64)
    return p[np.lexsort((p[:, 1], p[:, 0]))]


def _pair_terms(x, box, rc, chunk, fn):
    n = x.shape[1]
    for i0 in range(0, n, chunk):
        i1 = min(n, i0 + chunk)
        d = _images(x, box, i0, i1)
        s = np.einsum("ijsk,ijsk->ijs", d, d)
        idx = np.arange(i0, i1)
        self_img = np.zeros_like(s, dtype=bool)
        self_img[np.arange(i1 - i0), idx, SHIFTS.tolist().index([0.0, 0.0, 0.0])] = True
        m = (s < rc * rc) & ~self_img
        yield i0, i1, d, s, m


def lj(x, box, rc, eps=1.0, sigma=1.0, chunk=16):
    """Forces [3][N], energy, virial[6] of 12-6 LJ summed over all images."""
    n = x.shape[1]
    f = np.zeros((n, 3))
    e = 0.0
    w = np.zeros(6)
    for i0, i1, d, s, m in _pair_terms(x, box, rc, chunk, None):
        ss = np.where(m, s, 1.0)
        inv6 = (sigma * sigma / ss) ** 3
        phi = np.where(m, 4.0 * eps * (inv6 * inv6 - inv6), 0.0)
        # F_ij = -dphi/dr * d/r = 24 eps (2 (sigma/r)^12 - (sigma/r)^6) / r^2 * d
        g = np.where(m, 24.0 * eps * (2.0 * inv6 * inv6 - inv6) / ss, 0.0)
        f[i0:i1] += np.einsum("ijs,ijsk->ik", g, d)
        e += 0.5 * phi.sum()
        for q, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
            w[q] += 0.5 * np.sum(g * d[..., a] * d[..., b])
    return f.T.copy(), e, w


def sutton_chen(x, box, rc, eps, a, c, nexp, mexp, chunk=16):
    """Forces [3][N], energy, rho[N] of Sutton-Chen summed over all images,
    from E = eps [1/2 sum_ij (a/r)^n - c sum_i sqrt(rho_i)] by the chain rule."""
    n = x.shape[1]
    rho = np.zeros(n)
    rep = np.zeros(n)
    for i0, i1, d, s, m in _pair_terms(x, box, rc, chunk, None):
        r = np.sqrt(np.where(m, s, 1.0))
        rho[i0:i1] += np.where(m, (a / r) ** mexp, 0.0).sum(axis=(1, 2))
        rep[i0:i1] += np.where(m, (a / r) ** nexp, 0.0).sum(axis=(1, 2))
    energy = eps * float(np.sum(0.5 * rep - c * np.sqrt(rho)))
    # dE/dr_ij for one unordered pair: eps [ V'(r) - c/2 (1/sqrt(rho_i) + 1/sqrt(rho_j)) phi'(r) ]
    inv = np.where(rho > 0, 1.0 / np.sqrt(np.where(rho > 0, rho, 1.0)), 0.0)
    f = np.zeros((n, 3))
    for i0, i1, d, s, m in _pair_terms(x, box, rc, chunk, None):
        r = np.sqrt(np.where(m, s, 1.0))
        vp = -nexp * (a / r) ** nexp / r
        php = -mexp * (a / r) ** mexp / r
        emb = 0.5 * c * (inv[i0:i1, None, None] + inv[None, :, None])
        dedr = eps * (vp - emb * php)
        coef = np.where(m, -dedr / r, 0.0)
        f[i0:i1] += np.einsum("ijs,ijsk->ik", coef, d)
    return f.T.copy(), energy, rho


def fcc_shells(rmax, a):
    """Distances and multiplicities of fcc lattice vectors with 0 < r < rmax,
    by enumerating the integer points (h, k, l) of the a/2 grid with h+k+l even."""
    kmax = int(np.ceil(2.0 * rmax / a)) + 1
    rng = np.arange(-kmax, kmax + 1)
    h, k, l = np.meshgrid(rng, rng, rng, indexing="ij")
    m2 = (h * h + k * k + l * l).ravel()
    even = ((h + k + l) % 2 == 0).ravel()
    m2 = m2[even & (m2 > 0)]
    vals, counts = np.unique(m2, return_counts=True)
    r = 0.5 * a * np.sqrt(vals)
    keep = r < rmax
    return r[keep], counts[keep], vals[keep]
