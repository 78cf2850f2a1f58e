"""Shared setup for the GPU parity tests: seeded inputs are handed to both the
HIP path (through the C ABI binding) and the oracle, never from one to the
other."""
from __future__ import annotations

import math

import numpy as np
import torch

from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd import md

SC_KW = dict(eps=1.2382e-2, a=3.61, c=39.432, nexp=9, mexp=6)


def dev(a) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def ncell_of(box, rl):
    return int(np.prod([math.floor(L / rl) for L in box]))


def gpu_bin(x_np, box, rl):
    n = x_np.shape[1]
    x = dev(x_np)
    mbox = md.make_box(box)
    cells = md.Cells(n, ncell_of(box, rl))
    ws = md.workspace(n, mbox, rl)
    md.md_bin_cells(x, mbox, rl, cells, ws)
    return x, cells, ws, mbox


def gpu_list(x_np, box, rc, skin, layout, cap):
    """Bin (wrapping a device copy) and build a list; returns (x, cells, nl, ws, box)."""
    x, cells, ws, mbox = gpu_bin(x_np, box, rc + skin)
    nl = md.NList(x_np.shape[1], cap, layout)
    md.md_build_neighbors(x, mbox, cells, rc, skin, nl)
    return x, cells, nl, ws, mbox


def gpu_pairs(nl: md.NList) -> np.ndarray:
    rows = nl.rows().cpu().numpy()
    cnt = np.minimum(nl.numneigh.cpu().numpy(), nl.capacity)
    n = cnt.shape[0]
    i = np.repeat(np.arange(n, dtype=np.int64), cnt)
    mask = np.arange(nl.capacity)[None, :] < cnt[:, None]
    j = rows[mask].astype(np.int64)
    p = np.stack([i, j], axis=1)
    return p[np.lexsort((p[:, 1], p[:, 0]))]


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def lj_liquid(orc, ncell, seed, steps=40, temp=1.5):
    """A melted LJ configuration from the oracle's own NVE run (seeded)."""
    w = I.scaled(I.LJ_4K, ncell, temp=temp)
    x, v, box = I.initial_state(w, seed)
    if steps:
        res = orc.md_run(orc.params_for(w), x, v, box, steps, steps)
        x, v = res.x, res.v
    return x, v, box, w


def sc_solid(ncell, seed, amp=0.15):
    x = I.jitter(I.fcc_positions(ncell, 3.61), amp, seed)
    return x, (ncell * 3.61,) * 3


def forces_gpu(pot, x, mbox, nl, prec, kernel, ws, flags=md.MD_EFLAG | md.MD_VFLAG):
    n = x.shape[1]
    f = torch.zeros(3, n, dtype=torch.float64, device="cuda")
    ev = torch.zeros(7, dtype=torch.float64, device="cuda")
    md.md_compute_forces(pot, x, mbox, nl, prec, kernel, flags, f, ev, ws)
    torch.cuda.synchronize()
    return f.cpu().numpy(), ev.cpu().numpy()


def assert_fp64(got, want, bar: float = 1e-12, what: str = "forces") -> None:
    """FP64 parity of a per-atom [3][n] field: the norm-wise relative error
    over all components and the largest per-atom error (relative to the
    largest per-atom magnitude) both within bar.  The per-atom check keeps a
    few bad atoms from hiding in the norm of a large system."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    e = rel(got, want)
    assert e < bar, f"{what}: norm-wise relative error {e:.3e} >= {bar:.0e}"
    d = np.sqrt(((got - want) ** 2).sum(axis=0))
    m = float(np.sqrt((want ** 2).sum(axis=0)).max())
    assert d.max() <= bar * max(m, 1e-300), (
        f"{what}: largest per-atom error {d.max():.3e} > {bar:.0e} x {m:.3e}")
