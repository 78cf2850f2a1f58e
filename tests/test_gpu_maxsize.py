"""Parity at the largest size the bench times: the LJ melt at 2,048,000 atoms
(fcc 80^3), FP32-mixed md_step with the mini-benchmark's kernel against the
oracle's FP64 run of the same size (rebuild steps), then, at the oracle's
final positions, the library's list against the oracle's row by row (every
atom's neighbour set) and the MIXED and FP64 forces over all atoms."""
import math

import numpy as np
import pytest
import torch

from gpu_helpers import assert_fp64, rel
from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd import md
from paper_1009_4330_amd.system import MDSystem

pytestmark = pytest.mark.gpu

STEPS = 20


def sorted_rows(neigh: torch.Tensor, count: torch.Tensor, width: int) -> torch.Tensor:
    """[n][width] rows, entries past each atom's count replaced by INT32_MAX,
    sorted along each row (neighbour sets become comparable)."""
    n, cap = neigh.shape
    out = torch.full((n, width), 2147483647, dtype=torch.int32, device=neigh.device)
    m = torch.arange(cap, device=neigh.device)[None, :] < count[:, None]
    out[:, :cap] = torch.where(m, neigh.to(torch.int32), torch.full_like(out[:, :cap], 2147483647))
    return torch.sort(out, dim=1).values


def test_maxsize_lj_mixed_2m(orc):
    w = I.scaled(I.LJ_256K, 80)
    n = w.natoms
    assert n == 2048000
    x, v, box = I.initial_state(w)
    print(f"[maxsize] lj melt {n} atoms, mixed, {STEPS} steps", flush=True)
    sysm = MDSystem(w, x, v, "mixed", "auto")
    rows = np.concatenate([sysm.setup(True), sysm.run(STEPS, 5)])
    ref = orc.md_run(orc.params_for(w), x, v, box, STEPS, 5)
    assert np.array_equal(rows[:, 6].astype(int), ref.thermo[:, 6].astype(int))
    assert rows[-1, 6] > 1
    # the library's list at the oracle's final positions, against the oracle's
    rl = w.rc + w.skin
    xd = torch.as_tensor(ref.x, dtype=torch.float64, device="cuda").contiguous()
    mbox = md.make_box(box)
    cells = md.Cells(n, int(np.prod([math.floor(L / rl) for L in box])))
    ws = md.workspace(n, mbox, rl)
    md.md_bin_cells(xd, mbox, rl, cells, ws)
    nl = md.NList(n, 160, sysm.nl.layout)
    md.md_build_neighbors(xd, mbox, cells, w.rc, w.skin, nl)
    onl, oc = orc.build_nlist(ref.x, box, rl)
    got_n = nl.numneigh
    want_n = torch.as_tensor(onl.numneigh, device="cuda")
    assert torch.equal(got_n, want_n.to(got_n.dtype))
    width = max(nl.capacity, onl.cap)
    got = sorted_rows(nl.rows(), got_n, width)
    want = sorted_rows(torch.as_tensor(onl.neigh, device="cuda"), want_n, width)
    assert torch.equal(got, want)
    del got, want
    print(f"[maxsize] lists equal: {int(got_n.sum())} entries", flush=True)
    pot = md.lj_potential(w.rc, 1.0, 1.0, 1)
    f = torch.zeros(3, n, dtype=torch.float64, device="cuda")
    md.md_compute_forces(pot, xd, mbox, nl, md.MD_MIXED, md.MD_KERNEL_AUTO, 0, f, None, ws)
    err = rel(f.cpu().numpy(), ref.f)
    print(f"[maxsize] mixed force rel-RMS {err:.3e}", flush=True)
    assert err < 1e-6
    md.md_compute_forces(pot, xd, mbox, nl, md.MD_FP64, md.MD_KERNEL_AUTO, 0, f, None, ws)
    assert_fp64(f.cpu().numpy(), ref.f)
