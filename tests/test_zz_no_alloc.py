"""md_compute_forces_noalloc (fixed library scratch, no workspace) against
md_compute_forces (caller's workspace) on the same inputs: both run the same
kernels in the same order, so forces, energy and virial must agree bit for
bit.  Two calls in a row, the second on a smaller system, so the second call
reuses scratch the first one filled; then a Sutton-Chen call (the density
column in the scratch) and a half list (the atomic-add path)."""
import numpy as np
import pytest
import torch

from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd import md

from gpu_helpers import SC_KW, gpu_list, sc_solid

pytestmark = pytest.mark.gpu

EV = md.MD_EFLAG | md.MD_VFLAG


def both(pot, x, mbox, nl, prec, ws, flags=EV):
    n = x.shape[1]
    out = []
    for noalloc in (False, True):
        f = torch.full((3, n), np.nan, dtype=torch.float64, device="cuda")
        ev = torch.full((7,), np.nan, dtype=torch.float64, device="cuda")
        if noalloc:
            md.md_compute_forces_noalloc(pot, x, mbox, nl, prec, md.MD_KERNEL_AUTO, flags, f, ev)
        else:
            md.md_compute_forces(pot, x, mbox, nl, prec, md.MD_KERNEL_AUTO, flags, f, ev, ws)
        torch.cuda.synchronize()
        out.append((f.cpu().numpy(), ev.cpu().numpy()))
    return out


def lj_case(ncell, seed, layout):
    w = I.scaled(I.LJ_4K, ncell)
    x = I.jitter(I.fcc_positions(ncell, w.a), 0.3, seed)
    box = w.box
    xd, cells, nl, ws, mbox = gpu_list(x, box, w.rc, w.skin, layout, 160)
    return md.lj_potential(w.rc, 1.0, 1.0, 1), xd, mbox, nl, ws


@pytest.mark.parametrize("prec", [md.MD_FP64, md.MD_MIXED])
def test_noalloc_matches_workspace_call_twice_second_smaller(prec):
    for ncell, seed, layout in ((12, 11, 4), (6, 12, 1)):   # 6912 atoms, then 864
        pot, x, mbox, nl, ws = lj_case(ncell, seed, layout)
        (f_ws, ev_ws), (f_na, ev_na) = both(pot, x, mbox, nl, prec, ws)
        assert np.isfinite(f_ws).all() and np.isfinite(ev_ws).all()
        assert np.array_equal(f_na, f_ws), ncell
        assert np.array_equal(ev_na, ev_ws), ncell
        # forces only (no energy / virial columns in the scratch)
        (f_ws, _), (f_na, _) = both(pot, x, mbox, nl, prec, ws, flags=0)
        assert np.array_equal(f_na, f_ws), ncell


def test_noalloc_sutton_chen_and_half_list():
    x, box = sc_solid(5, 21)
    rc, skin = 7.22, 1.0
    xd, cells, nl, ws, mbox = gpu_list(x, box, rc, skin, 4, 260)
    pot = md.sc_potential(rc, SC_KW["eps"], SC_KW["a"], SC_KW["c"], SC_KW["nexp"], SC_KW["mexp"])
    for prec in (md.MD_FP64, md.MD_MIXED):
        (f_ws, ev_ws), (f_na, ev_na) = both(pot, xd, mbox, nl, prec, ws)
        assert np.array_equal(f_na, f_ws) and np.array_equal(ev_na, ev_ws)
    # half list: atomic adds make the last bits order-dependent, so compare
    # to the FP64 bar instead of bitwise
    w = I.scaled(I.LJ_4K, 8)
    xl = I.jitter(I.fcc_positions(8, w.a), 0.3, 5)
    xd, cells, nlh, ws, mbox = gpu_list(xl, w.box, w.rc, w.skin, 1, 160)
    nlh_half = md.NList(xl.shape[1], 160, 1, half=True)
    md.md_build_neighbors(xd, mbox, cells, w.rc, w.skin, nlh_half)
    pot = md.lj_potential(w.rc)
    (f_ws, ev_ws), (f_na, ev_na) = both(pot, xd, mbox, nlh_half, md.MD_FP64, ws)
    assert np.linalg.norm(f_na - f_ws) <= 1e-12 * np.linalg.norm(f_ws)
    assert np.allclose(ev_na, ev_ws, rtol=1e-12, atol=0)


def test_noalloc_rejects_more_than_its_scratch():
    """A call that needs more than the fixed scratch is refused before any
    launch, with MD_ERR_SCRATCH; the same call with a workspace runs."""
    n = md.MD_NOALLOC_SCRATCH_BYTES // 88 + 1000   # LJ with energy / virial: 88 B per atom
    assert md.md_compute_forces_noalloc_bytes(n, md.MD_POT_LJ, EV) > md.MD_NOALLOC_SCRATCH_BYTES
    assert md.md_compute_forces_noalloc_bytes(n, md.MD_POT_LJ, 0) <= md.MD_NOALLOC_SCRATCH_BYTES
    ncell = 1
    while 4 * ncell ** 3 < n:
        ncell += 1
    w = I.scaled(I.LJ_4K, ncell)
    x = torch.as_tensor(I.fcc_positions(ncell, w.a), device="cuda").contiguous()
    nl = md.NList(x.shape[1], 1, 1)
    mbox = md.make_box(w.box)
    f = torch.zeros_like(x)
    ev = torch.zeros(7, dtype=torch.float64, device="cuda")
    pot = md.lj_potential(w.rc)
    with pytest.raises(md.MDError) as e:
        md.md_compute_forces_noalloc(pot, x, mbox, nl, md.MD_FP64, 0, EV, f, ev)
    assert e.value.code == md.MD_ERR_SCRATCH
    assert np.all(f.cpu().numpy() == 0.0)   # nothing was enqueued
