"""The two remaining workloads at their full sizes, in FP32-mixed as well as
FP64, against the oracle over all atoms: the 108,000-atom LJ system at cutoff
5 sigma (several hundred neighbours per atom) with one lane, the
mini-benchmark's choice and a whole wavefront per atom, and the 500,000-atom
Sutton-Chen solid.  Positions are seeded jitters of the workloads' lattices,
handed to both sides; no input comes from the HIP path."""
import math

import numpy as np
import pytest
import torch

import mixed_bounds as MB
from gpu_helpers import assert_fp64, gpu_pairs, rel
from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd import md

pytestmark = pytest.mark.gpu


def binned(x_np, box, rl):
    n = x_np.shape[1]
    x = torch.as_tensor(np.ascontiguousarray(x_np), dtype=torch.float64, device="cuda")
    mbox = md.make_box(box)
    cells = md.Cells(n, int(np.prod([math.floor(L / rl) for L in box])))
    ws = md.workspace(n, mbox, rl)
    md.md_bin_cells(x, mbox, rl, cells, ws)
    return x, mbox, cells, ws


def forces(pot, x, mbox, nl, prec, ws):
    n = x.shape[1]
    f = torch.zeros(3, n, dtype=torch.float64, device="cuda")
    ev = torch.zeros(7, dtype=torch.float64, device="cuda")
    md.md_compute_forces(pot, x, mbox, nl, prec, md.MD_KERNEL_AUTO, md.MD_EFLAG | md.MD_VFLAG,
                         f, ev, ws)
    torch.cuda.synchronize()
    return f.cpu().numpy(), ev.cpu().numpy()


@pytest.mark.parametrize("kernel", [md.MD_KERNEL_TPA, md.MD_KERNEL_AUTO, md.MD_KERNEL_WPA],
                         ids=["k1", "auto", "k64"])
def test_lj_rc5_108k_both_precisions(orc, kernel):
    w = I.LJ_HI_108K
    x_np = I.jitter(I.fcc_positions(w.ncell, w.a), 0.25, 108)
    box = w.box
    rl = w.rc + w.skin
    print(f"[c3] {w.natoms} atoms rc {w.rc}, kernel {kernel}", flush=True)
    x, mbox, cells, ws = binned(x_np, box, rl)
    pot = md.lj_potential(w.rc, 1.0, 1.0, 1)
    nl = md.NList(w.natoms, 700, md.MD_LAYOUT_TPA if kernel == md.MD_KERNEL_AUTO else kernel)
    if kernel == md.MD_KERNEL_AUTO:
        lanes = md.md_autoselect(pot, x, mbox, cells, w.skin, nl, md.MD_MIXED, 3, ws)
        print(f"[c3] auto-selected {lanes} lanes per atom")
    else:
        md.md_build_neighbors(x, mbox, cells, w.rc, w.skin, nl)
    onl, oc = orc.build_nlist(x_np, box, rl)
    assert np.array_equal(gpu_pairs(nl), onl.pairs())
    ref = orc.lj_forces(oc.x, box, onl, w.rc, shift=1)
    f64, ev64 = forces(pot, x, mbox, nl, md.MD_FP64, ws)
    assert_fp64(f64, ref.f)
    assert ev64[0] == pytest.approx(ref.energy, rel=1e-12)
    assert rel(ev64[1:], ref.virial) < 1e-12
    fm, evm = forces(pot, x, mbox, nl, md.MD_MIXED, ws)
    err = rel(fm, ref.f)
    print(f"[c3] mixed force rel-RMS {err:.3e}")
    assert err < 1e-6
    mag = MB.lj_magnitudes(oc.x, box, onl, w.rc, 1.0, 1.0)
    MB.assert_vector(fm, ref.f, mag["f"], what="force")
    MB.assert_total(evm[0], ref.energy, mag["e"], what="energy")
    for c in range(6):
        MB.assert_total(evm[1 + c], ref.virial[c], mag["w"][c], what=f"virial {c}")


def test_sutton_chen_500k_both_precisions(orc):
    w = I.SC_500K
    x_np = I.jitter(I.fcc_positions(w.ncell, w.a), 0.12, 500)
    box = w.box
    rl = w.rc + w.skin
    print(f"[c4] {w.natoms} atoms", flush=True)
    x, mbox, cells, ws = binned(x_np, box, rl)
    pot = md.sc_potential(w.rc, w.sc_eps, w.sc_a, w.sc_c, w.sc_n, w.sc_m)
    nl = md.NList(w.natoms, 260, md.MD_LAYOUT_TPA)
    lanes = md.md_autoselect(pot, x, mbox, cells, w.skin, nl, md.MD_MIXED, 3, ws)
    print(f"[c4] auto-selected {lanes} lanes per atom")
    onl, oc = orc.build_nlist(x_np, box, rl)
    ref = orc.sc_forces(oc.x, box, onl, w.rc, w.sc_eps, w.sc_a, w.sc_c, w.sc_n, w.sc_m)
    f64, ev64 = forces(pot, x, mbox, nl, md.MD_FP64, ws)
    assert_fp64(f64, ref.f)
    assert ev64[0] == pytest.approx(ref.energy, rel=1e-12)
    fm, evm = forces(pot, x, mbox, nl, md.MD_MIXED, ws)
    err = rel(fm, ref.f)
    print(f"[c4] mixed force rel-RMS {err:.3e}")
    assert err < 1e-6
    mag = MB.sc_magnitudes(oc.x, box, onl, w.rc, w.sc_eps, w.sc_a, w.sc_c, w.sc_n, w.sc_m,
                           ref.rho)
    MB.assert_vector(fm, ref.f, mag["f"], what="force")
    MB.assert_total(evm[0], ref.energy, mag["e"], what="energy")
