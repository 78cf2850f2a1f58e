"""HIP path vs the CPU oracle, element by element, on the same seeded inputs.

Bars: integer work (wrap, cells, permutation, neighbour pair sets) bit-exact;
FP64 forces / energy / virial / adjoint within 1e-12 relative (norm-wise over
all components, the FP64 summation order being the only difference); MIXED
(FP32 pair function, FP64 separation, cutoff test and accumulation) within
1e-6 relative RMS of the FP64 oracle.
"""
import dataclasses

import numpy as np
import pytest
import torch

import mixed_bounds as MB
from gpu_helpers import (SC_KW, assert_fp64, dev, forces_gpu, gpu_bin, gpu_list, gpu_pairs,
                         lj_liquid, rel, sc_solid)
from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd import md
from paper_1009_4330_amd.system import MDSystem

pytestmark = pytest.mark.gpu

LAYOUTS = [(md.MD_LAYOUT_TPA, md.MD_KERNEL_TPA), (4, 4), (16, 16),
           (md.MD_LAYOUT_WPA, md.MD_KERNEL_WPA)]
IDS = ["tpa", "k4", "k16", "wpa"]


def jittered_lj(ncell, seed, amp=0.35, outside=0.15):
    x = I.jitter(I.fcc_positions(ncell, I.A_LJ), amp, seed)
    box = (ncell * I.A_LJ,) * 3
    rng = np.random.default_rng(seed)
    for d in range(3):
        k = rng.choice(x.shape[1], 16, replace=False)
        x[d, k[:8]] = -rng.uniform(0, outside, 8)
        x[d, k[8:]] = box[d] + rng.uniform(0, outside, 8)
    return x, box


# ----------------------------------------------------------- binning --


@pytest.mark.parametrize("ncell,seed", [(5, 1), (10, 2), (13, 3)])
def test_bin_cells_bit_exact(orc, ncell, seed):
    x_np, box = jittered_lj(ncell, seed)
    x, cells, ws, _ = gpu_bin(x_np, box, 2.8)
    want = orc.bin_cells(x_np, box, 2.8)
    assert tuple(cells.nc) == tuple(want.nc)
    assert np.array_equal(x.cpu().numpy(), want.x)          # wrapped coordinates, bitwise
    assert np.array_equal(cells.atom_cell.cpu().numpy(), want.atom_cell)
    ncell_tot = int(np.prod(want.nc))
    assert np.array_equal(cells.cell_start.cpu().numpy()[: ncell_tot + 1], want.cell_start)
    assert np.array_equal(cells.perm.cpu().numpy(), want.perm)


def test_sort_atoms_gathers_through_perm(orc):
    x_np, box = jittered_lj(6, 4)
    v_np = I.random_unit_vectors(x_np.shape[1], 5)
    x, cells, ws, mbox = gpu_bin(x_np, box, 2.8)
    st = md.State(x, dev(v_np), 1.0)
    st.f.copy_(dev(2.0 * v_np))
    xr = dev(x_np)
    md.md_sort_atoms(st, cells, xr, ws)
    perm = orc.bin_cells(x_np, box, 2.8).perm
    want_x = orc.bin_cells(x_np, box, 2.8).x[:, perm]
    assert np.array_equal(st.x.cpu().numpy(), want_x)
    assert np.array_equal(st.v.cpu().numpy(), v_np[:, perm])
    assert np.array_equal(st.f.cpu().numpy(), 2.0 * v_np[:, perm])
    assert np.array_equal(xr.cpu().numpy(), x_np[:, perm])
    assert np.array_equal(st.id.cpu().numpy(), perm)


# ---------------------------------------------------- neighbour lists --


@pytest.mark.parametrize("layout,kernel", LAYOUTS, ids=IDS)
@pytest.mark.parametrize("case", ["jitter500", "liquid4k", "jitter2k_nc3"])
def test_neighbor_pairs_bit_exact(orc, case, layout, kernel):
    if case == "jitter500":
        x_np, box = jittered_lj(5, 11)
    elif case == "liquid4k":
        x_np, _, box, _ = lj_liquid(orc, 10, 12)
    else:
        x_np, box = jittered_lj(8, 13)    # 4 cells per dimension
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 2.5, 0.3, layout, 160)
    ref, ocells = orc.build_nlist(x_np, box, 2.8)
    got = gpu_pairs(nl)
    assert got.shape == ref.pairs().shape
    assert np.array_equal(got, ref.pairs())
    assert np.array_equal(nl.numneigh.cpu().numpy(), ref.numneigh)
    assert np.array_equal(nl.x_ref.cpu().numpy(), ocells.x)
    words = md.md_nlist_status(nl)
    assert words[md.MD_ST_ERRORS] == 0 and words[md.MD_ST_MAXNEIGH] == ref.max_count


@pytest.mark.parametrize("case", ["liquid4k_nc5", "jitter864_nc3", "liquid4k_rc5",
                                  "liquid6912_nc7"])
def test_step_setup_list_bit_exact(orc, case):
    """md_step's own build (atoms sorted into cell order, lists built along x
    rows of cells; the rc = 5 case has slabs too large for that path and takes
    the per-cell one) against the oracle's list on the oracle's own wrapped,
    cell-sorted positions."""
    rc = 2.5
    if case == "liquid4k_nc5":
        x_np, v_np, box, w = lj_liquid(orc, 10, 21)
    elif case == "jitter864_nc3":
        x_np, box = jittered_lj(6, 22)
        w = I.scaled(I.LJ_4K, 6)
        v_np = I.random_unit_vectors(x_np.shape[1], 23)
    elif case == "liquid4k_rc5":
        rc = 5.0
        x_np, v_np, box, w = lj_liquid(orc, 10, 24)
        w = dataclasses.replace(w, rc=rc)
    else:
        x_np, v_np, box, w = lj_liquid(orc, 12, 25, steps=20)   # 7 cells per dimension
    s = MDSystem(w, x_np, v_np, "fp64", "k4", capacity=700 if rc > 3 else 160)
    s.setup(thermo=False)
    rl = rc + w.skin
    oc = orc.bin_cells(x_np, box, rl)
    xs = np.ascontiguousarray(oc.x[:, oc.perm])          # oracle's wrapped, sorted positions
    ref, _ = orc.build_nlist(xs, box, rl)
    assert np.array_equal(s.state.id.cpu().numpy(), oc.perm)
    assert np.array_equal(s.state.x.cpu().numpy(), xs)
    assert np.array_equal(s.nl.x_ref.cpu().numpy(), xs)
    assert np.array_equal(s.cells.cell_start.cpu().numpy()[: len(oc.cell_start)],
                          oc.cell_start)
    assert np.array_equal(gpu_pairs(s.nl), ref.pairs())
    assert np.array_equal(s.nl.numneigh.cpu().numpy(), ref.numneigh)
    words = md.md_nlist_status(s.nl)
    assert words[md.MD_ST_ERRORS] == 0 and words[md.MD_ST_MAXNEIGH] == ref.max_count


def test_neighbor_overflow_reports_required_capacity(orc):
    x_np, box = jittered_lj(5, 14)
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 2.5, 0.3, md.MD_LAYOUT_TPA, 20)
    ref, _ = orc.build_nlist(x_np, box, 2.8)
    words = md.md_nlist_status(nl)
    assert words[md.MD_ST_ERRORS] & 1
    assert words[md.MD_ST_MAXNEIGH] == ref.max_count
    assert np.array_equal(nl.numneigh.cpu().numpy(), ref.numneigh)


# -------------------------------------------------------------- forces --


def oracle_lj(orc, x_np, box, shift=0, eps=1.0, sigma=1.0, rc=2.5, skin=0.3):
    nl, cells = orc.build_nlist(x_np, box, rc + skin)
    return orc.lj_forces(cells.x, box, nl, rc, eps=eps, sigma=sigma, shift=shift), cells.x


@pytest.mark.parametrize("layout,kernel", LAYOUTS, ids=IDS)
@pytest.mark.parametrize("shift", [0, 1])
def test_lj_forces_fp64(orc, layout, kernel, shift):
    x_np, _, box, _ = lj_liquid(orc, 10, 21)
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 2.5, 0.3, layout, 160)
    pot = md.lj_potential(2.5, 1.0, 1.0, shift)
    f, ev = forces_gpu(pot, x, mbox, nl, md.MD_FP64, kernel, ws)
    ref, _ = oracle_lj(orc, x_np, box, shift)
    assert_fp64(f, ref.f)
    assert ev[0] == pytest.approx(ref.energy, rel=1e-12)
    assert rel(ev[1:], ref.virial) < 1e-12


@pytest.mark.parametrize("layout,kernel", LAYOUTS, ids=IDS)
def test_lj_forces_mixed(orc, layout, kernel):
    x_np, _, box, _ = lj_liquid(orc, 10, 22)
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 2.5, 0.3, layout, 160)
    f, ev = forces_gpu(md.lj_potential(2.5), x, mbox, nl, md.MD_MIXED, kernel, ws)
    ref, _ = oracle_lj(orc, x_np, box)
    err = rel(f, ref.f)
    print(f"mixed LJ force rel-RMS {err:.3e}")
    assert err < 1e-6
    onl, oc = orc.build_nlist(x_np, box, 2.8)
    mag = MB.lj_magnitudes(oc.x, box, onl, 2.5, 1.0, 1.0)
    MB.assert_vector(f, ref.f, mag["f"], what="force")
    MB.assert_total(ev[0], ref.energy, mag["e"], what="energy")
    for c in range(6):
        MB.assert_total(ev[1 + c], ref.virial[c], mag["w"][c], what=f"virial {c}")


def test_lj_nondefault_parameters_and_high_cutoff(orc):
    x_np, _, box, _ = lj_liquid(orc, 12, 23)
    for layout, kernel in LAYOUTS:
        x, cells, nl, ws, mbox = gpu_list(x_np, box, 5.0, 0.3, layout, 700)
        pot = md.lj_potential(5.0, 1.3, 0.93, 0)
        f, ev = forces_gpu(pot, x, mbox, nl, md.MD_FP64, kernel, ws)
        ref, _ = oracle_lj(orc, x_np, box, eps=1.3, sigma=0.93, rc=5.0)
        assert_fp64(f, ref.f)
        assert ev[0] == pytest.approx(ref.energy, rel=1e-12)


@pytest.mark.parametrize("layout,kernel", LAYOUTS, ids=IDS)
@pytest.mark.parametrize("prec", [md.MD_FP64, md.MD_MIXED], ids=["fp64", "mixed"])
def test_sutton_chen_forces(orc, layout, kernel, prec):
    x_np, box = sc_solid(6, 31)
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 7.22, 1.0, layout, 260)
    pot = md.sc_potential(7.22, SC_KW["eps"], SC_KW["a"], SC_KW["c"], 9, 6)
    f, ev = forces_gpu(pot, x, mbox, nl, prec, kernel, ws)
    onl, ocells = orc.build_nlist(x_np, box, 8.22)
    ref = orc.sc_forces(ocells.x, box, onl, 7.22, **SC_KW)
    if prec == md.MD_FP64:
        assert_fp64(f, ref.f)
        assert ev[0] == pytest.approx(ref.energy, rel=1e-12)
        assert rel(ev[1:], ref.virial) < 1e-12
    else:
        err = rel(f, ref.f)
        print(f"mixed SC force rel-RMS {err:.3e}")
        assert err < 1e-6
        mag = MB.sc_magnitudes(ocells.x, box, onl, 7.22, SC_KW["eps"], SC_KW["a"], SC_KW["c"],
                               9, 6, ref.rho)
        MB.assert_vector(f, ref.f, mag["f"], what="force")
        MB.assert_total(ev[0], ref.energy, mag["e"], what="energy")
        for c in range(6):
            MB.assert_total(ev[1 + c], ref.virial[c], mag["w"][c], what=f"virial {c}")


def test_sutton_chen_perfect_lattice_tie(orc):
    """The 8th shell sits exactly at rc = 2a: both sides must take the same
    FP64 decision for every one of those pairs."""
    x_np = I.fcc_positions(6, 3.61)
    box = (6 * 3.61,) * 3
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 7.22, 1.0, md.MD_LAYOUT_TPA, 260)
    pot = md.sc_potential(7.22, SC_KW["eps"], SC_KW["a"], SC_KW["c"], 9, 6)
    f, ev = forces_gpu(pot, x, mbox, nl, md.MD_FP64, md.MD_KERNEL_TPA, ws)
    onl, ocells = orc.build_nlist(x_np, box, 8.22)
    ref = orc.sc_forces(ocells.x, box, onl, 7.22, **SC_KW)
    assert ev[0] == pytest.approx(ref.energy, rel=1e-12)
    assert np.abs(f - ref.f).max() < 1e-12 * max(1.0, np.abs(ref.f).max())


# ------------------------------------------------------------- adjoint --


@pytest.mark.parametrize("layout,kernel", LAYOUTS, ids=IDS)
@pytest.mark.parametrize("prec", [md.MD_FP64, md.MD_MIXED], ids=["fp64", "mixed"])
def test_lj_vjp(orc, layout, kernel, prec):
    x_np, _, box, _ = lj_liquid(orc, 10, 41)
    n = x_np.shape[1]
    u_np = I.random_unit_vectors(n, 42)
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 2.5, 0.3, layout, 160)
    pot = md.lj_potential(2.5, 1.1, 1.05, 0)
    gx = torch.zeros(3, n, dtype=torch.float64, device="cuda")
    gp = torch.zeros(2, dtype=torch.float64, device="cuda")
    md.md_force_vjp(pot, x, mbox, nl, prec, dev(u_np), gx, gp, ws)
    onl, ocells = orc.build_nlist(x_np, box, 2.8)
    rgx, rgp = orc.lj_vjp(ocells.x, box, onl, 2.5, 1.1, 1.05, u_np)
    ggx, ggp = gx.cpu().numpy(), gp.cpu().numpy()
    mag = MB.lj_magnitudes(ocells.x, box, onl, 2.5, 1.1, 1.05, u_np)
    if prec == md.MD_FP64:
        assert_fp64(ggx, rgx, what="gx")
        MB.assert_total(ggp[0], rgp[0], mag["geps"], u=MB.U64, what="dL/deps")
        MB.assert_total(ggp[1], rgp[1], mag["gsig"], u=MB.U64, what="dL/dsigma")
    else:
        print(f"mixed vjp rel error {rel(ggx, rgx):.3e}, gparam {ggp} vs {rgp}")
        MB.assert_vector(ggx, rgx, mag["gx"], what="gx")
        MB.assert_total(ggp[0], rgp[0], mag["geps"], what="dL/deps")
        MB.assert_total(ggp[1], rgp[1], mag["gsig"], what="dL/dsigma")


# ------------------------------------------------------------ auto select --


def test_autoselect_choice_matches_layout(orc):
    x_np, _, box, _ = lj_liquid(orc, 10, 51)
    x, cells, ws, mbox = gpu_bin(x_np, box, 2.8)
    nl = md.NList(x_np.shape[1], 160)
    pot = md.lj_potential(2.5)
    choice = md.md_autoselect(pot, x, mbox, cells, 0.3, nl, md.MD_FP64, 3, ws)
    print(f"auto-selected {choice} lanes per atom")
    assert choice in md.LANES
    assert nl.layout == choice
    words = md.md_nlist_status(nl)
    assert words[md.MD_ST_BUILDS] == 0     # trial builds are not counted
    f, ev = forces_gpu(pot, x, mbox, nl, md.MD_FP64, md.MD_KERNEL_AUTO, ws)
    ref, _ = oracle_lj(orc, x_np, box)
    assert_fp64(f, ref.f)
