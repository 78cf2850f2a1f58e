"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and rejects invalid host arguments before touching the GPU;
plus the seeded input generators."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1009_4330_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "md.h")


@pytest.fixture(scope="module")
def mdlib():
    from paper_1009_4330_amd import md
    if not os.path.exists(md.LIB_PATH):
        from paper_1009_4330_amd import build
        build.build()
    return md


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(md_[a-z_]+)\s*\(", text)))


def test_header_declares_the_five_calls():
    names = declared_functions()
    for call in ("md_bin_cells", "md_build_neighbors", "md_compute_forces", "md_step",
                 "md_force_vjp"):
        assert call in names


def test_library_exports_every_declared_symbol(mdlib):
    lib = mdlib.lib()
    names = declared_functions()
    assert set(names) == set(mdlib.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(mdlib):
    for code in range(10):
        assert mdlib.status_string(code) != "unknown status"
    assert mdlib.status_string(3) == "neighbour list capacity exceeded"


def test_workspace_and_rows_host_logic(mdlib):
    lib = mdlib.lib()
    box = mdlib.make_box((16.8, 16.8, 16.8))
    b = lib.md_workspace_bytes(4000, ctypes.byref(box), 2.8)
    assert b > 4000 * (8 * 3 * 3 + 8 * 9) and b % 256 == 0
    assert lib.md_workspace_bytes(4000, ctypes.byref(mdlib.make_box((5.0, 16.8, 16.8))), 2.8) == 0
    assert lib.md_workspace_bytes(0, ctypes.byref(box), 2.8) == 0
    # atom-count limit (32-byte position records addressed with 32-bit offsets)
    big = mdlib.make_box((400.0, 400.0, 400.0))
    assert lib.md_workspace_bytes(mdlib.MD_MAX_ATOMS, ctypes.byref(big), 2.8) > 0
    assert lib.md_workspace_bytes(mdlib.MD_MAX_ATOMS + 1, ctypes.byref(big), 2.8) == 0
    # the neighbour buffer fits every lanes-per-atom layout K (see md.h)
    for n, cap in ((4000, 100), (1, 1), (100, 7), (256000, 130)):
        want = max(-(-n // (64 // k)) * -(-cap // k) * 64 for k in mdlib.LANES)
        assert mdlib.md_nlist_ints(n, cap) == want
    assert lib.md_nlist_ints(10, 0) == 0
    assert mdlib.md_thermo_rows(100, 10, 1) == 11
    assert mdlib.md_thermo_rows(100, 7, 0) == 14
    assert mdlib.md_thermo_rows(-1, 10, 0) == 0


def test_host_validation_precedes_any_launch(mdlib):
    """Each of these returns its code from host checks alone (no device)."""
    lib = mdlib.lib()
    fake = ctypes.c_void_p(0x1000)
    box = mdlib.make_box(I.LJ_4K.box)
    small = mdlib.make_box((5.0, 16.8, 16.8))
    cells = mdlib.md_cells(ncell_cap=125, cell_start=0x1000, atom_cell=0x1000, perm=0x1000)
    nl = mdlib.md_nlist(capacity=100, layout=1, rl=2.8, neigh=0x1000, numneigh=0x1000,
                        x_ref=0x1000, status=0x1000)
    lj = mdlib.lj_potential(2.5)
    R = ctypes.byref
    assert lib.md_bin_cells(None, 4000, R(box), 2.8, R(cells), fake, 1 << 30, None) == 1
    assert lib.md_bin_cells(fake, 4000, R(small), 2.8, R(cells), fake, 1 << 30, None) == 2
    assert lib.md_bin_cells(fake, 0, R(box), 2.8, R(cells), fake, 1 << 30, None) == 1
    assert lib.md_bin_cells(fake, 4000, R(box), 2.8, R(cells), fake, 16, None) == 7
    tiny_cells = mdlib.md_cells(ncell_cap=10, cell_start=0x1000, atom_cell=0x1000, perm=0x1000)
    assert lib.md_bin_cells(fake, 4000, R(box), 2.8, R(tiny_cells), fake, 1 << 30, None) == 1
    # wrong kernel / layout pairing, bad precision, bad flags
    assert lib.md_compute_forces(R(lj), fake, 4000, R(box), R(nl), 0, 2, 0, fake, None, fake,
                                 1 << 30, None) == 1
    assert lib.md_compute_forces(R(lj), fake, 4000, R(box), R(nl), 7, 1, 0, fake, None, fake,
                                 1 << 30, None) == 1
    assert lib.md_compute_forces(R(lj), fake, 4000, R(box), R(nl), 0, 1, 1, fake, None, fake,
                                 1 << 30, None) == 1
    bad = mdlib.lj_potential(-1.0)
    assert lib.md_compute_forces(R(bad), fake, 4000, R(box), R(nl), 0, 1, 0, fake, None, fake,
                                 1 << 30, None) == 1
    buck = mdlib.md_potential(kind=mdlib.MD_POT_BUCK, rc=2.5, qqr2e=14.4, type=0x1000)
    assert lib.md_force_vjp(R(buck), fake, 4000, R(box), R(nl), 0, fake, fake, None, fake,
                            1 << 30, None) == 5
    # Buckingham tables: species array required, tables symmetric
    nospecies = mdlib.md_potential(kind=mdlib.MD_POT_BUCK, rc=2.5, qqr2e=14.4)
    assert lib.md_compute_forces(R(nospecies), fake, 4000, R(box), R(nl), 0, 1, 0, fake, None,
                                 fake, 1 << 30, None) == 1
    asym = mdlib.md_potential(kind=mdlib.MD_POT_BUCK, rc=2.5, qqr2e=14.4, type=0x1000)
    asym.buck_A[1], asym.buck_rho[1] = 100.0, 0.3
    assert lib.md_compute_forces(R(asym), fake, 4000, R(box), R(nl), 0, 1, 0, fake, None,
                                 fake, 1 << 30, None) == 1
    nl0 = mdlib.md_nlist(capacity=0, layout=1, rl=2.8, neigh=0x1000, numneigh=0x1000,
                         x_ref=0x1000, status=0x1000)
    assert lib.md_build_neighbors(fake, 4000, R(box), R(cells), 2.5, 0.3, R(nl0), None) == 1
    st = mdlib.md_state(n=4000, x=0x1000, v=0x1000, f=0x1000, id=0x1000, mass=1.0, ftm2v=1.0,
                        mvv2e=1.0, boltz=1.0)
    assert lib.md_step(R(st), R(lj), R(small), R(cells), R(nl), 0, 1, 0.3, 0.005, 10, 10, 1,
                       fake, fake, 1 << 30, None) == 2
    assert lib.md_step(R(st), R(lj), R(box), R(cells), R(nl), 0, 1, 0.3, -0.005, 10, 10, 1,
                       fake, fake, 1 << 30, None) == 1
    assert lib.md_step(R(st), R(lj), R(box), R(cells), R(nl), 0, 1, 0.3, 0.005, 10, 0, 1,
                       None, fake, 1 << 30, None) == 1


# ------------------------------------------------------------ inputs --


def test_fcc_lattice_counts_and_spacing():
    x = I.fcc_positions(3, 2.0)
    assert x.shape == (3, 108)
    L = 6.0
    d = x[:, :, None] - x[:, None, :]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(axis=0))
    np.fill_diagonal(r, np.inf)
    assert np.allclose(r.min(axis=1), 2.0 / math.sqrt(2.0))
    assert np.all((r < 1.5).sum(axis=1) == 12)


def test_workload_sizes():
    assert I.LJ_4K.natoms == 4000 and I.LJ_256K.natoms == 256000
    assert I.LJ_HI_108K.natoms == 108000 and I.SC_500K.natoms == 500000
    assert I.LJ_FM_32K.natoms == 32000
    assert I.LJ_256K.box[0] == pytest.approx(40 * (4 / 0.8442) ** (1 / 3))
    assert 4 * I.LJ_4K.ncell ** 3 / I.LJ_4K.box[0] ** 3 == pytest.approx(0.8442)


def test_velocities_seeded_zero_momentum_exact_temperature():
    v1 = I.gaussian_velocities(4000, 3.0, 1.0, I.LJ_UNITS, 4000)
    v2 = I.gaussian_velocities(4000, 3.0, 1.0, I.LJ_UNITS, 4000)
    assert np.array_equal(v1, v2)
    assert np.abs(v1.sum(axis=1)).max() < 1e-10
    t = np.sum(v1 * v1) / (3 * 4000 - 3)
    assert t == pytest.approx(3.0, rel=1e-14)
    vm = I.gaussian_velocities(500, 600.0, 63.55, I.METAL_UNITS, 5)
    tm = 63.55 * I.METAL_MVV2E * np.sum(vm * vm) / ((3 * 500 - 3) * I.METAL_BOLTZ)
    assert tm == pytest.approx(600.0, rel=1e-14)


def test_binding_structs_match_the_header(mdlib, tmp_path):
    """Every ctypes structure of the Python binding has the size and field
    offsets the C compiler gives the header's struct (compiled here with gcc),
    and the binding's constants equal the header's."""
    structs = {"md_box": mdlib.md_box, "md_potential": mdlib.md_potential,
               "md_cells": mdlib.md_cells, "md_nlist": mdlib.md_nlist,
               "md_state": mdlib.md_state, "md_nhc": mdlib.md_nhc, "md_npt": mdlib.md_npt}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "md.h"', 'int main(void) {']
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    for const in ("MD_NHC_MAX", "MD_NHC_STATE", "MD_MAX_ATOMS", "MD_STATUS_WORDS",
                  "MD_POT_BUCK", "MD_LAYOUT_WPA", "MD_LAYOUT_TILE", "MD_NPT_STATE",
                  "MD_NOALLOC_SCRATCH_BYTES"):
        lines.append(f'  printf("const {const} %lld\\n", (long long){const});')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o",
                           str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
    for const in ("MD_NHC_MAX", "MD_NHC_STATE", "MD_MAX_ATOMS", "MD_STATUS_WORDS",
                  "MD_POT_BUCK", "MD_LAYOUT_WPA", "MD_LAYOUT_TILE", "MD_NPT_STATE",
                  "MD_NOALLOC_SCRATCH_BYTES"):
        assert got[("const", const)] == getattr(mdlib, const), const


def test_binding_rejects_a_list_sized_for_fewer_atoms(mdlib):
    """A list built for fewer atoms than the positions hold is refused on the
    host, before any pointer reaches a kernel (host tensors suffice: the
    check runs first)."""
    import torch
    nl = mdlib.NList(50, 8, mdlib.MD_LAYOUT_TPA, device="cpu")
    x = torch.zeros(3, 100, dtype=torch.float64)
    f = torch.zeros_like(x)
    ws = torch.zeros(16, dtype=torch.uint8)
    box = mdlib.make_box((20.0, 20.0, 20.0))
    pot = mdlib.lj_potential(2.5)
    for call in (lambda: mdlib.md_compute_forces(pot, x, box, nl, mdlib.MD_FP64, 0, 0, f, None, ws),
                 lambda: mdlib.md_force_vjp(pot, x, box, nl, mdlib.MD_FP64, x, f, None, ws),
                 lambda: mdlib.md_build_neighbors(x, box, None, 2.5, 0.3, nl)):
        with pytest.raises(ValueError, match="list holds 50 atoms"):
            call()
    # a list whose neigh buffer is too short for its capacity
    nl2 = mdlib.NList(100, 8, mdlib.MD_LAYOUT_TPA, device="cpu")
    nl2.neigh = nl2.neigh[:10]
    with pytest.raises(ValueError, match="neigh holds 10 ints"):
        mdlib.md_compute_forces(pot, x, box, nl2, mdlib.MD_FP64, 0, 0, f, None, ws)


def test_noalloc_scratch_limit_is_checked_on_the_host(mdlib):
    """md_compute_forces_noalloc refuses a call larger than its fixed scratch
    (MD_ERR_SCRATCH) from host checks alone, and sizes its scratch as its
    header states."""
    lib = mdlib.lib()
    fake = ctypes.c_void_p(0x1000)
    R = ctypes.byref
    box = mdlib.make_box(I.LJ_4K.box)
    nl = mdlib.md_nlist(capacity=100, layout=1, rl=2.8, neigh=0x1000, numneigh=0x1000,
                        x_ref=0x1000, status=0x1000)
    lj = mdlib.lj_potential(2.5)
    ev = mdlib.MD_EFLAG | mdlib.MD_VFLAG
    r256 = lambda b: -(-b // 256) * 256
    for n in (1, 4000, 256000):
        assert mdlib.md_compute_forces_noalloc_bytes(n, mdlib.MD_POT_LJ, 0) == r256(32 * n)
        assert mdlib.md_compute_forces_noalloc_bytes(n, mdlib.MD_POT_SC, ev) == (
            r256(32 * n) + r256(8 * n) + r256(8 * n) + r256(48 * n) + r256(512 * 8 * 8))
    assert mdlib.md_compute_forces_noalloc_bytes(0, mdlib.MD_POT_LJ, 0) == 0
    big = mdlib.MD_NOALLOC_SCRATCH_BYTES // 88 + 1000
    assert lib.md_compute_forces_noalloc(R(lj), fake, big, R(box), R(nl), 0, 1, ev, fake, fake,
                                         None) == mdlib.MD_ERR_SCRATCH
    # argument errors come first, as in md_compute_forces
    assert lib.md_compute_forces_noalloc(R(lj), fake, big, R(box), R(nl), 0, 2, ev, fake, fake,
                                         None) == mdlib.MD_ERR_INVALID_ARG
    assert mdlib.status_string(mdlib.MD_ERR_SCRATCH) != "unknown status"


def test_tile_entries_host_logic(mdlib):
    """The tiled layouts apply with at least 4 cells along x and 3 along y, z
    and a window that fits the LDS; their buffer covers every K they take."""
    lib = mdlib.lib()
    box = mdlib.make_box(I.LJ_256K.box)
    e = mdlib.md_nlist_tile_entries(256000, 160, box, 2.8)
    assert e > 0 and e % 128 == 0
    # at least one 32-bit word pair per row group and lane for each entry
    assert e >= 2 * 256000 * 160 // 2
    assert mdlib.md_nlist_tile_entries(4000, 160, mdlib.make_box(I.LJ_4K.box), 2.8) > 0
    # 3 cells along x (16.8 / 5.3): no tiled layout
    assert mdlib.md_nlist_tile_entries(4000, 160, mdlib.make_box((16.8, 16.8, 16.8)), 5.3) == 0
    # rc 5 sigma at density 0.8442: windows far larger than the LDS
    assert mdlib.md_nlist_tile_entries(108000, 700, mdlib.make_box(I.LJ_HI_108K.box), 5.3) == 0
    assert lib.md_nlist_tile_entries(0, 160, ctypes.byref(box), 2.8) == 0
    # a tiled layout is refused where the K-lane layout is the only option
    fake = ctypes.c_void_p(0x1000)
    R = ctypes.byref
    nl = mdlib.md_nlist(capacity=100, layout=mdlib.MD_LAYOUT_TILE | 16, rl=2.8, neigh=0x1000,
                        numneigh=0x1000, x_ref=0x1000, status=0x1000)
    lj = mdlib.lj_potential(2.5)
    bx = mdlib.make_box(I.LJ_4K.box)
    assert lib.md_compute_forces(R(lj), fake, 4000, R(bx), R(nl), 0, 0, 0, fake, None, fake,
                                 1 << 30, None) == mdlib.MD_ERR_INVALID_ARG


def test_npt_host_checks(mdlib):
    """md_step_npt refuses, before any launch, a continuing run whose box has
    shrunk below its cell grid (edges under nc rl) and invalid barostat
    parameters."""
    lib = mdlib.lib()
    fake = ctypes.c_void_p(0x1000)
    R = ctypes.byref
    cells = mdlib.md_cells(nc=(5, 5, 5), ncell_cap=125, cell_start=0x1000, atom_cell=0x1000,
                           perm=0x1000)
    nl = mdlib.md_nlist(capacity=100, layout=4, rl=2.8, neigh=0x1000, numneigh=0x1000,
                        x_ref=0x1000, status=0x1000)
    st = mdlib.md_state(n=4000, x=0x1000, v=0x1000, f=0x1000, id=0x1000, mass=1.0, ftm2v=1.0,
                        mvv2e=1.0, boltz=1.0)
    lj = mdlib.lj_potential(2.5)
    npt = mdlib.md_npt(t_target=1.5, t_damp=0.5, chain=3, p_target=1.0, p_damp=0.5,
                       state=0x1000)
    small = mdlib.make_box((5 * 2.8 * 0.99,) * 3)      # below 5 cells of 2.8
    assert lib.md_step_npt(R(st), R(lj), R(small), R(cells), R(nl), 0, 4, 0.3, 0.005, R(npt), 10,
                           10, 0, None, fake, 1 << 30, None) == mdlib.MD_ERR_BOX_TOO_SMALL
    bad = mdlib.md_npt(t_target=1.5, t_damp=0.5, chain=3, p_target=1.0, p_damp=0.0,
                       state=0x1000)
    box = mdlib.make_box(I.LJ_4K.box)
    assert lib.md_step_npt(R(st), R(lj), R(box), R(cells), R(nl), 0, 4, 0.3, 0.005, R(bad), 10,
                           10, 1, None, fake, 1 << 30, None) == mdlib.MD_ERR_INVALID_ARG
    assert lib.md_step_npt(R(st), R(lj), R(box), R(cells), R(nl), 0, 4, 0.3, 0.005, None, 10,
                           10, 1, None, fake, 1 << 30, None) == mdlib.MD_ERR_INVALID_ARG


def test_tiled_layout_needs_a_large_enough_tile_buffer(mdlib):
    """A tiled kernel is refused (MD_ERR_UNSUPPORTED) before any launch when
    the list's tile buffer is smaller than the run's grid needs, and in NPT
    runs, whose cell grid is not the box's."""
    lib = mdlib.lib()
    fake = ctypes.c_void_p(0x1000)
    R = ctypes.byref
    w = I.LJ_4K
    box = mdlib.make_box(w.box)
    need = mdlib.md_nlist_tile_entries(w.natoms, 160, box, 2.8)
    cells = mdlib.md_cells(ncell_cap=125, cell_start=0x1000, atom_cell=0x1000, perm=0x1000)
    st = mdlib.md_state(n=w.natoms, x=0x1000, v=0x1000, f=0x1000, id=0x1000, mass=1.0,
                        ftm2v=1.0, mvv2e=1.0, boltz=1.0)
    lj = mdlib.lj_potential(2.5)
    tiled = mdlib.MD_LAYOUT_TILE | 4
    short = mdlib.md_nlist(capacity=160, layout=1, rl=2.8, neigh=0x1000, numneigh=0x1000,
                           x_ref=0x1000, status=0x1000, tile=0x1000, tile_entries=need - 1)
    assert lib.md_step(R(st), R(lj), R(box), R(cells), R(short), 0, tiled, 0.3, 0.005, 10, 10, 1,
                       None, fake, 1 << 30, None) == mdlib.MD_ERR_UNSUPPORTED
    full = mdlib.md_nlist(capacity=160, layout=1, rl=2.8, neigh=0x1000, numneigh=0x1000,
                          x_ref=0x1000, status=0x1000, tile=0x1000, tile_entries=need)
    npt = mdlib.md_npt(t_target=1.5, t_damp=0.5, chain=3, p_target=1.0, p_damp=0.5,
                       state=0x1000)
    assert lib.md_step_npt(R(st), R(lj), R(box), R(cells), R(full), 0, tiled, 0.3, 0.005, R(npt),
                           10, 10, 1, None, fake, 1 << 30, None) == mdlib.MD_ERR_UNSUPPORTED
