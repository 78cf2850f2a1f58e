"""Degenerate and boundary inputs against the oracle: a single atom, the
two-atom minimum of md_step in a box of two cells per dimension, a clustered
system whose cells are mostly empty (listed from unsorted atoms, and by
md_step's row build with its crowded runs), and a slab of atoms on cell faces
and on the box faces (x = 0 and x = L before wrapping)."""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_helpers import assert_fp64, forces_gpu, gpu_list, gpu_pairs, rel
from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd import md
from paper_1009_4330_amd.system import MDSystem

pytestmark = pytest.mark.gpu


def test_single_atom(orc):
    box = (6.0, 6.0, 6.0)
    x_np = np.array([[1.0], [2.0], [3.0]])
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 2.5, 0.3, 1, 8)
    assert nl.numneigh.cpu().numpy().tolist() == [0]
    f, ev = forces_gpu(md.lj_potential(2.5), x, mbox, nl, md.MD_FP64, md.MD_KERNEL_TPA, ws)
    assert np.all(f == 0.0) and np.all(ev == 0.0)


@pytest.mark.parametrize("kernel", ["tpa", "wpa"])
def test_two_atoms_in_a_two_cell_box(orc, kernel):
    """md_step's smallest case: two atoms 1.2 sigma apart (one across the
    periodic face), 2 list cells per dimension, against the oracle's run."""
    w = dataclasses.replace(I.scaled(I.LJ_4K, 1), ncell=1, a=6.0, steps=50)
    box = (6.0, 6.0, 6.0)
    x = np.array([[0.3, 5.1], [3.0, 3.0], [3.0, 3.0]])
    v = np.array([[0.5, -0.5], [0.2, -0.2], [0.0, 0.0]])
    ref = orc.md_run(orc.params_for(w), x, v, box, 50, 5)
    s = MDSystem(w, x, v, "fp64", kernel, capacity=8)
    rows = np.concatenate([s.setup(True), s.run(50, 5)])
    for c in (1, 2, 3, 4, 5):
        assert rel(rows[:, c], ref.thermo[:, c]) < 1e-10, c
    gx, gv, gf = s.host_state()
    L = np.array(box)[:, None]
    d = gx - ref.x
    assert np.abs(d - L * np.round(d / L)).max() < 1e-9
    assert np.abs(gv - ref.v).max() < 1e-9


@pytest.mark.parametrize("layout", [1, 4])
def test_clustered_atoms_mostly_empty_cells(orc, layout):
    """A dense droplet in one corner of a large box: most cells are empty and
    the occupied ones are crowded; list and forces against the oracle."""
    rng = np.random.default_rng(31)
    base = I.fcc_positions(5, I.A_LJ)                       # 500 atoms, 8.4 sigma cube
    x_np = base + rng.uniform(-0.05, 0.05, base.shape) + 1.0
    box = (30.0, 30.0, 30.0)
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 2.5, 0.3, layout, 120)
    ref, oc = orc.build_nlist(x_np, box, 2.8)
    assert np.array_equal(gpu_pairs(nl), ref.pairs())
    f, ev = forces_gpu(md.lj_potential(2.5), x, mbox, nl, md.MD_FP64, md.MD_KERNEL_AUTO, ws)
    fr = orc.lj_forces(oc.x, box, ref, 2.5)
    assert_fp64(f, fr.f)
    assert ev[0] == pytest.approx(fr.energy, rel=1e-12)


def test_row_build_crowded_runs_against_oracle(orc):
    """A dense droplet in a dilute box: the mean occupancy (about 9 atoms per
    list cell) sends md_step's build down the row path, while the runs
    through the droplet (about 48 per cell) hold more candidates than a run's
    LDS and are built one cell at a time.  md_step's cell order and list
    against the oracle's on the same sorted positions."""
    w = I.scaled(I.LJ_4K, 14, temp=0.5)
    box = w.box
    rng = np.random.default_rng(11)
    ax = np.arange(-8.0, 8.0001, 0.8)
    g = np.stack(np.meshgrid(ax, ax, ax, indexing="ij")).reshape(3, -1)
    ball = g[:, (g * g).sum(0) < 64.0] + np.array(box)[:, None] / 2
    far = np.round(rng.uniform(0, box[0], (3, 200)) / 0.8) * 0.8
    x_np = np.unique(np.round(np.concatenate([ball, far], axis=1), 9), axis=1)
    x_np = np.ascontiguousarray(x_np + rng.uniform(-0.02, 0.02, x_np.shape))
    v_np = np.zeros_like(x_np)
    s = MDSystem(w, x_np, v_np, "fp64", "k4", capacity=400)
    s.setup(thermo=False)
    rl = w.rc + w.skin
    oc = orc.bin_cells(x_np, box, rl)
    ncell = len(oc.cell_start) - 1
    counts = np.diff(oc.cell_start)
    print(f"[crowded] {x_np.shape[1]} atoms, {ncell} cells, mean {x_np.shape[1] / ncell:.1f}, "
          f"largest {counts.max()} per cell", flush=True)
    assert 36 * x_np.shape[1] / ncell < 400 and 36 * np.sort(counts)[-27:].mean() > 960
    xs = np.ascontiguousarray(oc.x[:, oc.perm])
    ref, _ = orc.build_nlist(xs, box, rl)
    assert np.array_equal(s.state.id.cpu().numpy(), oc.perm)
    assert np.array_equal(gpu_pairs(s.nl), ref.pairs())
    assert np.array_equal(s.nl.numneigh.cpu().numpy(), ref.numneigh)


def test_atoms_on_cell_and_box_faces(orc):
    """Coordinates exactly on cell boundaries (k L / nc) and on both box
    faces (0 and L, which wraps to 0): binning and pair set bit for bit."""
    box = (16.8, 16.8, 16.8)
    nc = 6                                  # floor(16.8 / 2.8)
    edge = box[0] / nc
    g = np.arange(nc + 1) * edge            # includes L itself
    xs, ys, zs = np.meshgrid(g, g[::2], g[1::2], indexing="ij")
    x_np = np.stack([xs.ravel(), ys.ravel() + 0.37, zs.ravel() + 0.11])
    x_np = x_np[:, np.argsort(x_np[0] + 1e-3 * np.arange(x_np.shape[1]), kind="stable")]
    # drop the copies of x = 0 that x = L wraps onto
    keep = x_np[0] < box[0]
    x_np = np.ascontiguousarray(np.concatenate([x_np[:, keep], x_np[:, ~keep][:, :3]], axis=1))
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 2.5, 0.3, 1, 64)
    want = orc.bin_cells(x_np, box, 2.8)
    assert np.array_equal(x.cpu().numpy(), want.x)
    assert np.array_equal(cells.atom_cell.cpu().numpy(), want.atom_cell)
    ref, _ = orc.build_nlist(x_np, box, 2.8)
    assert np.array_equal(gpu_pairs(nl), ref.pairs())
