"""LDS-tiled LJ kernels (layouts MD_LAYOUT_TILE | K) in md_step.

The tiled kernel with K lanes per atom reads the same list entries in the same
order as the K-lane kernel and forms every separation with the same FP64
operations from the same position records (in LDS instead of memory), so
its forces -- and whole md_step trajectories -- equal the K-lane kernel's
bit for bit; the K-lane kernel is itself held to the oracle.  Also: the
tiled run against the oracle directly, the path for a window larger than the
LDS (a dense droplet in a dilute box), and the mini-benchmark's choice."""
import numpy as np
import pytest

from gpu_helpers import assert_fp64, lj_liquid, rel
from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd import md
from paper_1009_4330_amd.system import MDSystem

pytestmark = pytest.mark.gpu


def run(w, x, v, prec, kernel, steps, every):
    s = MDSystem(w, x, v, prec, kernel)
    rows = np.concatenate([s.setup(True), s.run(steps, every)])
    gx, gv, gf = s.host_state()
    return s, rows, gx, gv, gf


@pytest.mark.parametrize("k", md.TILE_LANES)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_tiled_run_equals_k_lane_run_bitwise(orc, k, prec):
    x, v, box, w = lj_liquid(orc, 12, 90 + k)          # 6912 atoms, 7 cells per edge
    s_t, rows_t, xt, vt, ft = run(w, x, v, prec, f"t{k}", 60, 10)
    s_k, rows_k, xk, vk, fk = run(w, x, v, prec, f"k{k}", 60, 10)
    assert s_t.nl.layout == (md.MD_LAYOUT_TILE | k)
    assert rows_t[-1, 6] > 3                            # several rebuilds
    assert np.array_equal(rows_t, rows_k)
    assert np.array_equal(xt, xk) and np.array_equal(vt, vk) and np.array_equal(ft, fk)


def test_tiled_c1_against_oracle(orc):
    """The 4,000-atom melt, FP64, 100 steps with the tiled K = 4 kernel
    against the oracle's run: rebuild steps, thermo rows, final state."""
    w = I.LJ_4K
    x, v, box = I.initial_state(w)
    s, rows, gx, gv, gf = run(w, x, v, "fp64", "t4", 100, 10)
    ref = orc.md_run(orc.params_for(w), x, v, box, 100, 10)
    assert np.array_equal(rows[:, 6].astype(int), ref.thermo[:, 6].astype(int))
    for c in (1, 2, 3, 4, 5):
        assert rel(rows[:, c], ref.thermo[:, c]) < 1e-10, c
    L = np.array(box)[:, None]
    d = gx - ref.x
    assert np.abs(d - L * np.round(d / L)).max() < 1e-9
    assert_fp64(gf, ref.f, 1e-9)


def test_tiled_melt_256k_equals_k4(orc):
    """The headline workload: 40 mixed steps, tiled K = 4 against K = 4."""
    w = I.LJ_256K
    x, v, box = I.initial_state(w)
    print("[tile] lj_melt_256k mixed 40 steps, t4 and k4", flush=True)
    _, rows_t, xt, vt, ft = run(w, x, v, "mixed", "t4", 40, 10)
    _, rows_k, xk, vk, fk = run(w, x, v, "mixed", "k4", 40, 10)
    assert np.array_equal(rows_t, rows_k)
    assert np.array_equal(xt, xk) and np.array_equal(ft, fk)


def test_window_larger_than_lds_reads_memory(orc):
    """A dense droplet in a dilute box: the mean occupancy sizes the runs for
    small windows, while the droplet's windows hold more atoms than the LDS
    and take the path that reads positions from memory; the forces equal the
    K-lane kernel's."""
    w = I.scaled(I.LJ_4K, 14, temp=0.5)
    box = w.box
    rng = np.random.default_rng(7)
    # a grid of spacing 0.8 inside a ball of radius 8 (about 4,200 atoms, about
    # 48 per cell) plus 200 scattered grid points elsewhere
    ax = np.arange(-8.0, 8.0001, 0.8)
    g = np.stack(np.meshgrid(ax, ax, ax, indexing="ij")).reshape(3, -1)
    ball = g[:, (g * g).sum(0) < 64.0] + np.array(box)[:, None] / 2
    far = np.round(rng.uniform(0, box[0], (3, 200)) / 0.8) * 0.8
    x = np.unique(np.round(np.concatenate([ball, far], axis=1), 9), axis=1)
    x = np.ascontiguousarray(x + rng.uniform(-0.02, 0.02, x.shape))
    v = np.zeros_like(x)
    print(f"[tile] droplet of {x.shape[1]} atoms", flush=True)
    s_t = MDSystem(w, x, v, "fp64", "t4", capacity=400)
    s_t.setup(False)
    s_k = MDSystem(w, x, v, "fp64", "k4", capacity=400)
    s_k.setup(False)
    assert s_t.nl.layout == (md.MD_LAYOUT_TILE | 4)
    assert np.array_equal(s_t.host_state()[2], s_k.host_state()[2])


def test_auto_considers_tiled_kernels(orc):
    w = I.scaled(I.LJ_4K, 16)
    x, v, box = I.initial_state(w)
    s = MDSystem(w, x, v, "mixed", "auto")
    s.setup(False)
    print(f"[tile] auto chose layout {s.nl.layout:#x}")
    s.run(20, 20)
    assert s.nl.layout in md.LANES or (s.nl.layout & ~md.MD_LAYOUT_TILE) in md.TILE_LANES
