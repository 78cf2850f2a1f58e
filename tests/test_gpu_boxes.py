"""Orthorhombic boxes: edges of different lengths, so the list cells per
dimension differ -- two in some dimension (the stencil's offsets -1 and +1
are then one cell), the row-path build (three or more along x) and the
general build (two along x) -- against the oracle: pair sets bit-exact in
three layouts, FP64 forces / energy / virial within 1e-12, MIXED within
1e-6 and the derived bound, and 40 steps of md_step (FP64 and FP32-mixed,
the mini-benchmark's kernel) against the oracle's run (rebuild steps, thermo
rows, final state)."""
import dataclasses

import numpy as np
import pytest

import mixed_bounds as MB
from gpu_helpers import assert_fp64, forces_gpu, gpu_list, gpu_pairs, rel
from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd import md
from paper_1009_4330_amd.system import MDSystem

pytestmark = pytest.mark.gpu

# fcc unit cells along x, y, z; in the comment the list cells per dimension
# at r_l = 2.8 (edge a = 1.6796)
SHAPES = [(4, 7, 9),     # 2, 4, 5: general build
          (9, 4, 5),     # 5, 2, 2: row build, two cells along y and along z
          (6, 11, 4),    # 3, 6, 2: row build with three cells along x, two along z
          (12, 6, 7),    # 7, 3, 4: row build; the tiled layouts also fit
          (4, 4, 13)]    # 2, 2, 7: general build
SIDS = ["x".join(map(str, s)) for s in SHAPES]
LAYOUTS = [(md.MD_LAYOUT_TPA, md.MD_KERNEL_TPA), (4, 4), (md.MD_LAYOUT_WPA, md.MD_KERNEL_WPA)]
LIDS = ["tpa", "k4", "wpa"]
STEPS = 40


def workload(shape):
    return dataclasses.replace(I.LJ_4K, name="lj_" + "x".join(map(str, shape)), shape=shape,
                               temp=1.5, steps=STEPS)


def min_image_diff(a, b, box):
    L = np.array(box)[:, None]
    d = a - b
    return d - L * np.round(d / L)


@pytest.mark.parametrize("layout,kernel", LAYOUTS, ids=LIDS)
@pytest.mark.parametrize("shape", SHAPES, ids=SIDS)
def test_lists_and_forces(orc, shape, layout, kernel):
    w = workload(shape)
    x, _, box = I.initial_state(w)
    x = I.jitter(x, 0.2, seed=sum(shape) * 7)
    rl = w.rc + w.skin
    print(f"[boxes] {shape} box {tuple(round(b, 3) for b in box)} layout {layout}", flush=True)
    xg, cells, nl, ws, mbox = gpu_list(x, box, w.rc, w.skin, layout, 160)
    onl, oc = orc.build_nlist(x, box, rl)
    assert np.array_equal(gpu_pairs(nl), onl.pairs())
    ref = orc.lj_forces(oc.x, box, onl, w.rc, eps=1.0, sigma=1.0, shift=0)
    f, ev = forces_gpu(md.lj_potential(w.rc, 1.0, 1.0, 0), xg, mbox, nl, md.MD_FP64, kernel, ws)
    assert_fp64(f, ref.f)
    assert ev[0] == pytest.approx(ref.energy, rel=1e-12)
    assert rel(ev[1:], ref.virial) < 1e-12
    f, ev = forces_gpu(md.lj_potential(w.rc, 1.0, 1.0, 0), xg, mbox, nl, md.MD_MIXED, kernel, ws)
    assert rel(f, ref.f) < 1e-6
    mag = MB.lj_magnitudes(oc.x, box, onl, w.rc, 1.0, 1.0)
    MB.assert_vector(f, ref.f, mag["f"], what="force")
    MB.assert_total(ev[0], ref.energy, mag["e"], what="energy")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", SHAPES, ids=SIDS)
def test_step_against_oracle_run(orc, shape, prec):
    w = workload(shape)
    x, v, box = I.initial_state(w)   # the perfect lattice, melting at T* = 1.5
    print(f"[boxes] md_step {shape} {prec}", flush=True)
    ref = orc.md_run(orc.params_for(w), x, v, box, STEPS, 5)
    sysm = MDSystem(w, x, v, prec, "auto")
    rows = np.concatenate([sysm.setup(True), sysm.run(STEPS, 5)])
    assert np.array_equal(rows[:, 6].astype(int), ref.thermo[:, 6].astype(int))
    assert rows[-1, 6] >= 2
    gx, gv, gf = sysm.host_state()
    if prec == "fp64":
        assert np.array_equal(rows[:, 7].astype(int), ref.thermo[:, 7].astype(int))
        for c in (1, 2, 3, 4, 5):
            assert rel(rows[:, c], ref.thermo[:, c]) < 1e-10, c
        assert np.abs(min_image_diff(gx, ref.x, box)).max() < 1e-9
        assert np.abs(gv - ref.v).max() < 1e-9
        assert_fp64(gf, ref.f, 1e-9)
    else:
        # the mixed run follows the FP64 one to the rounding level over 40 steps
        assert np.abs(min_image_diff(gx, ref.x, box)).max() < 1e-4
        for c in (1, 2, 3):
            assert rel(rows[:, c], ref.thermo[:, c]) < 1e-5, c
