"""Half neighbour lists (each pair once, Newton's third law) on the GPU: the
pair set is the oracle's full list restricted to i < j, bit for bit, and the
forces, energy and virial from it equal the oracle's full-list results."""
import numpy as np
import pytest
import torch

import mixed_bounds as MB
from gpu_helpers import (SC_KW, assert_fp64, forces_gpu, gpu_bin, gpu_pairs, lj_liquid, rel,
                         sc_solid)
from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd import md
from test_gpu_parity import jittered_lj

pytestmark = pytest.mark.gpu

LAYOUTS = [1, 4, 64]


def half_list(x_np, box, rc, skin, layout, cap):
    x, cells, ws, mbox = gpu_bin(x_np, box, rc + skin)
    nl = md.NList(x_np.shape[1], cap, layout, half=True)
    md.md_build_neighbors(x, mbox, cells, rc, skin, nl)
    return x, cells, nl, ws, mbox


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("case", ["jittered", "liquid"])
def test_half_list_pairs(orc, layout, case):
    if case == "jittered":
        x_np, box = jittered_lj(6, 21)
    else:
        x_np, _, box, _ = lj_liquid(orc, 10, 22)
    x, cells, nl, ws, mbox = half_list(x_np, box, 2.5, 0.3, layout, 160)
    ref, _ = orc.build_nlist(x_np, box, 2.8)
    want = ref.pairs()
    want = want[want[:, 0] < want[:, 1]]
    assert np.array_equal(gpu_pairs(nl), want)
    cnt = np.bincount(want[:, 0], minlength=x_np.shape[1])
    assert np.array_equal(nl.numneigh.cpu().numpy(), cnt)
    # the status word still reports the full rows' largest count
    assert md.md_nlist_status(nl)[md.MD_ST_MAXNEIGH] == ref.max_count


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("prec", [md.MD_FP64, md.MD_MIXED], ids=["fp64", "mixed"])
def test_half_list_lj_forces(orc, layout, prec):
    x_np, _, box, _ = lj_liquid(orc, 10, 23)
    x, cells, nl, ws, mbox = half_list(x_np, box, 2.5, 0.3, layout, 160)
    pot = md.lj_potential(2.5, 1.0, 1.0, 1)
    f, ev = forces_gpu(pot, x, mbox, nl, prec, md.MD_KERNEL_AUTO, ws)
    onl, oc = orc.build_nlist(x_np, box, 2.8)
    ref = orc.lj_forces(oc.x, box, onl, 2.5, shift=1)
    if prec == md.MD_FP64:
        assert_fp64(f, ref.f)
        assert ev[0] == pytest.approx(ref.energy, rel=1e-12)
        assert rel(ev[1:], ref.virial) < 1e-12
    else:
        print(f"half-list mixed LJ force rel-RMS {rel(f, ref.f):.3e}")
        mag = MB.lj_magnitudes(oc.x, box, onl, 2.5, 1.0, 1.0)
        MB.assert_vector(f, ref.f, mag["f"], what="force")
        MB.assert_total(ev[0], ref.energy, mag["e"], what="energy")
    # Newton's third law exactly per pair: the total force is zero up to
    # the rounding of the atomic sums
    assert np.abs(f.sum(axis=1)).max() < 1e-9 * np.abs(f).max() * np.sqrt(x_np.shape[1])


def test_half_list_unsupported_uses():
    x_np, box = sc_solid(5, 24)
    x, cells, nl, ws, mbox = half_list(x_np, box, 7.22, 1.0, 1, 260)
    pot = md.sc_potential(7.22, SC_KW["eps"], SC_KW["a"], SC_KW["c"], 9, 6)
    f = torch.zeros(3, x_np.shape[1], dtype=torch.float64, device="cuda")
    with pytest.raises(md.MDError) as e:
        md.md_compute_forces(pot, x, mbox, nl, md.MD_FP64, md.MD_KERNEL_AUTO, 0, f, None, ws)
    assert e.value.code == md.MD_ERR_UNSUPPORTED
    u = torch.zeros_like(f)
    with pytest.raises(md.MDError) as e:
        md.md_force_vjp(md.lj_potential(2.5), x, mbox, nl, md.MD_FP64, u, f, None, ws)
    assert e.value.code == md.MD_ERR_UNSUPPORTED
