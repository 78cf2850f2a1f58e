"""LJ force adjoint through torch autograd, and the force-matching fit it
serves: (eps, sigma) recovered from forces the oracle computed at the target
parameters."""
import numpy as np
import pytest
import torch

import mixed_bounds as MB
from gpu_helpers import assert_fp64, dev, gpu_list, lj_liquid, rel
from paper_1009_4330_amd import autograd as AG
from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd import md

pytestmark = pytest.mark.gpu


def test_autograd_gradients_match_oracle_vjp(orc):
    """d(sum u . F)/d(x, eps, sigma) through LJForces.backward against the
    oracle's VJP of the same list (FP64 bars of the VJP parity test)."""
    x_np, _, box, _ = lj_liquid(orc, 10, 61)
    n = x_np.shape[1]
    u_np = I.random_unit_vectors(n, 62)
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 2.5, 0.3, 4, 160)
    xg = x.clone().requires_grad_(True)
    eps = torch.tensor(1.1, dtype=torch.float64, device="cuda", requires_grad=True)
    sig = torch.tensor(1.05, dtype=torch.float64, device="cuda", requires_grad=True)
    f = AG.lj_forces(xg, eps, sig, mbox, nl, 2.5, md.MD_FP64, ws)
    (f * dev(u_np)).sum().backward()
    onl, ocells = orc.build_nlist(x_np, box, 2.8)
    rgx, rgp = orc.lj_vjp(ocells.x, box, onl, 2.5, 1.1, 1.05, u_np)
    assert_fp64(xg.grad.cpu().numpy(), rgx, what="gx")
    mag = MB.lj_magnitudes(ocells.x, box, onl, 2.5, 1.1, 1.05, u_np)
    MB.assert_total(eps.grad.item(), rgp[0], mag["geps"], u=MB.U64, what="dL/deps")
    MB.assert_total(sig.grad.item(), rgp[1], mag["gsig"], u=MB.U64, what="dL/dsigma")


@pytest.mark.parametrize("lanes", [1, 2, 8, 16, 32, 64])
def test_vjp_every_layout_against_oracle(orc, lanes):
    """md_force_vjp on lists in every layout K against the oracle's VJP (FP64
    bars): the workgroups leave their partial sums of the parameter
    gradients in rows whose number grows with K (n K / 256 of them)."""
    x_np, _, box, _ = lj_liquid(orc, 6, 63)
    n = x_np.shape[1]
    u_np = I.random_unit_vectors(n, 64)
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 2.5, 0.3, lanes, 160)
    pot = md.lj_potential(2.5, 1.1, 1.05, 0)
    gx = torch.zeros(3, n, dtype=torch.float64, device="cuda")
    gp = torch.zeros(2, dtype=torch.float64, device="cuda")
    md.md_force_vjp(pot, x, mbox, nl, md.MD_FP64, dev(u_np), gx, gp, ws)
    onl, ocells = orc.build_nlist(x_np, box, 2.8)
    rgx, rgp = orc.lj_vjp(ocells.x, box, onl, 2.5, 1.1, 1.05, u_np)
    assert_fp64(gx.cpu().numpy(), rgx, what="gx")
    mag = MB.lj_magnitudes(ocells.x, box, onl, 2.5, 1.1, 1.05, u_np)
    gp = gp.cpu().numpy()
    MB.assert_total(gp[0], rgp[0], mag["geps"], u=MB.U64, what="dL/deps")
    MB.assert_total(gp[1], rgp[1], mag["gsig"], u=MB.U64, what="dL/dsigma")


@pytest.mark.parametrize("prec", [md.MD_FP64, md.MD_MIXED], ids=["fp64", "mixed"])
def test_force_matching_fit_recovers_parameters(orc, prec):
    """Mean squared force error against the oracle's forces at (1.1, 1.05),
    minimised over (eps, sigma) from (1, 1) by L-BFGS on the library's forces
    and adjoint.  The pair set does not depend on the parameters (absolute
    cutoff), so the minimum is exact at the target."""
    x_np, _, box, _ = lj_liquid(orc, 10, 63)
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 2.5, 0.3, 4, 160)
    onl, ocells = orc.build_nlist(x_np, box, 2.8)
    target = dev(orc.lj_forces(ocells.x, box, onl, 2.5, eps=I.FM_TARGET[0],
                               sigma=I.FM_TARGET[1]).f)
    eps = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    sig = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    opt = torch.optim.LBFGS([eps, sig], lr=1.0, max_iter=60, tolerance_grad=1e-15,
                            tolerance_change=1e-18, history_size=10,
                            line_search_fn="strong_wolfe")

    def closure():
        opt.zero_grad()
        f = AG.lj_forces(x, eps, sig, mbox, nl, 2.5, prec, ws)
        loss = ((f - target) ** 2).mean()
        loss.backward()
        return loss

    for _ in range(3):
        loss = opt.step(closure)
    got = (eps.item(), sig.item())
    print(f"fit ({'fp64' if prec == md.MD_FP64 else 'mixed'}): eps {got[0]:.12f} "
          f"sigma {got[1]:.12f} loss {loss.item():.3e}")
    # FP64 reaches the target to rounding; MIXED to the FP32 pair function's accuracy
    tol = 1e-9 if prec == md.MD_FP64 else 2e-6
    assert abs(got[0] - I.FM_TARGET[0]) < tol
    assert abs(got[1] - I.FM_TARGET[1]) < tol
