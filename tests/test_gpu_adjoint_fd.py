"""The LJ adjoint against finite differences of the library's own FP64
forces, and the force-matching workload at its full size.

md_force_vjp returns gx = (dF/dx)^T u and dL/d(eps, sigma) for
L = sum_i u_i . F_i.  Central differences (h = 1e-5) of L over the same
frozen list check both: per coordinate of sampled atoms none of whose listed
pairs lies within 1e-4 of the cutoff (so the h-step moves no pair across it),
and per parameter.  torch.autograd.gradcheck exercises LJForces on a
256-atom box.  The eight 32,000-atom force-matching snapshots are thermalised
by the oracle's own NVE runs; targets are the oracle's forces at the target
parameters."""
import numpy as np
import pytest
import torch

from gpu_helpers import dev, gpu_list, lj_liquid, rel
from paper_1009_4330_amd import autograd as AG
from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd import md

pytestmark = pytest.mark.gpu

H = 1e-5


def pair_margin(orc, x_np, box, rc, rl):
    """Per atom: the smallest |r_ij - rc| over its listed pairs (oracle geometry)."""
    onl, oc = orc.build_nlist(x_np, box, rl)
    p = onl.pairs()
    L = np.asarray(box)[:, None]
    d = oc.x[:, p[:, 0]] - oc.x[:, p[:, 1]]
    d -= L * np.rint(d / L)
    gap = np.abs(np.sqrt((d * d).sum(0)) - rc)
    out = np.full(x_np.shape[1], np.inf)
    np.minimum.at(out, p[:, 0], gap)
    np.minimum.at(out, p[:, 1], gap)
    return out


def loss(pot, x, mbox, nl, u, ws):
    f = torch.empty_like(x)
    md.md_compute_forces(pot, x, mbox, nl, md.MD_FP64, md.MD_KERNEL_AUTO, 0, f, None, ws)
    return float((f * u).sum().item())


def test_vjp_matches_central_differences(orc):
    x_np, _, box, _ = lj_liquid(orc, 8, 71)
    n = x_np.shape[1]
    u_np = I.random_unit_vectors(n, 72)
    eps, sig, rc = 1.1, 1.05, 2.5
    x, cells, nl, ws, mbox = gpu_list(x_np, box, rc, 0.3, 4, 160)
    u = dev(u_np)
    pot = md.lj_potential(rc, eps, sig, 0)
    gx = torch.zeros(3, n, dtype=torch.float64, device="cuda")
    gp = torch.zeros(2, dtype=torch.float64, device="cuda")
    md.md_force_vjp(pot, x, mbox, nl, md.MD_FP64, u, gx, gp, ws)
    gx, gp = gx.cpu().numpy(), gp.cpu().numpy()
    # x on the device is wrapped by the binning; perturb that copy
    margin = pair_margin(orc, x_np, box, rc, rc + 0.3)
    atoms = np.flatnonzero(margin > 1e-4)[:24]
    assert len(atoms) == 24
    fd, an = [], []
    for a in atoms:
        for d in range(3):
            xp = x.clone()
            xp[d, a] += H
            xm = x.clone()
            xm[d, a] -= H
            fd.append((loss(pot, xp, mbox, nl, u, ws) - loss(pot, xm, mbox, nl, u, ws)) / (2 * H))
            an.append(gx[d, a])
    err = rel(an, fd)
    print(f"[fd] position VJP vs central differences: {err:.3e} over {len(fd)} coordinates")
    assert err < 1e-6
    # parameters: no pair crosses rc when eps or sigma moves
    for k, (pe, ps) in enumerate(((eps + H, sig), (eps, sig + H))):
        pm = (2 * eps - pe, 2 * sig - ps)
        lp = loss(md.lj_potential(rc, pe, ps, 0), x, mbox, nl, u, ws)
        lm = loss(md.lj_potential(rc, pm[0], pm[1], 0), x, mbox, nl, u, ws)
        g = (lp - lm) / (2 * H)
        print(f"[fd] dL/d{'eps' if k == 0 else 'sigma'}: adjoint {gp[k]:.12e} fd {g:.12e}")
        assert abs(gp[k] - g) <= 1e-6 * abs(g)


def test_gradcheck_256_atoms(orc):
    """torch.autograd.gradcheck of F(x, eps, sigma) on a 256-atom FP64 box
    (fcc 4^3 jittered; the seed is the first whose listed pairs all stay
    farther than 1e-5 from the cutoff, found with the oracle's geometry)."""
    box = (4 * I.A_LJ,) * 3
    for seed in range(1, 50):
        x_np = I.jitter(I.fcc_positions(4, I.A_LJ), 0.2, seed)
        if pair_margin(orc, x_np, box, 2.5, 2.8).min() > 1e-5:
            break
    x, cells, nl, ws, mbox = gpu_list(x_np, box, 2.5, 0.3, 1, 160)
    xg = x.clone().requires_grad_(True)
    eps = torch.tensor(1.1, dtype=torch.float64, device="cuda", requires_grad=True)
    sig = torch.tensor(1.05, dtype=torch.float64, device="cuda", requires_grad=True)

    def f(xx, e, s):
        return AG.lj_forces(xx, e, s, mbox, nl, 2.5, md.MD_FP64, ws)

    assert torch.autograd.gradcheck(f, (xg, eps, sig), eps=1e-6, atol=1e-6, rtol=1e-6)


_SNAPS = {}


def fm_snapshots(orc):
    """The eight thermalised 32k snapshots (oracle NVE runs from the seeded
    lattices) and the oracle's target forces at (1.1, 1.05) on each (made
    once per session)."""
    w = I.LJ_FM_32K
    if "fm" in _SNAPS:
        return w, _SNAPS["fm"]
    out = []
    for seed in I.FM_SEEDS:
        x, v, box = I.initial_state(w, seed)
        res = orc.md_run(orc.params_for(w), x, v, box, w.steps, w.steps)
        onl, oc = orc.build_nlist(res.x, box, w.rc + w.skin)
        tgt = orc.lj_forces(oc.x, box, onl, w.rc, eps=I.FM_TARGET[0], sigma=I.FM_TARGET[1]).f
        out.append((res.x, tgt))
    _SNAPS["fm"] = out
    return w, out


@pytest.mark.parametrize("prec", [md.MD_FP64, md.MD_MIXED], ids=["fp64", "mixed"])
def test_force_matching_8x32k(orc, prec):
    """Loss = mean squared force error over the eight snapshots, minimised
    over (eps, sigma) from (1, 1) by L-BFGS with the library's forces and
    adjoint; on the first snapshot the loss gradient at (1, 1) is checked
    against central differences of the FP64 loss."""
    print(f"[c5] eight 32k snapshots from the oracle", flush=True)
    w, snaps = fm_snapshots(orc)
    sys = []
    for xs, tgt in snaps:
        x, cells, nl, ws, mbox = gpu_list(xs, w.box, w.rc, w.skin, 4, 160)
        sys.append((x, nl, ws, mbox, dev(tgt)))

    def total(e, s, p=prec):
        out = 0.0
        for x, nl, ws, mbox, tgt in sys:
            out = out + ((AG.lj_forces(x, e, s, mbox, nl, w.rc, p, ws) - tgt) ** 2).mean()
        return out

    if prec == md.MD_FP64:
        x, nl, ws, mbox, tgt = sys[0]
        e = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
        s = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
        one = ((AG.lj_forces(x, e, s, mbox, nl, w.rc, prec, ws) - tgt) ** 2).mean()
        one.backward()

        def lval(ev, sv):
            with torch.no_grad():
                ee = torch.tensor(ev, dtype=torch.float64, device="cuda")
                ss = torch.tensor(sv, dtype=torch.float64, device="cuda")
                return float(((AG.lj_forces(x, ee, ss, mbox, nl, w.rc, prec, ws) - tgt) ** 2)
                             .mean().item())

        ge = (lval(1 + H, 1.0) - lval(1 - H, 1.0)) / (2 * H)
        gs = (lval(1.0, 1 + H) - lval(1.0, 1 - H)) / (2 * H)
        print(f"[c5] gradient at (1, 1): adjoint ({e.grad.item():.10e}, {s.grad.item():.10e}) "
              f"fd ({ge:.10e}, {gs:.10e})")
        assert abs(e.grad.item() - ge) <= 1e-6 * abs(ge)
        assert abs(s.grad.item() - gs) <= 1e-6 * abs(gs)
    eps = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    sig = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    opt = torch.optim.LBFGS([eps, sig], lr=1.0, max_iter=60, tolerance_grad=1e-15,
                            tolerance_change=1e-18, history_size=10,
                            line_search_fn="strong_wolfe")

    def closure():
        opt.zero_grad()
        l_ = total(eps, sig)
        l_.backward()
        return l_

    for _ in range(3):
        l_ = opt.step(closure)
    got = (eps.item(), sig.item())
    print(f"[c5] fit: eps {got[0]:.12f} sigma {got[1]:.12f} loss {float(l_):.3e}")
    tol = 1e-9 if prec == md.MD_FP64 else 2e-6
    assert abs(got[0] - I.FM_TARGET[0]) < tol
    assert abs(got[1] - I.FM_TARGET[1]) < tol
