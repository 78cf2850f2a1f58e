"""Throughput of the MD hot path on one MI355X.

Headline: atom-timesteps/s of the 256,000-atom LJ melt (fcc 40^3 at reduced
density 0.8442, rc 2.5, skin 0.3, T* 3.0, dt 0.005), 1,000 NVE steps (more if
--steps asks for more, never fewer: the workload is defined as a 1,000-step
run), in FP32-mixed precision with the force kernel the setup mini-benchmark
picks (K lanes per atom).  The plain FP64 path and the thread-per-atom kernel
(K = 1) on the same workload, and the LJ adjoint (force VJP) throughput in
atoms/s on eight 32,000-atom snapshots thermalised for 500 NVE steps, are
reported beside it; each of those extras is guarded so that its failure
cannot suppress the headline line.

Each "step" is one full velocity-Verlet step of md_step: the rebuild chain
when the half-skin check fired (sort, list), then the force
kernel, which also does the closing kick, the next kick, drift and check;
thermo output every min(100, steps) steps.  Inputs are resident in HBM before
the timed region starts.  The roofline object describes that force kernel
(its duration from events recorded inside its own dispatches) and, as
step_frac, the whole step.  The cpu_baseline leg times the oracle on the host
cores and checks the final state's forces against it.  Prints one JSON line on
stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth
THERMO_EVERY = 100
HEADLINE_STEPS = 1000          # the 256k melt is defined as a 1,000-step NVE run


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def force_bytes_per_atom(mean_neigh: float) -> float:
    """Algorithmic HBM bytes per atom of md_step's force kernel, which also
    integrates.  Force part: numneigh (4), the neighbour indices (4 per
    entry), x_i (24) and f_i (24); the neighbour positions are cache-served
    gathers (atoms are cell-sorted).  Fused integration (the closing kick of
    one step with the kick, drift and check of the next): x, v, f and x_ref
    read, x and v written, 144."""
    return 4.0 + 4.0 * mean_neigh + 24.0 + 24.0 + 144.0


def rebuild_bytes_per_atom(mean_neigh: float) -> float:
    """Algorithmic bytes per atom of one rebuild: binning and the permutation
    of the state (about 132), then the list build (x 24, the count 4, the
    entries 4 per neighbour, x_ref 24)."""
    return 132.0 + 24.0 + 4.0 + 4.0 * mean_neigh + 24.0


def step_bytes_per_atom(mean_neigh: float, rebuilds: int, steps: int) -> float:
    """Algorithmic bytes per atom-step of the whole fused step: the force
    kernel with its integration plus the rebuilds amortised over the run."""
    return force_bytes_per_atom(mean_neigh) + rebuild_bytes_per_atom(mean_neigh) * rebuilds / max(
        steps, 1)


def source_hash() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1009_4330_amd", "csrc", "md_forces.hip"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_name: str, launches_bytes: float):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current force-kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "force_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash():
        return None
    k = d.get("kernels", {}).get(kernel_name)
    return None if k is None else k.get("bytes_per_launch")


def run_md(w, x, v, prec, kernel, steps, warmup, nvt=None, thermo_every=THERMO_EVERY, npt=None):
    import torch
    from paper_1009_4330_amd import md
    from paper_1009_4330_amd.system import MDSystem

    sysm = MDSystem(w, x, v, prec, kernel, nvt=nvt, npt=npt)
    sysm.setup(thermo=False)
    every = max(1, min(thermo_every, steps))
    if warmup:
        sysm.run(warmup, every)
    torch.cuda.synchronize()
    md.md_timing_enable(10)
    builds0 = md.md_nlist_status(sysm.nl)[md.MD_ST_BUILDS]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rows = sysm.run(steps, every)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches, ms = md.md_timing_read()
    md.md_timing_enable(0)
    words = md.md_nlist_status(sysm.nl)
    nn = sysm.nl.numneigh.double().mean().item()
    return dict(elapsed=elapsed, rows=rows, force_launches=launches,
                force_ms_avg=ms / max(launches, 1), rebuilds=words[md.MD_ST_BUILDS] - builds0,
                mean_neigh=nn, max_neigh=words[md.MD_ST_MAXNEIGH], n=w.natoms,
                kernel=sysm.kernel, system=sysm, thermo_every=every)


def nve_drift(rows, n: int, dt: float):
    """Total-energy drift over the thermo rows of a timed run: largest
    |E - E0| / |E0| and the least-squares slope of E/N per time unit.  None
    below two rows (no drift is defined)."""
    rows = np.asarray(rows, dtype=np.float64)
    if rows.ndim != 2 or rows.shape[0] < 2:
        return None
    e = rows[:, 3]
    t = rows[:, 0] * dt
    slope = float(np.polyfit(t, e / n, 1)[0])
    return {"max_rel": float(np.max(np.abs(e - e[0])) / abs(e[0])), "slope_per_tau": slope,
            "rows": int(len(e)), "first_step": int(rows[0, 0]), "last_step": int(rows[-1, 0])}


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count(), "model": model}


def bench_vjp(reps: int):
    """Force-VJP atoms/s on the eight thermalised 32k-atom snapshots, each
    list in the layout the mini-benchmark picks (K = 4 here; thread per atom
    leaves a 32k system at 500 wavefronts, 0.72e9 atoms/s)."""
    import torch
    from paper_1009_4330_amd import inputs as I
    from paper_1009_4330_amd import md
    from paper_1009_4330_amd.system import MDSystem

    w = I.LJ_FM_32K
    out = {}
    for prec_name, prec in (("mixed", md.MD_MIXED), ("fp64", md.MD_FP64)):
        total_t, total_atoms = 0.0, 0
        for seed in I.FM_SEEDS:
            x, v, box = I.initial_state(w, seed)
            s = MDSystem(w, x, v, "fp64", "auto")
            s.setup(thermo=False)
            s.run(w.steps, w.steps)
            n = w.natoms
            u = torch.randn(3, n, dtype=torch.float64, device="cuda",
                            generator=torch.Generator(device="cuda").manual_seed(seed))
            gx = torch.empty_like(u)
            gp = torch.empty(2, dtype=torch.float64, device="cuda")
            pot = md.lj_potential(w.rc, I.FM_TARGET[0], I.FM_TARGET[1], 0)
            md.md_force_vjp(pot, s.state.x, s.box, s.nl, prec, u, gx, gp, s.ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                md.md_force_vjp(pot, s.state.x, s.box, s.nl, prec, u, gx, gp, s.ws)
            torch.cuda.synchronize()
            total_t += time.perf_counter() - t0
            total_atoms += n * reps
        out[prec_name] = total_atoms / total_t
    return out


def bench_sc_vjp(reps: int):
    """Sutton-Chen force-VJP atoms/s (three passes, positions and (eps, a, c))
    on the 500k-atom copper-like solid after its setup."""
    import torch
    from paper_1009_4330_amd import inputs as I
    from paper_1009_4330_amd import md
    from paper_1009_4330_amd.system import MDSystem

    w = I.SC_500K
    x, v, _ = I.initial_state(w)
    s = MDSystem(w, x, v, "fp64", "auto")
    s.setup(thermo=False)
    n = w.natoms
    u = torch.randn(3, n, dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(5))
    gx = torch.empty_like(u)
    gp = torch.empty(3, dtype=torch.float64, device="cuda")
    out = {"lanes_per_atom": s.nl.layout}
    for prec_name, prec in (("mixed", md.MD_MIXED), ("fp64", md.MD_FP64)):
        md.md_force_vjp(s.pot, s.state.x, s.box, s.nl, prec, u, gx, gp, s.ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            md.md_force_vjp(s.pot, s.state.x, s.box, s.nl, prec, u, gx, gp, s.ws)
        torch.cuda.synchronize()
        out[prec_name] = n * reps / (time.perf_counter() - t0)
    return out


def bench_half_list(reps: int = 20):
    """Force-kernel time (md_compute_forces, no energy) from full and half
    lists on the 256k LJ melt after 200 steps, per lanes-per-atom layout."""
    import math
    import torch
    from paper_1009_4330_amd import inputs as I
    from paper_1009_4330_amd import md
    from paper_1009_4330_amd.system import MDSystem

    w = I.LJ_256K
    x, v, _ = I.initial_state(w)
    s = MDSystem(w, x, v, "mixed", "k4")
    s.setup(thermo=False)
    s.run(200, 200)
    xs = s.state.x.clone()
    n = w.natoms
    box = md.make_box(w.box)
    rl = w.rc + w.skin
    ncell = int(np.prod([math.floor(L / rl) for L in w.box]))
    cells = md.Cells(n, ncell)
    ws = md.workspace(n, box, rl)
    md.md_bin_cells(xs, box, rl, cells, ws)
    pot = md.lj_potential(w.rc, 1.0, 1.0, 1)
    f = torch.empty(3, n, dtype=torch.float64, device="cuda")
    out = {}
    for half in (False, True):
        for k in (1, 4, 64):
            nl = md.NList(n, 160, k, half=half)
            md.md_build_neighbors(xs, box, cells, w.rc, w.skin, nl)
            for prec_name, prec in (("mixed", md.MD_MIXED), ("fp64", md.MD_FP64)):
                md.md_compute_forces(pot, xs, box, nl, prec, md.MD_KERNEL_AUTO, 0, f, None, ws)
                torch.cuda.synchronize()
                md.md_timing_enable(1)
                for _ in range(reps):
                    md.md_compute_forces(pot, xs, box, nl, prec, md.MD_KERNEL_AUTO, 0, f, None,
                                         ws)
                launches, ms = md.md_timing_read()
                md.md_timing_enable(0)
                key = f"{'half' if half else 'full'}_k{k}_{prec_name}_us"
                out[key] = 1e3 * ms / max(launches, 1)
    return out


def cpu_baseline(w, x, v, target_s: float = 15.0):
    """The oracle's own NVE run on the host cores, on a bounded number of
    steps of the same workload; setup (first build + forces) is subtracted.
    Returns the report and the oracle's final state (positions, forces)."""
    import oracle
    p = oracle.params_for(w)
    t0 = time.perf_counter()
    oracle.md_run(p, x, v, w.box, 0, 1)
    t_setup = time.perf_counter() - t0
    probe = 5
    t0 = time.perf_counter()
    oracle.md_run(p, x, v, w.box, probe, probe)
    per_step = max((time.perf_counter() - t0 - t_setup) / probe, 1e-4)
    steps = int(max(probe, min(400, target_s / per_step)))
    t0 = time.perf_counter()
    res = oracle.md_run(p, x, v, w.box, steps, steps)
    t = time.perf_counter() - t0 - t_setup
    return dict(value=steps * w.natoms / t, unit="atom-timesteps/s", cores=oracle.num_threads(),
                kind="oracle",
                sample=f"{steps} NVE steps of the {w.natoms}-atom LJ melt from the same seeded "
                       f"state (FP64, setup excluded, {t:.1f} s)"), res


def oracle_force_check(w, ores, kernel: int):
    """Forces at the end of the oracle's own timed run: the library's MIXED
    and FP64 forces (md_compute_forces on a list it builds from the oracle's
    positions, in the headline run's lanes-per-atom layout) against the
    oracle's FP64 forces there.  rel-RMS over all 3N components and the
    largest per-atom error relative to the largest force."""
    import math
    import torch
    from paper_1009_4330_amd import md
    n = w.natoms
    rl = w.rc + w.skin
    x = torch.as_tensor(ores.x, dtype=torch.float64, device="cuda").contiguous()
    box = md.make_box(w.box)
    cells = md.Cells(n, int(np.prod([math.floor(L / rl) for L in w.box])))
    ws = md.workspace(n, box, rl)
    md.md_bin_cells(x, box, rl, cells, ws)
    nl = md.NList(n, 160, kernel)
    md.md_build_neighbors(x, box, cells, w.rc, w.skin, nl)
    pot = md.lj_potential(w.rc, w.lj_eps, w.lj_sigma, w.lj_shift)
    ref = ores.f
    out = {"state": "end of the oracle's timed run"}
    for name, prec in (("mixed", md.MD_MIXED), ("fp64", md.MD_FP64)):
        f = torch.empty_like(x)
        md.md_compute_forces(pot, x, box, nl, prec, md.MD_KERNEL_AUTO, 0, f, None, ws)
        f = f.cpu().numpy()
        d = f - ref
        out[f"{name}_force_rel_rms_vs_oracle"] = float(np.linalg.norm(d) / np.linalg.norm(ref))
        out[f"{name}_force_max_atom_err_rel"] = float(
            np.sqrt((d * d).sum(0)).max() / np.sqrt((ref * ref).sum(0)).max())
    out["atoms"] = n
    return out


def profile_force(steps: int, kernel: str):
    """For hardware-counter passes: the headline state after a short warm-up,
    then `steps` md_step steps (their force kernels are the fused ones the
    bench times), then a plain device copy of known size (256 MiB read + 256
    MiB written, 4 times) that calibrates the byte counters."""
    import torch
    from paper_1009_4330_amd import inputs as I
    from paper_1009_4330_amd.system import MDSystem

    w = I.LJ_256K
    x, v, _ = I.initial_state(w)
    s = MDSystem(w, x, v, "mixed", kernel)
    s.setup(thermo=False)
    s.run(20, 20)
    torch.cuda.synchronize()
    s.run(steps, steps)
    torch.cuda.synchronize()
    nbytes = 256 << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"steps": steps, "atoms": w.natoms,
                      "mean_neighbors": s.nl.numneigh.double().mean().item(),
                      "lanes_per_atom": s.nl.layout, "copy_bytes_read": nbytes,
                      "copy_bytes_written": nbytes, "copy_launches": 4}), flush=True)


def copy_peak(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Device-to-device copy bandwidth (read + write bytes / s) of a plain
    torch copy: the measured stream peak the roofline is also compared with."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    return 2.0 * nbytes * reps / (time.perf_counter() - t0) / 1e9


def fit_timing(iters: int = 3):
    """Force matching on the eight thermalised 32k snapshots (sum of the mean
    squared force errors): L-BFGS over (eps, sigma) from (1, 1) towards forces
    generated at the target parameters; wall time of the fit."""
    import torch
    from paper_1009_4330_amd import autograd as AG
    from paper_1009_4330_amd import inputs as I
    from paper_1009_4330_amd import md
    from paper_1009_4330_amd.system import MDSystem

    w = I.LJ_FM_32K
    snaps = []
    for seed in I.FM_SEEDS:
        x, v, box = I.initial_state(w, seed)
        s = MDSystem(w, x, v, "fp64", "auto")
        s.setup(thermo=False)
        s.run(w.steps, w.steps)
        pot = md.lj_potential(w.rc, I.FM_TARGET[0], I.FM_TARGET[1], 0)
        f = torch.empty_like(s.state.f)
        md.md_compute_forces(pot, s.state.x, s.box, s.nl, md.MD_FP64, md.MD_KERNEL_AUTO, 0, f,
                             None, s.ws)
        snaps.append((s, f))
    out = {}
    for prec_name, prec in (("mixed", md.MD_MIXED), ("fp64", md.MD_FP64)):
        eps = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
        sig = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
        opt = torch.optim.LBFGS([eps, sig], lr=1.0, max_iter=60, tolerance_grad=1e-15,
                                tolerance_change=1e-18, line_search_fn="strong_wolfe")
        calls = [0]

        def closure():
            opt.zero_grad()
            loss = 0.0
            for s, target in snaps:
                f = AG.lj_forces(s.state.x, eps, sig, s.box, s.nl, w.rc, prec, s.ws)
                loss = loss + ((f - target) ** 2).mean()
            loss.backward()
            calls[0] += 1
            return loss

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(iters):
            loss = opt.step(closure)
        torch.cuda.synchronize()
        out[prec_name] = dict(seconds=time.perf_counter() - t0, evaluations=calls[0],
                              eps=eps.item(), sigma=sig.item(), loss=float(loss))
    return out


def oracle_one_thread(w, x, v, steps: int = 10):
    """The oracle at one host thread, in a child process (OMP_NUM_THREADS=1)."""
    import subprocess
    code = ("import sys, time, numpy as np; sys.path.insert(0, %r); import oracle; "
            "from paper_1009_4330_amd import inputs as I; w = I.WORKLOADS[%r]; "
            "x, v, _ = I.initial_state(w); p = oracle.params_for(w); "
            "t0 = time.perf_counter(); oracle.md_run(p, x, v, w.box, 0, 1); ts = time.perf_counter() - t0; "
            "t0 = time.perf_counter(); oracle.md_run(p, x, v, w.box, %d, %d); t = time.perf_counter() - t0 - ts; "
            "print(%d * w.natoms / t, oracle.num_threads())") % (ROOT, w.name, steps, steps, steps)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=600)
    rate, threads = res.stdout.split()
    return dict(value=float(rate), unit="atom-timesteps/s", cores=int(threads), kind="oracle",
                sample=f"{steps} NVE steps of {w.name}, setup excluded")


def suite(steps: int):
    """The other configurations of the measurement plan; one JSON line each."""
    import torch
    from paper_1009_4330_amd import inputs as I

    def emit(d):
        print(json.dumps(d), flush=True)

    emit({"item": "copy_peak_GBps", "value": copy_peak()})
    w = I.LJ_HI_108K
    x, v, _ = I.initial_state(w)
    for prec in ("fp64", "mixed"):
        for kern in ("tpa", "wpa", "auto"):
            r = run_md(w, x, v, prec, kern, steps, 10)
            emit({"item": "C3", "workload": w.name, "precision": prec, "kernel": kern,
                  "lanes_per_atom": r["kernel"], "atom_steps_per_s": steps * w.natoms / r["elapsed"],
                  "force_us": 1e3 * r["force_ms_avg"], "rebuilds": r["rebuilds"],
                  "mean_neighbors": r["mean_neigh"], "steps": steps})
    w = I.SC_500K
    x, v, _ = I.initial_state(w)
    for prec in ("fp64", "mixed"):
        r = run_md(w, x, v, prec, "auto", steps, 10)
        emit({"item": "C4", "workload": w.name, "precision": prec, "kernel": "auto",
              "lanes_per_atom": r["kernel"], "atom_steps_per_s": steps * w.natoms / r["elapsed"],
              "force_us": 1e3 * r["force_ms_avg"], "rebuilds": r["rebuilds"],
              "mean_neighbors": r["mean_neigh"], "steps": steps})
    w = I.BUCK_141K
    x, v, _ = I.initial_state(w)
    for prec in ("fp64", "mixed"):
        r = run_md(w, x, v, prec, "auto", steps, 10)
        emit({"item": "buck_coul", "workload": w.name, "precision": prec, "kernel": "auto",
              "lanes_per_atom": r["kernel"], "atom_steps_per_s": steps * w.natoms / r["elapsed"],
              "force_us": 1e3 * r["force_ms_avg"], "rebuilds": r["rebuilds"],
              "mean_neighbors": r["mean_neigh"], "steps": steps})
    w = I.LJ_256K
    x, v, _ = I.initial_state(w)
    for prec in ("mixed", "fp64"):
        r = run_md(w, x, v, prec, "auto", steps, 10, nvt=(w.temp, 100 * w.dt, 3))
        emit({"item": "nvt", "workload": w.name, "precision": prec, "kernel": "auto",
              "thermostat": "Nose-Hoover chain, 3 links, period 100 dt",
              "lanes_per_atom": r["kernel"], "atom_steps_per_s": steps * w.natoms / r["elapsed"],
              "ms_per_step": 1e3 * r["elapsed"] / steps, "force_us": 1e3 * r["force_ms_avg"],
              "rebuilds": r["rebuilds"], "steps": steps})
    for prec in ("mixed", "fp64"):
        r = run_md(w, x, v, prec, "auto", steps, 10, npt=(w.temp, 100 * w.dt, 3, 2.0, 1000 * w.dt))
        emit({"item": "npt", "workload": w.name, "precision": prec, "kernel": "auto",
              "barostat": "isotropic MTK, Nose-Hoover chains of 3 on particles and barostat, "
                          "P 2.0, periods 100 dt (thermostat) and 1000 dt (barostat)",
              "lanes_per_atom": r["kernel"], "atom_steps_per_s": steps * w.natoms / r["elapsed"],
              "ms_per_step": 1e3 * r["elapsed"] / steps, "force_us": 1e3 * r["force_ms_avg"],
              "rebuilds": r["rebuilds"], "steps": steps})
    emit({"item": "C4_sc_vjp_atoms_per_s", **bench_sc_vjp(20)})
    emit({"item": "half_vs_full_list_force_kernel", "workload": "lj_melt_256k",
          **bench_half_list()})
    emit({"item": "C5_fit", **{k: v for k, v in fit_timing().items()}})
    for nc in (10, 20, 30, 40, 60, 80):
        w = I.scaled(I.LJ_256K, nc)
        x, v, _ = I.initial_state(w)
        r = run_md(w, x, v, "mixed", "auto", steps, 10)
        emit({"item": "sweep", "atoms": w.natoms, "precision": "mixed", "kernel": "auto",
              "lanes_per_atom": r["kernel"], "atom_steps_per_s": steps * w.natoms / r["elapsed"],
              "force_us": 1e3 * r["force_ms_avg"], "rebuilds": r["rebuilds"], "steps": steps})
    w = I.LJ_256K
    x, v, _ = I.initial_state(w)
    emit({"item": "oracle_one_thread", **oracle_one_thread(w, x, v)})


def one_workload(name: str, kernel: str, steps: int, warmup: int, nvt: bool = False,
                 npt: bool = False):
    """Time one named workload in FP64 and FP32-mixed; one JSON line each.
    With nvt, under a Nose-Hoover chain of 3 at the workload's temperature
    with a period of 100 time steps."""
    from paper_1009_4330_amd import inputs as I

    if name not in I.WORKLOADS:
        print(f"unknown workload {name}; one of {sorted(I.WORKLOADS)}", file=sys.stderr)
        sys.exit(2)
    w = I.WORKLOADS[name]
    x, v, _ = I.initial_state(w)
    for prec in ("fp64", "mixed"):
        log(f"[bench] {w.name}: {w.natoms} atoms, {prec}, kernel {kernel}")
        r = run_md(w, x, v, prec, kernel, steps, warmup,
                   nvt=(w.temp, 100 * w.dt, 3) if nvt and not npt else None,
                   npt=(w.temp, 100 * w.dt, 3, 2.0, 1000 * w.dt) if npt else None)
        print(json.dumps({"item": "workload", "workload": w.name, "precision": prec,
                          "ensemble": "npt" if npt else ("nvt" if nvt else "nve"),
                          "kernel": kernel, "lanes_per_atom": r["kernel"],
                          "atom_steps_per_s": steps * w.natoms / r["elapsed"],
                          "ms_per_step": 1e3 * r["elapsed"] / steps,
                          "force_us": 1e3 * r["force_ms_avg"], "rebuilds": r["rebuilds"],
                          "mean_neighbors": r["mean_neigh"], "steps": steps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="time only the headline configuration")
    ap.add_argument("--kernel", default="auto",
                    help="force kernel: tpa, wpa, auto or kN (N lanes per atom)")
    ap.add_argument("--profile-force", type=int, default=0, metavar="N",
                    help="run N md_step steps and a calibration copy (for counters)")
    ap.add_argument("--workload", default="",
                    help="time one other workload by name (e.g. buck_coul_141k, sc_cu_500k) in "
                         "both precisions with --kernel; one JSON line per precision")
    ap.add_argument("--nvt", action="store_true",
                    help="with --workload: run under the Nose-Hoover chain thermostat")
    ap.add_argument("--npt", action="store_true",
                    help="with --workload: run under the barostat (P 2.0, LJ units)")
    ap.add_argument("--suite", action="store_true",
                    help="the other configurations (rc 5.0 LJ, Sutton-Chen, Buckingham + Coulomb, "
                         "the force-matching fit, a size sweep, copy peak, one-thread oracle); "
                         "JSON lines")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.profile_force:
        profile_force(args.profile_force, args.kernel)
        return
    if args.suite:
        suite(args.steps if args.steps != 1000 else 200)
        return
    if args.workload:
        one_workload(args.workload, args.kernel, args.steps if args.steps != 1000 else 200,
                     args.warmup, args.nvt, args.npt)
        return
    headline(args)


def guarded(name: str, fn, *a, **kw):
    """Run one extra measurement; a failure there is logged and reported as
    an error string, never allowed to suppress the headline line."""
    try:
        return fn(*a, **kw)
    except Exception as e:  # noqa: BLE001 -- any failure of an extra is reported, not raised
        log(f"[bench] {name} failed: {type(e).__name__}: {e}")
        return {"error": f"{type(e).__name__}: {e}"}


def headline(args):
    """The 256k LJ melt, 1,000 NVE steps (or more when --steps asks for more),
    FP32-mixed; FP64 and thread-per-atom runs, the adjoint, the step-level
    roofline and the oracle (timing and force check) beside it."""
    import torch
    from paper_1009_4330_amd import inputs as I

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    w = I.LJ_256K
    steps = max(args.steps, HEADLINE_STEPS)
    x, v, _ = I.initial_state(w)
    log(f"[bench] {w.name}: {w.natoms} atoms, mixed precision, kernel {args.kernel}, "
        f"{steps} timed steps after {args.warmup} warm-up steps")
    mixed = run_md(w, x, v, "mixed", args.kernel, steps, args.warmup)
    value = steps * w.natoms / mixed["elapsed"]
    lanes = mixed["kernel"]
    log(f"[bench] mixed K={lanes}: {value:.4g} atom-steps/s, "
        f"{1e3 * mixed['elapsed'] / steps:.4f} ms/step, "
        f"force avg {1e3 * mixed['force_ms_avg']:.2f} us, rebuilds {mixed['rebuilds']}")

    nn = mixed["mean_neigh"]
    bpa = force_bytes_per_atom(nn)
    alg_bytes = bpa * w.natoms
    avg_s = mixed["force_ms_avg"] * 1e-3
    achieved = alg_bytes / avg_s / 1e9 if avg_s > 0 else 0.0
    kname = f"k_lj<MIXED, no energy/virial, K={lanes}, fused step>"
    traffic = measured_traffic(kname, alg_bytes)
    b_step = step_bytes_per_atom(nn, mixed["rebuilds"], steps)
    step_gbs = b_step * value / 1e9
    copy_gbs = guarded("copy_peak", copy_peak)
    copy_gbs = copy_gbs if isinstance(copy_gbs, float) else None
    line = {
        "metric": "atom-timesteps/s, LJ 256k atoms FP32-mixed vs FP64; adjoint HVP atoms/s",
        "value": value,
        "unit": "atom-timesteps/s",
        "n_gpus": 1,
        "steps": steps,
        "steps_requested": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * mixed["elapsed"] / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair math, f64 positions/accumulation/integration",
        "data": "synthetic",
        "config": {"workload": "lj_melt_256k", "atoms": w.natoms, "lattice": "fcc 40^3",
                   "density": 0.8442, "rc": w.rc, "skin": w.skin, "dt": w.dt, "temp": w.temp,
                   "ensemble": "nve", "precision": "mixed", "kernel_selection": args.kernel,
                   "lanes_per_atom": lanes, "thermo_every": mixed["thermo_every"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kname, "bytes_per_atom": bpa,
                     "launch_us": 1e3 * mixed["force_ms_avg"],
                     "timed_launches": mixed["force_launches"],
                     "measured_copy_GBps": copy_gbs,
                     "frac_of_measured_copy": achieved / copy_gbs if copy_gbs else None,
                     "step_bytes_per_atom": b_step, "step_achieved": step_gbs,
                     "step_frac": step_gbs / HBM_PEAK_GBS},
        "rebuilds": mixed["rebuilds"],
        "mean_neighbors": nn,
        "nve_drift_mixed": nve_drift(mixed["rows"], w.natoms, w.dt),
    }
    if not args.no_extras:
        fp64 = guarded("fp64 run", run_md, w, x, v, "fp64", args.kernel, steps, args.warmup)
        if "error" not in fp64:
            v64 = steps * w.natoms / fp64["elapsed"]
            log(f"[bench] fp64 K={fp64['kernel']}: {v64:.4g} atom-steps/s, "
                f"force avg {1e3 * fp64['force_ms_avg']:.2f} us")
            line.update({"fp64_atom_timesteps_per_s": v64, "mixed_over_fp64": value / v64,
                         "nve_drift_fp64": nve_drift(fp64["rows"], w.natoms, w.dt),
                         "fp64_force_kernel_us": 1e3 * fp64["force_ms_avg"],
                         "fp64_lanes_per_atom": fp64["kernel"]})
            del fp64
        else:
            line["fp64_run"] = fp64
        tpa = guarded("thread-per-atom run", run_md, w, x, v, "mixed", "tpa", steps, args.warmup)
        if "error" not in tpa:
            vt = steps * w.natoms / tpa["elapsed"]
            log(f"[bench] mixed K=1 (thread per atom): {vt:.4g} atom-steps/s, "
                f"force avg {1e3 * tpa['force_ms_avg']:.2f} us")
            line.update({"mixed_tpa_atom_timesteps_per_s": vt,
                         "mixed_tpa_force_kernel_us": 1e3 * tpa["force_ms_avg"]})
            del tpa
        else:
            line["mixed_tpa_run"] = tpa
        vjp = guarded("adjoint", bench_vjp, reps=100)
        log(f"[bench] vjp atoms/s: {vjp}")
        if "error" not in vjp:
            line.update({"adjoint_hvp_atoms_per_s": vjp["mixed"],
                         "adjoint_hvp_atoms_per_s_fp64": vjp["fp64"]})
        else:
            line["adjoint"] = vjp
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        cbr = guarded("cpu baseline", cpu_baseline, w, x, v)
        if isinstance(cbr, tuple):
            cb, ores = cbr
            cb["host"] = host_info()
            fc = guarded("oracle force check", oracle_force_check, w, ores, lanes)
        else:
            cb, fc = cbr, {"error": "no oracle state"}
        line["cpu_baseline"] = cb
        line["force_check_oracle_state"] = fc
        if "error" not in fc:
            line["mixed_force_rel_rms_vs_oracle"] = fc["mixed_force_rel_rms_vs_oracle"]
        log(f"[bench] force check at the oracle's final state: {fc}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
