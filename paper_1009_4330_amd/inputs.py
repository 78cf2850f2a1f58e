"""Seeded synthetic inputs for the short-range MD path.

This module is the only code shared by the HIP path, its tests and the CPU
oracle.  It builds input *data* (lattice positions, velocity draws, jitter)
and the workload descriptions; it contains none of the method's arithmetic
(no binning, neighbour search, forces or integration).

The workloads stand in for the benchmark systems of the paper's Appendix A
(LJ melt, lj/cut with cutoff 2.5 sigma at density ~0.84; an EAM metal).  The
paper's own input scripts and tabulated EAM file are not available, so every
system is generated here: fcc lattices with Gaussian (Maxwell) velocities drawn
from numpy's PCG64 generator with a fixed seed, zero net momentum, scaled to the
target temperature exactly.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Metal-unit constants (LAMMPS "metal" style: eV, Angstrom, amu, ps, K).
# mvv2e converts amu*A^2/ps^2 to eV; ftm2v converts eV/A/amu to A/ps^2.
METAL_MVV2E = 1.0364269652e-4
METAL_FTM2V = 1.0 / 1.0364269652e-4
METAL_BOLTZ = 8.617333262e-5  # eV/K (CODATA 2018)

FCC_BASIS = ((0.0, 0.0, 0.0), (0.5, 0.5, 0.0), (0.5, 0.0, 0.5), (0.0, 0.5, 0.5))


@dataclasses.dataclass(frozen=True)
class Units:
    """Unit system: ftm2v (force*time/mass -> velocity), mvv2e, Boltzmann."""
    ftm2v: float = 1.0
    mvv2e: float = 1.0
    boltz: float = 1.0


LJ_UNITS = Units()
METAL_UNITS = Units(METAL_FTM2V, METAL_MVV2E, METAL_BOLTZ)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic MD system: lattice, potential and run parameters."""
    name: str
    ncell: int                 # fcc unit cells per box edge
    a: float                   # lattice constant
    potential: str             # "lj" or "sc"
    rc: float
    skin: float
    dt: float
    steps: int
    temp: float
    seed: int
    mass: float = 1.0
    units: Units = LJ_UNITS
    # Lennard-Jones parameters
    lj_eps: float = 1.0
    lj_sigma: float = 1.0
    lj_shift: int = 1          # NVE drift is judged on the shifted energy
    # Sutton-Chen parameters
    sc_eps: float = 0.0
    sc_a: float = 0.0
    sc_c: float = 0.0
    sc_n: int = 0
    sc_m: int = 0

    @property
    def natoms(self) -> int:
        return 4 * self.ncell ** 3

    @property
    def box(self) -> tuple:
        edge = self.ncell * self.a
        return (edge, edge, edge)


def lj_lattice_constant(rho: float) -> float:
    """fcc lattice constant for reduced number density rho (4 atoms per cell)."""
    return (4.0 / rho) ** (1.0 / 3.0)


RHO_LJ = 0.8442
A_LJ = lj_lattice_constant(RHO_LJ)

# The five workloads: a 4k LJ melt checked step by step, its 256k scale-up
# (throughput case), a high-neighbour-count LJ at cutoff 5 sigma, a 500k-atom
# Sutton-Chen copper-like metal standing in for the paper's EAM system, and a
# force-matching set of 8 x 32k LJ snapshots.
LJ_4K = Workload("lj_melt_4k", 10, A_LJ, "lj", 2.5, 0.3, 0.005, 100, 3.0, 4000)
LJ_256K = Workload("lj_melt_256k", 40, A_LJ, "lj", 2.5, 0.3, 0.005, 1000, 3.0, 256000)
LJ_HI_108K = Workload("lj_rc5_108k", 30, A_LJ, "lj", 5.0, 0.3, 0.005, 500, 1.5, 108000)
SC_500K = Workload("sc_cu_500k", 50, 3.61, "sc", 7.22, 1.0, 0.001, 200, 600.0, 500000,
                   mass=63.55, units=METAL_UNITS, sc_eps=1.2382e-2, sc_a=3.61,
                   sc_c=39.432, sc_n=9, sc_m=6)
LJ_FM_32K = Workload("lj_fm_32k", 20, A_LJ, "lj", 2.5, 0.3, 0.005, 500, 1.5, 1)
FM_SEEDS = tuple(range(1, 9))
FM_TARGET = (1.1, 1.05)        # (eps, sigma) that generate the target forces

WORKLOADS = {w.name: w for w in (LJ_4K, LJ_256K, LJ_HI_108K, SC_500K, LJ_FM_32K)}


def scaled(w: Workload, ncell: int, **kw) -> Workload:
    """The same workload on a different lattice size (parity and sweep cases)."""
    return dataclasses.replace(w, name=f"{w.name}@{ncell}", ncell=ncell, **kw)


def fcc_positions(ncell: int, a: float) -> np.ndarray:
    """fcc lattice, SoA float64 [3][N]; atom order: cell z, y, x, then basis."""
    idx = np.arange(ncell, dtype=np.float64)
    cz, cy, cx = np.meshgrid(idx, idx, idx, indexing="ij")
    out = np.empty((3, ncell, ncell, ncell, 4), dtype=np.float64)
    for b, (bx, by, bz) in enumerate(FCC_BASIS):
        out[0, ..., b] = (cx + bx) * a
        out[1, ..., b] = (cy + by) * a
        out[2, ..., b] = (cz + bz) * a
    return np.ascontiguousarray(out.reshape(3, -1))


def gaussian_velocities(n: int, temp: float, mass: float, units: Units,
                        seed: int) -> np.ndarray:
    """Gaussian velocities (SoA [3][N]) with zero net momentum, scaled so that
    the kinetic temperature with 3N-3 degrees of freedom equals temp exactly."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    v -= v.mean(axis=0)
    if temp <= 0.0 or n < 2:
        return np.zeros((3, n))
    dof = 3 * n - 3
    t_now = mass * units.mvv2e * float(np.sum(v * v)) / (dof * units.boltz)
    v *= math.sqrt(temp / t_now)
    return np.ascontiguousarray(v.T)


def jitter(x: np.ndarray, amp: float, seed: int) -> np.ndarray:
    """Uniform random displacements in [-amp, amp] per component (copy)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(x + rng.uniform(-amp, amp, size=x.shape))


def random_unit_vectors(n: int, seed: int) -> np.ndarray:
    """Random cotangent / direction field SoA [3][N] with unit RMS entries."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((3, n)))


def initial_state(w: Workload, seed: Optional[int] = None):
    """(x, v, box) for a workload: perfect lattice + Gaussian velocities."""
    x = fcc_positions(w.ncell, w.a)
    v = gaussian_velocities(w.natoms, w.temp, w.mass, w.units,
                            w.seed if seed is None else seed)
    return x, v, w.box
