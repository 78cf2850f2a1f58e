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
    ncell: int                 # cubic unit cells per box edge
    a: float                   # lattice constant
    potential: str             # "lj", "sc" or "buck"
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
    # Buckingham + cut Coulomb: {(a, b): value} per species pair, charges per
    # species, the Coulomb constant in the workload's units
    lattice: str = "fcc"       # "fcc" (4 atoms per cell) or "rocksalt" (8, two species)
    buck_A: tuple = ()
    buck_rho: tuple = ()
    buck_C: tuple = ()
    charges: tuple = ()
    qqr2e: float = 0.0
    # fcc unit cells along x, y, z for an orthorhombic box; () = ncell along each
    shape: tuple = ()

    @property
    def cells_xyz(self) -> tuple:
        return tuple(self.shape) if self.shape else (self.ncell,) * 3

    @property
    def natoms(self) -> int:
        c = self.cells_xyz
        return (8 if self.lattice == "rocksalt" else 4) * c[0] * c[1] * c[2]

    def species(self) -> np.ndarray:
        """Species per atom in the order of initial_state's positions."""
        if self.lattice != "rocksalt":
            return np.zeros(self.natoms, np.int32)
        return np.tile(np.array([0, 0, 0, 0, 1, 1, 1, 1], np.int32), self.ncell ** 3)

    @property
    def box(self) -> tuple:
        return tuple(c * self.a for c in self.cells_xyz)


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

# The paper's second system (Appendix A "Silicate (cutoff)") uses Buckingham +
# cut Coulomb at 15 A cutoff, number density 0.09 A^-3 and 600 K, with
# parameters it does not print.  Stand-in: a two-species rocksalt ionic
# crystal at that density (a = (8 / 0.09)^(1/3) A), charges +-2 e and
# Buckingham terms of magnitudes typical of oxide models; one mass for both
# species (the kernels assume uniform mass).  All values are synthetic.  At
# 26^3 cells the box holds 140,608 atoms, about the paper's 139,968.
# The lattice constant puts the 15 A cutoff between two shells of the ion
# lattice (spacing a/2: shells at a/2 sqrt(46) = 14.85 A and a/2 sqrt(48) =
# 15.16 A), so that thermal motion seldom carries a pair across it (with a
# plain cut Coulomb every crossing changes the energy by qqr2e q_a q_b / rc);
# number density 8 / a^3 = 0.0954 A^-3, close to the paper's 0.09.
A_BUCK = 4.377
QQR2E_METAL = 14.399645        # e^2 / (4 pi eps0) in eV A
BUCK_KW = dict(mass=20.0, units=METAL_UNITS, lattice="rocksalt",
               buck_A=(((0, 1), 1500.0), ((1, 1), 20000.0)),
               buck_rho=(((0, 1), 0.30), ((1, 1), 0.15)),
               buck_C=(((1, 1), 30.0),),
               charges=(2.0, -2.0), qqr2e=QQR2E_METAL)
BUCK_141K = Workload("buck_coul_141k", 26, A_BUCK, "buck", 15.0, 2.0, 0.001, 100, 600.0,
                     140608, **BUCK_KW)
FM_SEEDS = tuple(range(1, 9))
FM_TARGET = (1.1, 1.05)        # (eps, sigma) that generate the target forces

WORKLOADS = {w.name: w for w in (LJ_4K, LJ_256K, LJ_HI_108K, SC_500K, LJ_FM_32K, BUCK_141K)}


def scaled(w: Workload, ncell: int, **kw) -> Workload:
    """The same workload on a different lattice size (parity and sweep cases)."""
    return dataclasses.replace(w, name=f"{w.name}@{ncell}", ncell=ncell, **kw)


def fcc_positions(ncell, a: float) -> np.ndarray:
    """fcc lattice of ncell unit cells per edge, or (nx, ny, nz) cells along
    x, y, z; SoA float64 [3][N]; atom order: cell z, y, x, then basis."""
    nx, ny, nz = (ncell,) * 3 if np.isscalar(ncell) else tuple(ncell)
    cz, cy, cx = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nx, dtype=np.float64), indexing="ij")
    out = np.empty((3, nz, ny, nx, 4), dtype=np.float64)
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


def rocksalt_positions(ncell: int, a: float) -> np.ndarray:
    """Rocksalt lattice, SoA float64 [3][N]: per cubic cell the four fcc
    sites (species 0) then the same sites shifted by a/2 along x (species 1)."""
    idx = np.arange(ncell, dtype=np.float64)
    cz, cy, cx = np.meshgrid(idx, idx, idx, indexing="ij")
    out = np.empty((3, ncell, ncell, ncell, 8), dtype=np.float64)
    for s, shift in enumerate((0.0, 0.5)):
        for b, (bx, by, bz) in enumerate(FCC_BASIS):
            out[0, ..., 4 * s + b] = (cx + bx + shift) * a
            out[1, ..., 4 * s + b] = (cy + by) * a
            out[2, ..., 4 * s + b] = (cz + bz) * a
    return np.ascontiguousarray(out.reshape(3, -1))


def pair_table(w: Workload, which: str) -> np.ndarray:
    """Symmetric 4 x 4 table (flattened a * 4 + b) of a Buckingham parameter."""
    t = np.zeros(16)
    for (a, b), val in getattr(w, which):
        t[a * 4 + b] = val
        t[b * 4 + a] = val
    return t


def initial_state(w: Workload, seed: Optional[int] = None):
    """(x, v, box) for a workload: perfect lattice + Gaussian velocities."""
    if w.lattice == "rocksalt":
        if w.shape:
            raise ValueError("orthorhombic shapes are fcc only")
        x = rocksalt_positions(w.ncell, w.a)
    else:
        x = fcc_positions(w.cells_xyz, w.a)
    v = gaussian_velocities(w.natoms, w.temp, w.mass, w.units,
                            w.seed if seed is None else seed)
    return x, v, w.box
