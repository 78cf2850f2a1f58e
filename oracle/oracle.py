"""ctypes front end of the C oracle (md_oracle.c).  Test infrastructure only.

Each wrapper takes and returns numpy arrays in the oracle's conventions: SoA
positions/forces [3][N] float64, row-major neighbour lists [N][cap] int32.
Statuses other than 0 raise OracleError (3, list overflow, is reported with the
largest neighbour count so callers can grow the list and retry).
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "md_oracle.c")
LIB = os.path.join(HERE, "libmd_oracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall", "-Wno-unused-function"]
# AddressSanitizer + UndefinedBehaviorSanitizer build of the same source (a
# process loading it needs gcc's libasan preloaded); MD_ORACLE_LIB selects the
# library lib() loads.
SAN_LIB = os.path.join(HERE, "libmd_oracle_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-g"]


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str, max_count: int = -1):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code
        self.max_count = max_count


def build(force: bool = True) -> str:
    """Compile md_oracle.c into libmd_oracle.so with gcc (no FMA contraction)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def build_sanitized() -> str:
    """Compile md_oracle.c with the oracle's flags plus ASan and UBSan into
    libmd_oracle_san.so."""
    tmp = SAN_LIB + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, *SAN_FLAGS, "-o", tmp, SRC, "-lm"])
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


_lib = None


@contextlib.contextmanager
def using(path: str):
    """Temporarily route every wrapper through another build of the oracle
    (used by the tests that plant mistakes in a copy of the source)."""
    global _lib
    old = _lib
    L = ctypes.CDLL(path)
    _declare(L)
    _lib = L
    try:
        yield
    finally:
        _lib = old


def build_variant(source_text: str, out_path: str) -> str:
    """Compile an edited copy of md_oracle.c with the oracle's own flags."""
    src = out_path + ".c"
    with open(src, "w") as fh:
        fh.write(source_text)
    subprocess.check_call(["gcc", *CFLAGS, "-o", out_path, src, "-lm"])
    return out_path


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("MD_ORACLE_LIB")
        if not path:
            path = LIB
            if not os.path.exists(LIB):
                build()
        _lib = ctypes.CDLL(path)
        _declare(_lib)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i64 = ctypes.c_int64


class Params(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("rc", ctypes.c_double), ("skin", ctypes.c_double),
                ("lj_eps", ctypes.c_double), ("lj_sigma", ctypes.c_double),
                ("lj_shift", ctypes.c_int), ("sc_eps", ctypes.c_double),
                ("sc_a", ctypes.c_double), ("sc_c", ctypes.c_double), ("sc_n", ctypes.c_int),
                ("sc_m", ctypes.c_int), ("mass", ctypes.c_double), ("dt", ctypes.c_double),
                ("ftm2v", ctypes.c_double), ("mvv2e", ctypes.c_double),
                ("boltz", ctypes.c_double), ("buck_A", ctypes.c_double * 16),
                ("buck_rho", ctypes.c_double * 16), ("buck_C", ctypes.c_double * 16),
                ("q", ctypes.c_double * 4), ("qqr2e", ctypes.c_double),
                ("type", ctypes.c_void_p)]


def _declare(L):
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_cell_dims.argtypes = [_dp, ctypes.c_double, _ip]
    L.orc_bin.argtypes = [_i64, _dp, _dp, ctypes.c_double, _ip, _ip, _ip, _ip]
    L.orc_build_nlist.argtypes = [_i64, _dp, _dp, _ip, _ip, _ip, _ip, ctypes.c_double,
                                  ctypes.c_int, _ip, _ip, _ip]
    L.orc_lj_forces.argtypes = [_i64, _dp, _dp, _ip, _ip, ctypes.c_int, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp,
                                _dp, _dp]
    L.orc_sc_forces.argtypes = [_i64, _dp, _dp, _ip, _ip, ctypes.c_int, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_buck_forces.argtypes = [_i64, _dp, _dp, _ip, _ip, ctypes.c_int, ctypes.c_double,
                                  _ip, _dp, _dp, _dp, _dp, ctypes.c_double, _dp, _dp, _dp,
                                  _dp, _dp]
    L.orc_lj_vjp.argtypes = [_i64, _dp, _dp, _ip, _ip, ctypes.c_int, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
    L.orc_sc_vjp.argtypes = [_i64, _dp, _dp, _ip, _ip, ctypes.c_int, ctypes.c_double,
                             ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                             ctypes.c_int, _dp, _dp, _dp]
    L.orc_md_run.argtypes = [ctypes.POINTER(Params), _i64, _dp, _dp, _dp, ctypes.c_int,
                             ctypes.c_int, ctypes.c_int, _dp, _ip, _dp]
    L.orc_md_run_nvt.argtypes = [ctypes.POINTER(Params), _i64, _dp, _dp, _dp, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int, _dp, _dp, _ip, _dp]
    L.orc_md_run_npt.argtypes = [ctypes.POINTER(Params), _i64, _dp, _dp, _dp, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp, _ip,
                                 _dp]
    for name in ("orc_cell_dims", "orc_bin", "orc_build_nlist", "orc_lj_forces",
                 "orc_sc_forces", "orc_buck_forces", "orc_lj_vjp", "orc_sc_vjp",
                 "orc_md_run", "orc_md_run_nvt", "orc_md_run_npt"):
        getattr(L, name).restype = ctypes.c_int


def _d(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_dp)


def _i(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_ip)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


def cell_dims(box, rl: float):
    nc = np.zeros(3, np.int32)
    st = lib().orc_cell_dims(_d(_f64(box)), rl, _i(nc))
    if st:
        raise OracleError(st, "cell_dims")
    return nc


@dataclass
class Cells:
    x: np.ndarray            # wrapped positions [3][N]
    nc: np.ndarray           # cells per dimension
    atom_cell: np.ndarray    # [N]
    cell_start: np.ndarray   # [ncell+1]
    perm: np.ndarray         # [N]


def bin_cells(x, box, rl: float) -> Cells:
    """Wrap (on a copy) and bin; stable counting sort by cell."""
    x = _f64(x).copy()
    n = x.shape[1]
    L = _f64(box)
    nc = cell_dims(L, rl)
    ncell = int(nc[0]) * int(nc[1]) * int(nc[2])
    atom_cell = np.zeros(n, np.int32)
    cell_start = np.zeros(ncell + 1, np.int32)
    perm = np.zeros(n, np.int32)
    st = lib().orc_bin(n, _d(x), _d(L), rl, _i(nc), _i(atom_cell), _i(cell_start), _i(perm))
    if st:
        raise OracleError(st, "bin")
    return Cells(x, nc, atom_cell, cell_start, perm)


@dataclass
class NList:
    numneigh: np.ndarray     # [N]
    neigh: np.ndarray        # [N][cap]
    cap: int
    max_count: int

    def pairs(self) -> np.ndarray:
        """Sorted (i, j) pairs of the list as an [M][2] int64 array."""
        n = self.numneigh.shape[0]
        cnt = np.minimum(self.numneigh, self.cap)
        i = np.repeat(np.arange(n, dtype=np.int64), cnt)
        mask = np.arange(self.cap)[None, :] < cnt[:, None]
        j = self.neigh[mask].astype(np.int64)
        p = np.stack([i, j], axis=1)
        return p[np.lexsort((p[:, 1], p[:, 0]))]


def build_nlist(x, box, rl: float, cap: int = 0, cells: Optional[Cells] = None):
    """Bin (on a copy) and build the full list at radius rl.  Returns
    (NList, Cells); cells.x holds the wrapped positions the list refers to.
    cap = 0 sizes the list from a first counting pass."""
    if cells is None:
        cells = bin_cells(x, box, rl)
    n = cells.x.shape[1]
    L = _f64(box)
    if cap <= 0:
        cap = 1
        mc = np.zeros(1, np.int32)
        nn = np.zeros(n, np.int32)
        tmp = np.zeros((n, 1), np.int32)
        lib().orc_build_nlist(n, _d(cells.x), _d(L), _i(cells.nc), _i(cells.atom_cell),
                              _i(cells.cell_start), _i(cells.perm), rl, 1, _i(nn), _i(tmp),
                              _i(mc))
        cap = max(1, int(mc[0]))
    numneigh = np.zeros(n, np.int32)
    neigh = np.zeros((n, cap), np.int32)
    mc = np.zeros(1, np.int32)
    st = lib().orc_build_nlist(n, _d(cells.x), _d(L), _i(cells.nc), _i(cells.atom_cell),
                               _i(cells.cell_start), _i(cells.perm), rl, cap, _i(numneigh),
                               _i(neigh), _i(mc))
    if st:
        raise OracleError(st, "build_nlist", int(mc[0]))
    return NList(numneigh, neigh, cap, int(mc[0])), cells


@dataclass
class ForceResult:
    f: np.ndarray
    energy: float
    virial: np.ndarray
    eatom: np.ndarray
    vatom: np.ndarray
    rho: Optional[np.ndarray] = None


def lj_forces(x, box, nl: NList, rc, eps=1.0, sigma=1.0, shift=0) -> ForceResult:
    x = _f64(x)
    n = x.shape[1]
    f = np.zeros((3, n))
    ea = np.zeros(n)
    va = np.zeros((6, n))
    e = np.zeros(1)
    w = np.zeros(6)
    st = lib().orc_lj_forces(n, _d(x), _d(_f64(box)), _i(nl.numneigh), _i(nl.neigh), nl.cap,
                             rc, eps, sigma, int(shift), _d(f), _d(ea), _d(va), _d(e), _d(w))
    if st:
        raise OracleError(st, "lj_forces")
    return ForceResult(f, float(e[0]), w, ea, va)


def sc_forces(x, box, nl: NList, rc, eps, a, c, nexp, mexp) -> ForceResult:
    x = _f64(x)
    n = x.shape[1]
    f = np.zeros((3, n))
    rho = np.zeros(n)
    ea = np.zeros(n)
    va = np.zeros((6, n))
    e = np.zeros(1)
    w = np.zeros(6)
    st = lib().orc_sc_forces(n, _d(x), _d(_f64(box)), _i(nl.numneigh), _i(nl.neigh), nl.cap,
                             rc, eps, a, c, int(nexp), int(mexp), _d(f), _d(rho), _d(ea),
                             _d(va), _d(e), _d(w))
    if st:
        raise OracleError(st, "sc_forces")
    return ForceResult(f, float(e[0]), w, ea, va, rho)


def buck_tables(pairs):
    """Symmetric 4 x 4 table (flattened a * 4 + b) from ((a, b), value) pairs."""
    t = np.zeros(16)
    for (a, b), val in pairs:
        t[a * 4 + b] = val
        t[b * 4 + a] = val
    return t


def buck_forces(x, box, nl: NList, rc, types, A, rho, C, q, qqr2e) -> ForceResult:
    """Buckingham + cut Coulomb; A, rho, C: 16-entry tables (a * 4 + b), q: 4
    charges per species, types: species per atom.  Entries of rho for pairs
    that never occur may be anything nonzero."""
    x = _f64(x)
    n = x.shape[1]
    types = np.ascontiguousarray(types, dtype=np.int32)
    rho = np.where(np.asarray(rho, float) == 0.0, 1.0, np.asarray(rho, float))
    f = np.zeros((3, n))
    ea = np.zeros(n)
    va = np.zeros((6, n))
    e = np.zeros(1)
    w = np.zeros(6)
    st = lib().orc_buck_forces(n, _d(x), _d(_f64(box)), _i(nl.numneigh), _i(nl.neigh), nl.cap,
                               rc, _i(types), _d(_f64(A)), _d(_f64(rho)), _d(_f64(C)),
                               _d(_f64(q)), qqr2e, _d(f), _d(ea), _d(va), _d(e), _d(w))
    if st:
        raise OracleError(st, "buck_forces")
    return ForceResult(f, float(e[0]), w, ea, va)


def lj_vjp(x, box, nl: NList, rc, eps, sigma, u):
    """Returns (gx [3][N], gparam [2] = dL/deps, dL/dsigma)."""
    x = _f64(x)
    u = _f64(u)
    n = x.shape[1]
    gx = np.zeros((3, n))
    gp = np.zeros(2)
    st = lib().orc_lj_vjp(n, _d(x), _d(_f64(box)), _i(nl.numneigh), _i(nl.neigh), nl.cap,
                          rc, eps, sigma, _d(u), _d(gx), _d(gp))
    if st:
        raise OracleError(st, "lj_vjp")
    return gx, gp


def sc_vjp(x, box, nl: NList, rc, eps, a, c, nexp, mexp, u):
    """Returns (gx [3][N], gparam [3] = dL/deps, dL/da, dL/dc) for
    L = sum_i u_i . F_i of the Sutton-Chen forces."""
    x = _f64(x)
    u = _f64(u)
    n = x.shape[1]
    gx = np.zeros((3, n))
    gp = np.zeros(3)
    st = lib().orc_sc_vjp(n, _d(x), _d(_f64(box)), _i(nl.numneigh), _i(nl.neigh), nl.cap,
                          rc, eps, a, c, int(nexp), int(mexp), _d(u), _d(gx), _d(gp))
    if st:
        raise OracleError(st, "sc_vjp")
    return gx, gp


_KIND = {"lj": 0, "sc": 1, "buck": 2}


def params_for(w, **over) -> Params:
    """orc_params for a Workload (paper_1009_4330_amd.inputs.Workload).  For
    the Buckingham workload the species array (input order) is kept alive on
    the returned object."""
    p = Params(kind=_KIND[w.potential], rc=w.rc, skin=w.skin, lj_eps=w.lj_eps,
               lj_sigma=w.lj_sigma, lj_shift=w.lj_shift, sc_eps=w.sc_eps, sc_a=w.sc_a,
               sc_c=w.sc_c, sc_n=w.sc_n, sc_m=w.sc_m, mass=w.mass, dt=w.dt,
               ftm2v=w.units.ftm2v, mvv2e=w.units.mvv2e, boltz=w.units.boltz)
    if w.potential == "buck":
        p.buck_A[:] = buck_tables(w.buck_A)
        rho = buck_tables(w.buck_rho)
        p.buck_rho[:] = np.where(rho == 0.0, 1.0, rho)
        p.buck_C[:] = buck_tables(w.buck_C)
        p.q[:] = list(w.charges) + [0.0] * (4 - len(w.charges))
        p.qqr2e = w.qqr2e
        p._types = np.ascontiguousarray(w.species(), dtype=np.int32)
        p.type = p._types.ctypes.data
    for k, v in over.items():
        setattr(p, k, v)
    return p


@dataclass
class RunResult:
    x: np.ndarray
    v: np.ndarray
    f: np.ndarray
    thermo: np.ndarray       # rows: step, pe, ke, etot, temp, press, rebuilds, maxcount
    rebuilt: np.ndarray      # [nsteps+1] 0/1


def md_run(params: Params, x, v, box, nsteps: int, thermo_every: int = 1,
           cap: int = 0) -> RunResult:
    """Velocity-Verlet NVE run; x, v are copied.  cap = 0 picks a list capacity
    from the initial configuration with generous headroom."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    n = x.shape[1]
    if cap <= 0:
        nl, _ = build_nlist(x, box, params.rc + params.skin)
        cap = int(nl.max_count * 1.5) + 32
    rows = 1 + nsteps // thermo_every
    thermo = np.zeros((rows, 8))
    rebuilt = np.zeros(nsteps + 1, np.int32)
    f = np.zeros((3, n))
    st = lib().orc_md_run(ctypes.byref(params), n, _d(x), _d(v), _d(_f64(box)), nsteps,
                          thermo_every, cap, _d(thermo), _i(rebuilt), _d(f))
    if st:
        raise OracleError(st, "md_run")
    return RunResult(x, v, f, thermo, rebuilt)


def md_run_nvt(params: Params, x, v, box, nsteps: int, t_target: float, t_damp: float,
               chain_len: int = 3, chain=None, thermo_every: int = 1, cap: int = 0):
    """Nose-Hoover chain NVT run; x, v, chain are copied.  Returns
    (RunResult with nine-column thermo rows, final chain [eta..., veta...])."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    n = x.shape[1]
    ch = np.zeros(2 * chain_len) if chain is None else np.array(chain, dtype=np.float64)
    if cap <= 0:
        nl, _ = build_nlist(x, box, params.rc + params.skin)
        cap = int(nl.max_count * 1.5) + 32
    rows = 1 + nsteps // thermo_every
    thermo = np.zeros((rows, 9))
    rebuilt = np.zeros(nsteps + 1, np.int32)
    f = np.zeros((3, n))
    st = lib().orc_md_run_nvt(ctypes.byref(params), n, _d(x), _d(v), _d(_f64(box)), nsteps,
                              thermo_every, cap, t_target, t_damp, chain_len, _d(ch),
                              _d(thermo), _i(rebuilt), _d(f))
    if st:
        raise OracleError(st, "md_run_nvt")
    return RunResult(x, v, f, thermo, rebuilt), ch


def md_run_npt(params: Params, x, v, box, nsteps: int, t_target: float, t_damp: float,
               p_target: float, p_damp: float, chain_len: int = 3, chain=None,
               thermo_every: int = 1, cap: int = 0):
    """Isotropic NPT run (MTK barostat, Nose-Hoover chains on the particles and
    on the barostat); x, v, box, chain are copied.  chain holds eta[M],
    veta[M], xi[M], w[M], p_eps.  Returns (RunResult with ten-column thermo
    rows, final chain, final box)."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    L = np.array(box, dtype=np.float64)
    n = x.shape[1]
    ch = (np.zeros(4 * chain_len + 1) if chain is None
          else np.array(chain, dtype=np.float64))
    if cap <= 0:
        nl, _ = build_nlist(x, box, params.rc + params.skin)
        cap = int(nl.max_count * 1.6) + 48
    rows = 1 + nsteps // thermo_every
    thermo = np.zeros((rows, 10))
    rebuilt = np.zeros(nsteps + 1, np.int32)
    f = np.zeros((3, n))
    st = lib().orc_md_run_npt(ctypes.byref(params), n, _d(x), _d(v), _d(L), nsteps,
                              thermo_every, cap, t_target, t_damp, chain_len, p_target, p_damp,
                              _d(ch), _d(thermo), _i(rebuilt), _d(f))
    if st:
        raise OracleError(st, "md_run_npt")
    return RunResult(x, v, f, thermo, rebuilt), ch, L
