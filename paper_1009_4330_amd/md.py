"""Python binding of the C ABI in include/md.h (argument marshalling only).

Every function has the name of the C entry point it calls.  Device buffers are
torch tensors on the GPU; streams are torch's current stream.  There is no
fallback: if libmd_mi355x.so is missing or a call fails, an exception says so.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

# The in-tree build; MD_LIB_PATH selects another build of the same library
# (the sanitized host build the ABI tests load).
LIB_PATH = os.environ.get("MD_LIB_PATH") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libmd_mi355x.so")

MD_OK, MD_ERR_INVALID_ARG, MD_ERR_BOX_TOO_SMALL, MD_ERR_NLIST_OVERFLOW = 0, 1, 2, 3
MD_ERR_NONFINITE, MD_ERR_UNSUPPORTED, MD_ERR_HIP, MD_ERR_WORKSPACE = 4, 5, 6, 7
MD_ERR_UNSTABLE, MD_ERR_SCRATCH = 8, 9
MD_NOALLOC_SCRATCH_BYTES = 67108864   # md.h: fixed scratch of md_compute_forces_noalloc
MD_MAX_ATOMS = 134217727          # md.h: largest atom count
MD_FP64, MD_MIXED = 0, 1
MD_KERNEL_AUTO, MD_KERNEL_TPA, MD_KERNEL_WPA = 0, 1, 64
LANES = (1, 2, 4, 8, 16, 32, 64)
MD_EFLAG, MD_VFLAG = 1, 2
MD_POT_LJ, MD_POT_SC, MD_POT_BUCK = 0, 1, 2
MD_LAYOUT_TPA, MD_LAYOUT_WPA, MD_LAYOUT_TILE = 1, 64, 256
TILE_LANES = (1, 2, 4, 8)         # lanes per atom of the tiled layouts
MD_ST_ERRORS, MD_ST_MAXNEIGH, MD_ST_BUILDS, MD_ST_REBUILD, MD_STATUS_WORDS = 0, 1, 2, 3, 8
EXPORTS = ("md_workspace_bytes", "md_nlist_ints", "md_thermo_rows", "md_bin_cells", "md_sort_atoms",
           "md_build_neighbors", "md_compute_forces", "md_step", "md_step_nvt", "md_force_vjp",
           "md_autoselect", "md_nlist_status", "md_timing_enable", "md_timing_read",
           "md_status_string", "md_compute_forces_noalloc",
           "md_compute_forces_noalloc_bytes", "md_nlist_tile_entries", "md_step_npt")


class MDError(RuntimeError):
    def __init__(self, code: int, call: str):
        super().__init__(f"{call}: {status_string(code)} (status {code})")
        self.code = code


class md_box(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3)]


class md_potential(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("rc", ctypes.c_double), ("lj_eps", ctypes.c_double),
                ("lj_sigma", ctypes.c_double), ("lj_shift", ctypes.c_int),
                ("sc_eps", ctypes.c_double), ("sc_a", ctypes.c_double),
                ("sc_c", ctypes.c_double), ("sc_n", ctypes.c_int), ("sc_m", ctypes.c_int),
                ("buck_A", ctypes.c_double * 16), ("buck_rho", ctypes.c_double * 16),
                ("buck_C", ctypes.c_double * 16), ("q", ctypes.c_double * 4),
                ("qqr2e", ctypes.c_double), ("type", ctypes.c_void_p)]


class md_cells(ctypes.Structure):
    _fields_ = [("nc", ctypes.c_int * 3), ("ncell_cap", ctypes.c_int64),
                ("cell_start", ctypes.c_void_p), ("atom_cell", ctypes.c_void_p),
                ("perm", ctypes.c_void_p)]


class md_nlist(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int), ("layout", ctypes.c_int), ("rl", ctypes.c_double),
                ("neigh", ctypes.c_void_p), ("numneigh", ctypes.c_void_p),
                ("x_ref", ctypes.c_void_p), ("status", ctypes.c_void_p), ("half", ctypes.c_int),
                ("tile", ctypes.c_void_p), ("tile_entries", ctypes.c_size_t)]


MD_NHC_MAX, MD_NHC_STATE = 8, 20


class md_nhc(ctypes.Structure):
    _fields_ = [("t_target", ctypes.c_double), ("t_damp", ctypes.c_double),
                ("chain", ctypes.c_int), ("state", ctypes.c_void_p)]


MD_NPT_STATE = 64
NPT_L = 33            # md_npt.state: box edges at [33, 36)


class md_npt(ctypes.Structure):
    _fields_ = [("t_target", ctypes.c_double), ("t_damp", ctypes.c_double),
                ("chain", ctypes.c_int), ("p_target", ctypes.c_double),
                ("p_damp", ctypes.c_double), ("state", ctypes.c_void_p)]


class md_state(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("x", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("f", ctypes.c_void_p), ("id", ctypes.c_void_p), ("mass", ctypes.c_double),
                ("ftm2v", ctypes.c_double), ("mvv2e", ctypes.c_double),
                ("boltz", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """The HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_1009_4330_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        P, V, I64, D, I = (ctypes.POINTER, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                           ctypes.c_int)
        L.md_workspace_bytes.restype = ctypes.c_size_t
        L.md_workspace_bytes.argtypes = [I64, P(md_box), D]
        L.md_nlist_ints.restype = ctypes.c_size_t
        L.md_nlist_ints.argtypes = [I64, I]
        L.md_nlist_tile_entries.restype = ctypes.c_size_t
        L.md_nlist_tile_entries.argtypes = [I64, I, P(md_box), D]
        L.md_thermo_rows.restype = I
        L.md_thermo_rows.argtypes = [I, I, I]
        L.md_status_string.restype = ctypes.c_char_p
        L.md_status_string.argtypes = [I]
        L.md_bin_cells.argtypes = [V, I64, P(md_box), D, P(md_cells), V, ctypes.c_size_t, V]
        L.md_sort_atoms.argtypes = [P(md_state), P(md_cells), V, V, ctypes.c_size_t, V]
        L.md_build_neighbors.argtypes = [V, I64, P(md_box), P(md_cells), D, D, P(md_nlist), V]
        L.md_compute_forces.argtypes = [P(md_potential), V, I64, P(md_box), P(md_nlist), I, I, I,
                                        V, V, V, ctypes.c_size_t, V]
        L.md_compute_forces_noalloc.argtypes = [P(md_potential), V, I64, P(md_box), P(md_nlist),
                                                I, I, I, V, V, V]
        L.md_compute_forces_noalloc_bytes.restype = ctypes.c_size_t
        L.md_compute_forces_noalloc_bytes.argtypes = [I64, I, I]
        L.md_step.argtypes = [P(md_state), P(md_potential), P(md_box), P(md_cells), P(md_nlist),
                              I, I, D, D, I, I, I, V, V, ctypes.c_size_t, V]
        L.md_step_nvt.argtypes = [P(md_state), P(md_potential), P(md_box), P(md_cells),
                                  P(md_nlist), I, I, D, D, P(md_nhc), I, I, I, V, V,
                                  ctypes.c_size_t, V]
        L.md_step_npt.argtypes = [P(md_state), P(md_potential), P(md_box), P(md_cells),
                                  P(md_nlist), I, I, D, D, P(md_npt), I, I, I, V, V,
                                  ctypes.c_size_t, V]
        L.md_force_vjp.argtypes = [P(md_potential), V, I64, P(md_box), P(md_nlist), I, V, V, V,
                                   V, ctypes.c_size_t, V]
        L.md_autoselect.argtypes = [P(md_potential), V, I64, P(md_box), P(md_cells), D,
                                    P(md_nlist), I, I, P(I), V, ctypes.c_size_t, V]
        L.md_nlist_status.argtypes = [P(md_nlist), P(I), V]
        L.md_timing_enable.argtypes = [I]
        L.md_timing_read.argtypes = [P(I64), P(D)]
        for name in EXPORTS:
            if name not in ("md_workspace_bytes", "md_nlist_ints", "md_thermo_rows",
                            "md_status_string", "md_compute_forces_noalloc_bytes",
                            "md_nlist_tile_entries"):
                getattr(L, name).restype = I
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().md_status_string(int(code)).decode()


def _check(code: int, call: str) -> None:
    if code != MD_OK:
        raise MDError(code, call)


def _ptr(t: Optional[torch.Tensor], dtype=None, numel: Optional[int] = None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{dtype} tensor expected, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"tensor too small: {t.numel()} < {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _check_list(nl: "NList", n: int, call: str) -> None:
    """The list's buffers must cover n atoms: a list sized for fewer atoms
    would be read past its end by the kernels (the C descriptor carries no
    atom count to check against)."""
    if nl.numneigh.numel() < n:
        raise ValueError(f"{call}: list holds {nl.numneigh.numel()} atoms, positions have {n}")
    need = md_nlist_ints(n, nl.capacity)
    if nl.neigh.numel() < need:
        raise ValueError(f"{call}: neigh holds {nl.neigh.numel()} ints, {need} needed")
    if nl.x_ref.numel() < 3 * n:
        raise ValueError(f"{call}: x_ref holds {nl.x_ref.numel()} values, {3 * n} needed")


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def make_box(L: Sequence[float]) -> md_box:
    b = md_box()
    for d in range(3):
        b.L[d] = float(L[d])
    return b


def lj_potential(rc: float, eps: float = 1.0, sigma: float = 1.0, shift: int = 0) -> md_potential:
    return md_potential(kind=MD_POT_LJ, rc=rc, lj_eps=eps, lj_sigma=sigma, lj_shift=shift)


def sc_potential(rc, eps, a, c, n, m) -> md_potential:
    return md_potential(kind=MD_POT_SC, rc=rc, sc_eps=eps, sc_a=a, sc_c=c, sc_n=n, sc_m=m)


def buck_potential(rc, A, rho, C, q, qqr2e, type_tensor) -> md_potential:
    """Buckingham + cut Coulomb.  A, rho, C: 16 values each (species pair
    a * 4 + b); q: up to 4 charges; type_tensor: device int32 species per atom,
    which md_step permutes in place with the atoms (the descriptor keeps its
    address, so the tensor must outlive it)."""
    if type_tensor.dtype != torch.int32 or not type_tensor.is_contiguous():
        raise ValueError("species must be a contiguous int32 tensor")
    qs = list(q) + [0.0] * (4 - len(q))
    p = md_potential(kind=MD_POT_BUCK, rc=rc, qqr2e=qqr2e, type=type_tensor.data_ptr())
    for k in range(16):
        p.buck_A[k], p.buck_rho[k], p.buck_C[k] = float(A[k]), float(rho[k]), float(C[k])
    for k in range(4):
        p.q[k] = float(qs[k])
    return p


class Cells:
    """Device cell arrays + their md_cells descriptor."""

    def __init__(self, n: int, ncell_cap: int, device="cuda"):
        self.cell_start = torch.zeros(ncell_cap + 1, dtype=torch.int32, device=device)
        self.atom_cell = torch.zeros(n, dtype=torch.int32, device=device)
        self.perm = torch.zeros(n, dtype=torch.int32, device=device)
        self.c = md_cells(ncell_cap=ncell_cap, cell_start=self.cell_start.data_ptr(),
                          atom_cell=self.atom_cell.data_ptr(), perm=self.perm.data_ptr())

    @property
    def nc(self):
        return tuple(self.c.nc)


class NList:
    """Device neighbour-list arrays + their md_nlist descriptor.  The neigh
    buffer is sized for every layout K (md_nlist_ints); tile_entries > 0 adds
    the 16-bit buffer of the tiled layouts (md_nlist_tile_entries)."""

    def __init__(self, n: int, capacity: int, layout: int = MD_LAYOUT_TPA, device="cuda",
                 half: bool = False, tile_entries: int = 0):
        self.neigh = torch.zeros(md_nlist_ints(n, capacity), dtype=torch.int32, device=device)
        self.numneigh = torch.zeros(n, dtype=torch.int32, device=device)
        self.x_ref = torch.zeros(3, n, dtype=torch.float64, device=device)
        self.status = torch.zeros(MD_STATUS_WORDS, dtype=torch.int32, device=device)
        # torch has no uint16 arithmetic on every build: int16 storage, same bytes
        self.tile = (torch.zeros(tile_entries, dtype=torch.int16, device=device)
                     if tile_entries > 0 else None)
        self.c = md_nlist(capacity=capacity, layout=layout, rl=0.0,
                          neigh=self.neigh.data_ptr(), numneigh=self.numneigh.data_ptr(),
                          x_ref=self.x_ref.data_ptr(), status=self.status.data_ptr(),
                          half=1 if half else 0,
                          tile=self.tile.data_ptr() if self.tile is not None else None,
                          tile_entries=self.tile.numel() if self.tile is not None else 0)

    @property
    def capacity(self) -> int:
        return self.c.capacity

    @property
    def layout(self) -> int:
        return self.c.layout

    def rows(self) -> torch.Tensor:
        """The list as an [n][capacity] tensor (row i = neighbours of atom i),
        gathered through the layout-K index of include/md.h."""
        n, cap, k = self.numneigh.numel(), self.c.capacity, self.c.layout & ~MD_LAYOUT_TILE
        dev = self.neigh.device
        i = torch.arange(n, device=dev, dtype=torch.int64)[:, None]
        m = torch.arange(cap, device=dev, dtype=torch.int64)[None, :]
        g = 64 // k
        rows = (cap + k - 1) // k
        idx = ((i // g) * rows + m // k) * 64 + (i % g) * k + m % k
        return self.neigh[idx]


class State:
    """Dynamic state tensors (x, v, f [3][n] float64, id [n] int32) + md_state."""

    def __init__(self, x: torch.Tensor, v: torch.Tensor, mass: float, ftm2v=1.0, mvv2e=1.0,
                 boltz=1.0, ids: Optional[torch.Tensor] = None):
        n = x.shape[1]
        self.x = x.contiguous()
        self.v = v.contiguous()
        self.f = torch.zeros_like(self.x)
        self.id = (torch.arange(n, dtype=torch.int32, device=x.device) if ids is None
                   else ids.to(torch.int32).contiguous())
        self.c = md_state(n=n, x=self.x.data_ptr(), v=self.v.data_ptr(), f=self.f.data_ptr(),
                          id=self.id.data_ptr(), mass=mass, ftm2v=ftm2v, mvv2e=mvv2e,
                          boltz=boltz)

    @property
    def n(self) -> int:
        return self.c.n


def md_workspace_bytes(n: int, box: md_box, rl: float) -> int:
    b = lib().md_workspace_bytes(int(n), ctypes.byref(box), float(rl))
    if b == 0:
        raise MDError(MD_ERR_INVALID_ARG, "md_workspace_bytes")
    return int(b)


def workspace(n: int, box: md_box, rl: float, device="cuda") -> torch.Tensor:
    """A workspace tensor of md_workspace_bytes bytes (torch allocations are
    256-byte aligned)."""
    return torch.empty(md_workspace_bytes(n, box, rl), dtype=torch.uint8, device=device)


def md_nlist_ints(n: int, capacity: int) -> int:
    k = int(lib().md_nlist_ints(int(n), int(capacity)))
    if k == 0:
        raise MDError(MD_ERR_INVALID_ARG, "md_nlist_ints")
    return k


def md_nlist_tile_entries(n: int, capacity: int, box: md_box, rl: float) -> int:
    """Entries of the tiled layouts' 16-bit buffer (0: they do not apply)."""
    return int(lib().md_nlist_tile_entries(int(n), int(capacity), ctypes.byref(box), float(rl)))


def md_thermo_rows(nsteps: int, thermo_every: int, setup: int) -> int:
    return int(lib().md_thermo_rows(nsteps, thermo_every, setup))


def md_bin_cells(x: torch.Tensor, box: md_box, rl: float, cells: Cells, ws: torch.Tensor,
                 stream=None) -> None:
    n = x.shape[1]
    _check(lib().md_bin_cells(_ptr(x, torch.float64, 3 * n), n, ctypes.byref(box), rl,
                              ctypes.byref(cells.c), _ptr(ws), ws.numel(), _stream(stream)),
           "md_bin_cells")


def md_sort_atoms(state: State, cells: Cells, x_ref: Optional[torch.Tensor], ws: torch.Tensor,
                  stream=None) -> None:
    _check(lib().md_sort_atoms(ctypes.byref(state.c), ctypes.byref(cells.c),
                               _ptr(x_ref, torch.float64, 3 * state.n), _ptr(ws), ws.numel(),
                               _stream(stream)), "md_sort_atoms")


def md_build_neighbors(x: torch.Tensor, box: md_box, cells: Cells, rc: float, skin: float,
                       nl: NList, stream=None) -> None:
    n = x.shape[1]
    _check_list(nl, n, "md_build_neighbors")
    _check(lib().md_build_neighbors(_ptr(x, torch.float64, 3 * n), n, ctypes.byref(box),
                                    ctypes.byref(cells.c), rc, skin, ctypes.byref(nl.c),
                                    _stream(stream)), "md_build_neighbors")


def md_compute_forces(pot: md_potential, x: torch.Tensor, box: md_box, nl: NList, prec: int,
                      kernel: int, flags: int, f: torch.Tensor, ev: Optional[torch.Tensor],
                      ws: torch.Tensor, stream=None) -> None:
    n = x.shape[1]
    _check_list(nl, n, "md_compute_forces")
    _check(lib().md_compute_forces(ctypes.byref(pot), _ptr(x, torch.float64, 3 * n), n,
                                   ctypes.byref(box), ctypes.byref(nl.c), prec, kernel, flags,
                                   _ptr(f, torch.float64, 3 * n), _ptr(ev, torch.float64, 7),
                                   _ptr(ws), ws.numel(), _stream(stream)), "md_compute_forces")


def md_compute_forces_noalloc_bytes(n: int, kind: int, flags: int) -> int:
    return int(lib().md_compute_forces_noalloc_bytes(int(n), int(kind), int(flags)))


def md_compute_forces_noalloc(pot: md_potential, x: torch.Tensor, box: md_box, nl: NList,
                              prec: int, kernel: int, flags: int, f: torch.Tensor,
                              ev: Optional[torch.Tensor], stream=None) -> None:
    """md_compute_forces without a workspace (the library's fixed scratch)."""
    n = x.shape[1]
    _check_list(nl, n, "md_compute_forces_noalloc")
    _check(lib().md_compute_forces_noalloc(ctypes.byref(pot), _ptr(x, torch.float64, 3 * n), n,
                                           ctypes.byref(box), ctypes.byref(nl.c), prec, kernel,
                                           flags, _ptr(f, torch.float64, 3 * n),
                                           _ptr(ev, torch.float64, 7), _stream(stream)),
           "md_compute_forces_noalloc")


def md_step(state: State, pot: md_potential, box: md_box, cells: Cells, nl: NList, prec: int,
            kernel: int, skin: float, dt: float, nsteps: int, thermo_every: int, setup: int,
            thermo: Optional[torch.Tensor], ws: torch.Tensor, stream=None) -> None:
    rows = md_thermo_rows(nsteps, thermo_every, setup)
    _check(lib().md_step(ctypes.byref(state.c), ctypes.byref(pot), ctypes.byref(box),
                         ctypes.byref(cells.c), ctypes.byref(nl.c), prec, kernel, skin, dt,
                         nsteps, thermo_every, setup,
                         _ptr(thermo, torch.float64, 8 * rows) if rows else None, _ptr(ws),
                         ws.numel(), _stream(stream)), "md_step")


class NHC:
    """Nose-Hoover chain thermostat: parameters plus its device state (zero
    for a fresh thermostat; md_step_nvt updates it in place)."""

    def __init__(self, t_target: float, t_damp: float, chain: int = 3, device="cuda"):
        self.state = torch.zeros(MD_NHC_STATE, dtype=torch.float64, device=device)
        self.c = md_nhc(t_target=t_target, t_damp=t_damp, chain=chain,
                        state=self.state.data_ptr())

    @property
    def chain_energy(self) -> float:
        return float(self.state[2 * MD_NHC_MAX].item())


def md_step_nvt(state: State, pot: md_potential, box: md_box, cells: Cells, nl: NList, prec: int,
                kernel: int, skin: float, dt: float, nhc: NHC, nsteps: int, thermo_every: int,
                setup: int, thermo: Optional[torch.Tensor], ws: torch.Tensor,
                stream=None) -> None:
    """thermo: rows x 9 doubles (md_step's eight and the conserved energy)."""
    rows = md_thermo_rows(nsteps, thermo_every, setup)
    _check(lib().md_step_nvt(ctypes.byref(state.c), ctypes.byref(pot), ctypes.byref(box),
                             ctypes.byref(cells.c), ctypes.byref(nl.c), prec, kernel, skin, dt,
                             ctypes.byref(nhc.c), nsteps, thermo_every, setup,
                             _ptr(thermo, torch.float64, 9 * rows) if rows else None, _ptr(ws),
                             ws.numel(), _stream(stream)), "md_step_nvt")


class NPT:
    """Isotropic barostat with Nose-Hoover chains: parameters plus its device
    state (zero for a fresh barostat; md_step_npt updates it in place)."""

    def __init__(self, t_target: float, t_damp: float, chain: int, p_target: float,
                 p_damp: float, device="cuda"):
        self.state = torch.zeros(MD_NPT_STATE, dtype=torch.float64, device=device)
        self.c = md_npt(t_target=t_target, t_damp=t_damp, chain=chain, p_target=p_target,
                        p_damp=p_damp, state=self.state.data_ptr())


def md_step_npt(state: State, pot: md_potential, box: md_box, cells: Cells, nl: NList,
                prec: int, kernel: int, skin: float, dt: float, npt: NPT, nsteps: int,
                thermo_every: int, setup: int, thermo: Optional[torch.Tensor], ws: torch.Tensor,
                stream=None) -> None:
    """thermo: rows x 10 doubles (md_step's eight, the conserved extended
    energy, the volume).  box is updated in place to the final box."""
    rows = md_thermo_rows(nsteps, thermo_every, setup)
    _check(lib().md_step_npt(ctypes.byref(state.c), ctypes.byref(pot), ctypes.byref(box),
                             ctypes.byref(cells.c), ctypes.byref(nl.c), prec, kernel, skin, dt,
                             ctypes.byref(npt.c), nsteps, thermo_every, setup,
                             _ptr(thermo, torch.float64, 10 * rows) if rows else None, _ptr(ws),
                             ws.numel(), _stream(stream)), "md_step_npt")


def md_force_vjp(pot: md_potential, x: torch.Tensor, box: md_box, nl: NList, prec: int,
                 u: torch.Tensor, gx: torch.Tensor, gparam: Optional[torch.Tensor],
                 ws: torch.Tensor, stream=None) -> None:
    n = x.shape[1]
    _check_list(nl, n, "md_force_vjp")
    _check(lib().md_force_vjp(ctypes.byref(pot), _ptr(x, torch.float64, 3 * n), n,
                              ctypes.byref(box), ctypes.byref(nl.c), prec,
                              _ptr(u, torch.float64, 3 * n), _ptr(gx, torch.float64, 3 * n),
                              _ptr(gparam, torch.float64, 3 if pot.kind == MD_POT_SC else 2),
                              _ptr(ws), ws.numel(),
                              _stream(stream)), "md_force_vjp")


def md_autoselect(pot: md_potential, x: torch.Tensor, box: md_box, cells: Cells, skin: float,
                  nl: NList, prec: int, reps: int, ws: torch.Tensor, stream=None) -> int:
    n = x.shape[1]
    _check_list(nl, n, "md_autoselect")
    choice = ctypes.c_int(0)
    _check(lib().md_autoselect(ctypes.byref(pot), _ptr(x, torch.float64, 3 * n), n,
                               ctypes.byref(box), ctypes.byref(cells.c), skin, ctypes.byref(nl.c),
                               prec, reps, ctypes.byref(choice), _ptr(ws), ws.numel(),
                               _stream(stream)), "md_autoselect")
    return choice.value


def md_nlist_status(nl: NList, stream=None) -> list:
    words = (ctypes.c_int * MD_STATUS_WORDS)()
    _check(lib().md_nlist_status(ctypes.byref(nl.c), words, _stream(stream)), "md_nlist_status")
    return list(words)


def md_timing_enable(every: int) -> None:
    _check(lib().md_timing_enable(int(every)), "md_timing_enable")


def md_timing_read():
    """(timed launches, summed duration in ms) since the last read."""
    n = ctypes.c_int64(0)
    ms = ctypes.c_double(0.0)
    _check(lib().md_timing_read(ctypes.byref(n), ctypes.byref(ms)), "md_timing_read")
    return n.value, ms.value
