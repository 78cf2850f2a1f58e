"""Buffers and run loop for one MD system on the GPU (host-side plumbing).

MDSystem owns the device state, cell arrays, neighbour list and workspace for
a workload and drives md_step in chunks.  When a list build overflows its
capacity, the chunk is rerun from a device copy of the state taken before it,
with the capacity raised to the required count plus headroom.
"""
from __future__ import annotations

import json
import math
from typing import Optional

import numpy as np
import torch

from . import md
from .inputs import Workload, pair_table

PREC = {"fp64": md.MD_FP64, "mixed": md.MD_MIXED}

# Names of the thermo row columns md_step writes (NVE), and the ones the NVT
# and NPT variants append.
THERMO_COLUMNS = ("step", "pe", "ke", "etotal", "temp", "press", "builds", "maxneigh")
THERMO_NVT = THERMO_COLUMNS + ("conserved",)
THERMO_NPT = THERMO_COLUMNS + ("conserved", "volume")
_THERMO_INTS = ("step", "builds", "maxneigh")


def thermo_records(rows: np.ndarray, columns=THERMO_COLUMNS) -> list:
    """Thermo rows as dicts keyed by column name; step, build count and the
    largest neighbour count as integers, the rest as floats."""
    rows = np.asarray(rows, dtype=np.float64)
    if rows.ndim != 2 or rows.shape[1] != len(columns):
        raise ValueError(f"thermo rows of {len(columns)} columns expected, got shape {rows.shape}")
    return [{c: (int(v) if c in _THERMO_INTS else float(v)) for c, v in zip(columns, r)}
            for r in rows]


def write_thermo_jsonl(fh, rows: np.ndarray, columns=THERMO_COLUMNS) -> None:
    """Append thermo rows to an open text file, one JSON object per line
    (floats written with full round-trip precision)."""
    for rec in thermo_records(rows, columns):
        fh.write(json.dumps(rec) + "\n")
KERNEL = {"auto": md.MD_KERNEL_AUTO, "tpa": md.MD_KERNEL_TPA, "wpa": md.MD_KERNEL_WPA,
          **{f"k{k}": k for k in md.LANES},
          **{f"t{k}": md.MD_LAYOUT_TILE | k for k in md.TILE_LANES}}


def potential_of(w: Workload, type_tensor: Optional[torch.Tensor] = None,
                 **over) -> md.md_potential:
    """The workload's potential; Buckingham needs the device species tensor."""
    if w.potential == "lj":
        return md.lj_potential(w.rc, over.get("eps", w.lj_eps), over.get("sigma", w.lj_sigma),
                               w.lj_shift)
    if w.potential == "buck":
        if type_tensor is None:
            raise ValueError("Buckingham needs a species tensor")
        return md.buck_potential(w.rc, pair_table(w, "buck_A"), pair_table(w, "buck_rho"),
                                 pair_table(w, "buck_C"), w.charges, w.qqr2e, type_tensor)
    return md.sc_potential(w.rc, w.sc_eps, w.sc_a, w.sc_c, w.sc_n, w.sc_m)


def capacity_guess(w: Workload) -> int:
    """Neighbour capacity from the mean count in the list sphere, with
    headroom for density fluctuations of a liquid."""
    rho = (8.0 if w.lattice == "rocksalt" else 4.0) / w.a ** 3
    mean = rho * 4.0 / 3.0 * math.pi * (w.rc + w.skin) ** 3
    return int(mean * 1.35 + 4.0 * math.sqrt(mean) + 16)


class MDSystem:
    def __init__(self, w: Workload, x: np.ndarray, v: np.ndarray, prec: str = "fp64",
                 kernel: str = "tpa", capacity: Optional[int] = None, device="cuda",
                 nvt: Optional[tuple] = None, npt: Optional[tuple] = None,
                 thermo_jsonl: Optional[str] = None):
        """nvt = (t_target, t_damp, chain length) runs md_step_nvt (thermo rows
        of nine columns); npt = (t_target, t_damp, chain length, p_target,
        p_damp) runs md_step_npt (ten columns, the box in self.box follows the
        run) instead of NVE md_step.  thermo_jsonl: a file that every thermo
        row setup() and run() return is appended to, one JSON object per row
        (columns THERMO_COLUMNS, THERMO_NVT or THERMO_NPT)."""
        self.w = w
        self.device = device
        self.nhc = md.NHC(*nvt, device=device) if nvt else None
        self.npt = md.NPT(*npt, device=device) if npt else None
        self.cols = 10 if npt else (9 if nvt else 8)
        self.columns = THERMO_NPT if npt else (THERMO_NVT if nvt else THERMO_COLUMNS)
        self.thermo_jsonl = thermo_jsonl
        self.prec = PREC[prec]
        self.kernel = KERNEL[kernel]
        self.box = md.make_box(w.box)
        n = x.shape[1]
        # species, permuted by md_step along with the atoms (Buckingham only)
        self.type = (torch.as_tensor(w.species(), dtype=torch.int32, device=device)
                     if w.potential == "buck" else None)
        self.pot = potential_of(w, self.type)
        self.rl = w.rc + w.skin
        self.n = n
        u = w.units
        self.state = md.State(torch.as_tensor(x, dtype=torch.float64, device=device),
                              torch.as_tensor(v, dtype=torch.float64, device=device),
                              w.mass, u.ftm2v, u.mvv2e, u.boltz)
        ncell = int(np.prod([math.floor(L / self.rl) for L in w.box]))
        self.cells = md.Cells(n, ncell, device)
        self.nl = self._nlist(capacity or capacity_guess(w), md.MD_LAYOUT_TPA)
        self.ws = md.workspace(n, self.box, self.rl, device)
        self.ready = False
        self.steps_done = 0

    # -- helpers -------------------------------------------------------------
    def _nlist(self, cap: int, layout: int) -> md.NList:
        """A list of this capacity, with the tiled layouts' buffer where they
        apply (LJ; enough cells)."""
        tiles = (md.md_nlist_tile_entries(self.n, cap, self.box, self.rl)
                 if self.w.potential == "lj" else 0)
        return md.NList(self.n, cap, layout, self.device, tile_entries=tiles)

    def _tensors(self):
        s = self.state
        out = [s.x, s.v, s.f, s.id, self.nl.x_ref, self.nl.status]
        out += [self.type] if self.type is not None else []
        out += [self.npt.state] if self.npt is not None else []
        return out + ([self.nhc.state] if self.nhc is not None else [])

    def _snapshot(self):
        return tuple(t.clone() for t in self._tensors()), tuple(self.box.L)

    def _restore(self, snap):
        tensors, box = snap
        for dst, src in zip(self._tensors(), tensors):
            dst.copy_(src)
        for d in range(3):
            self.box.L[d] = box[d]

    def _grow(self, need: int):
        cap = int(need * 1.2) + 16
        self.nl = self._nlist(cap, self.nl.layout)

    def _step(self, kernel, nsteps, every, setup, rows):
        if self.npt is not None:
            md.md_step_npt(self.state, self.pot, self.box, self.cells, self.nl, self.prec, kernel,
                           self.w.skin, self.w.dt, self.npt, nsteps, every, setup, rows, self.ws)
        elif self.nhc is None:
            md.md_step(self.state, self.pot, self.box, self.cells, self.nl, self.prec, kernel,
                       self.w.skin, self.w.dt, nsteps, every, setup, rows, self.ws)
        else:
            md.md_step_nvt(self.state, self.pot, self.box, self.cells, self.nl, self.prec,
                           kernel, self.w.skin, self.w.dt, self.nhc, nsteps, every, setup, rows,
                           self.ws)

    def setup(self, thermo: bool = True) -> Optional[np.ndarray]:
        """Wrap, bin, sort, build and evaluate forces for the current state."""
        while True:
            snap = self._snapshot()
            rows = (torch.zeros(1, self.cols, dtype=torch.float64, device=self.device)
                    if thermo else None)
            try:
                self._step(self.kernel, 0, 1, 1, rows)
            except md.MDError as e:
                if e.code != md.MD_ERR_NLIST_OVERFLOW:
                    raise
                need = md.md_nlist_status(self.nl)[md.MD_ST_MAXNEIGH]
                self._restore(snap)
                self._grow(need)
                continue
            self.ready = True
            self.kernel = self.nl.layout      # lanes per atom the run settled on
            if not thermo:
                return None
            r = rows.cpu().numpy()
            r[:, 0] += self.steps_done
            self._log(r)
            return r

    def run(self, nsteps: int, thermo_every: int = 0, chunk: int = 0) -> np.ndarray:
        """Advance nsteps; returns thermo rows (every thermo_every steps)."""
        if not self.ready:
            self.setup(thermo=False)
        every = thermo_every if thermo_every > 0 else max(nsteps, 1)
        chunk = chunk or nsteps
        out = []
        done = 0
        while done < nsteps:
            k = min(chunk, nsteps - done)
            rows_n = md.md_thermo_rows(k, every, 0)
            snap = self._snapshot()
            th = torch.zeros(max(rows_n, 1), self.cols, dtype=torch.float64, device=self.device)
            try:
                self._step(self.kernel, k, every, 0, th if rows_n else None)
            except md.MDError as e:
                if e.code != md.MD_ERR_NLIST_OVERFLOW:
                    raise
                need = md.md_nlist_status(self.nl)[md.MD_ST_MAXNEIGH]
                self._restore(snap)
                self._grow(need)
                self.ready = False
                self.setup(thermo=False)
                continue
            if rows_n:
                r = th[:rows_n].cpu().numpy()
                r[:, 0] += self.steps_done
                self._log(r)
                out.append(r)
            done += k
            self.steps_done += k
        return np.concatenate(out) if out else np.zeros((0, self.cols))

    def _log(self, rows: np.ndarray) -> None:
        if self.thermo_jsonl and len(rows):
            with open(self.thermo_jsonl, "a") as fh:
                write_thermo_jsonl(fh, rows, self.columns)

    # -- checkpoint / resume ----------------------------------------------------
    def checkpoint(self, path: str) -> None:
        """Write everything a continuing md_step reads to an .npz file: the
        state (x, v, f, ids, species), the list (entries, lengths, reference
        positions, tile entries), the cell starts and cells of its build, the
        status words, thermostat / barostat state, box, layout and steps done.
        A run restored from it continues bit for bit as if never stopped."""
        if not self.ready:
            raise RuntimeError("checkpoint before setup: nothing to save")
        torch.cuda.synchronize()
        host = lambda t: t.detach().cpu().numpy()
        d = dict(x=host(self.state.x), v=host(self.state.v), f=host(self.state.f),
                 id=host(self.state.id), x_ref=host(self.nl.x_ref), neigh=host(self.nl.neigh),
                 numneigh=host(self.nl.numneigh), status=host(self.nl.status),
                 cell_start=host(self.cells.cell_start), atom_cell=host(self.cells.atom_cell),
                 perm=host(self.cells.perm), nc=np.array(list(self.cells.c.nc)),
                 box=np.array(list(self.box.L)), layout=np.array(self.nl.layout),
                 capacity=np.array(self.nl.capacity), rl=np.array(self.nl.c.rl),
                 steps_done=np.array(self.steps_done), prec=np.array(self.prec))
        if self.type is not None:
            d["type"] = host(self.type)
        if self.nl.tile is not None:
            d["tile"] = host(self.nl.tile)
        if self.nhc is not None:
            d["nhc"] = host(self.nhc.state)
        if self.npt is not None:
            d["npt"] = host(self.npt.state)
        np.savez(path, **d)

    def restore(self, path: str) -> None:
        """Load a checkpoint written by checkpoint() for a system of the same
        workload, atom count and ensemble; the next run() continues it."""
        with np.load(path, allow_pickle=False) as z:
            if int(z["prec"]) != self.prec:
                raise ValueError("checkpoint was taken in another precision")
            if ("nhc" in z) != (self.nhc is not None) or ("npt" in z) != (self.npt is not None):
                raise ValueError("checkpoint was taken in another ensemble")
            if z["x"].shape[1] != self.n:
                raise ValueError("checkpoint holds another atom count")
            layout = int(z["layout"])
            self.nl = self._nlist(int(z["capacity"]), layout)
            if ("tile" in z) and self.nl.tile is None:
                raise ValueError("checkpoint has a tiled list this system cannot hold")
            dev = lambda a, t: t.copy_(torch.as_tensor(a))
            dev(z["x"], self.state.x)
            dev(z["v"], self.state.v)
            dev(z["f"], self.state.f)
            dev(z["id"], self.state.id)
            dev(z["x_ref"], self.nl.x_ref)
            dev(z["neigh"], self.nl.neigh)
            dev(z["numneigh"], self.nl.numneigh)
            dev(z["status"], self.nl.status)
            dev(z["cell_start"], self.cells.cell_start)
            dev(z["atom_cell"], self.cells.atom_cell)
            dev(z["perm"], self.cells.perm)
            if "tile" in z:
                dev(z["tile"], self.nl.tile)
            if self.type is not None:
                dev(z["type"], self.type)
            if self.nhc is not None:
                dev(z["nhc"], self.nhc.state)
            if self.npt is not None:
                dev(z["npt"], self.npt.state)
            for q in range(3):
                self.cells.c.nc[q] = int(z["nc"][q])
                self.box.L[q] = float(z["box"][q])
            self.nl.c.layout = layout
            self.nl.c.rl = float(z["rl"])
            self.kernel = layout
            self.steps_done = int(z["steps_done"])
        torch.cuda.synchronize()
        self.ready = True

    def host_state(self):
        """(x, v, f) as numpy [3][n] arrays in the caller's original atom order."""
        order = torch.argsort(self.state.id.long())
        get = lambda t: t[:, order].cpu().numpy()
        return get(self.state.x), get(self.state.v), get(self.state.f)
