"""Checkpoint / resume: a run stopped after 40 steps, written to disk, loaded
into a fresh system and continued for 60 steps equals the same run never
stopped (md_step calls of 40 and 60 steps in one process) bit for bit --
thermo rows, positions, velocities, forces, box -- in NVE FP64 and
FP32-mixed, under the NVT thermostat and under the barostat.  In NVE the
split run also equals one 100-step call (the NVT and NPT calls re-sum the
kinetic energy from v at their start, a rounding-level difference)."""
import os
import tempfile

import numpy as np
import pytest

from paper_1009_4330_amd import inputs as I
from paper_1009_4330_amd.system import MDSystem

pytestmark = pytest.mark.gpu

W = I.scaled(I.LJ_4K, 10)


@pytest.mark.parametrize("prec,ens", [("fp64", "nve"), ("mixed", "nve"), ("fp64", "nvt"),
                                      ("fp64", "npt")])
def test_resume_is_bitwise(prec, ens):
    x, v, box = I.initial_state(W)
    kw = {}
    if ens == "nvt":
        kw["nvt"] = (1.5, 0.5, 3)
    elif ens == "npt":
        kw["npt"] = (1.5, 0.5, 3, 2.0, 0.25)
    a = MDSystem(W, x, v, prec, "auto", **kw)
    a.setup(False)
    ra = np.concatenate([a.run(40, 10), a.run(60, 10)])
    if ens == "nve":
        one = MDSystem(W, x, v, prec, "auto", **kw)
        one.setup(False)
        assert np.array_equal(one.run(100, 10), ra)
    b = MDSystem(W, x, v, prec, "auto", **kw)
    b.setup(False)
    rb = b.run(40, 10)
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "ckpt.npz")
        b.checkpoint(path)
        # a fresh system, started from other positions, takes the saved run over
        c = MDSystem(W, I.jitter(x, 0.1, 3), np.zeros_like(v), prec, "auto", **kw)
        c.restore(path)
    rc = c.run(60, 10)
    assert rb[-1, 6] > 2 and ra[-1, 6] > rb[-1, 6]            # rebuilds on both sides
    assert np.array_equal(np.concatenate([rb, rc]), ra)
    assert tuple(c.box.L) == tuple(a.box.L)
    for ta, tc in zip(a.host_state(), c.host_state()):
        assert np.array_equal(ta, tc)
