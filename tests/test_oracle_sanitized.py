"""The oracle's pin tests rerun against an AddressSanitizer + UBSan build of
md_oracle.c (no GPU): a child process with gcc's libasan preloaded loads the
sanitized library through MD_ORACLE_LIB and runs the oracle test files; any
out-of-bounds access, use after free or undefined behaviour aborts it."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = ["tests/test_oracle.py", "tests/test_oracle_buck.py", "tests/test_oracle_nvt.py",
         "tests/test_oracle_npt.py", "tests/test_oracle_pressure.py",
         "tests/test_oracle_sc_vjp.py"]


def test_oracle_pins_under_asan_and_ubsan():
    libasan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc has no libasan")
    san = oracle.oracle.build_sanitized()
    preload = [libasan] + ([os.environ["LD_PRELOAD"]] if os.environ.get("LD_PRELOAD") else [])
    env = dict(os.environ, LD_PRELOAD=":".join(preload), MD_ORACLE_LIB=san,
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS=os.environ.get("OMP_NUM_THREADS", "8"))
    which = subprocess.run([sys.executable, "-c", "import oracle; print(oracle.oracle.lib()._name)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert which.returncode == 0 and which.stdout.strip() == san, which.stdout + which.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        *FILES], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in r.stdout
