"""The ABI host tests rerun against a build of the library whose host code
for the boundary calls (md_api.hip: argument checks, layouts, workspace and
status handling) carries AddressSanitizer and UBSan (no GPU): a child process
with clang's ASan runtime preloaded loads it through MD_LIB_PATH.  Any
out-of-bounds access or undefined behaviour, an invalid enum value included,
fails the run."""
import glob
import os
import subprocess
import sys

import pytest

from paper_1009_4330_amd import build as hip_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_host_code_under_asan_and_ubsan():
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("no clang ASan runtime in /opt/rocm/llvm")
    try:
        san = hip_build.build_sanitized()
    except RuntimeError as e:   # the regular objects are not built
        pytest.skip(str(e))
    preload = [rt[-1]] + ([os.environ["LD_PRELOAD"]] if os.environ.get("LD_PRELOAD") else [])
    env = dict(os.environ, LD_PRELOAD=":".join(preload), MD_LIB_PATH=san,
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    which = subprocess.run([sys.executable, "-c",
                            "from paper_1009_4330_amd import md; print(md.lib()._name)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert which.returncode == 0 and which.stdout.strip() == san, which.stdout + which.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider",
                        "tests/test_abi.py"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in r.stdout
