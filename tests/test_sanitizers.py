"""CPU sanitizer run: the oracle and the library's host code (parameter
validation, layouts, the C ABI's argument checks) built with
AddressSanitizer and UndefinedBehaviorSanitizer, under which the ABI tests
and the oracle's exact pins run in a child process.  Any sanitizer report
fails the test.  No GPU: the host-sanitized library has no device code."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (the complex-step build's bit-for-bit comparison with the real build is a
# property of the gcc build, which the sanitizer build, made with clang, does
# not share; it is left out here)
TESTS = ["tests/test_abi.py", "tests/test_oracle_lattice.py", "tests/test_oracle_stencils.py",
         "tests/test_oracle_boundaries.py", "tests/test_oracle_budget.py", "tests/test_oracle_diagnostics.py"]


def _asan_runtime():
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.slow
def test_abi_and_oracle_pins_under_asan_ubsan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no clang AddressSanitizer runtime in this image")
    sys.path.insert(0, ROOT)
    from oracle import build as ob
    from paper_1310_1871_amd import build as pb
    ob.build(sanitize=True)
    lib = pb.build_host_sanitized()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": rt,
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "ORACLE_LIB_SUFFIX": "_san",
        "LBM_AXI_LIB": lib,
        "OMP_NUM_THREADS": "4",
    })
    # the ray-weight test compares with the oracle's diagnostics and calls
    # host code only; GPU-marked tests are not collected
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu and not slow", "-p", "no:cacheprovider",
           *TESTS]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
