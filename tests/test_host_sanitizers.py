"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

- The C-ABI library's host code (validation, sizes, index maps, work
  decomposition) is built with the host sanitizers together with a C++ driver
  (tests/host_sanitize/abi_driver.cpp) and stand-ins for the kernel launchers,
  which the driven entry points never reach; the driver must finish clean,
  leak check included.
- The oracle is built with the same sanitizers and runs its pin tests in a
  child Python process with the sanitizer runtime preloaded.  A copy with a
  planted out-of-bounds read shows the tier reports such a defect.

Device code is not sanitized here (GPU sanitizers are not part of this
build): the hipcc line keeps the sanitizers on the host side.
"""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

from oracle import build as oracle_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
PINS = ["tests/test_oracle_closed_form.py", "tests/test_oracle_wick.py", "tests/test_oracle_arrays.py",
        "tests/test_oracle_invariants.py", "tests/test_oracle_compensated.py", "tests/test_oracle_gsigma.py",
        "tests/test_oracle_spin_channels.py", "tests/test_oracle_multiorbital.py"]


def _libasan():
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_abi_host_code_under_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "abi_driver")
        src = [os.path.join(ROOT, "paper_2105_00027_amd", "csrc", "g4_abi.cpp"),
               os.path.join(ROOT, "tests", "host_sanitize", "launch_stubs.cpp"),
               os.path.join(ROOT, "tests", "host_sanitize", "abi_driver.cpp")]
        # host-only translation units: no device code is built, and
        # -fno-gpu-sanitize keeps the sanitizers off any device pass
        r = subprocess.run(["hipcc", "-std=c++17", *SAN, "-fno-gpu-sanitize", "-I", os.path.join(ROOT, "include"),
                            *src, "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        run = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                             env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                                      UBSAN_OPTIONS="print_stacktrace=1"))
        assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
        assert "host ABI checks passed" in run.stdout


def _sanitized_oracle(tmp, source_text, name):
    path = os.path.join(tmp, name + ".c")
    with open(path, "w") as f:
        f.write(source_text)
    lib = os.path.join(tmp, name + ".so")
    flags = [f for f in oracle_build.CFLAGS if f != "-O2"]
    subprocess.run(["gcc", *SAN, *flags, path, "-o", lib, "-lm"], check=True)
    return lib


def _run_pins(lib, asan):
    env = dict(os.environ, G4_ORACLE_LIB=lib, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0",
               OMP_NUM_THREADS="2", PYTHONDONTWRITEBYTECODE="1")
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "--capture=sys",
                           "-k", "not sampled", *PINS], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=900)


@pytest.mark.skipif(_libasan() is None, reason="gcc AddressSanitizer runtime not available")
def test_oracle_pins_under_sanitizers():
    asan = _libasan()
    with open(oracle_build.SRC) as f:
        src = f.read()
    with tempfile.TemporaryDirectory() as tmp:
        r = _run_pins(_sanitized_oracle(tmp, src, "oracle_san"), asan)
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
        # planted defect: read one complex value before the start of G
        old = "const double *p = g + 2 * (r * ng + c);"
        assert src.count(old) == 1
        bad = src.replace(old, "const double *p = g + 2 * (r * ng + c) - (r == 0 && c == 0 ? 2 : 0);")
        r = _run_pins(_sanitized_oracle(tmp, bad, "oracle_oob"), asan)
        assert r.returncode != 0 and "AddressSanitizer" in (r.stdout + r.stderr), r.stdout[-2000:]
