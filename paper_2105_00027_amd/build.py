"""Build the HIP C-ABI library paper_2105_00027_amd/libg4.so for gfx950.

Every source is compiled by hipcc (objects under _build/, kept out of the
repository history), then linked into one shared library next to this file.
All device code is built with packed FP32 instructions disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build", "g4")
LIB = os.path.join(HERE, "libg4.so")
# (source, object name, extra defines); the update kernel is instantiated once
# per (kind, K2 rows per thread) pair, the packed-operand kernel once per K2
# rows per thread
SOURCES = [("g4_abi.cpp", "g4_abi", []), ("g4_kernels.hip", "g4_kernels", []),
           ("g4_synth.hip", "g4_synth", []), ("g4_update_mfma.hip", "g4_update_mfma", []),
           ("g4_direct.hip", "g4_direct", []), ("g4_noalloc.hip", "g4_noalloc", []),
           ("g4_gsigma.hip", "g4_gsigma", []), ("g4_multiorbital.hip", "g4_multiorbital", [])] + [
    ("g4_update_inst.hip", "g4_update_k%d_e%d" % (k, e), ["-DG4_KIND=%d" % k, "-DG4_EPT=%d" % e])
    for k in (0, 1, 2) for e in (1, 2, 4, 8)] + [
    ("g4_update_packed.hip", "g4_update_packed_e%d" % e, ["-DG4_EPT=%d" % e]) for e in (1, 2, 4, 8)]
ARCH = os.environ.get("G4_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(ROOT, "include")]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build_id() -> str:
    """SHA-1 (first 16 hex digits) over the library's sources and its header:
    compiled into the library so that autotuner choices stored by another
    build of the kernels are not reused."""
    import hashlib
    h = hashlib.sha1()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp", ".cpp")))
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    with open(os.path.join(ROOT, "include", "g4.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def _stale(src: str, obj: str) -> bool:
    """True when obj is missing or older than its source or any header."""
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, src)] + [os.path.join(d, f) for d in (CSRC, os.path.join(ROOT, "include"))
                                        for f in os.listdir(d) if f.endswith((".hpp", ".h"))]
    return max(os.path.getmtime(f) for f in deps) > os.path.getmtime(obj)


def _compile(spec, verbose: bool, incremental: bool = False) -> str:
    src, name, defs = spec
    obj = os.path.join(BUILD, name + ".o")
    if incremental and not src.endswith(".cpp") and not _stale(src, obj):
        return obj
    cmd = ["hipcc", *COMMON, *DEVICE, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        # the host code carries the build id (always recompiled: it changes
        # with any source)
        defs = defs + ['-DG4_BUILD_ID="%s"' % build_id()]
        cmd = ["hipcc", *COMMON, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on " + src)
    warn = "\n".join(l for l in (r.stderr or "").splitlines()
                     if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    if verbose and warn.strip():
        sys.stderr.write(warn + "\n")
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental: only those whose object is older than
    the source or a header) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(os.cpu_count() or 4, 16, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, incremental), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
