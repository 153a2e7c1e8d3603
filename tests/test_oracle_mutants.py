"""Planted mistakes in the oracle: each must fail at least one pin.

A pin that a plausible mistake passes pins nothing.  Each case below copies
oracle/g4_oracle.c, plants one mistake by exact text substitution, builds the
copy with the oracle's own compiler flags into a temporary directory, and
runs the oracle's pin tests against it (G4_ORACLE_LIB points the oracle's
loader at the copy) in a child process, which must fail.  The pins are the
closed forms, the brute-force Wick contraction, the array formulation, the
invariants, the exact compensated sums and the G_sigma pins; the numpy per-entry oracle's
comparison with the C oracle is left out, so that only the pins count.

Everything runs on the CPU; the HIP library is not involved.
"""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

from oracle import build as oracle_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_closed_form.py", "tests/test_oracle_wick.py",
        "tests/test_oracle_arrays.py", "tests/test_oracle_invariants.py",
        "tests/test_oracle_compensated.py", "tests/test_oracle_gsigma.py",
        "tests/test_oracle_spin_channels.py", "tests/test_oracle_multiorbital.py"]

# name -> (text in the oracle source, replacement)
MUTANTS = {
    # compensated accumulation
    "compensation dropped": (
        "cc[j] += (sum - tt) + x[j];\n                        else\n"
        "                            cc[j] += (x[j] - tt) + sum;",
        "(void)0;\n                        else\n                            (void)0;"),
    "compensation sign flipped": (
        "cc[j] += (sum - tt) + x[j];", "cc[j] -= (sum - tt) + x[j];"),
    "compensation without the magnitude test": (
        "if (fabs(sum) >= fabs(x[j]))", "if (1)"),
    # particle-hole terms
    "exchange sign": (
        "t = c_sub(direct, c_add(ex_u, ex_d));", "t = c_add(direct, c_add(ex_u, ex_d));"),
    "k1-q for k1+q": (
        "g_index(s, mom_add(s, k1, q), n1 + m);   /* K1 + Q */", "g_index(s, mom_sub(s, k1, q), n1 + m);"),
    "transposed exchange operand": (
        "cplx ex_u = c_mul(g_at(gu, ng, r_k2, r_k1), g_at(gu, ng, r_k1q, r_k2q));",
        "cplx ex_u = c_mul(g_at(gu, ng, r_k2, r_k1), g_at(gu, ng, r_k2q, r_k1q));"),
    "transposed direct operand": (
        "cplx u1 = g_at(gu, ng, r_k1q, r_k1), d1 = g_at(gd, ng, r_k1q, r_k1);",
        "cplx u1 = g_at(gu, ng, r_k1, r_k1q), d1 = g_at(gd, ng, r_k1, r_k1q);"),
    "charge and magnetic spin weights swapped": (
        "            cplx a = channel == ORACLE_PH_MAGNETIC ? c_sub(u1, d1) : c_add(u1, d1);",
        "            cplx a = channel == ORACLE_PH_MAGNETIC ? c_add(u1, d1) : c_sub(u1, d1);"),
    # particle-particle term, Eq. (1)
    "transposed PP operand": (
        "cplx up = c_mul(g_at(gu, ng, r_qk2, r_qk1)", "cplx up = c_mul(g_at(gu, ng, r_qk1, r_qk2)"),
    "PP same spin for the opposite spin": (
        "g_at(gd, ng, r_k2, r_k1));\n        cplx dn", "g_at(gu, ng, r_k2, r_k1));\n        cplx dn"),
    "PP frequency n2 for n1 in Q-K1": (
        "mom_sub(s, q, k1), m - n1 - 1); /* Q - K1 */", "mom_sub(s, q, k1), m - n2 - 1);"),
    "PP frequency off by one": (
        "mom_sub(s, q, k2), m - n2 - 1); /* Q - K2 */", "mom_sub(s, q, k2), m - n2);"),
    # spin-resolved particle-hole channels
    "up-up exchange dropped": (
        "t = c_sub(direct, ex);", "t = direct;"),
    "up-down spins swapped": (
        "t = c_mul(g_at(gu, ng, r_k1q, r_k1), g_at(gd, ng, r_k2, r_k2q));",
        "t = c_mul(g_at(gd, ng, r_k1q, r_k1), g_at(gu, ng, r_k2, r_k2q));"),
    "transverse with equal spins": (
        "cplx ex_du = c_mul(g_at(gd, ng, r_k2, r_k1), g_at(gu, ng, r_k1q, r_k2q));",
        "cplx ex_du = c_mul(g_at(gu, ng, r_k2, r_k1), g_at(gu, ng, r_k1q, r_k2q));"),
    "transverse sign": (
        "t = c_sub(zero, c_add(ex_du, ex_ud));", "t = c_add(zero, c_add(ex_du, ex_ud));"),
    # PP singlet / triplet
    "PP crossed term with Q-K1 for K1": (
        "c_mul(g_at(gu, ng, r_qk2, r_k1), g_at(gd, ng, r_k2, r_qk1))",
        "c_mul(g_at(gu, ng, r_qk2, r_qk1), g_at(gd, ng, r_k2, r_qk1))"),
    "PP crossed term with equal spins": (
        "c_mul(g_at(gd, ng, r_qk2, r_k1), g_at(gu, ng, r_k2, r_qk1))",
        "c_mul(g_at(gu, ng, r_qk2, r_k1), g_at(gu, ng, r_k2, r_qk1))"),
    "PP singlet and triplet swapped": (
        "cplx sum = channel == ORACLE_PP_SINGLET ? c_add(t, crossed) : c_sub(t, crossed);",
        "cplx sum = channel == ORACLE_PP_SINGLET ? c_sub(t, crossed) : c_add(t, crossed);"),
    "PP projection without the 1/2": (
        "t.re = 0.5 * sum.re;", "t.re = sum.re;"),
    # multi-orbital labels
    "MO exchange with b1 and b4 swapped": (
        "mo_g(gu, ngb, r_k1q, b1, r_k2q, b4, nb));", "mo_g(gu, ngb, r_k1q, b4, r_k2q, b1, nb));"),
    "MO direct with b3 and b4 swapped": (
        "cplx u2 = mo_g(gu, ngb, r_k2, b3, r_k2q, b4, nb)", "cplx u2 = mo_g(gu, ngb, r_k2, b4, r_k2q, b3, nb)"),
    "MO PP with b1 and b2 swapped": (
        "cplx up = c_mul(mo_g(gu, ngb, r_qk2, b4, r_qk1, b2, nb), mo_g(gd, ngb, r_k2, b3, r_k1, b1, nb));",
        "cplx up = c_mul(mo_g(gu, ngb, r_qk2, b4, r_qk1, b1, nb), mo_g(gd, ngb, r_k2, b3, r_k1, b2, nb));"),
    "MO magnetic and charge spin weights swapped": (
        "\n        cplx a = channel == ORACLE_PH_MAGNETIC ? c_sub(u1, d1) : c_add(u1, d1);",
        "\n        cplx a = channel == ORACLE_PH_MAGNETIC ? c_add(u1, d1) : c_sub(u1, d1);"),
    "MO G index with the orbital slowest": (
        "return g_at(g, ngb, r * nb + br, c * nb + bc);",
        "return g_at(g, ngb, br * (ngb / nb) + r, bc * (ngb / nb) + c);"),
    # G_sigma from an expansion configuration
    "G_sigma: conjugate phase on the left factor": (
        "const cplx ea = {cos(tha), sin(tha)};", "const cplx ea = {cos(tha), -sin(tha)};"),
    "G_sigma: normalisation dropped": (
        "const double norm = 1.0 / (beta * (double)nc);", "const double norm = 1.0;"),
    "G_sigma: k.r with the wrong sign": (
        "const double tha = w1 * tau[a] + 2.0 * pi *", "const double tha = w1 * tau[a] - 2.0 * pi *"),
    "G_sigma: spin ignored in g0": (
        "const double sg = spin == 0 ? 1.0 : -1.0;", "const double sg = 1.0;"),
}


def _build_mutant(tmp, name, old, new):
    with open(oracle_build.SRC) as f:
        src = f.read()
    assert src.count(old) == 1, "mutation site not found once for %r" % name
    path = os.path.join(tmp, "mutant_%d.c" % abs(hash(name)))
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = path[:-2] + ".so"
    subprocess.run(["gcc", *oracle_build.CFLAGS, path, "-o", lib, "-lm"], check=True)
    return lib


def _run_pins(lib):
    # no bytecode writes: four child test runs share the tests' __pycache__
    env = dict(os.environ, G4_ORACLE_LIB=lib, OMP_NUM_THREADS="2", PYTHONDONTWRITEBYTECODE="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "--capture=sys",
                        "-k", "not sampled", *PINS], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout + r.stderr


def test_unmutated_copy_passes_the_pins():
    """The harness itself: an unchanged copy built the same way passes."""
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_mutant(tmp, "none", "int oracle_max_threads(void)", "int oracle_max_threads(void)")
        rc, out = _run_pins(lib)
    assert rc == 0, out[-3000:]


def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        libs = {name: _build_mutant(tmp, name, old, new) for name, (old, new) in MUTANTS.items()}
        with cf.ThreadPoolExecutor(max_workers=4) as ex:
            results = dict(zip(libs, ex.map(_run_pins, libs.values())))
    survivors = [name for name, (rc, _) in results.items() if rc == 0]
    assert not survivors, "planted mistakes that pass every pin: %s" % survivors
    # a mutant fails by a failed assertion, or by the oracle's own check that
    # every frequency it reads lies in the G window (an abort); nothing else
    for name, (rc, out) in results.items():
        window = rc in (-6, 134) and "outside the G window" in out
        assert rc == 1 or window, "%s: pytest exit %d\n%s" % (name, rc, out[-3000:])
