"""Pin of the oracle's compensated accumulation mode against exact sums.

The oracle's optional compensated mode adds each weighted term s_b T_b with
Neumaier's error-free update (the running sum and a separate running
compensation, value = sum + compensation).  Its use is to bound the oracle's
own rounding when long runs are compared, as the paper's accuracy analysis
does (Results section, "Accuracy Analysis", Eq. (2) and Eq. (3)).

Pinned here by what the mathematics fixes, independently of the oracle:
G matrices with small integer entries make every product T_b an exact small
Gaussian integer; weights that are signed powers of two (some near 2^60,
some of order one) make every s_b T_b exact in FP64.  The exact sum is then
computed with Python's arbitrary-precision rationals.  With huge terms that
cancel, the plain FP64 sum loses the small ones entirely, while a correct
compensated sum returns the exact value (its error bound, 2u|S| plus a term of
order n u^2 sum|x|, is far below one unit of the exact result here).  The
first test shows the plain sum fails that bound on these inputs, so the pin
has teeth; tests/test_oracle_mutants.py checks that a dropped, sign-flipped
or misapplied compensation fails it.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import ref
from synth import Workload

# 1x1 cluster, two frequencies, one plane: 4 entries, 2x2 G matrices
W = Workload("comp", lx=1, ly=1, nw=2, nwex=1, nq=1, beta=5.0)


def _inputs(seed, count):
    """Triples of measurements (big, small, -big): the first and third share
    their G matrices and carry opposite weights near 2^60, so their terms
    cancel exactly; the middle one has a weight of order one.  The plain sum
    rounds the middle term away against the big one; the exact sum is the sum
    of the middle terms."""
    rng = np.random.default_rng(seed)

    def draw():
        return (rng.integers(-3, 4, size=(W.ng, W.ng))
                + 1j * rng.integers(-3, 4, size=(W.ng, W.ng))).astype(np.complex128)

    gu = np.empty((count, W.ng, W.ng), dtype=np.complex128)
    gd = np.empty_like(gu)
    s = np.empty(count)
    for b in range(count):
        if b % 3 == 2:                      # undo the big term of b - 2
            gu[b], gd[b], s[b] = gu[b - 2], gd[b - 2], -s[b - 2]
            continue
        gu[b], gd[b] = draw(), draw()
        sgn = float(rng.choice([-1.0, 1.0]))
        s[b] = sgn * 2.0 ** int(rng.integers(55, 62) if b % 3 == 0 else rng.integers(-3, 3))
    return gu, gd, s


def _exact(channel, gu, gd, s):
    """Exact rational sum of s_b T_b per entry; T_b from one-measurement oracle
    calls (an exact Gaussian integer for these inputs, checked)."""
    out = [[Fraction(0), Fraction(0)] for _ in range(W.entries)]
    for b in range(len(s)):
        t = ref.accumulate(W, channel, gu[b:b + 1], gd[b:b + 1], np.ones(1)).reshape(-1)
        for e in range(W.entries):
            assert t[e].real == int(t[e].real) and t[e].imag == int(t[e].imag)
            out[e][0] += Fraction(s[b]) * int(t[e].real)
            out[e][1] += Fraction(s[b]) * int(t[e].imag)
    return out


def _max_abs_dev(val, exact):
    dev = 0.0
    for e in range(W.entries):
        for j, part in enumerate((val[e].real, val[e].imag)):
            dev = max(dev, abs(float(Fraction(part) - exact[e][j])))
    return dev


@pytest.mark.parametrize("channel", [ref.PH_MAGNETIC, ref.PH_CHARGE, ref.PP_UPDOWN])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_compensated_sum_is_exact_where_plain_is_not(channel, seed):
    count = 60
    gu, gd, s = _inputs(seed, count)
    exact = _exact(channel, gu, gd, s)
    plain = ref.accumulate(W, channel, gu, gd, s).reshape(-1)
    g4 = np.zeros((W.planes, W.n, W.n), dtype=np.complex128)
    comp = np.zeros_like(g4)
    ref.accumulate(W, channel, gu, gd, s, g4=g4, comp=comp)
    val = (g4 + comp).reshape(-1)
    # the compensated value is the exact sum (all exact sums here are small
    # dyadic rationals, representable in FP64)
    assert _max_abs_dev(val, exact) == 0.0
    # the plain sum is off by at least one of the O(1) terms: the test can tell
    assert _max_abs_dev(plain, exact) >= 0.125


def test_compensated_matches_plain_on_benign_inputs():
    """Without cancellation both modes agree to FP64 rounding (the compensation
    stays at rounding size)."""
    gu, gd, s = _inputs(9, 30)
    s = np.abs(s) / np.abs(s).max() + 0.5
    plain = ref.accumulate(W, ref.PH_MAGNETIC, gu, gd, s)
    g4 = np.zeros_like(plain)
    comp = np.zeros_like(plain)
    ref.accumulate(W, ref.PH_MAGNETIC, gu, gd, s, g4=g4, comp=comp)
    scale = np.abs(plain).max()
    assert np.abs((g4 + comp) - plain).max() <= 64 * np.finfo(float).eps * scale
    assert np.abs(comp).max() <= 64 * np.finfo(float).eps * scale
