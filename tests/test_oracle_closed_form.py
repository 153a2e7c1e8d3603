"""Pin: noninteracting closed forms.

With no interaction the measured G is diagonal, G_s(X, Y) = delta_XY g_s(X),
and Wick's theorem reduces every channel to products of g:

  PH magnetic  S [ delta_{Q,0} (g_u - g_d)(K1) (g_u - g_d)(K2) - delta_{K1,K2} sum_s g_s(K1) g_s(K1+Q) ]
  PH charge    S [ delta_{Q,0} (g_u + g_d)(K1) (g_u + g_d)(K2) - delta_{K1,K2} sum_s g_s(K1) g_s(K1+Q) ]
  PP (Eq. 1)   S   delta_{K1,K2} sum_s g_s(Q-K1) g_{-s}(K1)
  PH up-up     S [ delta_{Q,0} g_u(K1) g_u(K2) - delta_{K1,K2} g_u(K1) g_u(K1+Q) ]
  PH up-down   S   delta_{Q,0} g_u(K1) g_d(K2)
  PH transv.  -S   delta_{K1,K2} [ g_u(K1) g_d(K1+Q) + g_d(K1) g_u(K1+Q) ]
  PP singlet / triplet  S/2 [ delta_{K1,K2} sum_s g_s(Q-K1) g_{-s}(K1)
                              +/- delta_{K2,Q-K1} sum_s g_s(K1) g_{-s}(Q-K1) ]
    (the second term where Q-K1 lies in the G4 frequency range)

with S the sum of the measurement signs.  Here g is evaluated from physical
momenta and Matsubara frequencies in floating point (k+q as a vector,
w_n + nu_m as a sum), never through the integer index maps, and the dispersion
has odd terms so that k+q, k-q and q-k all give different values.
"""
import math

import numpy as np
import pytest

from oracle import ref
from synth import Workload

T = 1.0
MU = 0.3


def eps(kx, ky):
    return (-2.0 * T * (np.cos(kx) + np.cos(ky)) + 0.37 * np.sin(kx) - 0.21 * np.sin(ky)
            + 0.13 * np.sin(kx + 2.0 * ky))


def gfun(w, sigma, kx, ky, omega, h):
    return 1.0 / (1j * omega + MU + sigma * h - eps(kx, ky))


def kvec(w, k):
    return 2.0 * math.pi * (k % w.lx) / w.lx, 2.0 * math.pi * (k // w.lx) / w.ly


def diag_g(w, sigma, h):
    r = np.arange(w.ng)
    k = r // w.nwg
    n = r % w.nwg - w.nw // 2
    kx, ky = kvec(w, k)
    return gfun(w, sigma, kx, ky, (2 * n + 1) * math.pi / w.beta, h)


def closed_form(w, channel, h, S):
    out = np.zeros((w.planes, w.n, w.n), dtype=np.complex128)
    K = np.arange(w.n)
    k = K // w.nw
    n = K % w.nw - w.nw // 2
    kx, ky = kvec(w, k)
    om = (2 * n + 1) * math.pi / w.beta
    for p in range(w.planes):
        iQ = w.q0 + p
        q = w.qs[iQ // w.nwex]
        m = iQ % w.nwex
        qx, qy = kvec(w, q)
        nu = 2.0 * math.pi * m / w.beta
        gu = gfun(w, +1, kx, ky, om, h)
        gd = gfun(w, -1, kx, ky, om, h)
        gu_q = gfun(w, +1, kx + qx, ky + qy, om + nu, h)
        gd_q = gfun(w, -1, kx + qx, ky + qy, om + nu, h)
        gu_r = gfun(w, +1, qx - kx, qy - ky, nu - om, h)
        gd_r = gfun(w, -1, qx - kx, qy - ky, nu - om, h)
        if channel in (ref.PH_MAGNETIC, ref.PH_CHARGE):
            d = gu - gd if channel == ref.PH_MAGNETIC else gu + gd
            if q == 0 and m == 0:
                out[p] += np.outer(d, d)   # [K2][K1] = d(K2) d(K1)
            out[p][K, K] -= gu * gu_q + gd * gd_q
        elif channel == ref.PH_LONG_UPUP:
            if q == 0 and m == 0:
                out[p] += np.outer(gu, gu)
            out[p][K, K] -= gu * gu_q
        elif channel == ref.PH_LONG_UPDOWN:
            if q == 0 and m == 0:
                out[p] += np.outer(gd, gu)   # [K2][K1] = g_d(K2) g_u(K1)
        elif channel == ref.PH_TRANSVERSE:
            out[p][K, K] -= gu * gd_q + gd * gu_q
        elif channel in (ref.PP_SINGLET, ref.PP_TRIPLET):
            pm = 1.0 if channel == ref.PP_SINGLET else -1.0
            out[p][K, K] += 0.5 * (gu_r * gd + gd_r * gu)
            # K2 = Q - K1: momentum q - k1 (lattice coordinates), label m - n1 - 1
            k2 = ((q % w.lx - k % w.lx) % w.lx) + w.lx * ((q // w.lx - k // w.lx) % w.ly)
            n2 = m - n - 1
            ok = (n2 >= -(w.nw // 2)) & (n2 < w.nw // 2)
            K2 = k2 * w.nw + n2 + w.nw // 2
            out[p][K2[ok], K[ok]] += pm * 0.5 * (gu * gd_r + gd * gu_r)[ok]
        else:
            out[p][K, K] += gu_r * gd + gd_r * gu
    return S * out


SHAPES = [
    # rectangular cluster, every transfer momentum, whole array
    Workload("rect 3x4", lx=3, ly=4, nw=4, nwex=3, nq=12, beta=5.0),
    # reordered transfer list, slice cut through the middle of a transfer momentum
    Workload("cut slice", lx=4, ly=3, nw=6, nwex=3, nq=3, q_list=(5, 0, 7), q_begin=2, q_end=7,
             beta=7.0),
    # the tiny workload's shape
    Workload("2x2", lx=2, ly=2, nw=16, nwex=1, nq=1, beta=5.0),
]


@pytest.mark.parametrize("w", SHAPES, ids=lambda w: w.name)
@pytest.mark.parametrize("channel", [ref.PH_MAGNETIC, ref.PH_CHARGE, ref.PP_UPDOWN, ref.PH_LONG_UPUP,
                                     ref.PH_LONG_UPDOWN, ref.PH_TRANSVERSE, ref.PP_SINGLET, ref.PP_TRIPLET])
@pytest.mark.parametrize("h", [0.0, 0.25])
def test_noninteracting_closed_form(w, channel, h):
    gu = np.diag(diag_g(w, +1, h))
    gd = np.diag(diag_g(w, -1, h))
    sgn = np.array([1.0, 1.0, -1.0, 1.0])
    B = len(sgn)
    out = ref.accumulate(w, channel, np.broadcast_to(gu, (B,) + gu.shape),
                         np.broadcast_to(gd, (B,) + gd.shape), sgn)
    want = closed_form(w, channel, h, sgn.sum())
    scale = np.abs(want).max()
    assert scale > 0
    assert np.abs(out - want).max() <= 1e-13 * scale
    # the support is exactly the closed form's: no stray entries from a wrong map
    assert np.array_equal(np.abs(out) > 1e-12 * scale, np.abs(want) > 1e-12 * scale)


def test_paramagnetic_magnetic_direct_vanishes_polarized_does_not():
    w = SHAPES[0]
    for h, expect_zero in ((0.0, True), (0.25, False)):
        gu = np.diag(diag_g(w, +1, h))[None]
        gd = np.diag(diag_g(w, -1, h))[None]
        out = ref.accumulate(w, ref.PH_MAGNETIC, gu, gd, np.ones(1))
        offdiag = out[0][~np.eye(w.n, dtype=bool)]   # Q = 0 plane, K1 != K2: direct term only
        assert (np.abs(offdiag).max() == 0.0) == expect_zero
