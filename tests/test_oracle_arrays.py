"""Pin: the channels re-expressed with array operations.

With G viewed as a 6-index array [ky, kx, n | ky', kx', n'], the shift
X -> X + Q is a cyclic roll of the momentum axes plus a frequency offset, and
X -> Q - X is a momentum reflection (flip + roll) with a reversed frequency
window.  Then, per transfer plane Q,

  direct   = outer(b, a),  a(K1) = diag D(K1+Q, K1),  b(K2) = diag D(K2, K2+Q)
             summed over measurements as the matrix product B^T diag(s) A   (library matmul)
  exchange = sum_s X_s (.) Y_s^T,  X = G(K2, K1),  Y = G(K1+Q, K2+Q)   (Hadamard)
  PP       = sum_s Z_s (.) X_-s,   Z = G(Q-K2, Q-K1)

At Q = 0 the exchange is the textbook sum_s G_s (.) G_s^T restricted to the
window.  None of this uses the oracle's index arithmetic.
"""
import numpy as np
import pytest

from oracle import ref
from synth import Workload


def six(w, G):
    return G.reshape(w.ly, w.lx, w.nwg, w.ly, w.lx, w.nwg)


def shift_rows(w, G6, q, m):
    """rows X -> X + Q (G4 range of X), all columns"""
    qx, qy = q % w.lx, q // w.lx
    return np.roll(G6, (-qy, -qx), axis=(0, 1))[:, :, m:m + w.nw]


def shift_cols(w, G6, q, m):
    qx, qy = q % w.lx, q // w.lx
    return np.roll(G6, (-qy, -qx), axis=(3, 4))[:, :, :, :, :, m:m + w.nw]


def reflect_rows(w, G6, q, m):
    """rows X -> Q - X (G4 range of X): momentum flip + roll, reversed frequencies"""
    qx, qy = q % w.lx, q // w.lx
    t = np.roll(np.flip(G6, axis=(0, 1)), (qy + 1, qx + 1), axis=(0, 1))
    return t[:, :, m:m + w.nw][:, :, ::-1]


def reflect_cols(w, G6, q, m):
    qx, qy = q % w.lx, q // w.lx
    t = np.roll(np.flip(G6, axis=(3, 4)), (qy + 1, qx + 1), axis=(3, 4))
    return t[:, :, :, :, :, m:m + w.nw][:, :, :, :, :, ::-1]


def mat(w, A6):
    return A6.reshape(w.n, w.n)


def window(w, G6):
    return G6[:, :, :w.nw, :, :, :w.nw]


def array_channel(w, channel, gu, gd, sgn):
    out = np.zeros((w.planes, w.n, w.n), dtype=np.complex128)
    for p in range(w.planes):
        iQ = w.q0 + p
        q, m = w.qs[iQ // w.nwex], iQ % w.nwex
        if channel in (ref.PH_MAGNETIC, ref.PH_CHARGE):
            pm = -1.0 if channel == ref.PH_MAGNETIC else 1.0
            A = np.empty((len(sgn), w.n), dtype=np.complex128)
            Bv = np.empty((len(sgn), w.n), dtype=np.complex128)
            ex = np.zeros((w.n, w.n), dtype=np.complex128)
            for b in range(len(sgn)):
                D6 = six(w, gu[b] + pm * gd[b])
                A[b] = np.diagonal(mat(w, shift_rows(w, D6, q, m)[:, :, :, :, :, :w.nw]))
                Bv[b] = np.diagonal(mat(w, shift_cols(w, D6, q, m)[:, :, :w.nw]))
                for G in (gu[b], gd[b]):
                    G6 = six(w, G)
                    X = mat(w, window(w, G6))                               # [K2][K1]
                    Y = mat(w, shift_cols(w, shift_rows(w, G6, q, m), q, m))  # [K1][K2]
                    ex += sgn[b] * (X * Y.T)
            direct = Bv.T @ (sgn[:, None] * A)                              # [K2][K1]
            out[p] = direct - ex
        else:
            for b in range(len(sgn)):
                for G, Gother in ((gu[b], gd[b]), (gd[b], gu[b])):
                    Z = mat(w, reflect_cols(w, reflect_rows(w, six(w, G), q, m), q, m))
                    X = mat(w, window(w, six(w, Gother)))
                    out[p] += sgn[b] * (Z * X)
    return out


SHAPES = [
    Workload("4x3 all q", lx=4, ly=3, nw=4, nwex=3, nq=12),
    Workload("3x5 cut", lx=3, ly=5, nw=6, nwex=2, nq=4, q_list=(14, 0, 7, 3), q_begin=3, q_end=7),
    Workload("2x2 tiny shape", lx=2, ly=2, nw=16, nwex=1, nq=1),
]


@pytest.mark.parametrize("w", SHAPES, ids=lambda w: w.name)
@pytest.mark.parametrize("channel", [ref.PH_MAGNETIC, ref.PH_CHARGE, ref.PP_UPDOWN])
def test_array_formulation(w, channel):
    rng = np.random.default_rng(5 + channel)
    B = 3
    gu = rng.normal(size=(B, w.ng, w.ng)) + 1j * rng.normal(size=(B, w.ng, w.ng))
    gd = rng.normal(size=(B, w.ng, w.ng)) + 1j * rng.normal(size=(B, w.ng, w.ng))
    sgn = np.array([1.0, -1.0, 1.0])
    want = array_channel(w, channel, gu, gd, sgn)
    got = ref.accumulate(w, channel, gu, gd, sgn)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_q0_exchange_is_hadamard_with_transpose():
    w = Workload("q0", lx=3, ly=3, nw=4, nwex=1, nq=1)
    rng = np.random.default_rng(3)
    gu = rng.normal(size=(1, w.ng, w.ng)) + 1j * rng.normal(size=(1, w.ng, w.ng))
    gd = rng.normal(size=(1, w.ng, w.ng)) + 1j * rng.normal(size=(1, w.ng, w.ng))
    mag = ref.accumulate(w, ref.PH_MAGNETIC, gu, gd, np.ones(1))[0]
    ch = ref.accumulate(w, ref.PH_CHARGE, gu, gd, np.ones(1))[0]
    # Nwex = 1: the G window is the G4 range and G4 indices equal G indices
    ex = gu[0] * gu[0].T + gd[0] * gd[0].T
    dm = np.diag(gu[0] - gd[0])
    dp = np.diag(gu[0] + gd[0])
    assert np.allclose(mag, np.outer(dm, dm) - ex, rtol=0, atol=1e-13)
    assert np.allclose(ch, np.outer(dp, dp) - ex, rtol=0, atol=1e-13)
