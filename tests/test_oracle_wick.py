"""Pin: brute-force Wick contraction on tiny clusters.

For one measurement the fermions are noninteracting in the sampled auxiliary
field, so a four-operator expectation is the sum, over the ways of pairing each
creator with an annihilator, of the product of the pair contractions, times the
parity of the permutation that brings each pair together (creator first).  The
contraction of c+_X with c_Y is G(X, Y), spin-diagonal.

The channels are the operator strings

  PH magnetic  sum_{s1,s2} s1 s2 < c+_{K1+Q,s1} c_{K1,s1} c+_{K2,s2} c_{K2+Q,s2} >
  PH charge    sum_{s1,s2}       < c+_{K1+Q,s1} c_{K1,s1} c+_{K2,s2} c_{K2+Q,s2} >
  PP           sum_s < c+_{K2,-s} c+_{Q-K2,s} c_{Q-K1,s} c_{K1,-s} >   (gives Eq. (1))
  PH long. up-up     < c+_{K1+Q,u} c_{K1,u} c+_{K2,u} c_{K2+Q,u} >
  PH long. up-down   < c+_{K1+Q,u} c_{K1,u} c+_{K2,d} c_{K2+Q,d} >
  PH transverse      sum_s < c+_{K1+Q,s} c_{K1,-s} c+_{K2,-s} c_{K2+Q,s} >
  PP singlet / triplet  < P+(K2) P(K1) > with the pair operator
                     P+(K) = (c+_{K,u} c+_{Q-K,d} -/+ c+_{K,d} c+_{Q-K,u}) / sqrt(2)

This test enumerates every tuple of G-window indices, keeps the tuples whose
momenta and Matsubara frequencies are conserved (checked on physical values:
momentum vectors modulo 2 pi, frequencies as floats), contracts them with the
generic routine below, and compares with the oracle.  Nothing here uses the
oracle's index arithmetic, its formulas or its sign choices.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import ref
from synth import Workload


def parity(order):
    inv = sum(1 for i in range(len(order)) for j in range(i + 1, len(order)) if order[i] > order[j])
    return -1 if inv % 2 else 1


def wick(ops, G):
    """<prod ops> for ops = [(is_creator, window_index, spin)], G[spin][X, Y]."""
    cre = [i for i, o in enumerate(ops) if o[0]]
    ann = [i for i, o in enumerate(ops) if not o[0]]
    total = 0j
    for perm in itertools.permutations(ann):
        val = 1 + 0j
        order = []
        for c, a in zip(cre, perm):
            if ops[c][2] != ops[a][2]:
                val = 0
                break
            val *= G[ops[c][2]][ops[c][1], ops[a][1]]
            order += [c, a]
        if val != 0:
            total += parity(order) * val
    return total


def physical(w, r):
    """momentum vector and Matsubara frequency of a G-window index"""
    k = r // w.nwg
    n = r % w.nwg - w.nw // 2
    return (2 * math.pi * (k % w.lx) / w.lx, 2 * math.pi * (k // w.lx) / w.ly,
            (2 * n + 1) * math.pi / w.beta)


def in_g4_range(w, r):
    return r % w.nwg < w.nw


def g4_index(w, r):
    return (r // w.nwg) * w.nw + r % w.nwg


def same_angle(a, b):
    d = (a - b) / (2 * math.pi)
    return abs(d - round(d)) < 1e-9


def transfer_plane(w, dkx, dky, dom):
    """slice plane (relative) whose transfer (q, nu_m) equals the given physical one"""
    for iQ in range(w.q0, w.q1):
        q = w.qs[iQ // w.nwex]
        m = iQ % w.nwex
        qx, qy = 2 * math.pi * (q % w.lx) / w.lx, 2 * math.pi * (q // w.lx) / w.ly
        if same_angle(dkx, qx) and same_angle(dky, qy) and abs(dom - 2 * math.pi * m / w.beta) < 1e-9:
            return iQ - w.q0
    return None


def ph_strings(channel):
    """Spins of c+_{K1+Q} c_{K1} c+_{K2} c_{K2+Q} and the weight of each string."""
    if channel == ref.PH_MAGNETIC:
        return [((s1, s1, s2, s2), (1 - 2 * s1) * (1 - 2 * s2)) for s1 in (0, 1) for s2 in (0, 1)]
    if channel == ref.PH_CHARGE:
        return [((s1, s1, s2, s2), 1.0) for s1 in (0, 1) for s2 in (0, 1)]
    if channel == ref.PH_LONG_UPUP:
        return [((0, 0, 0, 0), 1.0)]
    if channel == ref.PH_LONG_UPDOWN:
        return [((0, 0, 1, 1), 1.0)]
    return [((s, 1 - s, 1 - s, s), 1.0) for s in (0, 1)]      # transverse


def pp_strings(channel):
    """Spins of c+_{K2} c+_{Q-K2} c_{Q-K1} c_{K1} and the weight of each string."""
    if channel == ref.PP_UPDOWN:
        return [((1 - s, s, s, 1 - s), 1.0) for s in (0, 1)]
    # P+(K2) = sum_a ca c+_{K2,sa} c+_{Q-K2,-sa};  P(K1) = sum_b cb c_{Q-K1,-sb} c_{K1,sb}
    sgn = -1.0 if channel == ref.PP_SINGLET else 1.0
    terms = []
    for sa, ca in ((0, 1.0), (1, sgn)):
        for sb, cb in ((0, 1.0), (1, sgn)):
            terms.append(((sa, 1 - sa, 1 - sb, sb), 0.5 * ca * cb))
    return terms


def brute_force(w, channel, Gs, sgn):
    P = [physical(w, r) for r in range(w.ng)]
    out = np.zeros((w.planes, w.n, w.n), dtype=np.complex128)
    hits = np.zeros(out.shape, dtype=int)
    rng = range(w.ng)
    if channel in (ref.PH_MAGNETIC, ref.PH_CHARGE, ref.PH_LONG_UPUP, ref.PH_LONG_UPDOWN, ref.PH_TRANSVERSE):
        left = {}   # (X1, Y1): transfer X1 - Y1, Y1 = K1
        right = {}  # (X2, Y2): transfer Y2 - X2, X2 = K2
        for x, y in itertools.product(rng, rng):
            d = (P[x][0] - P[y][0], P[x][1] - P[y][1], P[x][2] - P[y][2])
            if in_g4_range(w, y):
                p = transfer_plane(w, *d)
                if p is not None:
                    left.setdefault(p, []).append((x, y))
            if in_g4_range(w, x):
                p = transfer_plane(w, -d[0], -d[1], -d[2])
                if p is not None:
                    right.setdefault(p, []).append((x, y))
        for p in left:
            for (x1, y1), (x2, y2) in itertools.product(left[p], right.get(p, [])):
                K1, K2 = g4_index(w, y1), g4_index(w, x2)
                v = 0j
                for spins, wt in ph_strings(channel):
                    a1, a2, a3, a4 = spins
                    for b, s in enumerate(sgn):
                        v += s * wt * wick([(True, x1, a1), (False, y1, a2),
                                            (True, x2, a3), (False, y2, a4)], Gs[b])
                out[p, K2, K1] += v
                hits[p, K2, K1] += 1
    else:
        pairs = {}  # (A, B) with A + B = Q; A in the G4 range
        for a, bb in itertools.product(rng, rng):
            if in_g4_range(w, a):
                p = transfer_plane(w, P[a][0] + P[bb][0], P[a][1] + P[bb][1], P[a][2] + P[bb][2])
                if p is not None:
                    pairs.setdefault(p, []).append((a, bb))
        for p in pairs:
            for (A, B), (D, C) in itertools.product(pairs[p], pairs[p]):
                K2, K1 = g4_index(w, A), g4_index(w, D)
                v = 0j
                for (a1, a2, a3, a4), wt in pp_strings(channel):
                    for b, sg in enumerate(sgn):
                        v += sg * wt * wick([(True, A, a1), (True, B, a2), (False, C, a3),
                                             (False, D, a4)], Gs[b])
                out[p, K2, K1] += v
                hits[p, K2, K1] += 1
    return out, hits


SHAPES = [
    Workload("3x2 all q", lx=3, ly=2, nw=2, nwex=2, nq=6, beta=4.0),
    Workload("2x3 cut slice", lx=2, ly=3, nw=4, nwex=2, nq=3, q_list=(3, 0, 5), q_begin=1,
             q_end=5, beta=6.0),
]


@pytest.mark.parametrize("w", SHAPES, ids=lambda w: w.name)
@pytest.mark.parametrize("channel", [ref.PH_MAGNETIC, ref.PH_CHARGE, ref.PP_UPDOWN, ref.PH_LONG_UPUP,
                                     ref.PH_LONG_UPDOWN, ref.PH_TRANSVERSE, ref.PP_SINGLET, ref.PP_TRIPLET])
def test_brute_force_wick(w, channel):
    rng = np.random.default_rng(11 + channel)
    sgn = np.array([1.0, -1.0])
    gu = rng.normal(size=(2, w.ng, w.ng)) + 1j * rng.normal(size=(2, w.ng, w.ng))
    gd = rng.normal(size=(2, w.ng, w.ng)) + 1j * rng.normal(size=(2, w.ng, w.ng))
    Gs = [(gu[b], gd[b]) for b in range(2)]
    want, hits = brute_force(w, channel, Gs, sgn)
    # conservation picks exactly one operator tuple per G4 entry
    assert (hits == 1).all()
    got = ref.accumulate(w, channel, gu, gd, sgn)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
