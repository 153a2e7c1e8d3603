"""Pins of the oracle's multi-orbital G4.

- nb = 1 is the single-band oracle, bit for bit (separate code);
- brute-force Wick contraction on a tiny two-orbital cluster: every tuple of
  G-window indices and orbital labels conserving momentum and frequency,
  contracted by the generic routine of the single-band Wick test, for the
  operator strings the oracle's header names;
- the per-entry form equals the whole-slice form at sampled entries, bit for
  bit;
- orbital-diagonal, orbital-independent G: the entries with all four labels
  equal are the single-band values, bit for bit; entries with b1 = b2 and
  b3 = b4 but b2 != b3 keep only the direct term, those with b2 = b3 and
  b1 = b4 but b1 != b2 only the exchange term, the rest vanish.
"""
import itertools

import numpy as np
import pytest

from oracle import ref
from synth import Workload
from test_oracle_wick import g4_index, in_g4_range, physical, transfer_plane, wick

CH = [ref.PH_MAGNETIC, ref.PH_CHARGE, ref.PP_UPDOWN]


def rand_g(rng, shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


@pytest.mark.parametrize("channel", CH)
def test_one_orbital_is_single_band(channel):
    w = Workload("mo1", lx=3, ly=2, nw=4, nwex=3, nq=6, q_begin=2, q_end=14, beta=6.0)
    rng = np.random.default_rng(channel)
    gu, gd = rand_g(rng, (2, w.ng, w.ng)), rand_g(rng, (2, w.ng, w.ng))
    s = np.array([1.0, -1.0])
    assert np.array_equal(ref.accumulate_mo(w, 1, channel, gu, gd, s), ref.accumulate(w, channel, gu, gd, s))


def brute_force_mo(w, nb, channel, Gs, sgn):
    P = [physical(w, r) for r in range(w.ng)]
    side = w.n * nb * nb
    out = np.zeros((w.planes, side, side), dtype=np.complex128)
    hits = np.zeros(out.shape, dtype=int)
    rng = range(w.ng)
    orb = list(itertools.product(range(nb), repeat=4))

    def row(K2, b3, b4):
        return (K2 * nb + b3) * nb + b4

    def col(K1, b1, b2):
        return (K1 * nb + b1) * nb + b2

    if channel != ref.PP_UPDOWN:
        left, right = {}, {}
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
                for b1, b2, b3, b4 in orb:
                    v = 0j
                    for s1, s2 in itertools.product((0, 1), (0, 1)):
                        wt = 1.0 if channel == ref.PH_CHARGE else (1 - 2 * s1) * (1 - 2 * s2)
                        for b, sg in enumerate(sgn):
                            v += sg * wt * wick([(True, x1 * nb + b1, s1), (False, y1 * nb + b2, s1),
                                                 (True, x2 * nb + b3, s2), (False, y2 * nb + b4, s2)], Gs[b])
                    out[p, row(K2, b3, b4), col(K1, b1, b2)] += v
                    hits[p, row(K2, b3, b4), col(K1, b1, b2)] += 1
    else:
        pairs = {}
        for a, bb in itertools.product(rng, rng):
            if in_g4_range(w, a):
                p = transfer_plane(w, P[a][0] + P[bb][0], P[a][1] + P[bb][1], P[a][2] + P[bb][2])
                if p is not None:
                    pairs.setdefault(p, []).append((a, bb))
        for p in pairs:
            for (A, B), (D, C) in itertools.product(pairs[p], pairs[p]):
                K2, K1 = g4_index(w, A), g4_index(w, D)
                for b1, b2, b3, b4 in orb:
                    v = 0j
                    for s in (0, 1):
                        for b, sg in enumerate(sgn):
                            v += sg * wick([(True, A * nb + b3, 1 - s), (True, B * nb + b4, s),
                                            (False, C * nb + b2, s), (False, D * nb + b1, 1 - s)], Gs[b])
                    out[p, row(K2, b3, b4), col(K1, b1, b2)] += v
                    hits[p, row(K2, b3, b4), col(K1, b1, b2)] += 1
    return out, hits


@pytest.mark.parametrize("channel", CH)
def test_brute_force_wick_two_orbitals(channel):
    w = Workload("mo-wick", lx=2, ly=1, nw=2, nwex=2, nq=2, q_list=(1, 0), q_begin=1, q_end=4, beta=4.0)
    nb = 2
    rng = np.random.default_rng(70 + channel)
    sgn = np.array([1.0, -1.0])
    ngb = w.ng * nb
    gu, gd = rand_g(rng, (2, ngb, ngb)), rand_g(rng, (2, ngb, ngb))
    want, hits = brute_force_mo(w, nb, channel, [(gu[b], gd[b]) for b in range(2)], sgn)
    assert (hits == 1).all()
    got = ref.accumulate_mo(w, nb, channel, gu, gd, sgn)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("channel", [ref.PH_MAGNETIC, ref.PH_CHARGE])
def test_orbital_diagonal_g_factorises(channel):
    w = Workload("mo-diag", lx=2, ly=2, nw=4, nwex=2, nq=4, q_begin=1, q_end=7, beta=5.0)
    nb = 3
    rng = np.random.default_rng(5)
    g0u, g0d = rand_g(rng, (1, w.ng, w.ng)), rand_g(rng, (1, w.ng, w.ng))
    eye = np.eye(nb)
    gu = np.kron(g0u[0], eye)[None]     # G(K b, K' b') = delta_bb' G0(K, K'), index K*nb + b
    gd = np.kron(g0d[0], eye)[None]
    s = np.array([1.0])
    mo = ref.accumulate_mo(w, nb, channel, gu, gd, s).reshape(w.planes, w.n, nb, nb, w.n, nb, nb)
    single = ref.accumulate(w, channel, g0u, g0d, s)
    zero = np.zeros_like(single)
    for b1, b2, b3, b4 in itertools.product(range(nb), repeat=4):
        blk = mo[:, :, b3, b4, :, b1, b2]
        if b1 == b2 == b3 == b4:
            assert np.array_equal(blk, single)
        elif not ((b1 == b2 and b3 == b4) or (b2 == b3 and b1 == b4)):
            assert np.array_equal(blk, zero)
    # direct only / exchange only pieces add up to the single-band value
    d = mo[:, :, 1, 1, :, 0, 0]          # b1 = b2 = 0, b3 = b4 = 1: direct term
    x = mo[:, :, 0, 1, :, 1, 0]          # b2 = b3 = 0, b1 = b4 = 1: exchange term
    assert np.abs(d + x - single).max() <= 1e-13 * np.abs(single).max()


@pytest.mark.parametrize("channel", CH)
def test_entries_equal_whole_slice(channel):
    w = Workload("mo-ent", lx=2, ly=2, nw=4, nwex=2, nq=4, q_list=(3, 1, 0, 2), q_begin=1, q_end=6, beta=5.0)
    nb = 2
    rng = np.random.default_rng(9 + channel)
    ngb = w.ng * nb
    gu, gd = rand_g(rng, (3, ngb, ngb)), rand_g(rng, (3, ngb, ngb))
    s = np.array([1.0, -1.0, 1.0])
    full = ref.accumulate_mo(w, nb, channel, gu, gd, s).reshape(-1)
    idx = rng.integers(0, full.shape[0], size=200)
    assert np.array_equal(ref.entries_mo(w, nb, channel, gu, gd, s, idx), full[idx])
