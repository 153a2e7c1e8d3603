"""Pins of the oracle's channel variants: the spin-resolved particle-hole
channels and the singlet / triplet projections of the particle-particle one.

Longitudinal up-up, longitudinal up-down and transverse are separate code in
the oracle.  Besides the brute-force Wick contraction and the noninteracting
closed forms (their own test files), they are pinned here against the
magnetic and charge channels, whose code they share nothing with:

- spin decomposition: with dd and du the up-up and up-down channels of the
  spin-swapped input,  magnetic = uu + dd - ud - du  and
  charge = uu + dd + ud + du  (the sums over s1, s2 with weights s1 s2 or 1);
- SU(2): for equal spins (Gu = Gd) the transverse channel equals the
  magnetic one (both are then minus twice the exchange term);
- no down spin (Gd = 0): up-down and transverse vanish exactly, up-up is
  the magnetic channel of the same input;
- transverse is symmetric under the spin swap, bit for bit;
- PP singlet + PP triplet = PP up-down (Eq. (1)), and the two differ (the
  crossed term is not zero);
- the per-entry numpy oracle (regenerated inputs) agrees with the C one.
"""
import numpy as np
import pytest

from metrics import rel_fro
from oracle import ref, sampled
from synth import Workload, g_matrices, signs

W = Workload("spin", lx=3, ly=2, nw=4, nwex=3, nq=6, q_begin=2, q_end=16, beta=6.0, seed=31, wid=31,
             measurements=3)
SPIN = [ref.PH_LONG_UPUP, ref.PH_LONG_UPDOWN, ref.PH_TRANSVERSE, ref.PP_SINGLET, ref.PP_TRIPLET]


def inputs(w, count):
    return g_matrices(w, 0, count, 0), g_matrices(w, 0, count, 1), signs(w, 0, count)


def test_magnetic_and_charge_decompose_into_spin_pairs():
    gu, gd, s = inputs(W, 3)
    uu = ref.accumulate(W, ref.PH_LONG_UPUP, gu, gd, s)
    dd = ref.accumulate(W, ref.PH_LONG_UPUP, gd, gu, s)
    ud = ref.accumulate(W, ref.PH_LONG_UPDOWN, gu, gd, s)
    du = ref.accumulate(W, ref.PH_LONG_UPDOWN, gd, gu, s)
    mag = ref.accumulate(W, ref.PH_MAGNETIC, gu, gd, s)
    chg = ref.accumulate(W, ref.PH_CHARGE, gu, gd, s)
    assert rel_fro(uu + dd - ud - du, mag) < 1e-14
    assert rel_fro(uu + dd + ud + du, chg) < 1e-14


def test_equal_spins_transverse_equals_magnetic():
    gu, _, s = inputs(W, 2)
    tr = ref.accumulate(W, ref.PH_TRANSVERSE, gu, gu, s)
    mag = ref.accumulate(W, ref.PH_MAGNETIC, gu, gu, s)
    assert np.abs(tr).max() > 0
    assert rel_fro(tr, mag) < 1e-15


def test_no_down_spin():
    gu, _, s = inputs(W, 2)
    zero = np.zeros_like(gu)
    assert np.abs(ref.accumulate(W, ref.PH_LONG_UPDOWN, gu, zero, s)).max() == 0.0
    assert np.abs(ref.accumulate(W, ref.PH_TRANSVERSE, gu, zero, s)).max() == 0.0
    uu = ref.accumulate(W, ref.PH_LONG_UPUP, gu, zero, s)
    assert rel_fro(uu, ref.accumulate(W, ref.PH_MAGNETIC, gu, zero, s)) < 1e-15


def test_transverse_spin_swap_is_exact():
    gu, gd, s = inputs(W, 2)
    a = ref.accumulate(W, ref.PH_TRANSVERSE, gu, gd, s)
    b = ref.accumulate(W, ref.PH_TRANSVERSE, gd, gu, s)
    assert np.array_equal(a, b)


def test_singlet_and_triplet_sum_to_eq1():
    gu, gd, s = inputs(W, 3)
    st = ref.accumulate(W, ref.PP_SINGLET, gu, gd, s)
    tt = ref.accumulate(W, ref.PP_TRIPLET, gu, gd, s)
    pp = ref.accumulate(W, ref.PP_UPDOWN, gu, gd, s)
    assert rel_fro(st + tt, pp) < 1e-15
    assert rel_fro(st, tt) > 0.1


@pytest.mark.parametrize("channel", SPIN)
def test_sampled_oracle_matches_c_oracle(channel):
    gu, gd, s = inputs(W, 3)
    full = ref.accumulate(W, channel, gu, gd, s)
    idx = sampled.sample_indices(W, 300)
    got = sampled.entries(W, channel, idx)
    assert rel_fro(got, full.reshape(-1)[idx]) < 1e-15
    assert np.array_equal(ref.entries(W, channel, gu, gd, s, idx), full.reshape(-1)[idx])
