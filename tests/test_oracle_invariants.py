"""Pins: invariants of the accumulation, the slice partition, the measurement
order, the paper's printed sizes, and agreement of the two oracle forms."""
import json
import os

import numpy as np
import pytest

from metrics import paper_errors, rel_fro
from oracle import ref, sampled
from synth import C1_TINY, Workload, g_matrices, signs

HERE = os.path.dirname(os.path.abspath(__file__))
W = Workload("inv", lx=3, ly=2, nw=4, nwex=3, nq=6, beta=6.0, seed=9, wid=9)
CHANNELS = [ref.PH_MAGNETIC, ref.PH_CHARGE, ref.PP_UPDOWN]


def inputs(w, count, b0=0):
    return g_matrices(w, b0, count, 0), g_matrices(w, b0, count, 1), signs(w, b0, count)


@pytest.mark.parametrize("channel", CHANNELS)
def test_spin_swap_is_exact(channel):
    gu, gd, s = inputs(W, 4)
    a = ref.accumulate(W, channel, gu, gd, s)
    b = ref.accumulate(W, channel, gd, gu, s)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("channel", CHANNELS)
def test_sign_negates(channel):
    gu, gd, s = inputs(W, 3)
    a = ref.accumulate(W, channel, gu, gd, s)
    b = ref.accumulate(W, channel, gu, gd, -s)
    assert np.array_equal(a, -b)


@pytest.mark.parametrize("channel", CHANNELS)
def test_symmetric_g_gives_symmetric_g4(channel):
    gu, gd, s = inputs(W, 2)
    gu = gu + np.transpose(gu, (0, 2, 1))
    gd = gd + np.transpose(gd, (0, 2, 1))
    a = ref.accumulate(W, channel, gu, gd, s)
    assert np.allclose(a, np.transpose(a, (0, 2, 1)), rtol=0, atol=1e-13 * np.abs(a).max())


@pytest.mark.parametrize("channel", CHANNELS)
def test_additivity_and_continuation(channel):
    gu, gd, s = inputs(W, 6)
    whole = ref.accumulate(W, channel, gu, gd, s)
    cont = ref.accumulate(W, channel, gu[:2], gd[:2], s[:2])
    ref.accumulate(W, channel, gu[2:], gd[2:], s[2:], g4=cont)
    assert np.array_equal(whole, cont)            # same per-entry order: bit-exact
    parts = ref.accumulate(W, channel, gu[:4], gd[:4], s[:4]) + ref.accumulate(
        W, channel, gu[4:], gd[4:], s[4:])
    assert rel_fro(parts, whole) < 1e-14


@pytest.mark.parametrize("channel", CHANNELS)
def test_slice_union_is_bitwise(channel):
    gu, gd, s = inputs(W, 3)
    full = ref.accumulate(W, channel, gu, gd, s)
    nQ = W.nQ
    bounds = [0, 5, 7, 12, nQ]        # uneven cuts, some through the middle of a q
    pieces = [ref.accumulate(W.with_(q_begin=a, q_end=b), channel, gu, gd, s)
              for a, b in zip(bounds[:-1], bounds[1:])]
    assert np.array_equal(np.concatenate(pieces, axis=0), full)


def test_ring_order_rotation():
    # rank r of an S-ring applies walker buffers in the order r, r-1, ..., r-S+1 (mod S)
    S = 4
    gu, gd, s = inputs(W, S)
    base = ref.accumulate(W, ref.PH_MAGNETIC, gu, gd, s)
    for r in range(S):
        order = [(r - j) % S for j in range(S)]
        got = ref.accumulate(W, ref.PH_MAGNETIC, gu[order], gd[order], s[order])
        assert rel_fro(got, base) < 1e-15


@pytest.mark.parametrize("channel", CHANNELS)
def test_sampled_oracle_matches_c_oracle(channel):
    w = W.with_(measurements=5, q_begin=4, q_end=15)
    gu, gd, s = inputs(w, 5)
    full = ref.accumulate(w, channel, gu, gd, s)
    idx = sampled.sample_indices(w, 300)
    got = sampled.entries(w, channel, idx)
    assert rel_fro(got, full.reshape(-1)[idx]) < 1e-15
    ent = ref.entries(w, channel, gu, gd, s, idx)
    assert np.array_equal(ent, full.reshape(-1)[idx])


def test_compensated_mode_agrees():
    gu, gd, s = inputs(C1_TINY, 16)
    a = ref.accumulate(C1_TINY, ref.PH_MAGNETIC, gu, gd, s)
    g4 = np.zeros_like(a)
    comp = np.zeros_like(a)
    ref.accumulate(C1_TINY, ref.PH_MAGNETIC, gu, gd, s, g4=g4, comp=comp)
    assert rel_fro(g4 + comp, a) < 1e-14


def test_paper_printed_sizes():
    with open(os.path.join(HERE, "golden", "paper_sizes.json")) as f:
        p = json.load(f)
    w = Workload("paper", lx=6, ly=6, nw=64, nwex=1, nq=40)   # NQ = 40 planes (reading)
    assert w.entries == p["entries"]
    gb = w.entries * 16 / 1e9
    assert round(gb, 1) == p["bytes_approx_GB"]
    assert round(gb, 2) == p["original_GB"]
    assert round(gb / p["subring_size"], 2) == p["slice_GB_subring3"]


def test_paper_error_metrics():
    a = np.array([1 + 2j, -3 + 1j])
    b = np.array([1 + 2.5j, -2 + 1j])
    e = paper_errors(a, b)
    assert np.isclose(e["l1_re"], 1.0 / 3.0) and np.isclose(e["l1_im"], 0.5 / 3.5)
    assert np.isclose(e["l2_re"], 1.0 / np.sqrt(5.0))
