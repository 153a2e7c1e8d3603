"""Parity of the channel variants on the GPU with the FP64 oracle: the
spin-resolved particle-hole channels (longitudinal up-up, longitudinal
up-down, transverse) and the singlet / triplet projections of the PP channel.

These channels run on the register-staged (VALU) kernels in every kind:
plain FP64, batched FP64, batched FP32 into each accumulator kind.  Bars as
for the other channels: 1e-12 for FP64 products, 1e-6 for FP32 products
(relative Frobenius, Eq. (2)/(3) on real and imaginary parts, and the small
half of the entries).  Shapes span several work tiles, ragged K2 tails and
plane groups cut by the slice bounds; every channel subset shape is run
(single channels, pairs, all three).  The full-size 4x4 slice with each
family in the benchmark's pass size is checked on sampled entries.
"""
import numpy as np
import pytest

from gpu_common import config_for, g4mod, host_inputs, run_slice, to_dev
from metrics import check_entries
from oracle import ref, sampled
from synth import C3_BATCHED, Workload, signs

pytestmark = pytest.mark.gpu

UU, UD, TR = ref.PH_LONG_UPUP, ref.PH_LONG_UPDOWN, ref.PH_TRANSVERSE
PS, PT = ref.PP_SINGLET, ref.PP_TRIPLET
ALL = UU | UD | TR
PAIR = PS | PT
CHANNELS = (UU, UD, TR, PS, PT)
RAGGED = Workload("ragged-spin", lx=3, ly=2, nw=24, nwex=5, nq=6, q_list=(4, 0, 5, 1, 3, 2),
                  q_begin=3, q_end=27, beta=7.0, seed=41, wid=41, channels=ALL, h=0.2)
MULTI = Workload("multi-spin", lx=4, ly=2, nw=64, nwex=3, nq=8, q_begin=0, q_end=24,
                 beta=9.0, seed=42, wid=42, channels=ALL)
TINY = Workload("tiny-spin", lx=2, ly=2, nw=16, nwex=1, nq=1, beta=5.0, seed=43, wid=43, channels=ALL)

_cache = {}


def oracle_out(w, count):
    key = (w, count)
    if key not in _cache:
        gu, gd, s = host_inputs(w, count)
        _cache[key] = {ch: ref.accumulate(w, ch, gu, gd, s) for ch in CHANNELS if w.channels & ch}
    return _cache[key]


def check(got, want, tol):
    for ch, v in want.items():
        check_entries(got[ch], v, tol, what="channel %d" % ch)


def pair(w):
    return w.with_(name=w.name.replace("spin", "pair"), channels=PAIR)


@pytest.mark.parametrize("w,count", [(TINY, 6), (RAGGED, 4), (MULTI, 3), (pair(TINY), 6), (pair(RAGGED), 4),
                                     (pair(MULTI), 3)], ids=lambda x: getattr(x, "name", str(x)))
def test_plain_fp64(w, count):
    print("\ncase plain %s" % w.name, flush=True)
    gu, gd, s = host_inputs(w, count)
    got, st = run_slice(config_for(w, mode=0), to_dev(gu, 0), to_dev(gd, 0), s)
    assert st["launches"] == count and st["variant"] == 0
    check(got, oracle_out(w, count), 1e-12)


@pytest.mark.parametrize("w,count,B,tile", [(RAGGED, 7, 3, 0), (RAGGED, 5, 4, 20), (MULTI, 4, 4, 0),
                                            (pair(RAGGED), 7, 3, 0), (pair(RAGGED), 5, 4, 20),
                                            (pair(MULTI), 4, 4, 0)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_batched_fp64(w, count, B, tile):
    print("\ncase batched fp64 %s B=%d tile=%d" % (w.name, B, tile), flush=True)
    gu, gd, s = host_inputs(w, count)
    cfg = config_for(w, mode=1, prod=0, g_in=0, acc=0, batch=B, tile=tile)
    got, st = run_slice(cfg, to_dev(gu, 0), to_dev(gd, 0), s)
    assert st["launches"] == -(-count // B)
    check(got, oracle_out(w, count), 1e-12)


@pytest.mark.parametrize("acc", [0, 1, 2], ids=["acc-c128", "acc-kahan", "acc-c64"])
@pytest.mark.parametrize("w,count,B", [(RAGGED, 7, 3), (MULTI, 4, 4), (TINY, 8, 8), (pair(RAGGED), 7, 3),
                                       (pair(MULTI), 4, 4), (pair(TINY), 8, 8)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_batched_fp32(w, count, B, acc):
    print("\ncase batched fp32 %s B=%d acc=%d" % (w.name, B, acc), flush=True)
    gu, gd, s = host_inputs(w, count)
    cfg = config_for(w, mode=1, prod=1, g_in=1, acc=acc, batch=B)
    got, _ = run_slice(cfg, to_dev(gu, 1), to_dev(gd, 1), s)
    check(got, oracle_out(w, count), 1e-6)


@pytest.mark.parametrize("channels", [UU, UD, TR, UU | UD, UU | TR, UD | TR, PS, PT],
                         ids=["uu", "ud", "tr", "uu+ud", "uu+tr", "ud+tr", "singlet", "triplet"])
@pytest.mark.parametrize("mode", [0, 1], ids=["plain", "batched-fp32"])
def test_channel_subsets(channels, mode):
    print("\ncase subset %d mode %d" % (channels, mode), flush=True)
    full = RAGGED if channels & ALL else pair(RAGGED)
    w = full.with_(channels=channels)
    gu, gd, s = host_inputs(w, 4)
    if mode == 0:
        got, _ = run_slice(config_for(w, mode=0), to_dev(gu, 0), to_dev(gd, 0), s)
        tol = 1e-12
    else:
        got, _ = run_slice(config_for(w, mode=1, prod=1, g_in=1, batch=3), to_dev(gu, 1), to_dev(gd, 1), s)
        tol = 1e-6
    want = {ch: v for ch, v in oracle_out(full, 4).items() if channels & ch}
    assert set(got) == set(want)
    check(got, want, tol)


@pytest.mark.parametrize("fam", ["spin", "pair"])
def test_autotune_keeps_valu_plans(fam):
    """The autotuner's candidates for these families are VALU plans; the
    installed one meets its FP64 gate and the slice matches the oracle."""
    g4 = g4mod()
    w = RAGGED if fam == "spin" else pair(RAGGED)
    gu, gd, s = host_inputs(w, 8)
    h = g4.g4_init_slice(config_for(w, mode=1, prod=1, g_in=1, batch=8))
    try:
        du, dd = to_dev(gu, 1), to_dev(gd, 1)
        res = g4.g4_autotune(h, du, dd, s, tol=1e-6)
        assert res["variant"] == 0 and res["rel_err_fp64"] <= 1e-6
        g4.g4_accumulate(h, du, dd, s)
        g4.g4_sync(h)
        got = {ch: g4.g4_readback(h, ch).reshape(w.planes, w.n, w.n) for ch in CHANNELS if w.channels & ch}
    finally:
        g4.g4_destroy(h)
    check(got, oracle_out(w, 8), 1e-6)


@pytest.mark.parametrize("channels", [ALL, PAIR], ids=["spin", "pair"])
def test_full_size_slice(channels):
    """The 4x4, Nw 64, Nq 16, Nwex 8 slice (134M entries per channel) with all
    channels of a family, 256 measurements in passes of 64, complex64 G, FP32
    products: 96 sampled entries per channel against the per-entry oracle."""
    import torch
    g4 = g4mod()
    w = C3_BATCHED.with_(channels=channels, measurements=256)
    M, B = w.measurements, 64
    print("\ncase full-size spin channels", flush=True)
    tdt = torch.complex64
    gu = torch.empty((M, w.ng, w.ng), dtype=tdt, device="cuda")
    gd = torch.empty((M, w.ng, w.ng), dtype=tdt, device="cuda")
    for t, spin in ((gu, 0), (gd, 1)):
        g4.g4_synth_fill(t, 1, w.lx, w.ly, w.nw, w.nwex, w.beta, w.t, w.mu, w.h, w.noise, w.seed, w.wid, 0, M,
                         spin, None)
    s = signs(w, 0, M)
    h = g4.g4_init_slice(config_for(w, mode=1, prod=1, g_in=1, acc=0, batch=B))
    try:
        g4.g4_accumulate(h, gu, gd, s)
        g4.g4_sync(h)
        idx = sampled.sample_indices(w, 96, seed=8)
        chans = [ch for ch in CHANNELS if channels & ch]
        got = {ch: np.array([g4.g4_readback(h, ch, int(i), 1)[0] for i in idx]) for ch in chans}
    finally:
        g4.g4_destroy(h)
        del gu, gd
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    for ch in got:
        check_entries(got[ch], sampled.entries(w, ch, idx, 0, M), 1e-6, what="channel %d" % ch)
