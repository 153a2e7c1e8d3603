"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: FP64 products (plain and batched) 1e-12 relative Frobenius error per
channel; FP32 products 1e-6.  Integer index maps are checked bit-exactly by
one-hot probes (the output support must equal the oracle's).  Shapes span
several work tiles, ragged K2 tails, transfer groups cut by the slice bounds,
and ragged final passes."""
import numpy as np
import pytest

from gpu_common import config_for, g4mod, host_inputs, run_slice, to_dev
from metrics import check_entries, rel_fro
from oracle import ref
from synth import C1_TINY, PH_CHARGE, PH_MAGNETIC, PP_UPDOWN, Workload

pytestmark = pytest.mark.gpu

ALL = PH_MAGNETIC | PH_CHARGE | PP_UPDOWN
RAGGED = Workload("ragged", lx=3, ly=2, nw=24, nwex=5, nq=6, q_list=(4, 0, 5, 1, 3, 2),
                  q_begin=3, q_end=27, beta=7.0, seed=21, wid=21, channels=ALL)
MULTI = Workload("multi-tile", lx=4, ly=2, nw=64, nwex=3, nq=8, q_begin=0, q_end=24,
                 beta=9.0, seed=22, wid=22, channels=ALL)
NW128 = Workload("nw128", lx=2, ly=1, nw=128, nwex=9, nq=2, q_begin=4, q_end=15,
                 beta=10.0, seed=23, wid=23, channels=ALL)
TINY_ALL = C1_TINY.with_(channels=ALL)

_cache = {}


def oracle_out(w, count, channels):
    key = (w, count, channels)
    if key not in _cache:
        gu, gd, s = host_inputs(w, count)
        _cache[key] = {ch: ref.accumulate(w, ch, gu, gd, s) for ch in (1, 2, 4) if channels & ch}
    return _cache[key]


def check(got, want, tol):
    for ch, v in want.items():
        check_entries(got[ch], v, tol, what="channel %d" % ch)


@pytest.mark.parametrize("w,count", [(C1_TINY, 64), (TINY_ALL, 8), (RAGGED, 5), (MULTI, 3),
                                     (NW128, 3)], ids=lambda x: getattr(x, "name", str(x)))
def test_plain_fp64(w, count):
    gu, gd, s = host_inputs(w, count)
    cfg = config_for(w, mode=0)
    got, st = run_slice(cfg, to_dev(gu, 0), to_dev(gd, 0), s, chunks=[0, 1, count])
    assert st["measurements"] == count and st["launches"] == count
    assert st["sign_sum"] == s.sum()
    check(got, oracle_out(w, count, w.channels), 1e-12)


@pytest.mark.parametrize("w,count,B,tile", [(RAGGED, 7, 3, 0), (RAGGED, 7, 8, 20), (MULTI, 4, 4, 0),
                                            (NW128, 5, 2, 0), (TINY_ALL, 8, 8, 0)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_batched_fp64_inputs(w, count, B, tile):
    gu, gd, s = host_inputs(w, count)
    cfg = config_for(w, mode=1, prod=0, g_in=0, acc=0, batch=B, tile=tile)
    got, st = run_slice(cfg, to_dev(gu, 0), to_dev(gd, 0), s)
    assert st["launches"] == -(-count // B)
    check(got, oracle_out(w, count, w.channels), 1e-12)


@pytest.mark.parametrize("g_in", [0, 1], ids=["c128-in", "c64-in"])
@pytest.mark.parametrize("acc", [0, 1, 2], ids=["acc-c128", "acc-kahan", "acc-c64"])
@pytest.mark.parametrize("w,count,B", [(RAGGED, 7, 3), (MULTI, 4, 4), (NW128, 5, 4)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_batched_fp32(w, count, B, g_in, acc):
    gu, gd, s = host_inputs(w, count)
    cfg = config_for(w, mode=1, prod=1, g_in=g_in, acc=acc, batch=B)
    got, _ = run_slice(cfg, to_dev(gu, g_in), to_dev(gd, g_in), s)
    check(got, oracle_out(w, count, w.channels), 1e-6)


PACKED_KINDS = [(16, 2), (32, 3)]      # (flag, variant): packed, packed with deep blocks


@pytest.mark.parametrize("g_in", [0, 1], ids=["c128-in", "c64-in"])
@pytest.mark.parametrize("acc", [0, 1], ids=["acc-c128", "acc-kahan"])
@pytest.mark.parametrize("w,count,B,tile", [(RAGGED, 7, 3, 0), (RAGGED, 5, 4, 20), (MULTI, 4, 4, 0),
                                            (MULTI, 3, 3, 16), (NW128, 5, 4, 0), (TINY_ALL, 8, 8, 0)],
                         ids=lambda x: getattr(x, "name", str(x)))
@pytest.mark.parametrize("flag,variant", PACKED_KINDS, ids=["packed", "deep"])
def test_batched_fp32_packed(w, count, B, tile, g_in, acc, flag, variant):
    """Packed operands copied straight into LDS: same products, same bar;
    several passes with a ragged last one exercise the buffer rotation."""
    g4 = g4mod()
    if variant == 3 and tile == 20:
        tile = 42                        # deep blocks sweep 21 rows of nw = 24
    if variant == 3 and tile == 16:
        tile = 8                         # three channels x 16 rows x 3 buffers exceed the LDS
    if variant == 3 and w is NW128:
        w = w.with_(channels=PH_MAGNETIC | PH_CHARGE)   # with PP, 3 buffers exceed the LDS
    gu, gd, s = host_inputs(w, count)
    cfg = config_for(w, mode=1, prod=1, g_in=g_in, acc=acc, batch=B, tile=tile, flags=flag)
    got, st = run_slice(cfg, to_dev(gu, g_in), to_dev(gd, g_in), s)
    assert st["variant"] == variant and st["launches"] == -(-count // B)
    check(got, oracle_out(w, count, w.channels), 1e-6)


@pytest.mark.parametrize("channels", [PH_MAGNETIC, PH_CHARGE, PP_UPDOWN, PH_MAGNETIC | PP_UPDOWN],
                         ids=["mag", "chg", "pp", "mag+pp"])
@pytest.mark.parametrize("flag,variant", PACKED_KINDS, ids=["packed", "deep"])
def test_packed_channel_subsets(channels, flag, variant):
    w = RAGGED.with_(channels=channels)
    gu, gd, s = host_inputs(w, 5)
    cfg = config_for(w, mode=1, prod=1, g_in=1, acc=0, batch=3, flags=flag)
    got, st = run_slice(cfg, to_dev(gu, 1), to_dev(gd, 1), s)
    assert st["variant"] == variant
    check(got, oracle_out(w, 5, channels), 1e-6)


# Packed kernel with the direct vector a(Q, K1) read into registers instead of
# LDS: one PH channel, no PP, plane groups of 8, nw 128..256, at most two K2
# rows per thread.  NW128's groups start mid-transfer (m = 4) and end with one
# plane; NW256A has groups of 6 (nwex = 6): partial groups of the 8-plane kernel.
NW256A = Workload("nw256a", lx=2, ly=1, nw=256, nwex=6, nq=2, q_begin=2, q_end=11, beta=12.0,
                  seed=28, wid=28, channels=PH_MAGNETIC)


@pytest.mark.parametrize("g_in", [0, 1], ids=["c128-in", "c64-in"])
@pytest.mark.parametrize("acc", [0, 1, 2], ids=["acc-c128", "acc-kahan", "acc-c64"])
@pytest.mark.parametrize("w,count,B,tile", [(NW128.with_(channels=PH_MAGNETIC), 5, 2, 4),
                                            (NW128.with_(channels=PH_MAGNETIC), 4, 4, 2),
                                            (NW128.with_(channels=PH_CHARGE), 3, 2, 0),
                                            (NW256A, 3, 2, 0), (NW256A.with_(channels=PH_CHARGE), 4, 3, 2)],
                         ids=["nw128-mag-t4", "nw128-mag-t2", "nw128-chg", "nw256-mag", "nw256-chg-t2"])
def test_packed_direct_vector_in_registers(w, count, B, tile, g_in, acc):
    g4 = g4mod()
    gu, gd, s = host_inputs(w, count)
    cfg = config_for(w, mode=1, prod=1, g_in=g_in, acc=acc, batch=B, tile=tile, flags=g4.G4_F_PACKED)
    got, st = run_slice(cfg, to_dev(gu, g_in), to_dev(gd, g_in), s)
    assert st["variant"] == 2 and st["launches"] == -(-count // B)
    check(got, oracle_out(w, count, w.channels), 1e-6)


# Packed operands with the direct term on the matrix cores: nw = 64, 8-row
# tiles, plane pairs, PH channels; MULTI has plane groups of 3 (nwex = 3, partial groups of
# the 4-plane kernel), W8 groups of 8 starting mid-group (m = 3) and ending
# mid-group, over two lattice rows.
W8 = Workload("w8", lx=2, ly=2, nw=64, nwex=8, nq=4, q_begin=3, q_end=29, beta=6.0, seed=27, wid=27,
              channels=PH_MAGNETIC)


@pytest.mark.parametrize("g_in", [0, 1], ids=["c128-in", "c64-in"])
@pytest.mark.parametrize("acc", [0, 1, 2], ids=["acc-c128", "acc-kahan", "acc-c64"])
@pytest.mark.parametrize("w,count,B", [(MULTI.with_(channels=PH_MAGNETIC), 7, 3),
                                       (MULTI.with_(channels=PH_CHARGE), 4, 4),
                                       (MULTI.with_(channels=PH_MAGNETIC | PH_CHARGE), 5, 2),
                                       (W8, 9, 4), (W8.with_(channels=PH_CHARGE), 3, 3),
                                       (W8.with_(channels=PH_MAGNETIC | PH_CHARGE), 5, 3)],
                         ids=["multi-mag", "multi-chg", "multi-mag+chg", "w8-mag", "w8-chg", "w8-mag+chg"])
def test_batched_fp32_packed_mfma(w, count, B, g_in, acc):
    """Packed operands, direct term on MFMA (two planes per MFMA pair):
    several passes with a ragged last one, every accumulator kind."""
    g4 = g4mod()
    gu, gd, s = host_inputs(w, count)
    cfg = config_for(w, mode=1, prod=1, g_in=g_in, acc=acc, batch=B,
                     flags=g4.G4_F_PACKED | g4.G4_F_MFMA)
    got, st = run_slice(cfg, to_dev(gu, g_in), to_dev(gd, g_in), s)
    assert st["variant"] == g4.G4_VARIANT_PACKED_MFMA and st["tile"] == 8
    assert st["launches"] == -(-count // B)
    check(got, oracle_out(w, count, w.channels), 1e-6)


# 4x2 cluster, all 64 planes of Nwex = 8: 4096 work tiles of 8 rows, more than
# the device holds blocks at once, so a persistent grid walks several each
W8_BIG = Workload("w8-big", lx=4, ly=2, nw=64, nwex=8, nq=8, q_begin=0, q_end=64, beta=6.0, seed=28, wid=28,
                  channels=PH_MAGNETIC)


@pytest.mark.parametrize("acc", [0, 1], ids=["acc-c128", "acc-kahan"])
@pytest.mark.parametrize("w,flags,variant", [
    (W8_BIG, "packed", 2), (W8_BIG.with_(channels=PH_MAGNETIC | PH_CHARGE), "packed-mfma", 4),
    (W8_BIG, "packed-mfma", 4), (MULTI, "packed", 2), (MULTI.with_(channels=PH_MAGNETIC), "deep", 3)],
    ids=["w8big-packed", "w8big-mfma-mag+chg", "w8big-mfma", "multi-packed-all", "multi-deep"])
def test_persistent_grid(w, flags, variant, acc):
    """G4_F_PERSISTENT: the packed kernels on a persistent grid walking more
    work tiles than it has blocks (every tile of a block after its first
    reuses the block's LDS), passes with a ragged last one."""
    g4 = g4mod()
    f = {"packed": g4.G4_F_PACKED, "packed-mfma": g4.G4_F_PACKED | g4.G4_F_MFMA,
         "deep": g4.G4_F_PACKED_DEEP}[flags] | g4.G4_F_PERSISTENT
    count, B = 5, 2
    print(f"\ncase {w.name} {flags} channels={w.channels} acc={acc}", flush=True)
    gu, gd, s = host_inputs(w, count)
    cfg = config_for(w, mode=1, prod=1, g_in=1, acc=acc, batch=B, flags=f)
    got, st = run_slice(cfg, to_dev(gu, 1), to_dev(gd, 1), s)
    assert st["variant"] == variant
    assert st["launches"] == -(-count // B)
    check(got, oracle_out(w, count, w.channels), 1e-6)


@pytest.mark.parametrize("g_in", [0, 1], ids=["c128-in", "c64-in"])
@pytest.mark.parametrize("acc", [0, 1, 2], ids=["acc-c128", "acc-kahan", "acc-c64"])
@pytest.mark.parametrize("channels", [PH_MAGNETIC, PH_CHARGE, PH_MAGNETIC | PH_CHARGE],
                         ids=["mag", "chg", "mag+chg"])
def test_packed_nw64_tile8(channels, g_in, acc):
    """The packed kernel's compile-time copy for nw = 64, 8-row tiles and plane
    groups of 8 (W8: a partial group at each end of the slice, full ones
    between), three passes with a ragged last one."""
    g4 = g4mod()
    w = W8.with_(channels=channels)
    gu, gd, s = host_inputs(w, 7)
    cfg = config_for(w, mode=1, prod=1, g_in=g_in, acc=acc, batch=3, tile=8, flags=g4.G4_F_PACKED)
    got, st = run_slice(cfg, to_dev(gu, g_in), to_dev(gd, g_in), s)
    assert st["variant"] == 2 and st["tile"] == 8
    check(got, oracle_out(w, 7, channels), 1e-6)


def test_deep_long_pass():
    """Passes of 16 measurements: the three-buffer rotation wraps several times."""
    g4 = g4mod()
    w = MULTI.with_(channels=PH_MAGNETIC)
    gu, gd, s = host_inputs(w, 21)
    for flag in (16, 32):
        cfg = config_for(w, mode=1, prod=1, g_in=1, acc=0, batch=16, flags=flag)
        got, _ = run_slice(cfg, to_dev(gu, 1), to_dev(gd, 1), s)
        check(got, oracle_out(w, 21, PH_MAGNETIC), 1e-6)


# Split-precision direct term: per product the dropped lo*lo and the rounding
# of lo leave a relative error below 2^-15 (bf16 hi+lo) or 2^-21 (fp16 hi+lo,
# lo scaled by 2^11); the exchange and PP sums stay FP32 (1e-6 bar).
SPLIT_BAR = {2: 2.0 ** -15 + 1e-6, 3: 1e-6}


@pytest.mark.parametrize("prod", [2, 3], ids=["bf16x2", "f16x2"])
@pytest.mark.parametrize("flags", [0, 16], ids=["valu", "packed"])
@pytest.mark.parametrize("w,count,B", [(RAGGED, 11, 9), (MULTI, 4, 4), (NW128, 5, 4),
                                       (NW128.with_(channels=PH_MAGNETIC), 5, 4)],
                         ids=["ragged", "multi-tile", "nw128", "nw128-mag"])
def test_split_precision_direct_term(w, count, B, flags, prod):
    """Direct term as a GEMM over the pass on MFMA from hi+lo split operands;
    B = 9 leaves a partial chunk of 8 measurements in every pass.  nw128-mag
    runs the packed kernel form that reads the direct vector a into registers,
    with its direct term switched off (b read as zeros)."""
    gu, gd, s = host_inputs(w, count)
    cfg = config_for(w, mode=1, prod=prod, g_in=1, acc=1, batch=B, flags=flags)
    got, _ = run_slice(cfg, to_dev(gu, 1), to_dev(gd, 1), s)
    want = oracle_out(w, count, w.channels)
    check(got, want, SPLIT_BAR[prod])
    # the split really is coarser than FP32 products for bf16 and no worse for fp16
    ref32, _ = run_slice(config_for(w, mode=1, prod=1, g_in=1, acc=1, batch=B, flags=flags),
                         to_dev(gu, 1), to_dev(gd, 1), s)
    e_split = rel_fro(got[PH_MAGNETIC], want[PH_MAGNETIC])
    e32 = rel_fro(ref32[PH_MAGNETIC], want[PH_MAGNETIC])
    if prod == 2:
        assert e_split > e32
    else:
        assert e_split < 10 * e32 + 1e-7


@pytest.mark.parametrize("flags", [0, 16, 24, 16 | 64], ids=["valu", "packed", "packed-mfma", "packed-persistent"])
def test_graph_replay_matches_direct_passes(flags):
    """G4_F_GRAPH: passes on known inputs replay a recorded graph.  Every replay
    is checked, bit for bit, against a slice running the same passes directly,
    with eager work, input changes, new weights and synchronizations between
    replays, and across a plan change (which drops the recordings).  The
    packed MFMA plan takes the PH channels only."""
    import torch
    g4 = g4mod()
    w = MULTI.with_(channels=PH_MAGNETIC | PH_CHARGE) if flags & 8 else MULTI
    gu, gd, s = host_inputs(w, 6)
    du, dd = to_dev(gu, 1), to_dev(gd, 1)
    base = dict(mode=1, prod=1, g_in=1, acc=1, batch=3)
    hd = g4.g4_init_slice(config_for(w, flags=flags, **base))
    hg = g4.g4_init_slice(config_for(w, flags=flags | g4.G4_F_GRAPH | g4.G4_F_KERNEL_TIMING, **base))
    try:
        # per input half: direct, recorded, replayed, replayed; then after the
        # plan call: direct, recorded
        for it in range(12):
            half = slice(0, 3) if it % 2 == 0 else slice(3, 6)
            sg = s[half] * (1.0 if it < 5 else -0.5)
            if it == 6:
                du.mul_(0.75)                      # the graph must read the current contents
            if it == 8:
                g4.g4_set_plan(hg, 0, 0, -1)       # a plan call drops the recordings
                g4.g4_set_plan(hd, 0, 0, -1)
            for h in (hd, hg):
                g4.g4_accumulate(h, du[half], dd[half], sg)
            torch.cuda.synchronize()
            _ = (du.abs().sum() + dd.abs().sum()).item()    # eager work between replays
            for ch in (c for c in (1, 2, 4) if w.channels & c):
                a = g4.g4_readback(hd, ch)
                b = g4.g4_readback(hg, ch)
                assert np.array_equal(a, b), (it, ch)
        st = g4.g4_stats(hg)
        assert st["launches"] == 12 and st["measurements"] == 36 and st["timed_launches"] == 12
    finally:
        g4.g4_destroy(hd)
        g4.g4_destroy(hg)


@pytest.mark.parametrize("acc", [0, 1], ids=["acc-c128", "acc-kahan"])
def test_graph_replay_matches_oracle(acc):
    """G4_F_GRAPH on the packed plan: after every call (direct, recorded,
    replayed, ...) on two alternating input pairs, with eager work and
    synchronizations between replays, the slice equals the FP64 oracle of
    everything applied so far."""
    import torch
    g4 = g4mod()
    w = MULTI
    gu, gd, s = host_inputs(w, 6)
    du, dd = to_dev(gu, 1), to_dev(gd, 1)
    halves = (slice(0, 3), slice(3, 6))
    want = [{ch: ref.accumulate(w, ch, gu[hv], gd[hv], s[hv]) for ch in (1, 2, 4)} for hv in halves]
    h = g4.g4_init_slice(config_for(w, mode=1, prod=1, g_in=1, acc=acc, batch=3,
                                    flags=g4.G4_F_PACKED | g4.G4_F_GRAPH))
    counts = [0, 0]
    try:
        for it in range(8):
            j = it % 2
            g4.g4_accumulate(h, du[halves[j]], dd[halves[j]], s[halves[j]])
            counts[j] += 1
            torch.cuda.synchronize()
            _ = (du.abs().sum() + dd.abs().sum()).item()    # eager work between replays
            for ch in (1, 2, 4):
                got = g4.g4_readback(h, ch)
                exp = counts[0] * want[0][ch] + counts[1] * want[1][ch]
                check_entries(got, exp, 1e-6, what="call %d channel %d" % (it, ch))
        st = g4.g4_stats(h)
        assert st["launches"] == 8 and st["measurements"] == 24
    finally:
        g4.g4_destroy(h)


EDGE = [Workload("1x1-nw2", lx=1, ly=1, nw=2, nwex=1, nq=1, q_begin=0, q_end=1, beta=3.0,
                 seed=24, wid=24, channels=ALL),
        Workload("nw256", lx=2, ly=1, nw=256, nwex=2, nq=2, q_begin=1, q_end=4, beta=20.0,
                 seed=25, wid=25, channels=ALL),
        Workload("1x5-nwex9", lx=1, ly=5, nw=6, nwex=9, nq=5, q_list=(3, 1, 4, 0, 2), q_begin=7,
                 q_end=38, beta=4.0, seed=26, wid=26, channels=ALL)]


@pytest.mark.parametrize("w", EDGE, ids=lambda w: w.name)
def test_edge_shapes_every_variant(w):
    """Degenerate and maximum shapes: a 1x1 cluster with two frequencies, the
    largest frequency count (256, one K2 row per 256-thread sweep), a 1x5
    cluster with more transfers than a plane group holds; plain FP64 and every
    batched variant that accepts the shape, against the oracle."""
    g4 = g4mod()
    count = 3
    gu, gd, s = host_inputs(w, count)
    want = oracle_out(w, count, w.channels)
    got, _ = run_slice(config_for(w, mode=0), to_dev(gu, 0), to_dev(gd, 0), s)
    check(got, want, 1e-12)
    ran = 0
    for flags in (0, g4.G4_F_MFMA, g4.G4_F_PACKED, g4.G4_F_PACKED_DEEP, g4.G4_F_PACKED | g4.G4_F_MFMA):
        cfg = config_for(w, mode=1, prod=1, g_in=1, acc=0, batch=2, flags=flags)
        try:
            g4.g4_slice_size(cfg)
        except g4.G4Error as e:
            assert e.code == g4.G4_E_UNSUPPORTED, (flags, e)
            continue
        got, _ = run_slice(cfg, to_dev(gu, 1), to_dev(gd, 1), s)
        check(got, want, 1e-6)
        ran += 1
    assert ran >= 2


@pytest.mark.parametrize("accs", [(0, 0), (1, 1), (0, 1), (1, 0)],
                         ids=["c128+c128", "kahan+kahan", "c128+kahan", "kahan+c128"])
def test_merge_of_replicas_and_slice_files(tmp_path, accs):
    """Sub-ring reduction: two replicas of the same planes, each fed half of the
    measurements, merged into one; and a slice written to a file in ranges and
    read back into a fresh slice."""
    from paper_2105_00027_amd import slice_io
    g4 = g4mod()
    w = RAGGED
    gu, gd, s = host_inputs(w, 6)
    want = oracle_out(w, 6, w.channels)
    du, dd = to_dev(gu, 1), to_dev(gd, 1)
    mk = lambda acc: g4.g4_init_slice(config_for(w, mode=1, prod=1, g_in=1, acc=acc, batch=3,
                                                 flags=g4.G4_F_PACKED))
    a, b, c = mk(accs[0]), mk(accs[1]), mk(accs[0])
    try:
        g4.g4_accumulate(a, du[:3], dd[:3], s[:3])
        g4.g4_accumulate(b, du[3:], dd[3:], s[3:])
        slice_io.reduce_slices(a, b)
        st = g4.g4_stats(a)
        assert st["measurements"] == 6 and st["sign_sum"] == s.sum()
        got = {ch: g4.g4_readback(a, ch).reshape(want[ch].shape) for ch in (1, 2, 4)}
        check(got, want, 1e-6)
        slice_io.save_slice(a, str(tmp_path / "slice"), chunk=1000)
        slice_io.load_slice(c, str(tmp_path / "slice"), chunk=777)
        assert g4.g4_stats(c)["measurements"] == 6
        for ch in (1, 2, 4):
            back = g4.g4_readback(c, ch)
            if accs[0] == 0:
                assert np.array_equal(back, got[ch].reshape(-1))
            else:
                assert rel_fro(back, got[ch].reshape(-1)) < 1e-12
        with pytest.raises(g4.G4Error) as e:
            g4.g4_merge(a, a)
        assert e.value.code == g4.G4_E_ARG
    finally:
        for h in (a, b, c):
            g4.g4_destroy(h)
    other = g4.g4_init_slice(config_for(w.with_(q_begin=4), mode=1, prod=1, g_in=1, batch=3))
    d = mk(0)
    try:
        with pytest.raises(g4.G4Error) as e:
            g4.g4_merge(d, other)
        assert e.value.code == g4.G4_E_ARG
    finally:
        g4.g4_destroy(other)
        g4.g4_destroy(d)


ONE_HOT = [(0, 0, 0), (0, 5, 7), (1, 31, 2), (0, 167, 0), (1, 100, 167), (0, 27, 28)]


@pytest.mark.parametrize("mode,prod,flags", [(0, 0, 0), (1, 1, 0), (1, 1, 16), (1, 1, 32)],
                         ids=["plain-fp64", "batched-fp32", "packed", "deep"])
def test_one_hot_support(mode, prod, flags):
    w = RAGGED
    g_in = 0 if prod == 0 else 1
    for spin, r, c in ONE_HOT:
        gu = np.zeros((1, w.ng, w.ng), dtype=np.complex128)
        gd = np.zeros_like(gu)
        (gu if spin == 0 else gd)[0, r, c] = 1.0 + 0.5j
        # a second element on the diagonal of the other spin makes direct terms appear
        (gd if spin == 0 else gu)[0, (r * 7 + 3) % w.ng, (r * 7 + 3) % w.ng] = -0.75 + 0.25j
        s = np.ones(1)
        want = {ch: ref.accumulate(w, ch, gu, gd, s) for ch in (1, 2, 4)}
        got, _ = run_slice(config_for(w, mode=mode, prod=prod, g_in=g_in, batch=1, flags=flags),
                           to_dev(gu, g_in), to_dev(gd, g_in), s)
        for ch in want:
            assert np.array_equal(got[ch] != 0, want[ch] != 0), (spin, r, c, ch)


# one-hot probes through the packed kernels that need nw = 64: the
# compile-time-nw copy (8-row tiles, plane groups of 8) and the MFMA-direct
# kernel (also 8-row tiles); W8 has Ng = 4 x 71 = 284
ONE_HOT_W8 = [(0, 0, 0), (0, 5, 77), (1, 70, 71), (0, 283, 0), (1, 150, 283), (0, 142, 213)]


@pytest.mark.parametrize("flags,tile", [(16, 8), (24, 8)], ids=["packed-nw64-t8", "packed-mfma"])
@pytest.mark.parametrize("channels", [PH_MAGNETIC, PH_CHARGE], ids=["mag", "chg"])
def test_one_hot_support_nw64(flags, tile, channels):
    w = W8.with_(channels=channels)
    for spin, r, c in ONE_HOT_W8:
        gu = np.zeros((1, w.ng, w.ng), dtype=np.complex128)
        gd = np.zeros_like(gu)
        (gu if spin == 0 else gd)[0, r, c] = 1.0 + 0.5j
        (gd if spin == 0 else gu)[0, (r * 7 + 3) % w.ng, (r * 7 + 3) % w.ng] = -0.75 + 0.25j
        s = np.ones(1)
        want = ref.accumulate(w, channels, gu, gd, s)
        got, st = run_slice(config_for(w, mode=1, prod=1, g_in=1, batch=1, tile=tile, flags=flags),
                            to_dev(gu, 1), to_dev(gd, 1), s)
        assert st["tile"] == tile
        assert np.array_equal(got[channels] != 0, want != 0), (spin, r, c)


@pytest.mark.parametrize("group,flags", [(4, 16), (4, 24), (1, 0), (8, 16)],
                         ids=["g4-packed", "g4-packed-mfma", "g1-valu", "g8-packed-nwex3"])
def test_plane_group_override(group, flags, monkeypatch):
    """G4_PLANE_GROUP sets the transfer planes per work tile (a measurement
    aid): groups of 4 or 1 on Nwex = 8, groups of 8 on Nwex = 3 (always
    partial), against the oracle."""
    monkeypatch.setenv("G4_PLANE_GROUP", str(group))
    g4 = g4mod()
    w = MULTI.with_(channels=PH_MAGNETIC | PH_CHARGE) if group == 8 else W8.with_(channels=PH_MAGNETIC | PH_CHARGE)
    gu, gd, s = host_inputs(w, 5)
    cfg = config_for(w, mode=1, prod=1, g_in=1, acc=0, batch=2, flags=flags)
    got, st = run_slice(cfg, to_dev(gu, 1), to_dev(gd, 1), s)
    check(got, oracle_out(w, 5, w.channels), 1e-6)


def test_determinism_bitwise():
    """Every slice entry is written by one thread, no atomics: two runs agree
    bit for bit (also a race check of the LDS staging)."""
    mag = MULTI.with_(channels=PH_MAGNETIC)
    for w, kw in ((MULTI, dict(mode=0)), (MULTI, dict(mode=1, prod=1, g_in=1, acc=1, batch=3)),
                  (MULTI, dict(mode=1, prod=1, g_in=1, acc=0, batch=2, flags=16)),
                  (MULTI, dict(mode=1, prod=1, g_in=1, acc=0, batch=3, flags=32)),
                  (mag, dict(mode=1, prod=1, g_in=1, acc=0, batch=3, flags=24)),       # packed, MFMA direct
                  (NW128.with_(channels=PH_MAGNETIC),
                   dict(mode=1, prod=1, g_in=1, acc=0, batch=2, flags=16))):            # a in registers
        gu, gd, s = host_inputs(w, 3)
        cfg = config_for(w, **kw)
        a, _ = run_slice(cfg, to_dev(gu, cfg.c.g_in), to_dev(gd, cfg.c.g_in), s)
        b, _ = run_slice(cfg, to_dev(gu, cfg.c.g_in), to_dev(gd, cfg.c.g_in), s)
        for ch in a:
            assert np.array_equal(a[ch], b[ch])


def test_slice_union_bitwise():
    w = RAGGED
    gu, gd, s = host_inputs(w, 3)
    dgu, dgd = to_dev(gu, 0), to_dev(gd, 0)
    full, _ = run_slice(config_for(w, mode=0, q_begin=0, q_end=w.nQ), dgu, dgd, s)
    cuts = [0, 4, 5, 13, 22, w.nQ]
    parts = [run_slice(config_for(w, mode=0, q_begin=a, q_end=b), dgu, dgd, s)[0]
             for a, b in zip(cuts[:-1], cuts[1:])]
    for ch in full:
        assert np.array_equal(np.concatenate([p[ch] for p in parts]), full[ch])


@pytest.mark.parametrize("kw", [dict(mode=0), dict(mode=1, prod=1, g_in=1, acc=1, batch=2),
                                dict(mode=1, prod=1, g_in=1, acc=2, batch=2)],
                         ids=["plain", "kahan", "c64"])
def test_checkpoint_resume(kw):
    g4 = g4mod()
    w = RAGGED
    gu, gd, s = host_inputs(w, 6)
    cfg = config_for(w, **kw)
    dgu, dgd = to_dev(gu, cfg.c.g_in), to_dev(gd, cfg.c.g_in)
    whole, st_whole = run_slice(cfg, dgu, dgd, s)
    h = g4.g4_init_slice(cfg)
    g4.g4_accumulate(h, dgu[:4], dgd[:4], s[:4])
    saved = {ch: g4.g4_readback(h, ch) for ch in (1, 2, 4)}
    st = g4.g4_stats(h)
    g4.g4_destroy(h)
    h = g4.g4_init_slice(cfg)
    for ch, v in saved.items():
        g4.g4_load(h, ch, 0, v)
    g4.g4_set_counts(h, st["measurements"], st["sign_sum"])
    g4.g4_accumulate(h, dgu[4:], dgd[4:], s[4:])
    st2 = g4.g4_stats(h)
    res = {ch: g4.g4_readback(h, ch).reshape(whole[ch].shape) for ch in (1, 2, 4)}
    g4.g4_destroy(h)
    assert st2["measurements"] == 6 and st2["sign_sum"] == s.sum()
    for ch in whole:
        if kw["mode"] == 0:
            assert np.array_equal(res[ch], whole[ch])
        else:
            # a float accumulator restarts from its own rounded value
            assert rel_fro(res[ch], whole[ch]) < 1e-6


def test_device_generator_matches_host():
    import torch
    g4 = g4mod()
    w = RAGGED
    gu, gd, _ = host_inputs(w, 2, b0=5)
    for dtype, tdt in ((0, torch.complex128), (1, torch.complex64)):
        for spin, host in ((0, gu), (1, gd)):
            out = torch.empty((2, w.ng, w.ng), dtype=tdt, device="cuda")
            g4.g4_synth_fill(out, dtype, w.lx, w.ly, w.nw, w.nwex, w.beta, w.t, w.mu, w.h,
                             w.noise, w.seed, w.wid, 5, 2, spin)
            torch.cuda.synchronize()
            dev = out.cpu().numpy().astype(np.complex128)
            tol = 1e-14 if dtype == 0 else 1e-7
            assert np.abs(dev - host).max() <= tol * np.abs(host).max()


def test_argument_errors_on_device():
    import torch
    g4 = g4mod()
    w = RAGGED
    cfg = config_for(w, mode=0)
    h = g4.g4_init_slice(cfg)
    try:
        small = torch.zeros((1, w.ng, w.ng - 1), dtype=torch.complex128, device="cuda")
        with pytest.raises(g4.G4Error) as e:
            g4.g4_accumulate(h, small, small, [1.0])
        assert e.value.code == g4.G4_E_ARG
        wrong = torch.zeros((1, w.ng, w.ng), dtype=torch.complex64, device="cuda")
        with pytest.raises(g4.G4Error):
            g4.g4_accumulate(h, wrong, wrong, [1.0])
        with pytest.raises(g4.G4Error) as e:
            g4.g4_readback(h, 1, h.entries - 1, 2)
        assert e.value.code == g4.G4_E_ARG
        with pytest.raises(g4.G4Error) as e:
            g4.g4_readback(h, 8, 0, 1)
        assert e.value.code == g4.G4_E_ARG
        g4.g4_accumulate(h, torch.zeros((0,), dtype=torch.complex128, device="cuda"),
                         torch.zeros((0,), dtype=torch.complex128, device="cuda"), [], 0)
        assert g4.g4_stats(h)["measurements"] == 0
    finally:
        g4.g4_destroy(h)


@pytest.mark.parametrize("g_in", [0, 1], ids=["c128-in", "c64-in"])
def test_check_finite_screens_g(g_in):
    """G4_F_CHECK_FINITE: a call whose G_up or G_dn holds a NaN or an infinity
    (or whose signs are not finite) is rejected with G4_E_ARG and accumulates
    nothing; a clean call then accumulates as usual."""
    g4 = g4mod()
    w = RAGGED
    gu, gd, s = host_inputs(w, 3)
    mode = dict(mode=0) if g_in == 0 else dict(mode=1, prod=1, g_in=1, batch=3)
    h = g4.g4_init_slice(config_for(w, flags=g4.G4_F_CHECK_FINITE, **mode))
    try:
        for spin, bad in ((0, np.nan), (1, np.inf), (1, complex(0, -np.inf))):
            u, d = gu.copy(), gd.copy()
            (u if spin == 0 else d)[2, w.ng - 1, 7] = bad
            with pytest.raises(g4.G4Error) as e:
                g4.g4_accumulate(h, to_dev(u, g_in), to_dev(d, g_in), s)
            assert e.value.code == g4.G4_E_ARG and "finite" in str(e.value)
        with pytest.raises(g4.G4Error) as e:
            g4.g4_accumulate(h, to_dev(gu, g_in), to_dev(gd, g_in), [1.0, np.nan, 1.0])
        assert e.value.code == g4.G4_E_ARG
        st = g4.g4_stats(h)
        assert st["measurements"] == 0 and st["launches"] == 0
        for ch in (1, 2, 4):
            assert np.count_nonzero(g4.g4_readback(h, ch)) == 0
        g4.g4_accumulate(h, to_dev(gu, g_in), to_dev(gd, g_in), s)
        got = {ch: g4.g4_readback(h, ch).reshape(w.planes, w.n, w.n) for ch in (1, 2, 4)}
    finally:
        g4.g4_destroy(h)
    check(got, oracle_out(w, 3, w.channels), 1e-12 if g_in == 0 else 1e-6)


@pytest.mark.parametrize("w,count,B,channels", [(MULTI, 5, 4, ALL), (MULTI, 4, 3, PH_CHARGE),
                                               (MULTI, 3, 2, PH_MAGNETIC | PH_CHARGE),
                                               (NW128, 5, 4, PH_MAGNETIC)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_batched_fp32_mfma_direct(w, count, B, channels):
    """Direct term on the matrix cores (paired measurements, odd tails padded)."""
    g4 = g4mod()
    w = w.with_(channels=channels)
    gu, gd, s = host_inputs(w, count)
    cfg = config_for(w, mode=1, prod=1, g_in=1, acc=0, batch=B, flags=g4.G4_F_MFMA)
    got, st = run_slice(cfg, to_dev(gu, 1), to_dev(gd, 1), s)
    assert st["variant"] == 1 and st["tile"] == 16
    check(got, oracle_out(w, count, channels), 1e-6)


def test_mfma_register_budget_rejected():
    g4 = g4mod()
    w = NW128.with_(channels=PH_MAGNETIC | PH_CHARGE)     # 2 channels x 2 slabs x 8 planes
    with pytest.raises(g4.G4Error) as e:
        g4.g4_init_slice(config_for(w, mode=1, prod=1, g_in=1, batch=2, flags=g4.G4_F_MFMA))
    assert e.value.code == g4.G4_E_UNSUPPORTED


def test_set_plan_switches_variant_and_batch():
    g4 = g4mod()
    w = MULTI.with_(channels=PH_MAGNETIC)
    gu, gd, s = host_inputs(w, 11)
    want = oracle_out(w, 11, PH_MAGNETIC)
    h = g4.g4_init_slice(config_for(w, mode=1, prod=1, g_in=1, acc=0, batch=4))
    try:
        du, dd = to_dev(gu, 1), to_dev(gd, 1)
        g4.g4_accumulate(h, du[:2], dd[:2], s[:2])
        g4.g4_set_plan(h, 0, 3, 1)                    # MFMA, passes of 3
        assert g4.g4_stats(h)["variant"] == 1
        g4.g4_accumulate(h, du[2:5], dd[2:5], s[2:5])
        g4.g4_set_plan(h, 8, 1, 0)                    # back to VALU, tile 8, passes of 1
        st = g4.g4_stats(h)
        assert st["variant"] == 0 and st["tile"] == 8 and st["batch"] == 1
        g4.g4_accumulate(h, du[5:6], dd[5:6], s[5:6])
        g4.g4_set_plan(h, 0, 2, g4.G4_VARIANT_PACKED)  # packed operands, passes of 2
        st = g4.g4_stats(h)
        assert st["variant"] == 2 and st["batch"] == 2
        g4.g4_accumulate(h, du[6:8], dd[6:8], s[6:8])
        g4.g4_set_plan(h, 0, 0, g4.G4_VARIANT_PACKED_DEEP)  # deep blocks, same pass size
        assert g4.g4_stats(h)["variant"] == 3
        g4.g4_accumulate(h, du[8:9], dd[8:9], s[8:9])
        g4.g4_set_plan(h, 0, 0, g4.G4_VARIANT_PACKED_MFMA)  # packed, direct term on MFMA
        st = g4.g4_stats(h)
        assert st["variant"] == 4 and st["tile"] == 8
        g4.g4_accumulate(h, du[9:], dd[9:], s[9:])
        got = g4.g4_readback(h, 1).reshape(want[1].shape)
        with pytest.raises(g4.G4Error):
            g4.g4_set_plan(h, 0, 5, 0)                # above the allocated max_batch
    finally:
        g4.g4_destroy(h)
    assert rel_fro(got, want[1]) <= 1e-6


def test_autotune_installs_a_plan_and_keeps_parity(tmp_path, monkeypatch):
    g4 = g4mod()
    w = MULTI.with_(channels=PH_MAGNETIC)
    gu, gd, s = host_inputs(w, 8)
    du, dd = to_dev(gu, 1), to_dev(gd, 1)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("G4_AUTOTUNE_CACHE", str(cache))
    cfg = config_for(w, mode=1, prod=1, g_in=1, acc=0, batch=8)
    h = g4.g4_init_slice(cfg)
    try:
        r = g4.g4_autotune(h, du, dd, s, 8, 1e-6)
        assert r["candidates"] >= 4 and r["batch"] in (4, 8) and r["rel_err_fp64"] <= 1e-6
        st = g4.g4_stats(h)
        assert st["measurements"] == 0 and st["batch"] == r["batch"] and st["tile"] == r["tile"]
        assert np.count_nonzero(g4.g4_readback(h, 1)) == 0          # left zeroed
        g4.g4_accumulate(h, du, dd, s)
        got = g4.g4_readback(h, 1).reshape(w.planes, w.n, w.n)
        with pytest.raises(g4.G4Error) as e:
            g4.g4_autotune(h, du, dd, s, 8, 1e-6)
        assert e.value.code == g4.G4_E_STATE
    finally:
        g4.g4_destroy(h)
    assert rel_fro(got, oracle_out(w, 8, PH_MAGNETIC)[1]) <= 1e-6
    h = g4.g4_init_slice(cfg)
    try:
        r2 = g4.g4_autotune(h, du, dd, s, 8, 1e-6)          # from the cache
        assert r2["candidates"] == 0 and (r2["batch"], r2["tile"], r2["variant"]) == \
            (r["batch"], r["tile"], r["variant"])
    finally:
        g4.g4_destroy(h)
