"""The in-process ring delivery: order (CPU) and double-buffered streaming on the
GPU, which must give exactly the sequential result, be invariant, to
rounding, under the rank (rotation of the order), and match the FP64 oracle
applied to the same buffers in the same order."""
import numpy as np
import pytest

from gpu_common import config_for, g4mod
from metrics import check_entries, rel_fro
from oracle import ref
from paper_2105_00027_amd.ring import ring_order
from synth import Workload, g_matrices, signs


def test_ring_order_properties():
    S = 8
    for r in range(S):
        order = ring_order(r, S)
        assert order[0] == r and sorted(order) == list(range(S))
        assert order[1] == (r - 1) % S            # first buffer comes from the left
    # after S-1 steps each walker's buffer sits at the left neighbour of its birth rank
    for w in range(S):
        last = [r for r in range(S) if ring_order(r, S)[S - 1] == w]
        assert last == [(w - 1) % S]
    with pytest.raises(ValueError):
        ring_order(8, 8)


W = Workload("ring", lx=3, ly=2, nw=24, nwex=5, nq=6, q_begin=5, q_end=23, beta=7.0, seed=31,
             wid=31, channels=7)


@pytest.mark.gpu
def test_streamed_ring_matches_sequential_and_rotation():
    import torch
    from paper_2105_00027_amd import ring
    g4 = g4mod()
    S, per = 4, 3
    main = torch.cuda.Stream()
    copy = torch.cuda.Stream()
    sg = {wk: signs(W, wk * per, per) for wk in range(S)}

    def deliver(walker, bu, bd, stream):
        for spin, buf in ((0, bu), (1, bd)):
            g4.g4_synth_fill(buf, 0, W.lx, W.ly, W.nw, W.nwex, W.beta, W.t, W.mu, W.h, W.noise,
                             W.seed, W.wid, walker * per, per, spin, stream.cuda_stream)

    def run(rank, streamed):
        cfg = config_for(W, mode=1, prod=0, g_in=0, acc=0, batch=per, stream=main.cuda_stream)
        h = g4.g4_init_slice(cfg)
        bufs = [tuple(torch.empty((per, W.ng, W.ng), dtype=torch.complex128, device="cuda")
                      for _ in range(2)) for _ in range(2)]
        try:
            if streamed:
                ring.stream_ring(h, deliver, sg, rank, S, bufs, main, copy)
            else:
                for wk in ring.ring_order(rank, S):
                    with torch.cuda.stream(main):
                        deliver(wk, bufs[0][0], bufs[0][1], main)
                        g4.g4_accumulate(h, bufs[0][0], bufs[0][1], sg[wk])
            g4.g4_sync(h)
            return {ch: g4.g4_readback(h, ch) for ch in (1, 2, 4)}
        finally:
            torch.cuda.synchronize()
            g4.g4_destroy(h)

    seq = run(2, False)
    strm = run(2, True)
    rot = run(0, True)
    for ch in (1, 2, 4):
        assert np.array_equal(seq[ch], strm[ch])
        assert rel_fro(rot[ch], seq[ch]) <= 1e-15
    # the oracle on the same buffers, in rank 2's ring order
    want = oracle_ring(2, S, per)
    for ch in (1, 2, 4):
        check_entries(strm[ch], want[ch], 1e-12, what="channel %d" % ch)


def oracle_ring(rank, S, per):
    order = ring_order(rank, S)
    gu = np.concatenate([g_matrices(W, wk * per, per, 0) for wk in order])
    gd = np.concatenate([g_matrices(W, wk * per, per, 1) for wk in order])
    s = np.concatenate([signs(W, wk * per, per) for wk in order])
    return {ch: ref.accumulate(W, ch, gu, gd, s).reshape(-1) for ch in (1, 2, 4)}


@pytest.mark.gpu
@pytest.mark.parametrize("acc", [0, 1], ids=["acc-c128", "acc-kahan"])
def test_streamed_ring_fp32_packed_matches_oracle(acc):
    """The benchmark's product path (complex64 G, FP32 products, packed operands)
    fed by the double-buffered ring delivery: two passes per walker buffer."""
    import torch
    from paper_2105_00027_amd import ring
    g4 = g4mod()
    S, per, rank = 4, 3, 1
    main = torch.cuda.Stream()
    copy = torch.cuda.Stream()
    sg = {wk: signs(W, wk * per, per) for wk in range(S)}

    def deliver(walker, bu, bd, stream):
        for spin, buf in ((0, bu), (1, bd)):
            g4.g4_synth_fill(buf, 1, W.lx, W.ly, W.nw, W.nwex, W.beta, W.t, W.mu, W.h, W.noise,
                             W.seed, W.wid, walker * per, per, spin, stream.cuda_stream)

    cfg = config_for(W, mode=1, prod=1, g_in=1, acc=acc, batch=2, flags=g4.G4_F_PACKED,
                     stream=main.cuda_stream)
    h = g4.g4_init_slice(cfg)
    bufs = [tuple(torch.empty((per, W.ng, W.ng), dtype=torch.complex64, device="cuda")
                  for _ in range(2)) for _ in range(2)]
    try:
        ring.stream_ring(h, deliver, sg, rank, S, bufs, main, copy)
        g4.g4_sync(h)
        got = {ch: g4.g4_readback(h, ch) for ch in (1, 2, 4)}
        st = g4.g4_stats(h)
    finally:
        torch.cuda.synchronize()
        g4.g4_destroy(h)
    assert st["measurements"] == S * per and st["launches"] == 2 * S
    want = oracle_ring(rank, S, per)
    for ch in (1, 2, 4):
        check_entries(got[ch], want[ch], 1e-6, what="channel %d" % ch)


@pytest.mark.gpu
@pytest.mark.parametrize("k", [2, 3, 4])
def test_multi_threaded_ring_matches_oracle(k):
    """k walker threads per rank, k independent rings (each thread index with
    its own delivery stream and buffer pair): every buffer of every thread of
    every rank is applied once, in ring order per step and thread order within
    a step; the result matches the FP64 oracle applied in that order (FP32
    products, packed operands, compensated accumulator)."""
    import torch
    from paper_2105_00027_amd import ring
    g4 = g4mod()
    S, per, rank = 3, 2, 2
    main = torch.cuda.Stream()
    copies = [torch.cuda.Stream() for _ in range(k)]

    def b0(src, t):                      # first measurement of thread t of rank src
        return (src * k + t) * per

    sg = {(r, t): signs(W, b0(r, t), per) for r in range(S) for t in range(k)}

    def deliver(src, t, bu, bd, stream):
        for spin, buf in ((0, bu), (1, bd)):
            g4.g4_synth_fill(buf, 1, W.lx, W.ly, W.nw, W.nwex, W.beta, W.t, W.mu, W.h, W.noise,
                             W.seed, W.wid, b0(src, t), per, spin, stream.cuda_stream)

    cfg = config_for(W, mode=1, prod=1, g_in=1, acc=1, batch=per, flags=g4.G4_F_PACKED,
                     stream=main.cuda_stream)
    h = g4.g4_init_slice(cfg)
    bufs = [[tuple(torch.empty((per, W.ng, W.ng), dtype=torch.complex64, device="cuda")
                   for _ in range(2)) for _ in range(2)] for _ in range(k)]
    try:
        ring.stream_ring_threads(h, deliver, sg, rank, S, bufs, main, copies)
        g4.g4_sync(h)
        got = {ch: g4.g4_readback(h, ch) for ch in (1, 2, 4)}
        st = g4.g4_stats(h)
    finally:
        torch.cuda.synchronize()
        g4.g4_destroy(h)
    assert st["measurements"] == S * k * per
    seq = [(src, t) for src in ring_order(rank, S) for t in range(k)]
    gu = np.concatenate([g_matrices(W, b0(*x), per, 0) for x in seq])
    gd = np.concatenate([g_matrices(W, b0(*x), per, 1) for x in seq])
    s = np.concatenate([sg[x] for x in seq])
    for ch in (1, 2, 4):
        want = ref.accumulate(W, ch, gu, gd, s).reshape(-1)
        check_entries(got[ch], want, 1e-6, what="channel %d" % ch)
