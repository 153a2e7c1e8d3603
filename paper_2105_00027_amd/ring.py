"""In-process stand-in for the paper's pipeline ring on one rank (Implementation
section, "Pipeline Ring Algorithm", Algorithm 1).

In the paper a rank first updates its part of G_t with the G_sigma its own
walker produced, then, for ringSize - 1 steps, receives a buffer from its left
neighbour while sending the previous one to its right neighbour, updating with
each received buffer; send and receive buffers swap roles between steps, so
the next transfer overlaps the current update.  Each buffer ends at the left
neighbour of the rank that produced it.

Here there is one GPU and no transport: the walker buffers are delivered on a
second stream into one of two device buffers while the library accumulates
the other one on the main stream (the send/receive swap), in the order the
ring would deliver them to this rank: r, r-1, ..., r-S+1 (mod S).  Only the
ordering and the double buffering are reproduced; all arithmetic is in the
library.

With k walker-accumulator threads per rank (Implementation section,
"Multi-Threaded Ring Communication", Algorithm 3) there are k independent
rings, one per thread index, and each thread holds two buffers.  Here each
thread index has its own delivery stream and buffer pair; at every ring step
the k buffers of that step are applied in thread order on the slice's
stream, while the k streams deliver the next step's buffers.
"""
from __future__ import annotations

from typing import Callable, Sequence


def ring_order(rank: int, size: int) -> list:
    """Walkers whose buffers rank `rank` applies, in order: its own, then the
    ones arriving from the left, S - 1 steps."""
    if size < 1 or not 0 <= rank < size:
        raise ValueError("rank %d outside a ring of %d" % (rank, size))
    return [(rank - j) % size for j in range(size)]


def stream_ring(h, deliver: Callable, signs: Sequence, rank: int, size: int, bufs,
                main_stream, copy_stream) -> None:
    """Accumulate every walker's buffer into slice h in ring order.

    deliver(walker, buf_up, buf_dn, stream): enqueue on `stream` the work that
        fills the two device buffers with `walker`'s G_up and G_dn (the stand-in
        for the receive).
    signs[walker]: host array of that walker's measurement weights.
    bufs: two (buf_up, buf_dn) pairs of device tensors (the swap pair).
    main_stream must be the stream the slice was created on.
    """
    import torch
    from . import g4

    order = ring_order(rank, size)
    ready = [torch.cuda.Event(), torch.cuda.Event()]
    free = [torch.cuda.Event(), torch.cuda.Event()]
    deliver(order[0], bufs[0][0], bufs[0][1], copy_stream)
    ready[0].record(copy_stream)
    for step, walker in enumerate(order):
        cur = step % 2
        if step + 1 < len(order):
            nxt = 1 - cur
            if step >= 1:
                copy_stream.wait_event(free[nxt])      # its previous contents are consumed
            deliver(order[step + 1], bufs[nxt][0], bufs[nxt][1], copy_stream)
            ready[nxt].record(copy_stream)
        main_stream.wait_event(ready[cur])
        g4.g4_accumulate(h, bufs[cur][0], bufs[cur][1], signs[walker])
        free[cur].record(main_stream)


def stream_ring_threads(h, deliver: Callable, signs, rank: int, size: int, bufs, main_stream,
                        copy_streams) -> None:
    """Accumulate the buffers of k walker threads per rank into slice h, k
    independent rings in ring order.

    deliver(src_rank, thread, buf_up, buf_dn, stream): enqueue on `stream` the
        work that fills the two device buffers with the G_up and G_dn that
        thread `thread` of rank `src_rank` produced (the stand-in for that
        thread's receive).
    signs[(src_rank, thread)]: host array of that buffer's measurement weights.
    bufs[t]: the two (buf_up, buf_dn) pairs of thread t (send/receive swap).
    copy_streams[t]: the delivery stream of thread t; main_stream must be the
        stream the slice was created on.
    """
    import torch
    from . import g4

    k = len(copy_streams)
    if len(bufs) != k or k < 1:
        raise ValueError("one buffer pair set and one stream per thread")
    order = ring_order(rank, size)
    ready = [[torch.cuda.Event(), torch.cuda.Event()] for _ in range(k)]
    free = [[torch.cuda.Event(), torch.cuda.Event()] for _ in range(k)]
    for t in range(k):
        deliver(order[0], t, bufs[t][0][0], bufs[t][0][1], copy_streams[t])
        ready[t][0].record(copy_streams[t])
    for step, src in enumerate(order):
        cur = step % 2
        if step + 1 < len(order):
            nxt = 1 - cur
            for t in range(k):
                if step >= 1:
                    copy_streams[t].wait_event(free[t][nxt])     # its previous contents are consumed
                deliver(order[step + 1], t, bufs[t][nxt][0], bufs[t][nxt][1], copy_streams[t])
                ready[t][nxt].record(copy_streams[t])
        for t in range(k):
            main_stream.wait_event(ready[t][cur])
            g4.g4_accumulate(h, bufs[t][cur][0], bufs[t][cur][1], signs[(src, t)])
            free[t][cur].record(main_stream)
