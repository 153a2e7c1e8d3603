"""Helpers for the GPU tests: configurations from workloads, host and device
inputs, and a run through the C-ABI library."""
import numpy as np

from synth import Workload, g_matrices, signs


def g4mod():
    from paper_2105_00027_amd import g4
    return g4


def config_for(w: Workload, mode=0, prod=0, g_in=0, acc=0, batch=1, tile=0, flags=0,
               channels=None, stream=None, q_begin=None, q_end=None):
    g4 = g4mod()
    return g4.Config(lx=w.lx, ly=w.ly, nw=w.nw, nwex=w.nwex, nq=w.nq, q_list=w.q_list,
                     q_begin=w.q0 if q_begin is None else q_begin,
                     q_end=w.q1 if q_end is None else q_end,
                     channels=w.channels if channels is None else channels,
                     g_in=g_in, prod=prod, acc=acc, mode=mode, max_batch=batch, tile=tile,
                     flags=flags, stream=stream, beta=w.beta)


def host_inputs(w: Workload, count: int, b0: int = 0):
    return g_matrices(w, b0, count, 0), g_matrices(w, b0, count, 1), signs(w, b0, count)


def to_dev(a, g_in):
    import torch
    dt = torch.complex128 if g_in == 0 else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)


def run_slice(cfg, gu_dev, gd_dev, sgn, chunks=None):
    """Accumulate (optionally in several calls), return {channel: array [planes, n, n]}."""
    g4 = g4mod()
    h = g4.g4_init_slice(cfg)
    try:
        B = len(sgn)
        bounds = [0, B] if chunks is None else chunks
        for a, b in zip(bounds[:-1], bounds[1:]):
            g4.g4_accumulate(h, gu_dev[a:b], gd_dev[a:b], sgn[a:b])
        g4.g4_sync(h)
        out = {}
        for ch in (1, 2, 4, 8, 16, 32, 64, 128):
            if cfg.c.channels & ch:
                out[ch] = g4.g4_readback(h, ch).reshape(cfg.planes, cfg.n, cfg.n)
        st = g4.g4_stats(h)
    finally:
        g4.g4_destroy(h)
    return out, st
