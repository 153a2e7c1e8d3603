"""Slice files: a slice's accumulators streamed to disk and back in bounded
ranges through g4_readback / g4_load (the paper's optional end-of-run write of
each rank's part of G_t, Implementation section), and the reduction of
same-index slices kept by replicas (g4_merge).

A slice file is a directory holding meta.json (shape, plane range, channels,
measurement count and weight sum) and one complex128 .npy array per channel
in the documented entry order [plane][K2][K1] (K1 fastest).  Host memory in
use is one range of `chunk` entries at a time.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import g4

CHANNELS = {g4.G4_PH_MAGNETIC: "ph_magnetic", g4.G4_PH_CHARGE: "ph_charge", g4.G4_PP_UPDOWN: "pp_updown",
            g4.G4_PH_LONG_UPUP: "ph_long_upup", g4.G4_PH_LONG_UPDOWN: "ph_long_updown",
            g4.G4_PH_TRANSVERSE: "ph_transverse", g4.G4_PP_SINGLET: "pp_singlet",
            g4.G4_PP_TRIPLET: "pp_triplet"}


def _meta(h: g4.Slice) -> dict:
    c = h.cfg.c
    st = g4.g4_stats(h)
    q = h.cfg._q
    return {"lx": c.lx, "ly": c.ly, "nw": c.nw, "nwex": c.nwex, "nq": c.nq,
            "q_list": [int(x) for x in q] if q is not None else list(range(c.nq)),
            "q_begin": c.q_begin, "q_end": c.q_end, "channels": c.channels, "entries": h.entries,
            "measurements": st["measurements"], "sign_sum": st["sign_sum"]}


def save_slice(h: g4.Slice, path: str, chunk: int = 1 << 22) -> None:
    """Write every channel of slice h to the directory `path` (created).

    The device-to-host readback of one range overlaps the file write of the
    previous one (a writer thread; the readback and the copy into the mapped
    file both run outside the interpreter lock), so at most two ranges are
    held in host memory."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(path, exist_ok=True)
    meta = _meta(h)

    def put(out, first, data):
        out[first:first + data.shape[0]] = data

    with ThreadPoolExecutor(max_workers=1) as writer:
        for ch, name in CHANNELS.items():
            if not meta["channels"] & ch:
                continue
            out = np.lib.format.open_memmap(os.path.join(path, name + ".npy"), mode="w+",
                                            dtype=np.complex128, shape=(h.entries,))
            pending = None
            for first in range(0, h.entries, chunk):
                count = min(chunk, h.entries - first)
                data = g4.g4_readback(h, ch, first, count)
                if pending is not None:
                    pending.result()
                pending = writer.submit(put, out, first, data)
            if pending is not None:
                pending.result()
            out.flush()
            del out
    with open(os.path.join(path, "meta.json"), "w") as f:
        json.dump(meta, f, indent=1)


def load_slice(h: g4.Slice, path: str, chunk: int = 1 << 22) -> None:
    """Load the directory `path` into slice h (same shape, planes and channels),
    replacing its accumulators, measurement count and weight sum."""
    with open(os.path.join(path, "meta.json")) as f:
        meta = json.load(f)
    mine = _meta(h)
    for k in ("lx", "ly", "nw", "nwex", "nq", "q_list", "q_begin", "q_end", "channels", "entries"):
        if meta[k] != mine[k]:
            raise ValueError("slice file %s: %s is %r, the slice has %r" % (path, k, meta[k], mine[k]))
    # the device load reads each range straight from the mapped file (no
    # host copy of its own; a reader thread that copied the next range out
    # ahead took 0.21 s against 0.08 s for a 2.15 GB channel in page cache)
    for ch, name in CHANNELS.items():
        if not meta["channels"] & ch:
            continue
        src = np.load(os.path.join(path, name + ".npy"), mmap_mode="r")
        if src.shape != (h.entries,):
            raise ValueError("slice file %s: %s holds %r entries, the slice has %d"
                             % (path, name, src.shape, h.entries))
        for first in range(0, h.entries, chunk):
            count = min(chunk, h.entries - first)
            g4.g4_load(h, ch, first, np.asarray(src[first:first + count]))
        del src
    g4.g4_set_counts(h, meta["measurements"], meta["sign_sum"])


def reduce_slices(dst: g4.Slice, *others: g4.Slice) -> None:
    """Add the slices `others` (replicas of dst's planes) into dst."""
    for s in others:
        g4.g4_merge(dst, s)
