"""Benchmark of the G4 slice accumulation on one MI355X.

Headline workload: the 4x4-cluster slice (Nc=16, Nw=64 fermionic frequencies,
Nq=16 momentum transfers, Nwex=8 bosonic transfers; 134,217,728 entries of the
particle-hole magnetic channel), seeded synthetic Hubbard-shaped G.

A step is one g4_accumulate call of B measurements through the batched
mixed-precision path (G in complex64, FP32 products, complex128 accumulator):
the pass's staging kernel plus the fused slice-update kernel.  The timed
region is K steps; it is repeated three times and the median is reported.
The plain FP64 per-measurement path (complex128 G and accumulator, one pass
per measurement) is timed on the same slice for comparison.  Inputs are
resident in HBM before the timed region; the slice is zeroed after the
warm-up steps.

Further legs in the same JSON line (each with its rate, roofline and error):
  ring_share       one rank's 1/8 share of the 6x6, Nw=128, Nq=36, Nwex=16
                   array, fed by 8 walkers' buffers of 16 measurements in the
                   order the ring delivers them (batched FP32 and plain FP64);
  split_precision  a 1/4 slice of the 8x8, Nw=64, Nq=64, Nwex=4 array with PH
                   magnetic, PH charge and PP in one pass, compensated
                   complex64 accumulators, FP32 products and the fp16 / bf16
                   hi+lo split direct term;
  gsigma           G_sigma of the 4x4 window (Ng = 1136) from seeded expansion
                   configurations of order n = 512, 64 measurements per call,
                   complex64 and complex128 (the step before the slice update);
  multi_orbital    the whole multi-orbital G4 of a 2x2 cluster with 4 orbitals
                   (Nw = 32, Nwex = 4, all 16 transfer planes: 67M entries per
                   channel), PH magnetic, 64 measurements per launch, FP32.

Printed: one JSON line with the entry-update rate (entries x measurements per
second), the dominant kernel's roofline position (its average launch time from
HIP events recorded around each launch on the stream it runs on), the sampled
errors against the FP64 oracle (relative Frobenius and the paper's Eq. (2)
and (3) on real and imaginary parts), and the oracle's own rate on the host
cores (all of them, and one).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G4 entry-updates/s per GPU (plain FP64 vs batched mixed) at stated error; % HBM/MFMA peak"
HBM_PEAK = 8.0e12                                   # bytes/s, MI355X HBM3E
ALU_PEAK = 256 * 4 * 16 * 2 * 2.4e9                 # FP32 or FP64 FMA, non-packed: 78.6 TFLOP/s
MFMA_F32_PEAK = 157.3e12                            # dense FP32 MFMA
MFMA_F16_PEAK = 2.5e15                              # dense fp16 / bf16 MFMA
MFMA_F64_PEAK = 78.6e12                             # dense FP64 MFMA
FLOPS_PER_EU = {1: 24, 2: 24, 4: 16}                 # per channel: direct 8 + exchange 16; PP 16
DIRECT_FLOPS = 8                                     # the PH direct term's share
VARIANTS = ["valu", "mfma-direct", "packed-lds", "packed-lds-deep", "packed-lds-mfma-direct"]
KERNELS = ["update_kernel", "update_mfma_kernel", "update_packed_kernel", "update_packed_kernel",
           "update_packed_mfma_kernel"]
REPS = 3


def algorithmic(E, ng, B, g_bytes, acc_bytes, channels):
    """Bytes and flops one update launch must move/do: accumulator read+write
    for every entry, each G element of the pass read once; flops of the
    products and sums."""
    nch = bin(channels).count("1")
    bytes_ = 2 * acc_bytes * E * nch + 2 * B * ng * ng * g_bytes
    flops = sum(FLOPS_PER_EU[c] for c in (1, 2, 4) if channels & c) * E * B
    return bytes_, flops


def roofline(E, ng, B, g_bytes, acc_bytes, channels, launch_s, variant=0, direct_elsewhere=False):
    """Position of one update launch against its binding roof.  For plans whose
    PH direct term runs on the matrix cores (in the kernel, or in a separate
    GEMM pass) the VALU carries only the exchange and PP sums: the ALU figure
    counts those, and the direct term's flops are reported against the MFMA
    peak beside it."""
    by, fl = algorithmic(E, ng, B, g_bytes, acc_bytes, channels)
    nph = bin(channels & 3).count("1")
    mfma_direct = variant in (1, 4) or direct_elsewhere
    fl_direct = DIRECT_FLOPS * nph * E * B if mfma_direct else 0
    fl_valu = fl - fl_direct
    t_hbm = by / HBM_PEAK
    t_alu = fl_valu / ALU_PEAK
    if t_hbm >= t_alu:
        ach = by / launch_s / 1e9
        out = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
               "frac": ach / (HBM_PEAK / 1e9), "traffic": None,
               "algorithmic_bytes_per_launch": by}
    else:
        ach = fl_valu / launch_s / 1e12
        out = {"bound": "alu", "achieved": ach, "peak": ALU_PEAK / 1e12, "unit": "TFLOP/s",
               "frac": ach / (ALU_PEAK / 1e12), "traffic": None,
               "algorithmic_flops_per_launch": fl_valu}
    if fl_direct and not direct_elsewhere:
        a = fl_direct / launch_s / 1e12
        out["mfma_direct"] = {"achieved": a, "peak": MFMA_F32_PEAK / 1e12, "unit": "TFLOP/s",
                              "frac": a / (MFMA_F32_PEAK / 1e12), "flops_per_launch": fl_direct}
        # every term's flops against the vector peak: the figure a plan with the
        # direct term on the VALU reports as its frac, for comparison
        out["all_flops_vs_valu_peak"] = fl / launch_s / ALU_PEAK
    return out


def measured_traffic(plan):
    """HBM bytes per launch of the kernel that runs `plan`, from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary (scaled by its copy-kernel
    calibration), or None when no counter run covers this plan or the kernel
    sources have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
        h = hashlib.sha1()
        for name in d["source_files"]:
            with open(os.path.join(ROOT, "paper_2105_00027_amd", "csrc", name), "rb") as f:
                h.update(f.read())
    except (OSError, ValueError, KeyError):
        return None
    if h.hexdigest() != d.get("source_sha1"):
        return None
    for k in d["kernels"].values():
        if k["plan"] == plan:
            return k["bytes_per_launch"]
    return None


def paper_errors(got, want):
    """Relative Frobenius error and the paper's normalized L1 / L2 errors
    (Results section, "Accuracy Analysis", Eq. (2) and Eq. (3)) on the real
    and imaginary parts, as its Table 1 reports them."""
    def l1(a, b):
        return float(np.abs(a - b).sum() / np.abs(b).sum())

    def l2(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return {"rel_fro_vs_fp64_oracle": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
            "eq2_l1_re": l1(got.real, want.real), "eq2_l1_im": l1(got.imag, want.imag),
            "eq3_l2_re": l2(got.real, want.real), "eq3_l2_im": l2(got.imag, want.imag)}


def sampled_error(w, h, g4, channel, b_seq, sign_seq, nsample, gate):
    """Errors of sampled slice entries against the oracle, which sums the same
    measurement sequence in order."""
    from oracle import sampled
    idx = sampled.sample_indices(w, nsample, seed=777)
    got = np.array([g4.g4_readback(h, channel, int(i), 1)[0] for i in idx])
    want = np.zeros(len(idx), dtype=np.complex128)
    start = 0
    while start < len(b_seq):
        b0 = b_seq[start]
        run = 1
        while start + run < len(b_seq) and b_seq[start + run] == b0 + run:
            run += 1
        want += sampled.entries(w, channel, idx, b0=b0, count=run, sign=sign_seq[start:start + run])
        start += run
    out = paper_errors(got, want)
    out.update({"sampled_entries": int(len(idx)), "gate": gate})
    return out


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return None


def cpu_baseline(w, seconds):
    """The oracle, as it stands, on the host cores over a bounded sample: all
    threads OpenMP gives it, then one thread."""
    from oracle import ref
    from synth import g_matrices, signs
    nd = 2
    gu = g_matrices(w, 0, nd, 0)
    gd = g_matrices(w, 0, nd, 1)
    s = signs(w, 0, nd)
    g4 = np.zeros((w.planes, w.n, w.n), dtype=np.complex128)

    def rate(nthreads, budget):
        t0 = time.perf_counter()
        ref.accumulate(w, 1, gu[:1], gd[:1], s[:1], g4=g4, nthreads=nthreads)
        t1 = time.perf_counter() - t0
        m = max(1, int(budget / max(t1, 1e-3)))
        t0 = time.perf_counter()
        for j in range(m):
            ref.accumulate(w, 1, gu[j % nd:j % nd + 1], gd[j % nd:j % nd + 1], s[j % nd:j % nd + 1],
                           g4=g4, nthreads=nthreads)
        return w.entries * m / (time.perf_counter() - t0), m

    cores = ref.max_threads()
    v_all, m_all = rate(cores, seconds)
    v_one, m_one = rate(1, seconds / 4)
    ref.accumulate(w, 1, gu[:0], gd[:0], s[:0], g4=g4, nthreads=cores)   # restore the thread count
    return {"value": v_all, "unit": "entry-updates/s", "cores": cores, "kind": "oracle",
            "sample": "%d measurements (PH magnetic) over the whole %d-entry slice, C oracle, "
                      "OpenMP over slice rows, %d threads" % (m_all, w.entries, cores),
            "single_thread": {"value": v_one, "unit": "entry-updates/s", "cores": 1,
                              "sample": "%d measurement(s), same slice" % m_one},
            "cpu_model": cpu_model()}


class Bench:
    def __init__(self, args):
        import torch
        from paper_2105_00027_amd import g4
        self.torch, self.g4, self.args = torch, g4, args
        self.dev = torch.device("cuda:0")
        torch.cuda.set_device(self.dev)
        # an explicit stream (default priority): the library enqueues on it and
        # the timing events are recorded on it
        self.stream = torch.cuda.Stream(device=self.dev)
        torch.cuda.set_stream(self.stream)
        self.sptr = self.stream.cuda_stream

    def fill(self, w, buf, dtype, b0, count, spin):
        self.g4.g4_synth_fill(buf, dtype, w.lx, w.ly, w.nw, w.nwex, w.beta, w.t, w.mu, w.h, w.noise,
                              w.seed, w.wid, b0, count, spin, self.sptr)

    def cfg(self, w, flags=0, **kw):
        g4 = self.g4
        return g4.Config(lx=w.lx, ly=w.ly, nw=w.nw, nwex=w.nwex, nq=w.nq, q_begin=w.q0, q_end=w.q1,
                         channels=w.channels, beta=w.beta, stream=self.sptr,
                         flags=g4.G4_F_KERNEL_TIMING | flags, **kw)

    def timed(self, fn, steps):
        torch = self.torch
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        for i in range(steps):
            fn(i)
        e1.record(self.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    def batched(self, w, B, runs, steps, warmup, prod=1, acc=0, flags=0, tile=0, autotune=False,
                err_channels=(1,), nsample=256, gate=1e-6, reps=REPS):
        """Batched leg: the pool of measurements given by runs [(b0, n), ...]
        resident in HBM, steps of B measurements taken in pool order.  Returns
        the per-repetition times, statistics, errors and the roofline."""
        g4, torch = self.g4, self.torch
        pool = sum(n for _, n in runs)
        ids = np.concatenate([np.arange(b0, b0 + n) for b0, n in runs])
        gu = torch.empty((pool, w.ng, w.ng), dtype=torch.complex64, device=self.dev)
        gd = torch.empty_like(gu)
        pos = 0
        from synth import signs
        for b0, n in runs:
            self.fill(w, gu[pos:pos + n], g4.G4_IN_C64, b0, n, 0)
            self.fill(w, gd[pos:pos + n], g4.G4_IN_C64, b0, n, 1)
            pos += n
        sg = np.concatenate([signs(w, b0, n) for b0, n in runs])
        h = g4.g4_init_slice(self.cfg(w, mode=g4.G4_MODE_BATCHED, prod=prod, g_in=g4.G4_IN_C64, acc=acc,
                                      max_batch=B, tile=tile, flags=flags))
        out = {}
        try:
            if autotune:
                out["autotune"] = g4.g4_autotune(h, gu[:B], gd[:B], sg[:B], B, gate)
            nblk = pool // B

            def step(i):
                j = i % nblk
                g4.g4_accumulate(h, gu[j * B:(j + 1) * B], gd[j * B:(j + 1) * B], sg[j * B:(j + 1) * B])

            graph = bool(flags & g4.G4_F_GRAPH)
            for i in range(max(warmup, 2 * nblk if graph else 0)):
                step(i)
            g4.g4_sync(h)
            g4.g4_reset(h)
            torch.cuda.synchronize()
            b_seq, rep_ms = [], []
            i0 = warmup
            for _ in range(reps):
                rep_ms.append(self.timed(lambda i: step(i0 + i), steps))
                for i in range(steps):
                    j = (i0 + i) % nblk
                    b_seq.extend(range(j * B, (j + 1) * B))
                i0 += steps
            st = g4.g4_stats(h)
            out["rep_ms"] = rep_ms
            out["stats"] = st
            if not self.args.no_check and steps:
                out["errors"] = {ch: sampled_error(w, h, g4, ch, [int(ids[p]) for p in b_seq], sg[b_seq],
                                                   nsample, gate) for ch in err_channels}
        finally:
            g4.g4_destroy(h)
            del gu, gd
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
        return out

    def ring_threads(self, w, k, per, S, rank, pool_bufs, flags, tile, nsample=96):
        """The multi-threaded ring on one rank: k walker threads per rank, k
        independent rings; each thread's buffer of `per` measurements is
        delivered (a device-to-device copy from a resident pool of pool_bufs
        distinct buffers, the stand-in for the receive) on that thread's own
        stream into one of its two buffers while the slice accumulates on the
        main stream.  The timed region covers the whole ring, deliveries
        included."""
        g4, torch = self.g4, self.torch
        from paper_2105_00027_amd import ring
        from synth import signs
        pool = [tuple(torch.empty((per, w.ng, w.ng), dtype=torch.complex64, device=self.dev) for _ in range(2))
                for _ in range(pool_bufs)]
        for i, (pu, pd) in enumerate(pool):
            self.fill(w, pu, g4.G4_IN_C64, i * per, per, 0)
            self.fill(w, pd, g4.G4_IN_C64, i * per, per, 1)
        src_of = lambda r, t: (r * k + t) % pool_bufs
        sg = {(r, t): signs(w, src_of(r, t) * per, per) for r in range(S) for t in range(k)}
        bufs = [[tuple(torch.empty((per, w.ng, w.ng), dtype=torch.complex64, device=self.dev) for _ in range(2))
                 for _ in range(2)] for _ in range(k)]
        copies = [torch.cuda.Stream(device=self.dev) for _ in range(k)]

        def deliver(r, t, bu, bd, stream):
            with torch.cuda.stream(stream):
                pu, pd = pool[src_of(r, t)]
                bu.copy_(pu, non_blocking=True)
                bd.copy_(pd, non_blocking=True)

        h = g4.g4_init_slice(self.cfg(w, mode=g4.G4_MODE_BATCHED, prod=g4.G4_PROD_F32, g_in=g4.G4_IN_C64,
                                      acc=g4.G4_ACC_C128, max_batch=per, tile=tile, flags=flags))
        out = {}
        try:
            ring.stream_ring_threads(h, deliver, sg, rank, S, bufs, self.stream, copies)   # warm-up
            g4.g4_sync(h)
            g4.g4_reset(h)
            torch.cuda.synchronize()
            ms = self.timed(lambda i: ring.stream_ring_threads(h, deliver, sg, rank, S, bufs, self.stream, copies), 1)
            st = g4.g4_stats(h)
            out["ms"] = ms
            out["stats"] = st
            seq = [(r, t) for r in ring.ring_order(rank, S) for t in range(k)]
            b_seq = [src_of(*x) * per + j for x in seq for j in range(per)]
            sign_seq = np.concatenate([sg[x] for x in seq])
            if not self.args.no_check:
                out["error"] = sampled_error(w, h, g4, 1, b_seq, sign_seq, nsample, 1e-6)
        finally:
            g4.g4_destroy(h)
            del pool, bufs
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
        return out

    def gsigma(self, w, n, count, c128, steps=8, warmup=2, nsample=64, check=True):
        """G_sigma of `count` configurations per call for both spins: time per
        call (HIP events on the library's stream over `steps` calls after
        `warmup`), rate, and the sampled error of two measurements against the
        oracle."""
        torch, g4 = self.torch, self.g4
        from synth import expansion_configs
        dt = torch.complex128 if c128 else torch.complex64
        tau, site, M = expansion_configs(w, 4242, count, n)
        tau_d = torch.from_numpy(tau).to(self.dev)
        site_d = torch.from_numpy(site).to(self.dev)
        M_d = torch.from_numpy(M).to(device=self.dev, dtype=dt)
        G = [torch.empty((count, w.ng, w.ng), dtype=dt, device=self.dev) for _ in range(2)]
        dtype = g4.G4_IN_C128 if c128 else g4.G4_IN_C64
        ws = torch.empty(g4.g4_gsigma_workspace(w.lx, w.ly, w.nw, w.nwex, n, count, dtype), dtype=torch.uint8,
                         device=self.dev)

        def call(i):
            g4.g4_gsigma(w.lx, w.ly, w.nw, w.nwex, w.beta, w.mu, w.h, w.t, i % 2, tau_d, site_d, M_d,
                         G[i % 2], ws, self.sptr)
        for i in range(warmup):
            call(i)
        torch.cuda.synchronize()
        ms = [self.timed(call, steps) / steps for _ in range(REPS)]
        med = statistics.median(ms)
        flops = 8.0 * count * (w.ng * n * n + w.ng * w.ng * n)
        peak = MFMA_F64_PEAK if c128 else MFMA_F32_PEAK
        out = {"dtype": "c128" if c128 else "c64", "ms_per_call": med, "rep_ms": ms,
               "value": count / (med / 1e3), "unit": "measurements/s",
               "roofline": {"bound": "mfma", "achieved": flops / (med / 1e3) / 1e12, "peak": peak / 1e12,
                            "unit": "TFLOP/s", "frac": flops / (med / 1e3) / peak, "traffic": None,
                            "algorithmic_flops_per_call": flops,
                            "timed": "whole call (g0, phases and both complex products)"}}
        if check:
            from oracle import ref
            rng = np.random.default_rng(5)
            errs = []
            Gh = G[(warmup + steps - 1) % 2].cpu().numpy().astype(np.complex128)
            spin = (warmup + steps - 1) % 2
            Mo = M if c128 else M.astype(np.complex64).astype(np.complex128)
            for b in (0, count - 1):
                idx = rng.integers(0, w.ng * w.ng, size=nsample)
                want = ref.gsigma(w, spin, tau[b], site[b], Mo[b], idx)
                got = Gh[b].reshape(-1)[idx]
                errs.append(float(np.linalg.norm(got - want) / np.linalg.norm(want)))
            out["error"] = {"rel_fro_vs_fp64_oracle": max(errs), "sampled_entries": 2 * nsample}
        del G, ws, M_d
        torch.cuda.empty_cache()
        return out

    def multi_orbital(self, w, nb, B, steps=4, warmup=1, nsample=64, check=True):
        """Multi-orbital accumulation, PH magnetic, FP32 products, B measurements
        per call into a caller-owned complex128 accumulator."""
        torch, g4 = self.torch, self.g4
        ngb = w.ng * nb
        rng = np.random.default_rng(17)
        gu_h = ((rng.normal(size=(B, ngb, ngb)) + 1j * rng.normal(size=(B, ngb, ngb))) * 0.1).astype(np.complex64)
        gd_h = ((rng.normal(size=(B, ngb, ngb)) + 1j * rng.normal(size=(B, ngb, ngb))) * 0.1).astype(np.complex64)
        s = np.where(rng.random(B) < 0.95, 1.0, -1.0)
        gu = torch.from_numpy(gu_h).to(self.dev)
        gd = torch.from_numpy(gd_h).to(self.dev)
        side = w.n * nb * nb
        acc = torch.zeros((w.planes, side, side), dtype=torch.complex128, device=self.dev)

        def call(i):
            g4.g4_accumulate_mo(w.lx, w.ly, w.nw, w.nwex, nb, w.nq, None, w.q0, w.q1, g4.G4_PH_MAGNETIC,
                                g4.G4_PROD_F32, gu, gd, s, acc, None, None, self.sptr)
        for i in range(warmup):
            call(i)
        torch.cuda.synchronize()
        acc.zero_()
        ms = [self.timed(call, steps) / steps for _ in range(REPS)]
        med = statistics.median(ms)
        E = w.planes * side * side
        launch_s = med / 1e3
        flops = 24.0 * E * B
        byts = 32.0 * E + 2.0 * B * ngb * ngb * 8
        out = {"value": E * B / launch_s, "unit": "entry-updates/s", "ms_per_call": med, "rep_ms": ms,
               "entries": E, "measurements_per_call": B,
               "roofline": {"bound": "alu", "achieved": flops / launch_s / 1e12, "peak": ALU_PEAK / 1e12,
                            "unit": "TFLOP/s", "frac": flops / launch_s / ALU_PEAK, "traffic": None,
                            "algorithmic_flops_per_launch": flops,
                            "hbm_algorithmic_bytes_per_launch": byts,
                            "hbm_frac": byts / launch_s / HBM_PEAK}}
        if check:
            from oracle import ref
            torch.cuda.synchronize()
            idx = rng.integers(0, E, size=nsample)
            got = acc.reshape(-1)[torch.from_numpy(idx).to(self.dev)].cpu().numpy()
            # the accumulator holds REPS * steps calls of the same B measurements
            want = ref.entries_mo(w, nb, 1, gu_h.astype(np.complex128), gd_h.astype(np.complex128), s,
                                  idx) * (REPS * steps)
            out["error"] = {"rel_fro_vs_fp64_oracle": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
                            "sampled_entries": nsample}
        del gu, gd, acc
        torch.cuda.empty_cache()
        return out

    def plain(self, w, M, tile=0, reps=REPS):
        """Plain FP64 leg: M measurements, one pass each, timed `reps` times."""
        g4, torch = self.g4, self.torch
        from synth import signs
        pu = torch.empty((M, w.ng, w.ng), dtype=torch.complex128, device=self.dev)
        pd = torch.empty_like(pu)
        self.fill(w, pu, g4.G4_IN_C128, 0, M, 0)
        self.fill(w, pd, g4.G4_IN_C128, 0, M, 1)
        ps = signs(w, 0, M)
        hp = g4.g4_init_slice(self.cfg(w, mode=g4.G4_MODE_PLAIN, tile=tile))
        out = {}
        try:
            g4.g4_accumulate(hp, pu[:2], pd[:2], ps[:2])      # warm-up
            g4.g4_sync(hp)
            g4.g4_reset(hp)
            torch.cuda.synchronize()
            out["rep_ms"] = [self.timed(lambda i: g4.g4_accumulate(hp, pu, pd, ps), 1) for _ in range(reps)]
            out["stats"] = g4.g4_stats(hp)
            if not self.args.no_check:
                out["errors"] = {1: sampled_error(w, hp, g4, 1, list(range(M)) * reps, np.tile(ps, reps),
                                                  256, 1e-12)}
        finally:
            g4.g4_destroy(hp)
            del pu, pd
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
        return out


def leg_line(w, res, B, steps, g_bytes, acc_bytes, plan_acc, direct_elsewhere=False):
    """Summary of a batched leg: median rate over the repetitions, kernel
    timing, roofline with measured traffic when a counter run covers the plan."""
    st = res["stats"]
    med = statistics.median(res["rep_ms"])
    nch = bin(w.channels).count("1")
    launch_s = st["kernel_ms"] / max(1, st["timed_launches"]) / 1e3
    line = {"value": w.entries * nch * steps * B / (med / 1e3), "unit": "entry-updates/s",
            "ms_per_step": med / max(1, steps), "rep_ms": res["rep_ms"],
            "pass_batch": st["batch"], "tile": st["tile"], "kernel_variant": VARIANTS[st["variant"]],
            "kernel": {"name": KERNELS[st["variant"]], "avg_launch_ms": launch_s * 1e3,
                       "launches": st["timed_launches"]}}
    line["roofline"] = None
    if launch_s > 0:     # no timed launch (--no-batched): no kernel time to put against a roof
        line["roofline"] = roofline(w.entries, w.ng, st["batch"], g_bytes, acc_bytes, w.channels, launch_s,
                                    st["variant"], direct_elsewhere)
        line["roofline"]["traffic"] = measured_traffic(
            {"mode": 1, "acc": plan_acc, "batch": st["batch"], "tile": st["tile"], "variant": st["variant"],
             "channels": w.channels, "entries": w.entries})
    if "errors" in res:
        line["error"] = res["errors"][1] if list(res["errors"]) == [1] else \
            {"channel_%d" % ch: e for ch, e in res["errors"].items()}
    return line


def plain_line(w, res, M, nch=1):
    st = res["stats"]
    med = statistics.median(res["rep_ms"])
    plaunch = st["kernel_ms"] / max(1, st["timed_launches"]) / 1e3
    line = {"value": w.entries * nch * M / (med / 1e3), "unit": "entry-updates/s", "measurements": M,
            "ms_per_measurement": med / M, "rep_ms": res["rep_ms"], "dtype": "f64", "tile": st["tile"],
            "kernel_avg_launch_ms": plaunch * 1e3,
            "roofline": roofline(w.entries, w.ng, 1, 16, 16, w.channels, plaunch)}
    line["roofline"]["traffic"] = measured_traffic(
        {"mode": 0, "acc": 0, "batch": 1, "tile": st["tile"], "variant": 0, "channels": w.channels,
         "entries": w.entries})
    if "errors" in res:
        line["error"] = res["errors"][1]
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--batch", type=int, default=0,
                    help="measurements per step (the slice's max_batch); default 64, ring: 16 "
                         "(one walker's buffer; a multiple of 16 takes that many buffers per pass)")
    ap.add_argument("--workload", default="slice4x4", choices=["slice4x4", "ring6x6"],
                    help="headline: slice4x4 (default) or ring6x6 (rank 3's 1/8 share of the 6x6, "
                         "Nw=128 array as the headline, for profiling)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default plan instead of timing the candidates first")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--acc", default="c128", choices=["c128", "kahan"])
    ap.add_argument("--mfma", action="store_true",
                    help="direct term on the matrix cores (with --packed: the packed MFMA-direct kernel)")
    ap.add_argument("--packed", action="store_true",
                    help="packed operands copied straight into LDS (the autotuner may switch)")
    ap.add_argument("--deep", action="store_true",
                    help="packed operands, 512-thread blocks, three LDS buffers")
    ap.add_argument("--persistent", action="store_true",
                    help="packed plans launch a persistent grid walking the tiles (G4_F_PERSISTENT)")
    ap.add_argument("--graph", action="store_true",
                    help="replay recorded HIP graphs of the passes (warm-up covers the recording)")
    ap.add_argument("--plain-measurements", type=int, default=64)
    ap.add_argument("--plain-tile", type=int, default=0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ring", action="store_true", help="skip the ring-share leg")
    ap.add_argument("--no-split", action="store_true", help="skip the split-precision leg")
    ap.add_argument("--no-gsigma", action="store_true", help="skip the G_sigma leg")
    ap.add_argument("--no-mo", action="store_true", help="skip the multi-orbital leg")
    ap.add_argument("--gsigma-order", type=int, default=512, help="expansion order of the G_sigma leg")
    ap.add_argument("--legs-only", action="store_true",
                    help="run only the ring-share, split-precision and G_sigma legs (profiling)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--pool", type=int, default=1024, help="distinct measurements resident in HBM")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain elementwise copy of MIB MiB (known traffic) for "
                         "scaling hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the slice is one GPU's share and no "
              "multi-GPU path is built (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    bench = Bench(args)
    g4, torch = bench.g4, bench.torch
    from synth import C2_PLAIN, C4_RING, C5_SPLIT, Workload

    out = {"metric": METRIC, "unit": "entry-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic"}

    if args.calibrate_copy:
        nb = args.calibrate_copy << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device=bench.dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)          # reads nb bytes, writes nb bytes
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = nb
        del src, dst

    ring = args.workload == "ring6x6"
    acc = g4.G4_ACC_C128 if args.acc == "c128" else g4.G4_ACC_C64_KAHAN
    vflags = ((g4.G4_F_GRAPH if args.graph else 0) | (g4.G4_F_MFMA if args.mfma else 0) |
              (g4.G4_F_PACKED if args.packed else 0) | (g4.G4_F_PACKED_DEEP if args.deep else 0) |
              (g4.G4_F_PERSISTENT if args.persistent else 0))
    ring_w = C4_RING.with_(channels=g4.G4_PH_MAGNETIC, q_begin=3 * 72, q_end=4 * 72)
    ring_runs = [((3 - s) % 8 * 16, 16) for s in range(8)]   # rank 3's order: own, then from the left

    # ---- the headline: batched mixed precision ------------------------------
    if not args.legs_only:
        if ring:
            # rank 3 of 8: planes [216, 288) of 6x6 x 128 frequencies x (36 x 16) transfers
            w = ring_w
            B = args.batch or 16
            if B % 16 or 128 % B:
                ap.error("ring6x6: --batch must be 16, 32, 64 or 128")
            runs = ring_runs
            args.no_cpu_baseline = True   # the oracle's full-slice array would be 24.5 GB of host memory
        else:
            w = C2_PLAIN.with_(channels=g4.G4_PH_MAGNETIC)
            B = args.batch or 64
            total = (args.warmup + REPS * args.steps) * B
            pool = max(B, min(args.pool, total))
            pool -= pool % B
            runs = [(0, pool)]
        steps = 0 if args.no_batched else args.steps
        res = bench.batched(w, B, runs if not args.no_batched else [(0, B)], steps, args.warmup, acc=acc,
                            flags=vflags, tile=args.tile, autotune=not args.no_autotune and steps > 0)
        head = leg_line(w, res, B, steps, 8, 16, acc)
        if "autotune" in res:
            out["autotune"] = res["autotune"]
        out["value"] = head["value"] if steps else 0.0
        out["ms_per_step"] = head["ms_per_step"]
        out["rep_ms_per_step"] = [t / max(1, steps) for t in head["rep_ms"]]
        shape = ("%dx%d Hubbard cluster G4 slice: Nc=%d, Nw=%d, Nq=%d, Nwex=%d, planes [%d, %d)"
                 % (w.lx, w.ly, w.nc, w.nw, w.nq, w.nwex, w.q0, w.q1))
        if ring:
            shape += ", 8 walkers' buffers of 16 measurements in ring order"
        out["config"] = {"workload": shape +
                                     ", E=%d entries, PH magnetic, %d measurements per step in passes "
                                     "of %d, complex64 G, FP32 products, %s accumulator"
                                     % (w.entries, B, head["pass_batch"], args.acc),
                         "entries": w.entries, "measurements_per_step": B, "pass_batch": head["pass_batch"],
                         "tile": head["tile"], "accumulator": args.acc,
                         "kernel_variant": head["kernel_variant"],
                         "measurements_timed": REPS * steps * B, "timed_repetitions": REPS,
                         "value_is": "median of the repetitions"}
        out["kernel"] = head["kernel"]
        out["roofline"] = head["roofline"] if steps else None
        if "error" in head:
            out["error"] = head["error"]

        # ---- plain FP64, one pass per measurement ----------------------------
        if not args.no_plain:
            pw = w if not ring else ring_w
            M = args.plain_measurements if not ring else 8
            out["plain_fp64"] = plain_line(pw, bench.plain(pw, M, args.plain_tile), M)
            out["speedup_vs_plain_fp64"] = out["value"] / out["plain_fp64"]["value"] if out["value"] else None

    # ---- ring share: 8 walkers' buffers in ring order -------------------------
    if not args.no_ring and not ring:
        leg = {"workload": "6x6 Hubbard cluster, Nw=128, Nq=36, Nwex=16: rank 3's 1/8 slice, planes "
                           "[216, 288), E=%d entries, PH magnetic; 8 walkers' buffers of 16 measurements "
                           "in the ring's order (3, 2, 1, 0, 7, 6, 5, 4), one buffer per pass, complex64 G, "
                           "FP32 products, packed operands (4-row tiles, direct vector a in registers), "
                           "complex128 accumulator" % ring_w.entries}
        res = bench.batched(ring_w, 16, ring_runs, 8, 2, acc=0, flags=g4.G4_F_PACKED, tile=4,
                            nsample=96, reps=REPS)
        leg["batched"] = leg_line(ring_w, res, 16, 8, 8, 16, 0)
        # the multi-threaded ring: 2 walker threads per rank, deliveries on their
        # own streams overlapping the accumulation
        k, per = 2, 16
        rt = bench.ring_threads(ring_w, k, per, 8, 3, 4, g4.G4_F_PACKED, 4)
        n_meas = 8 * k * per
        leg["streamed_threads"] = {
            "threads": k, "measurements": n_meas, "ms": rt["ms"],
            "value": ring_w.entries * n_meas / (rt["ms"] / 1e3), "unit": "entry-updates/s",
            "delivery": "device-to-device copy of each thread's buffer (16 measurements, 2 x %.0f MB) on "
                        "that thread's stream into one of its two buffers" % (per * ring_w.ng ** 2 * 8 / 1e6),
            "timed": "the whole ring, deliveries included"}
        if "error" in rt:
            leg["streamed_threads"]["error"] = rt["error"]
        if not args.no_plain:
            leg["plain_fp64"] = plain_line(ring_w, bench.plain(ring_w, 8), 8)
            leg["speedup_vs_plain_fp64"] = leg["batched"]["value"] / leg["plain_fp64"]["value"]
        out["ring_share"] = leg

    # ---- split precision: 8x8, three channels in one pass ----------------------
    if not args.no_split and not ring:
        sw = C5_SPLIT.with_(q_begin=64, q_end=128)
        leg = {"workload": "8x8 Hubbard cluster, Nw=64, Nq=64, Nwex=4: a 1/4 slice, planes [64, 128), "
                           "E=%d entries per channel, PH magnetic + PH charge + PP in one pass, 64 "
                           "measurements in passes of 32, complex64 G, compensated complex64 "
                           "accumulators" % sw.entries}
        for name, prod, gate in (("f32", g4.G4_PROD_F32, 1e-6), ("f16x2", g4.G4_PROD_F16X2, 1e-6),
                                 ("bf16x2", g4.G4_PROD_BF16X2, 2.0 ** -15 + 1e-6)):
            # packed operands for every product kind (the split kinds imply them)
            res = bench.batched(sw, 32, [(0, 64)], 2, 1, prod=prod, acc=g4.G4_ACC_C64_KAHAN, flags=g4.G4_F_PACKED,
                                err_channels=(1, 2, 4), nsample=64, gate=gate)
            line = leg_line(sw, res, 32, 2, 8, 16, g4.G4_ACC_C64_KAHAN,
                            direct_elsewhere=prod in (g4.G4_PROD_F16X2, g4.G4_PROD_BF16X2))
            line["products"] = name
            leg[name] = line
        out["split_precision"] = leg

    # ---- G_sigma from expansion configurations (the step before the update) --
    if not args.no_gsigma and not ring:
        gw = C2_PLAIN
        n, count = args.gsigma_order, 64
        out["gsigma"] = {"workload": "G_sigma of the 4x4 window (Nc=16, Nw=64, Nwex=8, Ng=%d) from seeded expansion "
                                     "configurations of order n=%d, %d measurements per call, spins alternating"
                                     % (gw.ng, n, count),
                         "c64": bench.gsigma(gw, n, count, False, check=not args.no_check),
                         "c128": bench.gsigma(gw, n, count, True, check=not args.no_check)}

    # ---- multi-orbital G4 ------------------------------------------------------
    if not args.no_mo and not ring:
        mw = Workload("mo", lx=2, ly=2, nw=32, nwex=4, nq=4, beta=10.0)
        leg = {"workload": "multi-orbital G4 of a 2x2 cluster, 4 orbitals, Nw=32, Nwex=4, all 16 transfer planes "
                           "(%d entries), PH magnetic, 64 measurements per call, complex64 G, FP32 products, "
                           "complex128 accumulator" % (mw.planes * (mw.n * 16) ** 2)}
        leg.update(bench.multi_orbital(mw, 4, 64, check=not args.no_check))
        out["multi_orbital"] = leg

    if not args.no_cpu_baseline and not args.legs_only:
        out["cpu_baseline"] = cpu_baseline(C2_PLAIN.with_(channels=g4.G4_PH_MAGNETIC), args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
