"""Benchmark of the G4 slice accumulation on one MI355X.

Workload: the 4x4-cluster slice (Nc=16, Nw=64 fermionic frequencies, Nq=16
momentum transfers, Nwex=8 bosonic transfers; 134,217,728 entries of the
particle-hole magnetic channel), seeded synthetic Hubbard-shaped G.

A step is one g4_accumulate call of B measurements through the batched
mixed-precision path (G in complex64, FP32 products, complex128 accumulator):
direct-term gather plus the fused slice-update pass.  The plain FP64
per-measurement path (complex128 G and accumulator, one pass per measurement)
is timed on the same slice for comparison.  Inputs are resident in HBM before
the timed region; the slice is zeroed after the warm-up steps.

Printed: one JSON line with the entry-update rate (entries x measurements per
second), the dominant kernel's roofline position (its average launch time from
HIP events recorded around each launch on the stream it runs on), the sampled
error against the FP64 oracle, and the oracle's own rate on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G4 entry-updates/s per GPU (plain FP64 vs batched mixed) at stated error; % HBM/MFMA peak"
HBM_PEAK = 8.0e12                                   # bytes/s, MI355X HBM3E
ALU_PEAK = 256 * 4 * 16 * 2 * 2.4e9                 # FP32 or FP64 FMA, non-packed: 78.6 TFLOP/s
FLOPS_PER_EU = {1: 24, 2: 24, 4: 16}                 # per channel: direct 8 + exchange 16; PP 16
VARIANTS = ["valu", "mfma-direct", "packed-lds", "packed-lds-deep", "packed-lds-mfma-direct"]
KERNELS = ["update_kernel", "update_mfma_kernel", "update_packed_kernel", "update_packed_kernel",
           "update_packed_mfma_kernel"]


def algorithmic(E, ng, B, g_bytes, acc_bytes, channels):
    """Bytes and flops one update launch must move/do: accumulator read+write
    for every entry, each G element of the pass read once; flops of the
    products and sums."""
    nch = bin(channels).count("1")
    bytes_ = 2 * acc_bytes * E * nch + 2 * B * ng * ng * g_bytes
    flops = sum(FLOPS_PER_EU[c] for c in (1, 2, 4) if channels & c) * E * B
    return bytes_, flops


def roofline(E, ng, B, g_bytes, acc_bytes, channels, launch_s):
    by, fl = algorithmic(E, ng, B, g_bytes, acc_bytes, channels)
    t_hbm = by / HBM_PEAK
    t_alu = fl / ALU_PEAK
    if t_hbm >= t_alu:
        ach = by / launch_s / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": ach / (HBM_PEAK / 1e9), "traffic": None,
                "algorithmic_bytes_per_launch": by}
    ach = fl / launch_s / 1e12
    return {"bound": "alu", "achieved": ach, "peak": ALU_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": ach / (ALU_PEAK / 1e12), "traffic": None, "algorithmic_flops_per_launch": fl}


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


def sampled_error(w, h, g4, channel, b_seq, sign_seq, nsample):
    """Relative Frobenius error of sampled slice entries against the oracle."""
    from oracle import sampled
    idx = sampled.sample_indices(w, nsample, seed=777)
    got = np.array([g4.g4_readback(h, channel, int(i), 1)[0] for i in idx])
    want = np.zeros(len(idx), dtype=np.complex128)
    # the oracle sums in measurement order over the same sequence
    start = 0
    while start < len(b_seq):
        b0 = b_seq[start]
        run = 1
        while start + run < len(b_seq) and b_seq[start + run] == b0 + run:
            run += 1
        want += sampled.entries(w, channel, idx, b0=b0, count=run, sign=sign_seq[start:start + run])
        start += run
    err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    return err, len(idx)


def cpu_baseline(w, seconds):
    """The oracle, as it stands, on the host cores over a bounded sample."""
    from oracle import ref
    from synth import g_matrices, signs
    nd = 2
    gu = g_matrices(w, 0, nd, 0)
    gd = g_matrices(w, 0, nd, 1)
    s = signs(w, 0, nd)
    g4 = np.zeros((w.planes, w.n, w.n), dtype=np.complex128)
    t0 = time.perf_counter()
    ref.accumulate(w, 1, gu[:1], gd[:1], s[:1], g4=g4)
    t1 = time.perf_counter() - t0
    m = max(1, int(seconds / max(t1, 1e-3)))
    t0 = time.perf_counter()
    for j in range(m):
        ref.accumulate(w, 1, gu[j % nd:j % nd + 1], gd[j % nd:j % nd + 1], s[j % nd:j % nd + 1], g4=g4)
    t = time.perf_counter() - t0
    return {"value": w.entries * m / t, "unit": "entry-updates/s", "cores": ref.max_threads(),
            "kind": "oracle",
            "sample": "%d measurements (PH magnetic) over the whole %d-entry slice, C oracle, "
                      "OpenMP over slice rows" % (m, w.entries)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--batch", type=int, default=0,
                    help="measurements per step (the slice's max_batch); default 64, ring: 16 "
                         "(one walker's buffer; a multiple of 16 takes that many buffers per pass)")
    ap.add_argument("--workload", default="slice4x4", choices=["slice4x4", "ring6x6"],
                    help="slice4x4: the 4x4-cluster slice (default); ring6x6: rank 3's 1/8 share "
                         "of the 6x6, Nw=128 array, fed by 8 walkers' buffers of 16 measurements "
                         "in ring order")
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
    ap.add_argument("--graph", action="store_true",
                    help="replay recorded HIP graphs of the passes (warm-up covers the recording)")
    ap.add_argument("--plain-measurements", type=int, default=64)
    ap.add_argument("--plain-tile", type=int, default=0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    import torch
    from paper_2105_00027_amd import g4
    from synth import C2_PLAIN, C4_RING, signs

    ring = args.workload == "ring6x6"
    if ring:
        # rank 3 of 8: planes [216, 288) of 6x6 x 128 frequencies x (36 x 16) transfers
        w = C4_RING.with_(channels=g4.G4_PH_MAGNETIC, q_begin=3 * 72, q_end=4 * 72)
        args.batch = args.batch or 16
        args.no_cpu_baseline = True     # the oracle's full-slice array would be 24.5 GB of host memory
    else:
        w = C2_PLAIN.with_(channels=g4.G4_PH_MAGNETIC)
        args.batch = args.batch or 64
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # an explicit stream (default priority): the library enqueues on it and the
    # timing events are recorded on it
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    sptr = stream.cuda_stream
    E, ng, B = w.entries, w.ng, args.batch

    def fill(buf, dtype, b0, count, spin):
        g4.g4_synth_fill(buf, dtype, w.lx, w.ly, w.nw, w.nwex, w.beta, w.t, w.mu, w.h, w.noise,
                         w.seed, w.wid, b0, count, spin, sptr)

    def cfg(flags=0, **kw):
        return g4.Config(lx=w.lx, ly=w.ly, nw=w.nw, nwex=w.nwex, nq=w.nq, q_begin=w.q0, q_end=w.q1,
                         channels=w.channels, beta=w.beta, stream=sptr,
                         flags=g4.G4_F_KERNEL_TIMING | flags, **kw)

    out = {"metric": METRIC, "unit": "entry-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic"}

    if args.calibrate_copy:
        nb = args.calibrate_copy << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)          # reads nb bytes, writes nb bytes
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = nb
        del src, dst

    # ---- batched mixed precision (the headline) -------------------------------
    total = (args.warmup + args.steps) * B
    pool = max(B, min(args.pool, total))
    pool -= pool % B
    if ring:
        # the 8 walkers' buffers of 16 measurements, laid out in the order rank 3
        # receives them (its own walker's, then each from the left); a step takes
        # B / 16 of them in that order
        if B % 16 or 128 % B:
            ap.error("ring6x6: --batch must be 16, 32, 64 or 128")
        pool = 128
        runs = [((3 - s) % 8 * 16, 16) for s in range(8)]
    else:
        runs = [(0, pool)]
    if args.no_batched:
        args.steps = 0
        pool, runs = B, [(0, B)]
    # ids[p]: the measurement held at pool position p
    ids = np.concatenate([np.arange(b0, b0 + n) for b0, n in runs])
    gu = torch.empty((pool, ng, ng), dtype=torch.complex64, device=dev)
    gd = torch.empty_like(gu)
    pos = 0
    for b0, n in runs:
        fill(gu[pos:pos + n], g4.G4_IN_C64, b0, n, 0)
        fill(gd[pos:pos + n], g4.G4_IN_C64, b0, n, 1)
        pos += n
    sg = np.concatenate([signs(w, b0, n) for b0, n in runs])
    acc = g4.G4_ACC_C128 if args.acc == "c128" else g4.G4_ACC_C64_KAHAN
    h = g4.g4_init_slice(cfg(mode=g4.G4_MODE_BATCHED, prod=g4.G4_PROD_F32, g_in=g4.G4_IN_C64,
                             acc=acc, max_batch=B, tile=args.tile,
                             flags=(g4.G4_F_GRAPH if args.graph else 0) |
                                   (g4.G4_F_MFMA if args.mfma else 0) |
                                   (g4.G4_F_PACKED if args.packed else 0) |
                                   (g4.G4_F_PACKED_DEEP if args.deep else 0)))
    nblk = pool // B
    if not args.no_autotune:
        tune = g4.g4_autotune(h, gu[:B], gd[:B], sg[:B], B, 1e-6)
        out["autotune"] = tune

    def step(i):
        j = i % nblk
        g4.g4_accumulate(h, gu[j * B:(j + 1) * B], gd[j * B:(j + 1) * B], sg[j * B:(j + 1) * B])

    # with graphs every pool block is used twice before timing (run, then record)
    for i in range(max(args.warmup, 2 * nblk if args.graph else 0)):
        step(i)
    g4.g4_sync(h)
    g4.g4_reset(h)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    b_seq = []
    e0.record(stream)
    for i in range(args.steps):
        step(args.warmup + i)
        j = (args.warmup + i) % nblk
        b_seq.extend(range(j * B, (j + 1) * B))
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    st = g4.g4_stats(h)
    launch_s = st["kernel_ms"] / max(1, st["timed_launches"]) / 1e3
    value = E * args.steps * B / (ms / 1e3) if args.steps else 0.0
    out["value"] = value
    out["ms_per_step"] = ms / max(1, args.steps)
    shape = ("%dx%d Hubbard cluster G4 slice: Nc=%d, Nw=%d, Nq=%d, Nwex=%d, planes [%d, %d)"
             % (w.lx, w.ly, w.nc, w.nw, w.nq, w.nwex, w.q0, w.q1))
    if ring:
        shape += ", 8 walkers' buffers of 16 measurements in ring order"
    out["config"] = {"workload": shape +
                                 ", E=%d entries, PH magnetic, %d measurements per step in passes "
                                 "of %d, complex64 G, FP32 products, %s accumulator"
                                 % (E, B, st["batch"], args.acc),
                     "entries": E, "measurements_per_step": B, "pass_batch": st["batch"],
                     "tile": st["tile"], "accumulator": args.acc,
                     "kernel_variant": VARIANTS[st["variant"]],
                     "measurements_timed": args.steps * B}
    out["kernel"] = {"name": KERNELS[st["variant"]],
                     "avg_launch_ms": launch_s * 1e3, "launches": st["timed_launches"]}
    out["roofline"] = roofline(E, ng, st["batch"], 8, 16, w.channels, launch_s) if args.steps else None
    if out["roofline"]:
        out["roofline"]["traffic"] = measured_traffic(
            {"mode": 1, "acc": acc, "batch": st["batch"], "tile": st["tile"],
             "variant": st["variant"], "channels": w.channels, "entries": E})
    if not args.no_check and args.steps:
        err, ns = sampled_error(w, h, g4, 1, [int(ids[p]) for p in b_seq], sg[b_seq], 256)
        out["error"] = {"rel_fro_vs_fp64_oracle": err, "sampled_entries": ns, "gate": 1e-6}
    g4.g4_destroy(h)
    del gu, gd
    torch.cuda.empty_cache()

    # ---- plain FP64, one pass per measurement ------------------------------
    if not args.no_plain:
        M = args.plain_measurements
        pu = torch.empty((M, ng, ng), dtype=torch.complex128, device=dev)
        pd = torch.empty_like(pu)
        fill(pu, g4.G4_IN_C128, 0, M, 0)
        fill(pd, g4.G4_IN_C128, 0, M, 1)
        ps = signs(w, 0, M)
        hp = g4.g4_init_slice(cfg(mode=g4.G4_MODE_PLAIN, tile=args.plain_tile))
        g4.g4_accumulate(hp, pu[:2], pd[:2], ps[:2])      # warm-up
        g4.g4_sync(hp)
        g4.g4_reset(hp)
        torch.cuda.synchronize()
        e0.record(stream)
        g4.g4_accumulate(hp, pu, pd, ps)
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1)
        pst = g4.g4_stats(hp)
        plaunch = pst["kernel_ms"] / max(1, pst["timed_launches"]) / 1e3
        pval = E * M / (pms / 1e3)
        plain = {"value": pval, "unit": "entry-updates/s", "measurements": M,
                 "ms_per_measurement": pms / M, "dtype": "f64", "tile": pst["tile"],
                 "kernel_avg_launch_ms": plaunch * 1e3,
                 "roofline": roofline(E, ng, 1, 16, 16, w.channels, plaunch)}
        plain["roofline"]["traffic"] = measured_traffic(
            {"mode": 0, "acc": 0, "batch": 1, "tile": pst["tile"], "variant": 0,
             "channels": w.channels, "entries": E})
        if not args.no_check:
            err, ns = sampled_error(w, hp, g4, 1, list(range(M)), ps, 256)
            plain["error"] = {"rel_fro_vs_fp64_oracle": err, "sampled_entries": ns, "gate": 1e-12}
        g4.g4_destroy(hp)
        del pu, pd
        torch.cuda.empty_cache()
        out["plain_fp64"] = plain
        out["speedup_vs_plain_fp64"] = value / pval if value else None

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
