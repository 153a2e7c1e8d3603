/*
 * g4.h -- C ABI of the MI355X (gfx950) library that accumulates one GPU's
 * slice of the two-particle Green's function G4 (the paper's G_t) from
 * streamed single-particle Green's functions G_sigma.
 *
 * Paper: "Memory Reduction using a Ring Abstraction over GPU RDMA for
 * Distributed Quantum Monte Carlo Solver" (arXiv 2105.00027).
 *   - The update: Background section, "Memory-Bound Issue in DCA++", Eq. (1)
 *     (particle-particle channel), and its particle-hole counterparts
 *     (direct minus exchange Wick products; the paper prints only Eq. (1)).
 *   - The slice: Implementation section, "Distributed G_t in QMC Solver":
 *     each rank owns an even 1/p part of G_t and must see every G_sigma.
 *   - The stream of G_sigma buffers: Implementation section, "Pipeline Ring
 *     Algorithm" (Algorithm 1): a rank updates its part with its own G_sigma,
 *     then with each buffer received from its left neighbour.
 *   - Lifetime: G_t is allocated before the measurements and lives until the
 *     end of the run (Background section, the solver workflow).
 *
 * Conventions (all integer maps are exact):
 *   Cluster lx x ly, Nc = lx*ly momenta, k = ix + lx*iy.  k+q and q-k are
 *     taken coordinate-wise modulo the cluster.
 *   Fermionic Matsubara n in [-nw/2, nw/2-1] (nw even), w_n = (2n+1)pi/beta.
 *   Bosonic transfer m in [0, nwex-1], nu_m = 2 pi m/beta; so
 *     w_n + nu_m = w_{n+m} and nu_m - w_n = w_{m-n-1}.
 *   G4 combined index K = k*nw + (n + nw/2), N = Nc*nw.
 *   G frequency window n in [-nw/2, nw/2+nwex-2], Nwg = nw+nwex-1;
 *     G row/column index k*Nwg + (n + nw/2), Ng = Nc*Nwg.
 *   Transfer plane Q = (q, m), flattened iQ = iq*nwex + m, q = q_list[iq],
 *     NQ = nq*nwex planes in the full G4.
 *   The slice holds planes [q_begin, q_end); entry ((iQ-q_begin)*N + K2)*N + K1
 *     of each channel, K1 fastest.
 *
 * Per measurement b with weight s_b (the QMC sign, normally +-1):
 *   PH magnetic  G4 += s_b [ (Gu-Gd)(K1+Q,K1) (Gu-Gd)(K2,K2+Q) - sum_s G_s(K2,K1) G_s(K1+Q,K2+Q) ]
 *   PH charge    G4 += s_b [ (Gu+Gd)(K1+Q,K1) (Gu+Gd)(K2,K2+Q) - sum_s G_s(K2,K1) G_s(K1+Q,K2+Q) ]
 *   PP up-down   G4 += s_b   sum_s G_s(Q-K2,Q-K1) G_{-s}(K2,K1)          (Eq. (1), K3 -> Q)
 * and the spin-resolved particle-hole channels, from the same Wick rule on
 * c+_{K1+Q,s1} c_{K1,s2} c+_{K2,s3} c_{K2+Q,s4} with one spin assignment each:
 *   PH longitudinal up-up    G4 += s_b [ Gu(K1+Q,K1) Gu(K2,K2+Q) - Gu(K2,K1) Gu(K1+Q,K2+Q) ]
 *   PH longitudinal up-down  G4 += s_b   Gu(K1+Q,K1) Gd(K2,K2+Q)
 *   PH transverse            G4 += -s_b  sum_s G_{-s}(K2,K1) G_s(K1+Q,K2+Q)
 *     (spins (s, -s, -s, s) summed over s)
 * (magnetic = uu + dd - ud - du and charge = uu + dd + ud + du, with dd, du
 * the up-up and up-down channels of the spin-swapped pair), and the singlet
 * and triplet (S_z = 0) projections of the PP pair, with pair operators
 * (c+_{K,up} c+_{Q-K,dn} -/+ c+_{K,dn} c+_{Q-K,up})/sqrt(2):
 *   PP singlet   G4 += s_b/2 sum_s [ G_s(Q-K2,Q-K1) G_{-s}(K2,K1) + G_s(Q-K2,K1) G_{-s}(K2,Q-K1) ]
 *   PP triplet   G4 += s_b/2 sum_s [ G_s(Q-K2,Q-K1) G_{-s}(K2,K1) - G_s(Q-K2,K1) G_{-s}(K2,Q-K1) ]
 *   (singlet + triplet = PP up-down).
 * A slice holds channels of one family: a subset of {G4_PH_MAGNETIC,
 * G4_PH_CHARGE, G4_PP_UPDOWN}, of {G4_PH_LONG_UPUP, G4_PH_LONG_UPDOWN,
 * G4_PH_TRANSVERSE}, or of {G4_PP_SINGLET, G4_PP_TRIPLET}; the last two
 * families run on the register-staged (VALU) kernels.
 * The values kept are raw signed sums; g4_stats gives the measurement count
 * and the sum of weights for normalisation.
 *
 * Errors: every call returns G4_OK or a negative status, and leaves a
 * message for g4_last_error() (thread-local).  G4_E_ARG, G4_E_OOM and
 * G4_E_UNSUPPORTED change nothing.  G4_E_HIP poisons the handle: every
 * later call on it except g4_destroy returns G4_E_STATE.  Arguments are
 * validated before any HIP call.
 *
 * Threading: a handle is used by one host thread at a time.  Work is
 * enqueued on the handle's stream; calls return before the GPU finishes
 * unless documented as synchronous.
 */
#ifndef G4_H
#define G4_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define G4_ABI_VERSION 1u

enum {
    G4_OK = 0,
    G4_E_ARG = -1,          /* invalid argument or configuration */
    G4_E_OOM = -2,          /* the slice and its work buffers do not fit */
    G4_E_HIP = -3,          /* a HIP runtime call failed; handle poisoned */
    G4_E_STATE = -4,        /* poisoned handle, or call out of order */
    G4_E_UNSUPPORTED = -5   /* valid request this build does not implement */
};

/* channels (bitmask); accumulator slot 0: magnetic, up-up or PP singlet,
 * 1: charge, up-down or PP triplet, 2: PP or transverse */
enum {
    G4_PH_MAGNETIC = 1, G4_PH_CHARGE = 2, G4_PP_UPDOWN = 4,
    G4_PH_LONG_UPUP = 8, G4_PH_LONG_UPDOWN = 16, G4_PH_TRANSVERSE = 32,
    G4_PP_SINGLET = 64, G4_PP_TRIPLET = 128
};

/* element type of the G_up / G_dn buffers passed to g4_accumulate */
enum {
    G4_IN_C128 = 0,  /* complex double, interleaved (re, im): 16 bytes */
    G4_IN_C64 = 1    /* complex float, interleaved: 8 bytes */
};

/* precision of the products */
enum {
    G4_PROD_F64 = 0,     /* every product in FP64 */
    G4_PROD_F32 = 1,     /* G rounded to FP32, products and batch sums in FP32 */
    G4_PROD_BF16X2 = 2,  /* batched: exchange and PP as G4_PROD_F32; the PH direct term as a
                            complex GEMM over the pass on MFMA from split operands x = hi + lo,
                            hi = bf16(x), lo = bf16(x - hi), products hi*hi + hi*lo + lo*hi
                            (relative error per product below 2^-15), added to the slice in a
                            second read-modify-write.  Runs the packed kernels (G4_F_PACKED is
                            implied; G4_F_PACKED_DEEP may be given); not with G4_F_MFMA. */
    G4_PROD_F16X2 = 3    /* as G4_PROD_BF16X2 with hi = f16(x), lo = f16(2^11 (x - hi)) (relative
                            error per product below 2^-21); operands must stay below 65504 in
                            magnitude (fp16 range) */
};

/* accumulator held in device memory for every slice entry */
enum {
    G4_ACC_C128 = 0,        /* complex double */
    G4_ACC_C64_KAHAN = 1,   /* complex float value + complex float Kahan compensation */
    G4_ACC_C64 = 2          /* complex float, uncompensated (a control for drift studies) */
};

/* how measurements are applied */
enum {
    G4_MODE_PLAIN = 0,    /* one kernel pass over the slice per measurement */
    G4_MODE_BATCHED = 1   /* up to max_batch measurements fused in one pass */
};

/* flags */
enum {
    G4_F_CHECK_FINITE = 1u,   /* g4_accumulate rejects (G4_E_ARG, nothing accumulated) a call whose
                                 signs or G_up/G_dn elements are not all finite; G is screened by
                                 a device pass over both buffers followed by a wait, so the call
                                 returns only after the stream's earlier work has finished */
    G4_F_KERNEL_TIMING = 2u,  /* time every slice-update kernel with HIP events (see g4_stats) */
    G4_F_GRAPH = 4u,          /* batched: a pass on input pointers (and pass size) seen before is
                                 replayed as a HIP graph of its kernels, recorded on the second
                                 use (the first runs directly); the weights are uploaded before
                                 each launch.  Up to 64 recordings per slice, dropped when the
                                 plan changes.  With G4_F_KERNEL_TIMING a replayed pass is timed
                                 as a whole.  The caller's stream must not be capturing already. */
    G4_F_MFMA = 8u,           /* batched FP32: direct term on MFMA (nw = 64 or 128; 16-row tiles).
                                 With G4_F_PACKED: the packed operands of G4_F_PACKED and the
                                 direct term on MFMA in one kernel (nw = 64, 8-row tiles, PH
                                 magnetic and charge only, FP32 products). */
    G4_F_PACKED = 16u,        /* batched FP32: each pass first packs G_up and G_dn side by side
                                 (16 bytes per element, each momentum block of Nwg columns padded
                                 to a multiple of 8, with the pass's direct vectors) and the
                                 update kernel copies its operand blocks straight from that
                                 buffer into LDS; needs an even tile and max_batch * (Ng * ldp
                                 * 16 + direct vectors) more device bytes, ldp = Nc * pcb + 1
                                 rounded up to 8, pcb = Nwg rounded up to 8.  Combines with
                                 G4_F_MFMA only (see there). */
    G4_F_PACKED_DEEP = 32u,   /* as G4_F_PACKED, with 512-thread blocks and three LDS buffers
                                 (copies run two measurements ahead); one or two K2 rows per
                                 thread, tile = 512/nw or 1024/nw.  Exclusive with the others. */
    G4_F_PERSISTENT = 64u     /* packed plans (G4_F_PACKED, with or without G4_F_MFMA, and
                                 G4_F_PACKED_DEEP) launch a persistent grid: as many blocks as
                                 the device holds at once (the occupancy calculator's blocks per
                                 CU times the CU count, rounded down to a multiple of 8), each
                                 walking the pass's work tiles with a grid stride, in place of
                                 one block per tile; every pass still fuses all its measurements
                                 in one launch.  Other plans ignore the flag.  Slower than one
                                 block per tile on MI355X (tiles advance in a fixed stride instead
                                 of being handed to whichever block finishes first). */
};

/* slice-update kernel variants (g4_stats, g4_set_plan, g4_tune_result) */
enum {
    G4_VARIANT_VALU = 0,      /* operands staged through registers, all terms on the VALU */
    G4_VARIANT_MFMA = 1,      /* G4_F_MFMA */
    G4_VARIANT_PACKED = 2,    /* G4_F_PACKED */
    G4_VARIANT_PACKED_DEEP = 3, /* G4_F_PACKED_DEEP */
    G4_VARIANT_PACKED_MFMA = 4  /* G4_F_PACKED | G4_F_MFMA */
};

typedef struct g4_config {
    uint32_t abi_version;     /* G4_ABI_VERSION */
    int32_t lx, ly;           /* cluster extent, >= 1 each */
    int32_t nw;               /* G4 fermionic frequencies, even, >= 2 */
    int32_t nwex;             /* bosonic transfers, >= 1 */
    int32_t nq;               /* momentum transfers, 1..Nc */
    const int32_t *q_list;    /* host array of nq distinct momenta in [0,Nc), or NULL for 0..nq-1;
                                 copied by g4_init_slice */
    int64_t q_begin, q_end;   /* slice planes, 0 <= q_begin < q_end <= nq*nwex */
    uint32_t channels;        /* nonzero bitmask of G4_PH_MAGNETIC | G4_PH_CHARGE | G4_PP_UPDOWN,
                                 of G4_PH_LONG_UPUP | G4_PH_LONG_UPDOWN | G4_PH_TRANSVERSE, or
                                 of G4_PP_SINGLET | G4_PP_TRIPLET (one family; the last two on
                                 the VALU kernels only) */
    int32_t g_in;             /* G4_IN_* */
    int32_t prod;             /* G4_PROD_* ; G4_MODE_PLAIN requires G4_PROD_F64 */
    int32_t acc;              /* G4_ACC_* */
    int32_t mode;             /* G4_MODE_* */
    int32_t max_batch;        /* batched: measurements per pass, 1..256 (plain: ignored) */
    int32_t device;           /* HIP device ordinal */
    void *stream;             /* hipStream_t to enqueue on, or NULL for a library-owned blocking
                                 stream (ordered with work on the null stream) */
    uint32_t flags;           /* G4_F_* */
    int32_t tile;             /* rows of K2 frequencies per work tile; 0 = default */
    double beta;              /* inverse temperature; metadata only */
} g4_config;

typedef struct g4_slice g4_slice;   /* opaque; owned by the library */

typedef struct g4_stats_t {
    uint64_t measurements;     /* measurements accumulated since init/reset/load */
    double sign_sum;           /* sum of their weights */
    uint64_t launches;         /* slice-update kernel launches */
    double kernel_ms;          /* summed HIP-event time of those launches (G4_F_KERNEL_TIMING) */
    uint64_t timed_launches;   /* launches included in kernel_ms */
    uint64_t entries;          /* entries per channel in the slice */
    uint32_t channels;         /* channel bitmask */
    int32_t batch;             /* measurements per pass in use */
    int32_t tile;              /* K2 rows per tile in use */
    int32_t variant;           /* kernel variant in use (G4_VARIANT_*) */
} g4_stats_t;

/* Fill *cfg with defaults (magnetic channel, c128, FP64, plain, whole
 * slice of a 1x1 cluster).  Returns G4_E_ARG for NULL.
 * Paper: Implementation section, "Distributed G_t in QMC Solver" (the slice a
 * rank owns, which the configuration describes). */
int g4_config_init(g4_config *cfg);

/* Validate cfg and report entries per channel and the device bytes that
 * g4_init_slice would allocate.  No HIP call.  Either output may be NULL.
 * Paper: Results section, "Memory Analysis" (the G_t sizes it prints: the full array and its 1/p
 * part per rank, Implementation section, "Distributed G_t in QMC Solver"). */
int g4_slice_size(const g4_config *cfg, uint64_t *entries_per_channel, uint64_t *device_bytes);

/* Create a slice: validate, check device memory (also against the optional
 * cap G4_TEST_DEVICE_MEM_LIMIT, in bytes, from the environment), build and
 * upload the index tables, allocate and zero the accumulators.  Synchronous.
 * On success *out owns all device memory until g4_destroy.
 * Paper: Implementation section, "Distributed G_t in QMC Solver" (each rank
 * allocates an even 1/p part of G_t, a contiguous range of transfer planes
 * here); Background section, the solver workflow (G_t is allocated before the
 * measurements and kept for the whole run). */
int g4_init_slice(const g4_config *cfg, g4_slice **out);

/* Enqueue the accumulation of `batch` measurements.
 * Paper: Background section, "Memory-Bound Issue in DCA++", Eq. (1) (the
 * update of G_t by one G_sigma pair; PH channels by the same Wick rule, see the
 * top of this header); Implementation section, Algorithm 1 ("Pipeline Ring
 * Algorithm": a rank applies its own G_sigma, then each buffer that reaches it
 * from its left neighbour; here the buffers arrive as device pointers).
 * G_up, G_dn: DEVICE pointers to batch consecutive Ng x Ng row-major matrices
 *   of element type cfg.g_in (Ng = lx*ly*(nw+nwex-1)), one per spin.
 *   Borrowed: they must stay alive and unchanged until g4_sync returns (or
 *   until later work on the same stream has run).
 * sign: HOST array of batch weights s_b, copied before return.
 * batch >= 0 (0 is a no-op).  In batched mode the measurements are processed
 * in passes of at most max_batch; in plain mode one pass per measurement.
 * Asynchronous on the handle's stream. */
int g4_accumulate(g4_slice *h, const void *G_up, const void *G_dn, const double *sign,
                  int32_t batch);

/* Wait for all enqueued work on the handle's stream; folds event timings
 * into the statistics.
 * Paper: Implementation section, Algorithm 1 (the wait on the outstanding
 * transfers before a buffer is reused). */
int g4_sync(g4_slice *h);

/* Synchronous copy of entries [first, first+count) of one channel (a single
 * G4_* bit present in cfg.channels) into out_c128 (HOST, 2*count doubles,
 * interleaved).  A compensated accumulator entry is returned as its value in
 * double: the float sum minus the stored compensation term (which holds the
 * negated rounding remainder of the float sum).
 * Paper: Background section, the solver workflow (the accumulated G_t is
 * reduced or written out after the last measurement); Implementation section,
 * "Pipeline Ring Algorithm" (the optional write of each rank's part to a
 * file). */
int g4_readback(g4_slice *h, uint32_t channel, uint64_t first, uint64_t count, double *out_c128);

/* Synchronous overwrite of entries [first, first+count) of one channel from
 * in_c128 (HOST).  For float accumulators each value is split into a rounded
 * value and its rounding remainder (compensated) or rounded (plain float).
 * Paper: Implementation section, "Pipeline Ring Algorithm" (the inverse of the
 * per-rank file write: restoring a slice, e.g. to resume a run). */
int g4_load(g4_slice *h, uint32_t channel, uint64_t first, uint64_t count, const double *in_c128);

/* Add src's accumulators into dst, entry by entry, and its measurement count
 * and weight sum into dst's: the end-of-run reduction of same-index slices
 * that replicas (the paper's sub-rings, Implementation section) accumulate
 * separately.  Both slices must have the same shape, transfer list, plane
 * range and channels (G4_E_ARG otherwise) and live on the same device
 * (G4_E_UNSUPPORTED); their accumulator kinds may differ (each value is read
 * in src's kind and added in dst's; a compensated dst adds the float part and
 * its remainder).  Waits for src's stream, runs on dst's, and returns when
 * done; src is left unchanged.
 * Paper: Implementation section, "Sub-Ring Optimization" (ranks of different sub-rings hold
 * the same part of G_t; those parts are reduced at the end of the run). */
int g4_merge(g4_slice *dst, g4_slice *src);

/* Set the measurement count and weight sum (restoring a checkpoint).
 * Paper: Background section, the solver workflow (G_t is normalised by the
 * measurements taken; with g4_load, a resumed run continues that sum). */
int g4_set_counts(g4_slice *h, uint64_t measurements, double sign_sum);

/* Zero every accumulator and the statistics.  Enqueued.
 * Paper: Background section, the solver workflow (G_t starts from zero before
 * the measurement phase). */
int g4_reset(g4_slice *h);

/* Current statistics (synchronous: waits for the stream first).
 * Paper: Results section (measurement counts and timing of the runs it
 * reports); no interface is given there. */
int g4_stats(g4_slice *h, g4_stats_t *st);

/* Override the work tile (K2 rows; 0 keeps it, or takes the variant's default
 * when the variant changes), the pass size (batched mode, at most the
 * allocated max_batch; 0 keeps it) and the kernel variant (G4_VARIANT_*, -1
 * keeps it).  Selecting G4_VARIANT_PACKED allocates its buffer on first use
 * (G4_E_OOM if it does not fit).  G4_E_UNSUPPORTED if the combination cannot
 * run for this slice.  Waits for the handle's stream.
 * Paper: no passage (the paper gives no kernel design for the G_t update; the
 * plans are this library's own, all computing Eq. (1) and its PH analogues). */
int g4_set_plan(g4_slice *h, int32_t tile, int32_t batch, int32_t variant);

typedef struct g4_tune_result {
    int32_t batch;               /* measurements per pass chosen */
    int32_t tile;                /* K2 rows per work tile chosen */
    int32_t variant;             /* G4_VARIANT_* */
    int32_t candidates;          /* plans timed (0 when a stored choice passed the gate) */
    double ms_per_measurement;   /* pass time per measurement of the chosen plan, as measured here */
    double rel_err_fp64;         /* its largest relative Frobenius difference, over the channels, from
                                    an FP64 evaluation of the same measurements at up to 16384 slice
                                    entries spread over the slice */
} g4_tune_result;

/* Choose the plan (pass size up to min(max_batch, batch), work-tile height,
 * kernel variant) with the shortest pass time per measurement on the first
 * min(batch, max_batch) of `batch` caller-supplied measurements (same layout
 * and ownership as g4_accumulate), among those whose result at up to 16384
 * sampled slice entries differs from an FP64 evaluation of the same
 * measurements (computed on the device straight from G, per entry) by at most
 * tol (relative Frobenius, per channel), and install it.  With
 * G4_AUTOTUNE_CACHE naming a file in the environment, a choice stored there
 * for the same library build, GPU architecture and slice shape is installed
 * after one timed pass passes the same gate (else every plan is timed), and
 * new choices are appended.  G4_E_UNSUPPORTED if no plan meets tol.  Requires
 * a fresh or reset slice (G4_E_STATE otherwise); leaves the accumulators and
 * statistics zeroed.  Synchronous; allocates a few small work buffers.
 * Paper: no passage (as g4_set_plan). */
int g4_autotune(g4_slice *h, const void *G_up, const void *G_dn, const double *sign, int32_t batch,
                double tol, g4_tune_result *out);

/* Allocation-free accumulation, for callers that cannot allocate: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The work of g4_accumulate on a slice described by cfg, into accumulators
 * the caller owns, with no slice handle, no hipMalloc, no
 * hipFree and no allocating library call.  The library's workspace (index
 * tables, work tiles, direct-term vectors, weights) is a static device array
 * of 64 MiB per GPU (the GPU keeps it until the process ends); a
 * configuration whose workspace does not fit is rejected with
 * G4_E_UNSUPPORTED (the message gives the bytes needed: fewer planes or a
 * smaller max_batch fit).
 *   cfg: as for g4_init_slice; cfg->stream is the stream used (NULL: the null
 *     stream), cfg->device the GPU.  Runs the VALU kernels: plain mode, or
 *     batched with G4_PROD_F64 or G4_PROD_F32 (complex64 G for FP32); no
 *     G4_F_* flags (G4_E_UNSUPPORTED otherwise).
 *   acc_mag, acc_chg, acc_pp: DEVICE accumulators of slots 0, 1, 2, one per
 *     channel in cfg->channels (slot 0: magnetic, up-up or PP singlet; 1:
 *     charge, up-down or PP triplet; 2: PP or transverse; NULL for absent
 *     ones), each entries x 16 bytes (G4_ACC_C128,
 *     G4_ACC_C64_KAHAN) or x 8 bytes (G4_ACC_C64), in the library's device
 *     layout [plane][k2][k1][i2][i1] (K = k*nw + i), which g4_readback
 *     translates for a slice; the caller zeroes them before the first call.
 *   G_up, G_dn, sign, batch: as for g4_accumulate.
 * Synchronous: returns when the work on the stream is done.  Every call on a
 * GPU shares its static workspace, which keeps the last call's contents: calls
 * that overlap on one GPU (from two host threads) race; do not make them.
 * Errors as for g4_accumulate; validation happens before any HIP call. */
int g4_accumulate_into(const g4_config *cfg, void *acc_mag, void *acc_chg, void *acc_pp, const void *G_up,
                       const void *G_dn, const double *sign, int32_t batch);

/* ---- G_sigma from expansion configurations -----------------------------
 * For each of `count` measurements b, the walker's single-particle Green's
 * function of one spin on the G window from its expansion configuration:
 *   G_b(K1,K2) = g0(K1) d(K1,K2)
 *              - g0(K1) [sum_ij e^{i th_i(K1)} M_b(i,j) e^{-i th_j(K2)}] g0(K2) / (beta Nc),
 *   th_i(K) = w_n tau_i + k . r_i,  w_n = (2n+1) pi / beta,
 *   g0(K) = 1 / (i w_n + mu + s h - eps_k),  eps_k = -2t(cos kx + cos ky),
 *   s = +1 for spin 0, -1 for spin 1;
 * K = k*(Nw+Nwex-1) + (n + Nw/2) with k = kx_index + lx*ky_index, as for the
 * slice's G input, and the time-ordering conventions folded into M.
 * Computed as E_b M_b E_b^H with E_b(K,i) = e^{i th_i(K)}: phases and g0 in
 * FP64, the two complex products on MFMA in the precision of dtype.
 * Paper: Background section, the solver workflow (the walker's nonuniform
 * Fourier transform of G_sigma, implemented as matrix-matrix products).
 * Arguments (DEVICE pointers unless noted; all arrays row-major, packed):
 *   lx, ly        cluster (Nc = lx*ly <= 4096); nw even in [2, 4096]; nwex in
 *                 [1, 4096]; Ng = Nc*(Nw+Nwex-1) at most 46340;
 *   beta > 0, mu, h, t   model parameters; spin 0 or 1;
 *   n >= 0        vertices per configuration (the same for every b);
 *   count         measurements, 0..65535 (0: nothing is launched);
 *   tau           count x n doubles in [0, beta);
 *   site          count x n int32 cluster sites in [0, Nc), x + lx*y (not
 *                 checked: no memory is indexed by them);
 *   M             count x n x n complex of dtype (G4_IN_C128 or G4_IN_C64);
 *   G             count x Ng x Ng complex of dtype, written whole;
 *   workspace, workspace_bytes   device scratch of at least
 *                 g4_gsigma_workspace() bytes, owned by the caller, not to be
 *                 used by anything else until the stream reaches the end of
 *                 this call; its contents on entry do not matter;
 *   stream        hipStream_t or NULL (the null stream).
 * Asynchronous on stream.  G4_E_ARG for a bad shape, NULL pointers (except
 * tau/site/M when n = 0) or a short workspace; G4_E_UNSUPPORTED beyond the
 * limits above; G4_E_HIP if a launch fails.  No slice handle is involved. */
int g4_gsigma(int32_t lx, int32_t ly, int32_t nw, int32_t nwex, double beta, double mu, double h, double t,
              int32_t spin, int32_t n, int32_t count, const double *tau, const int32_t *site, const void *M,
              int32_t dtype, void *G, void *workspace, uint64_t workspace_bytes, void *stream);

/* Device workspace bytes g4_gsigma needs for these sizes, into *bytes (HOST):
 * Ng complex128 values of g0, then E and E M (count x Ng x n each, dtype);
 * 0 for count = 0.  No HIP call.  G4_E_ARG for a bad shape or dtype, or NULL bytes.
 * Paper: Background section, the solver workflow (the same transform). */
int g4_gsigma_workspace(int32_t lx, int32_t ly, int32_t nw, int32_t nwex, int32_t n, int32_t count,
                        int32_t dtype, uint64_t *bytes);

/* ---- multi-orbital G4 ---------------------------------------------------
 * Accumulate `batch` measurements of the multi-orbital G4 into caller-owned
 * accumulators: every single-particle index carries an orbital label b in
 * [0, nb), so an entry is (Q; K1, b1, b2; K2, b3, b4) and the array holds
 * planes x (N nb^2)^2 entries per channel.  Per measurement:
 *   PH magnetic/charge  s_b [ (Gu-/+Gd)(K1+Q b1, K1 b2) (Gu-/+Gd)(K2 b3, K2+Q b4)
 *                             - sum_s G_s(K2 b3, K1 b2) G_s(K1+Q b1, K2+Q b4) ]
 *   PP up-down          s_b sum_s G_s(Q-K2 b4, Q-K1 b2) G_{-s}(K2 b3, K1 b1)
 * (nb = 1: the single-band channels above).
 * Paper: Background section, "Memory-Bound Issue in DCA++" (Eq. (1), and the
 * multi-orbital case whose G_t grows with the fourth power of the orbital
 * count, which motivates distributing G_t).
 * Arguments: lx, ly, nw, nwex, nq, q_list (HOST, nq distinct momenta, or NULL
 *   for 0..nq-1), q_begin, q_end as in g4_config; nb in [1, 64];
 *   channels: bitmask of G4_PH_MAGNETIC | G4_PH_CHARGE | G4_PP_UPDOWN;
 *   prod: G4_PROD_F64 (G complex128, FP64 products) or G4_PROD_F32 (G
 *   complex64, FP32 products and sums over each launch's measurements);
 *   G_up, G_dn: DEVICE, batch matrices of (Ng nb) x (Ng nb), row-major, row
 *   and column index (k*Nwg + n + nw/2)*nb + b, borrowed until the stream
 *   reaches the end of this call's work;
 *   sign: HOST, batch weights (copied before return);
 *   acc_mag, acc_chg, acc_pp: DEVICE complex128 accumulators, one per channel
 *   in `channels` (NULL for the others), each (q_end-q_begin) x (N nb^2)^2
 *   entries, entry ((p*N + K2)*nb^2 + b3*nb + b4)*(N nb^2) + (K1*nb + b1)*nb
 *   + b2; owned by the caller, who zeroes them;
 *   stream: hipStream_t or NULL.
 * Asynchronous on stream; allocates nothing.  G4_E_ARG for bad shapes,
 * channels, pointers or accumulators not matching `channels`; G4_E_UNSUPPORTED
 * when (Ng nb)^2 >= 2^40 or N nb^2 > 2^30; G4_E_HIP if a launch fails. */
int g4_accumulate_mo(int32_t lx, int32_t ly, int32_t nw, int32_t nwex, int32_t nb, int32_t nq,
                     const int32_t *q_list, int64_t q_begin, int64_t q_end, uint32_t channels, int32_t prod,
                     const void *G_up, const void *G_dn, const double *sign, int32_t batch, void *acc_mag,
                     void *acc_chg, void *acc_pp, void *stream);

/* Release everything owned by h (waits for its stream).  NULL is a no-op.
 * Paper: Background section, the solver workflow (G_t is freed at the end of
 * the run). */
void g4_destroy(g4_slice *h);

/* Environment: G4_LOG=1 prints one line on stderr whenever a slice installs
 * a plan (init, g4_set_plan, g4_autotune); G4_AUTOTUNE_CACHE names the
 * autotuner's cache file; each pass of g4_accumulate is a roctx range
 * ("g4 pass: ...", seen by rocprofv3 --marker-trace) when the roctx library
 * is present, G4_ROCTX=0 turns the ranges off.  For measurements,
 * G4_TILE_ORDER=0..3 sets the order of the work tiles and G4_PLANE_GROUP=1|4|8
 * the transfer planes per tile (defaults: by variant; 8, 4 or 1 by Nwex).
 *
 * Message of the last failing call on this host thread ("" if none).
 * Paper: no passage (error reporting of this interface only). */
const char *g4_last_error(void);

/* ---- synthetic inputs (not part of the method) -------------------------
 * Fill a DEVICE buffer with `count` seeded Hubbard-shaped G matrices for
 * measurements b0..b0+count-1 of one spin (0 up, 1 down):
 *   G(r,c) = delta_rc / (i w_n + mu + s h - eps_k) + noise (x + i y),
 *   eps_k = -2t(cos kx + cos ky),  x, y ~ N(0,1) from Philox4x32-10 with
 *   key (seed, wid) and counter (r*Ng + c, b, spin, 0), Box-Muller in double.
 * dtype: G4_IN_C128 or G4_IN_C64 (rounded).  stream: hipStream_t or NULL
 * (the null stream).  Asynchronous.
 * Paper: Results section (the 6x6 single-band Hubbard runs whose G_sigma these
 * synthetic matrices stand in for; the QMC walker itself is not built). */
int g4_synth_fill(void *out, int32_t dtype, int32_t lx, int32_t ly, int32_t nw, int32_t nwex,
                  double beta, double t, double mu, double h, double noise, uint32_t seed,
                  uint32_t wid, int64_t b0, int32_t count, int32_t spin, void *stream);

/* ---- debug export of the integer index maps (no HIP call) --------------
 * kadd[k*Nc+q] = k+q, ksub[q*Nc+k] = q-k (Nc*Nc int32 each, HOST).
 * plane_q[i], plane_m[i] for the slice's planes i = 0..q_end-q_begin-1.
 * Any output may be NULL.
 * Paper: Background section, "Memory-Bound Issue in DCA++" (the combined
 * momentum-frequency indices K and the transfer K3 of Eq. (1)). */
int g4_index_maps(const g4_config *cfg, int32_t *kadd, int32_t *ksub, int32_t *plane_q,
                  int32_t *plane_m);

#ifdef __cplusplus
}
#endif

#endif /* G4_H */
