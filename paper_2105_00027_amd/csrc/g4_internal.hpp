// Internal declarations shared by the C-ABI host code and the kernel
// launchers of the G4 slice library (not installed, not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <utility>

namespace g4 {

// Shapes of one slice; every count is derived from the configuration.
struct Dims {
    int lx, ly, nc;      // cluster
    int nw, nwex, nwg;   // frequencies: G4 range, transfers, G window
    int ng, n;           // G side, G4 plane side
    int planes;          // planes in the slice
    int64_t q_begin;     // first plane (flattened iQ)
};

// A run of transfer planes sharing one momentum q: bosonic m in
// [m_lo, m_lo + count), slice-relative plane index of m_lo is p0.
// Stored as int4 {q, m_lo, count, p0}.

// One work tile of the slice-update kernel, int4 {group, k1, k2, c0}:
// momenta k1, k2 and K2-frequency rows [c0, c0 + tile) of that group.

// Device-resident index tables of a slice.
struct Tables {
    const int32_t *kadd;   // kadd[k*nc + q] = k + q
    const int32_t *ksub;   // ksub[q*nc + k] = q - k
    const int4 *groups;    // {q, m_lo, count, p0}
    const int4 *items;     // {group, k1, k2, c0}
    const int2 *plane_qm;  // per slice plane {q, m}
    const int32_t *qpos;   // qpos[q] = position of momentum q in the transfer list, or -1
};

enum AccKind { ACC_C128 = 0, ACC_C64_KAHAN = 1, ACC_C64 = 2 };

// Raise a kernel's dynamic-LDS limit once per (kernel, device): launches can
// then be recorded into a HIP graph with no attribute call in between.
inline hipError_t ensure_lds_limit(const void *fn, size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, size_t> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(mu);
    auto it = done.find({fn, dev});
    if (it != done.end() && it->second >= lds) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) done[{fn, dev}] = lds;
    return e;
}
enum { CH_MAG = 1, CH_CHG = 2, CH_PP = 4, CH_UU = 8, CH_UD = 16, CH_TR = 32, CH_PS = 64, CH_PT = 128 };
// Accumulator slot of each channel bit (0 magnetic / up-up / PP singlet,
// 1 charge / up-down / PP triplet, 2 PP / transverse) and the slots a channel
// set occupies.
__host__ __device__ constexpr int acc_slot_of(int ch) {
    return (ch & (CH_MAG | CH_UU | CH_PS)) ? 0 : (ch & (CH_CHG | CH_UD | CH_PT)) ? 1 : 2;
}
__host__ __device__ constexpr int acc_slots(int channels) {
    return (channels | (channels >> 3) | (channels >> 6)) & 7;
}
// Direct-vector recipes (GatherArgs::slots bits), in slot order:
// bit 0 magnetic a = s(Gu-Gd), b = Gu-Gd; bit 1 charge (sums); bit 2 up-up
// a = s Gu, b = Gu; bit 3 up-down a = s Gu, b = Gd.
__host__ __device__ constexpr int direct_recipes(int channels) {
    return (channels & (CH_MAG | CH_CHG)) | ((channels & CH_UU) ? 4 : 0) | ((channels & CH_UD) ? 8 : 0);
}

// Arguments of the slice-update kernel.  G elements are complex of the
// product precision (double2 for FP64, float2 for FP32).
struct UpdateArgs {
    const void *gu;           // batch of Ng x Ng matrices, spin up
    const void *gd;           // spin down
    int64_t g_stride;         // elements between consecutive matrices
    const void *dir_a;        // direct vectors a(slot, b, p, K) (sign folded), slot 0 mag, 1 charge
    const void *dir_b;        // direct vectors b(slot, b, p, K)
    int64_t dir_slot_stride;  // elements between slots
    int64_t dir_b_stride;     // elements between measurements (p, K contiguous: p*n + K)
    const double *sign;       // device, per measurement of this pass
    int batch;                // measurements in this pass
    void *acc[3];             // accumulators: magnetic, charge, pp (NULL if absent)
    int acc_kind;             // AccKind
    int tile;                 // K2 rows per work tile
    const void *pack;         // packed variant: spin-interleaved G of the pass (pack_kernel)
    int64_t pack_stride;      // bytes between consecutive packed matrices
    int ldp;                  // row pitch of a packed matrix, in 16-byte elements
    int pcb;                  // packed column pitch of one momentum block (nwg rounded up to 8)
    int nitems;               // work tiles in the list (one block per tile)
    int skip_direct;          // packed kernel: 1 = the PH direct term is added by
                              // direct_split_kernel; the tile's direct vectors read as zeros
    int persistent;           // packed kernels: 1 = a grid of co-resident blocks walks the tiles
                              // with a grid stride, 0 = one block per tile
    Dims d;
    Tables t;
};

// LDS geometry of one staging buffer of the packed-operand kernel, in 16-byte
// chunks (one chunk = one G element with both spins, or two direct-vector
// values).  Exchange block rows are padded to an odd pitch so that lanes
// walking K1 (one row apart) fall in distinct banks.  The G(K2,K1) rows are
// staged only when x_in_lds (the deep form); the two-buffer form reads them
// into registers.
struct PackedGeom {
    int ycs;        // exchange-block row pitch
    int nY, nZ, nX; // exchange block, PP block, G(K2,K1) rows
    int nG;         // nY + nZ + nX
    int nA, nB;     // direct vectors a (planes x nw) and b (planes x T2), chunks
    int nbuf;       // chunks per buffer
};
__host__ __device__ constexpr PackedGeom packed_geom(int nw, int T2, int M, int channels, bool x_in_lds,
                                                     bool a_in_regs = false) {
    PackedGeom g{};
    const int nph = ((channels & CH_MAG) ? 1 : 0) + ((channels & CH_CHG) ? 1 : 0);
    const int yc = T2 + M - 1;
    g.ycs = yc | 1;
    g.nY = nph ? (nw + M - 1) * g.ycs : 0;
    g.nZ = (channels & CH_PP) ? (T2 + M - 1) * (nw + M - 1) : 0;
    g.nX = x_in_lds ? T2 * nw : 0;
    g.nG = g.nY + g.nZ + g.nX;
    g.nA = a_in_regs ? 0 : nph * M * nw / 2;
    g.nB = nph * M * T2 / 2;
    g.nbuf = g.nG + g.nA + g.nB;
    return g;
}
// Two-buffer packed kernel, one PH channel and no PP, plane groups of 8,
// 128 <= nw <= 256 and at most two K2 rows per thread: the direct vector
// a(Q, K1) (8 x nw complex64, a quarter of the staged chunks at nw = 128) goes
// into registers one measurement ahead instead of LDS, so that three blocks
// fit a CU.  Such a tile stages at most (nw+7) x 9 + 8 chunks: 10 copy slots.
__host__ __device__ constexpr bool packed_a_in_regs(int nw, int tile, int mgroup, int channels, bool deep) {
    return !deep && nw >= 128 && nw <= 256 && mgroup == 8 && tile <= 2 * (256 / nw) && !(channels & CH_PP) &&
           ((channels & CH_MAG) ? 1 : 0) + ((channels & CH_CHG) ? 1 : 0) == 1;
}
constexpr int kPackedSlotsAReg = 10;
// per-thread staging slots of the packed kernel (256 threads, one chunk each)
constexpr int kPackedSlots = 16;
// measurements per pass at most (the packed kernel keeps the pass's weights in LDS)
constexpr int kMaxPassBatch = 256;
// Block shape of the packed kernel: threads and staging buffers (deep: 512
// threads, three buffers, for one or two K2 rows per thread; else 256, two).
inline int packed_threads(bool deep) { return deep ? 512 : 256; }
inline int packed_buffers(bool deep) { return deep ? 3 : 2; }
// Copy instructions per wave and measurement, covering a full tile.
inline int packed_slots(const PackedGeom &g, bool deep) {
    return (g.nbuf + packed_threads(deep) - 1) / packed_threads(deep);
}
// LDS bytes of the packed kernel: the buffers (a whole number of copy rounds
// each) and the pass's weights.
inline size_t packed_lds_bytes(const PackedGeom &g, bool deep) {
    return (size_t)packed_buffers(deep) * packed_slots(g, deep) * packed_threads(deep) * 16 + kMaxPassBatch * 4;
}

// Arguments of the split-precision direct-term GEMM (g4_direct.hip): direct
// vectors in the layout of UpdateArgs, one PH channel per slot.
struct DirectArgs {
    const void *dir_a, *dir_b;   // complex64
    int64_t dir_slot_stride, dir_b_stride;
    int batch;
    int nslots;                  // PH channels present (slot 0 magnetic or charge, slot 1 charge)
    void *acc[2];                // accumulator of each slot's channel
    int acc_kind;
    int p0;                      // first plane of the launch (0: the whole slice)
    Dims d;
};
hipError_t launch_direct_split(int split, const DirectArgs &a, hipStream_t s);

// Arguments of the direct-vector gather.
struct GatherArgs {
    const void *gu, *gd;
    int64_t g_stride;
    void *dir_a, *dir_b;
    int64_t dir_slot_stride;
    int64_t dir_b_stride;
    const double *sign;
    int batch;
    int slots;          // direct_recipes(): bit 0 magnetic (G_up - G_dn), bit 1 charge
                        // (G_up + G_dn), bit 2 up-up (G_up, G_up), bit 3 up-down (G_up, G_dn)
    Dims d;
    Tables t;
};

// Kernel launchers (g4_kernels.hip).  Gather `prec` 0 = FP64, 1 = FP32.
// Update `kind` 0 = plain FP64 (one measurement per pass), 1 = batched FP64,
// 2 = batched FP32.
hipError_t launch_gather(int prec, const GatherArgs &a, hipStream_t s);
// `variant` 0 = VALU kernel, 1 = MFMA direct term (kind 2, tile 16, nw % 64 == 0),
// 2 = packed operands staged straight into LDS (kind 2, even tile).
hipError_t launch_update(int kind, int channels, int ept, int mgroup, int nitems, int variant,
                         const UpdateArgs &a, hipStream_t s);
// LDS bytes of one update block (host arithmetic, also used by the validation)
inline size_t update_lds_bytes(int kind, int channels, int tile, int mgroup, const Dims &d, int variant) {
    if (variant == 2 || variant == 3 || variant == 4) {
        // staging buffers of 16-byte chunks, rotating by measurement
        const bool deep = variant == 3;
        const bool areg = variant == 2 && packed_a_in_regs(d.nw, tile, mgroup, channels, deep);
        return packed_lds_bytes(packed_geom(d.nw, tile < d.nw ? tile : d.nw, mgroup, channels, deep, areg), deep);
    }
    // [exchange block | PP block | G(K2,K1) rows] as spin pairs, then the direct
    // vectors (two copies, by measurement parity, for the MFMA variant)
    const size_t el = kind == 2 ? sizeof(float2) : sizeof(double2);
    const int T2 = tile < d.nw ? tile : d.nw;
    const int nph = __builtin_popcount(direct_recipes(channels));
    const bool ex = (channels & (CH_MAG | CH_CHG | CH_UU | CH_TR)) != 0;
    const bool pair = (channels & (CH_PS | CH_PT)) != 0;
    size_t pairs = (size_t)T2 * d.nw;
    if (ex) pairs += (size_t)(d.nw + mgroup - 1) * (T2 + mgroup - 1);
    if ((channels & CH_PP) || pair) pairs += (size_t)(T2 + mgroup - 1) * (d.nw + mgroup - 1);
    // singlet / triplet: G(Q-K2, K1) and G(K2, Q-K1) blocks
    if (pair) pairs += (size_t)(T2 + mgroup - 1) * d.nw + (size_t)T2 * (d.nw + mgroup - 1);
    const size_t vecs = (size_t)nph * mgroup * (d.nw + T2) * (variant == 1 ? 2 : 1);
    return pairs * 2 * el + vecs * el;
}

// Packed operands with the direct term on MFMA (variant 4): nw = 64, tile 8, plane groups of
// 4 or 8, PH channels.
hipError_t launch_update_packed_mfma(int channels, int mgroup, int nitems, size_t lds, const UpdateArgs &a,
                                     hipStream_t s);
// Packing of one pass for the packed-operand kernel, with the direct vectors
// built on the way: every element (b, r, c) of the pass's complex64 G pairs,
// column c = k*nwg + i, goes to pack[b*pack_stride16 + r*ldp + k*pcb + i] =
// {Re up, Im up, Re dn, Im dn} (16-byte units).  Each momentum block's columns
// start on a 128-byte boundary (pcb = nwg rounded up to 8), so the row runs the
// update kernel copies start on a cache line; the padding columns (i >= nwg and
// [nc*pcb, ldp), ldp >= nc*pcb + 1) hold zeros.  The elements that are
// direct-term operands are also written, combined over the spins, to the direct
// vectors of GatherArgs layout.
struct PackArgs {
    GatherArgs g;            // source G, direct-vector layout, weights, slots, shapes, tables
    void *pack;
    int64_t pack_stride16;   // 16-byte elements between consecutive packed matrices
    int ldp;
    int pcb;                 // column pitch of one momentum block, a multiple of 8 >= nwg
};
hipError_t launch_pack_gather(const PackArgs &a, hipStream_t s);
hipError_t launch_convert_c128_to_c64(const void *src, void *dst, int64_t count, hipStream_t s);
// Readback / load between the documented [plane][K2][K1] order (c128, dst/src)
// and the tile-contiguous device layout of the accumulators.
hipError_t launch_acc_to_c128(int acc_kind, const void *acc, uint64_t first, uint64_t count,
                              double *dst, int nc, int nw, hipStream_t s);
hipError_t launch_c128_to_acc(int acc_kind, const double *src, void *acc, uint64_t first,
                              uint64_t count, int nc, int nw, hipStream_t s);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
// *flag = 1 if any float (dbl = 0) or double (dbl = 1) in [p, p + bytes) is not
// finite; p and bytes aligned to the value size; *flag is not cleared
hipError_t launch_finite_check(const void *p, size_t bytes, int dbl, int *flag, hipStream_t s);
// dst += src over `count` entries of one channel (same geometry; any two accumulator kinds)
hipError_t launch_merge(int dkind, void *dst, int skind, const void *src, uint64_t count, hipStream_t s);

// FP64 evaluation, straight from the G matrices, of sum_b s_b T_ch at listed
// slice entries (documented [plane][K2][K1] order): the reference of the
// autotuner's accuracy gate.  G elements complex128 (g_in 0) or complex64
// (g_in 1, widened); `channel` one CH_* bit.
struct RefArgs {
    const void *gu, *gd;
    int g_in;
    int64_t g_stride;        // elements between consecutive matrices
    const double *sign;      // device, batch weights
    int batch;
    int channel;
    const uint64_t *idx;     // device, count entry indices
    int64_t count;
    double *out;             // device, count complex128 values
    Dims d;
    Tables t;
};
hipError_t launch_ref_entries(const RefArgs &a, hipStream_t s);
// out[j] = accumulator value at documented entry idx[j] (complex128; a
// compensated entry as sum - comp)
hipError_t launch_acc_gather(int acc_kind, const void *acc, const uint64_t *idx, int64_t count, double *out,
                             int nc, int nw, hipStream_t s);

// Synthetic-input generator (g4_synth.hip).
hipError_t launch_synth(void *out, int dtype, int lx, int ly, int nw, int nwex, double beta,
                        double t, double mu, double h, double noise, uint32_t seed, uint32_t wid,
                        int64_t b0, int count, int spin, hipStream_t s);

}  // namespace g4
