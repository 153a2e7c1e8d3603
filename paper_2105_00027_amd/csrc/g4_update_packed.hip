// Slice-update kernels with packed operands (batched FP32), for gfx950.
// Compiled once per G4_EPT (K2 rows per thread), for every channel
// combination and plane-group bound; with G4_EPT = 2 also the copies with the
// direct vector in registers (one PH channel, nw >= 128) and the copy for
// nw = 64 with 8-row tiles, and with G4_EPT = 4 the variant whose direct term
// runs on the matrix cores (update_packed_mfma_kernel).
//
// Same arithmetic, work tiles, thread mapping and accumulator epilogue as the
// batched FP32 VALU kernel in g4_update.hpp; what differs is how a tile's
// operands reach LDS.  Before the pass, pack_gather_kernel rewrites each of
// the pass's G matrix pairs as one block of 16-byte elements
// {Re G_up, Im G_up, Re G_dn, Im G_dn} with a padded row pitch, followed by
// that measurement's direct vectors.  Every operand a tile needs per
// measurement is then a set of contiguous row runs of that block (the
// exchange block, the PP block, the G(K2,K1) rows, the direct vectors), and
// each 16-byte chunk is moved by global_load_lds_dwordx4 straight from memory
// into LDS: no register round trip, no LDS store instructions.  Two LDS
// buffers alternate by measurement parity (three, two measurements ahead, in
// the deep form), so the copies for the next measurement are in flight while
// the current one is computed.
//
// LDS buffer (16-byte chunks, PackedGeom):
//   Y  exchange block G(k1+q rows, k2+q columns), row-major, odd row pitch:
//      lanes walk K1 down a column, one pitch apart, in distinct banks;
//   Z  PP block G(q-k2 rows, q-k1 columns), row-major (lanes read a
//      descending run of one row);
//   X  G(K2, K1) rows of the tile, row-major (lanes read a row): deep form only;
//      the two-buffer form reads them from the packed block into registers,
//      one measurement ahead, which leaves room for three blocks per CU;
//   A  a(Q, K1) per PH channel and plane, Bv b(Q, K2) per channel, plane, row
//      (complex64 pairs).
#include "g4_update.hpp"

#include <algorithm>

#if !defined(G4_EPT)
#error "G4_EPT must be defined"
#endif

namespace g4 {
namespace upd {
namespace {

typedef __attribute__((address_space(3))) unsigned char lds_t;

// global -> LDS, 16 bytes per lane: lane l copies base + off to LDS byte
// address lds + 16*l (base and lds wave-uniform).  Issued as inline assembly so
// that the compiler does not make LDS reads of the other buffer wait for these
// copies; the kernel waits for them itself (s_waitcnt before the barrier that
// publishes the buffer).  M0 carries the LDS address; one wait state separates
// its write from the copy.
__device__ __forceinline__ void dma16(const char *base, unsigned off, unsigned lds) {
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1"
                 :
                 : "v"(off), "s"(base), "s"(lds)
                 : "memory", "m0");
}

// Wait until at most n vector-memory operations of this wave are outstanding.
// n = 0 goes through the builtin so that the compiler knows every load of its
// own (the G(K2,K1) registers) has landed and adds no wait of its own later,
// where one would also wait for copies issued after this point.
__device__ __forceinline__ void wait_vm(int n) {
    if (n == 0) {
        __builtin_amdgcn_s_waitcnt(0);
        return;
    }
    switch (n) {
#define G4_W(k) case k: asm volatile("s_waitcnt vmcnt(" #k ")" ::: "memory"); break;
        G4_W(1) G4_W(2) G4_W(3) G4_W(4) G4_W(5) G4_W(6) G4_W(7) G4_W(8)
        G4_W(9) G4_W(10) G4_W(11) G4_W(12) G4_W(13) G4_W(14) G4_W(15) G4_W(16)
#undef G4_W
        default: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
    }
}

// One block per tile, or (a.persistent) as many blocks as the device holds at
// once, each walking the tile list with a grid stride.  The persistent grid
// is a multiple of 8, so that block i (dispatched to XCD i % 8) still takes
// the tiles the list's order put on that XCD.
hipError_t launch_block_per_tile(const void *fn, int nitems, int nth, size_t lds, const UpdateArgs &a,
                                 hipStream_t s) {
    if (hipError_t e = ensure_lds_limit(fn, lds); e != hipSuccess) return e;
    UpdateArgs arg = a;
    arg.nitems = nitems;
    void *params[] = {&arg};
    int grid = nitems;
    if (a.persistent) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipError_t e = hipGetDevice(&dev); e != hipSuccess) return e;
        if (hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            e != hipSuccess)
            return e;
        if (hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nth, lds); e != hipSuccess)
            return e;
        const int resident = std::max(8, per_cu * cus / 8 * 8);
        grid = std::max(1, std::min(nitems, resident));
    }
    return hipLaunchKernel(fn, dim3(grid), dim3(nth), params, lds, s);
}

// Geometry of a tile's staging buffer, known at run time (GeoRt) or, for
// full tiles of a compile-time-nw kernel copy, at compile time (GeoCt), where
// the divisions of the copy-slot table become multiply-shifts.
struct GeoRt {
    int nw, T2, M, zc;
    PackedGeom g;
};
template <int NW, int T2_, int M_, int CH, bool XL, bool AR>
struct GeoCt {
    static constexpr int nw = NW, T2 = T2_, M = M_, zc = NW + M_ - 1;
    static constexpr PackedGeom g = packed_geom(NW, T2_, M_, CH, XL, AR);
};

// Per-thread copy slots of a tile.  Chunk e = k*NTH + tid of the LDS buffer
// [Y | Z | X | A | Bv] comes from byte offset off[k] of a measurement's packed
// block (its G matrix followed by its direct vectors, see pack_gather_kernel);
// chunks past the tile's end take offset 0 and land in the buffer's padding.
// G rows are indexed k*nwg + i, packed columns k*pcb + i.
template <int NTH, int CH, int SLOTS, class GEO>
__device__ __forceinline__ void packed_offsets(const UpdateArgs &a, const GEO &geo, int tid, int q, int k1,
                                               int k2, int c0, int m_lo, int p0, unsigned (&off)[SLOTS]) {
    using CI = ChanInfo<CH>;
    const auto &pg = geo.g;
    const int nw = geo.nw, T2 = geo.T2, M = geo.M, zc = geo.zc;
    const int nwg = a.d.nwg, nc = a.d.nc, n = a.d.n;
    const int ldp = a.ldp, pcb = a.pcb;
    const int rowY = CI::ph ? a.t.kadd[k1 * nc + q] * nwg + m_lo : 0;
    const int colY = CI::ph ? a.t.kadd[k2 * nc + q] * pcb + c0 + m_lo : 0;
    const int rowZ = CI::pp ? a.t.ksub[q * nc + k2] * nwg + m_lo + nw - c0 - T2 : 0;
    const int colZ = CI::pp ? a.t.ksub[q * nc + k1] * pcb + m_lo : 0;
    const int rowX = k2 * nwg + c0, colX = k1 * pcb;
    const int64_t dslot = a.dir_slot_stride;                 // complex64 values
    const int64_t adelta = static_cast<const char *>(a.dir_a) - static_cast<const char *>(a.pack);
    const int64_t bdelta = static_cast<const char *>(a.dir_b) - static_cast<const char *>(a.pack);
    static_for<0, SLOTS>([&](auto k) {
        const int e = k * NTH + tid;
        int64_t o = 0;
        if (e < pg.nY) {
            const int r = e / pg.ycs, c = e - r * pg.ycs;
            o = ((int64_t)(rowY + r) * ldp + colY + c) * 16;
        } else if (e < pg.nY + pg.nZ) {
            const int f = e - pg.nY;
            const int r = f / zc, c = f - r * zc;
            o = ((int64_t)(rowZ + r) * ldp + colZ + c) * 16;
        } else if (e < pg.nG) {
            const int f = e - pg.nY - pg.nZ;
            const int r = f / nw, c = f - r * nw;
            o = ((int64_t)(rowX + r) * ldp + colX + c) * 16;
        } else if (e < pg.nbuf && a.skip_direct) {
            // direct term added elsewhere: the vectors read as zeros (the last
            // padding element of row 0, which the pack fills with zeros)
            o = (int64_t)(ldp - 1) * 16;
        } else if (e < pg.nG + pg.nA) {
            const int f = e - pg.nG, hw = nw / 2;
            const int sm = f / hw, cc = f - sm * hw;
            const int sl = sm / M, m = sm - sl * M;
            o = adelta + (sl * dslot + (int64_t)(p0 + m) * n + k1 * nw + 2 * cc) * 8;
        } else if (e < pg.nbuf) {
            const int f = e - pg.nG - pg.nA, ht = T2 / 2;
            const int sm = f / ht, cc = f - sm * ht;
            const int sl = sm / M, m = sm - sl * M;
            o = bdelta + (sl * dslot + (int64_t)(p0 + m) * n + k2 * nw + c0 + 2 * cc) * 8;
        }
        off[k] = (unsigned)o;
    });
}

// Copy slots of a PH tile in the full group's buffer layout g (MG planes,
// T2 rows) also when the group has only M < MG planes: rows, columns and
// planes past the group's end repeat its last one, so every copy stays inside
// the group's G window and the kernel reads a full tile's layout; entries of
// the absent planes are computed from those repeats and never stored.
template <int NTH, int CH, int SLOTS>
__device__ __forceinline__ void packed_offsets_full(const UpdateArgs &a, const PackedGeom &g, int tid, int q,
                                                    int k1, int k2, int c0, int T2, int M, int MG, int m_lo,
                                                    int p0, unsigned (&off)[SLOTS]) {
    const int nw = a.d.nw, nwg = a.d.nwg, nc = a.d.nc, n = a.d.n;
    const int ldp = a.ldp, pcb = a.pcb;
    const int rowY = a.t.kadd[k1 * nc + q] * nwg + m_lo;
    const int colY = a.t.kadd[k2 * nc + q] * pcb + c0 + m_lo;
    const int64_t dslot = a.dir_slot_stride;
    const int64_t adelta = static_cast<const char *>(a.dir_a) - static_cast<const char *>(a.pack);
    const int64_t bdelta = static_cast<const char *>(a.dir_b) - static_cast<const char *>(a.pack);
    static_for<0, SLOTS>([&](auto k) {
        const int e = k * NTH + tid;
        int64_t o = 0;
        if (e < g.nY) {
            const int r = min(e / g.ycs, nw + M - 2), c = min(e % g.ycs, T2 + M - 2);
            o = ((int64_t)(rowY + r) * ldp + colY + c) * 16;
        } else if (e < g.nG + g.nA) {
            const int f = e - g.nG, hw = nw / 2;
            const int sm = f / hw, cc = f - sm * hw;
            const int sl = sm / MG, m = min(sm - sl * MG, M - 1);
            o = adelta + (sl * dslot + (int64_t)(p0 + m) * n + k1 * nw + 2 * cc) * 8;
        } else if (e < g.nbuf) {
            const int f = e - g.nG - g.nA, ht = T2 / 2;
            const int sm = f / ht, cc = f - sm * ht;
            const int sl = sm / MG, m = min(sm - sl * MG, M - 1);
            o = bdelta + (sl * dslot + (int64_t)(p0 + m) * n + k2 * nw + c0 + 2 * cc) * 8;
        }
        off[k] = (unsigned)o;
    });
}

// NTH threads per block, NB staging buffers (copies run NB-1 measurements
// ahead).  Every wave issues the same number S of copy instructions per
// measurement (lanes past the tile's chunks copy the block's first chunk into
// the buffer's padding), and loads complete in issue order, so waiting until
// S*(copies issued after measurement b's) are outstanding means b's copies
// have landed.  AR: the direct vector a(Q, K1) is read into registers one
// measurement ahead instead of being staged in LDS (packed_a_in_regs).  NWC:
// nw fixed at compile time (0: taken from the arguments); the tile is then
// EPT * NTH / NWC rows, and a full tile's LDS operand addresses are one
// per-thread base plus constant offsets.
template <int EPT, int MG, int CH, int NTH, int NB, bool AR = false, int NWC = 0>
__global__ __launch_bounds__(NTH, AR ? 3 : 2) void update_packed_kernel(UpdateArgs a) {
    using V = float2;
    using CI = ChanInfo<CH>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nw = NWC ? NWC : a.d.nw, nwg = a.d.nwg, nc = a.d.nc, n = a.d.n;
    const int tile = NWC ? EPT * (NTH / NWC) : a.tile;

    // the pass's weights as floats after the NB buffers (sized for a full
    // tile); the measurement loop then has no memory read of its own that the
    // compiler would wait for (and with it for the copies in flight)
    constexpr bool XL = NB > 2;      // G(K2,K1) rows staged in LDS (deep form) or read into registers
    static_assert(!AR || (CI::nph == 1 && !XL), "a in registers: one PH channel, two-buffer form");
    const PackedGeom pgf = packed_geom(nw, min(tile, nw), MG, CH, XL, AR);   // a full tile
    const int S_full = (pgf.nbuf + NTH - 1) / NTH;
    float *sg = reinterpret_cast<float *>(smem_raw + NB * S_full * NTH * 16);
    if (tid < a.batch) sg[tid] = (float)a.sign[tid];

    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        __syncthreads();   // the previous tile's LDS reads are done (a persistent grid walks several)
        // ---- decode the tile -------------------------------------------------
        const int4 it = a.t.items[item];
        const int4 gr = a.t.groups[it.x];
        const int q = gr.x, m_lo = gr.y, M = gr.z, p0 = gr.w;
        const int k1 = it.y, k2 = it.z, c0 = it.w;
        const int T2 = min(tile, nw - c0);
        const PackedGeom pg = packed_geom(nw, T2, M, CH, XL, AR);

        // ---- per-thread copy slots (S cover a full tile) ------------------------
        const int S = S_full;
        const int ldp = a.ldp;
        const int rowX = k2 * nwg + c0, colX = k1 * a.pcb;
        constexpr int SLOTS = AR ? kPackedSlotsAReg : kPackedSlots;
        unsigned off[SLOTS];
        bool ct = false;
        if constexpr (NWC > 0) {
            if (T2 == tile && M == MG) {
                packed_offsets<NTH, CH, SLOTS>(a, GeoCt<NWC, EPT * (NTH / NWC), MG, CH, XL, AR>{}, tid, q, k1, k2,
                                               c0, m_lo, p0, off);
                ct = true;
            }
        }
        if (!ct) packed_offsets<NTH, CH, SLOTS>(a, GeoRt{nw, T2, M, nw + M - 1, pg}, tid, q, k1, k2, c0, m_lo, p0, off);
        const int bufb = S * NTH * 16;   // bytes per buffer
        const unsigned lds_base = (unsigned)(uintptr_t)(lds_t *)smem_raw;
        const unsigned lds0 = lds_base + wave * 64 * 16;
        auto issue = [&](int j) __attribute__((always_inline)) {
            const char *base = static_cast<const char *>(a.pack) + (int64_t)j * a.pack_stride;
            const unsigned buf = lds0 + (j % NB) * bufb;
            static_for<0, SLOTS>([&](auto k) {
                if (k < S) dma16(base, off[k], buf + k * NTH * 16);
            });
        };

        // ---- accumulation ----------------------------------------------------
        const int RP = NTH / nw;
        const bool act = tid < RP * nw;
        const int i1 = tid % nw;
        const int r0 = tid / nw;
        V acc[CI::count][EPT][MG];
        static_for<0, CI::count>([&](auto c) {
            static_for<0, EPT>([&](auto j) {
                static_for<0, MG>([&](auto m) { acc[c][j][m] = V{0.f, 0.f}; });
            });
        });
        const bool full = (T2 == tile) && (M == MG);
        // two-buffer form: this thread's G(K2,K1) values straight from the packed
        // block into registers, one measurement ahead (the loop waits for every
        // outstanding load before its barrier, so these add no wait)
        float4 xr[EPT];
        // a block base common to the wave plus this lane's fixed byte offsets
        unsigned xoff[EPT];
        static_for<0, EPT>([&](auto j) {
            const int r = min(r0 + j * RP, T2 - 1);
            xoff[j] = (unsigned)(((rowX + r) * ldp + colX + i1) * 16);
        });
        auto load_x = [&](int jb, float4 *dst) __attribute__((always_inline)) {
            const char *blk = static_cast<const char *>(a.pack) + (int64_t)jb * a.pack_stride;
            static_for<0, EPT>([&](auto j) { dst[j] = *reinterpret_cast<const float4 *>(blk + xoff[j]); });
        };
        static_for<0, EPT>([&](auto j) { xr[j] = float4{0.f, 0.f, 0.f, 0.f}; });
        // AR: this thread's a(Q, K1) for the group's planes (clamped to the
        // group's last plane, whose values the partial path does not use)
        V ar[AR ? MG : 1], an[AR ? MG : 1];
        auto load_a = [&](int jb, V *dst) __attribute__((always_inline)) {
            const V *pa = reinterpret_cast<const V *>(static_cast<const char *>(a.dir_a) +
                                                      (int64_t)jb * a.pack_stride) + k1 * nw + i1;
            static_for<0, MG>([&](auto m) { dst[m] = pa[(int64_t)(p0 + min((int)m, M - 1)) * n]; });
        };
        // a full tile's operands: this thread's byte offsets within a buffer;
        // plane and row then add constants (compile-time when nw is), so each
        // measurement costs one address add per operand
        const int zcf = nw + MG - 1;
        const unsigned fy = (unsigned)((i1 * pgf.ycs + r0) * 16);
        const unsigned fz = (unsigned)((pgf.nY + (tile - 1 - r0) * zcf + nw - 1 - i1) * 16);
        const unsigned fa = (unsigned)(pgf.nG * 16 + i1 * 8);
        const unsigned fb = (unsigned)(pgf.nG * 16 + pgf.nA * 16 + r0 * 8);
        for (int b = 0; b < NB - 1 && b < a.batch; ++b) issue(b);
        if (!XL && act && a.batch > 0) load_x(0, xr);
        if constexpr (AR) {
            if (act && a.batch > 0) load_a(0, ar);
        }
        for (int b = 0; b < a.batch; ++b) {
            // copies issued after b's: those of b+1 .. b+NB-2 that exist
            wait_vm(S * (min(b + NB - 2, a.batch - 1) - b));
            __syncthreads();                 // b's copies landed everywhere; b-1's buffer is free
            if (b + NB - 1 < a.batch) issue(b + NB - 1);
            if constexpr (AR) {
                if (act && b + 1 < a.batch) load_a(b + 1, an);
            }
            if (!act) continue;
            const float s = sg[b];
            const float4 *L = reinterpret_cast<const float4 *>(smem_raw + (b % NB) * bufb);
            const float4 *Lx = L + pg.nY + pg.nZ;
            // G(K2,K1) times -s_b for the PH exchange (its minus folded in), +s_b for PP
            V xu[EPT], xd[EPT];
            static_for<0, EPT>([&](auto j) {
                const float4 x = XL ? Lx[min(r0 + j * RP, T2 - 1) * nw + i1] : xr[j];
                const float f = CI::ph ? -s : s;
                xu[j] = V{x.x * f, x.y * f};
                xd[j] = V{x.z * f, x.w * f};
            });
            // xr is consumed: the next measurement's G(K2,K1) goes straight into
            // it (the last step reloads its own, in bounds, so that the load is
            // unconditional and its registers stay the loop's)
            if constexpr (!XL) {
                __builtin_amdgcn_sched_barrier(0);
                load_x(min(b + 1, a.batch - 1), xr);
            }
            // The plane loop is software-pipelined by hand: the LDS operands of
            // plane m+1 are read into registers before the arithmetic of plane m,
            // so the LDS latency is covered by that arithmetic even at two
            // resident blocks per CU.  Partial tiles clamp the reads (in bounds)
            // and skip the arithmetic of absent entries.
            struct Ops {
                float4 y[EPT], z[EPT];
                V a[CI::nph > 0 ? CI::nph : 1], bb[CI::nph > 0 ? CI::nph : 1][EPT];
            };
            auto run = [&](auto FULL) __attribute__((always_inline)) {
                constexpr bool F = decltype(FULL)::value;
                // a full tile's geometry is pgf (compile-time when nw is)
                const PackedGeom &g = F ? pgf : pg;
                const int Mx = F ? MG : M, T2x = F ? tile : T2, zcx = nw + Mx - 1;
                const float4 *Ly = L, *Lz = L + g.nY;
                const V *At = reinterpret_cast<const V *>(L + g.nG);
                const V *Bt = At + 2 * g.nA;
                auto load = [&](int m, Ops &o) __attribute__((always_inline)) {
                    if constexpr (F) {
                        const unsigned char *lb = smem_raw + (b % NB) * bufb;
                        static_for<0, EPT>([&](auto j) {
                            const int rj = NWC ? j * (NTH / (NWC ? NWC : NTH)) : j * RP;
                            if (CI::ph)
                                o.y[j] = *reinterpret_cast<const float4 *>(lb + fy + (m * (g.ycs + 1) + rj) * 16);
                            if (CI::pp)
                                o.z[j] = *reinterpret_cast<const float4 *>(lb + fz + (m * (zcx + 1) - rj * zcx) * 16);
                            static_for<0, CI::nph>([&](auto c) {
                                o.bb[c][j] = ld(reinterpret_cast<const V *>(lb + fb + ((c * MG + m) * tile + rj) * 8));
                            });
                        });
                        if constexpr (!AR)
                            static_for<0, CI::nph>([&](auto c) {
                                o.a[c] = ld(reinterpret_cast<const V *>(lb + fa + (c * MG + m) * nw * 8));
                            });
                        return;
                    }
                    const int mm = F ? m : min(m, M - 1);
                    static_for<0, EPT>([&](auto j) {
                        const int i2l = F ? r0 + j * RP : min(r0 + j * RP, T2 - 1);
                        if (CI::ph) o.y[j] = Ly[(i1 + mm) * g.ycs + i2l + mm];
                        if (CI::pp) o.z[j] = Lz[(mm + T2x - 1 - i2l) * zcx + mm + nw - 1 - i1];
                        static_for<0, CI::nph>([&](auto c) { o.bb[c][j] = ld(Bt + (c * Mx + mm) * T2x + i2l); });
                    });
                    if constexpr (!AR) static_for<0, CI::nph>([&](auto c) { o.a[c] = ld(At + (c * Mx + mm) * nw + i1); });
                };
                auto compute = [&](auto m, const Ops &o) __attribute__((always_inline)) {
                    static_for<0, EPT>([&](auto j) {
                        if (!F && !(m < M && r0 + j * RP < T2)) return;
                        if (CI::ph) {
                            const V yu{o.y[j].x, o.y[j].y}, yd{o.y[j].z, o.y[j].w};
                            if constexpr (CI::nph == 1) {
                                V &r = acc[0][j][m];
                                V av;
                                if constexpr (AR) av = ar[m];
                                else av = o.a[0];
                                cmac(r, av, o.bb[0][j]);
                                cmac(r, xu[j], yu);
                                cmac(r, xd[j], yd);
                            } else {
                                // magnetic and charge share the exchange sum: computed once
                                V ex = cmul(xu[j], yu);
                                cmac(ex, xd[j], yd);
                                static_for<0, CI::nph>([&](auto c) {
                                    V &r = acc[c][j][m];
                                    cmac(r, o.a[c], o.bb[c][j]);
                                    r.x += ex.x;
                                    r.y += ex.y;
                                });
                            }
                        }
                        if (CI::pp) {
                            const V zu{o.z[j].x, o.z[j].y}, zd{o.z[j].z, o.z[j].w};
                            V &r = acc[CI::slot_pp][j][m];
                            if (CI::ph) {
                                // the PP term takes +s_b: undo the PH negation folded into x
                                V w = cmul(zu, xd[j]);
                                cmac(w, zd, xu[j]);
                                r.x -= w.x;
                                r.y -= w.y;
                            } else {
                                cmac(r, zu, xd[j]);
                                cmac(r, zd, xu[j]);
                            }
                        }
                    });
                };
                Ops o[2];
                load(0, o[0]);
                static_for<0, MG>([&](auto m) {
                    if constexpr (m + 1 < MG) load(m + 1, o[(m + 1) & 1]);
                    __builtin_amdgcn_sched_barrier(0);
                    compute(m, o[m & 1]);
                    __builtin_amdgcn_sched_barrier(0);
                });
            };
            if (full && r0 + (EPT - 1) * RP < T2) run(std::true_type{});
            else run(std::false_type{});
            if constexpr (AR) static_for<0, MG>([&](auto m) { ar[m] = an[m]; });
        }
        if (!act) continue;
        const int64_t nn = (int64_t)n * n;
        const int64_t ebase = (((int64_t)p0 * nc + k2) * nc + k1) * nw * nw + (int64_t)(c0 + r0) * nw + i1;
        static_for<0, EPT>([&](auto j) {
            static_for<0, MG>([&](auto m) {
                if (!(r0 + j * RP < T2 && m < M)) return;
                const int64_t e = ebase + m * nn + (int64_t)j * RP * nw;
                if (CI::mag) acc_update(a.acc[0], a.acc_kind, e, acc[0][j][m]);
                if (CI::chg) acc_update(a.acc[1], a.acc_kind, e, acc[CI::slot_chg][j][m]);
                if (CI::pp) acc_update(a.acc[2], a.acc_kind, e, acc[CI::slot_pp][j][m]);
            });
        });

    }
}

#if G4_EPT == 2
// Packed operands with the PH direct term on the matrix cores: nw = 64, 8-row
// tiles, plane groups of MG = 4 or 8, PH channels.  Same copies into LDS as
// the packed kernel (buffer layout, copy-slot table, G(K2,K1) read into
// registers one measurement ahead, three blocks per CU) and the same vector
// mapping for the exchange term: lane l owns K1 column l of the tile, wave w
// K2 rows w and w + 4, every plane.  The vector units only do the exchange
// Hadamard sum, once for both PH channels.  The direct term
// D(K2, K1) += b(Q, K2) a(Q, K1) (sign folded into a) of each channel runs on
// v_mfma_f32_4x4x1_16b_f32: sixteen 4x4 rank-1 updates per instruction, block
// l/4 holding K1 columns 4(l/4)..4(l/4)+3, so that lane l again owns column l,
// here of K2 rows 4(w%2)..4(w%2)+3 (its four result registers) and of planes
// (MG/2)(w/2)..(MG/2)(w/2)+MG/2-1.  A complex update is four real ones:
//   Re D += Re b Re a, Re D += (-Im b) Im a, Im D += Re b Im a, Im D += Im b Re a.
// After the pass's last measurement the matrix-core sums go through LDS (the
// staging buffers are free then) into the exchange layout and each channel's
// accumulator entry is read, updated and written once.
template <int MG, int CH>
__global__ __launch_bounds__(256, CH == 3 ? 2 : 3) void update_packed_mfma_kernel(UpdateArgs a) {
    using V = float2;
    using CI = ChanInfo<CH>;
    static_assert(CI::ph && !CI::pp, "PH channels only");
    static_assert(MG == 4 || MG == 8, "plane groups of 4 or 8");
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int NTH = 256, NB = 2, TR = 8, NW = 64, EPT = 2, RP = 4, PW = MG / 2, NPH = CI::nph;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l = tid & 63;
    const int r0 = wave;                                   // exchange: K2 rows r0, r0 + RP
    const int rg = 4 * (wave & 1), pw0 = PW * (wave >> 1); // direct: K2 rows rg.., planes pw0..
    const int nwg = a.d.nwg, nc = a.d.nc, n = a.d.n;
    constexpr PackedGeom pgf = packed_geom(NW, TR, MG, CH, false);
    constexpr int S = (pgf.nbuf + NTH - 1) / NTH;
    static_assert(S <= kPackedSlots, "staging slots");
    constexpr int bufb = S * NTH * 16;
    static_assert(TR * MG * NW * 8 <= NB * bufb, "the direct sums' transpose fits the staging buffers");
    float *sg = reinterpret_cast<float *>(smem_raw + NB * bufb);
    if (tid < a.batch) sg[tid] = (float)a.sign[tid];
    // this lane's byte offsets within a buffer: exchange block (plane m adds
    // m (ycs + 1) chunks, row j adds RP), a(Q, K1) at column l and b(Q, K2) at
    // row rg + l%4 of plane pw0 (channel c and plane p add (c MG + p) rows)
    const unsigned fy = (unsigned)((l * pgf.ycs + r0) * 16);
    const unsigned fa = (unsigned)(pgf.nG * 16 + (pw0 * NW + l) * 8);
    const unsigned fb = (unsigned)(pgf.nG * 16 + pgf.nA * 16 + (pw0 * TR + rg + (l & 3)) * 8);

    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        __syncthreads();   // the previous tile's LDS reads are done (a persistent grid walks several)
        const int4 it = a.t.items[item];
        const int4 gr = a.t.groups[it.x];
        const int q = gr.x, m_lo = gr.y, M = gr.z, p0 = gr.w;
        const int k1 = it.y, k2 = it.z, c0 = it.w;
        const int ldp = a.ldp;
        const int rowX = k2 * nwg + c0, colX = k1 * a.pcb;
        unsigned off[S];
        packed_offsets_full<NTH, CH, S>(a, pgf, tid, q, k1, k2, c0, TR, M, MG, m_lo, p0, off);
        const unsigned lds0 = (unsigned)(uintptr_t)(lds_t *)smem_raw + wave * 64 * 16;
        auto issue = [&](int j) __attribute__((always_inline)) {
            const char *base = static_cast<const char *>(a.pack) + (int64_t)j * a.pack_stride;
            const unsigned buf = lds0 + (j % NB) * bufb;
            static_for<0, S>([&](auto k) { dma16(base, off[k], buf + k * NTH * 16); });
        };
        V ex[EPT][MG];
        f4 dre[NPH][PW], dim[NPH][PW];
        static_for<0, EPT>([&](auto j) { static_for<0, MG>([&](auto m) { ex[j][m] = V{0.f, 0.f}; }); });
        static_for<0, NPH>([&](auto c) {
            static_for<0, PW>([&](auto p) {
                dre[c][p] = f4{0.f, 0.f, 0.f, 0.f};
                dim[c][p] = f4{0.f, 0.f, 0.f, 0.f};
            });
        });
        // G(K2,K1) at this lane's two rows, one measurement ahead
        float4 xr[EPT];
        unsigned xoff[EPT];
        static_for<0, EPT>([&](auto j) { xoff[j] = (unsigned)(((rowX + r0 + j * RP) * ldp + colX + l) * 16); });
        auto load_x = [&](int jb, float4 *dst) __attribute__((always_inline)) {
            const char *blk = static_cast<const char *>(a.pack) + (int64_t)jb * a.pack_stride;
            static_for<0, EPT>([&](auto j) { dst[j] = *reinterpret_cast<const float4 *>(blk + xoff[j]); });
        };
        static_for<0, EPT>([&](auto j) { xr[j] = float4{0.f, 0.f, 0.f, 0.f}; });
        if (a.batch > 0) {
            issue(0);
            load_x(0, xr);
        }
        for (int b = 0; b < a.batch; ++b) {
            wait_vm(0);
            __syncthreads();                 // b's copies landed everywhere; b-1's buffer is free
            if (b + 1 < a.batch) issue(b + 1);
            const float s = sg[b];
            // G(K2,K1) times -s_b (the PH exchange's minus folded in)
            V xu[EPT], xd[EPT];
            static_for<0, EPT>([&](auto j) {
                xu[j] = V{xr[j].x * -s, xr[j].y * -s};
                xd[j] = V{xr[j].z * -s, xr[j].w * -s};
            });
            // xr is consumed: the next measurement's G(K2,K1) goes straight into
            // it (the last step reloads its own, in bounds)
            __builtin_amdgcn_sched_barrier(0);
            load_x(min(b + 1, a.batch - 1), xr);
            const unsigned char *lb = smem_raw + (b & 1) * bufb;
            struct MOps {
                float ar[NPH], ai[NPH], br[NPH], bi[NPH];
            };
            auto load_m = [&](int p, MOps &o) __attribute__((always_inline)) {
                static_for<0, NPH>([&](auto c) {
                    const V av = ld(reinterpret_cast<const V *>(lb + fa + (c * MG + p) * NW * 8));
                    const V bv = ld(reinterpret_cast<const V *>(lb + fb + (c * MG + p) * TR * 8));
                    o.ar[c] = av.x;
                    o.ai[c] = av.y;
                    o.br[c] = bv.x;
                    o.bi[c] = bv.y;
                });
            };
            auto load_y = [&](int m, float4 (&y)[EPT]) __attribute__((always_inline)) {
                static_for<0, EPT>([&](auto j) {
                    y[j] = *reinterpret_cast<const float4 *>(lb + fy + (m * (pgf.ycs + 1) + j * RP) * 16);
                });
            };
            // plane m+1's exchange operands, and plane group p+1's matrix-core
            // operands, are read before plane m's arithmetic
            float4 y[2][EPT];
            MOps mo[2];
            load_m(0, mo[0]);
            load_y(0, y[0]);
            static_for<0, MG>([&](auto m) {
                constexpr int p = m / 2;
                if constexpr (m + 1 < MG) load_y(m + 1, y[(m + 1) & 1]);
                if constexpr (m % 2 == 0 && p + 1 < PW) load_m(p + 1, mo[(p + 1) & 1]);
                __builtin_amdgcn_sched_barrier(0);
                static_for<0, EPT>([&](auto j) {
                    const float4 &yv = y[m & 1][j];
                    cmac(ex[j][m], xu[j], V{yv.x, yv.y});
                    cmac(ex[j][m], xd[j], V{yv.z, yv.w});
                });
                const MOps &o = mo[p & 1];
                static_for<0, NPH>([&](auto c) {
                    if constexpr (m % 2 == 0) {
                        dre[c][p] = __builtin_amdgcn_mfma_f32_4x4x1f32(o.br[c], o.ar[c], dre[c][p], 0, 0, 0);
                        dim[c][p] = __builtin_amdgcn_mfma_f32_4x4x1f32(o.br[c], o.ai[c], dim[c][p], 0, 0, 0);
                    } else {
                        dre[c][p] = __builtin_amdgcn_mfma_f32_4x4x1f32(-o.bi[c], o.ai[c], dre[c][p], 0, 0, 0);
                        dim[c][p] = __builtin_amdgcn_mfma_f32_4x4x1f32(o.bi[c], o.ar[c], dim[c][p], 0, 0, 0);
                    }
                });
                __builtin_amdgcn_sched_barrier(0);
            });
        }
        // the direct sums into the exchange layout through LDS, one channel at a
        // time: T[K2 row][plane][K1 column]
        const int64_t nn = (int64_t)n * n;
        const int64_t ebase = (((int64_t)p0 * nc + k2) * nc + k1) * NW * NW + (int64_t)(c0 + r0) * NW + l;
        V *T = reinterpret_cast<V *>(smem_raw);
        static_for<0, NPH>([&](auto c) {
            __syncthreads();                 // the buffers (or the previous channel's T) are free
            static_for<0, PW>([&](auto p) {
                static_for<0, 4>([&](auto r) {
                    T[((rg + r) * MG + pw0 + p) * NW + l] = V{dre[c][p][r()], dim[c][p][r()]};
                });
            });
            __syncthreads();
            static_for<0, EPT>([&](auto j) {
                static_for<0, MG>([&](auto m) {
                    if (m < M) {
                        const V d = T[((r0 + j * RP) * MG + m) * NW + l];
                        const int64_t e = ebase + m * nn + (int64_t)j * RP * NW;
                        const V v{ex[j][m].x + d.x, ex[j][m].y + d.y};
                        acc_update(a.acc[(c == 0 && CI::mag) ? 0 : 1], a.acc_kind, e, v);
                    }
                });
            });
        });
    }
}

template <int MG>
hipError_t launch_packed_mfma_ch(int channels, int nitems, size_t lds, const UpdateArgs &a, hipStream_t s) {
    const void *fn = nullptr;
    switch (channels) {
        case 1: fn = reinterpret_cast<const void *>(&update_packed_mfma_kernel<MG, 1>); break;
        case 2: fn = reinterpret_cast<const void *>(&update_packed_mfma_kernel<MG, 2>); break;
        case 3: fn = reinterpret_cast<const void *>(&update_packed_mfma_kernel<MG, 3>); break;
        default: return hipErrorInvalidValue;
    }
    return launch_block_per_tile(fn, nitems, 256, lds, a, s);
}
#endif

template <int MG, int NTH, int NB>
hipError_t launch_packed_ch(int channels, int nitems, size_t lds, const UpdateArgs &a, hipStream_t s,
                            bool areg) {
    const void *fn = nullptr;
#if G4_EPT <= 2
    if constexpr (MG == 8 && NB == 2) {
        if (areg) {
            switch (channels) {
                case 1: fn = reinterpret_cast<const void *>(&update_packed_kernel<G4_EPT, 8, 1, NTH, 2, true>); break;
                case 2: fn = reinterpret_cast<const void *>(&update_packed_kernel<G4_EPT, 8, 2, NTH, 2, true>); break;
                default: return hipErrorInvalidValue;
            }
        }
    }
#endif
#if G4_EPT == 2
    // nw = 64, 8-row tiles, plane groups of 8, PH channels: the compile-time-nw copy
    if constexpr (MG == 8 && NTH == 256 && NB == 2) {
        if (!areg && a.d.nw == 64 && a.tile == 8) {
            switch (channels) {
                case 1: fn = reinterpret_cast<const void *>(&update_packed_kernel<2, 8, 1, 256, 2, false, 64>); break;
                case 2: fn = reinterpret_cast<const void *>(&update_packed_kernel<2, 8, 2, 256, 2, false, 64>); break;
                case 3: fn = reinterpret_cast<const void *>(&update_packed_kernel<2, 8, 3, 256, 2, false, 64>); break;
                default: break;
            }
        }
    }
#endif
    if (areg && !fn) return hipErrorInvalidValue;
    if (!fn) switch (channels) {
#define G4_CASE(CHV)                                                                          \
    case CHV:                                                                                 \
        fn = reinterpret_cast<const void *>(&update_packed_kernel<G4_EPT, MG, CHV, NTH, NB>); \
        break;
        G4_CASE(1) G4_CASE(2) G4_CASE(3) G4_CASE(4) G4_CASE(5) G4_CASE(6) G4_CASE(7)
#undef G4_CASE
        default:
            return hipErrorInvalidValue;
    }
    return launch_block_per_tile(fn, nitems, NTH, lds, a, s);
}

template <int NTH, int NB>
hipError_t launch_packed_mg(int channels, int mgroup, int nitems, size_t lds, const UpdateArgs &a,
                            hipStream_t s, bool areg) {
    switch (mgroup) {
        case 1: return launch_packed_ch<1, NTH, NB>(channels, nitems, lds, a, s, areg);
        case 4: return launch_packed_ch<4, NTH, NB>(channels, nitems, lds, a, s, areg);
        case 8: return launch_packed_ch<8, NTH, NB>(channels, nitems, lds, a, s, areg);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace upd

#define G4_PNAME2(e) launch_update_packed_e##e
#define G4_PNAME(e) G4_PNAME2(e)

// deep = false: 256-thread blocks, two buffers; deep = true: 512-thread
// blocks, three buffers (built for one and two K2 rows per thread)
hipError_t G4_PNAME(G4_EPT)(int channels, int mgroup, int nitems, size_t lds, const UpdateArgs &a,
                            hipStream_t s, bool deep) {
    const bool areg = packed_a_in_regs(a.d.nw, a.tile, mgroup, channels, deep);
    if (!deep) return upd::launch_packed_mg<256, 2>(channels, mgroup, nitems, lds, a, s, areg);
#if G4_EPT <= 2
    return upd::launch_packed_mg<512, 3>(channels, mgroup, nitems, lds, a, s, false);
#else
    return hipErrorInvalidValue;
#endif
}

#if G4_EPT == 2
// packed operands, direct term on MFMA: nw = 64, 8-row tiles, PH channels
hipError_t launch_update_packed_mfma(int channels, int mgroup, int nitems, size_t lds, const UpdateArgs &a,
                                     hipStream_t s) {
    if (a.d.nw != 64 || a.tile != 8 || (channels & CH_PP)) return hipErrorInvalidValue;
    switch (mgroup) {
        case 4: return upd::launch_packed_mfma_ch<4>(channels, nitems, lds, a, s);
        case 8: return upd::launch_packed_mfma_ch<8>(channels, nitems, lds, a, s);
        default: return hipErrorInvalidValue;
    }
}
#endif

}  // namespace g4
