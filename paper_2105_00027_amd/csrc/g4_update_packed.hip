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

// Per-thread copy slots of a tile.  Chunk e = k*NTH + tid of the LDS buffer
// [Y | Z | X | A | Bv] comes from byte offset off[k] of a measurement's packed
// block (its G matrix followed by its direct vectors, see pack_gather_kernel);
// chunks past the tile's end take offset 0 and land in the buffer's padding.
// G rows are indexed k*nwg + i, packed columns k*pcb + i.
template <int NTH, int CH, int SLOTS>
__device__ __forceinline__ void packed_offsets(const UpdateArgs &a, const PackedGeom &pg, int tid, int q,
                                               int k1, int k2, int c0, int T2, int M, int m_lo, int p0,
                                               unsigned (&off)[SLOTS]) {
    using CI = ChanInfo<CH>;
    const int nw = a.d.nw, nwg = a.d.nwg, nc = a.d.nc, n = a.d.n;
    const int zc = nw + M - 1;
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
        __syncthreads();   // a previous tile's LDS reads are done (the launch uses one block per tile)
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
        packed_offsets<NTH, CH, SLOTS>(a, pg, tid, q, k1, k2, c0, T2, M, m_lo, p0, off);
        const int bufb = S * NTH * 16;   // bytes per buffer
        const unsigned lds_base = (unsigned)(uintptr_t)(lds_t *)smem_raw;
        const unsigned lds0 = lds_base + wave * 64 * 16;
        auto issue = [&](int b) __attribute__((always_inline)) {
            const char *base = static_cast<const char *>(a.pack) + (int64_t)b * a.pack_stride;
            const unsigned buf = lds0 + (b % NB) * bufb;
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
        float4 xr[EPT], xn[EPT];
        auto load_x = [&](int b, float4 *dst) __attribute__((always_inline)) {
            const float4 *blk = reinterpret_cast<const float4 *>(static_cast<const char *>(a.pack) +
                                                                 (int64_t)b * a.pack_stride);
            static_for<0, EPT>([&](auto j) {
                const int r = min(r0 + j * RP, T2 - 1);
                dst[j] = blk[(int64_t)(rowX + r) * ldp + colX + i1];
            });
        };
        static_for<0, EPT>([&](auto j) { xr[j] = xn[j] = float4{0.f, 0.f, 0.f, 0.f}; });
        // AR: this thread's a(Q, K1) for the group's planes (clamped to the
        // group's last plane, whose values the partial path does not use)
        V ar[AR ? MG : 1], an[AR ? MG : 1];
        auto load_a = [&](int b, V *dst) __attribute__((always_inline)) {
            const V *pa = reinterpret_cast<const V *>(static_cast<const char *>(a.dir_a) +
                                                      (int64_t)b * a.pack_stride) + k1 * nw + i1;
            static_for<0, MG>([&](auto m) { dst[m] = pa[(int64_t)(p0 + min((int)m, M - 1)) * n]; });
        };
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
            if (!XL && act && b + 1 < a.batch) load_x(b + 1, xn);
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
                            static_for<0, CI::nph>([&](auto c) {
                                V &r = acc[c][j][m];
                                V av;
                                if constexpr (AR) av = ar[m];
                                else av = o.a[c];
                                cmac(r, av, o.bb[c][j]);
                                cmac(r, xu[j], yu);
                                cmac(r, xd[j], yd);
                            });
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
            if (!XL) static_for<0, EPT>([&](auto j) { xr[j] = xn[j]; });
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

#if G4_EPT == 4
// Packed operands with the direct term on the matrix cores (nw = 64, 16-row
// tiles, PH channels).  The copies into LDS are those of the two-buffer packed
// kernel (same buffer layout, same slot table, G(K2,K1) read into registers one
// measurement ahead); the thread mapping is the MFMA accumulator layout of
// v_mfma_f32_16x16x4f32: lane l of wave w holds rows 4*(l/16) + t (t < 4) of
// column K1 = 16*w + l%16.  The direct term of plane m is the complex rank-B
// update D(K2, K1) += a_b(Q, K1) b_b(Q, K2); one MFMA pair per measurement and
// plane takes it with K = 4 = {re, im} of the measurement plus two zero slots:
//   A[K2][k] from b: (Re b, -Im b) for Re D, (Re b, Im b) for Im D;
//   B[k][K1] from a: (Re a, Im a) for Re D, (Im a, Re a) for Im D.
// The exchange Hadamard sum is added into the same registers on the VALU.
template <int MG, int CH>
__global__ __launch_bounds__(256, 2) void update_packed_mfma_kernel(UpdateArgs a) {
    using V = float2;
    using CI = ChanInfo<CH>;
    static_assert(CI::ph && !CI::pp, "PH channels only");
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int NTH = 256, NB = 2, TR = 16;     // threads, buffers, tile rows
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l = tid & 63, g4r = l >> 4, c16 = l & 15;
    constexpr int nw = 64;
    const int nwg = a.d.nwg, nc = a.d.nc, n = a.d.n;
    const int i1 = 16 * wave + c16;               // this lane's K1 column
    constexpr int S = (packed_geom(nw, TR, MG, CH, false).nbuf + NTH - 1) / NTH;   // copies per wave
    static_assert(S <= kPackedSlots, "staging slots");
    float *sg = reinterpret_cast<float *>(smem_raw + NB * S * NTH * 16);
    if (tid < a.batch) sg[tid] = (float)a.sign[tid];

    for (int item = blockIdx.x; item < a.nitems; item += gridDim.x) {
        __syncthreads();   // a previous tile's LDS reads are done (the launch uses one block per tile)
        const int4 it = a.t.items[item];
        const int4 gr = a.t.groups[it.x];
        const int q = gr.x, m_lo = gr.y, M = gr.z, p0 = gr.w;
        const int k1 = it.y, k2 = it.z, c0 = it.w;
        const PackedGeom pg = packed_geom(nw, TR, M, CH, false);
        const int ldp = a.ldp;
        const int rowX = k2 * nwg + c0, colX = k1 * a.pcb;
        unsigned off[S];
        packed_offsets<NTH, CH, S>(a, pg, tid, q, k1, k2, c0, TR, M, m_lo, p0, off);
        const int bufb = S * NTH * 16;
        const unsigned lds0 = (unsigned)(uintptr_t)(lds_t *)smem_raw + wave * 64 * 16;
        auto issue = [&](int b) __attribute__((always_inline)) {
            const char *base = static_cast<const char *>(a.pack) + (int64_t)b * a.pack_stride;
            const unsigned buf = lds0 + (b % NB) * bufb;
            static_for<0, S>([&](auto k) {
                dma16(base, off[k], buf + k * NTH * 16);
            });
        };
        f4 re[CI::count][MG], im[CI::count][MG];
        static_for<0, CI::count>([&](auto c) {
            static_for<0, MG>([&](auto m) {
                re[c][m] = f4{0.f, 0.f, 0.f, 0.f};
                im[c][m] = f4{0.f, 0.f, 0.f, 0.f};
            });
        });
        // G(K2,K1) at this lane's four rows, one measurement ahead
        float4 xr[4], xn[4];
        auto load_x = [&](int b, float4 *dst) __attribute__((always_inline)) {
            const float4 *blk = reinterpret_cast<const float4 *>(static_cast<const char *>(a.pack) +
                                                                 (int64_t)b * a.pack_stride);
            static_for<0, 4>([&](auto tt) { dst[tt] = blk[(int64_t)(rowX + 4 * g4r + tt) * ldp + colX + i1]; });
        };
        if (a.batch > 0) {
            issue(0);
            load_x(0, xr);
        }
        for (int b = 0; b < a.batch; ++b) {
            wait_vm(0);
            __syncthreads();                 // b's copies landed everywhere; b-1's buffer is free
            if (b + 1 < a.batch) {
                issue(b + 1);
                load_x(b + 1, xn);
            }
            const float s = sg[b];
            const float4 *Ly = reinterpret_cast<const float4 *>(smem_raw + (b % NB) * bufb);
            const V *At = reinterpret_cast<const V *>(Ly + pg.nG);
            const V *Bt = At + 2 * pg.nA;
            // G(K2,K1) times -s_b (the PH exchange's minus folded in)
            V xu[4], xd[4];
            static_for<0, 4>([&](auto tt) {
                xu[tt] = V{-s * xr[tt].x, -s * xr[tt].y};
                xd[tt] = V{-s * xr[tt].z, -s * xr[tt].w};
            });
            // direct operands: k slot g4r = {re, im} of measurement b for g4r < 2, zero above
            const bool live = g4r < 2, comp = g4r & 1;
            // One plane at a time, software-pipelined: plane m+1's LDS operands are
            // read before plane m's arithmetic (partial groups clamp the reads).
            struct Ops {
                float4 y[4];
                V a[CI::count], b[CI::count];
            };
            auto run = [&](auto FULL) __attribute__((always_inline)) {
                constexpr bool F = decltype(FULL)::value;
                auto load = [&](int m, Ops &o) __attribute__((always_inline)) {
                    const int mm = F ? m : min(m, M - 1);
                    static_for<0, 4>([&](auto tt) { o.y[tt] = Ly[(i1 + mm) * pg.ycs + 4 * g4r + tt + mm]; });
                    static_for<0, CI::count>([&](auto c) {
                        const int sm = c * M + mm;
                        o.b[c] = live ? ld(Bt + sm * TR + c16) : V{0.f, 0.f};
                        o.a[c] = live ? ld(At + sm * nw + i1) : V{0.f, 0.f};
                    });
                };
                auto compute = [&](auto m, const Ops &o) __attribute__((always_inline)) {
                    if (!F && !(m < M)) return;
                    // exchange: sum over spins of G(K2,K1) G(K1+Q,K2+Q), on the VALU
                    static_for<0, 4>([&](auto tt) {
                        V ex = cmul(xu[tt], V{o.y[tt].x, o.y[tt].y});
                        cmac(ex, xd[tt], V{o.y[tt].z, o.y[tt].w});
                        static_for<0, CI::count>([&](auto c) {
                            re[c][m][tt()] += ex.x;
                            im[c][m][tt()] += ex.y;
                        });
                    });
                    // direct: a_b(Q,K1) b_b(Q,K2) on the matrix cores
                    static_for<0, CI::count>([&](auto c) {
                        const V bv = o.b[c], av = o.a[c];
                        const float ar = comp ? -bv.y : bv.x, ai = comp ? bv.y : bv.x;
                        const float br = comp ? av.y : av.x, bi = comp ? av.x : av.y;
                        re[c][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, re[c][m], 0, 0, 0);
                        im[c][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, bi, im[c][m], 0, 0, 0);
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
            if (M == MG) run(std::true_type{});
            else run(std::false_type{});
            static_for<0, 4>([&](auto tt) { xr[tt] = xn[tt]; });
        }
        const int64_t nn = (int64_t)n * n;
        const int64_t ebase = (((int64_t)p0 * nc + k2) * nc + k1) * nw * nw + (int64_t)c0 * nw + i1;
        // one plane at a time, so that the accumulator reads in flight stay few
        static_for<0, MG>([&](auto m) {
            if (m >= M) return;
            static_for<0, 4>([&](auto tt) {
                const int64_t e = ebase + m * nn + (int64_t)(4 * g4r + tt) * nw;
                if (CI::mag) acc_update(a.acc[0], a.acc_kind, e, V{re[0][m][tt()], im[0][m][tt()]});
                if (CI::chg)
                    acc_update(a.acc[1], a.acc_kind, e, V{re[CI::slot_chg][m][tt()], im[CI::slot_chg][m][tt()]});
            });
            __builtin_amdgcn_sched_barrier(0);
        });
    }
}

template <int MG>
hipError_t launch_packed_mfma_ch(int channels, int nitems, size_t lds, const UpdateArgs &a, hipStream_t s) {
    const void *fn = nullptr;
    switch (channels) {
        case 1: fn = reinterpret_cast<const void *>(&update_packed_mfma_kernel<MG, 1>); break;
        case 2: fn = reinterpret_cast<const void *>(&update_packed_mfma_kernel<MG, 2>); break;
        case 3:   // both PH channels: register budget allows plane groups up to 4
            if constexpr (MG <= 4) fn = reinterpret_cast<const void *>(&update_packed_mfma_kernel<MG, 3>);
            else return hipErrorInvalidValue;
            break;
        default: return hipErrorInvalidValue;
    }
    if (hipError_t e = ensure_lds_limit(fn, lds); e != hipSuccess) return e;
    UpdateArgs arg = a;
    arg.nitems = nitems;
    void *params[] = {&arg};
    return hipLaunchKernel(fn, dim3(nitems), dim3(256), params, lds, s);
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
    if (hipError_t e = ensure_lds_limit(fn, lds); e != hipSuccess) return e;
    UpdateArgs arg = a;
    arg.nitems = nitems;
    void *params[] = {&arg};
    return hipLaunchKernel(fn, dim3(nitems), dim3(NTH), params, lds, s);
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

#if G4_EPT == 4
// packed operands, direct term on MFMA: nw = 64, 16-row tiles, PH channels
hipError_t launch_update_packed_mfma(int channels, int mgroup, int nitems, size_t lds, const UpdateArgs &a,
                                     hipStream_t s) {
    if (a.d.nw != 64 || a.tile != 16 || (channels & CH_PP)) return hipErrorInvalidValue;
    switch (mgroup) {
        case 1: return upd::launch_packed_mfma_ch<1>(channels, nitems, lds, a, s);
        case 4: return upd::launch_packed_mfma_ch<4>(channels, nitems, lds, a, s);
        case 8: return upd::launch_packed_mfma_ch<8>(channels, nitems, lds, a, s);
        default: return hipErrorInvalidValue;
    }
}
#endif

}  // namespace g4
