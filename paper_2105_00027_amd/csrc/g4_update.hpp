// Slice-update kernel template for gfx950, included by g4_update_inst.hip,
// which is compiled once per (kind, K2 rows per thread) pair.
//
// Per measurement b (weight s_b) and slice entry (Q, K2, K1):
//   PH magnetic/charge: s_b [ D(K1+Q,K1) D(K2,K2+Q) - sum_s G_s(K2,K1) G_s(K1+Q,K2+Q) ],
//                       D = G_up -/+ G_dn
//   PP (Eq. (1) of the paper, K3 -> Q): s_b sum_s G_s(Q-K2,Q-K1) G_{-s}(K2,K1)
//
// One work tile = (plane group {q, m-range}, k1, k2, K2-frequency rows
// [c0, c0+tile)).  Per measurement the block stages into LDS, both spins side
// by side, the G sub-blocks that hold the exchange operand (rows k1+q, columns
// k2+q; column-major so that lanes walking K1 read consecutive words), the PP
// operand (rows q-k2, columns q-k1; row-major, lanes read a descending run)
// and the tile's G(K2,K1) rows, plus the direct-term vectors a(Q,K1) and
// b(Q,K2); G(K2,K1) is reused from registers over the tile's planes, a over
// its rows.  Loads for the next measurement are held in registers while the
// current one is computed.  The pass's measurements are summed in registers;
// then every slice entry is read, updated and written exactly once (no
// atomics, deterministic).  In the plain FP64 kind (one measurement per pass)
// the accumulators are loaded before the tile is staged so that the HBM reads
// overlap the staging and the arithmetic.  The packed-operand kernel
// (g4_update_packed.hip) and the MFMA kernel below share the arithmetic.
// Lanes run along K1 frequencies, so each G4 access of a wavefront is one
// contiguous run of nw complex values.
#pragma once

#include <type_traits>

#include "g4_internal.hpp"

namespace g4 {
namespace upd {

template <typename R> struct Cx;
template <> struct Cx<double> { using V = double2; };
template <> struct Cx<float> { using V = float2; };


template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// acc += a * b
template <typename V>
__device__ __forceinline__ void cmac(V &acc, V a, V b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}

// Member-wise copies: whole-struct copies of double2 between address spaces
// become memcpy calls that keep register arrays in scratch.
template <typename V>
__device__ __forceinline__ V ld(const V *p) {
    V v;
    v.x = p->x;
    v.y = p->y;
    return v;
}
template <typename V>
__device__ __forceinline__ void st(V *p, V v) {
    p->x = v.x;
    p->y = v.y;
}

template <typename V, typename R>
__device__ __forceinline__ V cscale(V a, R s) {
    V r;
    r.x = a.x * s;
    r.y = a.y * s;
    return r;
}

// Accumulator access.  Every entry is read and written once per pass, so the
// accesses are marked non-temporal: the slice streams through without evicting
// the G blocks that the tiles share from L2 and the MALL.
template <typename T>
__device__ __forceinline__ T nt_ld(const T *p) {
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void nt_st(T *p, T v) {
    __builtin_nontemporal_store(v, p);
}
template <typename V>
__device__ __forceinline__ V acc_ld(const V *p) {
    V v;
    v.x = nt_ld(&p->x);
    v.y = nt_ld(&p->y);
    return v;
}
template <typename V>
__device__ __forceinline__ void acc_st(V *p, V v) {
    nt_st(&p->x, v.x);
    nt_st(&p->y, v.y);
}

// Accumulator read-modify-write of one entry.
template <typename V>
__device__ __forceinline__ void acc_update(void *base, int kind, int64_t e, V v) {
    if (kind == ACC_C128) {
        double2 *p = static_cast<double2 *>(base) + e;
        double2 o = acc_ld(p);
        o.x += (double)v.x;
        o.y += (double)v.y;
        acc_st(p, o);
    } else if (kind == ACC_C64_KAHAN) {
        // {sum.re, sum.im, comp.re, comp.im}; value = sum - comp
        typedef float f4 __attribute__((ext_vector_type(4)));
        f4 *p = reinterpret_cast<f4 *>(static_cast<float4 *>(base) + e);
        f4 o = nt_ld(p);
        float yr = (float)v.x - o.z;
        float tr = o.x + yr;
        o.z = (tr - o.x) - yr;
        o.x = tr;
        float yi = (float)v.y - o.w;
        float ti = o.y + yi;
        o.w = (ti - o.y) - yi;
        o.y = ti;
        nt_st(p, o);
    } else {
        float2 *p = static_cast<float2 *>(base) + e;
        float2 o = acc_ld(p);
        o.x += (float)v.x;
        o.y += (float)v.y;
        acc_st(p, o);
    }
}

// Calls f(integral_constant<int, I>) for I = B..E-1: array indices stay
// compile-time constants without relying on loop unrolling.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

constexpr int NT = 256;   // threads per block
constexpr int SX = 32;    // staging lanes along a G row
constexpr int SY = NT / SX;

// Channel set CH: magnetic / charge / PP, the spin-resolved PH channels
// (longitudinal up-up, up-down, transverse), or the PP singlet / triplet
// projections (the last two families on the VALU kernel only).  Register
// accumulators are numbered in bit order; direct-vector slots likewise over
// the channels with a direct term.
template <int CH>
struct ChanInfo {
    static constexpr bool mag = (CH & CH_MAG) != 0;
    static constexpr bool chg = (CH & CH_CHG) != 0;
    static constexpr bool pp = (CH & CH_PP) != 0;
    static constexpr bool uu = (CH & CH_UU) != 0;
    static constexpr bool ud = (CH & CH_UD) != 0;
    static constexpr bool tr = (CH & CH_TR) != 0;
    static constexpr bool ps = (CH & CH_PS) != 0;
    static constexpr bool pt = (CH & CH_PT) != 0;
    static constexpr bool pair = ps || pt;                  // needs the crossed PP blocks
    static constexpr bool ph = mag || chg || uu || ud || tr;
    static constexpr bool ex = mag || chg || uu || tr;      // needs the exchange block
    static constexpr int count = (mag ? 1 : 0) + (chg ? 1 : 0) + (pp ? 1 : 0) + (uu ? 1 : 0) + (ud ? 1 : 0) +
                                 (tr ? 1 : 0) + (ps ? 1 : 0) + (pt ? 1 : 0);
    static constexpr int nph = (mag ? 1 : 0) + (chg ? 1 : 0) + (uu ? 1 : 0) + (ud ? 1 : 0);
    static constexpr int slot_chg = mag ? 1 : 0;
    static constexpr int slot_pp = (mag ? 1 : 0) + (chg ? 1 : 0);
    static constexpr int slot_ud = uu ? 1 : 0;
    static constexpr int slot_tr = (uu ? 1 : 0) + (ud ? 1 : 0);
    static constexpr int slot_pt = ps ? 1 : 0;
};

// Kind: 0 plain FP64 (one measurement, c128 accumulator, prefetched);
//       1 batched FP64; 2 batched FP32.
template <int KIND> struct KindInfo;
template <> struct KindInfo<0> { using R = double; static constexpr bool prefetch = true; static constexpr int nsg = 6; static constexpr bool pipe = true; static constexpr int waves = 1; };
template <> struct KindInfo<1> { using R = double; static constexpr bool prefetch = false; static constexpr int nsg = 8; static constexpr bool pipe = true; static constexpr int waves = 1; };
template <> struct KindInfo<2> { using R = float; static constexpr bool prefetch = false; static constexpr int nsg = 8; static constexpr bool pipe = true; static constexpr int waves = 1; };

// Staging slots per thread held in registers across the compute of the
// previous measurement: NSG G-block elements (both spins) and NSV
// direct-vector elements.  Larger tiles copy the rest directly.
constexpr int NSV = 4;

// One work tile decoded, with its LDS layout and its operand staging.
//
// LDS: [Y | Z | X] G-block elements for both spins, then the direct vectors
// [A | Bv] (NVB copies, indexed by measurement parity when NVB = 2).
//   Y  exchange block, rows k1+q, columns k2+q, column-major (lanes walking
//      K1 read consecutive words);
//   Z  PP block, rows q-k2, columns q-k1, row-major (descending runs);
//   X  G(K2, K1) rows of the tile, row-major;
//   W  (PP singlet / triplet) G(Q-K2, K1): the PP block's rows, the K1 columns;
//   U  (PP singlet / triplet) G(K2, Q-K1): the tile's rows, the PP block's columns;
//   A  a(Q, K1) per PH channel and plane; Bv b(Q, K2) per channel, plane, row.
// FP32 spin pairs (16 bytes) sit side by side and are read with one 16-byte
// access; FP64 values are kept in two planes so that consecutive lanes stay
// 16 bytes apart (no bank conflicts).
template <typename V, typename CI, int NSG, int NVB>
struct Tile {
    int nw, nwg, nc, n, planes, ng;
    int q, m_lo, M, p0, k1, k2, c0, T2;
    int yr, yc, zr, zc, nY, nZ, nX, nW, nU, nG, nA, nB, nV;
    int rowY, colY, rowZ, colZ, rowX, colX;
    V *Gp, *Vt;
    const V *dA, *dB;
    int64_t vstride;
    int dir_slot;
    int sg_goff[NSG], sg_loff[NSG];
    int sv_goff[NSV], sv_loff[NSV];
    bool sv_isb[NSV];
    V rgu[NSG], rgd[NSG], rv[NSV];
    static constexpr bool SOA = sizeof(V) == 16;

    __device__ __forceinline__ int pu(int i) const { return SOA ? i : 2 * i; }
    __device__ __forceinline__ int pd(int i) const { return SOA ? nG + i : 2 * i + 1; }
    __device__ __forceinline__ V *At(int b) const { return Vt + (NVB == 2 ? (b & 1) * nV : 0); }
    __device__ __forceinline__ V *Bt(int b) const { return At(b) + nA; }

    __device__ __forceinline__ void init(const UpdateArgs &a, int tile, unsigned char *smem, int tid) {
        nw = a.d.nw; nwg = a.d.nwg; nc = a.d.nc; n = a.d.n; planes = a.d.planes; ng = a.d.ng;
        const int4 it = a.t.items[blockIdx.x];
        const int4 gr = a.t.groups[it.x];
        q = gr.x; m_lo = gr.y; M = gr.z; p0 = gr.w;
        k1 = it.y; k2 = it.z; c0 = it.w;
        T2 = min(tile, nw - c0);
        yr = nw + M - 1; yc = T2 + M - 1;
        zr = T2 + M - 1; zc = nw + M - 1;
        nY = CI::ex ? yr * yc : 0;
        nZ = (CI::pp || CI::pair) ? zr * zc : 0;
        nX = T2 * nw;
        nW = CI::pair ? zr * nw : 0;
        nU = CI::pair ? T2 * zc : 0;
        nG = nY + nZ + nX + nW + nU;
        nA = CI::nph * M * nw;
        nB = CI::nph * M * T2;
        nV = nA + nB;
        Gp = reinterpret_cast<V *>(smem);
        Vt = Gp + 2 * nG;
        rowY = CI::ex ? a.t.kadd[k1 * nc + q] * nwg + m_lo : 0;
        colY = CI::ex ? a.t.kadd[k2 * nc + q] * nwg + c0 + m_lo : 0;
        rowZ = (CI::pp || CI::pair) ? a.t.ksub[q * nc + k2] * nwg + m_lo + nw - c0 - T2 : 0;
        colZ = (CI::pp || CI::pair) ? a.t.ksub[q * nc + k1] * nwg + m_lo : 0;
        rowX = k2 * nwg + c0;
        colX = k1 * nwg;
        dA = static_cast<const V *>(a.dir_a);
        dB = static_cast<const V *>(a.dir_b);
        vstride = a.dir_b_stride;
        dir_slot = (int)a.dir_slot_stride;
        static_for<0, NSG>([&](auto k) {
            const int e = tid + k * NT;
            if (e < nG) g_slot(e, sg_goff[k], sg_loff[k]);
            else sg_goff[k] = sg_loff[k] = -1;
        });
        static_for<0, NSV>([&](auto k) {
            const int e = tid + k * NT;
            if (CI::ph && e < nV) v_slot(e, sv_goff[k], sv_loff[k], sv_isb[k]);
            else { sv_goff[k] = 0; sv_loff[k] = -1; sv_isb[k] = false; }
        });
    }
    // element e of the staged G blocks -> (offset in G, offset in LDS)
    __device__ __forceinline__ void g_slot(int e, int &goff, int &loff) const {
        if (e < nY) {
            const int r = e / yc, c = e - r * yc;
            goff = (rowY + r) * ng + colY + c;
            loff = c * yr + r;
        } else if (e < nY + nZ) {
            const int f = e - nY;
            const int r = f / zc, c = f - r * zc;
            goff = (rowZ + r) * ng + colZ + c;
            loff = nY + f;
        } else if (e < nY + nZ + nX) {
            const int f = e - nY - nZ;
            const int r = f / nw, c = f - r * nw;
            goff = (rowX + r) * ng + colX + c;
            loff = nY + nZ + f;
        } else if (e < nY + nZ + nX + nW) {
            const int f = e - nY - nZ - nX;          // W: rows of Q-K2, columns K1
            const int r = f / nw, c = f - r * nw;
            goff = (rowZ + r) * ng + colX + c;
            loff = nY + nZ + nX + f;
        } else {
            const int f = e - nY - nZ - nX - nW;     // U: rows K2, columns of Q-K1
            const int r = f / zc, c = f - r * zc;
            goff = (rowX + r) * ng + colZ + c;
            loff = nY + nZ + nX + nW + f;
        }
    }
    // element e of the staged direct vectors -> (offset at b = 0, LDS offset)
    __device__ __forceinline__ void v_slot(int e, int &goff, int &loff, bool &isb) const {
        isb = e >= nA;
        const int f = isb ? e - nA : e;
        const int w = isb ? T2 : nw;
        const int sm = f / w, c = f - sm * w;          // sm = slot * M + m
        const int sl = sm / M, m = sm - sl * M;
        goff = sl * dir_slot + (p0 + m) * n + (isb ? k2 * nw + c0 + c : k1 * nw + c);
        loff = f;
    }
    __device__ __forceinline__ void fetch(const UpdateArgs &a, int b) {
        const V *gu = static_cast<const V *>(a.gu) + (int64_t)b * a.g_stride;
        const V *gd = static_cast<const V *>(a.gd) + (int64_t)b * a.g_stride;
        static_for<0, NSG>([&](auto k) {
            if (sg_loff[k] >= 0) {
                rgu[k] = ld(gu + sg_goff[k]);
                rgd[k] = ld(gd + sg_goff[k]);
            }
        });
        if (CI::ph)
            static_for<0, NSV>([&](auto k) {
                if (sv_loff[k] >= 0) rv[k] = ld((sv_isb[k] ? dB : dA) + sv_goff[k] + b * vstride);
            });
    }
    __device__ __forceinline__ void store(const UpdateArgs &a, int b, int tid) {
        V *at = At(b);
        static_for<0, NSG>([&](auto k) {
            if (sg_loff[k] >= 0) {
                st(Gp + pu(sg_loff[k]), rgu[k]);
                st(Gp + pd(sg_loff[k]), rgd[k]);
            }
        });
        if (CI::ph)
            static_for<0, NSV>([&](auto k) {
                if (sv_loff[k] >= 0) st(at + (sv_isb[k] ? nA : 0) + sv_loff[k], rv[k]);
            });
        // elements beyond the register slots (large tiles): direct copy
        const V *gu = static_cast<const V *>(a.gu) + (int64_t)b * a.g_stride;
        const V *gd = static_cast<const V *>(a.gd) + (int64_t)b * a.g_stride;
        for (int e = tid + NSG * NT; e < nG; e += NT) {
            int go, lo;
            g_slot(e, go, lo);
            st(Gp + pu(lo), ld(gu + go));
            st(Gp + pd(lo), ld(gd + go));
        }
        if (CI::ph)
            for (int e = tid + NSV * NT; e < nV; e += NT) {
                int go, lo;
                bool isb;
                v_slot(e, go, lo, isb);
                st(at + (isb ? nA : 0) + lo, ld((isb ? dB : dA) + go + b * vstride));
            }
    }
    // operands of entry (row i2l, column i1, plane m) from LDS
    __device__ __forceinline__ void x_at(int i2l, int i1, V &u, V &d) const {
        const int i = nY + nZ + i2l * nw + i1;
        u = ld(Gp + pu(i));
        d = ld(Gp + pd(i));
    }
    __device__ __forceinline__ void y_at(int i2l, int i1, int m, V &u, V &d) const {
        const int i = (i2l + m) * yr + i1 + m;
        u = ld(Gp + pu(i));
        d = ld(Gp + pd(i));
    }
    __device__ __forceinline__ void z_at(int i2l, int i1, int m, V &u, V &d) const {
        const int i = nY + (m + T2 - 1 - i2l) * zc + m + nw - 1 - i1;
        u = ld(Gp + pu(i));
        d = ld(Gp + pd(i));
    }
    __device__ __forceinline__ void w_at(int i2l, int i1, int m, V &u, V &d) const {
        const int i = nY + nZ + nX + (m + T2 - 1 - i2l) * nw + i1;
        u = ld(Gp + pu(i));
        d = ld(Gp + pd(i));
    }
    __device__ __forceinline__ void u_at(int i2l, int i1, int m, V &u, V &d) const {
        const int i = nY + nZ + nX + nW + i2l * zc + m + nw - 1 - i1;
        u = ld(Gp + pu(i));
        d = ld(Gp + pd(i));
    }
    // physical accumulator index (tile-contiguous layout, see update_kernel)
    __device__ __forceinline__ int64_t entry(int m, int i2l, int i1) const {
        return (((int64_t)(p0 + m) * nc + k2) * nc + k1) * nw * nw + (int64_t)(c0 + i2l) * nw + i1;
    }
};

// Accumulator layout in device memory, tile-contiguous:
//   [plane][k2][k1][i2][i1]  (K2 = k2*nw + i2, K1 = k1*nw + i1),
// so one plane of a tile is a single run of T2*nw entries.  Readback and load
// translate to the documented [plane][K2][K1] order.
//
// VALU kernel: thread (r0 = tid / nw, i1 = tid % nw) owns rows
// r0 + j*RP (j < EPT, RP = 256/nw) of column i1 for every plane of the group.
template <int KIND, int EPT, int MG, int CH>
__global__ __launch_bounds__(NT, KindInfo<KIND>::waves) void update_kernel(UpdateArgs a) {
    using R = typename KindInfo<KIND>::R;
    using V = typename Cx<R>::V;
    using CI = ChanInfo<CH>;
    constexpr bool PF = KindInfo<KIND>::prefetch;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x;
    Tile<V, CI, KindInfo<KIND>::nsg, 1> t;
    t.init(a, a.tile, smem_raw, tid);
    const int nw = t.nw, T2 = t.T2, M = t.M;
    const int RP = NT / nw;            // K2 rows covered by one pass of the block
    const bool act = tid < RP * nw;
    const int i1 = tid % nw;
    const int r0 = tid / nw;
    const int64_t nn = (int64_t)t.n * t.n;
    const int64_t ebase = t.entry(0, r0, i1);   // + m*nn + j*RP*nw

    // register accumulators; in the plain kind they start from the slice values,
    // loaded here so that the HBM reads overlap the operand staging
    V acc[CI::count][EPT][MG];
    static_for<0, CI::count>([&](auto c) {
        static_for<0, EPT>([&](auto j) {
            static_for<0, MG>([&](auto m) { acc[c][j][m] = V{0, 0}; });
        });
    });
    if constexpr (PF) {
        if (act) {
            static_for<0, EPT>([&](auto j) {
                static_for<0, MG>([&](auto m) {
                    if (r0 + j * RP < T2 && m < M) {
                        const int64_t e = ebase + m * nn + (int64_t)j * RP * nw;
                        if (CI::mag) acc[0][j][m] = acc_ld(static_cast<const V *>(a.acc[0]) + e);
                        if (CI::chg) acc[CI::slot_chg][j][m] = acc_ld(static_cast<const V *>(a.acc[1]) + e);
                        if (CI::pp) acc[CI::slot_pp][j][m] = acc_ld(static_cast<const V *>(a.acc[2]) + e);
                        if (CI::uu) acc[0][j][m] = acc_ld(static_cast<const V *>(a.acc[0]) + e);
                        if (CI::ud) acc[CI::slot_ud][j][m] = acc_ld(static_cast<const V *>(a.acc[1]) + e);
                        if (CI::tr) acc[CI::slot_tr][j][m] = acc_ld(static_cast<const V *>(a.acc[2]) + e);
                        if (CI::ps) acc[0][j][m] = acc_ld(static_cast<const V *>(a.acc[0]) + e);
                        if (CI::pt) acc[CI::slot_pt][j][m] = acc_ld(static_cast<const V *>(a.acc[1]) + e);
                    }
                });
            });
        }
    }

    const bool full = (T2 == a.tile) && (M == MG);
    // PIPE: the next measurement's operands are loaded into registers while the
    // current one is computed; otherwise each measurement is staged on its own
    // and latency is covered by more resident blocks (fewer live registers).
    constexpr bool PIPE = KindInfo<KIND>::pipe;
    if (PIPE && a.batch > 0) t.fetch(a, 0);
    for (int b = 0; b < a.batch; ++b) {
        __syncthreads();          // the previous measurement's operands are consumed
        if (!PIPE) t.fetch(a, b);
        t.store(a, b, tid);
        __syncthreads();          // this measurement's operands are in LDS
        if (PIPE && b + 1 < a.batch) t.fetch(a, b + 1);
        if (!act) continue;
        const R s = (R)a.sign[b];
        const V *At = t.At(b), *Bt = t.Bt(b);
        // G(K2,K1) times -s_b for the PH exchange (its minus folded in), +s_b for PP
        V xu[EPT], xd[EPT];
        static_for<0, EPT>([&](auto j) {
            V u, d;
            t.x_at(min(r0 + j * RP, T2 - 1), i1, u, d);
            xu[j] = cscale(u, CI::ph ? -s : s);
            xd[j] = cscale(d, CI::ph ? -s : s);
        });
        auto body = [&](auto j, auto m) __attribute__((always_inline)) {
            const int i2l = r0 + j * RP;
            if (CI::pair) {
                // PP singlet / triplet: 1/2 [ s sum_s' G_s'(Q-K2,Q-K1) G_-s'(K2,K1)
                //                           +/- s sum_s' G_s'(Q-K2,K1) G_-s'(K2,Q-K1) ]
                // (xu, xd carry +s_b here)
                V zu, zd, wu, wd, uu_, ud_;
                t.z_at(i2l, i1, m, zu, zd);
                t.w_at(i2l, i1, m, wu, wd);
                t.u_at(i2l, i1, m, uu_, ud_);
                V same = cmul(zu, xd[j]);
                cmac(same, zd, xu[j]);
                V cr = cmul(wu, ud_);
                cmac(cr, wd, uu_);
                const R h = (R)0.5, hs = (R)0.5 * s;
                if (CI::ps) {
                    acc[0][j][m].x += h * same.x + hs * cr.x;
                    acc[0][j][m].y += h * same.y + hs * cr.y;
                }
                if (CI::pt) {
                    acc[CI::slot_pt][j][m].x += h * same.x - hs * cr.x;
                    acc[CI::slot_pt][j][m].y += h * same.y - hs * cr.y;
                }
            } else if (CI::uu || CI::ud || CI::tr) {
                // spin-resolved channels; xu, xd carry -s_b (the exchange sign)
                V yu{0, 0}, yd{0, 0};
                if (CI::ex) t.y_at(i2l, i1, m, yu, yd);
                if (CI::uu) {
                    cmac(acc[0][j][m], ld(At + m * nw + i1), ld(Bt + m * T2 + i2l));
                    cmac(acc[0][j][m], xu[j], yu);
                }
                if (CI::ud) {
                    const int sm = CI::slot_ud * M + m;
                    cmac(acc[CI::slot_ud][j][m], ld(At + sm * nw + i1), ld(Bt + sm * T2 + i2l));
                }
                if (CI::tr) {
                    cmac(acc[CI::slot_tr][j][m], xd[j], yu);
                    cmac(acc[CI::slot_tr][j][m], xu[j], yd);
                }
            } else if (CI::ph) {
                V yu, yd;
                t.y_at(i2l, i1, m, yu, yd);
                if constexpr (CI::mag && CI::chg) {
                    // both PH channels share the exchange sum: computed once
                    V ex = cmul(xu[j], yu);
                    cmac(ex, xd[j], yd);
                    cmac(acc[0][j][m], ld(At + m * nw + i1), ld(Bt + m * T2 + i2l));
                    acc[0][j][m].x += ex.x;
                    acc[0][j][m].y += ex.y;
                    const int sm = CI::slot_chg * M + m;
                    cmac(acc[CI::slot_chg][j][m], ld(At + sm * nw + i1), ld(Bt + sm * T2 + i2l));
                    acc[CI::slot_chg][j][m].x += ex.x;
                    acc[CI::slot_chg][j][m].y += ex.y;
                } else {
                    if (CI::mag) {
                        cmac(acc[0][j][m], ld(At + m * nw + i1), ld(Bt + m * T2 + i2l));
                        cmac(acc[0][j][m], xu[j], yu);
                        cmac(acc[0][j][m], xd[j], yd);
                    }
                    if (CI::chg) {
                        const int sm = CI::slot_chg * M + m;
                        cmac(acc[CI::slot_chg][j][m], ld(At + sm * nw + i1), ld(Bt + sm * T2 + i2l));
                        cmac(acc[CI::slot_chg][j][m], xu[j], yu);
                        cmac(acc[CI::slot_chg][j][m], xd[j], yd);
                    }
                }
            }
            if (CI::pp) {
                // the PP term takes +s_b: undo the PH negation when both are present
                V zu, zd;
                t.z_at(i2l, i1, m, zu, zd);
                if (CI::ph) {
                    V w = cmul(zu, xd[j]);
                    cmac(w, zd, xu[j]);
                    acc[CI::slot_pp][j][m].x -= w.x;
                    acc[CI::slot_pp][j][m].y -= w.y;
                } else {
                    cmac(acc[CI::slot_pp][j][m], zu, xd[j]);
                    cmac(acc[CI::slot_pp][j][m], zd, xu[j]);
                }
            }
        };
        if (full && r0 + (EPT - 1) * RP < T2) {
            static_for<0, MG>([&](auto m) { static_for<0, EPT>([&](auto j) { body(j, m); }); });
        } else {
            static_for<0, MG>([&](auto m) {
                static_for<0, EPT>([&](auto j) {
                    if (m < M && r0 + j * RP < T2) body(j, m);
                });
            });
        }
    }
    if (!act) return;
    static_for<0, EPT>([&](auto j) {
        static_for<0, MG>([&](auto m) {
            if (!(r0 + j * RP < T2 && m < M)) return;
            const int64_t e = ebase + m * nn + (int64_t)j * RP * nw;
            if constexpr (PF) {
                if (CI::mag) acc_st(static_cast<V *>(a.acc[0]) + e, acc[0][j][m]);
                if (CI::chg) acc_st(static_cast<V *>(a.acc[1]) + e, acc[CI::slot_chg][j][m]);
                if (CI::pp) acc_st(static_cast<V *>(a.acc[2]) + e, acc[CI::slot_pp][j][m]);
                if (CI::uu) acc_st(static_cast<V *>(a.acc[0]) + e, acc[0][j][m]);
                if (CI::ud) acc_st(static_cast<V *>(a.acc[1]) + e, acc[CI::slot_ud][j][m]);
                if (CI::tr) acc_st(static_cast<V *>(a.acc[2]) + e, acc[CI::slot_tr][j][m]);
                if (CI::ps) acc_st(static_cast<V *>(a.acc[0]) + e, acc[0][j][m]);
                if (CI::pt) acc_st(static_cast<V *>(a.acc[1]) + e, acc[CI::slot_pt][j][m]);
            } else {
                if (CI::mag) acc_update(a.acc[0], a.acc_kind, e, acc[0][j][m]);
                if (CI::chg) acc_update(a.acc[1], a.acc_kind, e, acc[CI::slot_chg][j][m]);
                if (CI::pp) acc_update(a.acc[2], a.acc_kind, e, acc[CI::slot_pp][j][m]);
                if (CI::uu) acc_update(a.acc[0], a.acc_kind, e, acc[0][j][m]);
                if (CI::ud) acc_update(a.acc[1], a.acc_kind, e, acc[CI::slot_ud][j][m]);
                if (CI::tr) acc_update(a.acc[2], a.acc_kind, e, acc[CI::slot_tr][j][m]);
                if (CI::ps) acc_update(a.acc[0], a.acc_kind, e, acc[0][j][m]);
                if (CI::pt) acc_update(a.acc[1], a.acc_kind, e, acc[CI::slot_pt][j][m]);
            }
        });
    });
}

// MFMA kernel (batched FP32, nw a multiple of 64, tile of 16 K2 rows): the
// direct term of each plane is a complex rank-B update, summed on the matrix
// cores with v_mfma_f32_16x16x4f32 (K = 4: two measurements x {re, im}):
//   Re D += sum_b [ Re b(K2) Re a(K1) - Im b(K2) Im a(K1) ]
//   Im D += sum_b [ Re b(K2) Im a(K1) + Im b(K2) Re a(K1) ]
// with A[row = K2][k] built from b and B[k][col = K1] from a.  Lane l of wave w
// holds rows 4*(l/16) + t (t < 4) of column 16*w + 64*s + l%16 (slab s), the
// MFMA accumulator layout; the exchange and PP Hadamard sums are added into
// the same registers on the VALU.  The direct vectors of two consecutive
// measurements are kept in LDS (indexed by parity) for the paired MFMA.
template <int SL, int MG, int CH>
__global__ __launch_bounds__(NT) void update_mfma_kernel(UpdateArgs a) {
    using V = float2;
    using CI = ChanInfo<CH>;
    typedef float f4 __attribute__((ext_vector_type(4)));
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x;
    Tile<V, CI, 8, 2> t;
    t.init(a, 16, smem_raw, tid);
    const int nw = t.nw, T2 = t.T2, M = t.M;
    const int w = tid / 64, l = tid % 64;
    const int g4r = l / 16, c16 = l % 16;
    const int64_t nn = (int64_t)t.n * t.n;

    f4 re[CI::count][SL][MG], im[CI::count][SL][MG];
    static_for<0, CI::count>([&](auto c) {
        static_for<0, SL>([&](auto s) {
            static_for<0, MG>([&](auto m) {
                re[c][s][m] = f4{0.f, 0.f, 0.f, 0.f};
                im[c][s][m] = f4{0.f, 0.f, 0.f, 0.f};
            });
        });
    });

    if (a.batch > 0) t.fetch(a, 0);
    for (int b = 0; b < a.batch; ++b) {
        __syncthreads();
        t.store(a, b, tid);
        __syncthreads();
        if (b + 1 < a.batch) t.fetch(a, b + 1);
        const float sg = (float)a.sign[b];
        // exchange / PP Hadamard terms on the VALU
        static_for<0, SL>([&](auto s) {
            const int i1 = 64 * s + 16 * w + c16;
            static_for<0, 4>([&](auto tt) {
                const int i2l = 4 * g4r + tt;
                if (i2l >= T2) return;
                V xu, xd;
                t.x_at(i2l, i1, xu, xd);
                xu = cscale(xu, CI::ph ? -sg : sg);
                xd = cscale(xd, CI::ph ? -sg : sg);
                static_for<0, MG>([&](auto m) {
                    if (m >= M) return;
                    if (CI::ph) {
                        V yu, yd;
                        t.y_at(i2l, i1, m, yu, yd);
                        V ex = cmul(xu, yu);
                        cmac(ex, xd, yd);
                        if (CI::mag) {
                            re[0][s][m][tt()] += ex.x;
                            im[0][s][m][tt()] += ex.y;
                        }
                        if (CI::chg) {
                            re[CI::slot_chg][s][m][tt()] += ex.x;
                            im[CI::slot_chg][s][m][tt()] += ex.y;
                        }
                    }
                    if (CI::pp) {
                        V zu, zd;
                        t.z_at(i2l, i1, m, zu, zd);
                        V w2 = cmul(zu, xd);
                        cmac(w2, zd, xu);
                        const float sgn = CI::ph ? -1.f : 1.f;
                        re[CI::slot_pp][s][m][tt()] += sgn * w2.x;
                        im[CI::slot_pp][s][m][tt()] += sgn * w2.y;
                    }
                });
            });
        });
        // direct term: one MFMA pair per two measurements
        if (CI::ph && ((b & 1) || b + 1 == a.batch)) {
            const int b0 = b & ~1;
            const int bk = b0 + (g4r >> 1);        // measurement of this lane's k slot
            const bool comp = g4r & 1;
            const bool live = bk <= b;             // an unpaired last measurement pads with 0
            const V *At = t.At(bk), *Bt = t.Bt(bk);
            static_for<0, CI::nph>([&](auto c) {
                static_for<0, MG>([&](auto m) {
                    if (m >= M) return;
                    const int sm = c * M + m;
                    V bv = live && c16 < T2 ? ld(Bt + sm * T2 + c16) : V{0.f, 0.f};
                    const float ar = comp ? -bv.y : bv.x;
                    const float ai = comp ? bv.y : bv.x;
                    static_for<0, SL>([&](auto s) {
                        const int i1 = 64 * s + 16 * w + c16;
                        V av = live ? ld(At + sm * nw + i1) : V{0.f, 0.f};
                        const float br = comp ? av.y : av.x;
                        const float bi = comp ? av.x : av.y;
                        re[c][s][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, re[c][s][m], 0, 0, 0);
                        im[c][s][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, bi, im[c][s][m], 0, 0, 0);
                    });
                });
            });
        }
    }
    static_for<0, SL>([&](auto s) {
        const int i1 = 64 * s + 16 * w + c16;
        static_for<0, 4>([&](auto tt) {
            const int i2l = 4 * g4r + tt;
            if (i2l >= T2) return;
            static_for<0, MG>([&](auto m) {
                if (m >= M) return;
                const int64_t e = t.entry(m, i2l, i1);
                static_for<0, CI::count>([&](auto c) {
                    const int ch = c == 0 ? (CI::mag ? 0 : (CI::chg ? 1 : 2)) : (c == 1 ? (CI::mag && CI::chg ? 1 : 2) : 2);
                    acc_update(a.acc[ch], a.acc_kind, e, V{re[c][s][m][tt()], im[c][s][m][tt()]});
                });
            });
        });
    });
}

// ---- dispatch over the compile-time parameters -----------------------------
template <int KIND, int EPT, int MG>
hipError_t launch_ch(int channels, int nitems, size_t lds, const UpdateArgs &a, hipStream_t s) {
    const void *fn = nullptr;
    switch (channels) {
#define G4_CASE(CHV)                                                                 \
    case CHV:                                                                        \
        fn = reinterpret_cast<const void *>(&update_kernel<KIND, EPT, MG, CHV>);     \
        break;
        G4_CASE(1) G4_CASE(2) G4_CASE(3) G4_CASE(4) G4_CASE(5) G4_CASE(6) G4_CASE(7)
        G4_CASE(8) G4_CASE(16) G4_CASE(24) G4_CASE(32) G4_CASE(40) G4_CASE(48) G4_CASE(56)
        G4_CASE(64) G4_CASE(128) G4_CASE(192)
#undef G4_CASE
        default:
            return hipErrorInvalidValue;
    }
    if (hipError_t e = ensure_lds_limit(fn, lds); e != hipSuccess) return e;
    UpdateArgs arg = a;
    void *params[] = {&arg};
    return hipLaunchKernel(fn, dim3(nitems), dim3(NT), params, lds, s);
}

template <int KIND, int EPT>
hipError_t launch_mg(int channels, int mgroup, int nitems, size_t lds, const UpdateArgs &a,
                     hipStream_t s) {
    switch (mgroup) {
        case 1: return launch_ch<KIND, EPT, 1>(channels, nitems, lds, a, s);
        case 4: return launch_ch<KIND, EPT, 4>(channels, nitems, lds, a, s);
        case 8: return launch_ch<KIND, EPT, 8>(channels, nitems, lds, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace upd
}  // namespace g4
