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
// k2+q; column-major so that lanes walking K1 read consecutive words) and the
// PP operand (rows q-k2, columns q-k1; row-major, lanes read a descending
// run), plus the direct-term vector b(Q,K2) of the tile's rows.  G(K2,K1) and
// a(Q,K1) are read straight from memory, coalesced along K1, and reused over
// the tile's planes and rows.  The pass's measurements are summed in
// registers; then every slice entry is read, updated and written exactly once
// (no atomics, deterministic).  In the plain FP64 kind (one measurement per
// pass) the accumulators are loaded before the tile is staged so that the
// HBM reads overlap the staging and the arithmetic.
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

template <int CH>
struct ChanInfo {
    static constexpr bool mag = (CH & CH_MAG) != 0;
    static constexpr bool chg = (CH & CH_CHG) != 0;
    static constexpr bool pp = (CH & CH_PP) != 0;
    static constexpr bool ph = mag || chg;
    static constexpr int count = (mag ? 1 : 0) + (chg ? 1 : 0) + (pp ? 1 : 0);
    static constexpr int nph = (mag ? 1 : 0) + (chg ? 1 : 0);
    static constexpr int slot_chg = mag ? 1 : 0;
    static constexpr int slot_pp = nph;
};

// Kind: 0 plain FP64 (one measurement, c128 accumulator, prefetched);
//       1 batched FP64; 2 batched FP32.
template <int KIND> struct KindInfo;
template <> struct KindInfo<0> { using R = double; static constexpr bool prefetch = true; static constexpr int nsg = 6; };
template <> struct KindInfo<1> { using R = double; static constexpr bool prefetch = false; static constexpr int nsg = 8; };
template <> struct KindInfo<2> { using R = float; static constexpr bool prefetch = false; static constexpr int nsg = 8; };

// Staging slots per thread held in registers across the compute of the
// previous measurement: KindInfo::nsg G-block elements (both spins) and NSV
// direct-vector elements.  Larger tiles copy the rest directly.
constexpr int NSV = 4;

template <int KIND, int EPT, int MG, int CH>
__global__ __launch_bounds__(NT) void update_kernel(UpdateArgs a) {
    using R = typename KindInfo<KIND>::R;
    using V = typename Cx<R>::V;
    using CI = ChanInfo<CH>;
    constexpr bool PF = KindInfo<KIND>::prefetch;
    constexpr int NSG = KindInfo<KIND>::nsg;
    extern __shared__ __align__(16) unsigned char smem_raw[];

    const int nw = a.d.nw, nwg = a.d.nwg, nc = a.d.nc, n = a.d.n, planes = a.d.planes;
    const int ng = a.d.ng;
    const int4 it = a.t.items[blockIdx.x];
    const int4 gr = a.t.groups[it.x];
    const int q = gr.x, m_lo = gr.y, M = gr.z, p0 = gr.w;
    const int k1 = it.y, k2 = it.z, c0 = it.w;
    const int T2 = min(a.tile, nw - c0);
    const int RP = NT / nw;            // K2 rows covered by one pass of the block
    const int tid = threadIdx.x;
    const bool act = tid < RP * nw;
    const int i1 = tid % nw;
    const int r0 = tid / nw;

    // ---- LDS layout: [Y | Z | X] spin pairs, then [A | Bv] direct vectors
    const int yr = nw + M - 1, yc = T2 + M - 1;    // exchange operand block
    const int zr = T2 + M - 1, zc = nw + M - 1;    // PP operand block
    const int nY = CI::ph ? yr * yc : 0;
    const int nZ = CI::pp ? zr * zc : 0;
    const int nX = T2 * nw;                        // G(K2, K1) rows of the tile
    const int nG = nY + nZ + nX;
    const int nA = CI::nph * M * nw;               // a(Q, K1) per PH channel
    const int nB = CI::nph * M * T2;               // b(Q, K2) per PH channel
    const int nV = nA + nB;
    // Spin pairs of the staged G blocks: element i of [Y | Z | X].  FP32 pairs
    // (16 bytes) sit side by side and are read with one 16-byte access; FP64
    // values are kept in two planes so that consecutive lanes stay 16 bytes
    // apart (no bank conflicts).
    constexpr bool SOA = sizeof(V) == 16;
    V *Gp = reinterpret_cast<V *>(smem_raw);
    V *At = Gp + 2 * nG;
    V *Bt = At + nA;
    auto pu = [&](int i) __attribute__((always_inline)) { return SOA ? i : 2 * i; };
    auto pd = [&](int i) __attribute__((always_inline)) { return SOA ? nG + i : 2 * i + 1; };

    const int rowY = CI::ph ? a.t.kadd[k1 * nc + q] * nwg + m_lo : 0;
    const int colY = CI::ph ? a.t.kadd[k2 * nc + q] * nwg + c0 + m_lo : 0;
    const int rowZ = CI::pp ? a.t.ksub[q * nc + k2] * nwg + m_lo + nw - c0 - T2 : 0;
    const int colZ = CI::pp ? a.t.ksub[q * nc + k1] * nwg + m_lo : 0;
    const int rowX = k2 * nwg + c0, colX = k1 * nwg;

    // element e of the staged G blocks -> (offset in G, offset in LDS)
    auto g_slot = [&](int e, int &goff, int &loff) __attribute__((always_inline)) {
        if (e < nY) {            // exchange block, stored column-major
            const int r = e / yc, c = e - r * yc;
            goff = (rowY + r) * ng + colY + c;
            loff = c * yr + r;
        } else if (e < nY + nZ) {   // PP block, row-major
            const int f = e - nY;
            const int r = f / zc, c = f - r * zc;
            goff = (rowZ + r) * ng + colZ + c;
            loff = nY + f;
        } else {                 // G(K2, K1) rows, row-major
            const int f = e - nY - nZ;
            const int r = f / nw, c = f - r * nw;
            goff = (rowX + r) * ng + colX + c;
            loff = nY + nZ + f;
        }
    };
    // element e of the staged direct vectors -> (offset in dir arrays at b = 0, LDS offset)
    auto v_slot = [&](int e, int &goff, int &loff, bool &isb) __attribute__((always_inline)) {
        isb = e >= nA;
        const int f = isb ? e - nA : e;
        const int w = isb ? T2 : nw;
        const int sm = f / w, c = f - sm * w;          // sm = slot * M + m
        const int sl = sm / M, m = sm - sl * M;
        goff = sl * (int)a.dir_slot_stride + (p0 + m) * n + (isb ? k2 * nw + c0 + c : k1 * nw + c);
        loff = f;
    };

    int sg_goff[NSG], sg_loff[NSG];
    static_for<0, NSG>([&](auto k) {
        const int e = tid + k * NT;
        if (e < nG) g_slot(e, sg_goff[k], sg_loff[k]);
        else sg_goff[k] = sg_loff[k] = -1;
    });
    int sv_goff[NSV];
    int sv_loff[NSV];
    bool sv_isb[NSV];
    static_for<0, NSV>([&](auto k) {
        const int e = tid + k * NT;
        if (CI::ph && e < nV) v_slot(e, sv_goff[k], sv_loff[k], sv_isb[k]);
        else { sv_goff[k] = 0; sv_loff[k] = -1; sv_isb[k] = false; }
    });

    const V *dA = static_cast<const V *>(a.dir_a);
    const V *dB = static_cast<const V *>(a.dir_b);
    const int64_t vstride = (int64_t)planes * n;     // direct vectors: per measurement
    V rgu[NSG], rgd[NSG];
    V rv[NSV];
    auto fetch = [&](int b) __attribute__((always_inline)) {
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
    };
    auto store = [&](int b) __attribute__((always_inline)) {
        static_for<0, NSG>([&](auto k) {
            if (sg_loff[k] >= 0) {
                st(Gp + pu(sg_loff[k]), rgu[k]);
                st(Gp + pd(sg_loff[k]), rgd[k]);
            }
        });
        if (CI::ph)
            static_for<0, NSV>([&](auto k) {
                if (sv_loff[k] >= 0) st((sv_isb[k] ? Bt : At) + sv_loff[k], rv[k]);
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
                st((isb ? Bt : At) + lo, ld((isb ? dB : dA) + go + b * vstride));
            }
    };

    // Accumulator layout in device memory, tile-contiguous:
    //   [plane][k2][k1][i2][i1]  (K2 = k2*nw + i2, K1 = k1*nw + i1),
    // so one plane of a tile is a single run of T2*nw entries.  Readback and
    // load translate to the documented [plane][K2][K1] order.
    // Physical index of (plane p0, row c0 + r0, column i1); + m*n*n + j*RP*nw.
    const int64_t ebase = (((int64_t)p0 * nc + k2) * nc + k1) * nw * nw + (int64_t)(c0 + r0) * nw + i1;
    const int64_t nn = (int64_t)n * n;

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
                    }
                });
            });
        }
    }

    const bool full = (T2 == a.tile) && (M == MG);
    if (a.batch > 0) fetch(0);
    for (int b = 0; b < a.batch; ++b) {
        __syncthreads();          // the previous measurement's operands are consumed
        store(b);
        __syncthreads();          // this measurement's operands are in LDS
        if (b + 1 < a.batch) fetch(b + 1);
        if (!act) continue;
        const R s = (R)a.sign[b];
        // G(K2,K1) times -s_b for the PH exchange (its minus folded in), +s_b for PP
        V xu[EPT], xd[EPT];
        static_for<0, EPT>([&](auto j) {
            const int i2l = min(r0 + j * RP, T2 - 1);
            const int ix = nY + nZ + i2l * nw + i1;
            xu[j] = cscale(ld(Gp + pu(ix)), CI::ph ? -s : s);
            xd[j] = cscale(ld(Gp + pd(ix)), CI::ph ? -s : s);
        });
        auto body = [&](auto j, auto m) __attribute__((always_inline)) {
            const int i2l = r0 + j * RP;
            if (CI::ph) {
                const int iy = (i2l + m) * yr + i1 + m;
                const V yu = ld(Gp + pu(iy)), yd = ld(Gp + pd(iy));
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
            if (CI::pp) {
                // the PP term takes +s_b: undo the PH negation when both are present
                const int iz = nY + (m + T2 - 1 - i2l) * zc + m + nw - 1 - i1;
                const V zu = ld(Gp + pu(iz)), zd = ld(Gp + pd(iz));
                if (CI::ph) {
                    V t = cmul(zu, xd[j]);
                    cmac(t, zd, xu[j]);
                    acc[CI::slot_pp][j][m].x -= t.x;
                    acc[CI::slot_pp][j][m].y -= t.y;
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
            } else {
                if (CI::mag) acc_update(a.acc[0], a.acc_kind, e, acc[0][j][m]);
                if (CI::chg) acc_update(a.acc[1], a.acc_kind, e, acc[CI::slot_chg][j][m]);
                if (CI::pp) acc_update(a.acc[2], a.acc_kind, e, acc[CI::slot_pp][j][m]);
            }
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
#undef G4_CASE
        default:
            return hipErrorInvalidValue;
    }
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
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
