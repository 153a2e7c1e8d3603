// Slice-update kernel template for gfx950, included by g4_update_inst.hip,
// which is compiled once per (precision, K2 rows per thread) pair.
//
// Per measurement b (weight s_b) and slice entry (Q, K2, K1):
//   PH magnetic/charge: s_b [ D(K1+Q,K1) D(K2,K2+Q) - sum_s G_s(K2,K1) G_s(K1+Q,K2+Q) ],
//                       D = G_up -/+ G_dn
//   PP (Eq. (1) of the paper, K3 -> Q): s_b sum_s G_s(Q-K2,Q-K1) G_{-s}(K2,K1)
//
// One work tile = (plane group {q, m-range}, k1, k2, K2-frequency rows
// [c0, c0+tile)).  Per measurement the block stages into LDS the G sub-blocks
// holding the exchange operand (rows k1+q, columns k2+q) and the PP operand
// (rows q-k2, columns q-k1), reads G(K2,K1) straight from memory (coalesced
// along K1), takes the direct-term vectors built by the gather kernel, and
// accumulates the pass's measurements in registers; then every slice entry
// is read, updated and written exactly once (no atomics, deterministic).
// Lanes run along K1 frequencies, so each G4 access of a wavefront is one
// contiguous run of nw complex values.
#pragma once

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

template <typename V, typename R>
__device__ __forceinline__ V cscale(V a, R s) {
    V r;
    r.x = a.x * s;
    r.y = a.y * s;
    return r;
}

// ---------------------------------------------------------------------------
// Accumulator read-modify-write of one entry.
template <typename V>
__device__ __forceinline__ void acc_update(void *base, int kind, int64_t e, V v) {
    if (kind == ACC_C128) {
        double2 *p = static_cast<double2 *>(base) + e;
        double2 o = *p;
        o.x += (double)v.x;
        o.y += (double)v.y;
        *p = o;
    } else if (kind == ACC_C64_KAHAN) {
        // {sum.re, sum.im, comp.re, comp.im}; comp holds the negated lost low part
        float4 *p = static_cast<float4 *>(base) + e;
        float4 o = *p;
        float yr = (float)v.x - o.z;
        float tr = o.x + yr;
        o.z = (tr - o.x) - yr;
        o.x = tr;
        float yi = (float)v.y - o.w;
        float ti = o.y + yi;
        o.w = (ti - o.y) - yi;
        o.y = ti;
        *p = o;
    } else {
        float2 *p = static_cast<float2 *>(base) + e;
        float2 o = *p;
        o.x += (float)v.x;
        o.y += (float)v.y;
        *p = o;
    }
}

constexpr int NT = 256;

template <int CH>
struct ChanInfo {
    static constexpr bool mag = (CH & CH_MAG) != 0;
    static constexpr bool chg = (CH & CH_CHG) != 0;
    static constexpr bool pp = (CH & CH_PP) != 0;
    static constexpr bool ph = mag || chg;
    static constexpr int count = (mag ? 1 : 0) + (chg ? 1 : 0) + (pp ? 1 : 0);
    static constexpr int slot_chg = mag ? 1 : 0;
    static constexpr int slot_pp = (mag ? 1 : 0) + (chg ? 1 : 0);
};

// LDS: PH exchange tiles Y_s stored column-major (row index fastest) so that
// lanes (consecutive K1 rows of G) read consecutive words; PP tiles Z_s
// row-major (lanes read descending consecutive columns).
template <typename R, int EPT, int MG, int CH>
__global__ __launch_bounds__(NT) void update_kernel(UpdateArgs a) {
    using V = typename Cx<R>::V;
    using CI = ChanInfo<CH>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V *smem = reinterpret_cast<V *>(smem_raw);

    const int nw = a.d.nw, nwg = a.d.nwg, nc = a.d.nc, n = a.d.n, planes = a.d.planes;
    const int64_t ng = a.d.ng;
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

    const int yr = nw + M - 1, yc = T2 + M - 1;    // exchange tile: rows x cols
    const int zr = T2 + M - 1, zc = nw + M - 1;    // PP tile
    V *Y0 = smem;
    V *Y1 = Y0 + (CI::ph ? yr * yc : 0);
    V *Z0 = Y1 + (CI::ph ? yr * yc : 0);
    V *Z1 = Z0 + (CI::pp ? zr * zc : 0);

    const int64_t rowY = CI::ph ? (int64_t)a.t.kadd[k1 * nc + q] * nwg + m_lo : 0;
    const int64_t colY = CI::ph ? (int64_t)a.t.kadd[k2 * nc + q] * nwg + c0 + m_lo : 0;
    const int64_t rowZ = CI::pp ? (int64_t)a.t.ksub[q * nc + k2] * nwg + m_lo + nw - c0 - T2 : 0;
    const int64_t colZ = CI::pp ? (int64_t)a.t.ksub[q * nc + k1] * nwg + m_lo : 0;
    const int64_t rowX = (int64_t)k2 * nwg + c0;
    const int64_t colX = (int64_t)k1 * nwg + i1;

    V acc[CI::count][EPT][MG];
#pragma unroll
    for (int c = 0; c < CI::count; ++c)
#pragma unroll
        for (int j = 0; j < EPT; ++j)
#pragma unroll
            for (int m = 0; m < MG; ++m) acc[c][j][m] = V{0, 0};

    const V *dA = static_cast<const V *>(a.dir_a);
    const V *dB = static_cast<const V *>(a.dir_b);

    for (int b = 0; b < a.batch; ++b) {
        const V *gu = static_cast<const V *>(a.gu) + (int64_t)b * a.g_stride;
        const V *gd = static_cast<const V *>(a.gd) + (int64_t)b * a.g_stride;
        __syncthreads();
        if (CI::ph) {
            const int cnt = yr * yc;
            for (int e = tid; e < cnt; e += NT) {
                const int r = e / yc, c = e - (e / yc) * yc;
                const int64_t g = (rowY + r) * ng + colY + c;
                Y0[c * yr + r] = gu[g];
                Y1[c * yr + r] = gd[g];
            }
        }
        if (CI::pp) {
            const int cnt = zr * zc;
            for (int e = tid; e < cnt; e += NT) {
                const int r = e / zc, c = e - (e / zc) * zc;
                const int64_t g = (rowZ + r) * ng + colZ + c;
                Z0[r * zc + c] = gu[g];
                Z1[r * zc + c] = gd[g];
            }
        }
        __syncthreads();
        if (!act) continue;
        const R s = (R)a.sign[b];
        V xu[EPT], xd[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int i2l = r0 + j * RP;
            if (i2l < T2) {
                const int64_t g = (rowX + i2l) * ng + colX;
                xu[j] = cscale(gu[g], s);
                xd[j] = cscale(gd[g], s);
            } else {
                xu[j] = V{0, 0};
                xd[j] = V{0, 0};
            }
        }
        const int64_t vbase = (int64_t)b * planes * n;
#pragma unroll
        for (int m = 0; m < MG; ++m) {
            if (m >= M) break;
            const int64_t vrow = vbase + (int64_t)(p0 + m) * n;
            V am{0, 0}, ac{0, 0};
            if (CI::mag) am = dA[vrow + k1 * nw + i1];
            if (CI::chg) ac = dA[(CI::mag ? a.dir_slot_stride : 0) + vrow + k1 * nw + i1];
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const int i2l = r0 + j * RP;
                if (i2l >= T2) break;
                if (CI::ph) {
                    const V yu = Y0[(i2l + m) * yr + i1 + m];
                    const V yd = Y1[(i2l + m) * yr + i1 + m];
                    V ex = cmul(xu[j], yu);
                    cmac(ex, xd[j], yd);
                    const int K2 = k2 * nw + c0 + i2l;
                    if (CI::mag) {
                        const V bm = dB[vrow + K2];
                        cmac(acc[0][j][m], am, bm);
                        acc[0][j][m].x -= ex.x;
                        acc[0][j][m].y -= ex.y;
                    }
                    if (CI::chg) {
                        const V bc = dB[(CI::mag ? a.dir_slot_stride : 0) + vrow + K2];
                        cmac(acc[CI::slot_chg][j][m], ac, bc);
                        acc[CI::slot_chg][j][m].x -= ex.x;
                        acc[CI::slot_chg][j][m].y -= ex.y;
                    }
                }
                if (CI::pp) {
                    const int zi = (m + T2 - 1 - i2l) * zc + m + nw - 1 - i1;
                    cmac(acc[CI::slot_pp][j][m], Z0[zi], xd[j]);
                    cmac(acc[CI::slot_pp][j][m], Z1[zi], xu[j]);
                }
            }
        }
    }
    if (!act) return;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int i2l = r0 + j * RP;
        if (i2l >= T2) break;
#pragma unroll
        for (int m = 0; m < MG; ++m) {
            if (m >= M) break;
            const int64_t e = ((int64_t)(p0 + m) * n + k2 * nw + c0 + i2l) * n + k1 * nw + i1;
            if (CI::mag) acc_update(a.acc[0], a.acc_kind, e, acc[0][j][m]);
            if (CI::chg) acc_update(a.acc[1], a.acc_kind, e, acc[CI::slot_chg][j][m]);
            if (CI::pp) acc_update(a.acc[2], a.acc_kind, e, acc[CI::slot_pp][j][m]);
        }
    }
}

// ---- dispatch of update_kernel instantiations ------------------------------
template <typename R, int EPT, int MG>
hipError_t launch_ch(int channels, int nitems, size_t lds, const UpdateArgs &a, hipStream_t s) {
    const void *fn = nullptr;
    switch (channels) {
#define G4_CASE(CHV)                                                             \
    case CHV:                                                                    \
        fn = reinterpret_cast<const void *>(&update_kernel<R, EPT, MG, CHV>);    \
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

template <typename R, int EPT>
hipError_t launch_mg(int channels, int mgroup, int nitems, size_t lds, const UpdateArgs &a,
                     hipStream_t s) {
    switch (mgroup) {
        case 1: return launch_ch<R, EPT, 1>(channels, nitems, lds, a, s);
        case 4: return launch_ch<R, EPT, 4>(channels, nitems, lds, a, s);
        case 8: return launch_ch<R, EPT, 8>(channels, nitems, lds, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace upd
}  // namespace g4
