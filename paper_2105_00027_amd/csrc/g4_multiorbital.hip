// Multi-orbital G4 accumulation for gfx950: every single-particle index
// carries an orbital label, so a G4 entry is (Q; K1, b1, b2; K2, b3, b4) and
// the array grows as nb^4 (the paper's motivating case for distributing G_t:
// Background section, "Memory-Bound Issue in DCA++").
//
// Per measurement b with weight s_b:
//   PH magnetic/charge  s_b [ (Gu -/+ Gd)(K1+Q b1, K1 b2) (Gu -/+ Gd)(K2 b3, K2+Q b4)
//                             - sum_s G_s(K2 b3, K1 b2) G_s(K1+Q b1, K2+Q b4) ]
//   PP up-down          s_b sum_s G_s(Q-K2 b4, Q-K1 b2) G_{-s}(K2 b3, K1 b1)
// G_sigma is (Ng nb) x (Ng nb), index (k*Nwg + n + Nw/2)*nb + b.  The slice is
// stored as documented: entry ((p*N + K2)*nb^2 + b3*nb + b4)*(N nb^2) +
// (K1*nb + b1)*nb + b2, complex128.
//
// A launch covers up to 32 measurements of one channel over up to 256 planes
// and keeps the sums over the measurements in registers, then reads, adds and
// writes each entry once.  For nb <= 8 (mo_rows_kernel) a thread owns one
// column (K1, b1, b2) of one (plane, K2) and all nb^2 rows (b3, b4): per
// measurement it loads the column's a = G(K1+Q b1, K1 b2) once and the nb
// exchange operands of each side (G(K2 b3, K1 b2) and G(K1+Q b1, K2+Q b4):
// one per b3, one per b4), both spins: 2 + 4 nb vector loads for nb^2 entry
// updates (18 for 16 at nb = 4) instead of eight per entry update; the nb^2
// values b = G(K2 b3, K2+Q b4) are
// the same for the whole block (a block covers one (plane, K2) row), which
// forms them once per launch into LDS.  Lanes run along the column, so each
// of the nb^2 output rows is written as one contiguous run.  Larger nb takes the
// one-thread-per-entry kernel (mo_kernel).  G elements come straight from
// global memory (L2-resident across a plane's rows).  Momenta are added on
// the lattice coordinates in the kernel (no tables).
#include "../../include/g4.h"
#include "g4_internal.hpp"

#include <algorithm>
#include <cstdio>
#include <vector>

namespace g4 {
namespace {

constexpr int kMoPlanes = 256;   // planes per launch
// measurements per launch: 32 keeps a launch's G (2 x 32 x 2.5 MB for the
// 2x2 cluster with 4 orbitals) in the last-level cache; 64 per launch took
// 3.27 ms per 64 measurements there, 32 3.18 ms
constexpr int kMoBatch = 32;

struct MoArgs {
    const void *gu, *gd;
    int64_t g_stride;            // elements between matrices
    double2 *acc;                // slice of this launch's first plane
    int64_t total;               // entries of this launch
    int64_t side;                // N nb^2
    int lx, ly, nw, nwg, nb, ngb, channel, batch, planes;
    int2 qm[kMoPlanes];          // (q, m) per plane of the launch
    double sign[kMoBatch];
};

template <typename R> struct MoCx;
template <> struct MoCx<double> { using V = double2; };
template <> struct MoCx<float> { using V = float2; };

template <typename V>
__device__ __forceinline__ V mo_ld(const V *g, int64_t i) { return g[i]; }

template <typename R>
__global__ __launch_bounds__(256) void mo_kernel(MoArgs a) {
    using V = typename MoCx<R>::V;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= a.total) return;
    const int nb = a.nb, nw = a.nw, nwg = a.nwg, lx = a.lx, ly = a.ly;
    const int64_t side = a.side, ngb = a.ngb;
    const int64_t col = e % side, rr = e / side;
    const int p = (int)(rr / side);
    const int64_t row = rr % side;
    const int K1 = (int)(col / (nb * nb)), b1 = (int)((col / nb) % nb), b2 = (int)(col % nb);
    const int K2 = (int)(row / (nb * nb)), b3 = (int)((row / nb) % nb), b4 = (int)(row % nb);
    const int q = a.qm[p].x, m = a.qm[p].y;
    const int k1 = K1 / nw, i1 = K1 % nw, k2 = K2 / nw, i2 = K2 % nw;
    const int qx = q % lx, qy = q / lx;
    auto kadd = [&](int k) { return (k % lx + qx) % lx + lx * ((k / lx + qy) % ly); };
    auto ksub = [&](int k) { return (qx - k % lx + lx) % lx + lx * ((qy - k / lx + ly) % ly); };
    // G row/column of (window index, orbital)
    auto gi = [&](int w, int b) { return (int64_t)w * nb + b; };
    const V *gu = static_cast<const V *>(a.gu);
    const V *gd = static_cast<const V *>(a.gd);
    R sr = 0, si = 0;
    if (a.channel == CH_PP) {
        const int w_qk1 = ksub(k1) * nwg + (m + nw - 1 - i1), w_qk2 = ksub(k2) * nwg + (m + nw - 1 - i2);
        const int64_t iz = gi(w_qk2, b4) * ngb + gi(w_qk1, b2);          // G(Q-K2 b4, Q-K1 b2)
        const int64_t ix = gi(k2 * nwg + i2, b3) * ngb + gi(k1 * nwg + i1, b1);   // G(K2 b3, K1 b1)
        for (int b = 0; b < a.batch; ++b) {
            const int64_t o = (int64_t)b * a.g_stride;
            const V zu = mo_ld(gu, o + iz), zd = mo_ld(gd, o + iz), xu = mo_ld(gu, o + ix), xd = mo_ld(gd, o + ix);
            const R s = (R)a.sign[b];
            const R tr = zu.x * xd.x - zu.y * xd.y + zd.x * xu.x - zd.y * xu.y;
            const R ti = zu.x * xd.y + zu.y * xd.x + zd.x * xu.y + zd.y * xu.x;
            sr += s * tr;
            si += s * ti;
        }
    } else {
        const R sg = a.channel == CH_MAG ? (R)-1 : (R)1;
        const int w_k1 = k1 * nwg + i1, w_k2 = k2 * nwg + i2;
        const int w_k1q = kadd(k1) * nwg + i1 + m, w_k2q = kadd(k2) * nwg + i2 + m;
        const int64_t i_a = gi(w_k1q, b1) * ngb + gi(w_k1, b2);    // G(K1+Q b1, K1 b2)
        const int64_t i_b = gi(w_k2, b3) * ngb + gi(w_k2q, b4);    // G(K2 b3, K2+Q b4)
        const int64_t i_x = gi(w_k2, b3) * ngb + gi(w_k1, b2);     // G(K2 b3, K1 b2)
        const int64_t i_y = gi(w_k1q, b1) * ngb + gi(w_k2q, b4);   // G(K1+Q b1, K2+Q b4)
        for (int b = 0; b < a.batch; ++b) {
            const int64_t o = (int64_t)b * a.g_stride;
            const V au = mo_ld(gu, o + i_a), ad = mo_ld(gd, o + i_a);
            const V bu = mo_ld(gu, o + i_b), bd = mo_ld(gd, o + i_b);
            const V xu = mo_ld(gu, o + i_x), xd = mo_ld(gd, o + i_x);
            const V yu = mo_ld(gu, o + i_y), yd = mo_ld(gd, o + i_y);
            const R ar = au.x + sg * ad.x, ai = au.y + sg * ad.y;
            const R br = bu.x + sg * bd.x, bi = bu.y + sg * bd.y;
            const R tr = ar * br - ai * bi - (xu.x * yu.x - xu.y * yu.y) - (xd.x * yd.x - xd.y * yd.y);
            const R ti = ar * bi + ai * br - (xu.x * yu.y + xu.y * yu.x) - (xd.x * yd.y + xd.y * yd.x);
            const R s = (R)a.sign[b];
            sr += s * tr;
            si += s * ti;
        }
    }
    double2 *pa = a.acc + e;
    double2 v = *pa;
    v.x += (double)sr;
    v.y += (double)si;
    *pa = v;
}

// Thread (plane p, K2, column (K1, b1, b2)) for all (b3, b4); NB = nb.  A
// block covers up to 256 columns of one (plane, K2) row, so the row-side
// direct operand b(Q; K2 b3, K2+Q b4) of every measurement is the same for
// the whole block: the block forms it once per launch, weight and spin
// combination folded in, into LDS, and the loop reads it from there.  The
// weight of the exchange term is folded into G(K2 b3, K1 b2) as it arrives,
// so each entry update is the twelve FMAs of its three complex products.
template <typename R, int NB>
__global__ __launch_bounds__(256) void mo_rows_kernel(MoArgs a) {
    using V = typename MoCx<R>::V;
    __shared__ V bsh[kMoBatch][NB * NB];
    const int64_t side = a.side;                       // N NB^2
    const int64_t n = side / (NB * NB);
    const int64_t bpr = (side + 255) / 256;            // blocks per (plane, K2) row
    const int64_t rowi = blockIdx.x / bpr;
    const int64_t col = (blockIdx.x % bpr) * 256 + threadIdx.x;
    const bool act = col < side;
    const int K2 = (int)(rowi % n), p = (int)(rowi / n);
    const int nw = a.nw, nwg = a.nwg, lx = a.lx, ly = a.ly;
    const int64_t ngb = a.ngb;
    const int64_t cl = act ? col : 0;
    const int K1 = (int)(cl / (NB * NB)), b1 = (int)((cl / NB) % NB), b2 = (int)(cl % NB);
    const int q = a.qm[p].x, m = a.qm[p].y;
    const int k1 = K1 / nw, i1 = K1 % nw, k2 = K2 / nw, i2 = K2 % nw;
    const int qx = q % lx, qy = q / lx;
    auto kadd = [&](int k) { return (k % lx + qx) % lx + lx * ((k / lx + qy) % ly); };
    auto ksub = [&](int k) { return (qx - k % lx + lx) % lx + lx * ((qy - k / lx + ly) % ly); };
    auto gi = [&](int w, int b) { return (int64_t)w * NB + b; };
    const V *gu = static_cast<const V *>(a.gu);
    const V *gd = static_cast<const V *>(a.gd);
    R sr[NB][NB], si[NB][NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) sr[i][j] = si[i][j] = 0;
    // Operands of one measurement, loaded one measurement ahead into the other
    // of two register sets (the loop alternates them, so nothing is copied).
    // Every product is added by a plain FMA: imaginary parts that enter with a
    // minus sign are negated once per measurement.
    struct Ops {
        V au, ad;
        V xu[NB], xd[NB], yu[NB], yd[NB];
    };
    auto run = [&](auto load, auto compute) __attribute__((always_inline)) {
        if (!act || a.batch == 0) return;
        Ops o0, o1;
        load(0, o0);
        int b = 0;
        for (; b + 1 < a.batch; b += 2) {
            load(b + 1, o1);
            compute(b, o0);
            load(min(b + 2, a.batch - 1), o0);
            compute(b + 1, o1);
        }
        if (b < a.batch) compute(b, o0);
    };
    if (a.channel == CH_PP) {
        const int w_qk1 = ksub(k1) * nwg + (m + nw - 1 - i1), w_qk2 = ksub(k2) * nwg + (m + nw - 1 - i2);
        const int w_k1 = k1 * nwg + i1, w_k2 = k2 * nwg + i2;
        const int64_t iz0 = gi(w_qk2, 0) * ngb + gi(w_qk1, b2);   // G(Q-K2 b4, Q-K1 b2) at b4 = 0 (yu, yd)
        const int64_t ix0 = gi(w_k2, 0) * ngb + gi(w_k1, b1);     // G(K2 b3, K1 b1) at b3 = 0 (xu, xd)
        auto load = [&](int b, Ops &o) __attribute__((always_inline)) {
            const V *pu = gu + (int64_t)b * a.g_stride, *pd = gd + (int64_t)b * a.g_stride;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                o.yu[j] = pu[iz0 + j * ngb];
                o.yd[j] = pd[iz0 + j * ngb];
                o.xu[j] = pu[ix0 + j * ngb];
                o.xd[j] = pd[ix0 + j * ngb];
            }
        };
        auto compute = [&](int b, const Ops &o) __attribute__((always_inline)) {
            const R s = (R)a.sign[b];
            // s G(Q-K2 b4, Q-K1 b2) and its negated imaginary part
            R zur[NB], zui[NB], zun[NB], zdr[NB], zdi[NB], zdn[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                zur[j] = s * o.yu[j].x;
                zui[j] = s * o.yu[j].y;
                zun[j] = -zui[j];
                zdr[j] = s * o.yd[j].x;
                zdi[j] = s * o.yd[j].y;
                zdn[j] = -zdi[j];
            }
#pragma unroll
            for (int b3 = 0; b3 < NB; ++b3)
#pragma unroll
                for (int b4 = 0; b4 < NB; ++b4) {
                    R r = sr[b3][b4], i = si[b3][b4];
                    r += zur[b4] * o.xd[b3].x;
                    r += zun[b4] * o.xd[b3].y;
                    r += zdr[b4] * o.xu[b3].x;
                    r += zdn[b4] * o.xu[b3].y;
                    i += zur[b4] * o.xd[b3].y;
                    i += zui[b4] * o.xd[b3].x;
                    i += zdr[b4] * o.xu[b3].y;
                    i += zdi[b4] * o.xu[b3].x;
                    sr[b3][b4] = r;
                    si[b3][b4] = i;
                }
        };
        run(load, compute);
    } else {
        const R sg = a.channel == CH_MAG ? (R)-1 : (R)1;
        const int w_k1 = k1 * nwg + i1, w_k2 = k2 * nwg + i2;
        const int w_k1q = kadd(k1) * nwg + i1 + m, w_k2q = kadd(k2) * nwg + i2 + m;
        // s_b (Gu -/+ Gd)(K2 b3, K2+Q b4) of every measurement of the launch
        for (int t = threadIdx.x; t < a.batch * NB * NB; t += 256) {
            const int b = t / (NB * NB), j = t % (NB * NB);
            const int64_t ib = (int64_t)b * a.g_stride + gi(w_k2, j / NB) * ngb + gi(w_k2q, j % NB);
            const V u = gu[ib], d = gd[ib];
            const R s = (R)a.sign[b];
            bsh[b][j] = V{s * (u.x + sg * d.x), s * (u.y + sg * d.y)};
        }
        __syncthreads();
        const int64_t ia = gi(w_k1q, b1) * ngb + gi(w_k1, b2);    // G(K1+Q b1, K1 b2)
        const int64_t ix0 = gi(w_k2, 0) * ngb + gi(w_k1, b2);     // G(K2 b3, K1 b2) at b3 = 0
        const int64_t iy0 = gi(w_k1q, b1) * ngb + gi(w_k2q, 0);   // G(K1+Q b1, K2+Q b4) at b4 = 0
        auto load = [&](int b, Ops &o) __attribute__((always_inline)) {
            const V *pu = gu + (int64_t)b * a.g_stride, *pd = gd + (int64_t)b * a.g_stride;
            o.au = pu[ia];
            o.ad = pd[ia];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                o.xu[j] = pu[ix0 + j * ngb];
                o.xd[j] = pd[ix0 + j * ngb];
                o.yu[j] = pu[iy0 + j];
                o.yd[j] = pd[iy0 + j];
            }
        };
        auto compute = [&](int b, const Ops &o) __attribute__((always_inline)) {
            const R s = (R)a.sign[b];
            const R ar = o.au.x + sg * o.ad.x, ai = o.au.y + sg * o.ad.y, an = -ai;
            // -s G(K2 b3, K1 b2) (the exchange's minus and weight), and G(K1+Q b1,
            // K2+Q b4) with its negated imaginary part
            R xur[NB], xui[NB], xdr[NB], xdi[NB], yun[NB], ydn[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                xur[j] = -s * o.xu[j].x;
                xui[j] = -s * o.xu[j].y;
                xdr[j] = -s * o.xd[j].x;
                xdi[j] = -s * o.xd[j].y;
                yun[j] = -o.yu[j].y;
                ydn[j] = -o.yd[j].y;
            }
#pragma unroll
            for (int b3 = 0; b3 < NB; ++b3)
#pragma unroll
                for (int b4 = 0; b4 < NB; ++b4) {
                    const V bb = bsh[b][b3 * NB + b4];
                    R r = sr[b3][b4], i = si[b3][b4];
                    r += ar * bb.x;
                    r += an * bb.y;
                    r += xur[b3] * o.yu[b4].x;
                    r += xui[b3] * yun[b4];
                    r += xdr[b3] * o.yd[b4].x;
                    r += xdi[b3] * ydn[b4];
                    i += ar * bb.y;
                    i += ai * bb.x;
                    i += xur[b3] * o.yu[b4].y;
                    i += xui[b3] * o.yu[b4].x;
                    i += xdr[b3] * o.yd[b4].y;
                    i += xdi[b3] * o.yd[b4].x;
                    sr[b3][b4] = r;
                    si[b3][b4] = i;
                }
        };
        run(load, compute);
    }
    if (!act) return;
    // entry ((p*N + K2)*NB^2 + b3*NB + b4)*side + col
#pragma unroll
    for (int b3 = 0; b3 < NB; ++b3)
#pragma unroll
        for (int b4 = 0; b4 < NB; ++b4) {
            double2 *pa = a.acc + (((int64_t)p * n + K2) * (NB * NB) + b3 * NB + b4) * side + col;
            double2 v = *pa;
            v.x += (double)sr[b3][b4];
            v.y += (double)si[b3][b4];
            *pa = v;
        }
}

template <typename R>
hipError_t launch_mo(const MoArgs &a, hipStream_t st) {
    const int64_t n = a.side / ((int64_t)a.nb * a.nb);
    // rows kernel: whole blocks per (plane, K2) row; entry kernel: one thread per entry
    const int64_t blocks = a.nb <= 8 ? (int64_t)a.planes * n * ((a.side + 255) / 256) : (a.total + 255) / 256;
    if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidConfiguration;
    const dim3 g((unsigned)blocks), b(256);
    switch (a.nb) {
        case 1: hipLaunchKernelGGL((mo_rows_kernel<R, 1>), g, b, 0, st, a); break;
        case 2: hipLaunchKernelGGL((mo_rows_kernel<R, 2>), g, b, 0, st, a); break;
        case 3: hipLaunchKernelGGL((mo_rows_kernel<R, 3>), g, b, 0, st, a); break;
        case 4: hipLaunchKernelGGL((mo_rows_kernel<R, 4>), g, b, 0, st, a); break;
        case 5: hipLaunchKernelGGL((mo_rows_kernel<R, 5>), g, b, 0, st, a); break;
        case 6: hipLaunchKernelGGL((mo_rows_kernel<R, 6>), g, b, 0, st, a); break;
        case 7: hipLaunchKernelGGL((mo_rows_kernel<R, 7>), g, b, 0, st, a); break;
        case 8: hipLaunchKernelGGL((mo_rows_kernel<R, 8>), g, b, 0, st, a); break;
        default: hipLaunchKernelGGL(mo_kernel<R>, g, b, 0, st, a); break;
    }
    return hipGetLastError();
}

}  // namespace

int set_error(int code, const char *msg);

}  // namespace g4

extern "C" int g4_accumulate_mo(int32_t lx, int32_t ly, int32_t nw, int32_t nwex, int32_t nb, int32_t nq,
                                const int32_t *q_list, int64_t q_begin, int64_t q_end, uint32_t channels,
                                int32_t prod, const void *G_up, const void *G_dn, const double *sign,
                                int32_t batch, void *acc_mag, void *acc_chg, void *acc_pp, void *stream) {
    using namespace g4;
    if (lx < 1 || ly < 1 || (int64_t)lx * ly > 4096 || nw < 2 || (nw & 1) || nw > 4096 || nwex < 1 ||
        nwex > 4096 || nb < 1 || nb > 64)
        return set_error(G4_E_ARG, "multi-orbital: bad cluster, frequency or orbital count");
    const int nc = lx * ly;
    if (nq < 1 || nq > nc) return set_error(G4_E_ARG, "multi-orbital: nq outside [1, Nc]");
    std::vector<int> ql(nq), seen(nc, 0);
    for (int i = 0; i < nq; ++i) {
        ql[i] = q_list ? q_list[i] : i;
        if (ql[i] < 0 || ql[i] >= nc || seen[ql[i]]) return set_error(G4_E_ARG, "multi-orbital: bad q_list");
        seen[ql[i]] = 1;
    }
    if (q_begin < 0 || q_end > (int64_t)nq * nwex || q_begin >= q_end)
        return set_error(G4_E_ARG, "multi-orbital: slice planes outside [0, nq*nwex)");
    if (channels == 0 || (channels & ~7u)) return set_error(G4_E_ARG, "multi-orbital: channels of 1|2|4 only");
    if (prod != G4_PROD_F64 && prod != G4_PROD_F32)
        return set_error(G4_E_ARG, "multi-orbital: prod must be G4_PROD_F64 or G4_PROD_F32");
    if (batch < 0) return set_error(G4_E_ARG, "multi-orbital: batch < 0");
    void *acc[3] = {acc_mag, acc_chg, acc_pp};
    for (int c = 0; c < 3; ++c)
        if (((channels >> c) & 1u) != (acc[c] != nullptr))
            return set_error(G4_E_ARG, "multi-orbital: one accumulator per channel, NULL for the others");
    const int64_t nwg = nw + nwex - 1;
    const int64_t ngb = (int64_t)nc * nwg * nb;
    const int64_t side = (int64_t)nc * nw * nb * nb;
    if (ngb * ngb >= ((int64_t)1 << 40) || side > ((int64_t)1 << 30))
        return set_error(G4_E_UNSUPPORTED, "multi-orbital: matrices too large");
    if (batch == 0) return G4_OK;
    if (!G_up || !G_dn || !sign) return set_error(G4_E_ARG, "multi-orbital: NULL G or sign");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t planes = q_end - q_begin;
    for (int c = 0; c < 3; ++c) {
        if (!acc[c]) continue;
        for (int64_t p0 = 0; p0 < planes; p0 += kMoPlanes) {
            const int np = (int)std::min<int64_t>(kMoPlanes, planes - p0);
            for (int b0 = 0; b0 < batch; b0 += kMoBatch) {
                MoArgs a{};
                a.g_stride = ngb * ngb;
                const size_t el = prod == G4_PROD_F64 ? 16 : 8;
                a.gu = static_cast<const char *>(G_up) + (size_t)b0 * a.g_stride * el;
                a.gd = static_cast<const char *>(G_dn) + (size_t)b0 * a.g_stride * el;
                a.acc = static_cast<double2 *>(acc[c]) + p0 * side * side;
                a.total = (int64_t)np * side * side;
                a.side = side;
                a.lx = lx; a.ly = ly; a.nw = nw; a.nwg = (int)nwg; a.nb = nb; a.ngb = (int)ngb;
                a.channel = 1 << c;
                a.batch = std::min(kMoBatch, batch - b0);
                a.planes = np;
                for (int i = 0; i < np; ++i) {
                    const int64_t iQ = q_begin + p0 + i;
                    a.qm[i] = int2{ql[(size_t)(iQ / nwex)], (int)(iQ % nwex)};
                }
                for (int j = 0; j < a.batch; ++j) a.sign[j] = sign[b0 + j];
                if ((a.total + 255) / 256 >= ((int64_t)1 << 31))
                    return set_error(G4_E_UNSUPPORTED, "multi-orbital: grid too large");
                const hipError_t e = prod == G4_PROD_F64 ? launch_mo<double>(a, st) : launch_mo<float>(a, st);
                if (e != hipSuccess) {
                    char msg[160];
                    std::snprintf(msg, sizeof(msg), "multi-orbital launch: %s", hipGetErrorString(e));
                    return set_error(G4_E_HIP, msg);
                }
            }
        }
    }
    return G4_OK;
}
