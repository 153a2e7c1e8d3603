// Direct term of the particle-hole channels as a complex GEMM over the pass's
// measurements on the matrix cores, with split-precision operands (gfx950).
//
// For one transfer plane Q and one PH channel the direct term of a pass is
//   D(K2, K1) = sum_b a_b(Q, K1) b_b(Q, K2),
// a_b = s_b (G_up -/+ G_dn)(K1+Q, K1), b_b = (G_up -/+ G_dn)(K2, K2+Q): a complex
// rank-B update, i.e. a GEMM with K = B.  Written over real numbers with the
// measurement's real and imaginary parts as two K indices,
//   Re D = sum_b [Re b Re a - Im b Im a],  Im D = sum_b [Re b Im a + Im b Re a],
// so one 16x16x16 MFMA covers 8 measurements.  Each FP32 operand x is split
// into a 16-bit high part and a 16-bit low part of the remainder; the products
// hi*hi + hi*lo + lo*hi (lo*lo dropped) are exact in the MFMA's FP32
// accumulate.  BF16: hi = bf16(x), lo = bf16(x - hi).  FP16: hi = f16(x),
// lo = f16(2^11 (x - hi)) (the scale keeps lo out of the subnormal range), and
// the cross products are summed apart and scaled by 2^-11 at the end.
//
// Block: 256 threads, a 64 x 64 tile (K2 rows x K1 columns) of one plane and
// one channel; wave w owns rows 16w..16w+15 as four 16x16 MFMA tiles.  MFMA
// operand layout (16x16x16): lane l holds A[l%16][4(l/16)+t] and
// B[4(l/16)+t][l%16], t < 4; the result D[4(l/16)+r][l%16], r < 4.  The sum is
// added to the slice accumulator (read-modify-write, once per entry and pass).
#include "g4_internal.hpp"

namespace g4 {
namespace {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// float -> bf16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short bf16_rn(float x) {
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// SPLIT 1: BF16 hi+lo, 2: FP16 hi+lo with the low part scaled by 2^11
template <int SPLIT>
struct Split {
    using V = typename std::conditional<SPLIT == 1, s4, h4>::type;
    static __device__ __forceinline__ void split4(const float x[4], V &hi, V &lo) {
        for (int t = 0; t < 4; ++t) {
            if constexpr (SPLIT == 1) {
                const unsigned short h = bf16_rn(x[t]);
                hi[t] = (short)h;
                lo[t] = (short)bf16_rn(x[t] - bf16_f(h));
            } else {
                const _Float16 h = (_Float16)x[t];
                hi[t] = h;
                lo[t] = (_Float16)((x[t] - (float)h) * 2048.f);
            }
        }
    }
    static __device__ __forceinline__ f4 mma(V a, V b, f4 c) {
        if constexpr (SPLIT == 1) return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
        else return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    }
};

template <int SPLIT>
__global__ __launch_bounds__(256) void direct_split_kernel(DirectArgs a) {
    using S = Split<SPLIT>;
    using V = typename S::V;
    const int n = a.d.n, nw = a.d.nw, nc = a.d.nc;
    const int tiles = (n + 63) / 64;
    const int t2 = blockIdx.x / tiles, t1 = blockIdx.x - t2 * tiles;
    const int p = blockIdx.y, sl = blockIdx.z;   // plane, direct-vector slot
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r16 = l & 15, kq = l >> 4;         // row/column within a 16x16 tile, k quarter
    const int K2 = t2 * 64 + 16 * w + r16;       // A row of this lane
    const float2 *pa = static_cast<const float2 *>(a.dir_a) + sl * a.dir_slot_stride + (int64_t)p * n;
    const float2 *pb = static_cast<const float2 *>(a.dir_b) + sl * a.dir_slot_stride + (int64_t)p * n;

    f4 hh_re[4], hh_im[4], x_re[4], x_im[4];     // x: cross products (FP16: scaled by 2^11)
    for (int s = 0; s < 4; ++s) {
        hh_re[s] = f4{0.f, 0.f, 0.f, 0.f};
        hh_im[s] = hh_re[s];
        x_re[s] = hh_re[s];
        x_im[s] = hh_re[s];
    }
    for (int b0 = 0; b0 < a.batch; b0 += 8) {
        // this lane's two measurements of the chunk: b0 + 2*kq + {0, 1}
        float2 bv[2];
        for (int u = 0; u < 2; ++u) {
            const int b = b0 + 2 * kq + u;
            bv[u] = (b < a.batch && K2 < n) ? pb[(int64_t)b * a.dir_b_stride + K2] : float2{0.f, 0.f};
        }
        // A for Re D: (Re b, -Im b) per measurement; for Im D: (Re b, Im b)
        const float are[4] = {bv[0].x, -bv[0].y, bv[1].x, -bv[1].y};
        const float aim[4] = {bv[0].x, bv[0].y, bv[1].x, bv[1].y};
        V are_h, are_l, aim_h, aim_l;
        S::split4(are, are_h, are_l);
        S::split4(aim, aim_h, aim_l);
        for (int s = 0; s < 4; ++s) {
            const int K1 = t1 * 64 + 16 * s + r16;   // B column of this lane
            float2 av[2];
            for (int u = 0; u < 2; ++u) {
                const int b = b0 + 2 * kq + u;
                av[u] = (b < a.batch && K1 < n) ? pa[(int64_t)b * a.dir_b_stride + K1] : float2{0.f, 0.f};
            }
            // B for Re D: (Re a, Im a); for Im D: (Im a, Re a)
            const float bre[4] = {av[0].x, av[0].y, av[1].x, av[1].y};
            const float bim[4] = {av[0].y, av[0].x, av[1].y, av[1].x};
            V bre_h, bre_l, bim_h, bim_l;
            S::split4(bre, bre_h, bre_l);
            S::split4(bim, bim_h, bim_l);
            hh_re[s] = S::mma(are_h, bre_h, hh_re[s]);
            x_re[s] = S::mma(are_h, bre_l, x_re[s]);
            x_re[s] = S::mma(are_l, bre_h, x_re[s]);
            hh_im[s] = S::mma(aim_h, bim_h, hh_im[s]);
            x_im[s] = S::mma(aim_h, bim_l, x_im[s]);
            x_im[s] = S::mma(aim_l, bim_h, x_im[s]);
        }
    }
    // accumulate: lane holds D[4*kq + r][r16] of each 16x16 tile
    const float xs = SPLIT == 2 ? 1.f / 2048.f : 1.f;
    void *acc = a.acc[sl];
    for (int s = 0; s < 4; ++s) {
        const int K1 = t1 * 64 + 16 * s + r16;
        for (int r = 0; r < 4; ++r) {
            const int K2o = t2 * 64 + 16 * w + 4 * kq + r;
            if (K1 >= n || K2o >= n) continue;
            const float re = hh_re[s][r] + x_re[s][r] * xs;
            const float im = hh_im[s][r] + x_im[s][r] * xs;
            // tile-contiguous slice layout [plane][k2][k1][i2][i1]
            const int k2 = K2o / nw, i2 = K2o - k2 * nw, k1 = K1 / nw, i1 = K1 - k1 * nw;
            const int64_t e = (((int64_t)(a.p0 + p) * nc + k2) * nc + k1) * nw * nw + (int64_t)i2 * nw + i1;
            if (a.acc_kind == ACC_C128) {
                double2 *q = static_cast<double2 *>(acc) + e;
                double2 o = *q;
                o.x += (double)re;
                o.y += (double)im;
                *q = o;
            } else if (a.acc_kind == ACC_C64_KAHAN) {
                float4 *q = static_cast<float4 *>(acc) + e;
                float4 o = *q;   // {sum.re, sum.im, comp.re, comp.im}, value = sum - comp
                const float yr = re - o.z, tr = o.x + yr;
                o.z = (tr - o.x) - yr;
                o.x = tr;
                const float yi = im - o.w, ti = o.y + yi;
                o.w = (ti - o.y) - yi;
                o.y = ti;
                *q = o;
            } else {
                float2 *q = static_cast<float2 *>(acc) + e;
                float2 o = *q;
                o.x += re;
                o.y += im;
                *q = o;
            }
        }
    }
}

}  // namespace

hipError_t launch_direct_split(int split, const DirectArgs &a, hipStream_t s) {
    if (a.batch == 0 || a.nslots == 0 || a.d.planes == 0) return hipSuccess;
    const int tiles = (a.d.n + 63) / 64;
    if ((int64_t)tiles * tiles > 0x7fffffff || a.d.planes > 65535) return hipErrorInvalidValue;
    const dim3 grid(tiles * tiles, a.d.planes, a.nslots);
    if (split == 1) hipLaunchKernelGGL(direct_split_kernel<1>, grid, dim3(256), 0, s, a);
    else if (split == 2) hipLaunchKernelGGL(direct_split_kernel<2>, grid, dim3(256), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace g4
