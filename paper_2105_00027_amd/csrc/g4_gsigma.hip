// G_sigma of a batch of measurements from their expansion configurations:
// the walker's nonuniform Fourier transform written as matrix products
// (Background section, the solver workflow), for gfx950.
//
// For measurement b with n vertices (imaginary times tau_i, cluster sites
// r_i) and the walker's n x n matrix M_b:
//   E_b[K][i] = exp(i (w_n tau_i + k . r_i))                 (Ng x n)
//   G_b       = diag(g0) - diag(g0) (E_b M_b E_b^H) diag(g0) / (beta Nc)
// Launches per call:
//   g0_kernel             g0 over the window, FP64, into the workspace;
//   phase_kernel          E_b, phases in FP64 (k . r as an exact fraction
//                         of 2 pi), stored in the output precision;
//   cgemm_kernel<N>       T_b = E_b M_b;
//   cgemm_kernel<H, G>    G_b from T_b E_b^H with the g0 scaling and the
//                         diagonal fused into the store.
// The complex GEMM runs on v_mfma_{f32,f64}_16x16x4: per step of two complex
// k, the four k slots hold (Re, Im) of both (Re C: A slots (Re a, -Im a),
// Im C: (Im a, Re a), B slots (Re b, Im b)).  A 256-thread block owns a
// 64 x 64 output tile (each wave 32 x 32: 2 x 2 MFMA tiles, Re and Im),
// staged through LDS in k chunks of 16, the next chunk held in registers
// while the current one is multiplied; LDS holds the operands in the form
// each lane hands to the MFMA, so the inner loop is LDS reads and MFMAs.
#include "../../include/g4.h"
#include "g4_internal.hpp"

#include <cstdio>

namespace g4 {
namespace {

template <typename T> struct Cx2;
template <> struct Cx2<float> { using V = float2; using V4 = float __attribute__((ext_vector_type(4))); };
template <> struct Cx2<double> { using V = double2; using V4 = double __attribute__((ext_vector_type(4))); };

__device__ __forceinline__ Cx2<float>::V4 mfma16(float a, float b, Cx2<float>::V4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ Cx2<double>::V4 mfma16(double a, double b, Cx2<double>::V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr double kPi = 3.14159265358979323846;

struct GsShape {
    int lx, ly, nc, nw, nwg, ng, n, count, spin;
    double beta, mu, h, t;
};

// g0(K) = 1 / (i w_n + mu + s h - eps_k) for every K of the window, in FP64
__global__ __launch_bounds__(256) void g0_kernel(GsShape s, double2 *g0) {
    const int K = blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= s.ng) return;
    const int k = K / s.nwg, nn = K % s.nwg - s.nw / 2;
    const double w = (2.0 * nn + 1.0) * kPi / s.beta;
    const double eps = -2.0 * s.t * (cos(2.0 * kPi * (k % s.lx) / s.lx) + cos(2.0 * kPi * (k / s.lx) / s.ly));
    const double r = s.mu + (s.spin == 0 ? s.h : -s.h) - eps;
    const double d = r * r + w * w;
    g0[K] = double2{r / d, -w / d};
}

template <typename T>
__global__ __launch_bounds__(256) void phase_kernel(GsShape s, const double *tau, const int32_t *site,
                                                    typename Cx2<T>::V *E) {
    using V = typename Cx2<T>::V;
    const int64_t total = (int64_t)s.count * s.ng * s.n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % s.n);
        const int64_t rest = idx / s.n;
        const int K = (int)(rest % s.ng);
        const int64_t b = rest / s.ng;
        const int k = K / s.nwg, nn = K % s.nwg - s.nw / 2;
        const double w = (2.0 * nn + 1.0) * kPi / s.beta;
        const int st = site[b * s.n + i];
        const int kx = k % s.lx, ky = k / s.lx, rx = st % s.lx, ry = st / s.lx;
        const double th = w * tau[b * s.n + i] +
                          2.0 * kPi * ((double)((kx * rx) % s.lx) / s.lx + (double)((ky * ry) % s.ly) / s.ly);
        double sn, cs;
        sincos(th, &sn, &cs);
        E[idx] = V{(T)cs, (T)sn};
    }
}

// Batched complex GEMM C_b = A_b op(B_b): A_b M x K (lda), op(B_b) = B_b
// (K x N, ldb) or, with BH, the conjugate transpose of B_b (N x K, ldb).
// With GEPI the store is G = (K1 == K2 ? g0(K1) : 0) - g0(K1) C g0(K2) * scale.
struct CgArgs {
    const void *A, *B;
    void *C;
    const double2 *g0;           // GEPI: g0 of every K
    int64_t sA, sB, sC;          // elements between batches
    int lda, ldb, ldc;
    int M, N, K;
    double scale;
};

constexpr int BN = 64, BK = 16;

// TM: 16-row MFMA tiles per wave along M; the block is (32 TM) x 64.
template <typename T, bool BH, bool GEPI, int TM>
__global__ __launch_bounds__(256) void cgemm_kernel(CgArgs a) {
    using V = typename Cx2<T>::V;
    using V4 = typename Cx2<T>::V4;
    constexpr int BM = 32 * TM;
    // Operands in LDS in the form each lane feeds the MFMA: A twice, as
    // (Re, Im) for the real-part slots and (-Im, Re) for the imaginary-part
    // slots; B split into its real and imaginary planes.
    __shared__ V Ap[2][BM][BK + 1];
    __shared__ T Bp[2][BK][BN + 4];
    constexpr int PA = BM * BK / 256, PB = BK * BN / 256;   // elements a thread stages per chunk
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int b = blockIdx.z;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const V *A = static_cast<const V *>(a.A) + (int64_t)b * a.sA;
    const V *B = static_cast<const V *>(a.B) + (int64_t)b * a.sB;
    const int wr = (w >> 1) * 16 * TM, wc = (w & 1) * 32;
    const int slot = l >> 4, comp = slot & 1, kh = slot >> 1, lr = l & 15;
    V4 re[TM][2], im[TM][2];
    for (int i = 0; i < TM; ++i)
        for (int j = 0; j < 2; ++j) {
            re[i][j] = V4{0, 0, 0, 0};
            im[i][j] = V4{0, 0, 0, 0};
        }
    // the next chunk's operands are loaded into registers while the current one is multiplied
    V ra[PA], rb[PB];
    auto load = [&](int k0) {
        for (int u = 0; u < PA; ++u) {
            const int e = tid + 256 * u;
            const int r = e / BK, c = e % BK;
            const int gr = m0 + r, gc = k0 + c;
            ra[u] = (gr < a.M && gc < a.K) ? A[(int64_t)gr * a.lda + gc] : V{0, 0};
        }
        for (int u = 0; u < PB; ++u) {
            const int e = tid + 256 * u;
            const int r = e / BK, c = e % BK;
            if (BH) {
                const int gj = n0 + r, gk = k0 + c;          // B_b row n0 + r, column k0 + c
                rb[u] = (gj < a.N && gk < a.K) ? B[(int64_t)gj * a.ldb + gk] : V{0, 0};
            } else {
                const int rr = e / BN, cc = e % BN;
                const int gk = k0 + rr, gj = n0 + cc;
                rb[u] = (gk < a.K && gj < a.N) ? B[(int64_t)gk * a.ldb + gj] : V{0, 0};
            }
        }
    };
    auto store = [&]() {
        for (int u = 0; u < PA; ++u) {
            const int e = tid + 256 * u;
            const int r = e / BK, c = e % BK;
            const V v = ra[u];
            Ap[0][r][c] = v;
            Ap[1][r][c] = V{-v.y, v.x};
        }
        for (int u = 0; u < PB; ++u) {
            const int e = tid + 256 * u;
            const int r = e / BK, c = e % BK;
            if (BH) {                 // conj(B_b(n0 + r, k0 + c)) at k = c, column r
                Bp[0][c][r] = rb[u].x;
                Bp[1][c][r] = -rb[u].y;
            } else {
                const int rr = e / BN, cc = e % BN;
                Bp[0][rr][cc] = rb[u].x;
                Bp[1][rr][cc] = rb[u].y;
            }
        }
    };
    if (a.K > 0) load(0);
    for (int k0 = 0; k0 < a.K; k0 += BK) {
        __syncthreads();      // the previous chunk's reads are done
        store();
        __syncthreads();
        if (k0 + BK < a.K) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 2) {
            const int kc = kk + kh;
            T are[TM], aim[TM], bv[2];
#pragma unroll
            for (int t = 0; t < TM; ++t) {
                const V av = Ap[comp][wr + 16 * t + lr][kc];
                are[t] = av.x;
                aim[t] = av.y;
            }
#pragma unroll
            for (int t = 0; t < 2; ++t) bv[t] = Bp[comp][kc][wc + 16 * t + lr];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    re[i][j] = mfma16(are[i], bv[j], re[i][j]);
                    im[i][j] = mfma16(aim[i], bv[j], im[i][j]);
                }
        }
    }
    // lane l holds rows 4(l/16) + r of column l % 16 of each 16 x 16 tile
    V *C = static_cast<V *>(a.C) + (int64_t)b * a.sC;
    for (int j = 0; j < 2; ++j) {
        const int col = n0 + wc + 16 * j + lr;
        if (col >= a.N) continue;
        double2 gc{0.0, 0.0};
        if (GEPI) gc = a.g0[col];
        for (int i = 0; i < TM; ++i)
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wr + 16 * i + 4 * slot + r;
                if (row >= a.M) continue;
                double cr = (double)re[i][j][r], ci = (double)im[i][j][r];
                if (GEPI) {
                    const double2 gr = a.g0[row];
                    // g0(row) c g0(col) * scale, subtracted from the diagonal g0
                    const double tr = gr.x * cr - gr.y * ci, ti = gr.x * ci + gr.y * cr;
                    double vr = -(tr * gc.x - ti * gc.y) * a.scale;
                    double vi = -(tr * gc.y + ti * gc.x) * a.scale;
                    if (row == col) {
                        vr += gr.x;
                        vi += gr.y;
                    }
                    cr = vr;
                    ci = vi;
                }
                C[(int64_t)row * a.ldc + col] = V{(T)cr, (T)ci};
            }
    }
}

// Workspace: g0 of the window (Ng complex128), then E and T (count x Ng x n each)
uint64_t workspace_bytes(int64_t ng, int64_t n, int64_t count, int esize) {
    return count == 0 ? 0 : (uint64_t)ng * 16 + 2ull * (uint64_t)count * ng * n * esize;
}

template <typename T>
hipError_t run_gsigma(const GsShape &s, const double *tau, const int32_t *site, const void *M, void *G, void *ws,
                      hipStream_t st) {
    using V = typename Cx2<T>::V;
    constexpr int kTM = sizeof(T) == 4 ? 4 : 2, kBM = 32 * kTM;   // FP64: registers and LDS allow 64-row blocks
    const int64_t per_e = (int64_t)s.ng * s.n;
    double2 *g0 = static_cast<double2 *>(ws);
    V *E = reinterpret_cast<V *>(g0 + s.ng);
    V *Tm = E + (int64_t)s.count * per_e;
    hipLaunchKernelGGL(g0_kernel, dim3((s.ng + 255) / 256), dim3(256), 0, st, s, g0);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    const int64_t total = (int64_t)s.count * per_e;
    if (total > 0) {
        int64_t grid = (total + 255) / 256;
        if (grid > 65536) grid = 65536;
        hipLaunchKernelGGL(phase_kernel<T>, dim3((unsigned)grid), dim3(256), 0, st, s, tau, site, E);
        if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
        CgArgs a1{};
        a1.A = E; a1.B = M; a1.C = Tm;
        a1.sA = per_e; a1.sB = (int64_t)s.n * s.n; a1.sC = per_e;
        a1.lda = s.n; a1.ldb = s.n; a1.ldc = s.n;
        a1.M = s.ng; a1.N = s.n; a1.K = s.n; a1.scale = 1.0;
        hipLaunchKernelGGL((cgemm_kernel<T, false, false, kTM>), dim3((s.n + BN - 1) / BN, (s.ng + kBM - 1) / kBM, s.count),
                           dim3(256), 0, st, a1);
        if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    }
    CgArgs a2{};
    a2.A = Tm; a2.B = E; a2.C = G; a2.g0 = g0;
    a2.sA = per_e; a2.sB = per_e; a2.sC = (int64_t)s.ng * s.ng;
    a2.lda = s.n; a2.ldb = s.n; a2.ldc = s.ng;
    a2.M = s.ng; a2.N = s.ng; a2.K = s.n; a2.scale = 1.0 / (s.beta * s.nc);
    // n = 0 still writes G = diag(g0) (the k loop is empty)
    hipLaunchKernelGGL((cgemm_kernel<T, true, true, kTM>), dim3((s.ng + BN - 1) / BN, (s.ng + kBM - 1) / kBM, s.count),
                       dim3(256), 0, st, a2);
    return hipGetLastError();
}

}  // namespace

int set_error(int code, const char *msg);

}  // namespace g4

extern "C" {

int g4_gsigma_workspace(int32_t lx, int32_t ly, int32_t nw, int32_t nwex, int32_t n, int32_t count, int32_t dtype,
                        uint64_t *bytes) {
    if (!bytes) return g4::set_error(G4_E_ARG, "bytes is NULL");
    if (lx < 1 || ly < 1 || (int64_t)lx * ly > 4096 || nw < 2 || (nw & 1) || nw > 4096 || nwex < 1 ||
        nwex > 4096 || n < 0 || count < 0 || (dtype != G4_IN_C128 && dtype != G4_IN_C64))
        return g4::set_error(G4_E_ARG, "bad G_sigma shape");
    *bytes = g4::workspace_bytes((int64_t)lx * ly * (nw + nwex - 1), n, count, dtype == G4_IN_C128 ? 16 : 8);
    return G4_OK;
}

int g4_gsigma(int32_t lx, int32_t ly, int32_t nw, int32_t nwex, double beta, double mu, double h, double t,
              int32_t spin, int32_t n, int32_t count, const double *tau, const int32_t *site, const void *M,
              int32_t dtype, void *G, void *workspace, uint64_t workspace_bytes, void *stream) {
    uint64_t need = 0;
    if (int rc = g4_gsigma_workspace(lx, ly, nw, nwex, n, count, dtype, &need); rc) return rc;
    if (!(beta > 0) || (spin != 0 && spin != 1)) return g4::set_error(G4_E_ARG, "beta must be positive, spin 0 or 1");
    const int64_t ng = (int64_t)lx * ly * (nw + nwex - 1);
    if (ng * ng >= ((int64_t)1 << 31)) return g4::set_error(G4_E_UNSUPPORTED, "G side above 46340");
    if (count > 65535) return g4::set_error(G4_E_UNSUPPORTED, "more than 65535 measurements per call");
    if (count == 0) return G4_OK;
    if (!G || (n > 0 && (!tau || !site || !M))) return g4::set_error(G4_E_ARG, "NULL pointer");
    if (!workspace || workspace_bytes < need)
        return g4::set_error(G4_E_ARG, "workspace too small (g4_gsigma_workspace gives the size)");
    g4::GsShape s;
    s.lx = lx; s.ly = ly; s.nc = lx * ly; s.nw = nw; s.nwg = nw + nwex - 1; s.ng = (int)ng; s.n = n;
    s.count = count; s.spin = spin; s.beta = beta; s.mu = mu; s.h = h; s.t = t;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const hipError_t e = dtype == G4_IN_C128 ? g4::run_gsigma<double>(s, tau, site, M, G, workspace, st)
                                             : g4::run_gsigma<float>(s, tau, site, M, G, workspace, st);
    if (e != hipSuccess) {
        char msg[160];
        std::snprintf(msg, sizeof(msg), "G_sigma launch: %s", hipGetErrorString(e));
        return g4::set_error(G4_E_HIP, msg);
    }
    return G4_OK;
}

}  // extern "C"
