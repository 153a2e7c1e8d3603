// Seeded synthetic input generator (device side).  Not part of the method:
// it fills G buffers shaped like a 2D Hubbard cluster measurement,
//   G(r,c) = delta_rc / (i w_n + mu + s h - eps_k) + noise (x + i y),
// with x, y ~ N(0,1) from Philox4x32-10 (Salmon et al., SC'11; key (seed, wid),
// counter (r*Ng + c, b, spin, 0)) and Box-Muller in double precision.
#include "g4_internal.hpp"

namespace g4 {
namespace {

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

struct SynthArgs {
    void *out;
    int dtype;
    int lx, ly, nw, nwex, nwg;
    int64_t ng;
    double beta, t, mu, h, noise;
    uint32_t seed, wid;
    int64_t b0;
    int count, spin;
};

__global__ __launch_bounds__(256) void synth_kernel(SynthArgs a) {
    const int64_t per = a.ng * a.ng;
    const int64_t total = per * a.count;
    const double pi = 3.141592653589793;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(idx / per);
        const int64_t e = idx - (int64_t)j * per;
        uint32_t c[4] = {(uint32_t)e, (uint32_t)(a.b0 + j), (uint32_t)a.spin, 0u};
        philox10(c, a.seed, a.wid);
        const double u1 = u53(c[0], c[1]), u2 = u53(c[2], c[3]);
        const double rad = sqrt(-2.0 * log1p(-u1));
        const double ang = 2.0 * pi * u2;
        double re = a.noise * (rad * cos(ang));
        double im = a.noise * (rad * sin(ang));
        const int64_t r = e / a.ng, col = e - r * a.ng;
        if (r == col) {
            const int k = (int)(r / a.nwg);
            const int n = (int)(r - (int64_t)k * a.nwg) - a.nw / 2;
            const int ix = k % a.lx, iy = k / a.lx;
            const double eps = -2.0 * a.t * (cos(2.0 * pi * ix / a.lx) + cos(2.0 * pi * iy / a.ly));
            const double wn = (2.0 * n + 1.0) * pi / a.beta;
            const double zr = a.mu + (a.spin == 0 ? a.h : -a.h) - eps, zi = wn;
            const double den = zr * zr + zi * zi;
            re += zr / den;
            im += -zi / den;
        }
        if (a.dtype == 0)
            static_cast<double2 *>(a.out)[idx] = double2{re, im};
        else
            static_cast<float2 *>(a.out)[idx] = float2{(float)re, (float)im};
    }
}

}  // namespace

hipError_t launch_synth(void *out, int dtype, int lx, int ly, int nw, int nwex, double beta,
                        double t, double mu, double h, double noise, uint32_t seed, uint32_t wid,
                        int64_t b0, int count, int spin, hipStream_t s) {
    SynthArgs a;
    a.out = out;
    a.dtype = dtype;
    a.lx = lx;
    a.ly = ly;
    a.nw = nw;
    a.nwex = nwex;
    a.nwg = nw + nwex - 1;
    a.ng = (int64_t)lx * ly * a.nwg;
    a.beta = beta;
    a.t = t;
    a.mu = mu;
    a.h = h;
    a.noise = noise;
    a.seed = seed;
    a.wid = wid;
    a.b0 = b0;
    a.count = count;
    a.spin = spin;
    const int64_t total = a.ng * a.ng * count;
    if (total == 0) return hipSuccess;
    int64_t g = (total + 255) / 256;
    if (g > 131072) g = 131072;
    hipLaunchKernelGGL(synth_kernel, dim3((unsigned)g), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace g4
