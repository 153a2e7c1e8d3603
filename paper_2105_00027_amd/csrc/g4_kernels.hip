// Helper kernels of the G4 slice library for gfx950 (CDNA4): the direct-term
// gather, the pack of a pass for the packed-operand kernels (which builds the
// direct vectors on the way), precision staging, accumulator conversion for
// readback/load, a fill kernel, and the dispatch to the slice-update kernel
// instantiations (g4_update.hpp, g4_update_inst.hip, g4_update_mfma.hip,
// g4_update_packed.hip).
//
// The gather builds, for every plane Q of the slice and every K, the
// direct-term vectors a_b(Q,K) = s_b D(K+Q,K) and b_b(Q,K) = D(K,K+Q) with
// D = G_up - G_dn (magnetic) or G_up + G_dn (charge), so the update kernel
// reads them coalesced instead of gathering diagonals of G per entry.
#include "g4_internal.hpp"

namespace g4 {
namespace {

template <typename R> struct Cx;
template <> struct Cx<double> { using V = double2; };
template <> struct Cx<float> { using V = float2; };

// ---------------------------------------------------------------------------
// Direct-term vectors: element (slot, b, p, K) at slot*dir_slot_stride +
// b*dir_b_stride + p*n + K; slot 0 = magnetic (G_up - G_dn), slot 1 = charge
// (G_up + G_dn), present when the slot bit is set.
template <typename R>
__global__ __launch_bounds__(256) void gather_kernel(GatherArgs a) {
    using V = typename Cx<R>::V;
    const int n = a.d.n, nw = a.d.nw, nwg = a.d.nwg, nc = a.d.nc, planes = a.d.planes;
    const int64_t ng = a.d.ng;
    const int64_t total = (int64_t)a.batch * planes * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int K = (int)(idx % n);
        const int64_t rest = idx / n;
        const int p = (int)(rest % planes);
        const int b = (int)(rest / planes);
        const int2 qm = a.t.plane_qm[p];
        const int k = K / nw, i = K % nw;
        const int kq = a.t.kadd[k * nc + qm.x];
        const int64_t rK = (int64_t)k * nwg + i;
        const int64_t rKQ = (int64_t)kq * nwg + i + qm.y;
        const V *gu = static_cast<const V *>(a.gu) + (int64_t)b * a.g_stride;
        const V *gd = static_cast<const V *>(a.gd) + (int64_t)b * a.g_stride;
        const V au = gu[rKQ * ng + rK], ad = gd[rKQ * ng + rK];
        const V bu = gu[rK * ng + rKQ], bd = gd[rK * ng + rKQ];
        const R s = (R)a.sign[b];
        V *da = static_cast<V *>(a.dir_a);
        V *db = static_cast<V *>(a.dir_b);
        int64_t o = (int64_t)b * a.dir_b_stride + (int64_t)p * n + K;
        if (a.slots & 1) {
            da[o] = V{s * (au.x - ad.x), s * (au.y - ad.y)};
            db[o] = V{bu.x - bd.x, bu.y - bd.y};
            o += a.dir_slot_stride;
        }
        if (a.slots & 2) {
            da[o] = V{s * (au.x + ad.x), s * (au.y + ad.y)};
            db[o] = V{bu.x + bd.x, bu.y + bd.y};
            o += a.dir_slot_stride;
        }
        if (a.slots & 4) {          // longitudinal up-up
            da[o] = V{s * au.x, s * au.y};
            db[o] = bu;
            o += a.dir_slot_stride;
        }
        if (a.slots & 8) {          // longitudinal up-down
            da[o] = V{s * au.x, s * au.y};
            db[o] = bd;
        }
    }
}

// Packing of one pass for the packed-operand kernel (see PackArgs).  Block
// (R, b) handles row R of matrix b: it copies the row into the packed layout
// (element pairs, 16-byte loads, when Ng is even), zeroes its padding columns,
// and writes the direct-term vector elements that lie in
// the row.
// Row R = kr*Nwg + rho holds
//   a_b(Q, K) = s_b D(K+Q, K) at column k*Nwg + i, K = k*nw + i, q = kr - k,
//                for every m = rho - i that is a bosonic index;
//   b_b(Q, K) = D(K, K+Q) at column kq*Nwg + rho + m, K = kr*nw + rho (rho < nw),
//                q = kq - kr, for every bosonic m;
// for the planes (q, m) in the slice: one thread per (column block, m).  Each
// (plane, K) pair is written exactly once for a and once for b.
__global__ __launch_bounds__(256) void pack_gather_kernel(PackArgs pa) {
    const GatherArgs &a = pa.g;
    const int64_t b = blockIdx.y;
    const int ng = a.d.ng, nwg = a.d.nwg, nw = a.d.nw, nwex = a.d.nwex, nc = a.d.nc, n = a.d.n;
    // Blocks are dealt to the 8 XCDs in turn; each XCD takes a contiguous run of
    // rows, so the direct-vector elements that consecutive rows write into one
    // cache line meet in the same L2 instead of leaving it as partial lines.
    const int per = (ng + 7) / 8;
    const int R = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (R >= ng) return;
    const float2 *su = static_cast<const float2 *>(a.gu) + b * a.g_stride + (int64_t)R * ng;
    const float2 *sd = static_cast<const float2 *>(a.gd) + b * a.g_stride + (int64_t)R * ng;
    float4 *d = static_cast<float4 *>(pa.pack) + b * pa.pack_stride16 + (int64_t)R * pa.ldp;
    const int pcb = pa.pcb, pad = pcb - nwg;
    // source column c = k*nwg + i -> packed column k*pcb + i
    auto dcol = [&](int c) { const int k = c / nwg; return c + k * pad; };
    // lane c: source column c of both spins (8-byte loads, contiguous across
    // the wave) into packed column dcol(c), so that each store instruction
    // writes one contiguous run (16-byte loads of two columns, whose stores
    // then alternate between chunks, took 0.71 against 0.66 ms per pass)
    for (int c = threadIdx.x; c < ng; c += 256) {
        const float2 u = su[c], w = sd[c];
        d[dcol(c)] = float4{u.x, u.y, w.x, w.y};
    }
    // zeros: each block's padding columns, then the row's tail [nc*pcb, ldp)
    for (int e = threadIdx.x; e < nc * pad; e += 256) {
        const int k = e / pad;
        d[k * pcb + nwg + (e - k * pad)] = float4{0.f, 0.f, 0.f, 0.f};
    }
    for (int c = nc * pcb + threadIdx.x; c < pa.ldp; c += 256) d[c] = float4{0.f, 0.f, 0.f, 0.f};
    if (!a.slots) return;
    const int kr = R / nwg, rho = R - kr * nwg;
    const float s = (float)a.sign[b];
    float2 *da = static_cast<float2 *>(a.dir_a) + b * a.dir_b_stride;
    float2 *db = static_cast<float2 *>(a.dir_b) + b * a.dir_b_stride;
    for (int e = threadIdx.x; e < 2 * nc * nwex; e += 256) {
        const int kind = e >= nc * nwex;                 // 0: operand a, 1: operand b
        const int f = e - kind * nc * nwex;
        const int kb = f / nwex, m = f - kb * nwex;      // column block, bosonic index
        int i, col, kk, q;
        if (kind == 0) {
            i = rho - m;
            if (i < 0 || i >= nw) continue;
            col = kb * nwg + i;
            kk = kb;
            q = a.t.ksub[kr * nc + kb];
        } else {
            if (rho >= nw) continue;
            i = rho;
            col = kb * nwg + rho + m;
            kk = kr;
            q = a.t.ksub[kb * nc + kr];
        }
        const int iq = a.t.qpos[q];
        if (iq < 0) continue;
        const int64_t p = (int64_t)iq * nwex + m - a.d.q_begin;
        if (p < 0 || p >= a.d.planes) continue;
        const float2 u = su[col], w = sd[col];
        const float g = kind == 0 ? s : 1.f;
        float2 *out = kind == 0 ? da : db;
        int64_t o = p * n + (int64_t)kk * nw + i;
        if (a.slots & 1) {
            out[o] = float2{g * (u.x - w.x), g * (u.y - w.y)};
            o += a.dir_slot_stride;
        }
        if (a.slots & 2) out[o] = float2{g * (u.x + w.x), g * (u.y + w.y)};
    }
}

__global__ void convert_kernel(const double2 *src, float2 *dst, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 v = src[i];
        dst[i] = float2{(float)v.x, (float)v.y};
    }
}

// Entry j of the documented [plane][K2][K1] order -> its place in the
// tile-contiguous device layout [plane][k2][k1][i2][i1].
__device__ __forceinline__ uint64_t phys_index(uint64_t j, uint64_t nc, uint64_t nw) {
    const uint64_t n = nc * nw;
    const uint64_t K1 = j % n, t = j / n;
    const uint64_t K2 = t % n, p = t / n;
    return ((p * nc + K2 / nw) * nc + K1 / nw) * nw * nw + (K2 % nw) * nw + (K1 % nw);
}

__global__ void acc_to_c128_kernel(int kind, const void *acc, uint64_t first, uint64_t count,
                                   double2 *dst, int nc, int nw) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t e = phys_index(first + i, nc, nw);
        if (kind == ACC_C128) {
            dst[i] = static_cast<const double2 *>(acc)[e];
        } else if (kind == ACC_C64_KAHAN) {
            const float4 v = static_cast<const float4 *>(acc)[e];
            // value = sum - comp (comp is the negated remainder)
            dst[i] = double2{(double)v.x - (double)v.z, (double)v.y - (double)v.w};
        } else {
            const float2 v = static_cast<const float2 *>(acc)[e];
            dst[i] = double2{(double)v.x, (double)v.y};
        }
    }
}

__global__ void c128_to_acc_kernel(int kind, const double2 *src, void *acc, uint64_t first,
                                   uint64_t count, int nc, int nw) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t e = phys_index(first + i, nc, nw);
        const double2 v = src[i];
        if (kind == ACC_C128) {
            static_cast<double2 *>(acc)[e] = v;
            continue;
        }
        const float hr = (float)v.x, hi = (float)v.y;
        if (kind == ACC_C64_KAHAN) {
            const float cr = (float)((double)hr - v.x), ci = (float)((double)hi - v.y);
            static_cast<float4 *>(acc)[e] = float4{hr, hi, cr, ci};
        } else {
            static_cast<float2 *>(acc)[e] = float2{hr, hi};
        }
    }
}

// dst += src entry by entry (same slice geometry, so the same physical index);
// each side in its own accumulator kind.  A compensated destination takes the
// source value's float part and its remainder as two compensated additions.
__device__ __forceinline__ void kahan_add(float &s, float &c, float v) {
    const float y = v - c, t = s + y;
    c = (t - s) - y;
    s = t;
}
__global__ void merge_kernel(int dkind, void *dst, int skind, const void *src, uint64_t count) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (uint64_t)gridDim.x * blockDim.x) {
        double2 v;
        if (skind == ACC_C128) {
            v = static_cast<const double2 *>(src)[e];
        } else if (skind == ACC_C64_KAHAN) {
            const float4 x = static_cast<const float4 *>(src)[e];
            v = double2{(double)x.x - (double)x.z, (double)x.y - (double)x.w};
        } else {
            const float2 x = static_cast<const float2 *>(src)[e];
            v = double2{(double)x.x, (double)x.y};
        }
        if (dkind == ACC_C128) {
            double2 &o = static_cast<double2 *>(dst)[e];
            o.x += v.x;
            o.y += v.y;
        } else if (dkind == ACC_C64_KAHAN) {
            float4 o = static_cast<float4 *>(dst)[e];
            const float hx = (float)v.x, hy = (float)v.y;
            kahan_add(o.x, o.z, hx);
            kahan_add(o.x, o.z, (float)(v.x - (double)hx));
            kahan_add(o.y, o.w, hy);
            kahan_add(o.y, o.w, (float)(v.y - (double)hy));
            static_cast<float4 *>(dst)[e] = o;
        } else {
            float2 &o = static_cast<float2 *>(dst)[e];
            o.x = (float)((double)o.x + v.x);
            o.y = (float)((double)o.y + v.y);
        }
    }
}

// Accumulator values at listed entries of the documented order.
__global__ void acc_gather_kernel(int kind, const void *acc, const uint64_t *idx, int64_t count, double2 *out,
                                  int nc, int nw) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t e = phys_index(idx[j], nc, nw);
        if (kind == ACC_C128) {
            out[j] = static_cast<const double2 *>(acc)[e];
        } else if (kind == ACC_C64_KAHAN) {
            const float4 v = static_cast<const float4 *>(acc)[e];
            out[j] = double2{(double)v.x - (double)v.z, (double)v.y - (double)v.w};
        } else {
            const float2 v = static_cast<const float2 *>(acc)[e];
            out[j] = double2{(double)v.x, (double)v.y};
        }
    }
}

// Reference values for the autotuner: one thread per listed entry sums
// s_b T_ch over the pass in FP64, reading the G elements it needs directly
// (no staging, no tables beyond the momentum maps and the plane decode).
__device__ __forceinline__ double2 ref_g(const void *g, int g_in, int64_t off) {
    if (g_in == 0) return static_cast<const double2 *>(g)[off];
    const float2 v = static_cast<const float2 *>(g)[off];
    return double2{(double)v.x, (double)v.y};
}
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__global__ void ref_entries_kernel(RefArgs a) {
    const int n = a.d.n, nw = a.d.nw, nwg = a.d.nwg, nc = a.d.nc;
    const int64_t ng = a.d.ng;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.count;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t e = a.idx[j];
        const int K1 = (int)(e % (uint64_t)n), K2 = (int)((e / (uint64_t)n) % (uint64_t)n);
        const int p = (int)(e / ((uint64_t)n * n));
        const int2 qm = a.t.plane_qm[p];
        const int q = qm.x, m = qm.y;
        const int k1 = K1 / nw, i1 = K1 % nw, k2 = K2 / nw, i2 = K2 % nw;
        const int64_t r1 = (int64_t)k1 * nwg + i1, r2 = (int64_t)k2 * nwg + i2;
        double2 acc{0.0, 0.0};
        for (int b = 0; b < a.batch; ++b) {
            const int64_t base = (int64_t)b * a.g_stride;
            double2 t;
            if (a.channel == CH_PP || a.channel == CH_PS || a.channel == CH_PT) {
                // Q-K: momentum q-k, local frequency m + nw - 1 - i
                const int64_t s1 = (int64_t)a.t.ksub[q * nc + k1] * nwg + (m + nw - 1 - i1);
                const int64_t s2 = (int64_t)a.t.ksub[q * nc + k2] * nwg + (m + nw - 1 - i2);
                const double2 up = zmul(ref_g(a.gu, a.g_in, base + s2 * ng + s1), ref_g(a.gd, a.g_in, base + r2 * ng + r1));
                const double2 dn = zmul(ref_g(a.gd, a.g_in, base + s2 * ng + s1), ref_g(a.gu, a.g_in, base + r2 * ng + r1));
                t = double2{up.x + dn.x, up.y + dn.y};
                if (a.channel != CH_PP) {
                    // crossed: sum_s G_s(Q-K2, K1) G_-s(K2, Q-K1); singlet (t + c)/2, triplet (t - c)/2
                    const double2 c1 = zmul(ref_g(a.gu, a.g_in, base + s2 * ng + r1), ref_g(a.gd, a.g_in, base + r2 * ng + s1));
                    const double2 c2 = zmul(ref_g(a.gd, a.g_in, base + s2 * ng + r1), ref_g(a.gu, a.g_in, base + r2 * ng + s1));
                    const double pm = a.channel == CH_PS ? 1.0 : -1.0;
                    t = double2{0.5 * (t.x + pm * (c1.x + c2.x)), 0.5 * (t.y + pm * (c1.y + c2.y))};
                }
            } else {
                // K+Q: momentum k+q, local frequency i + m
                const int64_t p1 = (int64_t)a.t.kadd[k1 * nc + q] * nwg + i1 + m;
                const int64_t p2 = (int64_t)a.t.kadd[k2 * nc + q] * nwg + i2 + m;
                const double2 u1 = ref_g(a.gu, a.g_in, base + p1 * ng + r1), d1 = ref_g(a.gd, a.g_in, base + p1 * ng + r1);
                const double2 u2 = ref_g(a.gu, a.g_in, base + r2 * ng + p2), d2 = ref_g(a.gd, a.g_in, base + r2 * ng + p2);
                const double2 xu = ref_g(a.gu, a.g_in, base + r2 * ng + r1), xd = ref_g(a.gd, a.g_in, base + r2 * ng + r1);
                const double2 yu = ref_g(a.gu, a.g_in, base + p1 * ng + p2), yd = ref_g(a.gd, a.g_in, base + p1 * ng + p2);
                if (a.channel == CH_MAG || a.channel == CH_CHG) {
                    const double sg = a.channel == CH_MAG ? -1.0 : 1.0;
                    const double2 dir = zmul(double2{u1.x + sg * d1.x, u1.y + sg * d1.y},
                                             double2{u2.x + sg * d2.x, u2.y + sg * d2.y});
                    const double2 eu = zmul(xu, yu), ed = zmul(xd, yd);
                    t = double2{dir.x - eu.x - ed.x, dir.y - eu.y - ed.y};
                } else if (a.channel == CH_UU) {
                    const double2 dir = zmul(u1, u2), eu = zmul(xu, yu);
                    t = double2{dir.x - eu.x, dir.y - eu.y};
                } else if (a.channel == CH_UD) {
                    t = zmul(u1, d2);
                } else {
                    const double2 e1 = zmul(xd, yu), e2 = zmul(xu, yd);
                    t = double2{-(e1.x + e2.x), -(e1.y + e2.y)};
                }
            }
            const double s = a.sign[b];
            acc.x += s * t.x;
            acc.y += s * t.y;
        }
        reinterpret_cast<double2 *>(a.out)[j] = acc;
    }
}

// Sets *flag when any value in the `nwords` 32-bit words is not finite (all
// exponent bits set): every word is an fp32 value (dbl = 0), or the words pair
// up into doubles whose odd words hold sign and exponent (dbl = 1).  Lanes that
// find one store 1; nothing clears the flag here.
__global__ void finite_check_kernel(const uint32_t *p, size_t nwords, int dbl, int *flag) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const uint32_t mask = dbl ? 0x7ff00000u : 0x7f800000u;
    const size_t step = dbl ? 2 : 1;
    bool bad = false;
    for (size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * step + (dbl ? 1 : 0); i < nwords;
         i += stride * step)
        bad |= (p[i] & mask) == mask;
    if (bad) *flag = 1;
}

__global__ void fill_zero_kernel(uint4 *p, size_t n16, unsigned char *tail, size_t ntail) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t i = i0; i < n16; i += stride) p[i] = uint4{0u, 0u, 0u, 0u};
    if (i0 < ntail) tail[i0] = 0;
}

int grid_for(int64_t work, int threads) {
    int64_t g = (work + threads - 1) / threads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

#define G4_DECL(k, e)                                                                        \
    hipError_t launch_update_k##k##_e##e(int channels, int mgroup, int nitems, size_t lds, \
                                         const UpdateArgs &a, hipStream_t s);
#define G4_DECL_KIND(k) G4_DECL(k, 1) G4_DECL(k, 2) G4_DECL(k, 4) G4_DECL(k, 8)
G4_DECL_KIND(0) G4_DECL_KIND(1) G4_DECL_KIND(2)
#undef G4_DECL_KIND
#undef G4_DECL

hipError_t launch_update_mfma(int channels, int slabs, int mgroup, int nitems, size_t lds,
                              const UpdateArgs &a, hipStream_t s);
#define G4_PDECL(e)                                                                            \
    hipError_t launch_update_packed_e##e(int channels, int mgroup, int nitems, size_t lds,    \
                                         const UpdateArgs &a, hipStream_t s, bool deep);
G4_PDECL(1) G4_PDECL(2) G4_PDECL(4) G4_PDECL(8)
#undef G4_PDECL

hipError_t launch_gather(int prec, const GatherArgs &a, hipStream_t s) {
    const int64_t total = (int64_t)a.batch * a.d.planes * a.d.n;
    if (total == 0) return hipSuccess;
    const int g = grid_for(total, 256);
    if (prec == 0)
        hipLaunchKernelGGL(gather_kernel<double>, dim3(g), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(gather_kernel<float>, dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_update(int kind, int channels, int ept, int mgroup, int nitems, int variant,
                         const UpdateArgs &a, hipStream_t s) {
    if (nitems == 0) return hipSuccess;
    const size_t lds = update_lds_bytes(kind, channels, a.tile, mgroup, a.d, variant);
    if (variant == 1) {
        if (kind != 2 || a.tile != 16 || a.d.nw % 64) return hipErrorInvalidValue;
        return launch_update_mfma(channels, a.d.nw / 64, mgroup, nitems, lds, a, s);
    }
    if (variant == 4) {
        if (kind != 2 || !a.pack) return hipErrorInvalidValue;
        return launch_update_packed_mfma(channels, mgroup, nitems, lds, a, s);
    }
    if (variant == 2 || variant == 3) {
        if (kind != 2 || !a.pack) return hipErrorInvalidValue;
        const bool deep = variant == 3;
        switch (ept) {
            case 1: return launch_update_packed_e1(channels, mgroup, nitems, lds, a, s, deep);
            case 2: return launch_update_packed_e2(channels, mgroup, nitems, lds, a, s, deep);
            case 4: return launch_update_packed_e4(channels, mgroup, nitems, lds, a, s, deep);
            case 8: return launch_update_packed_e8(channels, mgroup, nitems, lds, a, s, deep);
            default: return hipErrorInvalidValue;
        }
    }
#define G4_K(k)                                                                     \
    case k * 16 + 1: return launch_update_k##k##_e1(channels, mgroup, nitems, lds, a, s); \
    case k * 16 + 2: return launch_update_k##k##_e2(channels, mgroup, nitems, lds, a, s); \
    case k * 16 + 4: return launch_update_k##k##_e4(channels, mgroup, nitems, lds, a, s); \
    case k * 16 + 8: return launch_update_k##k##_e8(channels, mgroup, nitems, lds, a, s);
    switch (kind * 16 + ept) {
        G4_K(0) G4_K(1) G4_K(2)
        default: return hipErrorInvalidValue;
    }
#undef G4_K
}

hipError_t launch_pack_gather(const PackArgs &a, hipStream_t s) {
    const int count = a.g.batch, ng = a.g.d.ng;
    if (count == 0) return hipSuccess;
    if (a.pcb < a.g.d.nwg || a.pcb % 8 || a.ldp < a.g.d.nc * a.pcb + 1 || a.pack_stride16 < (int64_t)ng * a.ldp ||
        count > 65535)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(pack_gather_kernel, dim3(8 * ((ng + 7) / 8), count), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_convert_c128_to_c64(const void *src, void *dst, int64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(convert_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s,
                       static_cast<const double2 *>(src), static_cast<float2 *>(dst), count);
    return hipGetLastError();
}

hipError_t launch_acc_to_c128(int acc_kind, const void *acc, uint64_t first, uint64_t count,
                              double *dst, int nc, int nw, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(acc_to_c128_kernel, dim3(grid_for((int64_t)count, 256)), dim3(256), 0, s,
                       acc_kind, acc, first, count, reinterpret_cast<double2 *>(dst), nc, nw);
    return hipGetLastError();
}

hipError_t launch_c128_to_acc(int acc_kind, const double *src, void *acc, uint64_t first,
                              uint64_t count, int nc, int nw, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(c128_to_acc_kernel, dim3(grid_for((int64_t)count, 256)), dim3(256), 0, s,
                       acc_kind, reinterpret_cast<const double2 *>(src), acc, first, count, nc, nw);
    return hipGetLastError();
}

hipError_t launch_merge(int dkind, void *dst, int skind, const void *src, uint64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(merge_kernel, dim3(grid_for((int64_t)count, 256)), dim3(256), 0, s, dkind, dst, skind,
                       src, count);
    return hipGetLastError();
}

hipError_t launch_ref_entries(const RefArgs &a, hipStream_t s) {
    if (a.count == 0) return hipSuccess;
    hipLaunchKernelGGL(ref_entries_kernel, dim3(grid_for(a.count, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_acc_gather(int acc_kind, const void *acc, const uint64_t *idx, int64_t count, double *out,
                             int nc, int nw, hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(acc_gather_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, acc_kind, acc, idx, count,
                       reinterpret_cast<double2 *>(out), nc, nw);
    return hipGetLastError();
}

hipError_t launch_finite_check(const void *p, size_t bytes, int dbl, int *flag, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (bytes % (dbl ? 8 : 4) || reinterpret_cast<uintptr_t>(p) % (dbl ? 8 : 4)) return hipErrorInvalidValue;
    const size_t nwords = bytes / 4;
    hipLaunchKernelGGL(finite_check_kernel, dim3(grid_for((int64_t)(nwords / (dbl ? 2 : 1)), 256)), dim3(256), 0, s,
                       static_cast<const uint32_t *>(p), nwords, dbl, flag);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const size_t n16 = bytes / 16, ntail = bytes % 16;
    unsigned char *tail = static_cast<unsigned char *>(p) + n16 * 16;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for((int64_t)(n16 > ntail ? n16 : ntail), 256)),
                       dim3(256), 0, s, static_cast<uint4 *>(p), n16, tail, ntail);
    return hipGetLastError();
}

}  // namespace g4
