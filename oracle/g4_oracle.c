/*
 * FP64 CPU oracle for one GPU's slice of the two-particle Green's function
 * (G4, the paper's G_t) accumulation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code, header
 * or table with the HIP library; it is the plain definition written out, entry
 * by entry, in double precision, with every index computed from cluster
 * coordinates and integer Matsubara labels (no lookup tables).
 *
 * What it computes (per measurement b with weight s_b, for every entry of the
 * slice):
 *
 *   G4_ch(K1, K2, Q) += s_b * T_ch(K1, K2, Q)
 *
 *   PH magnetic  T = (Gu-Gd)(K1+Q,K1) (Gu-Gd)(K2,K2+Q) - sum_s G_s(K2,K1) G_s(K1+Q,K2+Q)
 *   PH charge    T = (Gu+Gd)(K1+Q,K1) (Gu+Gd)(K2,K2+Q) - sum_s G_s(K2,K1) G_s(K1+Q,K2+Q)
 *   PP up-down   T = sum_s G_s(Q-K2,Q-K1) G_{-s}(K2,K1)
 *
 * and the spin-resolved particle-hole channels (one spin pair each, the
 * same Wick rule on the same operator strings):
 *
 *   PH longitudinal up-up    s1 = s2 = up:
 *       T = Gu(K1+Q,K1) Gu(K2,K2+Q) - Gu(K2,K1) Gu(K1+Q,K2+Q)
 *   PH longitudinal up-down  s1 = up, s2 = down (no exchange contraction):
 *       T = Gu(K1+Q,K1) Gd(K2,K2+Q)
 *   PH transverse            c+_{K1+Q,s} c_{K1,-s} c+_{K2,-s} c_{K2+Q,s}, summed over s
 *       (no direct contraction):
 *       T = - sum_s G_{-s}(K2,K1) G_s(K1+Q,K2+Q)
 *
 * and the singlet and triplet (S_z = 0) projections of the PP up-down pair,
 * with the pair operators (c+_{K,up} c+_{Q-K,dn} -/+ c+_{K,dn} c+_{Q-K,up})/sqrt(2):
 *
 *   PP singlet  T = 1/2 sum_s [ G_s(Q-K2,Q-K1) G_{-s}(K2,K1) + G_s(Q-K2,K1) G_{-s}(K2,Q-K1) ]
 *   PP triplet  T = 1/2 sum_s [ G_s(Q-K2,Q-K1) G_{-s}(K2,K1) - G_s(Q-K2,K1) G_{-s}(K2,Q-K1) ]
 *
 * (singlet + triplet = PP up-down, Eq. (1)).
 *
 * The PP term is the paper's Eq. (1) (Background section, "Memory-Bound Issue
 * in DCA++") with K3 read as the transfer Q.  The particle-hole terms are the
 * direct-minus-exchange Wick contractions of c+_{K1+Q,s1} c_{K1,s1}
 * c+_{K2,s2} c_{K2+Q,s2}, weighted by s1*s2 (magnetic) or 1 (charge); the
 * paper prints only Eq. (1), so these are a reading, pinned by the brute-force
 * Wick test.  The slice is the paper's distributed G^d_t (Implementation
 * section, "Distributed G_t in QMC Solver"): a contiguous range of transfer
 * planes out of the full array.
 *
 * Conventions:
 *   cluster Lx x Ly, momentum index k = ix + Lx*iy, k+q and q-k taken
 *     coordinate-wise modulo the cluster;
 *   fermionic n in [-Nw/2, Nw/2-1] (w_n = (2n+1) pi/beta), bosonic m in
 *     [0, Nwex-1] (nu_m = 2 pi m/beta), so w_n + nu_m = w_{n+m} and
 *     nu_m - w_n = w_{m-n-1};
 *   G4 combined index K = k*Nw + (n + Nw/2);
 *   G window n in [-Nw/2, Nw/2+Nwex-2], Nwg = Nw+Nwex-1, G row/column index
 *     k*Nwg + (n + Nw/2), G stored row-major, complex interleaved (re, im);
 *   transfer plane iQ = iq*Nwex + m, q = q_list[iq];
 *   slice entry ((iQ - q_begin)*N + K2)*N + K1 with N = Nc*Nw.
 *
 * Compile: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * No FMA contraction: each product is a plain complex multiply, each sum is
 * taken in measurement order.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int lx, ly;          /* cluster extent */
    int nw;              /* G4 fermionic frequencies (even, total count) */
    int nwex;            /* bosonic transfers m = 0..nwex-1 */
    int nq;              /* number of momentum transfers */
    const int *q_list;   /* nq momentum indices */
    long q_begin, q_end; /* slice: planes [q_begin, q_end) of nq*nwex */
} oracle_shape;

enum {
    ORACLE_PH_MAGNETIC = 1, ORACLE_PH_CHARGE = 2, ORACLE_PP_UPDOWN = 4,
    ORACLE_PH_LONG_UPUP = 8, ORACLE_PH_LONG_UPDOWN = 16, ORACLE_PH_TRANSVERSE = 32,
    ORACLE_PP_SINGLET = 64, ORACLE_PP_TRIPLET = 128
};

typedef struct { double re, im; } cplx;

static cplx c_mul(cplx a, cplx b) {
    cplx r;
    r.re = a.re * b.re - a.im * b.im;
    r.im = a.re * b.im + a.im * b.re;
    return r;
}
static cplx c_add(cplx a, cplx b) { cplx r = {a.re + b.re, a.im + b.im}; return r; }
static cplx c_sub(cplx a, cplx b) { cplx r = {a.re - b.re, a.im - b.im}; return r; }

static int wrap(int a, int n) { int r = a % n; return r < 0 ? r + n : r; }

/* momentum k + q: add the lattice coordinates, wrap around the cluster */
static int mom_add(const oracle_shape *s, int k, int q) {
    int ix = k % s->lx, iy = k / s->lx;
    int jx = q % s->lx, jy = q / s->lx;
    return wrap(ix + jx, s->lx) + s->lx * wrap(iy + jy, s->ly);
}

/* momentum q - k */
static int mom_sub(const oracle_shape *s, int q, int k) {
    int ix = k % s->lx, iy = k / s->lx;
    int jx = q % s->lx, jy = q / s->lx;
    return wrap(jx - ix, s->lx) + s->lx * wrap(jy - iy, s->ly);
}

/* G row/column index of (momentum k, fermionic Matsubara label n) */
static long g_index(const oracle_shape *s, int k, int n) {
    int nwg = s->nw + s->nwex - 1;
    int loc = n + s->nw / 2;
    if (loc < 0 || loc >= nwg) {
        fprintf(stderr, "oracle: frequency n=%d outside the G window\n", n);
        abort();
    }
    return (long)k * nwg + loc;
}

static cplx g_at(const double *g, long ng, long r, long c) {
    const double *p = g + 2 * (r * ng + c);
    cplx v = {p[0], p[1]};
    return v;
}

/* T_ch for one measurement (G_up, G_dn of that measurement) and one entry */
static cplx entry_term(const oracle_shape *s, int channel, const double *gu, const double *gd,
                       long ng, long iQ, long K2, long K1) {
    int nw = s->nw;
    int iq = (int)(iQ / s->nwex), m = (int)(iQ % s->nwex);
    int q = s->q_list[iq];
    int k1 = (int)(K1 / nw), n1 = (int)(K1 % nw) - nw / 2;
    int k2 = (int)(K2 / nw), n2 = (int)(K2 % nw) - nw / 2;
    long r_k1 = g_index(s, k1, n1), r_k2 = g_index(s, k2, n2);
    cplx t = {0.0, 0.0};
    if (channel == ORACLE_PH_MAGNETIC || channel == ORACLE_PH_CHARGE || channel == ORACLE_PH_LONG_UPUP ||
        channel == ORACLE_PH_LONG_UPDOWN || channel == ORACLE_PH_TRANSVERSE) {
        long r_k1q = g_index(s, mom_add(s, k1, q), n1 + m);   /* K1 + Q */
        long r_k2q = g_index(s, mom_add(s, k2, q), n2 + m);   /* K2 + Q */
        if (channel == ORACLE_PH_MAGNETIC || channel == ORACLE_PH_CHARGE) {
            cplx u1 = g_at(gu, ng, r_k1q, r_k1), d1 = g_at(gd, ng, r_k1q, r_k1);
            cplx u2 = g_at(gu, ng, r_k2, r_k2q), d2 = g_at(gd, ng, r_k2, r_k2q);
            cplx a = channel == ORACLE_PH_MAGNETIC ? c_sub(u1, d1) : c_add(u1, d1);
            cplx b = channel == ORACLE_PH_MAGNETIC ? c_sub(u2, d2) : c_add(u2, d2);
            cplx direct = c_mul(a, b);
            cplx ex_u = c_mul(g_at(gu, ng, r_k2, r_k1), g_at(gu, ng, r_k1q, r_k2q));
            cplx ex_d = c_mul(g_at(gd, ng, r_k2, r_k1), g_at(gd, ng, r_k1q, r_k2q));
            t = c_sub(direct, c_add(ex_u, ex_d));
        } else if (channel == ORACLE_PH_LONG_UPUP) {
            cplx direct = c_mul(g_at(gu, ng, r_k1q, r_k1), g_at(gu, ng, r_k2, r_k2q));
            cplx ex = c_mul(g_at(gu, ng, r_k2, r_k1), g_at(gu, ng, r_k1q, r_k2q));
            t = c_sub(direct, ex);
        } else if (channel == ORACLE_PH_LONG_UPDOWN) {
            t = c_mul(g_at(gu, ng, r_k1q, r_k1), g_at(gd, ng, r_k2, r_k2q));
        } else {
            cplx ex_du = c_mul(g_at(gd, ng, r_k2, r_k1), g_at(gu, ng, r_k1q, r_k2q));
            cplx ex_ud = c_mul(g_at(gu, ng, r_k2, r_k1), g_at(gd, ng, r_k1q, r_k2q));
            cplx zero = {0.0, 0.0};
            t = c_sub(zero, c_add(ex_du, ex_ud));
        }
    } else if (channel == ORACLE_PP_UPDOWN || channel == ORACLE_PP_SINGLET || channel == ORACLE_PP_TRIPLET) {
        long r_qk1 = g_index(s, mom_sub(s, q, k1), m - n1 - 1); /* Q - K1 */
        long r_qk2 = g_index(s, mom_sub(s, q, k2), m - n2 - 1); /* Q - K2 */
        cplx up = c_mul(g_at(gu, ng, r_qk2, r_qk1), g_at(gd, ng, r_k2, r_k1));
        cplx dn = c_mul(g_at(gd, ng, r_qk2, r_qk1), g_at(gu, ng, r_k2, r_k1));
        t = c_add(up, dn);
        if (channel != ORACLE_PP_UPDOWN) {
            cplx crossed = c_add(c_mul(g_at(gu, ng, r_qk2, r_k1), g_at(gd, ng, r_k2, r_qk1)),
                                 c_mul(g_at(gd, ng, r_qk2, r_k1), g_at(gu, ng, r_k2, r_qk1)));
            cplx sum = channel == ORACLE_PP_SINGLET ? c_add(t, crossed) : c_sub(t, crossed);
            t.re = 0.5 * sum.re;
            t.im = 0.5 * sum.im;
        }
    }
    return t;
}

static int check_shape(const oracle_shape *s, int channel) {
    if (!s || s->lx < 1 || s->ly < 1 || s->nw < 2 || (s->nw & 1) || s->nwex < 1 || s->nq < 1)
        return -1;
    if (!s->q_list || s->q_begin < 0 || s->q_end > (long)s->nq * s->nwex || s->q_begin >= s->q_end)
        return -1;
    for (int i = 0; i < s->nq; ++i)
        if (s->q_list[i] < 0 || s->q_list[i] >= s->lx * s->ly) return -1;
    if (channel != ORACLE_PH_MAGNETIC && channel != ORACLE_PH_CHARGE && channel != ORACLE_PP_UPDOWN &&
        channel != ORACLE_PH_LONG_UPUP && channel != ORACLE_PH_LONG_UPDOWN && channel != ORACLE_PH_TRANSVERSE &&
        channel != ORACLE_PP_SINGLET && channel != ORACLE_PP_TRIPLET)
        return -1;
    return 0;
}

/*
 * Accumulate `batch` measurements into the slice g4 (complex interleaved,
 * (q_end-q_begin)*N*N values).  g_up/g_dn hold batch matrices of Ng x Ng.
 * If comp is non-NULL the sums are Neumaier-compensated per real component and
 * comp (same size as g4) holds the running compensation; value = g4 + comp.
 * (Pinned against exact rational sums of inputs whose plain FP64 sum loses
 * whole terms.)
 * nthreads <= 0 uses the OpenMP default.  Returns 0, or -1 on a bad shape.
 */
int oracle_accumulate(const oracle_shape *s, int channel, const double *g_up, const double *g_dn,
                      const double *sign, int batch, double *g4, double *comp, int nthreads) {
    if (check_shape(s, channel) || batch < 0 || !g_up || !g_dn || !sign || !g4) return -1;
    long nc = (long)s->lx * s->ly;
    long ng = nc * (s->nw + s->nwex - 1);
    long n = nc * s->nw;
    long planes = s->q_end - s->q_begin;
    long rows = planes * n;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    for (int b = 0; b < batch; ++b) {
        const double *gu = g_up + 2 * (size_t)b * ng * ng;
        const double *gd = g_dn + 2 * (size_t)b * ng * ng;
        double sb = sign[b];
#pragma omp parallel for schedule(dynamic, 4)
        for (long row = 0; row < rows; ++row) {
            long iQ = s->q_begin + row / n;
            long K2 = row % n;
            for (long K1 = 0; K1 < n; ++K1) {
                cplx t = entry_term(s, channel, gu, gd, ng, iQ, K2, K1);
                double x[2] = {sb * t.re, sb * t.im};
                double *acc = g4 + 2 * (row * n + K1);
                if (!comp) {
                    acc[0] += x[0];
                    acc[1] += x[1];
                } else {
                    double *cc = comp + 2 * (row * n + K1);
                    for (int j = 0; j < 2; ++j) {
                        double sum = acc[j], tt = sum + x[j];
                        if (fabs(sum) >= fabs(x[j]))
                            cc[j] += (sum - tt) + x[j];
                        else
                            cc[j] += (x[j] - tt) + sum;
                        acc[j] = tt;
                    }
                }
            }
        }
    }
    return 0;
}

/*
 * Sum over the batch, in measurement order, of s_b * T_ch at `count` slice
 * entries given by their flattened slice index.  out: count complex values.
 */
int oracle_entries(const oracle_shape *s, int channel, const double *g_up, const double *g_dn,
                   const double *sign, int batch, const int64_t *idx, long count, double *out) {
    if (check_shape(s, channel) || batch < 0 || !g_up || !g_dn || !sign || (!idx && count) || (!out && count))
        return -1;
    long nc = (long)s->lx * s->ly;
    long ng = nc * (s->nw + s->nwex - 1);
    long n = nc * s->nw;
    long total = (s->q_end - s->q_begin) * n * n;
    for (long j = 0; j < count; ++j)
        if (idx[j] < 0 || idx[j] >= total) return -1;
#pragma omp parallel for schedule(static)
    for (long j = 0; j < count; ++j) {
        long e = idx[j];
        long K1 = e % n, K2 = (e / n) % n, iQ = s->q_begin + e / (n * n);
        double re = 0.0, im = 0.0;
        for (int b = 0; b < batch; ++b) {
            cplx t = entry_term(s, channel, g_up + 2 * (size_t)b * ng * ng,
                                g_dn + 2 * (size_t)b * ng * ng, ng, iQ, K2, K1);
            re += sign[b] * t.re;
            im += sign[b] * t.im;
        }
        out[2 * j] = re;
        out[2 * j + 1] = im;
    }
    return 0;
}

/*
 * The step before the accumulation: a walker's single-particle Green's
 * function G_sigma from its expansion configuration, by the nonuniform
 * Fourier transform that the paper's walker computes with matrix products
 * (Background section, the solver workflow).  For n vertices with imaginary
 * times tau_i and cluster sites r_i = rx + Lx*ry, and the walker's n x n
 * matrix M (row-major complex), for entries (K1, K2) of the G window:
 *
 *   G(K1, K2) = g0(K1) delta_{K1,K2}
 *               - g0(K1) [ sum_{i,j} e^{+i th_i(K1)} M_ij e^{-i th_j(K2)} ] g0(K2) / (beta Nc)
 *   th_i(K) = w_n tau_i + k . r_i,   k . r = 2 pi (kx rx / Lx + ky ry / Ly),
 *   g0(k, n) = 1 / (i w_n + mu + s h - eps_k),  eps_k = -2 t (cos kx + cos ky),
 *
 * s = +1 for spin 0 (up), -1 for spin 1 (down); K = k*Nwg + (n + Nw/2) over
 * the G window n in [-Nw/2, Nw/2+Nwex-2].  Each entry is the double sum
 * written out (O(n^2) per entry), every exponential evaluated by itself.
 * idx: count flattened entries K1*Ng + K2; out: count complex values.
 * Returns 0, or -1 on bad arguments.
 */
int oracle_gsigma(int lx, int ly, int nw, int nwex, double beta, double mu, double h, double t, int spin,
                  int n, const double *tau, const int *site, const double *M, const int64_t *idx, long count,
                  double *out) {
    if (lx < 1 || ly < 1 || nw < 2 || (nw & 1) || nwex < 1 || !(beta > 0) || (spin != 0 && spin != 1) ||
        n < 0 || (n && (!tau || !site || !M)) || (count && (!idx || !out)))
        return -1;
    const long nc = (long)lx * ly, nwg = nw + nwex - 1, ng = nc * nwg;
    for (int i = 0; i < n; ++i)
        if (site[i] < 0 || site[i] >= nc) return -1;
    for (long j = 0; j < count; ++j)
        if (idx[j] < 0 || idx[j] >= ng * ng) return -1;
    const double pi = 3.14159265358979323846;
    const double sg = spin == 0 ? 1.0 : -1.0;
#pragma omp parallel for schedule(static)
    for (long j = 0; j < count; ++j) {
        const long K1 = idx[j] / ng, K2 = idx[j] % ng;
        const long k1 = K1 / nwg, k2 = K2 / nwg;
        const long n1 = K1 % nwg - nw / 2, n2 = K2 % nwg - nw / 2;
        const double w1 = (2.0 * n1 + 1.0) * pi / beta, w2 = (2.0 * n2 + 1.0) * pi / beta;
        const long k1x = k1 % lx, k1y = k1 / lx, k2x = k2 % lx, k2y = k2 / lx;
        /* g0 at both ends */
        cplx g0a, g0b;
        {
            const double ea = -2.0 * t * (cos(2.0 * pi * k1x / lx) + cos(2.0 * pi * k1y / ly));
            const double eb = -2.0 * t * (cos(2.0 * pi * k2x / lx) + cos(2.0 * pi * k2y / ly));
            const double ra = mu + sg * h - ea, rb = mu + sg * h - eb;   /* 1/(i w + r) = (r - i w)/(r^2 + w^2) */
            g0a.re = ra / (ra * ra + w1 * w1);
            g0a.im = -w1 / (ra * ra + w1 * w1);
            g0b.re = rb / (rb * rb + w2 * w2);
            g0b.im = -w2 / (rb * rb + w2 * w2);
        }
        cplx sum = {0.0, 0.0};
        for (int a = 0; a < n; ++a) {
            const long rax = site[a] % lx, ray = site[a] / lx;
            const double tha = w1 * tau[a] + 2.0 * pi * ((double)(k1x * rax) / lx + (double)(k1y * ray) / ly);
            const cplx ea = {cos(tha), sin(tha)};
            for (int b = 0; b < n; ++b) {
                const long rbx = site[b] % lx, rby = site[b] / lx;
                const double thb = w2 * tau[b] + 2.0 * pi * ((double)(k2x * rbx) / lx + (double)(k2y * rby) / ly);
                const cplx eb = {cos(thb), -sin(thb)};
                const cplx m = {M[2 * ((long)a * n + b)], M[2 * ((long)a * n + b) + 1]};
                sum = c_add(sum, c_mul(c_mul(ea, m), eb));
            }
        }
        const double norm = 1.0 / (beta * (double)nc);
        const cplx corr = c_mul(c_mul(g0a, sum), g0b);
        cplx g = {-corr.re * norm, -corr.im * norm};
        if (K1 == K2) g = c_add(g, g0a);
        out[2 * j] = g.re;
        out[2 * j + 1] = g.im;
    }
    return 0;
}

/*
 * Multi-orbital G4: every single-particle index carries an orbital label,
 * (K, b) with b in [0, nb); G_sigma is (Ng nb) x (Ng nb), row/column index
 * (k*Nwg + n + Nw/2)*nb + b.  A G4 entry carries four labels: (K1, b1, b2),
 * (K2, b3, b4).  By the same Wick rule as the single-band channels, on the
 * strings c+_{K1+Q,b1,s1} c_{K1,b2,s1} c+_{K2,b3,s2} c_{K2+Q,b4,s2} (PH) and
 * c+_{K2,b3,-s} c+_{Q-K2,b4,s} c_{Q-K1,b2,s} c_{K1,b1,-s} (PP):
 *
 *   PH magnetic/charge  T = (Gu -/+ Gd)(K1+Q b1, K1 b2) (Gu -/+ Gd)(K2 b3, K2+Q b4)
 *                           - sum_s G_s(K2 b3, K1 b2) G_s(K1+Q b1, K2+Q b4)
 *   PP up-down          T = sum_s G_s(Q-K2 b4, Q-K1 b2) G_{-s}(K2 b3, K1 b1)
 *
 * nb = 1 is the single-band definition above.  Slice entry
 * ((p*N + K2)*nb*nb + b3*nb + b4) * (N*nb*nb) + (K1*nb + b1)*nb + b2, p the
 * plane within the slice; the slice holds planes*(N nb^2)^2 entries.
 */
static cplx mo_g(const double *g, long ngb, long r, int br, long c, int bc, int nb) {
    return g_at(g, ngb, r * nb + br, c * nb + bc);
}

static cplx mo_term(const oracle_shape *s, int nb, int channel, const double *gu, const double *gd, long ngb,
                    long iQ, long K2, int b3, int b4, long K1, int b1, int b2) {
    int nw = s->nw;
    int iq = (int)(iQ / s->nwex), m = (int)(iQ % s->nwex);
    int q = s->q_list[iq];
    int k1 = (int)(K1 / nw), n1 = (int)(K1 % nw) - nw / 2;
    int k2 = (int)(K2 / nw), n2 = (int)(K2 % nw) - nw / 2;
    long r_k1 = g_index(s, k1, n1), r_k2 = g_index(s, k2, n2);
    cplx t = {0.0, 0.0};
    if (channel == ORACLE_PH_MAGNETIC || channel == ORACLE_PH_CHARGE) {
        long r_k1q = g_index(s, mom_add(s, k1, q), n1 + m);
        long r_k2q = g_index(s, mom_add(s, k2, q), n2 + m);
        cplx u1 = mo_g(gu, ngb, r_k1q, b1, r_k1, b2, nb), d1 = mo_g(gd, ngb, r_k1q, b1, r_k1, b2, nb);
        cplx u2 = mo_g(gu, ngb, r_k2, b3, r_k2q, b4, nb), d2 = mo_g(gd, ngb, r_k2, b3, r_k2q, b4, nb);
        cplx a = channel == ORACLE_PH_MAGNETIC ? c_sub(u1, d1) : c_add(u1, d1);
        cplx b = channel == ORACLE_PH_MAGNETIC ? c_sub(u2, d2) : c_add(u2, d2);
        cplx ex_u = c_mul(mo_g(gu, ngb, r_k2, b3, r_k1, b2, nb), mo_g(gu, ngb, r_k1q, b1, r_k2q, b4, nb));
        cplx ex_d = c_mul(mo_g(gd, ngb, r_k2, b3, r_k1, b2, nb), mo_g(gd, ngb, r_k1q, b1, r_k2q, b4, nb));
        t = c_sub(c_mul(a, b), c_add(ex_u, ex_d));
    } else if (channel == ORACLE_PP_UPDOWN) {
        long r_qk1 = g_index(s, mom_sub(s, q, k1), m - n1 - 1);
        long r_qk2 = g_index(s, mom_sub(s, q, k2), m - n2 - 1);
        cplx up = c_mul(mo_g(gu, ngb, r_qk2, b4, r_qk1, b2, nb), mo_g(gd, ngb, r_k2, b3, r_k1, b1, nb));
        cplx dn = c_mul(mo_g(gd, ngb, r_qk2, b4, r_qk1, b2, nb), mo_g(gu, ngb, r_k2, b3, r_k1, b1, nb));
        t = c_add(up, dn);
    }
    return t;
}

/*
 * Accumulate `batch` measurements of the multi-orbital slice into g4
 * (complex interleaved, planes*(N nb^2)^2 values).  Channels: magnetic,
 * charge, PP up-down.  Returns 0, or -1 on a bad shape or argument.
 */
int oracle_accumulate_mo(const oracle_shape *s, int nb, int channel, const double *g_up, const double *g_dn,
                         const double *sign, int batch, double *g4) {
    if (check_shape(s, channel) || nb < 1 || batch < 0 || !g_up || !g_dn || !sign || !g4) return -1;
    if (channel != ORACLE_PH_MAGNETIC && channel != ORACLE_PH_CHARGE && channel != ORACLE_PP_UPDOWN) return -1;
    long nc = (long)s->lx * s->ly;
    long ngb = nc * (s->nw + s->nwex - 1) * nb;
    long n = nc * s->nw;
    long side = n * nb * nb;
    long planes = s->q_end - s->q_begin;
    for (int b = 0; b < batch; ++b) {
        const double *gu = g_up + 2 * (size_t)b * ngb * ngb;
        const double *gd = g_dn + 2 * (size_t)b * ngb * ngb;
#pragma omp parallel for schedule(dynamic, 4)
        for (long row = 0; row < planes * side; ++row) {
            long iQ = s->q_begin + row / side;
            long r = row % side;
            long K2 = r / (nb * nb);
            int b3 = (int)((r / nb) % nb), b4 = (int)(r % nb);
            for (long col = 0; col < side; ++col) {
                long K1 = col / (nb * nb);
                int b1 = (int)((col / nb) % nb), b2 = (int)(col % nb);
                cplx t = mo_term(s, nb, channel, gu, gd, ngb, iQ, K2, b3, b4, K1, b1, b2);
                double *acc = g4 + 2 * (row * side + col);
                acc[0] += sign[b] * t.re;
                acc[1] += sign[b] * t.im;
            }
        }
    }
    return 0;
}

/*
 * Sum over the batch, in measurement order, of s_b * T_ch of the
 * multi-orbital slice at `count` entries given by their flattened index
 * (layout of oracle_accumulate_mo).  out: count complex values.
 */
int oracle_entries_mo(const oracle_shape *s, int nb, int channel, const double *g_up, const double *g_dn,
                      const double *sign, int batch, const int64_t *idx, long count, double *out) {
    if (check_shape(s, channel) || nb < 1 || batch < 0 || !g_up || !g_dn || !sign || (count && (!idx || !out)))
        return -1;
    if (channel != ORACLE_PH_MAGNETIC && channel != ORACLE_PH_CHARGE && channel != ORACLE_PP_UPDOWN) return -1;
    long nc = (long)s->lx * s->ly;
    long ngb = nc * (s->nw + s->nwex - 1) * nb;
    long side = nc * s->nw * nb * nb;
    long total = (s->q_end - s->q_begin) * side * side;
    for (long j = 0; j < count; ++j)
        if (idx[j] < 0 || idx[j] >= total) return -1;
#pragma omp parallel for schedule(static)
    for (long j = 0; j < count; ++j) {
        long e = idx[j];
        long col = e % side, row = (e / side) % side, iQ = s->q_begin + e / (side * side);
        long K1 = col / (nb * nb), K2 = row / (nb * nb);
        int b1 = (int)((col / nb) % nb), b2 = (int)(col % nb), b3 = (int)((row / nb) % nb), b4 = (int)(row % nb);
        double re = 0.0, im = 0.0;
        for (int b = 0; b < batch; ++b) {
            cplx t = mo_term(s, nb, channel, g_up + 2 * (size_t)b * ngb * ngb, g_dn + 2 * (size_t)b * ngb * ngb,
                             ngb, iQ, K2, b3, b4, K1, b1, b2);
            re += sign[b] * t.re;
            im += sign[b] * t.im;
        }
        out[2 * j] = re;
        out[2 * j + 1] = im;
    }
    return 0;
}

/* Threads OpenMP would use (for reporting the CPU-baseline core count). */
int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
