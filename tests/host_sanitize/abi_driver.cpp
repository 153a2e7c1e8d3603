// Drives the HIP-free part of the C ABI (configuration defaults, validation,
// sizes, index maps, error messages) so that the library's host code runs
// under AddressSanitizer and UndefinedBehaviorSanitizer.  Exit status 0 when
// every check holds.
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/g4.h"

static int failures = 0;
#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

static g4_config base() {
    g4_config c;
    g4_config_init(&c);
    c.lx = c.ly = 4;
    c.nw = 64;
    c.nwex = 8;
    c.nq = 16;
    c.q_begin = 0;
    c.q_end = 128;
    return c;
}

int main() {
    CHECK(g4_config_init(nullptr) == G4_E_ARG);
    CHECK(std::strlen(g4_last_error()) > 0);
    uint64_t e = 0, bytes = 0;
    g4_config c = base();
    CHECK(g4_slice_size(&c, &e, &bytes) == G4_OK);
    CHECK(e == 128ull * 1024 * 1024 && bytes > e * 16);
    CHECK(g4_slice_size(nullptr, &e, &bytes) == G4_E_ARG);

    // invalid configurations
    int32_t dup[16];
    for (int i = 0; i < 16; ++i) dup[i] = i;
    dup[2] = 1;
    struct Bad { const char *what; void (*edit)(g4_config &); int code; };
    const Bad bad[] = {
        {"abi", [](g4_config &x) { x.abi_version = 7; }, G4_E_ARG},
        {"lx", [](g4_config &x) { x.lx = 0; }, G4_E_ARG},
        {"nw odd", [](g4_config &x) { x.nw = 63; }, G4_E_ARG},
        {"nwex", [](g4_config &x) { x.nwex = 0; }, G4_E_ARG},
        {"nq", [](g4_config &x) { x.nq = 17; }, G4_E_ARG},
        {"empty slice", [](g4_config &x) { x.q_begin = x.q_end = 5; }, G4_E_ARG},
        {"slice end", [](g4_config &x) { x.q_end = 129; }, G4_E_ARG},
        {"channels", [](g4_config &x) { x.channels = 256; }, G4_E_ARG},
        {"PP and singlet families", [](g4_config &x) { x.channels = G4_PP_UPDOWN | G4_PP_SINGLET; }, G4_E_ARG},
        {"mixed channel families", [](g4_config &x) { x.channels = G4_PH_MAGNETIC | G4_PH_LONG_UPUP; }, G4_E_ARG},
        {"spin channels on packed", [](g4_config &x) { x.mode = G4_MODE_BATCHED; x.max_batch = 8; x.prod = G4_PROD_F32;
                                                       x.g_in = G4_IN_C64; x.channels = G4_PH_TRANSVERSE;
                                                       x.flags = G4_F_PACKED; }, G4_E_UNSUPPORTED},
        {"g_in", [](g4_config &x) { x.g_in = 2; }, G4_E_ARG},
        {"prod", [](g4_config &x) { x.prod = 9; }, G4_E_ARG},
        {"acc", [](g4_config &x) { x.acc = 3; }, G4_E_ARG},
        {"mode", [](g4_config &x) { x.mode = 2; }, G4_E_ARG},
        {"flags", [](g4_config &x) { x.flags = 1u << 9; }, G4_E_ARG},
        {"max_batch", [](g4_config &x) { x.mode = 1; x.prod = 1; x.g_in = 1; x.max_batch = 257; }, G4_E_ARG},
        {"plain fp32", [](g4_config &x) { x.prod = 1; }, G4_E_ARG},
        {"tile", [](g4_config &x) { x.tile = -1; }, G4_E_ARG},
        {"nw above 256", [](g4_config &x) { x.nw = 258; x.lx = x.ly = 1; x.nq = 1; x.q_end = 8; }, G4_E_UNSUPPORTED},
        {"packed fp64", [](g4_config &x) { x.mode = 1; x.max_batch = 4; x.flags = G4_F_PACKED; }, G4_E_UNSUPPORTED},
        {"packed mfma pp", [](g4_config &x) { x.mode = 1; x.prod = 1; x.g_in = 1; x.max_batch = 4;
                                               x.channels = G4_PP_UPDOWN; x.flags = G4_F_PACKED | G4_F_MFMA; },
         G4_E_UNSUPPORTED},
    };
    for (const Bad &b : bad) {
        g4_config x = base();
        b.edit(x);
        const int rc = g4_slice_size(&x, &e, &bytes);
        if (rc != b.code) std::fprintf(stderr, "%s: rc %d\n", b.what, rc);
        CHECK(rc == b.code);
        CHECK(std::strlen(g4_last_error()) > 0);
    }
    {
        g4_config x = base();
        x.q_list = dup;
        CHECK(g4_slice_size(&x, &e, &bytes) == G4_E_ARG);
    }

    // valid plans of the workloads, every variant that fits
    struct Shape { int lx, ly, nw, nwex, nq; int64_t q0, q1; uint32_t ch; };
    const Shape shapes[] = {{2, 2, 16, 1, 1, 0, 1, 1}, {4, 4, 64, 8, 16, 0, 128, 1}, {6, 6, 128, 16, 36, 216, 288, 1},
                            {8, 8, 64, 4, 64, 64, 128, 7}, {3, 2, 24, 5, 6, 3, 27, 7}, {1, 5, 6, 9, 5, 7, 38, 7}};
    for (const Shape &s : shapes) {
        for (int mode = 0; mode < 2; ++mode)
            for (uint32_t fl : {0u, (uint32_t)G4_F_MFMA, (uint32_t)G4_F_PACKED, (uint32_t)G4_F_PACKED_DEEP,
                                (uint32_t)(G4_F_PACKED | G4_F_MFMA)}) {
                g4_config x;
                g4_config_init(&x);
                x.lx = s.lx; x.ly = s.ly; x.nw = s.nw; x.nwex = s.nwex; x.nq = s.nq;
                x.q_begin = s.q0; x.q_end = s.q1; x.channels = s.ch;
                x.mode = mode;
                if (mode == 1) { x.prod = 1; x.g_in = 1; x.acc = 1; x.max_batch = 64; x.flags = fl; }
                else if (fl) continue;
                const int rc = g4_slice_size(&x, &e, &bytes);
                CHECK(rc == G4_OK || rc == G4_E_UNSUPPORTED);
                if (rc == G4_OK) {
                    const uint64_t n = (uint64_t)s.lx * s.ly * s.nw;
                    CHECK(e == (uint64_t)(s.q1 - s.q0) * n * n);
                }
            }
        // index maps against coordinate arithmetic
        g4_config x;
        g4_config_init(&x);
        x.lx = s.lx; x.ly = s.ly; x.nw = s.nw; x.nwex = s.nwex; x.nq = s.nq; x.q_begin = s.q0; x.q_end = s.q1;
        const int nc = s.lx * s.ly;
        std::vector<int32_t> kadd(nc * nc), ksub(nc * nc), pq(s.q1 - s.q0), pm(s.q1 - s.q0);
        CHECK(g4_index_maps(&x, kadd.data(), ksub.data(), pq.data(), pm.data()) == G4_OK);
        for (int k = 0; k < nc; ++k)
            for (int q = 0; q < nc; ++q) {
                const int kx = k % s.lx, ky = k / s.lx, qx = q % s.lx, qy = q / s.lx;
                CHECK(kadd[k * nc + q] == (kx + qx) % s.lx + s.lx * ((ky + qy) % s.ly));
                CHECK(ksub[q * nc + k] == (qx - kx + s.lx) % s.lx + s.lx * ((qy - ky + s.ly) % s.ly));
            }
        for (int64_t p = 0; p < s.q1 - s.q0; ++p) {
            CHECK(pq[p] == (int)((s.q0 + p) / s.nwex));
            CHECK(pm[p] == (int)((s.q0 + p) % s.nwex));
        }
    }
    if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
    else std::printf("host ABI checks passed\n");
    return failures ? 1 : 0;
}
