// Instantiations of the MFMA slice-update kernel (batched FP32, direct term on
// the matrix cores): SL 64-column slabs per wave (nw = 64*SL), every channel
// combination and plane-group bound.
#include "g4_update.hpp"

namespace g4 {
namespace {

template <int SL, int MG>
hipError_t launch_mfma_ch(int channels, int nitems, size_t lds, const UpdateArgs &a, hipStream_t s) {
    const void *fn = nullptr;
    switch (channels) {
#define G4_CASE(CHV)                                                                   \
    case CHV:                                                                          \
        fn = reinterpret_cast<const void *>(&upd::update_mfma_kernel<SL, MG, CHV>);    \
        break;
        G4_CASE(1) G4_CASE(2) G4_CASE(3) G4_CASE(4) G4_CASE(5) G4_CASE(6) G4_CASE(7)
#undef G4_CASE
        default:
            return hipErrorInvalidValue;
    }
    if (hipError_t e = ensure_lds_limit(fn, lds); e != hipSuccess) return e;
    UpdateArgs arg = a;
    void *params[] = {&arg};
    return hipLaunchKernel(fn, dim3(nitems), dim3(upd::NT), params, lds, s);
}

template <int SL>
hipError_t launch_mfma_mg(int channels, int mgroup, int nitems, size_t lds, const UpdateArgs &a,
                          hipStream_t s) {
    switch (mgroup) {
        case 1: return launch_mfma_ch<SL, 1>(channels, nitems, lds, a, s);
        case 4: return launch_mfma_ch<SL, 4>(channels, nitems, lds, a, s);
        case 8: return launch_mfma_ch<SL, 8>(channels, nitems, lds, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_update_mfma(int channels, int slabs, int mgroup, int nitems, size_t lds,
                              const UpdateArgs &a, hipStream_t s) {
    switch (slabs) {
        case 1: return launch_mfma_mg<1>(channels, mgroup, nitems, lds, a, s);
        case 2: return launch_mfma_mg<2>(channels, mgroup, nitems, lds, a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace g4
