// One instantiation set of the slice-update kernel: kind G4_KIND (0 plain
// FP64, 1 batched FP64, 2 batched FP32) and G4_EPT K2 rows per thread, for
// every channel combination and plane-group bound.  Compiled once per pair so
// that the build parallelises.
#include "g4_update.hpp"

#if !defined(G4_KIND) || !defined(G4_EPT)
#error "G4_KIND and G4_EPT must be defined"
#endif

#define G4_NAME3(k, e) launch_update_k##k##_e##e
#define G4_NAME(k, e) G4_NAME3(k, e)

namespace g4 {

hipError_t G4_NAME(G4_KIND, G4_EPT)(int channels, int mgroup, int nitems, size_t lds,
                                    const UpdateArgs &a, hipStream_t s) {
    return upd::launch_mg<G4_KIND, G4_EPT>(channels, mgroup, nitems, lds, a, s);
}

}  // namespace g4
