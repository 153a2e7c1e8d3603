// One instantiation set of the slice-update kernel: precision G4_PREC (0 FP64,
// 1 FP32) and G4_EPT K2 rows per thread, for every channel combination and
// plane-group bound.  Compiled once per pair so the build parallelises.
#include "g4_update.hpp"

#if !defined(G4_PREC) || !defined(G4_EPT)
#error "G4_PREC and G4_EPT must be defined"
#endif

#define G4_NAME3(p, e) launch_update_p##p##_e##e
#define G4_NAME(p, e) G4_NAME3(p, e)

namespace g4 {

#if G4_PREC == 0
using g4_real_t = double;
#else
using g4_real_t = float;
#endif

hipError_t G4_NAME(G4_PREC, G4_EPT)(int channels, int mgroup, int nitems, size_t lds,
                                    const UpdateArgs &a, hipStream_t s) {
    return upd::launch_mg<g4_real_t, G4_EPT>(channels, mgroup, nitems, lds, a, s);
}

}  // namespace g4
