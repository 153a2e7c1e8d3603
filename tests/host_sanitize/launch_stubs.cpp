// Host-only stand-ins for the kernel launchers of the G4 library, so that its
// C-ABI host code (validation, index maps, work decomposition) can be built
// and run under the host sanitizers on a machine without a GPU.  None of the
// driven entry points reaches a launcher; each stand-in reports an error.
#include "../../paper_2105_00027_amd/csrc/g4_internal.hpp"

namespace g4 {
hipError_t launch_direct_split(int, const DirectArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_gather(int, const GatherArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_update(int, int, int, int, int, int, const UpdateArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_update_packed_mfma(int, int, int, size_t, const UpdateArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_pack_gather(const PackArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_convert_c128_to_c64(const void *, void *, int64_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_acc_to_c128(int, const void *, uint64_t, uint64_t, double *, int, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_c128_to_acc(int, const double *, void *, uint64_t, uint64_t, int, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_fill_zero(void *, size_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_finite_check(const void *, size_t, int, int *, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_merge(int, void *, int, const void *, uint64_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_ref_entries(const RefArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_acc_gather(int, const void *, const uint64_t *, int64_t, double *, int, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_synth(void *, int, int, int, int, int, double, double, double, double, double, uint32_t, uint32_t,
                        int64_t, int, int, hipStream_t) { return hipErrorInvalidValue; }
}  // namespace g4
