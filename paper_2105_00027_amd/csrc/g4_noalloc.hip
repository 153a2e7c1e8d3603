// Allocation-free accumulation entry point (g4_accumulate_into).  Its
// workspace (index tables, work tiles, direct-term vectors, weights) is a
// file-scope device array, one copy per GPU the library runs on, held until
// the process ends.  Host code never uses the array's name as an address:
// on the first call on a device, with that device current, its address is
// taken with hipGetSymbolAddress and kept per device; the kernels receive
// that address.  Every call on a GPU shares its array: calls that overlap on
// one GPU (two host threads, or two streams) race and must not be made.
#include "../../include/g4.h"

#include <hip/hip_runtime.h>

#include <mutex>

#include "g4_internal.hpp"

namespace g4 {
int noalloc_accumulate_entry(const g4_config *cfg, void *const acc[3], const void *G_up, const void *G_dn,
                             const double *sign, int32_t batch, void *ws, uint64_t ws_bytes);
int set_error(int code, const char *msg);
}  // namespace g4

namespace {

constexpr uint64_t kStaticWorkspaceBytes = 64ull << 20;   // 64 MiB per GPU
__device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

extern "C" int g4_accumulate_into(const g4_config *cfg, void *acc_mag, void *acc_chg, void *acc_pp,
                                  const void *G_up, const void *G_dn, const double *sign, int32_t batch) {
    // the configuration is validated before any HIP call
    if (int rc = g4_slice_size(cfg, nullptr, nullptr); rc != G4_OK) return rc;
    if (cfg->device >= kMaxDevices) return g4::set_error(G4_E_UNSUPPORTED, "device ordinal above 63");
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        ptr = g_ptr[cfg->device];
        if (!ptr) {
            int cur = 0;
            if (hipGetDevice(&cur) != hipSuccess) return g4::set_error(G4_E_HIP, "hipGetDevice failed");
            if (hipSetDevice(cfg->device) != hipSuccess)
                return g4::set_error(G4_E_HIP, "hipSetDevice failed");
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            (void)hipSetDevice(cur);
            if (e != hipSuccess || !ptr) {
                (void)hipGetLastError();
                return g4::set_error(G4_E_HIP, "hipGetSymbolAddress of the static workspace failed");
            }
            g_ptr[cfg->device] = ptr;
        }
    }
    void *const acc[3] = {acc_mag, acc_chg, acc_pp};
    return g4::noalloc_accumulate_entry(cfg, acc, G_up, G_dn, sign, batch, ptr, kStaticWorkspaceBytes);
}
