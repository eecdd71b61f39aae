// hfmm_direct_noalloc: the direct sum of hfmm_direct with its staging
// records in a fixed device array of the library instead of a caller arena,
// for callers that cannot allocate device memory.
//
// The array lives in the code object: every GPU the library runs on holds
// its own copy, at its own address, until the process ends.  Host code never
// passes the array's name to a kernel (on the host it only names a stand-in
// symbol); the device address is looked up once per device with
// hipGetSymbolAddress and kept.
#include "common.hpp"

#include <mutex>

namespace hfmm {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[HFMM_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on the first
// call on that device)
static int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return HFMM_E_HIP;
    if (dev < 0 || dev >= kMaxDevices) return HFMM_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HFMM_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HFMM_OK;
}

}  // namespace hfmm

using namespace hfmm;

extern "C" int hfmm_direct_noalloc(const double* x, const double* y, const double* z,
                                   const double* m, int64_t n_src, const double* tx,
                                   const double* ty, const double* tz, int64_t n_tgt,
                                   int precision, double eps2, void* phi, void* ax, void* ay,
                                   void* az, void* stream) {
    size_t need = 0;
    int rc = hfmm_direct_bytes(n_src, n_tgt, precision, &need);
    if (rc != HFMM_OK) return rc;
    if (need > (size_t)HFMM_SCRATCH_BYTES) return HFMM_E_NOMEM;
    void* ptr = nullptr;
    rc = scratch_address(&ptr);
    if (rc != HFMM_OK) return rc;
    // the same checks and kernels as hfmm_direct, on the scratch array
    return hfmm_direct(x, y, z, m, n_src, tx, ty, tz, n_tgt, precision, eps2, ptr,
                       (size_t)HFMM_SCRATCH_BYTES, phi, ax, ay, az, stream);
}
