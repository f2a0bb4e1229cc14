// gga_simulate for callers that cannot allocate device memory: the workspace
// of the slab-form sides lives in a fixed file-scope device array instead of a
// caller buffer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gga_internal.h"

namespace {

// The scratch array.  Host code never passes its name to a kernel or a copy:
// on the host the name is only a stand-in, and the device address comes from
// hipGetSymbolAddress, once per device (each GPU holds its own copy).
static __device__ __align__(256) unsigned char scratch[GGA_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[MAX_DEVICES] = {};

// The current device's address of `scratch`, looked up on the first call on
// that device with it current.
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" int gga_simulate_noalloc(const gga_params* params, const gga_sim_cfg* cfg, const float* dose_d,
                                    const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P, int32_t K,
                                    int32_t* live_d, float* fitness_d, int32_t* traj_d, hipStream_t stream) {
    // the argument checks that decide the size come first; gga_simulate's own
    // checks then run on the same arguments
    if (!cfg || cfg->struct_size != sizeof(gga_sim_cfg)) return cfg ? GGA_E_ABI : GGA_E_ARG;
    const size_t need = gga_workspace_bytes(cfg, P);
    if (need > GGA_NOALLOC_SCRATCH_BYTES) return GGA_E_SCRATCH;
    void* ws = nullptr;
    if (need > 0) {
        const hipError_t e = scratch_address(&ws);
        if (e != hipSuccess) return gga::hip_error(e);
    }
    return gga::simulate_checked(params, cfg, dose_d, gap_h_d, nfrac_d, P, K, ws, need > 0 ? GGA_NOALLOC_SCRATCH_BYTES : 0,
                                 live_d, fitness_d, traj_d, stream);
}
