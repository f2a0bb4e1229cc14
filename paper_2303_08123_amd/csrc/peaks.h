// Library-internal interface of the microbenchmarks (peaks.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace gga {

// Lane-ops/s of full-rate VALU FMAs, LDS read bytes/s and HBM read bytes/s of
// `buf` (bytes >= 256 MiB + 256; its last 256 bytes are reserved).
// Synchronous.
hipError_t measure_peaks(void* buf, size_t bytes, double* valu_ops, double* lds_bytes, double* hbm_bytes,
                         hipStream_t s);

}  // namespace gga
