// Microbenchmarks of the three resources the kernels are measured against:
// full-rate 32-bit VALU issue, LDS read bandwidth and HBM read bandwidth.
// Each kernel runs a fixed, bounded amount of work whose result is kept alive
// by a store that only an impossible value triggers; the host times each with
// HIP events after one warm-up launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "peaks.h"

namespace gga {
namespace {

constexpr int PEAK_THREADS = 256;
constexpr int VALU_CHAINS = 8;            // independent FMA chains per lane
constexpr int LDS_VECS = 2048;            // 32 KB of 16-byte vectors per workgroup
constexpr int LDS_UNROLL = 8;

// VALU: VALU_CHAINS independent FMA chains per lane, 4 x VALU_CHAINS FMAs per
// loop trip (each a full-rate v_fma_f32 / v_fmac_f32: one lane-op).
__global__ __launch_bounds__(PEAK_THREADS) void valu_peak_kernel(uint32_t* sink, int trips, float a, float b) {
    float x[VALU_CHAINS];
#pragma unroll
    for (int q = 0; q < VALU_CHAINS; ++q) x[q] = 1e-3f * (float)threadIdx.x + (float)q;
    for (int i = 0; i < trips; ++i) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < VALU_CHAINS; ++q) x[q] = fmaf(x[q], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int q = 0; q < VALU_CHAINS; ++q) s += x[q];
    if (s == -1.0f) sink[blockIdx.x & 63] = __float_as_uint(s);
}

// LDS: every lane reads 16-byte vectors, consecutive lanes consecutive
// vectors (no bank conflicts), LDS_UNROLL reads per loop trip, folded with
// two three-input XORs per vector.
__global__ __launch_bounds__(PEAK_THREADS) void lds_peak_kernel(uint32_t* sink, int trips) {
    __shared__ uint4 buf[LDS_VECS];
    const int t = threadIdx.x;
    for (int k = t; k < LDS_VECS; k += PEAK_THREADS) buf[k] = make_uint4(k, k * 3u, k * 5u, k * 7u);
    __syncthreads();
    uint32_t a0 = 0, a1 = 0;
    int base = 0;
    for (int i = 0; i < trips; ++i) {
#pragma unroll
        for (int u = 0; u < LDS_UNROLL; ++u) {
            const uint4 v = buf[(base + u * PEAK_THREADS + t) & (LDS_VECS - 1)];
            a0 ^= v.x ^ v.y;
            a1 ^= v.z ^ v.w;
        }
        base = (base + 7 * PEAK_THREADS) & (LDS_VECS - 1);
    }
    if ((a0 ^ a1) == 0xFFFFFFFFu) sink[blockIdx.x & 63] = a0;
}

// HBM: a grid-stride read of n 16-byte vectors.
__global__ __launch_bounds__(PEAK_THREADS) void hbm_read_kernel(const uint4* p, size_t n, uint32_t* sink) {
    uint32_t acc = 0;
    for (size_t i = (size_t)blockIdx.x * PEAK_THREADS + threadIdx.x; i < n; i += (size_t)gridDim.x * PEAK_THREADS) {
        const uint4 v = p[i];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == 0x9E3779B9u && threadIdx.x == 0) sink[blockIdx.x & 63] = acc;
}

template <class F>
hipError_t time_launch(F launch, hipStream_t s, float* ms) {
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    launch();                                             // warm-up
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e;
}

}  // namespace

hipError_t measure_peaks(void* buf, size_t bytes, double* valu_ops, double* lds_bytes, double* hbm_bytes,
                         hipStream_t s) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    // the last 256 bytes of the buffer take the (never written) sink stores
    uint32_t* sink = reinterpret_cast<uint32_t*>(static_cast<char*>(buf) + bytes - 256);
    const size_t nvec = (bytes - 256) / 16;
    float ms = 0.0f;
    // VALU: 8 workgroups (8 waves per SIMD) per CU
    const int vblocks = 8 * cus, vtrips = 20000;
    e = time_launch([&] { hipLaunchKernelGGL(valu_peak_kernel, dim3(vblocks), dim3(PEAK_THREADS), 0, s, sink, vtrips,
                                             0.999f, 1e-3f); }, s, &ms);
    if (e != hipSuccess) return e;
    *valu_ops = (double)vblocks * PEAK_THREADS * vtrips * 4.0 * VALU_CHAINS / (ms * 1e-3);
    // LDS: 4 workgroups (32 KB each) per CU
    const int lblocks = 4 * cus, ltrips = 20000;
    e = time_launch([&] { hipLaunchKernelGGL(lds_peak_kernel, dim3(lblocks), dim3(PEAK_THREADS), 0, s, sink,
                                             ltrips); }, s, &ms);
    if (e != hipSuccess) return e;
    *lds_bytes = (double)lblocks * PEAK_THREADS * ltrips * LDS_UNROLL * 16.0 / (ms * 1e-3);
    // HBM: 8 workgroups per CU stream the buffer once
    const int hblocks = 8 * cus;
    e = time_launch([&] { hipLaunchKernelGGL(hbm_read_kernel, dim3(hblocks), dim3(PEAK_THREADS), 0, s,
                                             static_cast<const uint4*>(buf), nvec, sink); }, s, &ms);
    if (e != hipSuccess) return e;
    *hbm_bytes = (double)nvec * 16.0 / (ms * 1e-3);
    return hipSuccess;
}

}  // namespace gga
