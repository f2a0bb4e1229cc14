// Population generator: random protocols uniform over the feasible set.
//
// A protocol is k (dose, delay) pairs with the total dose under a cap
// (Results, "Defining the search problem").  For protocol p: k is uniform on
// kmin..kmax; the doses are drawn position by position, value v taken with
// probability C[k-i-1][b-v] / C[k-i][b], where C[j][s] counts length-j dose
// sequences with total <= s quanta and b is the remaining budget -- uniform
// over all feasible length-k sequences; every delay is uniform over the
// allowed delays.  Each workgroup builds the counting table in LDS and each
// thread draws one protocol from Philox blocks (p, i, POP_TAG, 0).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gga_device.h"
#include "gga_internal.h"

namespace gga {
namespace {

constexpr uint32_t POP_TAG = 0x504F5055u;
constexpr uint32_t KPOS = 0xFFFFFFFFu;

#pragma clang fp contract(off)
__global__ __launch_bounds__(256) void population_kernel(PopArgs a) {
    extern __shared__ double C[];                // [kmax + 1][cap_q + 1]
    const int W = a.cap_q + 1;
    for (int s = threadIdx.x; s < W; s += blockDim.x) C[s] = 1.0;
    __syncthreads();
    for (int j = 1; j <= a.kmax; ++j) {
        for (int s = threadIdx.x; s < W; s += blockDim.x) {
            double acc = 0.0;
            for (int v = 0; v < a.n_dose; ++v)
                if (a.dose_q[v] <= s) acc += C[(j - 1) * W + s - a.dose_q[v]];
            C[j * W + s] = acc;
        }
        __syncthreads();
    }
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    const Block4 bk = philox10(p, KPOS, POP_TAG, 0, a.seed_lo, a.seed_hi);
    const int k = a.kmin + (int)(((uint64_t)bk.w0 * (uint32_t)(a.kmax - a.kmin + 1)) >> 32);
    int budget = a.cap_q;
    for (int i = 0; i < a.K; ++i) {
        float d = 0.0f;
        int g = 0;
        if (i < k) {
            const Block4 b = philox10(p, i, POP_TAG, 0, a.seed_lo, a.seed_hi);
            const double u = ((double)(b.w0 >> 5) * 67108864.0 + (double)(b.w1 >> 6)) *
                             (1.0 / 9007199254740992.0);
            const double x = u * C[(k - i) * W + budget];
            double acc = 0.0;
            int pick = 0;
            for (int v = 0; v < a.n_dose; ++v) {
                const int q = a.dose_q[v];
                if (q > budget) break;
                const double cnt = C[(k - i - 1) * W + budget - q];
                if (cnt == 0.0) break;
                acc += cnt;
                pick = q;
                if (x < acc) break;
            }
            budget -= pick;
            d = (float)((double)pick * (double)a.quantum);
            g = a.gaps[(int)(((uint64_t)b.w2 * (uint32_t)a.n_gap) >> 32)];
        }
        a.dose[(size_t)p * a.K + i] = d;
        a.gap[(size_t)p * a.K + i] = g;
    }
    a.nfrac[p] = k;
}
#pragma clang fp contract(on)

}  // namespace

hipError_t launch_population(const PopArgs& a, hipStream_t stream) {
    if (a.P <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * (size_t)(a.kmax + 1) * (size_t)(a.cap_q + 1);
    hipLaunchKernelGGL(population_kernel, dim3((a.P + 255) / 256), dim3(256), lds, stream, a);
    return hipGetLastError();
}

}  // namespace gga
