// Device GA over fixed-length protocols (K genes of dose and delay).
//
// The paper's loop (Materials and Methods, "The Main GA Loop"; appendix "GA
// Operators: additional details"): the best protocols are copied unchanged,
// parents are selected (k-way tournament by default; rank-based, roulette or
// truncation), recombined by crossover (one point by default; middle cut,
// two-point or uniform), mutated (per gene by default; dose swap, dose raise),
// and repaired by a guard that lowers the largest dose while the total exceeds
// the cap.  Lower fitness (mean live count) is better.
//
// Kernels: rank (position of each protocol in (fitness, index) order, NaN
// last), history (best and mean fitness of the generation), offspring (one
// thread per child pair), and the generation counter used by replayed graphs.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gga_device.h"
#include "gga_internal.h"
#include "ga_select.h"

namespace gga {
namespace {

__device__ __forceinline__ float rank_key(float f) { return isnan(f) ? INFINITY : f; }

__global__ __launch_bounds__(256) void rank_kernel(const float* fitness, int N, int32_t* order,
                                                   int32_t* position) {
    __shared__ float tile[256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float ki = (i < N) ? rank_key(fitness[i]) : 0.0f;
    int pos = 0;
    for (int base = 0; base < N; base += 256) {
        const int j = base + threadIdx.x;
        tile[threadIdx.x] = (j < N) ? rank_key(fitness[j]) : 0.0f;
        __syncthreads();
        const int n = min(256, N - base);
        for (int t = 0; t < n; ++t) {
            const float kj = tile[t];
            pos += (kj < ki) || (kj == ki && base + t < i);
        }
        __syncthreads();
    }
    if (i < N) {
        position[i] = pos;
        order[pos] = i;
    }
}

// hist[g] = (best fitness, mean fitness over finite entries) of this generation;
// with an archive, its row g receives the best protocol's genes.
__global__ __launch_bounds__(256) void history_kernel(const float* fitness, int N, const int32_t* order,
                                                      const int32_t* generation, float* hist, int hist_cap,
                                                      Archive arc) {
    __shared__ double s_sum[256];
    __shared__ int s_cnt[256];
    double sum = 0.0;
    int cnt = 0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const float f = fitness[i];
        if (!isnan(f)) { sum += f; ++cnt; }
    }
    s_sum[threadIdx.x] = sum;
    s_cnt[threadIdx.x] = cnt;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            s_sum[threadIdx.x] += s_sum[threadIdx.x + s];
            s_cnt[threadIdx.x] += s_cnt[threadIdx.x + s];
        }
        __syncthreads();
    }
    const int g = *generation;
    if (g < 0 || g >= hist_cap) return;
    const int best = order ? order[0] : 0;
    if (threadIdx.x == 0) {
        hist[2 * g] = fitness[best];
        hist[2 * g + 1] = s_cnt[0] ? (float)(s_sum[0] / s_cnt[0]) : __builtin_nanf("");
    }
    if (arc.best_dose && (int)threadIdx.x < arc.K) {
        arc.best_dose[(size_t)g * arc.K + threadIdx.x] = arc.dose[(size_t)best * arc.K + threadIdx.x];
        arc.best_gap[(size_t)g * arc.K + threadIdx.x] = arc.gap[(size_t)best * arc.K + threadIdx.x];
    }
}

__global__ __launch_bounds__(128) void offspring_kernel(GaArgs a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int K = a.K;
    const uint32_t g = (uint32_t)*a.generation;
    if (t < a.n_elite) {                                   // elites: copied unchanged
        const int src = a.order[t];
        for (int j = 0; j < K; ++j) {
            a.next_dose[(size_t)t * K + j] = a.dose[(size_t)src * K + j];
            a.next_gap[(size_t)t * K + j] = a.gap[(size_t)src * K + j];
        }
        return;
    }
    const int c = t - a.n_elite;                           // child pair
    const int n_pairs = (a.n_out - a.n_elite + 1) / 2;
    if (c < 0 || c >= n_pairs) return;
    const int nb = (selection_words(a) + 3) / 4;
    const int parent[2] = {select_parent(c, g, 0, a), select_parent(c, g, nb, a)};
    // crossover: the genes child 0 takes from parent 1 (bit j), child 1 the complement
    uint64_t from_b = 0;
    const Block4 bc = ga_words(c, g, (uint32_t)(2 * nb), a.seed_lo, a.seed_hi);
    if (bc.w0 < a.t_cross && K > 1) {
        const uint64_t all = (K == 64) ? ~0ull : ((1ull << K) - 1ull);
        if (a.crossover == GGA_X_ONE_POINT || a.crossover == GGA_X_MIDDLE) {
            int lo = 1, hi = K - 1;
            if (a.crossover == GGA_X_MIDDLE) {
                lo = max(1, K / 4);
                hi = max(lo, min(K - 1, 3 * K / 4));
            }
            const int cut = lo + pick_of(bc.w1, hi - lo + 1);
            from_b = all & ~((1ull << cut) - 1ull);
        } else if (a.crossover == GGA_X_TWO_POINT) {
            const int c1 = K / 4 + pick_of(bc.w1, K / 2 - K / 4 + 1);
            const int c2 = K / 2 + pick_of(bc.w2, 3 * K / 4 - K / 2 + 1);
            if (c1 < c2) from_b = ((1ull << c2) - 1ull) & ~((1ull << c1) - 1ull);
        } else {
            from_b = ((uint64_t)bc.w1 | ((uint64_t)bc.w2 << 32)) & all;
        }
    }
    for (int ch = 0; ch < 2; ++ch) {
        const int slot = a.n_elite + 2 * c + ch;
        if (slot >= a.n_out) break;
        int q[GGA_KMAX], gp[GGA_KMAX];
        int total = 0;
        for (int j = 0; j < K; ++j) {
            const bool other = ((from_b >> j) & 1ull) != 0;
            const int src = (other == (ch == 0)) ? parent[1] : parent[0];
            int qd = (int)rintf(a.dose[(size_t)src * K + j] / a.quantum);
            int gg = a.gap[(size_t)src * K + j];
            if (a.mutation & GGA_MUT_GENE) {
                const Block4 bm = ga_words(c, g, (uint32_t)(2 * nb + 1 + ch * K + j), a.seed_lo, a.seed_hi);
                if (bm.w0 < a.t_mut) qd = a.dose_q[pick_of(bm.w1, a.n_dose)];
                if (bm.w2 < a.t_mut) gg = a.gaps[pick_of(bm.w3, a.n_gap)];
            }
            q[j] = qd;
            gp[j] = gg;
            total += qd;
        }
        if ((a.mutation & GGA_MUT_SWAP) && K > 1) {       // two doses exchange places
            const Block4 bs = ga_words(c, g, (uint32_t)(2 * nb + 1 + 2 * K + 2 * ch), a.seed_lo, a.seed_hi);
            if (bs.w0 < a.t_mut) {
                const int i = pick_of(bs.w1, K);
                int j = pick_of(bs.w2, K - 1);
                j += (j >= i);
                const int tmp = q[i];
                q[i] = q[j];
                q[j] = tmp;
            }
        }
        if (a.mutation & GGA_MUT_RAISE) {                 // one dose rises to a larger alphabet value
            const Block4 br = ga_words(c, g, (uint32_t)(2 * nb + 2 + 2 * K + 2 * ch), a.seed_lo, a.seed_hi);
            if (br.w0 < a.t_mut && total < a.cap_q) {
                const int i = pick_of(br.w1, K);
                int first = 0;                             // alphabet doses are increasing
                while (first < a.n_dose && a.dose_q[first] <= q[i]) ++first;
                if (first < a.n_dose) {
                    const int nq = a.dose_q[first + pick_of(br.w2, a.n_dose - first)];
                    total += nq - q[i];
                    q[i] = nq;
                }
            }
        }
        // guard: the largest dose (first among equals) steps down the alphabet
        while (total > a.cap_q) {
            bool moved = false;
            int skip_above = 0x7FFFFFFF, skip_from = -1;     // doses that cannot move
            while (!moved) {
                int jm = -1;
                for (int j = 0; j < K; ++j) {
                    const bool eligible = q[j] < skip_above || (q[j] == skip_above && j > skip_from);
                    if (eligible && (jm < 0 || q[j] > q[jm])) jm = j;
                }
                if (jm < 0) break;                          // nothing can move (host rejects such alphabets)
                int lower = -1;
                for (int v = 0; v < a.n_dose; ++v)
                    if (a.dose_q[v] < q[jm]) lower = a.dose_q[v];
                if (lower >= 0) {
                    total -= q[jm] - lower;
                    q[jm] = lower;
                    moved = true;
                } else {
                    skip_above = q[jm];
                    skip_from = jm;
                }
            }
            if (!moved) break;
        }
        for (int j = 0; j < K; ++j) {
            a.next_dose[(size_t)slot * K + j] = (float)((double)q[j] * (double)a.quantum);
            a.next_gap[(size_t)slot * K + j] = gp[j];
        }
    }
}

// dst rows i < n = src rows idx[i] (or row i when idx is null), K genes each,
// plus an optional float per row.
__global__ void gather_kernel(const float* sd, const int32_t* sg, const float* sf, const int32_t* idx, int n, int K,
                              float* dd, int32_t* dg, float* df) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int src = idx ? idx[i] : i;
    for (int j = 0; j < K; ++j) {
        dd[(size_t)i * K + j] = sd[(size_t)src * K + j];
        dg[(size_t)i * K + j] = sg[(size_t)src * K + j];
    }
    if (sf && df) df[i] = sf[src];
}

// Uniform random keys (Philox blocks (i, generation, 0x53435245, 0)): the
// screening ablation that picks candidates without the surrogate.
__global__ void random_key_kernel(int n, const int32_t* generation, uint32_t k0, uint32_t k1, float* key) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Block4 b = philox10((uint32_t)i, (uint32_t)*generation, 0x53435245u, 0u, k0, k1);
    key[i] = (float)(b.w0 >> 8);
}

// fill an int32 array with a value
__global__ void fill_kernel(int32_t* p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void iota_kernel(int32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = i;
}

__global__ void counter_kernel(int32_t* generation, int32_t value, int32_t add) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *generation = add ? *generation + value : value;
}

__global__ void counter_copy_kernel(int32_t* dst, const int32_t* src, int32_t add) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src + add;
}

}  // namespace

hipError_t launch_rank(const float* fitness, int N, int32_t* order, int32_t* position, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(rank_kernel, dim3((N + 255) / 256), dim3(256), 0, s, fitness, N, order, position);
    return hipGetLastError();
}

hipError_t launch_history(const float* fitness, int N, const int32_t* order, const int32_t* generation,
                          float* hist, int hist_cap, const Archive& arc, hipStream_t s) {
    if (N <= 0 || !hist) return hipSuccess;
    if (arc.best_dose && (arc.K > 256 || !arc.best_gap || !arc.dose || !arc.gap)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(history_kernel, dim3(1), dim3(256), 0, s, fitness, N, order, generation, hist, hist_cap, arc);
    return hipGetLastError();
}

hipError_t launch_offspring(const GaArgs& a, hipStream_t s) {
    const int threads = a.n_elite + (a.n_out - a.n_elite + 1) / 2;
    if (threads <= 0) return hipSuccess;
    hipLaunchKernelGGL(offspring_kernel, dim3((threads + 127) / 128), dim3(128), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gather(const float* sd, const int32_t* sg, const float* sf, const int32_t* idx, int n, int K,
                         float* dd, int32_t* dg, float* df, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_kernel, dim3((n + 127) / 128), dim3(128), 0, s, sd, sg, sf, idx, n, K, dd, dg, df);
    return hipGetLastError();
}

hipError_t launch_random_keys(int n, const int32_t* generation, uint64_t seed, float* key, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(random_key_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, generation, (uint32_t)seed,
                       (uint32_t)(seed >> 32), key);
    return hipGetLastError();
}

hipError_t launch_fill(int32_t* p, int n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(iota_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_counter(int32_t* generation, int32_t value, int32_t add, hipStream_t s) {
    hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, s, generation, value, add);
    return hipGetLastError();
}

hipError_t launch_counter_copy(int32_t* dst, const int32_t* src, int32_t add, hipStream_t s) {
    hipLaunchKernelGGL(counter_copy_kernel, dim3(1), dim3(64), 0, s, dst, src, add);
    return hipGetLastError();
}

}  // namespace gga
