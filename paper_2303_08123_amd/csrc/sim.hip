// Resident variants of the simulation kernel (see sim_kernel.h), the fitness
// reduction, the Philox test fill, and the per-lattice variant choice.
#include <atomic>

#include "sim_kernel.h"

namespace gga {
namespace {

__global__ void fitness_kernel(const int32_t* live, int P, int R, float* fitness) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    long long sum = 0;
    bool bad = false;
    for (int r = 0; r < R; ++r) {
        const int v = live[(size_t)p * R + r];
        bad |= v < 0;
        sum += v;
    }
    fitness[p] = bad ? __builtin_nanf("") : (float)((double)sum / (double)R);
}

__global__ void philox_fill_kernel(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                                   long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Block4 b = philox10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
    out[4 * i] = b.w0;
    out[4 * i + 1] = b.w1;
    out[4 * i + 2] = b.w2;
    out[4 * i + 3] = b.w3;
}

template <int CPL, int RPT, int NW, int LW = 64 * CPL>
hipError_t launch_sim(const SimArgs& a, int n_blocks, hipStream_t stream) {
    using G = Geo<CPL, RPT, NW, LW>;
    static_assert(!G::SLAB, "slab variants are built in sim_slab.hip");
    if (a.prm.oer_max > 1.0 || a.prm.mitotic_death)   // the extended radiobiology instantiation
        hipLaunchKernelGGL((sim_kernel<CPL, RPT, NW, LW, true>), dim3(n_blocks), dim3(G::NT), 0, stream, a);
    else
        hipLaunchKernelGGL((sim_kernel<CPL, RPT, NW, LW, false>), dim3(n_blocks), dim3(G::NT), 0, stream, a);
    return hipGetLastError();
}

// chosen variant per lattice side 64, 96, .., 256 (index into SIM_VARIANTS):
// [0] any form, [1] resident only (-1: the side has no resident variant)
std::atomic<int> g_choice[2][N_SIDES] = {{{0}, {9}, {2}, {22}, {24}, {16}, {6}},
                                         {{0}, {9}, {2}, {-1}, {-1}, {-1}, {-1}}};

}  // namespace

bool sim_supported(int L) { return side_index(L) >= 0 && g_choice[1][side_index(L)].load() >= 0; }

hipError_t launch_variant(int v, const SimArgs& a, int n_blocks, hipStream_t stream) {
    if (n_blocks <= 0) return hipSuccess;
    switch (v) {
        case 0: return launch_sim<1, 4, 16>(a, n_blocks, stream);
        case 2: return launch_sim<2, 8, 16>(a, n_blocks, stream);
        case 3: return launch_sim<2, 16, 8>(a, n_blocks, stream);
        case 7: return launch_sim<1, 8, 8>(a, n_blocks, stream);
        case 8: return launch_sim<1, 16, 4>(a, n_blocks, stream);
        case 9: return launch_sim<2, 6, 16, 96>(a, n_blocks, stream);
        case 10: return launch_sim<2, 12, 8, 96>(a, n_blocks, stream);
        default:
            if (v >= 0 && v < N_SIM_VARIANTS && variant_is_slab(v)) return launch_slab_variant(v, a, n_blocks, stream);
            return hipErrorInvalidValue;
    }
}

int side_index(int L) { return (L % 32 == 0 && L >= 64 && L <= 256) ? L / 32 - 2 : -1; }

int variant_choice(int L, bool resident_only) {
    const int i = side_index(L);
    return i < 0 ? -1 : g_choice[resident_only ? 1 : 0][i].load();
}

int set_variant_choice(int L, int v) {
    const int i = side_index(L);
    if (i < 0 || v < 0 || v >= N_SIM_VARIANTS || SIM_VARIANTS[v].L != L) return -1;
    g_choice[0][i].store(v);
    if (!variant_is_slab(v)) g_choice[1][i].store(v);
    return 0;
}

hipError_t launch_simulation(const SimArgs& a, int L, int n_inst, hipStream_t stream) {
    if (n_inst <= 0) return hipSuccess;
    const int v = variant_choice(L, true);
    return v < 0 ? hipErrorInvalidValue : launch_variant(v, a, n_inst, stream);
}

hipError_t launch_fitness(const int32_t* live, int P, int R, float* fitness, hipStream_t stream) {
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(fitness_kernel, dim3((P + 255) / 256), dim3(256), 0, stream, live, P, R, fitness);
    return hipGetLastError();
}

hipError_t launch_philox_fill(const uint32_t* ctr, uint64_t seed, uint32_t* out, long long n,
                              hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const long long blocks = (n + 255) / 256;
    hipLaunchKernelGGL(philox_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, ctr,
                       (uint32_t)seed, (uint32_t)(seed >> 32), out, n);
    return hipGetLastError();
}

}  // namespace gga
