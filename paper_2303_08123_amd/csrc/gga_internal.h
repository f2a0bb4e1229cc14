// Library-internal interface between the host ABI code and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gga.h"

namespace gga {

enum : int { MODE_LOAD = 1, MODE_STORE = 2 };

// Arguments of one simulation launch (passed by value as the kernel argument).
struct SimArgs {
    gga_params prm;
    const float* dose;      // [P][K]
    const int32_t* gap;     // [P][K]
    const int32_t* nfrac;   // [P]
    int32_t K, R, substeps, n0, nsteps, mode;
    uint32_t seed_lo, seed_hi;
    double dose_cap;
    float* fields;          // [P*R][3][L][L] when mode has LOAD or STORE
    uint16_t* cells;        // [P*R][L][L]
    int32_t* live;          // [P*R] or null
    int32_t* traj;          // [P*R][nsteps] or null
};

bool sim_supported(int L);
hipError_t launch_simulation(const SimArgs& a, int L, int n_inst, hipStream_t stream);
hipError_t launch_fitness(const int32_t* live, int P, int R, float* fitness, hipStream_t stream);
hipError_t launch_philox_fill(const uint32_t* ctr, uint64_t seed, uint32_t* out, long long n,
                              hipStream_t stream);

struct PopArgs {
    int32_t n_dose, n_gap, kmin, kmax, cap_q, K, P;
    float quantum;
    uint32_t seed_lo, seed_hi;
    int32_t dose_q[GGA_ALPHABET_MAX];
    int32_t gaps[GGA_ALPHABET_MAX];
    float* dose;
    int32_t* gap;
    int32_t* nfrac;
};
constexpr int POP_TABLE_MAX = 8192;   // (kmax + 1) * (cap_q + 1) doubles in LDS
hipError_t launch_population(const PopArgs& a, hipStream_t stream);

}  // namespace gga
