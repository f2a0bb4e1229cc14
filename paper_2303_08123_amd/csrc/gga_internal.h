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
    // When set, the Philox key is seed + g * 0x9E3779B97F4A7C15 (mod 2^64) with
    // g read from this device counter (replayed GA generations).
    const int32_t* generation;
    uint64_t seed;
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

struct GaArgs {
    int32_t N, K, n_elite, k, n_dose, n_gap, cap_q;
    uint32_t t_cross, t_mut, seed_lo, seed_hi;
    float quantum;
    int32_t dose_q[GGA_ALPHABET_MAX];
    int32_t gaps[GGA_ALPHABET_MAX];
    const float* dose;
    const int32_t* gap;
    const int32_t* order;
    const int32_t* position;
    const int32_t* generation;
    float* next_dose;
    int32_t* next_gap;
};
hipError_t launch_rank(const float* fitness, int N, int32_t* order, int32_t* position, hipStream_t s);
hipError_t launch_history(const float* fitness, int N, const int32_t* order, const int32_t* generation,
                          float* hist, int hist_cap, hipStream_t s);
hipError_t launch_offspring(const GaArgs& a, hipStream_t s);
hipError_t launch_counter(int32_t* generation, int32_t value, int32_t add, hipStream_t s);

}  // namespace gga
