// Device GA over the time-slot genome: kernel arguments and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gga_internal.h"

namespace gga {

constexpr int SLOTS_MAX = 256;

struct SlotArgs {
    GaArgs sel;                 // selection and crossover settings, ranks, fitness, generation counter
    int32_t S, g_min, dmax, cap_q, mutation;
    float quantum;
    const uint8_t* pop;         // [N][S]
    uint8_t* next;              // [n_out][S]
};

// Next population: rows 0 .. n_elite-1 the best members, the rest children.
hipError_t launch_slot_offspring(const SlotArgs& a, hipStream_t s);
// dose[P][K], gap[P][K], nfrac[P] of genomes pop[P][S].
hipError_t launch_slot_decode(const uint8_t* pop, int P, int S, int K, float quantum, float* dose, int32_t* gap,
                              int32_t* nfrac, hipStream_t s);
// Guarded genomes pop[P][S] of protocols (dose, gap, nfrac).
hipError_t launch_slot_encode(const float* dose, const int32_t* gap, const int32_t* nfrac, int P, int K, int S,
                              float quantum, int g_min, int dmax, int cap_q, uint8_t* pop, hipStream_t s);

}  // namespace gga
