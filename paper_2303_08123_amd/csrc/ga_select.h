// Parent selection of the device GAs (fixed-length genes and time slots):
// the Philox words of a child pair and the four selection rules of the
// paper's appendix on the GA operators ("Selection").  Included by the GA
// kernels' translation units only.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gga_device.h"
#include "gga_internal.h"

namespace gga {
namespace {

constexpr uint32_t GA_TAG = 0x47414741u;

__device__ __forceinline__ Block4 ga_words(int c, uint32_t g, uint32_t sub, uint32_t k0, uint32_t k1) {
    return philox10((uint32_t)c, g, GA_TAG, sub, k0, k1);
}

__device__ __forceinline__ uint32_t word_of(const Block4& b, int i) {
    return i == 0 ? b.w0 : i == 1 ? b.w1 : i == 2 ? b.w2 : b.w3;
}

// Word i of the selection words of one parent (blocks base .. base + nb - 1).
__device__ __forceinline__ uint32_t sel_word(int c, uint32_t g, int base, int i, const GaArgs& a) {
    return word_of(ga_words(c, g, (uint32_t)(base + i / 4), a.seed_lo, a.seed_hi), i & 3);
}

__device__ __forceinline__ int pick_of(uint32_t w, int n) { return (int)(((uint64_t)w * (uint32_t)n) >> 32); }

// One parent (an index into the population) by the configured selection.
#pragma clang fp contract(off)
__device__ int select_parent(int c, uint32_t g, int base, const GaArgs& a) {
    const int N = a.N, k = a.k;
    if (a.selection == GGA_SEL_TOURNAMENT) {
        int best = -1, best_pos = 0x7FFFFFFF;
        for (int i = 0; i < k; ++i) {
            const int pick = pick_of(sel_word(c, g, base, i, a), N);
            const int pos = a.position[pick];
            if (pos < best_pos) { best_pos = pos; best = pick; }
        }
        return best;
    }
    if (a.selection == GGA_SEL_RANK) {
        // k picks sorted by rank position (insertion sort), then the j-th best
        // is taken with probability q (1 - q)^j, the last with the rest
        int pos[64];
        for (int i = 0; i < k; ++i) {
            const int p = a.position[pick_of(sel_word(c, g, base, i, a), N)];
            int j = i;
            while (j > 0 && pos[j - 1] > p) { pos[j] = pos[j - 1]; --j; }
            pos[j] = p;
        }
        int take = k - 1;
        for (int j = 0; j < k - 1; ++j)
            if (sel_word(c, g, base, k + j, a) < a.t_q) { take = j; break; }
        return a.order[pos[take]];
    }
    const uint32_t w0 = sel_word(c, g, base, 0, a);
    if (a.selection == GGA_SEL_TRUNCATION) return a.order[pick_of(w0, a.trunc_m)];
    // roulette over max(base - fitness, 0), sums in index order in float64
    double total = 0.0;
    for (int i = 0; i < N; ++i) {
        const float f = a.fitness[i];
        total += isnan(f) ? 0.0 : fmax(a.roulette_base - (double)f, 0.0);
    }
    if (!(total > 0.0)) return pick_of(w0, N);
    const double u = ((double)w0 * total) * 2.3283064365386963e-10;   // w0 total / 2^32
    double run = 0.0;
    int last = 0;
    for (int i = 0; i < N; ++i) {
        const float f = a.fitness[i];
        const double v = isnan(f) ? 0.0 : fmax(a.roulette_base - (double)f, 0.0);
        run += v;
        if (v > 0.0) last = i;
        if (run > u) return i;
    }
    return last;
}
#pragma clang fp contract(on)

__device__ __forceinline__ int selection_words(const GaArgs& a) {
    return a.selection == GGA_SEL_TOURNAMENT ? a.k : a.selection == GGA_SEL_RANK ? 2 * a.k - 1 : 1;
}

}  // namespace
}  // namespace gga
