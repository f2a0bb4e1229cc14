// Device GA over the paper's sparse time-slot genome (Materials and Methods,
// "GA Resolution, constraints" and "Protocol Representation"; appendix "GA
// Operators: additional details"): a protocol is S slots of one hour, each
// holding a dose in quanta (0: none), under a maximal single dose, a cap on
// the total and a minimal interval between doses.
//
// One thread per child.  Its genome lives in LDS, slot j of thread t at byte
// j * SLOT_BLOCK + t, so the lanes of a wave touch consecutive bytes.  Child
// pair c shares its parents and crossover words; child ch of the pair takes
// its own mutation blocks.  Random words: the GA's Philox blocks
// (pair, generation, 0x47414741, sub):
//   subs 0 .. 2nb-1       parent selection (as the fixed-length GA)
//   sub 2nb               crossover: w0 against p_cross, w1, w2 cut points
//   subs 2nb+1 ..         uniform crossover mask, one block per 128 slots
//   B + 8 ch + m          mutation m of child ch, B = 2nb + 1 + ceil(S / 128):
//                         m = 0 swap, 1 and 2 split, 3 dose time, 4 dose value
// Guards after the mutations: clamp to the maximal dose, the interval guard
// (a dose too close to the previous kept one moves to the first later slot
// with no dose within g_min - 1 slots on either side, or is dropped), and the
// total guard (the largest dose, first among equals, loses a quantum while the
// total exceeds the cap), computed here in closed form as a water level.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ga_select.h"
#include "gga_device.h"
#include "gga_internal.h"
#include "slots.h"

namespace gga {
namespace {

constexpr int SLOT_BLOCK = 64;          // threads per workgroup (one wave)
constexpr int MUT_BLOCKS = 8;           // Philox blocks reserved per child for mutations

// One thread's genome in LDS.
struct Genome {
    uint8_t* p;
    __device__ int operator[](int j) const { return p[j * SLOT_BLOCK]; }
    __device__ void set(int j, int v) const { p[j * SLOT_BLOCK] = (uint8_t)v; }
};

__device__ int count_at_least(const Genome& v, int S, int least) {
    int n = 0;
    for (int j = 0; j < S; ++j) n += v[j] >= least;
    return n;
}

// Slot of the i-th entry (slot order, from 0) holding at least `least`; the
// caller guarantees i < count_at_least(v, S, least).
__device__ int nth_at_least(const Genome& v, int S, int i, int least) {
    for (int j = 0; j < S; ++j)
        if (v[j] >= least && i-- == 0) return j;
    return S - 1;
}

__device__ void guard_clamp(const Genome& v, int S, int dmax) {
    for (int j = 0; j < S; ++j)
        if (v[j] > dmax) v.set(j, dmax);
}

__device__ void guard_interval(const Genome& v, int S, int g) {
    int last = -1;                                   // slot of the last kept dose
    for (int s = 0; s < S; ++s) {
        const int d = v[s];
        if (d == 0) continue;
        if (last < 0 || s - last >= g) {
            last = s;
            continue;
        }
        v.set(s, 0);
        // every dose before s is kept and `last` is the latest of them; scan
        // forward with prev = latest dose before t, nxt = first dose at or after t
        int prev = last, nxt = s + 1;
        while (nxt < S && v[nxt] == 0) ++nxt;
        for (int t = s + 1; t < S; ++t) {
            if (t == nxt) {
                prev = t;
                ++nxt;
                while (nxt < S && v[nxt] == 0) ++nxt;
                continue;
            }
            if (t - prev >= g && (nxt >= S || nxt - t >= g)) {
                v.set(t, d);
                break;
            }
        }
    }
}

__device__ int sum_min(const Genome& v, int S, int L) {
    int s = 0;
    for (int j = 0; j < S; ++j) s += min(v[j], L);
    return s;
}

// Repeatedly lowering the largest dose (first among equals) by one quantum
// until the total is within the cap ends at the water level L, the largest
// with sum(min(v, L)) <= cap: doses above L become L, except the last
// e = cap - sum(min(v, L)) of them in slot order, which keep L + 1.
__device__ void guard_total(const Genome& v, int S, int cap) {
    int total = 0, vmax = 0;
    for (int j = 0; j < S; ++j) {
        total += v[j];
        vmax = max(vmax, v[j]);
    }
    if (total <= cap) return;
    int lo = 0, hi = vmax - 1;                       // sum_min(0) = 0 <= cap < sum_min(vmax)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sum_min(v, S, mid) <= cap) lo = mid;
        else hi = mid - 1;
    }
    int e = cap - sum_min(v, S, lo);
    for (int j = S - 1; j >= 0; --j) {
        if (v[j] <= lo) continue;
        v.set(j, e > 0 ? lo + 1 : lo);
        e -= e > 0;
    }
}

__device__ void guards(const Genome& v, int S, int g, int dmax, int cap) {
    guard_clamp(v, S, dmax);
    guard_interval(v, S, g);
    guard_total(v, S, cap);
}

// A part of a split dose goes to slot r, or on from r, cyclically, to the
// first slot where it fits under dmax; the emptied source slot s always does
// for a clamped genome.
__device__ void place_part(const Genome& v, int S, int part, int r, int s, int dmax) {
    for (int step = 0; step < S; ++step) {
        const int t = (r + step) % S;
        if (v[t] + part <= dmax) {
            v.set(t, v[t] + part);
            return;
        }
    }
    v.set(s, v[s] + part);
}

__device__ void mutate(const Genome& v, const SlotArgs& a, int c, uint32_t g, uint32_t sub0) {
    const int S = a.S, dmax = a.dmax;
    const uint32_t k0 = a.sel.seed_lo, k1 = a.sel.seed_hi, t_mut = a.sel.t_mut;
    if (a.mutation & GGA_SMUT_SWAP) {                // a dose and another slot exchange contents
        const Block4 b = ga_words(c, g, sub0 + 0, k0, k1);
        if (b.w0 < t_mut) {
            const int n = count_at_least(v, S, 1);
            if (n > 0 && S >= 2) {
                const int i = nth_at_least(v, S, pick_of(b.w1, n), 1);
                int j = pick_of(b.w2, S - 1);
                j += j >= i;
                const int x = v[i];
                v.set(i, v[j]);
                v.set(j, x);
            }
        }
    }
    if (a.mutation & GGA_SMUT_SPLIT) {               // a dose of >= 2 quanta splits in two
        const Block4 b = ga_words(c, g, sub0 + 1, k0, k1);
        if (b.w0 < t_mut) {
            const int n = count_at_least(v, S, 2);
            if (n > 0) {
                const int s = nth_at_least(v, S, pick_of(b.w1, n), 2);
                const int total = v[s];
                v.set(s, 0);
                const int part = 1 + pick_of(b.w2, total - 1);
                const uint32_t r2 = ga_words(c, g, sub0 + 2, k0, k1).w0;
                place_part(v, S, part, pick_of(b.w3, S), s, dmax);
                place_part(v, S, total - part, pick_of(r2, S), s, dmax);
            }
        }
    }
    if (a.mutation & GGA_SMUT_TIME) {                // a dose moves; what does not fit stays
        const Block4 b = ga_words(c, g, sub0 + 3, k0, k1);
        if (b.w0 < t_mut) {
            const int n = count_at_least(v, S, 1);
            if (n > 0) {
                const int s = nth_at_least(v, S, pick_of(b.w1, n), 1);
                const int t = pick_of(b.w2, S);
                if (t != s) {
                    const int m = max(0, min(v[s], dmax - v[t]));
                    v.set(t, v[t] + m);
                    v.set(s, v[s] - m);
                }
            }
        }
    }
    if (a.mutation & GGA_SMUT_VALUE) {               // a dose grows while the total is under the cap
        const Block4 b = ga_words(c, g, sub0 + 4, k0, k1);
        if (b.w0 < t_mut) {
            int n = 0, total = 0;
            for (int j = 0; j < S; ++j) {
                n += v[j] > 0;
                total += v[j];
            }
            if (n > 0 && total < a.cap_q) {
                const int s = nth_at_least(v, S, pick_of(b.w1, n), 1);
                const int h = min(dmax, v[s] + a.cap_q - total);
                if (h > v[s]) v.set(s, v[s] + 1 + pick_of(b.w2, h - v[s]));
            }
        }
    }
}

// Dynamic LDS of both genome kernels: S * SLOT_BLOCK bytes.
__global__ __launch_bounds__(SLOT_BLOCK) void slot_offspring_kernel(SlotArgs a) {
    extern __shared__ uint8_t lds[];
    const int row = blockIdx.x * SLOT_BLOCK + threadIdx.x;
    const int S = a.S, n_elite = a.sel.n_elite;
    if (row >= a.sel.n_out) return;
    if (row < n_elite) {                             // elites: copied unchanged
        const uint8_t* src = a.pop + (size_t)a.sel.order[row] * S;
        for (int j = 0; j < S; ++j) a.next[(size_t)row * S + j] = src[j];
        return;
    }
    const uint32_t g = (uint32_t)*a.sel.generation;
    const int c = (row - n_elite) >> 1, ch = (row - n_elite) & 1;
    const int nb = (selection_words(a.sel) + 3) / 4;
    const uint8_t* pa = a.pop + (size_t)select_parent(c, g, 0, a.sel) * S;
    const uint8_t* pb = a.pop + (size_t)select_parent(c, g, nb, a.sel) * S;
    if (ch == 1) {                                   // child 1 starts from parent b
        const uint8_t* t = pa;
        pa = pb;
        pb = t;
    }
    // crossover: slots in [x0, x1) come from the other parent; uniform uses the mask
    const Block4 bc = ga_words(c, g, (uint32_t)(2 * nb), a.sel.seed_lo, a.sel.seed_hi);
    const bool cross = bc.w0 < a.sel.t_cross && S > 1;
    int x0 = S, x1 = S;
    if (cross && (a.sel.crossover == GGA_X_ONE_POINT || a.sel.crossover == GGA_X_MIDDLE)) {
        int lo = 1, hi = S - 1;
        if (a.sel.crossover == GGA_X_MIDDLE) {
            lo = max(1, S / 4);
            hi = max(lo, min(S - 1, 3 * S / 4));
        }
        x0 = lo + pick_of(bc.w1, hi - lo + 1);
    } else if (cross && a.sel.crossover == GGA_X_TWO_POINT) {
        x0 = S / 4 + pick_of(bc.w1, S / 2 - S / 4 + 1);
        x1 = S / 2 + pick_of(bc.w2, 3 * S / 4 - S / 2 + 1);
    }
    const bool uniform = cross && a.sel.crossover == GGA_X_UNIFORM;
    const Genome v{lds + threadIdx.x};
    Block4 mask{0, 0, 0, 0};
    for (int j = 0; j < S; ++j) {
        bool other;
        if (uniform) {
            if ((j & 127) == 0)
                mask = ga_words(c, g, (uint32_t)(2 * nb + 1 + (j >> 7)), a.sel.seed_lo, a.sel.seed_hi);
            other = (word_of(mask, (j >> 5) & 3) >> (j & 31)) & 1u;
        } else {
            other = a.sel.crossover == GGA_X_TWO_POINT ? (j >= x0 && j < x1) : j >= x0;
        }
        v.set(j, other ? pb[j] : pa[j]);
    }
    const uint32_t sub0 = (uint32_t)(2 * nb + 1 + (S + 127) / 128 + MUT_BLOCKS * ch);
    mutate(v, a, c, g, sub0);
    guards(v, S, a.g_min, a.dmax, a.cap_q);
    for (int j = 0; j < S; ++j) a.next[(size_t)row * S + j] = (uint8_t)v[j];
}

// One thread per genome: the doses in slot order; delay_1 is the slot of the
// first dose, later delays the slot differences; at most K doses are taken.
__global__ __launch_bounds__(256) void slot_decode_kernel(const uint8_t* pop, int P, int S, int K, float quantum,
                                                          float* dose, int32_t* gap, int32_t* nfrac) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const uint8_t* v = pop + (size_t)p * S;
    int n = 0, prev = 0;
    for (int s = 0; s < S && n < K; ++s) {
        const int x = v[s];
        if (x == 0) continue;
        dose[(size_t)p * K + n] = (float)x * quantum;
        gap[(size_t)p * K + n] = s - prev;
        prev = s;
        ++n;
    }
    nfrac[p] = n;
    for (int j = n; j < K; ++j) {
        dose[(size_t)p * K + j] = 0.0f;
        gap[(size_t)p * K + j] = 0;
    }
}

// One thread per protocol: fraction j adds round(dose_j / quantum) quanta at
// slot delay_1 + .. + delay_j until a slot falls outside the window; then the
// guards.
__global__ __launch_bounds__(SLOT_BLOCK) void slot_encode_kernel(const float* dose, const int32_t* gap,
                                                                 const int32_t* nfrac, int P, int K, int S,
                                                                 float quantum, int g_min, int dmax, int cap_q,
                                                                 uint8_t* pop) {
    extern __shared__ uint8_t lds[];
    const int p = blockIdx.x * SLOT_BLOCK + threadIdx.x;
    if (p >= P) return;
    const Genome v{lds + threadIdx.x};
    for (int j = 0; j < S; ++j) v.set(j, 0);
    const int n = min(max(nfrac[p], 0), K);
    long long t = 0;
    for (int j = 0; j < n; ++j) {
        t += gap[(size_t)p * K + j];
        if (t < 0 || t >= S) break;
        const float x = dose[(size_t)p * K + j] / quantum;
        const int q = x > 0.0f ? (int)fminf(rintf(x), 255.0f) : 0;
        v.set((int)t, min(255, v[(int)t] + q));
    }
    guards(v, S, g_min, dmax, cap_q);
    for (int j = 0; j < S; ++j) pop[(size_t)p * S + j] = (uint8_t)v[j];
}

}  // namespace

hipError_t launch_slot_offspring(const SlotArgs& a, hipStream_t s) {
    if (a.S < 1 || a.S > SLOTS_MAX) return hipErrorInvalidValue;
    if (a.sel.n_out <= 0) return hipSuccess;
    hipLaunchKernelGGL(slot_offspring_kernel, dim3((a.sel.n_out + SLOT_BLOCK - 1) / SLOT_BLOCK), dim3(SLOT_BLOCK),
                       (size_t)a.S * SLOT_BLOCK, s, a);
    return hipGetLastError();
}

hipError_t launch_slot_decode(const uint8_t* pop, int P, int S, int K, float quantum, float* dose, int32_t* gap,
                              int32_t* nfrac, hipStream_t s) {
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(slot_decode_kernel, dim3((P + 255) / 256), dim3(256), 0, s, pop, P, S, K, quantum, dose, gap,
                       nfrac);
    return hipGetLastError();
}

hipError_t launch_slot_encode(const float* dose, const int32_t* gap, const int32_t* nfrac, int P, int K, int S,
                              float quantum, int g_min, int dmax, int cap_q, uint8_t* pop, hipStream_t s) {
    if (S < 1 || S > SLOTS_MAX) return hipErrorInvalidValue;
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(slot_encode_kernel, dim3((P + SLOT_BLOCK - 1) / SLOT_BLOCK), dim3(SLOT_BLOCK),
                       (size_t)S * SLOT_BLOCK, s, dose, gap, nfrac, P, K, S, quantum, g_min, dmax, cap_q, pop);
    return hipGetLastError();
}

}  // namespace gga
