// Library-internal interface between the host ABI code and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gga.h"

namespace gga {

enum : int { MODE_LOAD = 1, MODE_STORE = 2 };

// One positive-dose fraction of the slab form's event table (16 bytes).
struct EventFraction {
    float dose;
    int32_t pad;
    double prior;           // unrepaired dose of the earlier fractions (incomplete repair)
};

// Arguments of one simulation launch (passed by value as the kernel argument).
struct SimArgs {
    gga_params prm;
    const float* dose;      // [P][K]
    const int32_t* gap;     // [P][K]
    const int32_t* nfrac;   // [P]
    int32_t K, R, substeps, n0, nsteps, mode;
    int32_t half;           // delays count half-hours (GGA_SIM_HALF_HOUR)
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
    // Uneven batches.  Resident form: instance of block b = inst_list[b] (or b),
    // steps = horizon[p] (or nsteps).  Slab form: list position k and slab s of
    // block b (XCD-grouped, see the kernel), instance inst_list[k], one step n0
    // from fields/cells (state row k) to
    // fields_out/cells_out, the event table below instead of decoding the
    // protocol, and the live count added into live[inst] at step horizon[p] - 1.
    const int32_t* inst_list;
    const int32_t* horizon;   // [P]
    float* fields_out;
    uint16_t* cells_out;
    int32_t n_slabs;
    int32_t n_active;         // slab form: list positions 0 .. n_active-1 run this launch
    int32_t slab_ys[16], slab_i0[16], slab_i1[16];   // first lattice row; own rows [i0, i1) of the slab
    const int32_t* ev_valid;  // [P]
    const int32_t* ev_count;  // [P]
    const int32_t* ev_step;   // [P][K] times of the positive-dose fractions in half-hours, in order
    const EventFraction* ev_frac;   // [P][K] dose and unrepaired dose of each of those fractions
    int32_t count_at;         // slab form without horizon[]: the step whose end is counted (and the
                              // row length of traj, which then receives every slab's count per step)
    int32_t lib_n;            // resident form with MODE_LOAD: replica r loads state r mod lib_n (0: its own)
    // Teams (slab form over whole horizons): per slab the own rows it publishes
    // for its neighbours, [i0, exA) and [exB, i1); per list position and slab
    // the published step count; the bounded wait's spin count (< 0: every wait fails)
    int32_t slab_exA[16], slab_exB[16];
    int32_t* team_flags;      // [n_active][n_slabs], zero before the launch
    int32_t spin_limit;
};
constexpr int MAX_SLABS = 16;

// Kernel variants: lattice side L, columns per lane, rows per thread, waves;
// RR = rpt * nw rows per workgroup (slab form when RR < L); row pitch on the
// CU 64 * cpl >= L.  Sides 64, 96, .., 256 (N_SIDES of them).
struct SimVariant {
    int L, cpl, rpt, nw;
    const char* name;
};
constexpr SimVariant SIM_VARIANTS[] = {
    {64, 1, 4, 16, "L64 resident 4x1 x16 waves"},
    {64, 1, 2, 16, "L64 slabs of 32 rows, 2x1 x16 waves"},
    {128, 2, 8, 16, "L128 resident 8x2 x16 waves"},
    {128, 2, 16, 8, "L128 resident 16x2 x8 waves"},
    {128, 2, 4, 16, "L128 slabs of 64 rows, 4x2 x16 waves"},
    {256, 4, 4, 16, "L256 slabs of 64 rows, 4x4 x16 waves"},
    {256, 4, 8, 8, "L256 slabs of 64 rows, 8x4 x8 waves"},
    {64, 1, 8, 8, "L64 resident 8x1 x8 waves"},
    {64, 1, 16, 4, "L64 resident 16x1 x4 waves"},
    // sides below the row pitch 64 * cpl: the lanes past the lattice hold padding
    {96, 2, 6, 16, "L96 resident 6x2 x16 waves (48 of 64 lanes)"},
    {96, 2, 12, 8, "L96 resident 12x2 x8 waves (48 of 64 lanes)"},
    {160, 4, 4, 16, "L160 slabs of 64 rows, 4x4 x16 waves (40 of 64 lanes)"},
    {160, 4, 8, 8, "L160 slabs of 64 rows, 8x4 x8 waves (40 of 64 lanes)"},
    {192, 4, 4, 16, "L192 slabs of 64 rows, 4x4 x16 waves (48 of 64 lanes)"},
    {192, 4, 8, 8, "L192 slabs of 64 rows, 8x4 x8 waves (48 of 64 lanes)"},
    {224, 4, 4, 16, "L224 slabs of 64 rows, 4x4 x16 waves (56 of 64 lanes)"},
    {224, 4, 8, 8, "L224 slabs of 64 rows, 8x4 x8 waves (56 of 64 lanes)"},
    {96, 2, 4, 16, "L96 slabs of 64 rows, 4x2 x16 waves (48 of 64 lanes)"},
    // three columns per lane: 192 columns, no padding at 192, 160 of 192 at 160
    {160, 3, 4, 16, "L160 slabs of 64 rows, 4x3 x16 waves (160 of 192 columns)"},
    {160, 3, 8, 8, "L160 slabs of 64 rows, 8x3 x8 waves (160 of 192 columns)"},
    {192, 3, 4, 16, "L192 slabs of 64 rows, 4x3 x16 waves"},
    {192, 3, 8, 8, "L192 slabs of 64 rows, 8x3 x8 waves"},
    // taller slabs (fewer of them per instance, so less halo recomputed)
    {160, 3, 9, 8, "L160 slabs of 72 rows, 9x3 x8 waves (160 of 192 columns)"},
    {192, 3, 9, 8, "L192 slabs of 72 rows, 9x3 x8 waves"},
    {192, 3, 10, 8, "L192 slabs of 80 rows, 10x3 x8 waves"},
};
constexpr int N_SIM_VARIANTS = sizeof(SIM_VARIANTS) / sizeof(SIM_VARIANTS[0]);
constexpr bool variant_is_slab(int v) { return SIM_VARIANTS[v].rpt * SIM_VARIANTS[v].nw < SIM_VARIANTS[v].L; }

// GGA_E_HIP for e, kept as the thread's last HIP error (gga_last_hip_error)
int hip_error(hipError_t e);
// gga_simulate's checks and work, for the entry points that share them
int simulate_checked(const gga_params* params, const gga_sim_cfg* cfg, const float* dose_d, const int32_t* gap_h_d,
                     const int32_t* nfrac_d, int32_t P, int32_t K, void* ws_d, size_t ws_bytes, int32_t* live_d,
                     float* fitness_d, int32_t* traj_d, hipStream_t stream);

constexpr int N_SIDES = 7;
// index of lattice side L in 64, 96, .., 256, or -1
int side_index(int L);
// sides with a resident variant (gga_simulate's path)
bool sim_supported(int L);
// resident launch with the variant chosen for L (gga_simulate's path)
hipError_t launch_simulation(const SimArgs& a, int L, int n_inst, hipStream_t stream);
// launch variant v over n_blocks workgroups (slab form: n_blocks = slab_blocks(n_active, n_slabs))
inline int slab_blocks(int n_active, int n_slabs) { return ((n_active + 7) / 8) * 8 * n_slabs; }
hipError_t launch_variant(int v, const SimArgs& a, int n_blocks, hipStream_t stream);
hipError_t launch_slab_variant(int v, const SimArgs& a, int n_blocks, hipStream_t stream);
// team form of slab variant v (a cooperative launch of n_blocks workgroups; the
// slab mapping of the kernel with n_active teams); n_blocks = 0 only reports in
// *capacity how many workgroups of it the device holds at once
hipError_t launch_team_variant(int v, const SimArgs& a, int n_blocks, int* capacity, hipStream_t stream);
// instances per team launch at most (exchange buffers are sized for this many)
constexpr int TEAM_MAX = 128;
// process-wide variant choice per lattice side: resident (gga_simulate) and any (uneven batches)
int variant_choice(int L, bool resident_only);
int set_variant_choice(int L, int v);
// event table of P protocols for the slab form (validity as the resident kernel decides it)
hipError_t launch_event_table(const SimArgs& a, int P, int32_t* valid, int32_t* count, int32_t* step,
                              EventFraction* frac, hipStream_t stream);
// live[inst] = 0 (-1 for invalid protocols) for instances inst_list[0 .. n-1] (or 0 .. n-1)
hipError_t launch_slab_live(const SimArgs& a, int n, hipStream_t stream);
// initial state of the slab-form instances inst_list[0 .. n-1] into state rows 0 .. n-1, live
// counts set to 0 (-1 for invalid protocols; the initial count when horizon is 0)
hipError_t launch_slab_init(const SimArgs& a, int L, int n, float* fields, uint16_t* cells, hipStream_t stream);
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
    int32_t n_out;                  // children written: slots n_elite .. n_out-1 (n_out = N for a generation)
    uint32_t t_cross, t_mut, seed_lo, seed_hi;
    int32_t selection, crossover, mutation, trunc_m;   // operators (GGA_SEL_*, GGA_X_*, GGA_MUT_* bits)
    uint32_t t_q;
    double roulette_base;
    const float* fitness;           // [N], read by roulette selection
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
// Per-generation record of the best protocol: best_dose/best_gap row g = genes
// of the best row of dose/gap (K per row); inactive when best_dose is null.
struct Archive {
    const float* dose;
    const int32_t* gap;
    int K;
    float* best_dose;
    int32_t* best_gap;
};
hipError_t launch_history(const float* fitness, int N, const int32_t* order, const int32_t* generation,
                          float* hist, int hist_cap, const Archive& arc, hipStream_t s);
hipError_t launch_offspring(const GaArgs& a, hipStream_t s);
hipError_t launch_counter(int32_t* generation, int32_t value, int32_t add, hipStream_t s);
// *dst = *src + add
hipError_t launch_counter_copy(int32_t* dst, const int32_t* src, int32_t add, hipStream_t s);
hipError_t launch_gather(const float* sd, const int32_t* sg, const float* sf, const int32_t* idx, int n, int K,
                         float* dd, int32_t* dg, float* df, hipStream_t s);
hipError_t launch_random_keys(int n, const int32_t* generation, uint64_t seed, float* key, hipStream_t s);
hipError_t launch_fill(int32_t* p, int n, int32_t v, hipStream_t s);
// p[i] = i for i < n
hipError_t launch_iota(int32_t* p, int n, hipStream_t s);

}  // namespace gga
