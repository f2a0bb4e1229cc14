/*
 * gga.h - C ABI of the MI355X (gfx950) lattice tumour / irradiation simulator.
 *
 * The calls follow the paper's statement of the search problem (Results,
 * "Defining the search problem"): a protocol is a sequence of k (dose, delay)
 * pairs whose first delay counts from the start of the simulation, the total
 * dose is capped, and a protocol's fitness comes from the number of occupied
 * lattice sites at the end of the simulated period, averaged over replicate
 * simulations (Materials and Methods, "The fitness function", equation
 * final_fit_fun).  A caller creates a population of protocols, simulates each
 * one R times and reads back the fitness.
 *
 * Conventions for every call:
 *   - return GGA_OK (0) on success or a negative GGA_E_* code; never abort and
 *     never throw across the ABI;
 *   - pointers named *_d are device pointers (hipMalloc'ed or torch tensors);
 *     the caller owns all memory and no call allocates or frees any;
 *   - stream-ordered calls enqueue on `stream` and return; outputs are valid
 *     once the stream has completed the work.  No call synchronises a stream;
 *   - arrays are dense and row-major, shapes given in brackets;
 *   - identical inputs give bit-identical outputs on every run.
 *
 * Cell words (uint16): bits 0-1 state (0 EMPTY, 1 PROLIF, 2 QUIESC, 3 DEAD),
 * bits 2-9 age in hours (saturating at 255), bit 14 the mark of a lethally hit
 * cell awaiting mitotic death (gga_params.mitotic_death); EMPTY sites hold 0.
 * Field state (float32): [instance][3][L][L], planes oxygen, glucose, acidity,
 * in normalised units.  Instance i = p * R + r (protocol p, replica r).
 */
#ifndef GGA_H
#define GGA_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GGA_ABI_VERSION 2

/* Error codes. */
#define GGA_OK 0
#define GGA_E_ARG (-1)          /* null pointer, negative size, size overflow   */
#define GGA_E_ABI (-2)          /* struct_size does not match this library      */
#define GGA_E_UNSUPPORTED (-3)  /* no kernel for this lattice side / sub-steps  */
#define GGA_E_HIP (-4)          /* HIP runtime error; see gga_last_hip_error()  */
#define GGA_E_PARAM (-5)        /* model constant out of range (e.g. lambda)    */
#define GGA_E_ALPHABET (-6)     /* alphabet admits no protocol / too large      */
#define GGA_E_SCRATCH (-7)      /* batch exceeds gga_simulate_noalloc's scratch */

/* Per-protocol status written by gga_validate (and used by gga_simulate). */
#define GGA_PROTO_OK 0
#define GGA_PROTO_NFRAC 1       /* nfrac < 0 or nfrac > K                       */
#define GGA_PROTO_DOSE 2        /* a used dose is negative or not finite        */
#define GGA_PROTO_CAP 3         /* total dose > dose_cap + 1e-6 Gy              */
#define GGA_PROTO_GAP 4         /* delay_1 < 0, or delay_j < 1 h for j >= 2     */

/* Model constants (the paper defers the model's equations to earlier work;
 * these are the synthetic model's inputs).  Set struct_size =
 * sizeof(gga_params). */
typedef struct gga_params {
    uint32_t struct_size;
    float lambda[3];        /* FTCS numbers D dtau / h^2 for O, G, H; each in [0, 1/4] */
    float kappa[3];         /* O and G uptake, H production per sub-step at activity 1;
                               all > 0, kappa[1] / kappa[0] and kappa[2] / kappa[0]
                               in [1e-12, 1e12]                                        */
    float ghost[3];         /* Dirichlet values outside the lattice                      */
    float init[3];          /* initial uniform field values                              */
    float activity[4];      /* activity of EMPTY, PROLIF, QUIESC, DEAD sites             */
    float theta_O_quiesce, theta_G_quiesce;              /* quiescent below these */
    float theta_O_death, theta_G_death, theta_H_death;   /* necrosis beyond these */
    int32_t T_min;          /* minimum age (h) before a cell may divide                  */
    int32_t T_lys;          /* hours from death to lysis                                  */
    int32_t A0;             /* initial ages uniform on 0 .. A0-1                          */
    int32_t seed_radius;    /* initial disc (x-c)^2 + (y-c)^2 <= r^2, c = L/2             */
    int32_t class_age[2];   /* sensitivity classes: age < a0, a0 <= age < a1, age >= a1   */
    double P_div;           /* hourly division probability once age >= T_min             */
    double alpha, beta;     /* linear-quadratic survival exp(-alpha x - beta x^2)        */
    double m[4];            /* x = m[class] * dose; classes young, mid, old, quiescent   */
    double repair_half_time;/* hours, finite, >= 0.  0: sublethal damage is repaired
                               between fractions (plain law per fraction).  > 0:
                               incomplete repair: fraction j survives with
                               exp(-alpha x - beta x (x + 2 y)), y = m D_j,
                               D_j = sum over earlier fractions i of
                               d_i 2^(-(t_j - t_i) / repair_half_time)          */
    double oer_max;         /* oxygen effect: finite, >= 1; 1 turns it off.  > 1: a cell's
                               dose d and unrepaired dose D are scaled by
                               OMF = (oer_max o + oer_k) / (oer_max (o + oer_k)), o the
                               midpoint of the oxygen bin of the site's current O
                               (GGA_OER_BINS bins of O / ghost[0] over [0, 1], the
                               last also above 1; ghost[0] > 0 required)               */
    double oer_k;           /* oxygen level of half the effect, same units as O; > 0  */
    int32_t mitotic_death;  /* 0: a lethally hit cell dies at once.  1: it is marked (bit
                               14 of its cell word) and dies when it next becomes ready
                               to divide (age >= T_min and its draw below P_div), free
                               neighbours or not; marked cells never divide          */
    int32_t reserved;       /* 0                                                      */
} gga_params;
#define GGA_OER_BINS 16

/*
 * Fill *out from a model file: a flat JSON object whose values are numbers or
 * arrays of numbers, keys lambda[3], kappa[3], ghost[3], init_fields[3],
 * activity[4], theta_O_quiesce, theta_G_quiesce, theta_O_death,
 * theta_G_death, theta_H_death, T_min, T_lys, A0, seed_radius (integers),
 * class_age[2] (integers), P_div, alpha, beta, m[4], and optionally
 * repair_half_time (default 0), oer_max (default 1), oer_k (default
 * 0.05) and mitotic_death (default 0) (the package's
 * data/model_default.json).  Other keys are ignored.  out->struct_size must
 * be sizeof(gga_params) (GGA_E_ABI otherwise); *out is written only on
 * success.  Host only, no device work.  Errors: GGA_E_ARG (null pointer,
 * unreadable file or malformed JSON), GGA_E_ABI, GGA_E_PARAM (a key missing,
 * of the wrong length or not integral where an integer is needed, or values
 * the simulation calls would refuse).
 */
int gga_params_from_json(const char* path, gga_params* out);

/* One simulation batch.  Set struct_size = sizeof(gga_sim_cfg).
 * GGA_SIM_HALF_HOUR: protocol delays count 30-minute units, the paper's slot
 * length (Materials and Methods, "GA Resolution, constraints"); the model
 * still steps in hours.  A fraction at an odd half-hour 2n + 1 is applied in
 * step n after substeps / 2 of its diffusion sub-steps (its survival words
 * from the Philox block of step word n | 2^31), and the reaction term is
 * rebuilt from the surviving cells for the rest of the hour.  Horizons are at
 * most 2^30 steps. */
#define GGA_SIM_HALF_HOUR 1u
typedef struct gga_sim_cfg {
    uint32_t struct_size;
    int32_t L;              /* lattice side: 64, 96, .., 256 (multiples of 32);
                               resident (state on one CU): 64, 96, 128; the other
                               sides run as slabs through device memory        */
    int32_t horizon;        /* steps (model hours) simulated by gga_simulate     */
    int32_t substeps;       /* diffusion sub-steps per step, 1 .. 64             */
    int32_t R;              /* replicas per protocol, >= 1                       */
    uint32_t flags;         /* 0 or GGA_SIM_HALF_HOUR                            */
    uint64_t seed;          /* Philox key (lo, hi words)                         */
    double dose_cap;        /* total-dose cap in Gy                              */
} gga_sim_cfg;

/* Alphabet for gga_population_random.  Set struct_size = sizeof(gga_alphabet). */
#define GGA_ALPHABET_MAX 64
#define GGA_KMAX 64
typedef struct gga_alphabet {
    uint32_t struct_size;
    int32_t n_dose;                      /* number of allowed doses, 1 .. 64        */
    int32_t n_gap;                       /* number of allowed delays, 1 .. 64       */
    int32_t kmin, kmax;                  /* fraction-count range, 0 <= kmin <= kmax */
    float dose_quantum;                  /* Gy per dose unit                        */
    float cap;                           /* total-dose cap in Gy                    */
    int32_t dose_q[GGA_ALPHABET_MAX];    /* allowed doses in quanta, increasing, >0 */
    int32_t gaps[GGA_ALPHABET_MAX];      /* allowed delays in hours, >= 1           */
} gga_alphabet;

/* ABI version (GGA_ABI_VERSION). */
int gga_version(void);

/* Static description of an error code; never NULL. */
const char* gga_strerror(int code);

/* hipError_t of the last call on this thread that returned GGA_E_HIP. */
int gga_last_hip_error(void);

/*
 * Validate protocols on the host (Results, "Defining the search problem": a
 * protocol is k (dose, delay) pairs, the first delay counted from the start,
 * under a cap on the total dose; Materials and Methods, "GA Resolution,
 * constraints").  dose[P][K], gap_h[P][K], nfrac[P] and
 * status[P] are HOST pointers.  Writes one GGA_PROTO_* code per protocol; the
 * rules are checked in the order nfrac, then per fraction dose and delay, then
 * the cap (total summed in double in index order).  Synchronous.
 * Errors: GGA_E_ARG, GGA_E_ABI.
 */
int gga_validate(const gga_sim_cfg* cfg, const float* dose, const int32_t* gap_h,
                 const int32_t* nfrac, int32_t P, int32_t K, int32_t* status);

/*
 * Create a population (Results, "Defining the search problem": the feasible
 * protocols are the dose sequences under the total-dose cap with delays from
 * the allowed set; Materials and Methods, "The Main GA Loop": a GA run starts
 * from a random population): P random protocols drawn on the device.  For protocol
 * p the fraction count k is uniform on kmin..kmax; the k doses are uniform
 * over all length-k sequences from the alphabet whose total is within the cap
 * (sequential sampling from a counting table, equal in law to rejection
 * sampling); the k delays are independent and uniform over the allowed delays.
 * Random words come from Philox4x32-10 blocks (p, i, 0x504F5055, 0) keyed by
 * `seed`, i = position, i = 0xFFFFFFFF for the fraction count.
 * Outputs dose_d[P][K] (Gy), gap_h_d[P][K], nfrac_d[P]; entries past nfrac
 * are 0.  Requires kmax <= K <= GGA_KMAX.
 * Errors: GGA_E_ARG, GGA_E_ABI, GGA_E_ALPHABET, GGA_E_HIP.
 */
int gga_population_random(const gga_alphabet* a, int32_t P, int32_t K, uint64_t seed,
                          float* dose_d, int32_t* gap_h_d, int32_t* nfrac_d,
                          hipStream_t stream);

/*
 * Device workspace gga_simulate needs for P protocols (any K <= GGA_KMAX) of
 * cfg->R replicas on a cfg->L lattice: 0 for the resident sides 64, 96 and
 * 128, whose state stays on the compute unit; for the other sides the event
 * table and two state buffers of P * R instances ((12 + 2) L^2 bytes each,
 * 256-byte aligned blocks).  0 also for invalid arguments (a NULL or
 * mismatched cfg, P < 0, an unsupported side).  Host only.
 */
size_t gga_workspace_bytes(const gga_sim_cfg* cfg, int32_t P);

/*
 * Simulate and score (Materials and Methods, "The fitness function &
 * experimental setup": a protocol's fitness is read from the number of
 * occupied sites at the end of the simulated period, averaged over repeated
 * simulations, equation final_fit_fun; "GPU implementation": many simulations
 * of a batch run at once).  Runs every (protocol, replica) instance from the
 * initial state for cfg->horizon steps on the device: fraction j of protocol
 * p (dose > 0, time t_j = delay_1 + .. + delay_j < horizon) is applied at the
 * start of step t_j; each step diffuses the fields cfg->substeps times and then
 * updates the cells.
 *   dose_d[P][K], gap_h_d[P][K], nfrac_d[P]  protocols (device)
 *   ws_d, ws_bytes   device workspace of at least gga_workspace_bytes(cfg, P)
 *                    bytes, 16-byte aligned, contents ignored; may be NULL
 *                    with 0 bytes when that is 0 (resident sides)
 *   live_d[P][R]     live (PROLIF + QUIESC) sites after the last step
 *   fitness_d[P]     mean of live over replicas (the fitness to minimise; the
 *                    paper's score is L*L - fitness)
 *   traj_d[P][R][horizon]  live count after every step, or NULL
 * Resident sides run one launch for the whole horizon; the other sides run
 * over slabs of rows, as teams of co-resident slab workgroups that keep their
 * rows on the compute units for the whole horizon (or, with the team form
 * switched off by gga_set_team_options, one launch per step); results are
 * bit-identical to a resident run of the same lattice (see the kernel
 * variants below).
 * A protocol that breaks a GGA_PROTO_* rule is not simulated: its live entries
 * are -1 and its fitness is NaN.
 * Errors: GGA_E_ARG (also a missing or small workspace), GGA_E_ABI,
 * GGA_E_UNSUPPORTED (side not a multiple of 32 in 64 .. 256, sub-steps above
 * what the slab plan allows), GGA_E_PARAM, GGA_E_HIP.
 */
int gga_simulate(const gga_params* params, const gga_sim_cfg* cfg,
                 const float* dose_d, const int32_t* gap_h_d, const int32_t* nfrac_d,
                 int32_t P, int32_t K, void* ws_d, size_t ws_bytes,
                 int32_t* live_d, float* fitness_d, int32_t* traj_d, hipStream_t stream);

/*
 * gga_simulate for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments without the workspace, and the same kernels and results.
 * The slab-form sides use a fixed scratch array of GGA_NOALLOC_SCRATCH_BYTES
 * in device memory instead, one per GPU the library runs on, held until the
 * process ends; batches whose gga_workspace_bytes(cfg, P) exceeds it return
 * GGA_E_SCRATCH before any work is enqueued (at most 36 instances at
 * 256 x 256, 47 at 224, 64 at 192, 93 at 160, one replica each).  Resident sides use no scratch.  The call allocates and
 * frees nothing (its first call on a device looks up that device's scratch
 * address).  Calls share their GPU's scratch: two calls whose work overlaps
 * on one GPU (other streams, other host threads) race; calls ordered on one
 * stream do not.  Errors: as gga_simulate, and GGA_E_SCRATCH.
 */
#define GGA_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int gga_simulate_noalloc(const gga_params* params, const gga_sim_cfg* cfg,
                         const float* dose_d, const int32_t* gap_h_d, const int32_t* nfrac_d,
                         int32_t P, int32_t K, int32_t* live_d, float* fitness_d, int32_t* traj_d,
                         hipStream_t stream);

/*
 * Write the initial state of P * cfg->R instances: fields_d[P*R][3][L][L]
 * (float32) and cells_d[P*R][L][L] (uint16 words).  Same kernel as
 * gga_simulate, run for zero steps; resident sides (64, 96, 128) only.
 *
 * State buffers (here, gga_state_run, the tumour library and the variant
 * runs) hold each field f in the kernel's units c^ = (c - ghost[f]) / rho_f,
 * rho_f = kappa'_f / kappa'_O with kappa' = (-kappa[0], -kappa[1], +kappa[2]):
 * shifted by its boundary value and scaled so that all three fields share one
 * reaction term.  Physical values are c = rho_f c^ + ghost[f].
 * Errors: as gga_simulate.
 */
int gga_state_init(const gga_params* params, const gga_sim_cfg* cfg, int32_t P,
                   float* fields_d, uint16_t* cells_d, hipStream_t stream);

/*
 * Advance the given states of P * cfg->R instances by `nsteps` steps, from
 * step n0 (events and random words are those of steps n0 .. n0+nsteps-1), in
 * place.  live_d[P][R] receives the final live counts and traj_d (or NULL)
 * [P][R][nsteps] the count after every step.  Invalid protocols leave their
 * states untouched and get live = -1.  Same kernel as gga_simulate; a test
 * hook for stepping from a known state.
 * Errors: as gga_simulate.
 */
int gga_state_run(const gga_params* params, const gga_sim_cfg* cfg,
                  const float* dose_d, const int32_t* gap_h_d, const int32_t* nfrac_d,
                  int32_t P, int32_t K, int32_t n0, int32_t nsteps,
                  float* fields_d, uint16_t* cells_d, int32_t* live_d, int32_t* traj_d,
                  hipStream_t stream);

/* GA settings.  Set struct_size = sizeof(gga_ga_cfg). */
/* Operator variants (the paper's appendix on the GA operators describes
 * simple, roulette and rank-based tournament selection, one-point (cut between
 * 25 % and 75 %), two-point and uniform crossover, and swap and dose-raising
 * mutations among others; zero selects the defaults). */
#define GGA_SEL_TOURNAMENT 0    /* best of k uniform picks                                 */
#define GGA_SEL_RANK 1          /* j-th best of k picks with probability q (1 - q)^j       */
#define GGA_SEL_ROULETTE 2      /* proportional to max(roulette_base - fitness, 0)         */
#define GGA_SEL_TRUNCATION 3    /* uniform over the best floor(trunc_frac N)               */
#define GGA_X_ONE_POINT 0       /* cut uniform on 1 .. K-1                                  */
#define GGA_X_MIDDLE 1          /* cut uniform on max(1, K/4) .. min(K-1, 3K/4)             */
#define GGA_X_TWO_POINT 2       /* genes [c1, c2) exchanged, c1 in K/4..K/2, c2 in K/2..3K/4 */
#define GGA_X_UNIFORM 3         /* each gene exchanged with probability 1/2                 */
#define GGA_MUT_GENE 1          /* per gene: dose and delay redrawn with probability p_mut  */
#define GGA_MUT_SWAP 2          /* per child: two doses exchanged with probability p_mut    */
#define GGA_MUT_RAISE 4         /* per child: one dose raised (if under the cap), p_mut     */
typedef struct gga_ga_cfg {
    uint32_t struct_size;
    int32_t n_elite;        /* best protocols copied unchanged, 0 .. N            */
    int32_t tournament_k;   /* picks per tournament (GGA_SEL_TOURNAMENT, _RANK), 1 .. 64 */
    double p_cross;         /* crossover probability, [0, 1]                       */
    double p_mut;           /* mutation probability (see GGA_MUT_*), [0, 1]        */
    uint64_t seed;          /* key of the GA's Philox blocks                        */
    int32_t selection;      /* GGA_SEL_*                                           */
    int32_t crossover;      /* GGA_X_*                                             */
    int32_t mutation;       /* GGA_MUT_* bits applied in the order gene, swap, raise; 0 = GGA_MUT_GENE */
    int32_t reserved;       /* 0                                                   */
    double q;               /* GGA_SEL_RANK: (0, 1]                                */
    double trunc_frac;      /* GGA_SEL_TRUNCATION: (0, 1]                          */
    double roulette_base;   /* GGA_SEL_ROULETTE: finite                            */
} gga_ga_cfg;

/*
 * One GA breeding step over fixed-length protocols (K genes of dose and delay;
 * the paper's loop, Materials and Methods, "The Main GA Loop", and its
 * appendix on the operators): rank by (fitness, index) with NaN last, copy the
 * n_elite best, and fill the other slots pairwise: tournament selection of two
 * parents, one-point crossover with probability p_cross, per-gene mutation
 * over the alphabet, and a guard that lowers the largest dose one alphabet
 * step until the total is within the cap.  Lower fitness is better.  Random
 * words: Philox blocks (pair, generation, 0x47414741, sub) keyed by
 * cfg->seed, generation read from *generation_d.
 *   fitness_d[N], dose_d[N][K], gap_h_d[N][K]   current population (device)
 *   order_d[N], position_d[N]                   rank outputs (device)
 *   next_dose_d[N][K], next_gap_h_d[N][K]       next population (device)
 * Requires 2 <= N, 1 <= K <= GGA_KMAX, doses on the alphabet's quantum grid.
 * Errors: GGA_E_ARG, GGA_E_ABI, GGA_E_ALPHABET, GGA_E_HIP.
 */
int gga_ga_breed(const gga_ga_cfg* ga, const gga_alphabet* a, const float* fitness_d,
                 const float* dose_d, const int32_t* gap_h_d, int32_t N, int32_t K,
                 const int32_t* generation_d, int32_t* order_d, int32_t* position_d,
                 float* next_dose_d, int32_t* next_gap_h_d, hipStream_t stream);

/* Device workspace of gga_ga_generation / gga_ga_run for N protocols x R replicas. */
size_t gga_ga_workspace_bytes(int32_t N, int32_t R);

/* Stream-ordered: store g in the workspace's generation counter.
 * Errors: GGA_E_ARG, GGA_E_HIP. */
int gga_ga_set_generation(void* ws_d, int32_t g, hipStream_t stream);

/*
 * One whole GA generation, stream-ordered: simulate every protocol of the
 * current population R times (Philox key cfg->seed + g * 0x9E3779B97F4A7C15,
 * g the generation counter held in the workspace), reduce the fitness, record
 * hist_d[g] = (best, mean fitness) when g < hist_cap, and breed the next
 * population.  With advance != 0 the counter is then incremented, so the same
 * enqueued work can be captured once in a hipGraph and replayed.  nfrac_d[N]
 * must hold K for every protocol.  Set the counter with gga_ga_set_generation.
 * Errors: as gga_simulate and gga_ga_breed; GGA_E_ARG for a small workspace.
 */
int gga_ga_generation(const gga_params* params, const gga_sim_cfg* cfg, const gga_ga_cfg* ga,
                      const gga_alphabet* a, const float* dose_d, const int32_t* gap_h_d,
                      const int32_t* nfrac_d, int32_t N, int32_t K, float* next_dose_d,
                      int32_t* next_gap_h_d, void* ws_d, size_t ws_bytes, float* hist_d,
                      int32_t hist_cap, int32_t advance, hipStream_t stream);

/*
 * Run generations g0 .. g0 + n_gen - 1 from population A (dose_a_d, gap_a_d),
 * alternating A -> B and B -> A; the last bred population is in A when n_gen
 * is even and in B otherwise.  A run continued with g0 = previous g0 + n_gen
 * from the previous result reproduces one longer run exactly.  use_graph = 0: each generation is enqueued and the host
 * waits for it before the next one (host-driven loop); use_graph = 1: the two
 * alternating generations are captured once into hipGraphs and replayed with
 * no host wait in between.  gen_ms_h[g] (HOST, or NULL) receives the time from
 * the start of the run to the end of generation g0 + g, from HIP events on
 * `stream`.  hist_d[g0 + n_gen][2] receives (best, mean) fitness at row g for
 * generation g.  Optional archive (both NULL, or both device arrays of
 * [g0 + n_gen][K]): best_dose_d / best_gap_d row g receive the genes of the
 * protocol with the best fitness of generation g.
 * Synchronous: returns after the stream has finished.  Creates and destroys
 * HIP graphs and events (host-side objects); allocates no device memory.
 * Errors: as gga_ga_generation.
 */
int gga_ga_run(const gga_params* params, const gga_sim_cfg* cfg, const gga_ga_cfg* ga,
               const gga_alphabet* a, float* dose_a_d, int32_t* gap_a_d, float* dose_b_d,
               int32_t* gap_b_d, const int32_t* nfrac_d, int32_t N, int32_t K, int32_t g0,
               int32_t n_gen, int32_t use_graph, void* ws_d, size_t ws_bytes, float* hist_d,
               float* best_dose_d, int32_t* best_gap_d, float* gen_ms_h, hipStream_t stream);

/*
 * GA over the paper's sparse time-slot genome (Materials and Methods, "GA
 * Resolution, constraints" and "Protocol Representation"; appendix "GA
 * Operators: additional details").  A genome is S bytes, one per hour of the
 * treatment window: the dose given at the start of that hour in quanta of
 * `quantum` Gy (0: no dose).  Guarded genomes hold no dose above dmax_q, no two
 * doses closer than g_min hours, and at most cap_q quanta in total.
 * Set struct_size = sizeof(gga_slot_cfg).
 */
#define GGA_SLOTS_MAX 256
#define GGA_SMUT_SWAP 1         /* a dose and another slot exchange contents          */
#define GGA_SMUT_SPLIT 2        /* a dose of >= 2 quanta splits into two placed doses  */
#define GGA_SMUT_TIME 4         /* a dose moves to another slot (what fits)            */
#define GGA_SMUT_VALUE 8        /* a dose grows, while the total is under the cap      */
typedef struct gga_slot_cfg {
    uint32_t struct_size;
    int32_t S;              /* slots (hours) in the window, 1 .. GGA_SLOTS_MAX        */
    int32_t g_min;          /* minimal interval between doses in hours, 1 .. S         */
    int32_t dmax_q;         /* maximal single dose in quanta, 1 .. 255                */
    int32_t cap_q;          /* cap on the total in quanta, 0 .. 65535                 */
    int32_t mutation;       /* GGA_SMUT_* bits, applied in the order swap, split, time,
                               value; 0 = swap | split | time (the operators of the
                               paper's final GA experiments)                         */
    float quantum;          /* Gy per quantum, finite, > 0                             */
    int32_t reserved;       /* 0                                                      */
} gga_slot_cfg;

/*
 * One GA breeding step over slot genomes, stream-ordered: rank by (fitness,
 * index) with NaN last, copy the ga->n_elite best to rows 0 .. n_elite - 1,
 * and fill the other rows with children: parents by ga->selection (as
 * gga_ga_breed), crossover by ga->crossover over slots (one point, the middle
 * cut between 25 % and 75 % of the window, two points with the first in
 * 25 .. 50 % and the second in 50 .. 75 %, or uniform), each mutation of
 * sc->mutation with probability ga->p_mut, then the guards: clamp to dmax_q;
 * a dose less than g_min after the last kept one moves to the first later
 * slot with no dose within g_min - 1 hours, or is dropped when there is none;
 * while the total exceeds cap_q the largest dose (first among equals) loses a
 * quantum.  Random words: Philox blocks (pair, generation, 0x47414741, sub)
 * keyed by ga->seed, generation read from *generation_d.
 *   fitness_d[N], pop_d[N][S]      current population (device)
 *   order_d[N], position_d[N]      rank outputs (device)
 *   next_d[N][S]                   next population (device; not pop_d)
 * Requires 2 <= N, ga->mutation == 0 (sc->mutation selects the operators).
 * Errors: GGA_E_ARG, GGA_E_ABI, GGA_E_HIP.
 */
int gga_slots_breed(const gga_ga_cfg* ga, const gga_slot_cfg* sc, const float* fitness_d,
                    const uint8_t* pop_d, int32_t N, const int32_t* generation_d, int32_t* order_d,
                    int32_t* position_d, uint8_t* next_d, hipStream_t stream);

/*
 * Slot genomes to simulation protocols, stream-ordered: the doses in slot
 * order, dose_d[p][j] = quanta x quantum (float32 product), delay_1 = slot of
 * the first dose and later delays the slot differences; nfrac_d[p] = number of
 * doses, at most K (a genome with more doses gives its first K; a guarded one
 * holds at most ceil(S / g_min)).  Entries past nfrac are 0.
 *   pop_d[P][S] (device) -> dose_d[P][K], gap_h_d[P][K], nfrac_d[P] (device)
 * Requires 1 <= K <= GGA_KMAX.  Errors: GGA_E_ARG, GGA_E_ABI, GGA_E_HIP.
 */
int gga_slots_decode(const gga_slot_cfg* sc, const uint8_t* pop_d, int32_t P, int32_t K, float* dose_d,
                     int32_t* gap_h_d, int32_t* nfrac_d, hipStream_t stream);

/*
 * Simulation protocols to guarded slot genomes, stream-ordered: fraction j
 * (j < nfrac, nfrac clipped to 0 .. K) adds round(dose_j / quantum) quanta
 * (float32 quotient, ties to even; 0 unless positive; a slot saturates at 255)
 * at hour delay_1 + .. + delay_j, until that hour falls outside 0 .. S - 1;
 * then the three guards run.
 *   dose_d[P][K], gap_h_d[P][K], nfrac_d[P] (device) -> pop_d[P][S] (device)
 * Requires 1 <= K <= GGA_KMAX.  Errors: GGA_E_ARG, GGA_E_ABI, GGA_E_HIP.
 */
int gga_slots_encode(const gga_slot_cfg* sc, const float* dose_d, const int32_t* gap_h_d,
                     const int32_t* nfrac_d, int32_t P, int32_t K, uint8_t* pop_d, hipStream_t stream);

/* Device workspace of gga_slots_run for N genomes x R replicas, K fractions. */
size_t gga_slots_workspace_bytes(int32_t N, int32_t R, int32_t K);

/*
 * Run generations g0 .. g0 + n_gen - 1 of the slot GA from population A,
 * alternating A -> B and B -> A (the last bred population is in A when n_gen
 * is even, in B otherwise).  Each generation decodes its genomes (K fraction
 * slots), simulates each R times (Philox key cfg->seed + g x
 * 0x9E3779B97F4A7C15), reduces the fitness, records hist_d[g] = (best, mean)
 * and the best protocol's decoded genes (best_dose_d / best_gap_d row g, both
 * NULL or both [g0 + n_gen][K] device arrays), and breeds the next population
 * as gga_slots_breed.  use_graph as gga_ga_run; gen_ms_h as gga_ga_run.
 *   pop_a_d[N][S], pop_b_d[N][S] (device), hist_d[g0 + n_gen][2] (device)
 * Requires K >= ceil(S / g_min) (every guarded dose is simulated) and
 * cap_q x quantum <= cfg->dose_cap + 1e-6 Gy (guarded genomes are valid
 * protocols).  With cfg->flags = GGA_SIM_HALF_HOUR the slots are 30 minutes.
 * Synchronous.  Errors: as gga_simulate and gga_slots_breed; GGA_E_ARG for a
 * small workspace or the requirements above.
 */
int gga_slots_run(const gga_params* params, const gga_sim_cfg* cfg, const gga_ga_cfg* ga,
                  const gga_slot_cfg* sc, uint8_t* pop_a_d, uint8_t* pop_b_d, int32_t N, int32_t K,
                  int32_t g0, int32_t n_gen, int32_t use_graph, void* ws_d, size_t ws_bytes, float* hist_d,
                  float* best_dose_d, int32_t* best_gap_d, float* gen_ms_h, hipStream_t stream);

/*
 * Surrogate of the simulation for pre-screening GA offspring (not part of the
 * paper's method): an MLP from an encoded protocol (40 fractions x (dose / 5
 * Gy, delay / 60 h, present), zero-padded to 128 features) through three
 * hidden layers of 512 with GELU(x) = x Phi(x) to one output, the normalised
 * fitness.  BF16 weights and activations on MFMA with FP32 accumulation; FP32
 * master weights and Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 *
 * Net buffer (device, caller-owned, gga_mlp_net_bytes() bytes), 256-byte
 * aligned blocks in this order: norm f32[2] (mu, sigma of the training
 * targets) and int32 Adam step count in one block, params f32[591873], Adam
 * m, Adam v, gradients (same size), then
 * bf16 copies W1 [128][512], W1^T, W2 [512][512], W2^T, W3, W3^T.  Parameter
 * order: W1 [128][512], b1[512], W2 [512][512], b2, W3 [512][512], b3,
 * w4[512], b4[1].  Work buffer: gga_mlp_work_bytes(B) bytes for batch B.
 * Net and work buffers (and the screened GA's workspace) must be 16-byte
 * aligned, as hipMalloc returns them: GGA_E_ARG otherwise.
 */
size_t gga_mlp_net_bytes(void);
size_t gga_mlp_work_bytes(int32_t B);

/* Test hook: byte offsets into a work buffer of batch B (B >= 0) of what the
 * passes leave there, written to offsets[12] (host): X bf16[B][128] (encoded
 * inputs), Z1, Z2, Z3 f32[B][512] (pre-activations), H1, H2, H3 bf16[B][512]
 * (activations), y f32[B] (outputs), dy f32[B] (loss gradient), dZa, dZb
 * bf16[B][512] (backward activation gradients), part (reduction partials).
 * After gga_mlp_grad, dZa holds dZ1 and dZb holds dZ2; Z3 is overwritten by
 * weight-gradient partials when B >= 1024.  Host only.  Errors: GGA_E_ARG. */
int gga_mlp_work_layout(int32_t B, size_t* offsets);

/* Initialise: weights uniform on +-1/sqrt(fan_in) from Philox keyed by seed,
 * biases and Adam state 0, norm (0, 1).  Synchronous.  Errors: GGA_E_ARG,
 * GGA_E_HIP. */
int gga_mlp_init(void* net_d, uint64_t seed, hipStream_t stream);

/* Set the target normalisation (mean, standard deviation) from n fitness
 * values (device).  Errors: GGA_E_ARG, GGA_E_HIP. */
int gga_mlp_set_norm(void* net_d, const float* target_d, int32_t n, hipStream_t stream);

/* Predicted fitness pred_d[B] (de-normalised) of protocols dose_d[B][K],
 * gap_h_d[B][K], nfrac_d[B] (K <= GGA_KMAX; fractions past 40 are ignored).
 * Errors: GGA_E_ARG, GGA_E_HIP. */
int gga_mlp_predict(const void* net_d, const float* dose_d, const int32_t* gap_h_d,
                    const int32_t* nfrac_d, int32_t B, int32_t K, void* work_d, size_t work_bytes,
                    float* pred_d, hipStream_t stream);

/* Forward and backward pass of the loss mean((y - (t - mu)/sigma)^2) over a
 * batch with targets target_d[B]; gradients land in the net buffer's gradient
 * block, the loss in loss_d[0] (or NULL).  Errors: GGA_E_ARG, GGA_E_HIP. */
int gga_mlp_grad(void* net_d, const float* dose_d, const int32_t* gap_h_d, const int32_t* nfrac_d,
                 const float* target_d, int32_t B, int32_t K, void* work_d, size_t work_bytes,
                 float* loss_d, hipStream_t stream);

/* gga_mlp_grad, then one Adam step (step counts from 1) with learning rate lr
 * and a refresh of the bf16 copies.  Errors: GGA_E_ARG, GGA_E_HIP. */
int gga_mlp_train_step(void* net_d, const float* dose_d, const int32_t* gap_h_d,
                       const int32_t* nfrac_d, const float* target_d, int32_t B, int32_t K,
                       int32_t step, float lr, void* work_d, size_t work_bytes, float* loss_d,
                       hipStream_t stream);

/* Test hook of the MLP's MFMA GEMM: C_d[M][N] (f32) = A * B with bf16 inputs
 * A stored [M][K] (or [K][M] if a_trans) and B stored [K][N] (or [N][K] if
 * b_trans).  Errors: GGA_E_ARG, GGA_E_HIP. */
int gga_mlp_gemm(int32_t M, int32_t N, int32_t K, const void* A_d, int32_t a_trans, const void* B_d,
                 int32_t b_trans, float* C_d, hipStream_t stream);

/*
 * Microbenchmarks of the resources the kernels are measured against, on the
 * current device: valu_ops_h[0] = full-rate 32-bit VALU lane-operations per
 * second (independent FMA chains, an FMA counted as one operation),
 * lds_bytes_h[0] = LDS read bytes per second (conflict-free 16-byte reads),
 * hbm_bytes_h[0] = HBM read bytes per second (one pass over buf_d).  buf_d:
 * device buffer of `bytes` >= 256 MiB + 256, 16-byte aligned, contents
 * ignored (its last 256 bytes are reserved).  Results are HOST doubles.
 * Synchronous.  Errors: GGA_E_ARG, GGA_E_HIP.
 */
int gga_measure_peaks(void* buf_d, size_t bytes, double* valu_ops_h, double* lds_bytes_h, double* hbm_bytes_h,
                      hipStream_t stream);

/* Surrogate-screened GA settings.  Set struct_size = sizeof(gga_sga_cfg). */
typedef struct gga_sga_cfg {
    uint32_t struct_size;
    int32_t n_candidates;   /* C: offspring bred and screened per generation, >= 2      */
    int32_t n_simulated;    /* S: screened offspring fully simulated, 1 .. C            */
    int32_t screen;         /* 1: the S best predicted by the surrogate; 0: S random     */
    int32_t refine_steps;   /* Adam steps per generation on the N + S simulated pairs, 0 .. 64 (screen = 1) */
    float refine_lr;        /* their learning rate (> 0 when refine_steps > 0)           */
} gga_sga_cfg;

/* Device workspace of the surrogate-screened GA. */
size_t gga_sga_workspace_bytes(int32_t N, int32_t K, int32_t R, int32_t C, int32_t S);

/*
 * Prepare a surrogate-screened GA: simulate the initial population
 * pop_dose_d[N][K], pop_gap_d[N][K] (R replicas, Philox key cfg->seed) into
 * pop_fit_d[0 .. N-1] and set the generation counter to 0.  The population
 * arrays have N + S rows; rows N .. N+S-1 are working space.
 * Errors: as gga_simulate; GGA_E_ARG for a small workspace.
 */
int gga_sga_init(const gga_params* params, const gga_sim_cfg* cfg, const gga_sga_cfg* sga,
                 float* pop_dose_d, int32_t* pop_gap_d, float* pop_fit_d, int32_t N, int32_t K,
                 void* ws_d, size_t ws_bytes, hipStream_t stream);

/*
 * One surrogate-screened generation, stream-ordered: rank the population by
 * its simulated fitness, breed C candidates with the GA operators (as
 * gga_ga_breed, no elites), predict their fitness with the surrogate net_d
 * (gga_mlp_*), fully simulate the S best-predicted candidates as members of
 * population g + 1 (Philox key cfg->seed + (g + 1) * 0x9E3779B97F4A7C15, the
 * initial population being population 0), and keep the best N of the N + S
 * evaluated protocols, sorted, in rows 0 .. N-1.  With refine_steps > 0 the
 * surrogate first takes that many Adam steps (on the net's own step count) on
 * the N + S simulated pairs: the simulation checks the surrogate's error and
 * corrects it where the search is.  hist_d[g] = (best, mean) fitness of the
 * kept population.  With screen = 0 the S candidates are
 * picked at random instead (the same loop without the surrogate).
 * Errors: as gga_ga_generation.
 */
int gga_sga_generation(const gga_params* params, const gga_sim_cfg* cfg, const gga_ga_cfg* ga,
                       const gga_alphabet* a, const gga_sga_cfg* sga, void* net_d,
                       float* pop_dose_d, int32_t* pop_gap_d, float* pop_fit_d, int32_t N, int32_t K,
                       void* ws_d, size_t ws_bytes, float* hist_d, int32_t hist_cap,
                       hipStream_t stream);

/*
 * Generations g0 .. g0+n_gen-1 of gga_sga_generation, host-driven
 * (use_graph = 0) or as a captured hipGraph replayed (use_graph = 1); timing,
 * history and the optional best-protocol archive as gga_ga_run (the archived
 * protocol of generation g is row 0 of the kept population).  Synchronous;
 * creates and destroys HIP graphs and events; allocates no device memory.
 * Errors: as gga_sga_generation.
 */
int gga_sga_run(const gga_params* params, const gga_sim_cfg* cfg, const gga_ga_cfg* ga,
                const gga_alphabet* a, const gga_sga_cfg* sga, void* net_d, float* pop_dose_d,
                int32_t* pop_gap_d, float* pop_fit_d, int32_t N, int32_t K, int32_t g0, int32_t n_gen,
                int32_t use_graph, void* ws_d, size_t ws_bytes, float* hist_d, float* best_dose_d,
                int32_t* best_gap_d, float* gen_ms_h, hipStream_t stream);

/*
 * gga_simulate from a library of pre-grown tumours instead of the seed disc
 * (Materials and Methods, "The tumour case library": protocols are evaluated
 * on tumours grown beforehand without treatment); resident sides only, no
 * workspace.  Replica r of every
 * protocol starts from library state r mod n_lib: lib_fields_d[n_lib][3][L][L]
 * (f32) and lib_cells_d[n_lib][L][L] (u16 words), for example states grown by
 * gga_state_init and gga_state_run; the library is read, never written.
 * Treatment steps count from 0; Philox counters as gga_simulate.
 * Errors: as gga_simulate; GGA_E_ARG for n_lib < 1.
 */
int gga_simulate_library(const gga_params* params, const gga_sim_cfg* cfg, const float* dose_d,
                         const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P, int32_t K,
                         const float* lib_fields_d, const uint16_t* lib_cells_d, int32_t n_lib, int32_t* live_d,
                         float* fitness_d, hipStream_t stream);

/*
 * Philox4x32-10 blocks (Salmon et al., SC'11) from the device implementation
 * the simulator uses: out_d[i][0..3] = Philox(counter ctr_d[i][0..3], key
 * (seed lo, seed hi)) for i < n.  A test hook.
 * Errors: GGA_E_ARG, GGA_E_HIP.
 */
int gga_philox_fill(const uint32_t* ctr_d, uint64_t seed, uint32_t* out_d, int64_t n,
                    hipStream_t stream);

/*
 * Kernel variants and uneven batches.  The paper simulates many instances
 * within and across GPUs (Materials and Methods, "GPU implementation"); a
 * batch here may mix lattice sides, fraction counts and horizons.
 *
 * Variants of the simulation kernel, numbered 0 .. gga_variant_count()-1, each
 * for one lattice side.  Resident variants keep an instance's whole state on
 * one compute unit for its whole horizon; slab variants (the only form for
 * L = 160 .. 256, whose state exceeds a compute unit) advance slabs of rows of a
 * lattice one step per launch between two state buffers in device memory,
 * each slab recomputing `substeps + 2` halo rows at its inner edges.  Every
 * variant gives bit-identical results.  Sides below a variant's row pitch of
 * 64 * columns-per-lane (96 in 128, 160 .. 224 in 256) hold padding lanes.
 * gga_state_run uses the chosen resident variant of L; gga_simulate the chosen
 * resident variant, or the chosen variant of any form for sides without one;
 * gga_simulate_uneven the chosen variant of any form.  Choices are process-wide; gga_autotune sets them by timing.
 */
int gga_variant_count(void);
int32_t gga_variant_side(int32_t v);      /* lattice side of variant v, -1 if none    */
int32_t gga_variant_is_slab(int32_t v);   /* 1 slab form, 0 resident, -1 no variant   */
const char* gga_variant_name(int32_t v);  /* static string                           */
/* Chosen variant for side L (resident_only != 0: the one gga_simulate uses).
 * Returns the variant, or GGA_E_UNSUPPORTED. */
int gga_get_variant(int32_t L, int32_t resident_only);
/* Choose variant v for its side (a resident v also becomes the resident
 * choice).  Returns GGA_OK or GGA_E_ARG. */
int gga_set_variant(int32_t L, int32_t v);

/*
 * Device workspace of gga_simulate_uneven for these HOST arrays lattice_h[P]
 * (64, 96, .., 256) and horizon_h[P] (>= 0 steps), R replicas and `substeps`
 * diffusion sub-steps per step (cfg->substeps of the call) under the current
 * variant choices and team setting; 0 for invalid arguments.
 */
size_t gga_uneven_workspace_bytes(const int32_t* lattice_h, const int32_t* horizon_h, int32_t P, int32_t K,
                                  int32_t R, int32_t substeps);

/*
 * Slab groups (sides without a resident variant, in gga_simulate and
 * gga_simulate_uneven) run as teams by default: the slabs of one instance are
 * co-resident workgroups of a cooperative launch that keep their rows on the
 * compute unit for the instance's whole horizon and exchange halo rows
 * through device memory after every step, each waiting for its neighbours'
 * step count with a bounded spin.  A wait that runs out leaves the instance's
 * live count negative (so its fitness is NaN) and every workgroup exits.
 * Test hook, process-wide: use_teams = 0 runs slab groups as one launch per
 * step instead (bit-identical results, larger workspace); spin_limit bounds
 * each wait (default 2^21 polls; negative: every wait fails).  Workspace
 * sizes depend on use_teams.  Returns GGA_OK or GGA_E_ARG.
 */
int gga_set_team_options(int32_t use_teams, int32_t spin_limit);

/*
 * gga_simulate for a batch whose protocol p runs on a lattice_h[p] x
 * lattice_h[p] lattice for horizon_h[p] steps (HOST arrays; cfg->L and
 * cfg->horizon are not used).  Instances are grouped by lattice side and
 * launched longest horizon first; slab-form groups run as teams (cooperative
 * launches of as many instances as the device holds at once, each instance's
 * slabs resident for its whole horizon), or with the team form switched off
 * take one launch per step over the instances still running.  live_d[P][R], fitness_d[P] as
 * gga_simulate (-1 / NaN for invalid protocols).  The instance order is
 * uploaded from host memory, and the call waits for that copy (and the work
 * already on `stream`) before enqueueing the kernels; it returns without
 * waiting for them.  Errors: as gga_simulate; GGA_E_UNSUPPORTED for another
 * side or too many sub-steps for the slab plan; GGA_E_ARG for a small
 * workspace.
 */
int gga_simulate_uneven(const gga_params* params, const gga_sim_cfg* cfg, const float* dose_d,
                        const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P, int32_t K,
                        const int32_t* lattice_h, const int32_t* horizon_h, void* ws_d, size_t ws_bytes,
                        int32_t* live_d, float* fitness_d, hipStream_t stream);

/* Workspace of gga_state_run_variant's event table. */
size_t gga_event_table_bytes(int32_t P, int32_t K);

/*
 * Test hook: gga_state_run with kernel variant `variant` (side cfg->L).  Slab
 * variants need nsteps >= 1, second state buffers fields2_d / cells2_d of the
 * same shape (overwritten) and ws_d of gga_event_table_bytes(P, K) bytes; the
 * result is in fields_d / cells_d.  live_d[P][R] (or NULL) receives the live
 * counts after the last step.  Errors: as gga_state_run; GGA_E_ARG for a
 * variant of another side.
 */
int gga_state_run_variant(const gga_params* params, const gga_sim_cfg* cfg, int32_t variant,
                          const float* dose_d, const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P,
                          int32_t K, int32_t n0, int32_t nsteps, float* fields_d, uint16_t* cells_d,
                          float* fields2_d, uint16_t* cells2_d, void* ws_d, size_t ws_bytes, int32_t* live_d,
                          hipStream_t stream);

/* Workspace of gga_autotune: the largest uneven workspace over L's variants. */
size_t gga_autotune_workspace_bytes(int32_t L, int32_t P, int32_t K, int32_t R, int32_t horizon, int32_t substeps);

/*
 * Autotuner: simulate the protocols on side cfg->L for cfg->horizon steps with
 * every variant of that side (one warm-up run, then the faster of two timed
 * runs, HIP events on `stream`), write each variant's milliseconds to ms_h
 * (HOST, gga_variant_count() entries, NaN for variants not timed), and make
 * the fastest the choice for L (and the fastest resident one the resident
 * choice).  live_d[P][R] and fitness_d[P] hold the last run's results.
 * Synchronous.  Returns the chosen variant, or an error as
 * gga_simulate_uneven.
 */
int gga_autotune(const gga_params* params, const gga_sim_cfg* cfg, const float* dose_d, const int32_t* gap_h_d,
                 const int32_t* nfrac_d, int32_t P, int32_t K, void* ws_d, size_t ws_bytes, int32_t* live_d,
                 float* fitness_d, float* ms_h, hipStream_t stream);

/*
 * Quasi-3D variant (the paper's model is quasi-three-dimensional, a site
 * holding many cells: Introduction, and Materials and Methods on the cells
 * per site).  Every site holds C cell slots (1 <= C <= GGA_Q3_MAX_SLOTS,
 * C L^2 <= 2^23, 8 <= L <= 512); the fields stay two-dimensional.  With C = 1
 * every rule is gga_simulate's.  Rules the paper does not print, fixed here:
 *   - slot z of site s = y L + x draws the Philox block of site counter
 *     z L^2 + s (slot 0 draws what the 2D model draws);
 *   - initial state: slot 0 is the 2D seed disc, the other slots EMPTY;
 *   - a fraction treats every live cell as the 2D model does (class by its
 *     age; oxygen bin of its site);
 *   - a site's activity is the mean over its C slots of activity[state];
 *   - cell update: every cell as in the 2D model with its site's fields; the
 *     free places of a cell are the EMPTY slots of its own site and of its four
 *     von Neumann neighbours, in the order own, N, E, S, W and by slot within a
 *     site; m counts them, a ready cell proposes the k-th, k = floor(w0 m /
 *     2^32), with the 64-bit key ((w2 >> 3) << 8) | (d << 5) | z (d = 4 for its
 *     own site, else its direction seen from the target, N 0, E 1, S 2, W 3),
 *     and each EMPTY slot takes the smallest key (daughter and winning parent
 *     get age 0);
 *   - live counts count PROLIF and QUIESC cells over all slots.
 * State: fields_d[P*R][3][L][L] (float32, field units as gga_state_init) and
 * cells_d[P*R][C][L][L] (uint16 words, slot planes).  cfg->flags may hold
 * GGA_SIM_HALF_HOUR.  Every parameter option of gga_params applies.
 * Workspace: gga_q3_workspace_bytes(L, C, P, R, K) bytes of device memory,
 * 16-byte aligned, caller-owned, contents not preserved between calls; calls
 * sharing a workspace must not overlap.
 * Errors: GGA_E_ARG (null or misaligned pointer, small workspace, C out of
 * range, n0 + nsteps > 2^30, P R ceil(L^2 / 256) >= 2^31), GGA_E_ABI,
 * GGA_E_PARAM, GGA_E_UNSUPPORTED (L, substeps or C L^2 out of range),
 * GGA_E_HIP.
 */
#define GGA_Q3_MAX_SLOTS 32
size_t gga_q3_workspace_bytes(int32_t L, int32_t C, int32_t P, int32_t R, int32_t K);

/* Initial state of P * cfg->R quasi-3D instances (no workspace). */
int gga_q3_init(const gga_params* params, const gga_sim_cfg* cfg, int32_t C, int32_t P, float* fields_d,
                uint16_t* cells_d, hipStream_t stream);

/*
 * Advance the given quasi-3D states by nsteps steps from step n0, in place.
 * live_d[P][R] (or NULL) receives the final live counts and traj_d (or NULL)
 * [P][R][nsteps] the count after every step (with nsteps = 0, live_d gets the
 * count of the given state).  Invalid protocols leave their states untouched
 * and get -1 in live_d and traj_d.
 */
int gga_q3_run(const gga_params* params, const gga_sim_cfg* cfg, int32_t C, const float* dose_d,
               const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P, int32_t K, int32_t n0, int32_t nsteps,
               float* fields_d, uint16_t* cells_d, void* ws_d, size_t ws_bytes, int32_t* live_d, int32_t* traj_d,
               hipStream_t stream);

/*
 * gga_simulate for the quasi-3D variant: the initial state, cfg->horizon
 * steps, live_d[P][R] (-1 for invalid protocols), fitness_d[P] (the mean over
 * replicas, NaN for invalid protocols) and traj_d[P][R][horizon] or NULL.
 * The state is held in the workspace.
 */
int gga_simulate_q3(const gga_params* params, const gga_sim_cfg* cfg, int32_t C, const float* dose_d,
                    const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P, int32_t K, void* ws_d, size_t ws_bytes,
                    int32_t* live_d, float* fitness_d, int32_t* traj_d, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GGA_H */
