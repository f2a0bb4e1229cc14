// Host side of the C ABI: argument checks, the host validator and launches.
// Every simulation step runs in the kernels; this file only checks and
// marshals arguments.
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "gga_internal.h"

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
    g_last_hip = static_cast<int>(e);
    return GGA_E_HIP;
}

bool finite_in(float v, float lo, float hi) { return std::isfinite(v) && v >= lo && v <= hi; }

int check_params(const gga_params* p) {
    if (!p) return GGA_E_ARG;
    if (p->struct_size != sizeof(gga_params)) return GGA_E_ABI;
    for (int f = 0; f < 3; ++f) {
        if (!finite_in(p->lambda[f], 0.0f, 0.25f)) return GGA_E_PARAM;
        if (!finite_in(p->kappa[f], f == 0 ? 1e-30f : 0.0f, 1e30f)) return GGA_E_PARAM;
        if (!std::isfinite(p->ghost[f]) || !std::isfinite(p->init[f])) return GGA_E_PARAM;
    }
    for (int s = 0; s < 4; ++s)
        if (!finite_in(p->activity[s], 0.0f, 1e30f)) return GGA_E_PARAM;
    if (p->T_min < 0 || p->T_lys < 0 || p->A0 < 1 || p->seed_radius < 0) return GGA_E_PARAM;
    if (p->class_age[0] < 0 || p->class_age[1] < p->class_age[0]) return GGA_E_PARAM;
    if (!(p->P_div >= 0.0 && p->P_div <= 1.0)) return GGA_E_PARAM;
    if (!std::isfinite(p->alpha) || !std::isfinite(p->beta)) return GGA_E_PARAM;
    for (int c = 0; c < 4; ++c)
        if (!std::isfinite(p->m[c])) return GGA_E_PARAM;
    return GGA_OK;
}

int check_cfg(const gga_sim_cfg* c) {
    if (!c) return GGA_E_ARG;
    if (c->struct_size != sizeof(gga_sim_cfg)) return GGA_E_ABI;
    if (c->flags != 0 || c->R < 1 || c->horizon < 0) return GGA_E_ARG;
    if (!std::isfinite(c->dose_cap)) return GGA_E_ARG;
    if (!gga::sim_supported(c->L) || c->substeps < 1 || c->substeps > 64) return GGA_E_UNSUPPORTED;
    return GGA_OK;
}

int check_batch(int32_t P, int32_t K, int32_t R) {
    if (P < 0 || K < 0 || K > GGA_KMAX) return GGA_E_ARG;
    if ((long long)P * R > std::numeric_limits<int32_t>::max()) return GGA_E_ARG;
    return GGA_OK;
}

gga::SimArgs make_args(const gga_params* prm, const gga_sim_cfg* cfg, const float* dose,
                       const int32_t* gap, const int32_t* nfrac, int32_t K) {
    gga::SimArgs a;
    std::memset(&a, 0, sizeof(a));
    a.prm = *prm;
    a.dose = dose;
    a.gap = gap;
    a.nfrac = nfrac;
    a.K = K;
    a.R = cfg->R;
    a.substeps = cfg->substeps;
    a.seed_lo = static_cast<uint32_t>(cfg->seed);
    a.seed_hi = static_cast<uint32_t>(cfg->seed >> 32);
    a.dose_cap = cfg->dose_cap;
    return a;
}

}  // namespace

extern "C" {

int gga_version(void) { return GGA_ABI_VERSION; }

const char* gga_strerror(int code) {
    switch (code) {
        case GGA_OK: return "success";
        case GGA_E_ARG: return "invalid argument (null pointer, negative or oversized size)";
        case GGA_E_ABI: return "struct_size does not match this library's ABI";
        case GGA_E_UNSUPPORTED: return "unsupported lattice side or sub-step count";
        case GGA_E_HIP: return "HIP runtime error (see gga_last_hip_error)";
        case GGA_E_PARAM: return "model constant out of range";
        case GGA_E_ALPHABET: return "alphabet admits no protocol or exceeds the table limit";
        default: return "unknown error code";
    }
}

int gga_last_hip_error(void) { return g_last_hip; }

int gga_validate(const gga_sim_cfg* cfg, const float* dose, const int32_t* gap_h,
                 const int32_t* nfrac, int32_t P, int32_t K, int32_t* status) {
    if (!cfg) return GGA_E_ARG;
    if (cfg->struct_size != sizeof(gga_sim_cfg)) return GGA_E_ABI;
    if (P < 0 || K < 0) return GGA_E_ARG;
    if (P > 0 && (!nfrac || !status || (K > 0 && (!dose || !gap_h)))) return GGA_E_ARG;
    for (int32_t p = 0; p < P; ++p) {
        const int32_t k = nfrac[p];
        if (k < 0 || k > K) {
            status[p] = GGA_PROTO_NFRAC;
            continue;
        }
        int st = GGA_PROTO_OK;
        double total = 0.0;
        for (int32_t j = 0; j < k; ++j) {
            const float d = dose[(size_t)p * K + j];
            if (!std::isfinite(d) || d < 0.0f) { st = GGA_PROTO_DOSE; break; }
            if (gap_h[(size_t)p * K + j] < (j == 0 ? 0 : 1)) { st = GGA_PROTO_GAP; break; }
            total += static_cast<double>(d);
        }
        if (st == GGA_PROTO_OK && total > cfg->dose_cap + 1e-6) st = GGA_PROTO_CAP;
        status[p] = st;
    }
    return GGA_OK;
}

int gga_population_random(const gga_alphabet* a, int32_t P, int32_t K, uint64_t seed,
                          float* dose_d, int32_t* gap_h_d, int32_t* nfrac_d, hipStream_t stream) {
    if (!a) return GGA_E_ARG;
    if (a->struct_size != sizeof(gga_alphabet)) return GGA_E_ABI;
    if (P < 0 || K < 0 || K > GGA_KMAX) return GGA_E_ARG;
    if (P > 0 && (!nfrac_d || (K > 0 && (!dose_d || !gap_h_d)))) return GGA_E_ARG;
    if (a->n_dose < 1 || a->n_dose > GGA_ALPHABET_MAX || a->n_gap < 1 || a->n_gap > GGA_ALPHABET_MAX)
        return GGA_E_ALPHABET;
    if (a->kmin < 0 || a->kmin > a->kmax || a->kmax > K) return GGA_E_ALPHABET;
    if (!(std::isfinite(a->dose_quantum) && a->dose_quantum > 0.0f) || !(std::isfinite(a->cap) && a->cap >= 0.0f))
        return GGA_E_ALPHABET;
    for (int i = 0; i < a->n_dose; ++i)
        if (a->dose_q[i] < 1 || (i > 0 && a->dose_q[i] <= a->dose_q[i - 1])) return GGA_E_ALPHABET;
    for (int i = 0; i < a->n_gap; ++i)
        if (a->gaps[i] < 1) return GGA_E_ALPHABET;
    const double capq = std::floor((double)a->cap / (double)a->dose_quantum + 1e-9);
    if (capq > 1e6) return GGA_E_ALPHABET;
    const int cap_q = static_cast<int>(capq);
    if ((long long)(a->kmax + 1) * (cap_q + 1) > gga::POP_TABLE_MAX) return GGA_E_ALPHABET;
    if ((long long)a->kmax * a->dose_q[0] > cap_q) return GGA_E_ALPHABET;   // no feasible protocol
    if (P == 0) return GGA_OK;
    gga::PopArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    pa.n_dose = a->n_dose;
    pa.n_gap = a->n_gap;
    pa.kmin = a->kmin;
    pa.kmax = a->kmax;
    pa.cap_q = cap_q;
    pa.K = K;
    pa.P = P;
    pa.quantum = a->dose_quantum;
    pa.seed_lo = static_cast<uint32_t>(seed);
    pa.seed_hi = static_cast<uint32_t>(seed >> 32);
    std::memcpy(pa.dose_q, a->dose_q, sizeof(pa.dose_q));
    std::memcpy(pa.gaps, a->gaps, sizeof(pa.gaps));
    pa.dose = dose_d;
    pa.gap = gap_h_d;
    pa.nfrac = nfrac_d;
    const hipError_t e = gga::launch_population(pa, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_simulate(const gga_params* params, const gga_sim_cfg* cfg, const float* dose_d,
                 const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P, int32_t K,
                 int32_t* live_d, float* fitness_d, int32_t* traj_d, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    if ((rc = check_batch(P, K, cfg->R))) return rc;
    if (P == 0) return GGA_OK;
    if (!nfrac_d || !live_d || !fitness_d || (K > 0 && (!dose_d || !gap_h_d))) return GGA_E_ARG;
    gga::SimArgs a = make_args(params, cfg, dose_d, gap_h_d, nfrac_d, K);
    a.n0 = 0;
    a.nsteps = cfg->horizon;
    a.mode = 0;
    a.live = live_d;
    a.traj = traj_d;
    hipError_t e = gga::launch_simulation(a, cfg->L, P * cfg->R, stream);
    if (e != hipSuccess) return hip_fail(e);
    e = gga::launch_fitness(live_d, P, cfg->R, fitness_d, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_state_init(const gga_params* params, const gga_sim_cfg* cfg, int32_t P, float* fields_d,
                   uint16_t* cells_d, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    if ((rc = check_batch(P, 0, cfg->R))) return rc;
    if (P == 0) return GGA_OK;
    if (!fields_d || !cells_d) return GGA_E_ARG;
    // No protocol: the kernel reads a null nfrac as zero fractions.
    gga::SimArgs a = make_args(params, cfg, nullptr, nullptr, nullptr, 0);
    a.nsteps = 0;
    a.mode = gga::MODE_STORE;
    a.fields = fields_d;
    a.cells = cells_d;
    const hipError_t e = gga::launch_simulation(a, cfg->L, P * cfg->R, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_state_run(const gga_params* params, const gga_sim_cfg* cfg, const float* dose_d,
                  const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P, int32_t K, int32_t n0,
                  int32_t nsteps, float* fields_d, uint16_t* cells_d, int32_t* live_d,
                  int32_t* traj_d, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    if ((rc = check_batch(P, K, cfg->R))) return rc;
    if (n0 < 0 || nsteps < 0 || (long long)n0 + nsteps > std::numeric_limits<int32_t>::max())
        return GGA_E_ARG;
    if (P == 0) return GGA_OK;
    if (!nfrac_d || !fields_d || !cells_d || (K > 0 && (!dose_d || !gap_h_d))) return GGA_E_ARG;
    gga::SimArgs a = make_args(params, cfg, dose_d, gap_h_d, nfrac_d, K);
    a.n0 = n0;
    a.nsteps = nsteps;
    a.mode = gga::MODE_LOAD | gga::MODE_STORE;
    a.fields = fields_d;
    a.cells = cells_d;
    a.live = live_d;
    a.traj = traj_d;
    const hipError_t e = gga::launch_simulation(a, cfg->L, P * cfg->R, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_philox_fill(const uint32_t* ctr_d, uint64_t seed, uint32_t* out_d, int64_t n,
                    hipStream_t stream) {
    if (n < 0 || (n > 0 && (!ctr_d || !out_d))) return GGA_E_ARG;
    if (n > (int64_t)1 << 40) return GGA_E_ARG;
    const hipError_t e = gga::launch_philox_fill(ctr_d, seed, out_d, (long long)n, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

}  // extern "C"

// ------------------------------------------------------------------ GA

namespace {

// Workspace of the GA: generation counter, live counts, fitness, rank arrays.
struct GaWorkspace {
    int32_t* generation;
    int32_t* live;
    float* fitness;
    int32_t* order;
    int32_t* position;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t ga_ws_bytes(int32_t N, int32_t R) {
    return align256(sizeof(int32_t)) + align256(sizeof(int32_t) * (size_t)N * R) +
           3 * align256(sizeof(int32_t) * (size_t)N);
}

GaWorkspace ga_ws(void* ws, int32_t N, int32_t R) {
    char* p = static_cast<char*>(ws);
    GaWorkspace w;
    w.generation = reinterpret_cast<int32_t*>(p);
    p += align256(sizeof(int32_t));
    w.live = reinterpret_cast<int32_t*>(p);
    p += align256(sizeof(int32_t) * (size_t)N * R);
    w.fitness = reinterpret_cast<float*>(p);
    p += align256(sizeof(int32_t) * (size_t)N);
    w.order = reinterpret_cast<int32_t*>(p);
    p += align256(sizeof(int32_t) * (size_t)N);
    w.position = reinterpret_cast<int32_t*>(p);
    return w;
}

uint32_t prob_threshold(double p) {
    const double t = std::floor(p * 4294967296.0);
    return t >= 4294967295.0 ? 0xFFFFFFFFu : static_cast<uint32_t>(t);
}

int check_ga(const gga_ga_cfg* ga, const gga_alphabet* a, int32_t N, int32_t K, gga::GaArgs* out) {
    if (!ga || !a) return GGA_E_ARG;
    if (ga->struct_size != sizeof(gga_ga_cfg) || a->struct_size != sizeof(gga_alphabet)) return GGA_E_ABI;
    if (N < 2 || K < 1 || K > GGA_KMAX) return GGA_E_ARG;
    if (ga->n_elite < 0 || ga->n_elite > N || ga->tournament_k < 1 || ga->tournament_k > 64) return GGA_E_ARG;
    if (!(ga->p_cross >= 0.0 && ga->p_cross <= 1.0) || !(ga->p_mut >= 0.0 && ga->p_mut <= 1.0)) return GGA_E_ARG;
    if (a->n_dose < 1 || a->n_dose > GGA_ALPHABET_MAX || a->n_gap < 1 || a->n_gap > GGA_ALPHABET_MAX)
        return GGA_E_ALPHABET;
    if (!(std::isfinite(a->dose_quantum) && a->dose_quantum > 0.0f) || !(std::isfinite(a->cap) && a->cap >= 0.0f))
        return GGA_E_ALPHABET;
    for (int i = 0; i < a->n_dose; ++i)
        if (a->dose_q[i] < 1 || (i > 0 && a->dose_q[i] <= a->dose_q[i - 1])) return GGA_E_ALPHABET;
    for (int i = 0; i < a->n_gap; ++i)
        if (a->gaps[i] < 1) return GGA_E_ALPHABET;
    const double capq = std::floor((double)a->cap / (double)a->dose_quantum + 1e-9);
    if (capq > 1e6 || (long long)K * a->dose_q[0] > capq) return GGA_E_ALPHABET;   // guard must succeed
    std::memset(out, 0, sizeof(*out));
    out->N = N;
    out->K = K;
    out->n_elite = ga->n_elite;
    out->k = ga->tournament_k;
    out->n_dose = a->n_dose;
    out->n_gap = a->n_gap;
    out->cap_q = static_cast<int32_t>(capq);
    out->t_cross = prob_threshold(ga->p_cross);
    out->t_mut = prob_threshold(ga->p_mut);
    out->seed_lo = static_cast<uint32_t>(ga->seed);
    out->seed_hi = static_cast<uint32_t>(ga->seed >> 32);
    out->quantum = a->dose_quantum;
    std::memcpy(out->dose_q, a->dose_q, sizeof(out->dose_q));
    std::memcpy(out->gaps, a->gaps, sizeof(out->gaps));
    return GGA_OK;
}

// Enqueue one generation; all arguments already checked.
hipError_t enqueue_generation(const gga_params* params, const gga_sim_cfg* cfg, gga::GaArgs ga_args,
                              const float* dose, const int32_t* gap, const int32_t* nfrac, int32_t N,
                              int32_t K, float* next_dose, int32_t* next_gap, const GaWorkspace& w,
                              float* hist, int32_t hist_cap, int32_t advance, hipStream_t stream) {
    gga::SimArgs sa = make_args(params, cfg, dose, gap, nfrac, K);
    sa.n0 = 0;
    sa.nsteps = cfg->horizon;
    sa.mode = 0;
    sa.live = w.live;
    sa.generation = w.generation;
    sa.seed = cfg->seed;
    hipError_t e = gga::launch_simulation(sa, cfg->L, N * cfg->R, stream);
    if (e == hipSuccess) e = gga::launch_fitness(w.live, N, cfg->R, w.fitness, stream);
    if (e == hipSuccess) e = gga::launch_rank(w.fitness, N, w.order, w.position, stream);
    if (e == hipSuccess) e = gga::launch_history(w.fitness, N, w.order, w.generation, hist, hist_cap, stream);
    ga_args.dose = dose;
    ga_args.gap = gap;
    ga_args.order = w.order;
    ga_args.position = w.position;
    ga_args.generation = w.generation;
    ga_args.next_dose = next_dose;
    ga_args.next_gap = next_gap;
    if (e == hipSuccess) e = gga::launch_offspring(ga_args, stream);
    if (e == hipSuccess && advance) e = gga::launch_counter(w.generation, 1, 1, stream);
    return e;
}

}  // namespace

extern "C" {

size_t gga_ga_workspace_bytes(int32_t N, int32_t R) {
    if (N < 0 || R < 1) return 0;
    return ga_ws_bytes(N, R);
}

int gga_ga_set_generation(void* ws_d, int32_t g, hipStream_t stream) {
    if (!ws_d) return GGA_E_ARG;
    const hipError_t e = gga::launch_counter(static_cast<int32_t*>(ws_d), g, 0, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_ga_breed(const gga_ga_cfg* ga, const gga_alphabet* a, const float* fitness_d, const float* dose_d,
                 const int32_t* gap_h_d, int32_t N, int32_t K, const int32_t* generation_d, int32_t* order_d,
                 int32_t* position_d, float* next_dose_d, int32_t* next_gap_h_d, hipStream_t stream) {
    gga::GaArgs ga_args;
    const int rc = check_ga(ga, a, N, K, &ga_args);
    if (rc) return rc;
    if (!fitness_d || !dose_d || !gap_h_d || !generation_d || !order_d || !position_d || !next_dose_d ||
        !next_gap_h_d)
        return GGA_E_ARG;
    hipError_t e = gga::launch_rank(fitness_d, N, order_d, position_d, stream);
    ga_args.dose = dose_d;
    ga_args.gap = gap_h_d;
    ga_args.order = order_d;
    ga_args.position = position_d;
    ga_args.generation = generation_d;
    ga_args.next_dose = next_dose_d;
    ga_args.next_gap = next_gap_h_d;
    if (e == hipSuccess) e = gga::launch_offspring(ga_args, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_ga_generation(const gga_params* params, const gga_sim_cfg* cfg, const gga_ga_cfg* ga,
                      const gga_alphabet* a, const float* dose_d, const int32_t* gap_h_d,
                      const int32_t* nfrac_d, int32_t N, int32_t K, float* next_dose_d,
                      int32_t* next_gap_h_d, void* ws_d, size_t ws_bytes, float* hist_d,
                      int32_t hist_cap, int32_t advance, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    if ((rc = check_batch(N, K, cfg->R))) return rc;
    gga::GaArgs ga_args;
    if ((rc = check_ga(ga, a, N, K, &ga_args))) return rc;
    if (!dose_d || !gap_h_d || !nfrac_d || !next_dose_d || !next_gap_h_d || !ws_d) return GGA_E_ARG;
    if (ws_bytes < ga_ws_bytes(N, cfg->R) || hist_cap < 0 || (hist_cap > 0 && !hist_d)) return GGA_E_ARG;
    const hipError_t e = enqueue_generation(params, cfg, ga_args, dose_d, gap_h_d, nfrac_d, N, K, next_dose_d,
                                            next_gap_h_d, ga_ws(ws_d, N, cfg->R), hist_d, hist_cap, advance,
                                            stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_ga_run(const gga_params* params, const gga_sim_cfg* cfg, const gga_ga_cfg* ga, const gga_alphabet* a,
               float* dose_a_d, int32_t* gap_a_d, float* dose_b_d, int32_t* gap_b_d, const int32_t* nfrac_d,
               int32_t N, int32_t K, int32_t g0, int32_t n_gen, int32_t use_graph, void* ws_d,
               size_t ws_bytes, float* hist_d, float* gen_ms_h, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    if ((rc = check_batch(N, K, cfg->R))) return rc;
    gga::GaArgs ga_args;
    if ((rc = check_ga(ga, a, N, K, &ga_args))) return rc;
    if (!dose_a_d || !gap_a_d || !dose_b_d || !gap_b_d || !nfrac_d || !ws_d || n_gen < 0 || g0 < 0) return GGA_E_ARG;
    if ((long long)g0 + n_gen > std::numeric_limits<int32_t>::max()) return GGA_E_ARG;
    const int32_t hist_cap = g0 + n_gen;
    if (ws_bytes < ga_ws_bytes(N, cfg->R) || (n_gen > 0 && !hist_d)) return GGA_E_ARG;
    const GaWorkspace w = ga_ws(ws_d, N, cfg->R);
    float* pd[2] = {dose_a_d, dose_b_d};
    int32_t* pg[2] = {gap_a_d, gap_b_d};
    std::vector<hipEvent_t> ev(static_cast<size_t>(n_gen) + 1, nullptr);
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (auto& x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    if (e == hipSuccess && use_graph) {
        for (int d = 0; d < 2 && e == hipSuccess; ++d) {
            e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) break;
            const hipError_t ee = enqueue_generation(params, cfg, ga_args, pd[d], pg[d], nfrac_d, N, K, pd[1 - d],
                                                     pg[1 - d], w, hist_d, hist_cap, 1, stream);
            e = hipStreamEndCapture(stream, &graph[d]);
            if (ee != hipSuccess) e = ee;
            if (e == hipSuccess) e = hipGraphInstantiate(&exec[d], graph[d], nullptr, nullptr, 0);
        }
    }
    if (e == hipSuccess) e = gga::launch_counter(w.generation, g0, 0, stream);
    if (e == hipSuccess) e = hipEventRecord(ev[0], stream);
    for (int g = 0; g < n_gen && e == hipSuccess; ++g) {
        const int d = g & 1;
        if (use_graph) {
            e = hipGraphLaunch(exec[d], stream);
        } else {
            e = enqueue_generation(params, cfg, ga_args, pd[d], pg[d], nfrac_d, N, K, pd[1 - d], pg[1 - d], w,
                                   hist_d, hist_cap, 1, stream);
        }
        if (e == hipSuccess) e = hipEventRecord(ev[g + 1], stream);
        if (e == hipSuccess && !use_graph) e = hipStreamSynchronize(stream);   // host-driven loop
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    for (int g = 0; g < n_gen && e == hipSuccess && gen_ms_h; ++g) e = hipEventElapsedTime(&gen_ms_h[g], ev[0], ev[g + 1]);
    for (int d = 0; d < 2; ++d) {
        if (exec[d]) (void)hipGraphExecDestroy(exec[d]);
        if (graph[d]) (void)hipGraphDestroy(graph[d]);
    }
    for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

}  // extern "C"
