// Host side of the C ABI: argument checks, the host validator and launches.
// Every simulation step runs in the kernels; this file only checks and
// marshals arguments.
#include <cmath>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <limits>
#include <vector>

#include "gga_internal.h"
#include "quasi3d.h"
#include "mlp_internal.h"
#include "peaks.h"
#include "slots.h"

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
        if (!finite_in(p->kappa[f], 1e-30f, 1e30f)) return GGA_E_PARAM;   // positive: the field units divide by them
        if (!std::isfinite(p->ghost[f]) || !std::isfinite(p->init[f])) return GGA_E_PARAM;
    }
    for (int f = 1; f < 3; ++f) {   // rho_f = kappa_f / kappa_O, the field units' scale, well inside float range
        const double r = (double)p->kappa[f] / (double)p->kappa[0];
        if (!(r >= 1e-12 && r <= 1e12)) return GGA_E_PARAM;
    }
    for (int s = 0; s < 4; ++s)
        if (!finite_in(p->activity[s], 0.0f, 1e30f)) return GGA_E_PARAM;
    if (p->T_min < 0 || p->T_lys < 0 || p->A0 < 1 || p->seed_radius < 0) return GGA_E_PARAM;
    if (p->class_age[0] < 0 || p->class_age[1] < p->class_age[0]) return GGA_E_PARAM;
    if (!(p->P_div >= 0.0 && p->P_div <= 1.0)) return GGA_E_PARAM;
    if (!std::isfinite(p->alpha) || !std::isfinite(p->beta)) return GGA_E_PARAM;
    for (int c = 0; c < 4; ++c)
        if (!std::isfinite(p->m[c])) return GGA_E_PARAM;
    if (!(std::isfinite(p->repair_half_time) && p->repair_half_time >= 0.0)) return GGA_E_PARAM;
    if (!(std::isfinite(p->oer_max) && p->oer_max >= 1.0 && std::isfinite(p->oer_k) && p->oer_k > 0.0))
        return GGA_E_PARAM;
    if (p->oer_max > 1.0 && !(p->ghost[0] > 0.0f)) return GGA_E_PARAM;   // oxygen bins are fractions of ghost[0]
    if ((p->mitotic_death != 0 && p->mitotic_death != 1) || p->reserved != 0) return GGA_E_PARAM;
    return GGA_OK;
}

int check_cfg(const gga_sim_cfg* c) {
    if (!c) return GGA_E_ARG;
    if (c->struct_size != sizeof(gga_sim_cfg)) return GGA_E_ABI;
    if ((c->flags & ~GGA_SIM_HALF_HOUR) != 0 || c->R < 1 || c->horizon < 0 || c->horizon > (1 << 30)) return GGA_E_ARG;
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
    a.half = (cfg->flags & GGA_SIM_HALF_HOUR) ? 1 : 0;
    return a;
}

int check_any_side_cfg(const gga_sim_cfg* c) {
    if (!c) return GGA_E_ARG;
    if (c->struct_size != sizeof(gga_sim_cfg)) return GGA_E_ABI;
    if ((c->flags & ~GGA_SIM_HALF_HOUR) != 0 || c->R < 1 || c->horizon < 0 || c->horizon > (1 << 30)) return GGA_E_ARG;
    if (!std::isfinite(c->dose_cap)) return GGA_E_ARG;
    if (gga::side_index(c->L) < 0 || c->substeps < 1 || c->substeps > 64) return GGA_E_UNSUPPORTED;
    return GGA_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
bool misaligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) != 0; }

int slab_plan(int L, int RR, int H, gga::SimArgs* a);

// gga_simulate's workspace for a side without a resident variant: the event
// table (rows of GGA_KMAX fractions, so the size does not depend on K) and two
// state buffers of P * R instances (one read, the other written each step).
// Slab groups run as teams (the slabs of an instance co-resident, state kept
// on the CU for the whole horizon, halo rows exchanged through device memory)
// unless switched off by the test hook; the spin count bounds each wait.
std::atomic<int> g_use_teams{1};
std::atomic<int> g_spin_limit{1 << 21};

// Export rows of a slab plan for the team form: slab s publishes its own rows
// [i0, exA) (the slab above's bottom halo) and [exB, i1) (the slab below's top
// halo).  False when a halo row is not an own row of the adjacent slab.
bool team_plan(gga::SimArgs* a, int RR) {
    const int S = a->n_slabs;
    for (int s = 0; s < S; ++s) {
        const int ys = a->slab_ys[s], i0 = a->slab_i0[s], i1 = a->slab_i1[s];
        int exA = i0, exB = i1;
        if (s > 0) {
            const int lo = a->slab_ys[s - 1] + a->slab_i1[s - 1] - ys, hi = a->slab_ys[s - 1] + RR - ys;
            if (lo < i0 || hi > i1) return false;
            exA = hi;
        }
        if (s < S - 1) {
            const int lo = a->slab_ys[s + 1] - ys, hi = a->slab_ys[s + 1] + a->slab_i0[s + 1] - ys;
            if (lo < i0 || hi > i1) return false;
            exB = lo;
        }
        a->slab_exA[s] = exA;
        a->slab_exB[s] = exB;
    }
    return true;
}

// Whether slab variant v runs lattice side L with `substeps` sub-steps as teams.
bool uses_teams(int v, int L, int substeps) {
    if (!g_use_teams.load() || v < 0 || !gga::variant_is_slab(v)) return false;
    gga::SimArgs a;
    std::memset(&a, 0, sizeof(a));
    const int RR = gga::SIM_VARIANTS[v].rpt * gga::SIM_VARIANTS[v].nw;
    return slab_plan(L, RR, substeps + 2, &a) > 0 && team_plan(&a, RR);
}

// Instances whose state buffers a slab group keeps: all of them one step per
// launch, a team launch's worth as teams.
int32_t state_rows(bool teams, int32_t n) { return teams ? std::min<int32_t>(n, gga::TEAM_MAX) : n; }

// gga_simulate's workspace for a side without a resident variant: the event
// table (rows of GGA_KMAX fractions, so the size does not depend on K), the
// instance list, the teams' step counts and two state buffers (one per step
// parity) of the instances held at once.
struct SimWs {
    size_t off_valid, off_count, off_step, off_frac, off_list, off_flags, off_state, state_bytes, total;
    int32_t rows;
    bool teams;
};
SimWs simulate_ws_layout(int L, int substeps, int32_t P, int32_t R) {
    SimWs w{};
    w.teams = uses_teams(gga::variant_choice(L, false), L, substeps);
    w.rows = state_rows(w.teams, P * R);
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t at = off; off += align256(bytes); return at; };
    w.off_valid = take(sizeof(int32_t) * (size_t)P);
    w.off_count = take(sizeof(int32_t) * (size_t)P);
    w.off_step = take(sizeof(int32_t) * (size_t)P * GGA_KMAX);
    w.off_frac = take(sizeof(gga::EventFraction) * (size_t)P * GGA_KMAX);
    w.off_list = take(w.teams ? sizeof(int32_t) * (size_t)P * R : 0);
    w.off_flags = take(w.teams ? sizeof(int32_t) * (size_t)gga::TEAM_MAX * gga::MAX_SLABS : 0);
    w.state_bytes = align256((size_t)L * L * (3 * sizeof(float) + sizeof(uint16_t)) * (size_t)w.rows);
    w.off_state = take(2 * w.state_bytes);
    w.total = off;
    return w;
}

// The instances at list positions 0 .. n-1 of a.inst_list as teams of slab
// variant v, in cooperative launches of as many teams as the device holds at
// once (at most `rows`, the instances the state buffers hold), each for its
// instances' whole horizons.  a carries the slab plan with its export rows.
hipError_t enqueue_teams(gga::SimArgs a, int v, int n, int rows, char* state, size_t state_bytes, int L,
                         int32_t* flags, hipStream_t stream) {
    int cap = 0;
    hipError_t e = gga::launch_team_variant(v, a, 0, &cap, stream);
    if (e != hipSuccess) return e;
    const int teams = std::min(8 * (cap / (8 * a.n_slabs)), rows);
    if (teams < 1) return hipErrorInvalidConfiguration;
    const size_t fbytes = (size_t)L * L * 3 * sizeof(float) * (size_t)rows;
    a.fields = reinterpret_cast<float*>(state);
    a.cells = reinterpret_cast<uint16_t*>(state + fbytes);
    a.fields_out = reinterpret_cast<float*>(state + state_bytes);
    a.cells_out = reinterpret_cast<uint16_t*>(state + state_bytes + fbytes);
    a.team_flags = flags;
    a.spin_limit = g_spin_limit.load();
    a.mode = 0;
    a.n0 = 0;
    const int32_t* list = a.inst_list;
    for (int k0 = 0; k0 < n && e == hipSuccess; k0 += teams) {
        const int m = std::min(teams, n - k0);
        a.inst_list = list + k0;
        a.n_active = m;
        e = gga::launch_fill(flags, m * a.n_slabs, 0, stream);
        if (e == hipSuccess) e = gga::launch_team_variant(v, a, gga::slab_blocks(m, a.n_slabs), &cap, stream);
    }
    return e;
}

// Slab-form simulation of all P * R instances for cfg->horizon steps: event
// table and live counts, then teams over whole horizons, or (teams off) the
// initial state and one launch per step alternating the two state buffers;
// the live count of the last step (and of every step into traj) is summed
// over the slabs.
hipError_t enqueue_simulate_slabs(gga::SimArgs a, const gga_sim_cfg* cfg, int32_t P, int32_t K, char* ws,
                                  const SimWs& w, hipStream_t stream) {
    const int v = gga::variant_choice(cfg->L, false);
    if (v < 0 || !gga::variant_is_slab(v)) return hipErrorInvalidValue;
    const gga::SimVariant& var = gga::SIM_VARIANTS[v];
    const int RR = var.rpt * var.nw;
    if (slab_plan(cfg->L, RR, cfg->substeps + 2, &a) <= 0) return hipErrorInvalidValue;
    if (w.teams && !team_plan(&a, RR)) return hipErrorInvalidValue;
    int32_t* valid = reinterpret_cast<int32_t*>(ws + w.off_valid);
    int32_t* count = reinterpret_cast<int32_t*>(ws + w.off_count);
    int32_t* step = reinterpret_cast<int32_t*>(ws + w.off_step);
    gga::EventFraction* frac = reinterpret_cast<gga::EventFraction*>(ws + w.off_frac);
    a.ev_valid = valid;
    a.ev_count = count;
    a.ev_step = step;
    a.ev_frac = frac;
    a.count_at = cfg->horizon;
    a.mode = 0;
    const int n = P * cfg->R;
    hipError_t e = gga::launch_event_table(a, P, valid, count, step, frac, stream);
    if (e == hipSuccess && a.traj) e = gga::launch_fill(a.traj, n * cfg->horizon, 0, stream);
    if (w.teams) {
        int32_t* list = reinterpret_cast<int32_t*>(ws + w.off_list);
        if (e == hipSuccess) e = gga::launch_iota(list, n, stream);
        a.inst_list = list;
        a.nsteps = cfg->horizon;
        if (e == hipSuccess) e = gga::launch_slab_live(a, n, stream);
        if (e == hipSuccess)
            e = enqueue_teams(a, v, n, w.rows, ws + w.off_state, w.state_bytes, cfg->L,
                              reinterpret_cast<int32_t*>(ws + w.off_flags), stream);
        return e;
    }
    const size_t fbytes = (size_t)cfg->L * cfg->L * 3 * sizeof(float) * (size_t)n;
    char* s0 = ws + w.off_state;
    char* s1 = s0 + w.state_bytes;
    float* fa = reinterpret_cast<float*>(s0);
    uint16_t* ca = reinterpret_cast<uint16_t*>(s0 + fbytes);
    float* fb = reinterpret_cast<float*>(s1);
    uint16_t* cb = reinterpret_cast<uint16_t*>(s1 + fbytes);
    if (e == hipSuccess) e = gga::launch_slab_init(a, cfg->L, n, fa, ca, stream);
    for (int32_t t = 0; t < cfg->horizon && e == hipSuccess; ++t) {
        a.n0 = t;
        a.nsteps = 1;
        a.fields = (t & 1) ? fb : fa;
        a.cells = (t & 1) ? cb : ca;
        a.fields_out = (t & 1) ? fa : fb;
        a.cells_out = (t & 1) ? ca : cb;
        a.n_active = n;
        e = gga::launch_variant(v, a, gga::slab_blocks(n, a.n_slabs), stream);
    }
    return e;
}

}  // namespace

namespace gga {
int hip_error(hipError_t e) { return hip_fail(e); }

// The parameter check of the simulation calls, for the JSON reader.
int check_params_host(const gga_params* p) { return check_params(p); }
}  // namespace gga

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
        case GGA_E_SCRATCH: return "batch needs more than the no-allocation entry point's fixed scratch";
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

size_t gga_workspace_bytes(const gga_sim_cfg* cfg, int32_t P) {
    if (!cfg || cfg->struct_size != sizeof(gga_sim_cfg) || check_batch(P, 0, cfg->R) || cfg->R < 1) return 0;
    if (gga::side_index(cfg->L) < 0 || gga::sim_supported(cfg->L)) return 0;   // resident: state stays on the CU
    return simulate_ws_layout(cfg->L, cfg->substeps, P, cfg->R).total;
}

int gga_simulate(const gga_params* params, const gga_sim_cfg* cfg, const float* dose_d,
                 const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P, int32_t K, void* ws_d,
                 size_t ws_bytes, int32_t* live_d, float* fitness_d, int32_t* traj_d, hipStream_t stream) {
    return gga::simulate_checked(params, cfg, dose_d, gap_h_d, nfrac_d, P, K, ws_d, ws_bytes, live_d, fitness_d,
                                 traj_d, stream);
}

}  // extern "C"

int gga::simulate_checked(const gga_params* params, const gga_sim_cfg* cfg, const float* dose_d,
                          const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P, int32_t K, void* ws_d,
                          size_t ws_bytes, int32_t* live_d, float* fitness_d, int32_t* traj_d, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_any_side_cfg(cfg))) return rc;
    if ((rc = check_batch(P, K, cfg->R))) return rc;
    if (P == 0) return GGA_OK;
    if (!nfrac_d || !live_d || !fitness_d || (K > 0 && (!dose_d || !gap_h_d))) return GGA_E_ARG;
    gga::SimArgs a = make_args(params, cfg, dose_d, gap_h_d, nfrac_d, K);
    a.live = live_d;
    a.traj = traj_d;
    hipError_t e = hipSuccess;
    if (gga::sim_supported(cfg->L)) {                // resident: one launch for the whole horizon
        a.n0 = 0;
        a.nsteps = cfg->horizon;
        a.mode = 0;
        e = gga::launch_simulation(a, cfg->L, P * cfg->R, stream);
    } else {                                         // slabs: state in the workspace, as teams or per step
        const SimWs w = simulate_ws_layout(cfg->L, cfg->substeps, P, cfg->R);
        if (!ws_d || misaligned16(ws_d) || ws_bytes < w.total) return GGA_E_ARG;
        if (traj_d && (long long)P * cfg->R * cfg->horizon > std::numeric_limits<int32_t>::max()) return GGA_E_ARG;
        e = enqueue_simulate_slabs(a, cfg, P, K, static_cast<char*>(ws_d), w, stream);
    }
    if (e == hipSuccess) e = gga::launch_fitness(live_d, P, cfg->R, fitness_d, stream);
    return e == hipSuccess ? GGA_OK : (e == hipErrorInvalidValue ? GGA_E_UNSUPPORTED : hip_fail(e));
}

extern "C" {

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

int gga_simulate_library(const gga_params* params, const gga_sim_cfg* cfg, const float* dose_d,
                         const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P, int32_t K,
                         const float* lib_fields_d, const uint16_t* lib_cells_d, int32_t n_lib, int32_t* live_d,
                         float* fitness_d, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    if ((rc = check_batch(P, K, cfg->R))) return rc;
    if (n_lib < 1) return GGA_E_ARG;
    if (P == 0) return GGA_OK;
    if (!nfrac_d || !live_d || !fitness_d || !lib_fields_d || !lib_cells_d || (K > 0 && (!dose_d || !gap_h_d)))
        return GGA_E_ARG;
    gga::SimArgs a = make_args(params, cfg, dose_d, gap_h_d, nfrac_d, K);
    a.n0 = 0;
    a.nsteps = cfg->horizon;
    a.mode = gga::MODE_LOAD;                       // read-only: the library is not written
    a.fields = const_cast<float*>(lib_fields_d);
    a.cells = const_cast<uint16_t*>(lib_cells_d);
    a.lib_n = n_lib;
    a.live = live_d;
    hipError_t e = gga::launch_simulation(a, cfg->L, P * cfg->R, stream);
    if (e == hipSuccess) e = gga::launch_fitness(live_d, P, cfg->R, fitness_d, stream);
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

// Selection, crossover and probability settings shared by both GAs; fills the
// matching fields of *out (zeroing the rest).
int check_ga_ops(const gga_ga_cfg* ga, int32_t N, gga::GaArgs* out) {
    if (!ga) return GGA_E_ARG;
    if (ga->struct_size != sizeof(gga_ga_cfg)) return GGA_E_ABI;
    if (N < 2) return GGA_E_ARG;
    if (ga->n_elite < 0 || ga->n_elite > N || ga->tournament_k < 1 || ga->tournament_k > 64) return GGA_E_ARG;
    if (!(ga->p_cross >= 0.0 && ga->p_cross <= 1.0) || !(ga->p_mut >= 0.0 && ga->p_mut <= 1.0)) return GGA_E_ARG;
    if (ga->selection < 0 || ga->selection > 3 || ga->crossover < 0 || ga->crossover > 3 || ga->reserved != 0)
        return GGA_E_ARG;
    if (ga->selection == GGA_SEL_RANK && !(ga->q > 0.0 && ga->q <= 1.0)) return GGA_E_ARG;
    if (ga->selection == GGA_SEL_TRUNCATION && !(ga->trunc_frac > 0.0 && ga->trunc_frac <= 1.0)) return GGA_E_ARG;
    if (ga->selection == GGA_SEL_ROULETTE && !std::isfinite(ga->roulette_base)) return GGA_E_ARG;
    std::memset(out, 0, sizeof(*out));
    out->N = N;
    out->n_out = N;
    out->n_elite = ga->n_elite;
    out->k = ga->tournament_k;
    out->t_cross = prob_threshold(ga->p_cross);
    out->t_mut = prob_threshold(ga->p_mut);
    out->selection = ga->selection;
    out->crossover = ga->crossover;
    out->t_q = ga->selection == GGA_SEL_RANK ? prob_threshold(ga->q) : 0u;
    out->trunc_m = ga->selection == GGA_SEL_TRUNCATION
                       ? std::max(1, std::min(N, static_cast<int>(std::floor(ga->trunc_frac * N))))
                       : 0;
    out->roulette_base = ga->roulette_base;
    out->seed_lo = static_cast<uint32_t>(ga->seed);
    out->seed_hi = static_cast<uint32_t>(ga->seed >> 32);
    return GGA_OK;
}

int check_ga(const gga_ga_cfg* ga, const gga_alphabet* a, int32_t N, int32_t K, gga::GaArgs* out) {
    if (!ga || !a) return GGA_E_ARG;
    if (ga->struct_size != sizeof(gga_ga_cfg) || a->struct_size != sizeof(gga_alphabet)) return GGA_E_ABI;
    if (K < 1 || K > GGA_KMAX || ga->mutation < 0 || ga->mutation > 7) return GGA_E_ARG;
    const int rc = check_ga_ops(ga, N, out);
    if (rc) return rc;
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
    out->K = K;
    out->n_dose = a->n_dose;
    out->n_gap = a->n_gap;
    out->cap_q = static_cast<int32_t>(capq);
    out->mutation = ga->mutation ? ga->mutation : GGA_MUT_GENE;
    out->quantum = a->dose_quantum;
    std::memcpy(out->dose_q, a->dose_q, sizeof(out->dose_q));
    std::memcpy(out->gaps, a->gaps, sizeof(out->gaps));
    return GGA_OK;
}

int check_slots(const gga_slot_cfg* sc) {
    if (!sc) return GGA_E_ARG;
    if (sc->struct_size != sizeof(gga_slot_cfg)) return GGA_E_ABI;
    if (sc->S < 1 || sc->S > GGA_SLOTS_MAX || sc->g_min < 1 || sc->g_min > sc->S) return GGA_E_ARG;
    if (sc->dmax_q < 1 || sc->dmax_q > 255 || sc->cap_q < 0 || sc->cap_q > 65535) return GGA_E_ARG;
    if (sc->mutation < 0 || sc->mutation > 15 || sc->reserved != 0) return GGA_E_ARG;
    if (!(std::isfinite(sc->quantum) && sc->quantum > 0.0f)) return GGA_E_ARG;
    return GGA_OK;
}

// Slot GA arguments from checked settings.
gga::SlotArgs slot_args(const gga::GaArgs& ops, const gga_slot_cfg* sc) {
    gga::SlotArgs a;
    std::memset(&a, 0, sizeof(a));
    a.sel = ops;
    a.S = sc->S;
    a.g_min = sc->g_min;
    a.dmax = sc->dmax_q;
    a.cap_q = sc->cap_q;
    a.mutation = sc->mutation ? sc->mutation : (GGA_SMUT_SWAP | GGA_SMUT_SPLIT | GGA_SMUT_TIME);
    a.quantum = sc->quantum;
    return a;
}

// Enqueue one generation; all arguments already checked.
hipError_t enqueue_generation(const gga_params* params, const gga_sim_cfg* cfg, gga::GaArgs ga_args,
                              const float* dose, const int32_t* gap, const int32_t* nfrac, int32_t N,
                              int32_t K, float* next_dose, int32_t* next_gap, const GaWorkspace& w,
                              float* hist, int32_t hist_cap, float* best_dose, int32_t* best_gap, int32_t advance,
                              hipStream_t stream) {
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
    const gga::Archive arc{dose, gap, K, best_dose, best_gap};
    if (e == hipSuccess) e = gga::launch_history(w.fitness, N, w.order, w.generation, hist, hist_cap, arc, stream);
    ga_args.fitness = w.fitness;
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

// Run generations g0 .. g0+n_gen-1 of enqueue(d) (d = generation parity):
// host-driven (enqueue, wait) or as two captured hipGraphs replayed back to
// back.  gen_ms[g] = time from the start to the end of generation g0 + g.
template <class F>
hipError_t run_generations(F enqueue, int32_t* counter, int32_t g0, int32_t n_gen, int32_t use_graph,
                           float* gen_ms, hipStream_t stream) {
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
            const hipError_t ee = enqueue(d);
            e = hipStreamEndCapture(stream, &graph[d]);
            if (ee != hipSuccess) e = ee;
            if (e == hipSuccess) e = hipGraphInstantiate(&exec[d], graph[d], nullptr, nullptr, 0);
        }
    }
    if (e == hipSuccess) e = gga::launch_counter(counter, g0, 0, stream);
    if (e == hipSuccess) e = hipEventRecord(ev[0], stream);
    for (int g = 0; g < n_gen && e == hipSuccess; ++g) {
        e = use_graph ? hipGraphLaunch(exec[g & 1], stream) : enqueue(g & 1);
        if (e == hipSuccess) e = hipEventRecord(ev[g + 1], stream);
        if (e == hipSuccess && !use_graph) e = hipStreamSynchronize(stream);   // host-driven loop
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    for (int g = 0; g < n_gen && e == hipSuccess && gen_ms; ++g) e = hipEventElapsedTime(&gen_ms[g], ev[0], ev[g + 1]);
    for (int d = 0; d < 2; ++d) {
        if (exec[d]) (void)hipGraphExecDestroy(exec[d]);
        if (graph[d]) (void)hipGraphDestroy(graph[d]);
    }
    for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    return e;
}

struct SlotWorkspace {
    GaWorkspace ga;
    float* dose;
    int32_t* gap;
    int32_t* nfrac;
};

size_t slots_ws_bytes(int32_t N, int32_t R, int32_t K) {
    return ga_ws_bytes(N, R) + 2 * align256(sizeof(int32_t) * (size_t)N * K) + align256(sizeof(int32_t) * (size_t)N);
}

SlotWorkspace slots_ws(void* ws, int32_t N, int32_t R, int32_t K) {
    SlotWorkspace w;
    w.ga = ga_ws(ws, N, R);
    char* p = static_cast<char*>(ws) + ga_ws_bytes(N, R);
    w.dose = reinterpret_cast<float*>(p);
    p += align256(sizeof(int32_t) * (size_t)N * K);
    w.gap = reinterpret_cast<int32_t*>(p);
    p += align256(sizeof(int32_t) * (size_t)N * K);
    w.nfrac = reinterpret_cast<int32_t*>(p);
    return w;
}

// Enqueue one slot-GA generation (decode, simulate, fitness, rank, history,
// breed); all arguments already checked.
hipError_t enqueue_slot_generation(const gga_params* params, const gga_sim_cfg* cfg, gga::SlotArgs sl,
                                   const uint8_t* pop, int32_t N, int32_t K, uint8_t* next, const SlotWorkspace& w,
                                   float* hist, int32_t hist_cap, float* best_dose, int32_t* best_gap,
                                   int32_t advance, hipStream_t stream) {
    hipError_t e = gga::launch_slot_decode(pop, N, sl.S, K, sl.quantum, w.dose, w.gap, w.nfrac, stream);
    gga::SimArgs sa = make_args(params, cfg, w.dose, w.gap, w.nfrac, K);
    sa.n0 = 0;
    sa.nsteps = cfg->horizon;
    sa.mode = 0;
    sa.live = w.ga.live;
    sa.generation = w.ga.generation;
    sa.seed = cfg->seed;
    if (e == hipSuccess) e = gga::launch_simulation(sa, cfg->L, N * cfg->R, stream);
    if (e == hipSuccess) e = gga::launch_fitness(w.ga.live, N, cfg->R, w.ga.fitness, stream);
    if (e == hipSuccess) e = gga::launch_rank(w.ga.fitness, N, w.ga.order, w.ga.position, stream);
    const gga::Archive arc{w.dose, w.gap, K, best_dose, best_gap};
    if (e == hipSuccess)
        e = gga::launch_history(w.ga.fitness, N, w.ga.order, w.ga.generation, hist, hist_cap, arc, stream);
    sl.sel.fitness = w.ga.fitness;
    sl.sel.order = w.ga.order;
    sl.sel.position = w.ga.position;
    sl.sel.generation = w.ga.generation;
    sl.pop = pop;
    sl.next = next;
    if (e == hipSuccess) e = gga::launch_slot_offspring(sl, stream);
    if (e == hipSuccess && advance) e = gga::launch_counter(w.ga.generation, 1, 1, stream);
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
    ga_args.fitness = fitness_d;
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
                                            next_gap_h_d, ga_ws(ws_d, N, cfg->R), hist_d, hist_cap, nullptr,
                                            nullptr, advance, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_ga_run(const gga_params* params, const gga_sim_cfg* cfg, const gga_ga_cfg* ga, const gga_alphabet* a,
               float* dose_a_d, int32_t* gap_a_d, float* dose_b_d, int32_t* gap_b_d, const int32_t* nfrac_d,
               int32_t N, int32_t K, int32_t g0, int32_t n_gen, int32_t use_graph, void* ws_d,
               size_t ws_bytes, float* hist_d, float* best_dose_d, int32_t* best_gap_d, float* gen_ms_h,
               hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    if ((rc = check_batch(N, K, cfg->R))) return rc;
    if (!best_dose_d != !best_gap_d) return GGA_E_ARG;
    gga::GaArgs ga_args;
    if ((rc = check_ga(ga, a, N, K, &ga_args))) return rc;
    if (!dose_a_d || !gap_a_d || !dose_b_d || !gap_b_d || !nfrac_d || !ws_d || n_gen < 0 || g0 < 0) return GGA_E_ARG;
    if ((long long)g0 + n_gen > std::numeric_limits<int32_t>::max()) return GGA_E_ARG;
    const int32_t hist_cap = g0 + n_gen;
    if (ws_bytes < ga_ws_bytes(N, cfg->R) || (n_gen > 0 && !hist_d)) return GGA_E_ARG;
    const GaWorkspace w = ga_ws(ws_d, N, cfg->R);
    float* pd[2] = {dose_a_d, dose_b_d};
    int32_t* pg[2] = {gap_a_d, gap_b_d};
    auto enqueue = [&](int d) {
        return enqueue_generation(params, cfg, ga_args, pd[d], pg[d], nfrac_d, N, K, pd[1 - d], pg[1 - d], w,
                                  hist_d, hist_cap, best_dose_d, best_gap_d, 1, stream);
    };
    const hipError_t e = run_generations(enqueue, w.generation, g0, n_gen, use_graph, gen_ms_h, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_slots_breed(const gga_ga_cfg* ga, const gga_slot_cfg* sc, const float* fitness_d, const uint8_t* pop_d,
                    int32_t N, const int32_t* generation_d, int32_t* order_d, int32_t* position_d, uint8_t* next_d,
                    hipStream_t stream) {
    int rc = check_slots(sc);
    if (rc) return rc;
    gga::GaArgs ops;
    if ((rc = check_ga_ops(ga, N, &ops))) return rc;
    if (ga->mutation != 0) return GGA_E_ARG;
    if (!fitness_d || !pop_d || !generation_d || !order_d || !position_d || !next_d || next_d == pop_d)
        return GGA_E_ARG;
    gga::SlotArgs a = slot_args(ops, sc);
    a.sel.fitness = fitness_d;
    a.sel.order = order_d;
    a.sel.position = position_d;
    a.sel.generation = generation_d;
    a.pop = pop_d;
    a.next = next_d;
    hipError_t e = gga::launch_rank(fitness_d, N, order_d, position_d, stream);
    if (e == hipSuccess) e = gga::launch_slot_offspring(a, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_slots_decode(const gga_slot_cfg* sc, const uint8_t* pop_d, int32_t P, int32_t K, float* dose_d,
                     int32_t* gap_h_d, int32_t* nfrac_d, hipStream_t stream) {
    const int rc = check_slots(sc);
    if (rc) return rc;
    if (P < 0 || K < 1 || K > GGA_KMAX || (long long)P * std::max(sc->S, K) > std::numeric_limits<int32_t>::max())
        return GGA_E_ARG;
    if (P > 0 && (!pop_d || !dose_d || !gap_h_d || !nfrac_d)) return GGA_E_ARG;
    const hipError_t e = gga::launch_slot_decode(pop_d, P, sc->S, K, sc->quantum, dose_d, gap_h_d, nfrac_d, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_slots_encode(const gga_slot_cfg* sc, const float* dose_d, const int32_t* gap_h_d, const int32_t* nfrac_d,
                     int32_t P, int32_t K, uint8_t* pop_d, hipStream_t stream) {
    const int rc = check_slots(sc);
    if (rc) return rc;
    if (P < 0 || K < 1 || K > GGA_KMAX || (long long)P * std::max(sc->S, K) > std::numeric_limits<int32_t>::max())
        return GGA_E_ARG;
    if (P > 0 && (!pop_d || !dose_d || !gap_h_d || !nfrac_d)) return GGA_E_ARG;
    const hipError_t e = gga::launch_slot_encode(dose_d, gap_h_d, nfrac_d, P, K, sc->S, sc->quantum, sc->g_min,
                                                 sc->dmax_q, sc->cap_q, pop_d, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

size_t gga_slots_workspace_bytes(int32_t N, int32_t R, int32_t K) {
    if (N < 0 || R < 1 || K < 1 || K > GGA_KMAX) return 0;
    return slots_ws_bytes(N, R, K);
}

int gga_slots_run(const gga_params* params, const gga_sim_cfg* cfg, const gga_ga_cfg* ga, const gga_slot_cfg* sc,
                  uint8_t* pop_a_d, uint8_t* pop_b_d, int32_t N, int32_t K, int32_t g0, int32_t n_gen,
                  int32_t use_graph, void* ws_d, size_t ws_bytes, float* hist_d, float* best_dose_d,
                  int32_t* best_gap_d, float* gen_ms_h, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    if ((rc = check_slots(sc))) return rc;
    if (K < 1 || (rc = check_batch(N, K, cfg->R))) return rc ? rc : GGA_E_ARG;
    if ((long long)K * sc->g_min < sc->S) return GGA_E_ARG;              // K >= ceil(S / g_min)
    if ((double)sc->cap_q * (double)sc->quantum > cfg->dose_cap + 1e-6) return GGA_E_ARG;
    gga::GaArgs ops;
    if ((rc = check_ga_ops(ga, N, &ops))) return rc;
    if (ga->mutation != 0) return GGA_E_ARG;
    if (!best_dose_d != !best_gap_d) return GGA_E_ARG;
    if (!pop_a_d || !pop_b_d || pop_a_d == pop_b_d || !ws_d || n_gen < 0 || g0 < 0) return GGA_E_ARG;
    if ((long long)g0 + n_gen > std::numeric_limits<int32_t>::max()) return GGA_E_ARG;
    if ((long long)N * sc->S > std::numeric_limits<int32_t>::max()) return GGA_E_ARG;
    const int32_t hist_cap = g0 + n_gen;
    if (ws_bytes < slots_ws_bytes(N, cfg->R, K) || (n_gen > 0 && !hist_d)) return GGA_E_ARG;
    const SlotWorkspace w = slots_ws(ws_d, N, cfg->R, K);
    const gga::SlotArgs sl = slot_args(ops, sc);
    uint8_t* pop[2] = {pop_a_d, pop_b_d};
    auto enqueue = [&](int d) {
        return enqueue_slot_generation(params, cfg, sl, pop[d], N, K, pop[1 - d], w, hist_d, hist_cap, best_dose_d,
                                       best_gap_d, 1, stream);
    };
    const hipError_t e = run_generations(enqueue, w.ga.generation, g0, n_gen, use_graph, gen_ms_h, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

}  // extern "C"

// ------------------------------------------------------------------ surrogate MLP

namespace gga {

namespace {
struct Layout {
    size_t norm, p, m, v, g, wb[3], wtb[3], total;
};
Layout net_layout() {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t at = off; off += align256(bytes); return at; };
    L.norm = take(2 * sizeof(float) + sizeof(int32_t));
    L.p = take(sizeof(float) * MLP_PARAMS);
    L.m = take(sizeof(float) * MLP_PARAMS);
    L.v = take(sizeof(float) * MLP_PARAMS);
    L.g = take(sizeof(float) * MLP_PARAMS);
    for (int l = 0; l < 3; ++l) {
        const size_t k = l == 0 ? MLP_IN : MLP_HID;
        L.wb[l] = take(sizeof(uint16_t) * k * MLP_HID);
        L.wtb[l] = take(sizeof(uint16_t) * k * MLP_HID);
    }
    L.total = off;
    return L;
}
}  // namespace

size_t mlp_net_bytes() { return net_layout().total; }

MlpNet mlp_net(void* base) {
    const Layout L = net_layout();
    char* c = static_cast<char*>(base);
    MlpNet n{};
    n.norm = reinterpret_cast<float*>(c + L.norm);
    n.step = reinterpret_cast<int32_t*>(c + L.norm + 2 * sizeof(float));
    n.p = reinterpret_cast<float*>(c + L.p);
    n.m = reinterpret_cast<float*>(c + L.m);
    n.v = reinterpret_cast<float*>(c + L.v);
    n.g = reinterpret_cast<float*>(c + L.g);
    float* p = n.p;
    float* g = n.g;
    for (int l = 0; l < 3; ++l) {
        const long k = l == 0 ? MLP_IN : MLP_HID;
        n.Wf[l] = p;
        n.gW[l] = g;
        p += k * MLP_HID;
        g += k * MLP_HID;
        n.b[l] = p;
        n.gb[l] = g;
        p += MLP_HID;
        g += MLP_HID;
        n.W[l] = reinterpret_cast<__bf16*>(c + L.wb[l]);
        n.WT[l] = reinterpret_cast<__bf16*>(c + L.wtb[l]);
    }
    n.w4 = p;
    n.gw4 = g;
    n.b4 = p + MLP_HID;
    n.gb4 = g + MLP_HID;
    return n;
}

// Byte offsets of X, Z[3], H[3], y, dy, dZ[2] and part in a work buffer of batch B.
void mlp_work_offsets(int B, size_t (&off)[12]) {
    const size_t b = static_cast<size_t>(B);
    size_t at = 0;
    auto take = [&](size_t bytes) { const size_t o = at; at += align256(bytes); return o; };
    off[0] = take(2 * b * MLP_IN);
    for (int l = 0; l < 3; ++l) off[1 + l] = take(4 * b * MLP_HID);
    for (int l = 0; l < 3; ++l) off[4 + l] = take(2 * b * MLP_HID);
    off[7] = take(4 * b);
    off[8] = take(4 * b);
    for (int l = 0; l < 2; ++l) off[9 + l] = take(2 * b * MLP_HID);
    off[11] = take(4 * MLP_RED_CHUNKS * (MLP_HID + 1));
}

size_t mlp_work_bytes(int B) {
    size_t off[12];
    mlp_work_offsets(B, off);
    return off[11] + align256(4 * MLP_RED_CHUNKS * (MLP_HID + 1));
}

MlpWork mlp_work(void* base, int B) {
    size_t off[12];
    mlp_work_offsets(B, off);
    char* c = static_cast<char*>(base);
    MlpWork w{};
    w.X = reinterpret_cast<__bf16*>(c + off[0]);
    for (int l = 0; l < 3; ++l) w.Z[l] = reinterpret_cast<float*>(c + off[1 + l]);
    for (int l = 0; l < 3; ++l) w.H[l] = reinterpret_cast<__bf16*>(c + off[4 + l]);
    w.y = reinterpret_cast<float*>(c + off[7]);
    w.dy = reinterpret_cast<float*>(c + off[8]);
    for (int l = 0; l < 2; ++l) w.dZ[l] = reinterpret_cast<__bf16*>(c + off[9 + l]);
    w.part = reinterpret_cast<float*>(c + off[11]);
    return w;
}

}  // namespace gga

namespace {

int mlp_check(const void* net, int32_t B, int32_t K, const float* dose, const int32_t* gap, const int32_t* nfrac,
              const void* work, size_t work_bytes) {
    if (!net || misaligned16(net) || misaligned16(work) || B < 0 || K < 0 || K > GGA_KMAX) return GGA_E_ARG;
    if (B > 0 && (!nfrac || !work || (K > 0 && (!dose || !gap)))) return GGA_E_ARG;
    if ((long long)B * gga::MLP_HID > std::numeric_limits<int32_t>::max()) return GGA_E_ARG;
    if (B > 0 && work_bytes < gga::mlp_work_bytes(B)) return GGA_E_ARG;
    return GGA_OK;
}
}  // namespace

extern "C" {

size_t gga_mlp_net_bytes(void) { return gga::mlp_net_bytes(); }

size_t gga_mlp_work_bytes(int32_t B) { return B < 0 ? 0 : gga::mlp_work_bytes(B); }

int gga_mlp_work_layout(int32_t B, size_t* offsets) {
    if (B < 0 || !offsets) return GGA_E_ARG;
    size_t off[12];
    gga::mlp_work_offsets(B, off);
    for (int i = 0; i < 12; ++i) offsets[i] = off[i];
    return GGA_OK;
}

int gga_mlp_init(void* net_d, uint64_t seed, hipStream_t stream) {
    if (!net_d || misaligned16(net_d)) return GGA_E_ARG;
    const gga::MlpNet net = gga::mlp_net(net_d);
    hipError_t e = gga::mlp_init(net, seed, stream);
    // normalisation defaults to (0, 1) until gga_mlp_set_norm; Adam step 0
    static const float unit[3] = {0.0f, 1.0f, 0.0f};
    if (e == hipSuccess) e = hipMemcpyAsync(net.norm, unit, sizeof(unit), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_mlp_set_norm(void* net_d, const float* target_d, int32_t n, hipStream_t stream) {
    if (!net_d || misaligned16(net_d) || n < 1 || !target_d) return GGA_E_ARG;
    const hipError_t e = gga::mlp_set_norm(gga::mlp_net(net_d), target_d, n, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_mlp_predict(const void* net_d, const float* dose_d, const int32_t* gap_h_d, const int32_t* nfrac_d,
                    int32_t B, int32_t K, void* work_d, size_t work_bytes, float* pred_d, hipStream_t stream) {
    const int rc = mlp_check(net_d, B, K, dose_d, gap_h_d, nfrac_d, work_d, work_bytes);
    if (rc) return rc;
    if (B == 0) return GGA_OK;
    if (!pred_d) return GGA_E_ARG;
    const hipError_t e = gga::mlp_forward(gga::mlp_net(const_cast<void*>(net_d)), dose_d, gap_h_d, nfrac_d, B, K,
                                          gga::mlp_work(work_d, B), pred_d, true, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_mlp_grad(void* net_d, const float* dose_d, const int32_t* gap_h_d, const int32_t* nfrac_d,
                 const float* target_d, int32_t B, int32_t K, void* work_d, size_t work_bytes, float* loss_d,
                 hipStream_t stream) {
    const int rc = mlp_check(net_d, B, K, dose_d, gap_h_d, nfrac_d, work_d, work_bytes);
    if (rc) return rc;
    if (B < 1 || !target_d) return GGA_E_ARG;
    const gga::MlpNet net = gga::mlp_net(net_d);
    const gga::MlpWork w = gga::mlp_work(work_d, B);
    hipError_t e = gga::mlp_forward(net, dose_d, gap_h_d, nfrac_d, B, K, w, w.y, false, stream);
    if (e == hipSuccess) e = gga::mlp_backward(net, B, target_d, w, loss_d, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_mlp_train_step(void* net_d, const float* dose_d, const int32_t* gap_h_d, const int32_t* nfrac_d,
                       const float* target_d, int32_t B, int32_t K, int32_t step, float lr, void* work_d,
                       size_t work_bytes, float* loss_d, hipStream_t stream) {
    if (step < 1 || !(lr > 0.0f) || !std::isfinite(lr)) return GGA_E_ARG;
    int rc = gga_mlp_grad(net_d, dose_d, gap_h_d, nfrac_d, target_d, B, K, work_d, work_bytes, loss_d, stream);
    if (rc) return rc;
    const hipError_t e = gga::mlp_adam_refresh(gga::mlp_net(net_d), step, lr, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_measure_peaks(void* buf_d, size_t bytes, double* valu_ops_h, double* lds_bytes_h, double* hbm_bytes_h,
                      hipStream_t stream) {
    if (!buf_d || (reinterpret_cast<uintptr_t>(buf_d) & 15) || bytes < ((size_t)256 << 20) + 256 || !valu_ops_h ||
        !lds_bytes_h || !hbm_bytes_h)
        return GGA_E_ARG;
    const hipError_t e = gga::measure_peaks(buf_d, bytes, valu_ops_h, lds_bytes_h, hbm_bytes_h, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_mlp_gemm(int32_t M, int32_t N, int32_t K, const void* A_d, int32_t a_trans, const void* B_d,
                 int32_t b_trans, float* C_d, hipStream_t stream) {
    if (M < 0 || N < 0 || K < 0 || (M > 0 && N > 0 && (!C_d || (K > 0 && (!A_d || !B_d))))) return GGA_E_ARG;
    gga::MlpGemm g{};
    g.M = M; g.N = N; g.K = K;
    g.A = static_cast<const __bf16*>(A_d);
    g.sa_m = a_trans ? 1 : K;        // A stored [M][K], or [K][M] when transposed
    g.sa_k = a_trans ? M : 1;
    g.B = static_cast<const __bf16*>(B_d);
    g.sb_k = b_trans ? 1 : N;        // B stored [K][N], or [N][K] when transposed
    g.sb_n = b_trans ? K : 1;
    g.mode = gga::MLP_PLAIN;
    g.C = C_d;
    g.ldc = N;
    const hipError_t e = gga::launch_gemm(g, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

}  // extern "C"

// ------------------------------------------------------------------ surrogate-screened GA

namespace {

struct SgaWorkspace {
    int32_t* generation;
    int32_t* sim_key;       // generation + 1: offspring of generation g join population g + 1
    float* cand_dose;
    int32_t* cand_gap;
    float* pred;
    int32_t *order_c, *pos_c, *order_p, *pos_p;
    int32_t* live;
    int32_t* nfrac;
    float* tmp_dose;
    int32_t* tmp_gap;
    float* tmp_fit;
    float* loss;
    void* mlp_work;
    size_t mlp_work_bytes;
};

struct SgaDims {
    int32_t N, K, R, C, S;
};

size_t sga_layout(const SgaDims& d, SgaWorkspace* w, void* base) {
    char* p = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t at = off; off += align256(bytes); return p ? p + at : nullptr; };
    const size_t C = d.C, K = d.K, NS = (size_t)d.N + d.S, MX = std::max<size_t>(C, NS);
    SgaWorkspace s{};
    s.generation = reinterpret_cast<int32_t*>(take(sizeof(int32_t)));
    s.sim_key = reinterpret_cast<int32_t*>(take(sizeof(int32_t)));
    s.cand_dose = reinterpret_cast<float*>(take(4 * C * K));
    s.cand_gap = reinterpret_cast<int32_t*>(take(4 * C * K));
    s.pred = reinterpret_cast<float*>(take(4 * C));
    s.order_c = reinterpret_cast<int32_t*>(take(4 * C));
    s.pos_c = reinterpret_cast<int32_t*>(take(4 * C));
    s.order_p = reinterpret_cast<int32_t*>(take(4 * NS));
    s.pos_p = reinterpret_cast<int32_t*>(take(4 * NS));
    s.live = reinterpret_cast<int32_t*>(take(4 * (size_t)std::max(d.N, d.S) * d.R));
    s.nfrac = reinterpret_cast<int32_t*>(take(4 * MX));
    s.tmp_dose = reinterpret_cast<float*>(take(4 * (size_t)d.N * K));
    s.tmp_gap = reinterpret_cast<int32_t*>(take(4 * (size_t)d.N * K));
    s.tmp_fit = reinterpret_cast<float*>(take(4 * (size_t)d.N));
    s.loss = reinterpret_cast<float*>(take(sizeof(float)));
    s.mlp_work_bytes = gga::mlp_work_bytes(std::max<int32_t>(d.C, d.N + d.S));
    s.mlp_work = take(s.mlp_work_bytes);
    if (w) *w = s;
    return off;
}

int check_sga(const gga_sga_cfg* sga, int32_t N, int32_t K, int32_t R, SgaDims* d) {
    if (!sga) return GGA_E_ARG;
    if (sga->struct_size != sizeof(gga_sga_cfg)) return GGA_E_ABI;
    if (sga->n_candidates < 2 || sga->n_simulated < 1 || sga->n_simulated > sga->n_candidates) return GGA_E_ARG;
    if (sga->screen != 0 && sga->screen != 1) return GGA_E_ARG;
    if (sga->refine_steps < 0 || sga->refine_steps > 64 || (sga->refine_steps > 0 && !sga->screen)) return GGA_E_ARG;
    if (sga->refine_steps > 0 && !(sga->refine_lr > 0.0f && std::isfinite(sga->refine_lr))) return GGA_E_ARG;
    if (N < 2 || K < 1 || K > GGA_KMAX || R < 1) return GGA_E_ARG;
    if ((long long)sga->n_candidates * gga::MLP_HID > std::numeric_limits<int32_t>::max()) return GGA_E_ARG;
    if ((long long)(N + sga->n_simulated) * R > std::numeric_limits<int32_t>::max()) return GGA_E_ARG;
    *d = SgaDims{N, K, R, sga->n_candidates, sga->n_simulated};
    return GGA_OK;
}

hipError_t sim_rows(const gga_params* params, const gga_sim_cfg* cfg, const float* dose, const int32_t* gap,
                    const int32_t* nfrac, int32_t P, int32_t K, const int32_t* generation, int32_t* live, float* fit,
                    hipStream_t stream) {
    gga::SimArgs sa = make_args(params, cfg, dose, gap, nfrac, K);
    sa.n0 = 0;
    sa.nsteps = cfg->horizon;
    sa.mode = 0;
    sa.live = live;
    sa.generation = generation;
    sa.seed = cfg->seed;
    hipError_t e = gga::launch_simulation(sa, cfg->L, P * cfg->R, stream);
    if (e == hipSuccess) e = gga::launch_fitness(live, P, cfg->R, fit, stream);
    return e;
}

hipError_t enqueue_sga(const gga_params* params, const gga_sim_cfg* cfg, gga::GaArgs ga_args, const gga_sga_cfg* sga,
                       void* net, float* pop_dose, int32_t* pop_gap, float* pop_fit, const SgaDims& d,
                       const SgaWorkspace& w, float* hist, int32_t hist_cap, float* best_dose, int32_t* best_gap,
                       hipStream_t stream) {
    const int N = d.N, K = d.K, C = d.C, S = d.S;
    // breed C candidates from the ranked population
    hipError_t e = gga::launch_rank(pop_fit, N, w.order_p, w.pos_p, stream);
    ga_args.n_elite = 0;
    ga_args.n_out = C;
    ga_args.fitness = pop_fit;
    ga_args.dose = pop_dose;
    ga_args.gap = pop_gap;
    ga_args.order = w.order_p;
    ga_args.position = w.pos_p;
    ga_args.generation = w.generation;
    ga_args.next_dose = w.cand_dose;
    ga_args.next_gap = w.cand_gap;
    if (e == hipSuccess) e = gga::launch_offspring(ga_args, stream);
    // screen: surrogate prediction (or random keys for the ablation), keep the best S
    if (e == hipSuccess) {
        e = sga->screen ? gga::mlp_forward(gga::mlp_net(net), w.cand_dose, w.cand_gap, w.nfrac, C, K,
                                           gga::mlp_work(w.mlp_work, C), w.pred, true, stream)
                        : gga::launch_random_keys(C, w.generation, ((uint64_t)ga_args.seed_hi << 32) | ga_args.seed_lo,
                                                  w.pred, stream);
    }
    if (e == hipSuccess) e = gga::launch_rank(w.pred, C, w.order_c, w.pos_c, stream);
    if (e == hipSuccess)
        e = gga::launch_gather(w.cand_dose, w.cand_gap, nullptr, w.order_c, S, K, pop_dose + (size_t)N * K,
                               pop_gap + (size_t)N * K, nullptr, stream);
    // simulate the S survivors of the screen, keyed as members of population g + 1
    if (e == hipSuccess) e = gga::launch_counter_copy(w.sim_key, w.generation, 1, stream);
    if (e == hipSuccess)
        e = sim_rows(params, cfg, pop_dose + (size_t)N * K, pop_gap + (size_t)N * K, w.nfrac, S, K, w.sim_key,
                     w.live, pop_fit + N, stream);
    // online refinement: Adam steps on the N + S simulated protocols (the
    // population and the new candidates), where the search now is
    for (int k = 0; k < sga->refine_steps && e == hipSuccess; ++k) {
        const gga::MlpNet mnet = gga::mlp_net(net);
        const gga::MlpWork mw = gga::mlp_work(w.mlp_work, N + S);
        e = gga::mlp_forward(mnet, pop_dose, pop_gap, w.nfrac, N + S, K, mw, mw.y, false, stream);
        if (e == hipSuccess) e = gga::mlp_backward(mnet, N + S, pop_fit, mw, w.loss, stream);
        if (e == hipSuccess) e = gga::mlp_adam_refresh(mnet, 0, sga->refine_lr, stream);
    }
    // keep the best N of the N + S evaluated protocols
    if (e == hipSuccess) e = gga::launch_rank(pop_fit, N + S, w.order_p, w.pos_p, stream);
    if (e == hipSuccess)
        e = gga::launch_gather(pop_dose, pop_gap, pop_fit, w.order_p, N, K, w.tmp_dose, w.tmp_gap, w.tmp_fit, stream);
    if (e == hipSuccess)
        e = gga::launch_gather(w.tmp_dose, w.tmp_gap, w.tmp_fit, nullptr, N, K, pop_dose, pop_gap, pop_fit, stream);
    const gga::Archive arc{pop_dose, pop_gap, K, best_dose, best_gap};
    if (e == hipSuccess) e = gga::launch_history(pop_fit, N, nullptr, w.generation, hist, hist_cap, arc, stream);
    if (e == hipSuccess) e = gga::launch_counter(w.generation, 1, 1, stream);
    return e;
}

}  // namespace

extern "C" {

size_t gga_sga_workspace_bytes(int32_t N, int32_t K, int32_t R, int32_t C, int32_t S) {
    if (N < 1 || K < 1 || R < 1 || C < 1 || S < 1) return 0;
    return sga_layout(SgaDims{N, K, R, C, S}, nullptr, nullptr);
}

int gga_sga_init(const gga_params* params, const gga_sim_cfg* cfg, const gga_sga_cfg* sga, float* pop_dose_d,
                 int32_t* pop_gap_d, float* pop_fit_d, int32_t N, int32_t K, void* ws_d, size_t ws_bytes,
                 hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    SgaDims d;
    if ((rc = check_sga(sga, N, K, cfg->R, &d))) return rc;
    if (!pop_dose_d || !pop_gap_d || !pop_fit_d || !ws_d || ws_bytes < sga_layout(d, nullptr, nullptr))
        return GGA_E_ARG;
    SgaWorkspace w;
    sga_layout(d, &w, ws_d);
    hipError_t e = gga::launch_fill(w.nfrac, std::max(d.C, d.N + d.S), K, stream);
    if (e == hipSuccess) e = gga::launch_counter(w.generation, 0, 0, stream);
    if (e == hipSuccess) e = sim_rows(params, cfg, pop_dose_d, pop_gap_d, w.nfrac, N, K, w.generation, w.live, pop_fit_d, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_sga_generation(const gga_params* params, const gga_sim_cfg* cfg, const gga_ga_cfg* ga,
                       const gga_alphabet* a, const gga_sga_cfg* sga, void* net_d, float* pop_dose_d,
                       int32_t* pop_gap_d, float* pop_fit_d, int32_t N, int32_t K, void* ws_d, size_t ws_bytes,
                       float* hist_d, int32_t hist_cap, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    SgaDims d;
    if ((rc = check_sga(sga, N, K, cfg->R, &d))) return rc;
    gga::GaArgs ga_args;
    if ((rc = check_ga(ga, a, N, K, &ga_args))) return rc;
    if (!pop_dose_d || !pop_gap_d || !pop_fit_d || !ws_d || (sga->screen && !net_d)) return GGA_E_ARG;
    if (misaligned16(ws_d) || (sga->screen && misaligned16(net_d))) return GGA_E_ARG;
    if (ws_bytes < sga_layout(d, nullptr, nullptr) || hist_cap < 0 || (hist_cap > 0 && !hist_d)) return GGA_E_ARG;
    SgaWorkspace w;
    sga_layout(d, &w, ws_d);
    const hipError_t e = enqueue_sga(params, cfg, ga_args, sga, net_d, pop_dose_d, pop_gap_d, pop_fit_d, d, w, hist_d,
                                     hist_cap, nullptr, nullptr, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_sga_run(const gga_params* params, const gga_sim_cfg* cfg, const gga_ga_cfg* ga, const gga_alphabet* a,
                const gga_sga_cfg* sga, void* net_d, float* pop_dose_d, int32_t* pop_gap_d, float* pop_fit_d,
                int32_t N, int32_t K, int32_t g0, int32_t n_gen, int32_t use_graph, void* ws_d, size_t ws_bytes,
                float* hist_d, float* best_dose_d, int32_t* best_gap_d, float* gen_ms_h, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_cfg(cfg))) return rc;
    if (!best_dose_d != !best_gap_d) return GGA_E_ARG;
    SgaDims d;
    if ((rc = check_sga(sga, N, K, cfg->R, &d))) return rc;
    gga::GaArgs ga_args;
    if ((rc = check_ga(ga, a, N, K, &ga_args))) return rc;
    if (!pop_dose_d || !pop_gap_d || !pop_fit_d || !ws_d || (sga->screen && !net_d) || n_gen < 0 || g0 < 0)
        return GGA_E_ARG;
    if (misaligned16(ws_d) || (sga->screen && misaligned16(net_d))) return GGA_E_ARG;
    if ((long long)g0 + n_gen > std::numeric_limits<int32_t>::max()) return GGA_E_ARG;
    if (ws_bytes < sga_layout(d, nullptr, nullptr) || (n_gen > 0 && !hist_d)) return GGA_E_ARG;
    SgaWorkspace w;
    sga_layout(d, &w, ws_d);
    const int32_t hist_cap = g0 + n_gen;
    auto enqueue = [&](int) {
        return enqueue_sga(params, cfg, ga_args, sga, net_d, pop_dose_d, pop_gap_d, pop_fit_d, d, w, hist_d, hist_cap,
                           best_dose_d, best_gap_d, stream);
    };
    const hipError_t e = run_generations(enqueue, w.generation, g0, n_gen, use_graph, gen_ms_h, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

}  // extern "C"

// ------------------------------------------------------------------ kernel variants, uneven batches

namespace {

// Slab rows for lattice side L, RR rows per workgroup and a halo of H rows:
// the first and last slab own RR - H rows at the lattice edges, middle slabs
// at most RR - 2H.  Returns the slab count (0: RR >= L, resident; -1: no plan).
int slab_plan(int L, int RR, int H, gga::SimArgs* a) {
    if (RR >= L) return 0;
    const int own_edge = RR - H;
    if (own_edge < 1) return -1;
    int ns = 0;
    auto add = [&](int ys, int i0, int i1) {
        if (ns < gga::MAX_SLABS) {
            a->slab_ys[ns] = ys;
            a->slab_i0[ns] = i0;
            a->slab_i1[ns] = i1;
        }
        ++ns;
    };
    if (2 * own_edge >= L) {                      // the two edge slabs meet
        const int half = L / 2;
        add(0, 0, half);
        add(L - RR, half - (L - RR), RR);
    } else {
        const int mid = RR - 2 * H;
        if (mid < 1) return -1;
        const int m = L - 2 * own_edge;
        const int nm = (m + mid - 1) / mid;
        add(0, 0, own_edge);
        int at = own_edge;
        for (int j = 0; j < nm; ++j) {
            const int len = m / nm + (j < m % nm ? 1 : 0);
            add(at - H, H, H + len);
            at += len;
        }
        add(L - RR, H, RR);
    }
    a->n_slabs = ns;
    return ns <= gga::MAX_SLABS ? ns : -1;
}

int side_ok(int L) { return gga::side_index(L) >= 0; }

size_t state_bytes(int L) { return (size_t)L * L * (3 * sizeof(float) + sizeof(uint16_t)); }

// One group of instances that share a lattice side (and so a kernel variant).
struct Group {
    int L, variant, first, count, max_h;   // instances list[first .. first+count), horizon-descending
    bool teams;                            // slab form as teams over whole horizons
    int rows;                              // slab form: instances the state buffers hold
    size_t state_off, flags_off;           // slab form: two state buffers of `rows` instances; team step counts
};

struct UnevenPlan {
    std::vector<int32_t> host;             // instance lists then horizons, uploaded together
    std::vector<Group> groups;
    size_t off_lists, off_horizon, off_valid, off_count, off_step, off_frac, total;
};

// Group the P*R instances by lattice side, each group sorted by horizon
// (longest first, then by index), and lay out the workspace.
int plan_uneven(const int32_t* lattice_h, const int32_t* horizon_h, int32_t P, int32_t K, int32_t R,
                int32_t substeps, const int* force, UnevenPlan* plan) {
    for (int32_t p = 0; p < P; ++p) {
        if (!side_ok(lattice_h[p])) return GGA_E_UNSUPPORTED;
        if (horizon_h[p] < 0 || horizon_h[p] > (1 << 30)) return GGA_E_ARG;
    }
    plan->host.clear();
    plan->groups.clear();
    for (int si = 0; si < gga::N_SIDES; ++si) {
        const int L = 64 + 32 * si;
        std::vector<int32_t> list;
        for (int32_t p = 0; p < P; ++p)
            if (lattice_h[p] == L)
                for (int32_t r = 0; r < R; ++r) list.push_back(p * R + r);
        if (list.empty()) continue;
        std::stable_sort(list.begin(), list.end(),
                         [&](int32_t x, int32_t y) { return horizon_h[x / R] > horizon_h[y / R]; });
        const int v = force && force[si] >= 0 ? force[si] : gga::variant_choice(L, false);
        if (v < 0) return GGA_E_UNSUPPORTED;
        const bool teams = uses_teams(v, L, substeps);
        Group g{L, v, (int)plan->host.size(), (int)list.size(), horizon_h[list[0] / R], teams,
                state_rows(teams, (int32_t)list.size()), 0, 0};
        plan->groups.push_back(g);
        plan->host.insert(plan->host.end(), list.begin(), list.end());
    }
    const size_t n_inst = plan->host.size();
    plan->host.insert(plan->host.end(), horizon_h, horizon_h + P);
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t at = off; off += align256(bytes); return at; };
    plan->off_lists = take(sizeof(int32_t) * n_inst);
    plan->off_horizon = take(sizeof(int32_t) * (size_t)P);
    plan->off_valid = take(sizeof(int32_t) * (size_t)P);
    plan->off_count = take(sizeof(int32_t) * (size_t)P);
    plan->off_step = take(sizeof(int32_t) * (size_t)P * K);
    plan->off_frac = take(sizeof(gga::EventFraction) * (size_t)P * K);
    for (auto& g : plan->groups)
        if (gga::variant_is_slab(g.variant)) {
            g.state_off = take(2 * align256(state_bytes(g.L) * (size_t)g.rows));
            if (g.teams) g.flags_off = take(sizeof(int32_t) * (size_t)gga::TEAM_MAX * gga::MAX_SLABS);
        }
    plan->total = off;
    return GGA_OK;
}

// Enqueue the uneven batch (the plan's host part already uploaded).
hipError_t enqueue_uneven(const gga::SimArgs& base, const UnevenPlan& plan, char* ws, int32_t P, int32_t R,
                          int32_t* live_d, float* fitness_d, hipStream_t stream) {
    gga::SimArgs a = base;
    a.live = live_d;
    a.horizon = reinterpret_cast<const int32_t*>(ws + plan.off_horizon);
    a.ev_valid = reinterpret_cast<const int32_t*>(ws + plan.off_valid);
    a.ev_count = reinterpret_cast<const int32_t*>(ws + plan.off_count);
    a.ev_step = reinterpret_cast<const int32_t*>(ws + plan.off_step);
    a.ev_frac = reinterpret_cast<const gga::EventFraction*>(ws + plan.off_frac);
    hipError_t e = gga::launch_event_table(a, P, reinterpret_cast<int32_t*>(ws + plan.off_valid),
                                           reinterpret_cast<int32_t*>(ws + plan.off_count),
                                           reinterpret_cast<int32_t*>(ws + plan.off_step),
                                           reinterpret_cast<gga::EventFraction*>(ws + plan.off_frac), stream);
    const int32_t* lists = reinterpret_cast<const int32_t*>(ws + plan.off_lists);
    for (const Group& g : plan.groups) {
        if (e != hipSuccess) break;
        a.inst_list = lists + g.first;
        if (!gga::variant_is_slab(g.variant)) {
            a.n0 = 0;
            a.nsteps = 0;                          // steps come from horizon[]
            a.mode = 0;
            e = gga::launch_variant(g.variant, a, g.count, stream);
            continue;
        }
        const gga::SimVariant& v = gga::SIM_VARIANTS[g.variant];
        if (slab_plan(g.L, v.rpt * v.nw, a.substeps + 2, &a) <= 0) return hipErrorInvalidValue;
        if (g.teams) {
            if (!team_plan(&a, v.rpt * v.nw)) return hipErrorInvalidValue;
            a.nsteps = 0;                          // steps come from horizon[]
            e = gga::launch_slab_live(a, g.count, stream);
            if (e == hipSuccess)
                e = enqueue_teams(a, g.variant, g.count, g.rows, ws + g.state_off,
                                  align256(state_bytes(g.L) * (size_t)g.rows), g.L,
                                  reinterpret_cast<int32_t*>(ws + g.flags_off), stream);
            continue;
        }
        const size_t sb = align256(state_bytes(g.L) * (size_t)g.count);
        float* fa = reinterpret_cast<float*>(ws + g.state_off);
        uint16_t* ca = reinterpret_cast<uint16_t*>(ws + g.state_off + (size_t)g.count * g.L * g.L * 3 * sizeof(float));
        float* fb = reinterpret_cast<float*>(ws + g.state_off + sb);
        uint16_t* cb = reinterpret_cast<uint16_t*>(ws + g.state_off + sb + (size_t)g.count * g.L * g.L * 3 * sizeof(float));
        e = gga::launch_slab_init(a, g.L, g.count, fa, ca, stream);
        // step n: the instances with horizon > n are a prefix of the group's list
        int active = g.count;
        for (int n = 0; n < g.max_h && e == hipSuccess; ++n) {
            while (active > 0 && plan.host[plan.host.size() - P + plan.host[g.first + active - 1] / R] <= n) --active;
            if (active == 0) break;
            a.n0 = n;
            a.nsteps = 1;
            a.fields = (n & 1) ? fb : fa;
            a.cells = (n & 1) ? cb : ca;
            a.fields_out = (n & 1) ? fa : fb;
            a.cells_out = (n & 1) ? ca : cb;
            a.n_active = active;
            e = gga::launch_variant(g.variant, a, gga::slab_blocks(active, a.n_slabs), stream);
        }
    }
    if (e == hipSuccess) e = gga::launch_fitness(live_d, P, R, fitness_d, stream);
    return e;
}

}  // namespace

namespace {

int upload_plan(const UnevenPlan& plan, char* ws, int32_t P, hipStream_t stream) {
    const size_t n_inst = plan.host.size() - (size_t)P;
    hipError_t e = hipSuccess;
    if (n_inst) e = hipMemcpyAsync(ws + plan.off_lists, plan.host.data(), sizeof(int32_t) * n_inst,
                                   hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && P)
        e = hipMemcpyAsync(ws + plan.off_horizon, plan.host.data() + n_inst, sizeof(int32_t) * (size_t)P,
                           hipMemcpyHostToDevice, stream);
    // the host vector is released on return
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int check_uneven_cfg(const gga_sim_cfg* c) {
    if (!c) return GGA_E_ARG;
    if (c->struct_size != sizeof(gga_sim_cfg)) return GGA_E_ABI;
    if ((c->flags & ~GGA_SIM_HALF_HOUR) != 0 || c->R < 1 || !std::isfinite(c->dose_cap)) return GGA_E_ARG;
    if (c->substeps < 1 || c->substeps > 64) return GGA_E_UNSUPPORTED;
    return GGA_OK;
}

}  // namespace

extern "C" {

int gga_variant_count(void) { return gga::N_SIM_VARIANTS; }

int gga_set_team_options(int32_t use_teams, int32_t spin_limit) {
    if (use_teams != 0 && use_teams != 1) return GGA_E_ARG;
    g_use_teams.store(use_teams);
    g_spin_limit.store(spin_limit);
    return GGA_OK;
}

int32_t gga_variant_side(int32_t v) { return (v >= 0 && v < gga::N_SIM_VARIANTS) ? gga::SIM_VARIANTS[v].L : -1; }

int32_t gga_variant_is_slab(int32_t v) {
    return (v >= 0 && v < gga::N_SIM_VARIANTS) ? (gga::variant_is_slab(v) ? 1 : 0) : -1;
}

const char* gga_variant_name(int32_t v) {
    return (v >= 0 && v < gga::N_SIM_VARIANTS) ? gga::SIM_VARIANTS[v].name : "no such variant";
}

int gga_get_variant(int32_t L, int32_t resident_only) {
    const int v = gga::variant_choice(L, resident_only != 0);
    return v < 0 ? GGA_E_UNSUPPORTED : v;
}

int gga_set_variant(int32_t L, int32_t v) { return gga::set_variant_choice(L, v) == 0 ? GGA_OK : GGA_E_ARG; }

size_t gga_uneven_workspace_bytes(const int32_t* lattice_h, const int32_t* horizon_h, int32_t P, int32_t K,
                                  int32_t R, int32_t substeps) {
    if (check_batch(P, K, R) || R < 1 || (P > 0 && (!lattice_h || !horizon_h))) return 0;
    if (substeps < 1 || substeps > 64) return 0;
    UnevenPlan plan;
    if (plan_uneven(lattice_h, horizon_h, P, K, R, substeps, nullptr, &plan)) return 0;
    return plan.total;
}

int gga_simulate_uneven(const gga_params* params, const gga_sim_cfg* cfg, const float* dose_d,
                        const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P, int32_t K,
                        const int32_t* lattice_h, const int32_t* horizon_h, void* ws_d, size_t ws_bytes,
                        int32_t* live_d, float* fitness_d, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_uneven_cfg(cfg))) return rc;
    if ((rc = check_batch(P, K, cfg->R))) return rc;
    if (P == 0) return GGA_OK;
    if (!lattice_h || !horizon_h || !nfrac_d || !live_d || !fitness_d || !ws_d || misaligned16(ws_d) ||
        (K > 0 && (!dose_d || !gap_h_d)))
        return GGA_E_ARG;
    UnevenPlan plan;
    if ((rc = plan_uneven(lattice_h, horizon_h, P, K, cfg->R, cfg->substeps, nullptr, &plan))) return rc;
    if (ws_bytes < plan.total) return GGA_E_ARG;
    char* ws = static_cast<char*>(ws_d);
    if ((rc = upload_plan(plan, ws, P, stream))) return rc;
    const gga::SimArgs base = make_args(params, cfg, dose_d, gap_h_d, nfrac_d, K);
    const hipError_t e = enqueue_uneven(base, plan, ws, P, cfg->R, live_d, fitness_d, stream);
    return e == hipSuccess ? GGA_OK : (e == hipErrorInvalidValue ? GGA_E_UNSUPPORTED : hip_fail(e));
}

size_t gga_event_table_bytes(int32_t P, int32_t K) {
    if (P < 0 || K < 0 || K > GGA_KMAX) return 0;
    return align256(sizeof(int32_t) * 2 * (size_t)P) + align256(sizeof(int32_t) * (size_t)P * K) +
           align256(sizeof(gga::EventFraction) * (size_t)P * K);
}

int gga_state_run_variant(const gga_params* params, const gga_sim_cfg* cfg, int32_t variant,
                          const float* dose_d, const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P,
                          int32_t K, int32_t n0, int32_t nsteps, float* fields_d, uint16_t* cells_d,
                          float* fields2_d, uint16_t* cells2_d, void* ws_d, size_t ws_bytes, int32_t* live_d,
                          hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_uneven_cfg(cfg))) return rc;
    if ((rc = check_batch(P, K, cfg->R))) return rc;
    if (variant < 0 || variant >= gga::N_SIM_VARIANTS || gga::SIM_VARIANTS[variant].L != cfg->L) return GGA_E_ARG;
    if (n0 < 0 || nsteps < 0 || (long long)n0 + nsteps > (1LL << 30)) return GGA_E_ARG;   // half-hour event times fit int32
    if (P == 0) return GGA_OK;
    if (!nfrac_d || !fields_d || !cells_d || (K > 0 && (!dose_d || !gap_h_d))) return GGA_E_ARG;
    gga::SimArgs a = make_args(params, cfg, dose_d, gap_h_d, nfrac_d, K);
    a.live = live_d;
    hipError_t e = hipSuccess;
    if (!gga::variant_is_slab(variant)) {
        a.n0 = n0;
        a.nsteps = nsteps;
        a.mode = gga::MODE_LOAD | gga::MODE_STORE;
        a.fields = fields_d;
        a.cells = cells_d;
        e = gga::launch_variant(variant, a, P * cfg->R, stream);
        return e == hipSuccess ? GGA_OK : hip_fail(e);
    }
    if (nsteps < 1 || !fields2_d || !cells2_d || !ws_d || misaligned16(ws_d) || ws_bytes < gga_event_table_bytes(P, K))
        return GGA_E_ARG;
    const gga::SimVariant& v = gga::SIM_VARIANTS[variant];
    if (slab_plan(cfg->L, v.rpt * v.nw, cfg->substeps + 2, &a) <= 0) return GGA_E_UNSUPPORTED;
    char* ws = static_cast<char*>(ws_d);
    int32_t* valid = reinterpret_cast<int32_t*>(ws);
    int32_t* count = valid + P;
    int32_t* step = reinterpret_cast<int32_t*>(ws + align256(sizeof(int32_t) * 2 * (size_t)P));
    gga::EventFraction* frac = reinterpret_cast<gga::EventFraction*>(
        ws + align256(sizeof(int32_t) * 2 * (size_t)P) + align256(sizeof(int32_t) * (size_t)P * K));
    a.ev_valid = valid;
    a.ev_count = count;
    a.ev_step = step;
    a.ev_frac = frac;
    a.count_at = n0 + nsteps;
    e = gga::launch_event_table(a, P, valid, count, step, frac, stream);
    if (e == hipSuccess) e = gga::launch_slab_live(a, P * cfg->R, stream);
    for (int32_t n = n0; n < n0 + nsteps && e == hipSuccess; ++n) {
        const bool odd = ((n - n0) & 1) != 0;
        a.n0 = n;
        a.nsteps = 1;
        a.fields = odd ? fields2_d : fields_d;
        a.cells = odd ? cells2_d : cells_d;
        a.fields_out = odd ? fields_d : fields2_d;
        a.cells_out = odd ? cells_d : cells2_d;
        a.n_active = P * cfg->R;
        e = gga::launch_variant(variant, a, gga::slab_blocks(a.n_active, a.n_slabs), stream);
    }
    if (e == hipSuccess && (nsteps & 1)) {         // the result is in the second buffers
        const size_t plane = (size_t)cfg->L * cfg->L, inst = (size_t)P * cfg->R;
        e = hipMemcpyAsync(fields_d, fields2_d, sizeof(float) * 3 * plane * inst, hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(cells_d, cells2_d, sizeof(uint16_t) * plane * inst, hipMemcpyDeviceToDevice, stream);
    }
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

size_t gga_autotune_workspace_bytes(int32_t L, int32_t P, int32_t K, int32_t R, int32_t horizon, int32_t substeps) {
    if (!side_ok(L) || P < 1 || R < 1 || horizon < 0 || check_batch(P, K, R)) return 0;
    if (substeps < 1 || substeps > 64) return 0;
    std::vector<int32_t> lat((size_t)P, L), hor((size_t)P, horizon);
    size_t most = 0;
    const int si = gga::side_index(L);
    for (int v = 0; v < gga::N_SIM_VARIANTS; ++v) {
        if (gga::SIM_VARIANTS[v].L != L) continue;
        int force[gga::N_SIDES] = {-1, -1, -1, -1, -1, -1, -1};
        force[si] = v;
        UnevenPlan plan;
        if (plan_uneven(lat.data(), hor.data(), P, K, R, substeps, force, &plan) == GGA_OK)
            most = std::max(most, plan.total);
    }
    return most;
}

int gga_autotune(const gga_params* params, const gga_sim_cfg* cfg, const float* dose_d, const int32_t* gap_h_d,
                 const int32_t* nfrac_d, int32_t P, int32_t K, void* ws_d, size_t ws_bytes, int32_t* live_d,
                 float* fitness_d, float* ms_h, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_uneven_cfg(cfg))) return rc;
    if ((rc = check_batch(P, K, cfg->R))) return rc;
    if (!side_ok(cfg->L)) return GGA_E_UNSUPPORTED;
    if (P < 1 || cfg->horizon < 0 || !nfrac_d || !live_d || !fitness_d || !ws_d || (K > 0 && (!dose_d || !gap_h_d)))
        return GGA_E_ARG;
    const int L = cfg->L, si = gga::side_index(L);
    std::vector<int32_t> lat((size_t)P, L), hor((size_t)P, cfg->horizon);
    const gga::SimArgs base = make_args(params, cfg, dose_d, gap_h_d, nfrac_d, K);
    char* ws = static_cast<char*>(ws_d);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    hipError_t e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    int best = -1, best_res = -1;
    float best_ms = 0.0f, best_res_ms = 0.0f;
    for (int v = 0; v < gga::N_SIM_VARIANTS && e == hipSuccess; ++v) {
        if (ms_h) ms_h[v] = std::numeric_limits<float>::quiet_NaN();
        if (gga::SIM_VARIANTS[v].L != L) continue;
        int force[gga::N_SIDES] = {-1, -1, -1, -1, -1, -1, -1};
        force[si] = v;
        UnevenPlan plan;
        if (plan_uneven(lat.data(), hor.data(), P, K, cfg->R, cfg->substeps, force, &plan) != GGA_OK) continue;
        if (ws_bytes < plan.total) { rc = GGA_E_ARG; break; }
        if ((rc = upload_plan(plan, ws, P, stream))) break;
        float ms = 0.0f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {    // the first run warms up
            e = hipEventRecord(t0, stream);
            if (e == hipSuccess) e = enqueue_uneven(base, plan, ws, P, cfg->R, live_d, fitness_d, stream);
            if (e == hipSuccess) e = hipEventRecord(t1, stream);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, t0, t1);
            if (rep == 1 || (rep == 2 && t < ms)) ms = t;
        }
        if (e == hipErrorInvalidValue) { e = hipSuccess; continue; }   // no slab plan for these sub-steps
        if (e != hipSuccess) break;
        if (ms_h) ms_h[v] = ms;
        if (best < 0 || ms < best_ms) { best = v; best_ms = ms; }
        if (!gga::variant_is_slab(v) && (best_res < 0 || ms < best_res_ms)) { best_res = v; best_res_ms = ms; }
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (e != hipSuccess) return hip_fail(e);
    if (rc) return rc;
    if (best < 0) return GGA_E_UNSUPPORTED;
    if (best_res >= 0) gga::set_variant_choice(L, best_res);
    gga::set_variant_choice(L, best);
    return best;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Quasi-3D variant: C cell slots per site.
namespace {

int check_q3_cfg(const gga_sim_cfg* c, int32_t C) {
    if (!c) return GGA_E_ARG;
    if (c->struct_size != sizeof(gga_sim_cfg)) return GGA_E_ABI;
    if ((c->flags & ~GGA_SIM_HALF_HOUR) != 0 || c->R < 1 || c->horizon < 0 || c->horizon > (1 << 30)) return GGA_E_ARG;
    if (!std::isfinite(c->dose_cap)) return GGA_E_ARG;
    if (C < 1 || C > gga::Q3_MAX_SLOTS) return GGA_E_ARG;
    if (c->L < gga::Q3_MIN_L || c->L > gga::Q3_MAX_L || c->substeps < 1 || c->substeps > 64) return GGA_E_UNSUPPORTED;
    if ((long long)C * c->L * c->L > gga::Q3_MAX_SLOT_SITES) return GGA_E_UNSUPPORTED;
    return GGA_OK;
}

// instances x blocks per instance must stay below 2^31 (one-dimensional grid)
bool q3_grid_ok(int32_t L, long long n_inst) {
    const long long nbx = ((long long)L * L + 255) / 256;
    return n_inst * nbx <= (1LL << 31) - 8;
}

struct Q3Plan {
    size_t off_step, off_frac, off_f2, off_react, off_emask, off_tmask, off_pmask, off_svec, off_keys, off_prop,
        off_fields, off_cells, total;
};

Q3Plan q3_plan(int32_t L, int32_t C, int32_t P, int32_t R, int32_t K) {
    Q3Plan q;
    const size_t n = (size_t)P * R, L2 = (size_t)L * L, CL2 = (size_t)C * L2;
    size_t o = align256(sizeof(int32_t) * 2 * (size_t)P);
    q.off_step = o;
    o += align256(sizeof(int32_t) * (size_t)P * K);
    q.off_frac = o;
    o += align256(sizeof(gga::EventFraction) * (size_t)P * K);
    q.off_f2 = o;
    o += align256(sizeof(float) * 3 * L2 * n);
    q.off_react = o;
    o += align256(sizeof(float) * L2 * n);
    q.off_emask = o;
    o += align256(sizeof(uint32_t) * L2 * n);
    q.off_tmask = o;
    o += align256(sizeof(uint32_t) * 2 * L2 * n);
    q.off_pmask = o;
    o += align256(sizeof(uint32_t) * L2 * n);
    q.off_svec = o;
    o += align256(sizeof(unsigned long long) * L2 * n);
    q.off_keys = o;
    o += align256(sizeof(unsigned long long) * CL2 * n);
    q.off_prop = o;
    o += align256(sizeof(uint32_t) * CL2 * n);
    q.off_fields = o;
    o += align256(sizeof(float) * 3 * L2 * n);
    q.off_cells = o;
    o += align256(sizeof(uint16_t) * CL2 * n);
    q.total = o;
    return q;
}

gga::Q3Args q3_args(const gga_params* prm, const gga_sim_cfg* cfg, int32_t C, int32_t P, int32_t K) {
    gga::Q3Args a;
    std::memset(&a, 0, sizeof(a));
    a.prm = *prm;
    a.L = cfg->L;
    a.C = C;
    a.R = cfg->R;
    a.K = K;
    a.substeps = cfg->substeps;
    a.half = (cfg->flags & GGA_SIM_HALF_HOUR) ? 1 : 0;
    a.n_inst = P * cfg->R;
    a.seed_lo = static_cast<uint32_t>(cfg->seed);
    a.seed_hi = static_cast<uint32_t>(cfg->seed >> 32);
    return a;
}

// Carves the workspace, builds the event table and runs steps n0 .. n0+nsteps-1
// on the state in a.fields / a.cells.
hipError_t q3_enqueue(gga::Q3Args a, const gga_params* prm, const gga_sim_cfg* cfg, const float* dose,
                      const int32_t* gap, const int32_t* nfrac, int32_t P, int32_t K, char* ws, const Q3Plan& q,
                      int32_t n0, int32_t nsteps, bool init, hipStream_t stream) {
    int32_t* valid = reinterpret_cast<int32_t*>(ws);
    int32_t* count = valid + P;
    int32_t* step = reinterpret_cast<int32_t*>(ws + q.off_step);
    gga::EventFraction* frac = reinterpret_cast<gga::EventFraction*>(ws + q.off_frac);
    gga::SimArgs s = make_args(prm, cfg, dose, gap, nfrac, K);
    hipError_t e = gga::launch_event_table(s, P, valid, count, step, frac, stream);
    if (e != hipSuccess) return e;
    a.ev_valid = valid;
    a.ev_count = count;
    a.ev_step = step;
    a.ev_frac = frac;
    a.fields2 = reinterpret_cast<float*>(ws + q.off_f2);
    a.react = reinterpret_cast<float*>(ws + q.off_react);
    a.emask = reinterpret_cast<uint32_t*>(ws + q.off_emask);
    a.tmask = reinterpret_cast<uint32_t*>(ws + q.off_tmask);
    a.pmask = reinterpret_cast<uint32_t*>(ws + q.off_pmask);
    a.svec = reinterpret_cast<unsigned long long*>(ws + q.off_svec);
    a.keys = reinterpret_cast<unsigned long long*>(ws + q.off_keys);
    a.prop = reinterpret_cast<uint32_t*>(ws + q.off_prop);
    if (init && (e = gga::q3_init(a, stream)) != hipSuccess) return e;
    return gga::q3_run(a, n0, nsteps, stream);
}

}  // namespace

extern "C" {

size_t gga_q3_workspace_bytes(int32_t L, int32_t C, int32_t P, int32_t R, int32_t K) {
    if (L < gga::Q3_MIN_L || L > gga::Q3_MAX_L || C < 1 || C > gga::Q3_MAX_SLOTS || R < 1 ||
        (long long)C * L * L > gga::Q3_MAX_SLOT_SITES || check_batch(P, K, R))
        return 0;
    return q3_plan(L, C, P, R, K).total;
}

int gga_q3_init(const gga_params* params, const gga_sim_cfg* cfg, int32_t C, int32_t P, float* fields_d,
                uint16_t* cells_d, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_q3_cfg(cfg, C))) return rc;
    if ((rc = check_batch(P, 0, cfg->R))) return rc;
    if (!q3_grid_ok(cfg->L, (long long)P * cfg->R)) return GGA_E_ARG;
    if (P == 0) return GGA_OK;
    if (!fields_d || !cells_d) return GGA_E_ARG;
    gga::Q3Args a = q3_args(params, cfg, C, P, 0);
    a.fields = fields_d;
    a.cells = cells_d;
    const hipError_t e = gga::q3_init(a, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_q3_run(const gga_params* params, const gga_sim_cfg* cfg, int32_t C, const float* dose_d,
               const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P, int32_t K, int32_t n0, int32_t nsteps,
               float* fields_d, uint16_t* cells_d, void* ws_d, size_t ws_bytes, int32_t* live_d, int32_t* traj_d,
               hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_q3_cfg(cfg, C))) return rc;
    if ((rc = check_batch(P, K, cfg->R))) return rc;
    if (n0 < 0 || nsteps < 0 || (long long)n0 + nsteps > (1LL << 30)) return GGA_E_ARG;
    if (!q3_grid_ok(cfg->L, (long long)P * cfg->R)) return GGA_E_ARG;
    if (P == 0) return GGA_OK;
    if (!nfrac_d || !fields_d || !cells_d || !ws_d || misaligned16(ws_d) || (K > 0 && (!dose_d || !gap_h_d)))
        return GGA_E_ARG;
    const Q3Plan q = q3_plan(cfg->L, C, P, cfg->R, K);
    if (ws_bytes < q.total) return GGA_E_ARG;
    gga::Q3Args a = q3_args(params, cfg, C, P, K);
    a.fields = fields_d;
    a.cells = cells_d;
    a.live = live_d;
    a.traj = traj_d;
    const hipError_t e = q3_enqueue(a, params, cfg, dose_d, gap_h_d, nfrac_d, P, K, static_cast<char*>(ws_d), q, n0,
                                    nsteps, false, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

int gga_simulate_q3(const gga_params* params, const gga_sim_cfg* cfg, int32_t C, const float* dose_d,
                    const int32_t* gap_h_d, const int32_t* nfrac_d, int32_t P, int32_t K, void* ws_d, size_t ws_bytes,
                    int32_t* live_d, float* fitness_d, int32_t* traj_d, hipStream_t stream) {
    int rc = check_params(params);
    if (rc) return rc;
    if ((rc = check_q3_cfg(cfg, C))) return rc;
    if ((rc = check_batch(P, K, cfg->R))) return rc;
    if (!q3_grid_ok(cfg->L, (long long)P * cfg->R)) return GGA_E_ARG;
    if (P == 0) return GGA_OK;
    if (!nfrac_d || !live_d || !fitness_d || !ws_d || misaligned16(ws_d) || (K > 0 && (!dose_d || !gap_h_d)))
        return GGA_E_ARG;
    const Q3Plan q = q3_plan(cfg->L, C, P, cfg->R, K);
    if (ws_bytes < q.total) return GGA_E_ARG;
    char* ws = static_cast<char*>(ws_d);
    gga::Q3Args a = q3_args(params, cfg, C, P, K);
    a.fields = reinterpret_cast<float*>(ws + q.off_fields);
    a.cells = reinterpret_cast<uint16_t*>(ws + q.off_cells);
    a.live = live_d;
    a.traj = traj_d;
    hipError_t e = q3_enqueue(a, params, cfg, dose_d, gap_h_d, nfrac_d, P, K, ws, q, 0, cfg->horizon, true, stream);
    if (e == hipSuccess) e = gga::launch_fitness(live_d, P, cfg->R, fitness_d, stream);
    return e == hipSuccess ? GGA_OK : hip_fail(e);
}

}  // extern "C"
