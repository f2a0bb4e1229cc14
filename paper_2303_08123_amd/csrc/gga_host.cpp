// Host side of the C ABI: argument checks, the host validator and launches.
// Every simulation step runs in the kernels; this file only checks and
// marshals arguments.
#include <cmath>
#include <cstring>
#include <limits>

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
