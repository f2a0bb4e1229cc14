// The simulation kernel template.  Resident form (RR = L): one workgroup
// advances one (protocol, replica) instance through all of its steps without
// leaving the compute unit.  Slab form (RR < L): one workgroup advances RR
// rows of a larger lattice by one step, from one state buffer in device memory
// to the other (see Geo).
//
// Layout.  Row pitch L = 64 * CPL; the lattice side LW <= L is a multiple of
// CPL.  Wave w owns rows [w*RPT, (w+1)*RPT) of the workgroup's RR rows; lane l
// owns columns [l*CPL, (l+1)*CPL).  The three
// float32 fields of a thread's RPT x CPL sites live in VGPRs for the whole run
// (resident) or step (slab); the uint16 cell words live in LDS.  One diffusion sub-step needs, per wave, only the row above and the
// row below its slab from the neighbouring waves (an LDS exchange of 2 rows),
// while left/right neighbours come from the adjacent lane through DPP lane
// shifts fused into the VALU adds.  A wave's 64 lanes span a whole lattice row,
// so the lane shifts' zero fill at lanes 0 and 63 is exactly the missing
// neighbour outside the lattice (the Dirichlet value is 0 in field units).
//
// Padding.  When LW < L the columns past the lattice hold padding sites:
// fields 0 with a diffusion number of 0 and no clamp, so they stay 0 and the
// last lattice column reads the boundary value from its right neighbour as
// lane 63 does; cell words EMPTY, never free and never irradiated.  Whole
// lanes are padding when LW is a multiple of CPL; otherwise one lane holds
// both kinds and keeps its diffusion numbers and clamps per column.  Philox
// counters and device-memory state use lattice coordinates (row pitch LW).
//
// Slabs.  A slab edge that is not a lattice edge is treated as if it were
// one; the error this makes reaches `substeps` rows into the slab through the
// diffusion and two rows further through the division proposals and their
// conflicts, so the rows within substeps + 2 of such an edge are a halo:
// computed, not stored, and owned by the neighbouring slab.  Every site's
// arithmetic is the resident form's, so both give identical results.
//
// Teams (TEAM): the slabs of one instance are a team of co-resident
// workgroups (a cooperative launch) that keep their rows on the CU for the
// whole horizon.  After each step a workgroup publishes the own rows its
// neighbours hold as halo (into one of two exchange buffers, by step parity)
// and a per-slab step count; before the next step it waits for both
// neighbours' counts, with a bounded spin, and reloads only its halo rows.
// A wait that runs out marks the instance's live count negative and the
// workgroup leaves; its neighbours then run out too, so every workgroup exits.
//
// The method (Materials and Methods: nutrient and waste diffusion, cell
// cycle, quiescence and death driven by the local environment, irradiation
// damage; fitness from the final number of occupied sites, equation
// final_fit_fun) with the synthetic model's rules:
//   step n:  (1) fraction at n?  live cell of class c survives iff w1 < T_c
//            (2) activity a = act[state], frozen until the next fraction
//            (3) `substeps` FTCS sub-steps
//                c' = c + lam (N + S + E + W - 4c) - kappa a  (O, G; then max(., 0))
//                H' = H + lam (N + S + E + W - 4H) + kappa a
//                (protocols timed in half-hours, the paper's 30-minute slots:
//                a fraction at the half hour runs (1) and (2) again after
//                substeps / 2 of them)
//            (4) synchronous cell update from the snapshot (lysis, environment,
//                division proposals into free von Neumann neighbours, conflict
//                resolution by the smallest key)
//            (5) live count (PROLIF + QUIESC) by wave reduction.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "gga_device.h"
#include "gga_internal.h"

namespace gga {
namespace {

constexpr uint32_t NONE_KEY = 0xFFFFFFFFu;
constexpr uint32_t INIT_STEP = 0xFFFFFFFFu;
constexpr int EMPTY = 0, PROLIF = 1, QUIESC = 2, DEAD = 3;
constexpr uint32_t DOOM_BIT = 1u << 14;    // cell word: lethally hit, awaiting mitotic death

// 32-bit linear-quadratic survival threshold, evaluated in float64 exactly as
// written: x = m d, y = m D, S = exp(-alpha x - beta x (x + 2 y)),
// T = min(floor(S 2^32), 2^32-1).  D is the unrepaired dose of earlier
// fractions (incomplete repair, see prior_damage); D = 0 is the plain law.
#pragma clang fp contract(off)
__device__ uint32_t lq_threshold(double d, double m, double alpha, double beta, double D) {
    const double x = m * d, y = m * D;
    const double e = -(alpha * x) - (beta * x) * (x + 2.0 * y);
    const double s = exp(e) * 4294967296.0;
    const double f = floor(s);
    return f >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)f;
}

// Unrepaired dose before fraction j of protocol p: the sum over earlier
// fractions i of d_i 2^(-(t_j - t_i) / half_time), in index order (times in
// hours, or half-hours scaled by 0.5); 0 when half_time is 0.
__device__ double prior_damage(const float* dose, const int32_t* gap, int j, long long tj, double half_time,
                               double unit) {
    if (!(half_time > 0.0)) return 0.0;
    double acc = 0.0;
    long long ti = 0;
    for (int i = 0; i < j; ++i) {
        ti += gap[i];
        const float di = dose[i];
        if (di > 0.0f) acc += (double)di * exp2(-(((double)(tj - ti) * unit) / half_time));
    }
    return acc;
}

// Oxygen modification factor of oxygen bin b (the oxygen effect, oer_max > 1):
// (oer_max o + K) / (oer_max (o + K)) at the bin's midpoint
// o = (b + 1/2) ghost_O / GGA_OER_BINS.
__device__ double oxygen_modification(const gga_params& P, int b) {
    const double o = (((double)b + 0.5) * (double)P.ghost[0]) / GGA_OER_BINS;
    return (P.oer_max * o + P.oer_k) / (P.oer_max * (o + P.oer_k));
}

// Oxygen bin of a site from its O in field units (O = o^ + ghost_O, rho_O = 1):
// floor(GGA_OER_BINS O / ghost_O) clamped to 0 .. GGA_OER_BINS - 1, in float64.
__device__ __forceinline__ int oxygen_bin(float o_hat, const gga_params& P) {
    const double q = ((double)o_hat + (double)P.ghost[0]) / (double)P.ghost[0];
    const double b = floor(q * GGA_OER_BINS);
    return b < 0.0 ? 0 : (b > GGA_OER_BINS - 1 ? GGA_OER_BINS - 1 : (int)b);
}
#pragma clang fp contract(on)

// CPL consecutive uint16 cell words of one row, read or written with one
// LDS access (the address is 2*CPL-byte aligned: x0 = lane * CPL; three
// columns per lane take one access per word).
template <int CPL>
__device__ __forceinline__ void load_words(const uint16_t* p, uint32_t (&w)[CPL]) {
    if constexpr (CPL == 1) {
        w[0] = p[0];
    } else if constexpr (CPL == 2) {
        const uint32_t v = *reinterpret_cast<const uint32_t*>(p);
        w[0] = v & 0xFFFFu; w[1] = v >> 16;
    } else if constexpr (CPL == 3) {
        w[0] = p[0]; w[1] = p[1]; w[2] = p[2];
    } else {
        static_assert(CPL == 4, "CPL must be 1, 2, 3 or 4");
        const uint2 v = *reinterpret_cast<const uint2*>(p);
        w[0] = v.x & 0xFFFFu; w[1] = v.x >> 16; w[2] = v.y & 0xFFFFu; w[3] = v.y >> 16;
    }
}
template <int CPL>
__device__ __forceinline__ void store_words(uint16_t* p, const uint32_t (&w)[CPL]) {
    if constexpr (CPL == 1) {
        p[0] = (uint16_t)w[0];
    } else if constexpr (CPL == 2) {
        *reinterpret_cast<uint32_t*>(p) = w[0] | (w[1] << 16);
    } else if constexpr (CPL == 3) {
        p[0] = (uint16_t)w[0]; p[1] = (uint16_t)w[1]; p[2] = (uint16_t)w[2];
    } else {
        *reinterpret_cast<uint2*>(p) = make_uint2(w[0] | (w[1] << 16), w[2] | (w[3] << 16));
    }
}

// Fields are held in kernel units c^ = (c - g_f) / rho_f: shifted by the
// field's Dirichlet boundary value g_f and scaled by rho_f = kappa'_f / kappa'_O
// (kappa' the signed reaction rate: -uptake for O and G, +production for H).
// In these units the boundary is 0 and every field's reaction term is the
// oxygen one, kappa'_O a, so one per-site term serves all three fields.  The
// FTCS update keeps its form: c' = lam S + (1 - 4 lam) c + r carries over to
// c^' = lam S^ + (1 - 4 lam) c^ + r / rho_f, because the shift g_f cancels
// (4 lam + (1 - 4 lam) - 1 = 0) and a neighbour on the boundary is g_f, i.e. 0.
__device__ __forceinline__ double field_rho(const gga_params& P, int f) {
    const double k0 = -(double)P.kappa[0];
    const double kf = f < 2 ? -(double)P.kappa[f] : (double)P.kappa[f];
    return kf / k0;
}
__device__ __forceinline__ float to_field_units(const gga_params& P, int f, double c) {
    return (float)((c - (double)P.ghost[f]) / field_rho(P, f));
}

// Constants of the cell update.  They sit in LDS and are read at their point
// of use after a barrier, so they do not occupy scalar registers across the
// diffusion loop.
struct CellConst {
    float thOq, thGq, thOd, thGd, thHd;
    int T_min, T_lys, ca0, ca1;
    uint32_t T_div;
};

template <int CPL>
__device__ __forceinline__ void store_keys(uint32_t* p, const uint32_t (&k)[CPL]) {
    if constexpr (CPL == 1) {
        p[0] = k[0];
    } else if constexpr (CPL == 2) {
        *reinterpret_cast<uint2*>(p) = make_uint2(k[0], k[1]);
    } else if constexpr (CPL == 3) {
        p[0] = k[0]; p[1] = k[1]; p[2] = k[2];
    } else {
        *reinterpret_cast<uint4*>(p) = make_uint4(k[0], k[1], k[2], k[3]);
    }
}

// L = 64 * CPL columns (LW of them the lattice's); NW waves of RPT rows hold
// RR = NW * RPT rows.  RR = LW: the whole lattice (resident).  RR < LW: a slab of a larger lattice advanced by
// one step per launch (the rows within `substeps + 2` of a slab edge that is
// not a lattice edge are a halo, recomputed by the neighbouring slab).
// Register slot of row i after k forward rotating sub-steps (S = RPT + 1 slots).
template <int S>
constexpr int rot_slot(int i, int k) { return ((i - k) % S + S) % S; }

template <int CPL, int RPT, int NW, int LW = 64 * CPL>
struct Geo {
    static constexpr int L = 64 * CPL;                // row pitch on the CU
    static constexpr int SIDE = LW;                   // lattice side
    static constexpr bool PAD = LW < L;               // columns past the lattice hold padding
    static constexpr bool PADC = PAD && LW % CPL != 0; // one lane holds lattice and padding columns
    static constexpr int NWAVE = NW;
    static constexpr int RR = NW * RPT;
    static constexpr bool SLAB = RR < LW;
    static constexpr int NT = 64 * NWAVE;
    static constexpr int BLK = 2 * 3 * L;             // one wave's halo block: [top/bottom][field][L]
    // Halo area [ghost][buffer 0: NW blocks][ghost]([buffer 1][ghost]): the ghost
    // blocks hold the boundary values, so the first and last wave read their
    // outer neighbour row like every other wave.  Double buffer when it fits
    // beside the cells and claim bits in LDS.
    static constexpr int area(int nbuf) { return (nbuf * (NWAVE + 1) + 1) * BLK; }
    static constexpr int NBUF = (RR * L * 2 + area(2) * 4 + RR * L / 8 + 4096 <= 160 * 1024) ? 2 : 1;
    static constexpr int AREA = area(NBUF);
    static constexpr int POOL = (AREA > RR * L) ? AREA : RR * L;
    static_assert(RR <= LW && NWAVE <= 16, "workgroup above 1024 threads");
    static_assert(LW <= L && L % 32 == 0, "rows of whole claim words");
    static_assert(RPT * CPL <= 32, "per-thread site masks are 32 bits wide");
    static constexpr uint32_t ALL = (RPT * CPL == 32) ? 0xFFFFFFFFu : ((1u << (RPT * CPL)) - 1u);
    // mask bits of the first / last column of every row (bit idx = i * CPL + c)
    static constexpr uint32_t col_bits(int c) {
        uint32_t m = 0;
        for (int i = 0; i < RPT; ++i) m |= 1u << (i * CPL + c);
        return m;
    }
    static constexpr uint32_t COL_FIRST = col_bits(0);
    static constexpr uint32_t COL_LAST = col_bits(CPL - 1);
};

// EXT: the extended radiobiology (the oxygen effect on radiosensitivity,
// gga_params.oer_max > 1, and mitotic death, gga_params.mitotic_death), a
// separate instantiation so that runs without them keep their register budget.
template <int CPL, int RPT, int NW, int LW, bool EXT, bool TEAM = false>
__global__ __launch_bounds__(64 * NW) void sim_kernel(SimArgs a) {
    using G = Geo<CPL, RPT, NW, LW>;
    constexpr int L = G::L;
    constexpr bool PAD = G::PAD, PADC = G::PADC;
    static_assert(!TEAM || G::SLAB, "teams are made of slabs");
    constexpr int RR = G::RR;
    constexpr int NWAVE = G::NWAVE;
    constexpr bool SLAB = G::SLAB;
    constexpr uint32_t ALL_SITES = G::ALL;

    __shared__ __attribute__((aligned(16))) uint16_t s_cell[RR * L];
    __shared__ __attribute__((aligned(16))) uint32_t s_pool[G::POOL];   // halo buffer(s), then claim slots
    __shared__ uint32_t s_claim[RR * L / 32 + 1];  // one "has a daughter" bit per site (and a spare word)
    __shared__ uint32_t s_ev_step[GGA_KMAX];   // half-hours since step n0 (2 (n - n0), + 1 at the half hour)
    __shared__ float s_ev_dose[GGA_KMAX];
    __shared__ double s_ev_prior[GGA_KMAX];    // unrepaired dose of the earlier fractions (incomplete repair)
    __shared__ uint32_t s_ev_thr[GGA_KMAX][4];
    // the current fraction's thresholds per class and oxygen bin (oxygen effect only)
    __shared__ uint32_t s_oer_thr[EXT ? 4 : 1][EXT ? GGA_OER_BINS : 1];
    __shared__ int s_nev, s_valid, s_evj[2];
    __shared__ int s_count[2];
    __shared__ int s_team_ok;
    __shared__ float s_react[4];               // reaction term per cell state
    __shared__ CellConst s_k;                  // cell-update constants, read where used

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    // instance (and slab) of this workgroup
    int inst, slab = 0, slab_row = 0;
    if constexpr (SLAB) {
        // Workgroups are dealt to the 8 XCDs in turn (block b to XCD b mod 8), so
        // all slabs of list position k go to XCD k mod 8: slab rows shared by
        // neighbouring slabs come from that XCD's L2.  b = (y * 8 + x) with
        // x = k mod 8 and y = (k / 8) * n_slabs + slab; positions past the list
        // are idle workgroups.
        const int x = (int)(blockIdx.x & 7u), y = (int)(blockIdx.x >> 3);
        const int kq = y / a.n_slabs;
        slab = y - kq * a.n_slabs;
        slab_row = kq * 8 + x;
        if (slab_row >= a.n_active) return;              // uniform across the workgroup
        inst = a.inst_list ? a.inst_list[slab_row] : slab_row;
    } else {
        inst = a.inst_list ? a.inst_list[blockIdx.x] : (int)blockIdx.x;
    }
    const int p = inst / a.R;
    const int r = inst - p * a.R;
    // state buffer row: the slab's list position; a library tumour (replica r
    // starts from library state r mod lib_n); or the instance
    const int slot = SLAB ? slab_row : (a.lib_n ? r % a.lib_n : inst);
    // the slab's first lattice row, and its own (non-halo) rows [iy0, iy1) of the slab
    const int ys = SLAB ? a.slab_ys[slab] : 0;
    const int iy0 = SLAB ? a.slab_i0[slab] : 0, iy1 = SLAB ? a.slab_i1[slab] : RR;
    const int lat0 = ys * LW;                        // lattice index of the slab's first site
    const int nsteps = ((!SLAB || TEAM) && a.horizon) ? a.horizon[p] : a.nsteps;
    const int y0 = wave * RPT;
    const int x0 = lane * CPL;
    // columns past the lattice hold padding: column x0 + c is the lattice's
    // when realc(c); real: the lane holds at least one lattice column
    auto realc = [&](int c) { return !PAD || x0 + c < LW; };
    const bool real = realc(0);
    // lattice index (the Philox site counter) of slab site index `site` (pitch L)
    auto lat_id = [&](int site) { return PAD ? (site / L) * LW + site % L + lat0 : site + lat0; };
    const gga_params& P = a.prm;
    // Philox key; `a` itself stays unmodified (a written kernel argument would
    // be copied to scratch memory)
    uint32_t seed_lo = a.seed_lo, seed_hi = a.seed_hi;
    if (a.generation) {             // per-generation key of a replayed GA generation
        const uint64_t key = a.seed + (uint64_t)(uint32_t)*a.generation * 0x9E3779B97F4A7C15ull;
        seed_lo = (uint32_t)key;
        seed_hi = (uint32_t)(key >> 32);
    }

    // ---- protocol: validity and irradiation events ----
    if constexpr (SLAB && !TEAM) {
        // event table (times in half-hours; at most one fraction at the start of
        // step n0 and one at its middle): lane j of wave 0 checks fraction j
        if (wave == 0) {
            const int k = a.ev_count[p];
            int j0 = -1, j1 = -1;
            for (int j = lane; j < k; j += 64) {
                const int tau = a.ev_step[(size_t)p * a.K + j];
                if (tau == 2 * a.n0) j0 = j;
                if (tau == 2 * a.n0 + 1) j1 = j;
            }
            const uint64_t m0 = __builtin_amdgcn_ballot_w64(j0 >= 0), m1 = __builtin_amdgcn_ballot_w64(j1 >= 0);
            const int J0 = m0 ? __shfl(j0, __builtin_ctzll(m0)) : -1;
            const int J1 = m1 ? __shfl(j1, __builtin_ctzll(m1)) : -1;
            if (lane == 0) {
                s_valid = a.ev_valid[p];
                int e = 0;
                if (J0 >= 0) { s_ev_step[e] = 0u; s_evj[e] = J0; ++e; }
                if (J1 >= 0) { s_ev_step[e] = 1u; s_evj[e] = J1; ++e; }
                s_nev = e;
            }
        }
    }
    if (tid == 0) {
        const int k = a.nfrac ? a.nfrac[p] : 0;
        int valid = (k >= 0 && k <= a.K);
        int nev = 0;
        double total = 0.0;
        long long t = 0;
        for (int j = 0; (!SLAB || TEAM) && valid && j < k; ++j) {
            const float d = a.dose[(size_t)p * a.K + j];
            const int g = a.gap[(size_t)p * a.K + j];
            if (!(d >= 0.0f) || !isfinite(d)) { valid = 0; break; }
            if (g < (j == 0 ? 0 : 1)) { valid = 0; break; }
            total += (double)d;
            t += g;
            // event time in half-hours (delays count half-hours with a.half)
            const long long tau = a.half ? t : 2 * t;
            if (d > 0.0f && tau >= 2LL * a.n0 && tau < 2LL * ((long long)a.n0 + nsteps)) {
                s_ev_step[nev] = (uint32_t)(tau - 2LL * a.n0);
                s_ev_dose[nev] = d;
                s_ev_prior[nev] = prior_damage(a.dose + (size_t)p * a.K, a.gap + (size_t)p * a.K, j, t,
                                               a.prm.repair_half_time, a.half ? 0.5 : 1.0);
                ++nev;
            }
        }
        if (valid && total > a.dose_cap + 1e-6) valid = 0;
        if (!SLAB || TEAM) {
            s_valid = valid;
            s_nev = nev;
        }
        const gga_params& Q = a.prm;
        // thresholds in field units (rho_O = 1, rho_G > 0, rho_H < 0: the host
        // requires positive rates, so "H above its threshold" reads H^ < th^)
        s_k.thOq = to_field_units(Q, 0, Q.theta_O_quiesce); s_k.thGq = to_field_units(Q, 1, Q.theta_G_quiesce);
        s_k.thOd = to_field_units(Q, 0, Q.theta_O_death); s_k.thGd = to_field_units(Q, 1, Q.theta_G_death);
        s_k.thHd = to_field_units(Q, 2, Q.theta_H_death);
        s_k.T_min = Q.T_min; s_k.T_lys = Q.T_lys;
        s_k.ca0 = Q.class_age[0]; s_k.ca1 = Q.class_age[1];
        s_k.T_div = (Q.P_div >= 1.0) ? 0xFFFFFFFFu : (uint32_t)floor(Q.P_div * 4294967296.0);
        s_count[0] = 0;
        s_count[1] = 0;
    }
    __syncthreads();
    if (!s_valid) {
        if (!SLAB && tid == 0 && a.live) a.live[inst] = -1;   // slabs: set before the first step
        return;                                   // uniform across the workgroup
    }
    const int nev = s_nev;
    if constexpr (SLAB && !TEAM) {
        if (tid < nev) {
            const EventFraction ef = a.ev_frac[(size_t)p * a.K + s_evj[tid]];
            s_ev_dose[tid] = ef.dose;
            s_ev_prior[tid] = ef.prior;
        }
        __syncthreads();
    }
    for (int e = tid; e < 4 * nev; e += G::NT)
        s_ev_thr[e >> 2][e & 3] = lq_threshold((double)s_ev_dose[e >> 2], P.m[e & 3], P.alpha, P.beta,
                                               s_ev_prior[e >> 2]);

    // ---- state: fields in registers, cells in LDS ----
    float F[3][RPT + 1][CPL];                  // slot RPT: spare row for the rotating sub-steps
    const size_t plane = (size_t)LW * LW;      // device-memory state: [3][LW][LW] fields, [LW][LW] cells
    if ((SLAB && !TEAM) || (a.mode & MODE_LOAD)) {
        const float* src = a.fields + (size_t)slot * 3 * plane + lat0;
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int i = 0; i < RPT; ++i)
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    F[f][i][c] = realc(c) ? src[f * plane + (size_t)(y0 + i) * LW + x0 + c] : 0.0f;
        const uint16_t* cs = a.cells + (size_t)slot * plane + lat0;
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int c = 0; c < CPL; ++c)
                s_cell[(y0 + i) * L + x0 + c] = realc(c) ? cs[(size_t)(y0 + i) * LW + x0 + c] : (uint16_t)0;
    } else {
        const int ctr = LW / 2;
        const int rad2 = P.seed_radius * P.seed_radius;
        float f0[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) f0[f] = to_field_units(P, f, P.init[f]);
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int i = 0; i < RPT; ++i)
#pragma unroll
                for (int c = 0; c < CPL; ++c) F[f][i][c] = realc(c) ? f0[f] : 0.0f;
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int y = ys + y0 + i, x = x0 + c;       // lattice row and column
                uint16_t w = 0;
                if (realc(c) && (x - ctr) * (x - ctr) + (y - ctr) * (y - ctr) <= rad2) {
                    const Block4 b = philox10(y * LW + x, INIT_STEP, r, p, seed_lo, seed_hi);
                    const uint32_t age = (uint32_t)(((uint64_t)b.w0 * (uint32_t)P.A0) >> 32);
                    w = (uint16_t)(PROLIF | (age << 2));
                }
                s_cell[(y0 + i) * L + x] = w;
            }
    }

    // Per-field constants (field units, see to_field_units): the update and the
    // lower clamp of O and G (c >= 0 reads c^ >= -g / rho, rho_O = 1 and
    // rho_G > 0); the one reaction rate kappa'_O enters through s_react.
    // Padding columns take lam = 0 and no clamp, so their fields stay 0 (per
    // column when a lane holds both kinds, else per lane).
    constexpr int NC = PADC ? CPL : 1;
    float lam[3][NC], cen[3], lo[2][NC];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
#pragma unroll
        for (int c = 0; c < NC; ++c) lam[f][c] = realc(c) ? P.lambda[f] : 0.0f;
        cen[f] = 1.0f - 4.0f * P.lambda[f];
    }
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int c = 0; c < NC; ++c) lo[f][c] = realc(c) ? to_field_units(P, f, 0.0) : -INFINITY;
    // reaction term per cell state, -kappa'_O a[state], looked up in LDS by
    // each site's state (one LDS read instead of a chain of selects)
    if (tid < 4) s_react[tid] = -P.kappa[0] * P.activity[tid];

    int ev = 0;
    int count = 0;
    __syncthreads();

    for (int n = a.n0; n < a.n0 + nsteps; ++n) {
        if constexpr (TEAM) {
            // the neighbouring slabs' rows of step n: wait for their step
            // counts, then reload this slab's halo rows from the exchange
            if (n > a.n0) {
                const int t = n - a.n0;
                // Polls are relaxed device-scope loads; one acquire fence
                // follows the last (an acquire per poll would invalidate the
                // caches on every iteration).  The compute unit's caches are
                // shared by the workgroup's waves, and none of them reads the
                // exchange rows before the barrier that follows the fence.
                // Both neighbours' counts are read in each poll, so a poll that
                // finds both published costs one memory round trip.
                if (tid == 0) {
                    int ok = a.spin_limit >= 0;
                    const int32_t* flags = a.team_flags + (size_t)slot * a.n_slabs;
                    const bool up = slab > 0, dn = slab + 1 < a.n_slabs;
                    int k = 0;
                    while (ok) {
                        const int fu = up ? __hip_atomic_load(flags + slab - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : t;
                        const int fd = dn ? __hip_atomic_load(flags + slab + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : t;
                        if (fu >= t && fd >= t) break;
                        if (++k > a.spin_limit) { ok = 0; break; }
                        __builtin_amdgcn_s_sleep(1);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    s_team_ok = ok;
                }
                __syncthreads();
                if (!s_team_ok) {                        // uniform: this workgroup leaves
                    if (tid == 0 && a.live) atomicExch(&a.live[inst], (int)0x80000000);
                    return;
                }
                const float* src = ((t & 1) ? a.fields_out : a.fields) + (size_t)slot * 3 * plane + lat0;
                const uint16_t* cs = ((t & 1) ? a.cells_out : a.cells) + (size_t)slot * plane + lat0;
                // Per halo row (wave-uniform): the cell words go from the
                // exchange straight into the LDS row by LDS DMA (lane l moves
                // the row's 32-bit word d0 + l; padding columns past LW are
                // not touched and stay EMPTY), so no register holds them and
                // no LDS write waits for its load: the rows' loads are all in
                // flight together.  The fields load into F.
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int y = y0 + i;
                    if (y < iy0 || y >= iy1) {
                        const uint32_t* gw = reinterpret_cast<const uint32_t*>(cs + (size_t)y * LW);
                        uint32_t* lw = reinterpret_cast<uint32_t*>(s_cell + y * L);
#pragma unroll
                        for (int d0 = 0; d0 < LW / 2; d0 += 64)
                            if (d0 + lane < LW / 2)
                                __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)(gw + d0 + lane),
                                                                 (__attribute__((address_space(3))) void*)(lw + d0), 4, 0, 0);
                        if (real) {
#pragma unroll
                            for (int f = 0; f < 3; ++f)
#pragma unroll
                                for (int c = 0; c < CPL; ++c)
                                    if (realc(c)) F[f][i][c] = src[f * plane + (size_t)y * LW + x0 + c];
                        }
                    }
                }
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the DMA writes have landed in LDS
                __syncthreads();                          // halo cells in before anyone reads them
            }
        }
        // Every LDS access below addresses a row as base + constant offset.  The
        // base is opaque to the compiler at the top of each step, so per-row
        // addresses are not hoisted out of the loop into registers.
        int own = y0 * L + x0;
        asm volatile("" : "+v"(own));
        uint16_t* const cellp = s_cell + own;            // row i: cellp + i * L
        float Ro[RPT][CPL];                              // reaction term, set below
        // (3) diffusion sub-steps, in pairs over the RPT + 1 register slots with
        // no row copied: a forward sub-step (rows top to bottom) writes new row
        // i over old row i - 1, which row i was the last to read, moving every
        // row one slot down; the reverse sub-step that follows (rows bottom to
        // top) writes new row i over old row i + 1 and moves them back, so after
        // each pair every row is in its own slot again.  An odd last sub-step
        // runs in the plain form with a copy of the row above.
        // Per field and column: the halo rows of this wave's neighbours, then
        // c' = lam (up + below + west + east) + (c cen + r).
        auto halo = [&](auto slot0, auto slotL, int par, float (&up)[3][CPL], float (&dn)[3][CPL]) {
            // Ro is opaque here, so nothing derived from it is hoisted out of
            // the sub-step loop to hold VGPRs across it.
#pragma unroll
            for (int i = 0; i < RPT; ++i)
#pragma unroll
                for (int c = 0; c < CPL; ++c) asm volatile("" : "+v"(Ro[i][c]));
            // this wave's halo block: [top/bottom][field][L] at wave * 6 L
            float* const hw = reinterpret_cast<float*>(s_pool) + ((G::NBUF == 2 ? par * (NWAVE + 1) : 0) + 1 + wave) * G::BLK + x0;
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    hw[f * L + c] = F[f][decltype(slot0)::value][c];
                    hw[(3 + f) * L + c] = F[f][decltype(slotL)::value][c];
                }
            __syncthreads();
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    up[f][c] = hw[(f - 3) * L + c];     // bottom row of wave-1 (or a ghost block)
                    dn[f][c] = hw[(6 + f) * L + c];     // top row of wave+1 (or a ghost block)
                }
            if constexpr (G::NBUF == 1) __syncthreads();   // one buffer: all reads before the next writes
        };
        auto update = [&](int f, int i, int c, float up, float below, float west, float east, float cur) {
            const float sum = (up + below) + (west + east);
            float v = fmaf(lam[f][PADC ? c : 0], sum, fmaf(cur, cen[f], Ro[i][c]));
            if (f < 2) v = fmaxf(v, lo[f][PADC ? c : 0]);
            return v;
        };
        auto rotating_substep = [&](auto KC, int par) {
            constexpr int k = decltype(KC)::value;
            // sub-steps stay in order: no work moves across this point
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int j = 0; j <= RPT; ++j)
#pragma unroll
                    for (int c = 0; c < CPL; ++c) asm volatile("" : "+v"(F[f][j][c]));
            float up[3][CPL], dn[3][CPL];
            halo(std::integral_constant<int, rot_slot<RPT + 1>(0, k)>{},
                 std::integral_constant<int, rot_slot<RPT + 1>(RPT - 1, k)>{}, par, up, dn);
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int si = rot_slot<RPT + 1>(i, k), sa = rot_slot<RPT + 1>(i - 1, k);
#pragma unroll
                for (int f = 0; f < 3; ++f)
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const float above = (i == 0) ? up[f][c] : F[f][sa][c];
                        const float below = (i < RPT - 1) ? F[f][rot_slot<RPT + 1>(i + 1, k)][c] : dn[f][c];
                        const float west = (c > 0) ? F[f][si][c - 1] : lane_from_left(F[f][si][CPL - 1]);
                        const float east = (c < CPL - 1) ? F[f][si][c + 1] : lane_from_right(F[f][si][0]);
                        // old row i - 1 (slot sa) is dead once row i has read it
                        F[f][sa][c] = update(f, i, c, above, below, west, east, F[f][si][c]);
                    }
            }
        };
        // Reverse sub-step with the map of the forward one k (row i in slot
        // rot_slot(i, k)); afterwards row i is in slot rot_slot(i, k - 1).
        auto reverse_substep = [&](auto KC, int par) {
            constexpr int k = decltype(KC)::value;
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int j = 0; j <= RPT; ++j)
#pragma unroll
                    for (int c = 0; c < CPL; ++c) asm volatile("" : "+v"(F[f][j][c]));
            float up[3][CPL], dn[3][CPL];
            halo(std::integral_constant<int, rot_slot<RPT + 1>(0, k)>{},
                 std::integral_constant<int, rot_slot<RPT + 1>(RPT - 1, k)>{}, par, up, dn);
#pragma unroll
            for (int i = RPT - 1; i >= 0; --i) {
                const int si = rot_slot<RPT + 1>(i, k), sb = rot_slot<RPT + 1>(i + 1, k);
#pragma unroll
                for (int f = 0; f < 3; ++f)
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const float above = (i == 0) ? up[f][c] : F[f][rot_slot<RPT + 1>(i - 1, k)][c];
                        const float below = (i < RPT - 1) ? F[f][sb][c] : dn[f][c];
                        const float west = (c > 0) ? F[f][si][c - 1] : lane_from_left(F[f][si][CPL - 1]);
                        const float east = (c < CPL - 1) ? F[f][si][c + 1] : lane_from_right(F[f][si][0]);
                        // old row i + 1 (slot sb; the spare slot for the last row) is dead once row i has read it
                        F[f][sb][c] = update(f, i, c, above, below, west, east, F[f][si][c]);
                    }
            }
        };
        auto plain_substep = [&](int par) {
            float up[3][CPL], dn[3][CPL];
            halo(std::integral_constant<int, 0>{}, std::integral_constant<int, RPT - 1>{}, par, up, dn);
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                float nw[3][CPL];
#pragma unroll
                for (int f = 0; f < 3; ++f)
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const float below = (i < RPT - 1) ? F[f][i + 1][c] : dn[f][c];
                        const float west = (c > 0) ? F[f][i][c - 1] : lane_from_left(F[f][i][CPL - 1]);
                        const float east = (c < CPL - 1) ? F[f][i][c + 1] : lane_from_right(F[f][i][0]);
                        nw[f][c] = update(f, i, c, up[f][c], below, west, east, F[f][i][c]);
                    }
#pragma unroll
                for (int f = 0; f < 3; ++f)
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        up[f][c] = F[f][i][c];
                        F[f][i][c] = nw[f][c];
                    }
            }
        };
        // ghost blocks (the cell update's claim slots share this memory); the
        // first sub-step's barrier orders these writes before any read
        for (int k = tid; k < (G::NBUF + 1) * G::BLK; k += G::NT) {
            const int blk = k / G::BLK, off = k - blk * G::BLK;
            reinterpret_cast<float*>(s_pool)[blk * (NWAVE + 1) * G::BLK + off] = 0.0f;   // the boundary, in field units
        }
        const uint32_t rel = 2u * (uint32_t)(n - a.n0);  // the hour's start, in half-hours since step n0
        int s = 0;
#pragma nounroll
        for (uint32_t half = 0;; half = 1) {
            // (1) irradiation: every live cell draws w1 against its class
            // threshold, at the start of the hour or, for a fraction timed at
            // the half hour, after half of the hour's sub-steps (its words from
            // the block of step word n | 2^31)
            if (ev < nev && s_ev_step[ev] == rel + half) {
                // with the oxygen effect: this fraction's thresholds per class
                // and oxygen bin, and each site's bin from its current O
                const bool oer = EXT && P.oer_max > 1.0, mitotic = EXT && P.mitotic_death != 0;
                if (oer) {
                    __syncthreads();                      // the previous fraction's table is read
                    if (tid < 4 * GGA_OER_BINS) {
                        const double f = oxygen_modification(P, tid % GGA_OER_BINS);
                        s_oer_thr[tid / GGA_OER_BINS][tid % GGA_OER_BINS] =
                            lq_threshold(f * (double)s_ev_dose[ev], P.m[tid / GGA_OER_BINS], P.alpha, P.beta,
                                         f * s_ev_prior[ev]);
                    }
                    __syncthreads();
                }
                const uint32_t t0 = s_ev_thr[ev][0], t1 = s_ev_thr[ev][1];
                const uint32_t t2 = s_ev_thr[ev][2], t3 = s_ev_thr[ev][3];
                const int ca0 = s_k.ca0, ca1 = s_k.ca1;
                uint32_t live_mask = 0;
#pragma unroll
                for (int i = 0; i < RPT; ++i)
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const uint32_t w = cellp[i * L + c];
                        const int st = w & 3;
                        if (st == PROLIF || st == QUIESC) {
                            live_mask |= 1u << (i * CPL + c);
                            // the site's oxygen bin rides in the word's free bits 10-13
                            // until this fraction is done
                            if (oer) cellp[i * L + c] = (uint16_t)(w | ((uint32_t)oxygen_bin(F[0][i][c], P) << 10));
                        }
                    }
                while (live_mask) {
                    const int idx = __builtin_ctz(live_mask);
                    live_mask &= live_mask - 1;
                    const int site = own + (idx / CPL) * L + idx % CPL;
                    const uint32_t w = s_cell[site];
                    const int st = w & 3, age = EXT ? (w >> 2) & 255 : w >> 2;
                    uint32_t thr = (st == QUIESC) ? t3 : (age < ca0 ? t0 : (age < ca1 ? t1 : t2));
                    if (oer) {
                        const int cls = (st == QUIESC) ? 3 : (age < ca0 ? 0 : (age < ca1 ? 1 : 2));
                        thr = s_oer_thr[cls][(w >> 10) & 15u];
                    }
                    const Block4 b = philox10(lat_id(site), (uint32_t)n | (half << 31), r, p, seed_lo, seed_hi);
                    // mitotic death: the cell lives on, marked, until it next divides
                    if (b.w1 >= thr) s_cell[site] = mitotic ? (uint16_t)(w | DOOM_BIT) : (uint16_t)DEAD;
                }
                if (oer) {
#pragma unroll
                    for (int i = 0; i < RPT; ++i)
#pragma unroll
                        for (int c = 0; c < CPL; ++c) cellp[i * L + c] = (uint16_t)(cellp[i * L + c] & ~0x3C00u);
                }
                ++ev;
            }

            // (2) reaction term until the next fraction or the end of the hour,
            // one per site for all three fields in field units: Ro = -kappa_O a.
#pragma unroll
            for (int i = 0; i < RPT; ++i)
#pragma unroll
                for (int c = 0; c < CPL; ++c) Ro[i][c] = realc(c) ? s_react[cellp[i * L + c] & 3] : 0.0f;
            // (3) the sub-steps up to a fraction at the half hour, or to the end of the hour
            const int stop = (half == 0 && ev < nev && s_ev_step[ev] == rel + 1) ? a.substeps / 2 : a.substeps;
            for (; s + 2 <= stop; s += 2) {
                rotating_substep(std::integral_constant<int, 0>{}, s & 1);
                reverse_substep(std::integral_constant<int, 1>{}, (s + 1) & 1);
            }
            if (s < stop) {
                plain_substep(s & 1);
                ++s;
            }
            if (stop == a.substeps) break;
        }
        if constexpr (TEAM) {
            // The fields of the rows the neighbours hold as halo are final
            // now (the cell update does not change them): their stores go out
            // here and drain during the cell update; the cell words and the
            // step count follow it.
            if (n + 1 < a.n0 + nsteps) {
                const int t1 = n + 1 - a.n0;
                float* fd = ((t1 & 1) ? a.fields_out : a.fields) + (size_t)slot * 3 * plane + lat0;
                const int exA = a.slab_exA[slab], exB = a.slab_exB[slab];
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int y = y0 + i;
                    if (real && y >= iy0 && y < iy1 && (y < exA || y >= exB)) {
#pragma unroll
                        for (int f = 0; f < 3; ++f)
#pragma unroll
                            for (int c = 0; c < CPL; ++c)
                                if (realc(c)) fd[f * plane + (size_t)y * LW + x0 + c] = F[f][i][c];
                    }
                }
            }
        }

        // (4) cell update, bit-parallel over the thread's RPT x CPL sites
        // (bit idx = i * CPL + c of 32-bit masks).  Proposers claim an EMPTY
        // target with ds_min_u32 on best[t] (one slot per site, sharing the
        // halo pool) and set the target's bit in s_claim; the smallest key's
        // low two bits name the winner's direction, so no key is kept.
        __syncthreads();   // the last sub-step's halo reads are done
        uint32_t* best = s_pool;
        uint32_t* const bestp = best + own;              // row i: bestp + i * L
        // From the snapshot: the EMPTY state of the rows just above and below
        // this slab (owned by the neighbouring waves) and whether any of this
        // wave's sites holds a cell.
        uint32_t top = 0, bot = 0, occupied = 0;
        if (wave > 0) {
            uint32_t w[CPL];
            load_words<CPL>(cellp - L, w);
#pragma unroll
            for (int c = 0; c < CPL; ++c) top |= (uint32_t)((w[c] & 3u) == EMPTY) << c;
        }
        if (wave < NWAVE - 1) {
            uint32_t w[CPL];
            load_words<CPL>(cellp + RPT * L, w);
#pragma unroll
            for (int c = 0; c < CPL; ++c) bot |= (uint32_t)((w[c] & 3u) == EMPTY) << c;
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            uint32_t w[CPL];
            load_words<CPL>(cellp + i * L, w);
#pragma unroll
            for (int c = 0; c < CPL; ++c) occupied |= w[c];
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            uint32_t none[CPL];
#pragma unroll
            for (int c = 0; c < CPL; ++c) none[c] = NONE_KEY;
            store_keys<CPL>(bestp + i * L, none);
        }
        for (int k = tid; k < RR * L / 32; k += G::NT) s_claim[k] = 0u;
        __syncthreads();   // boundary rows read, claims reset: own rows may now be rewritten
        // Per site: lysis and environment transitions, written back row by row.
        // padding sites are never free
        uint32_t real_m = real ? ALL_SITES : 0u;
        if constexpr (PADC) {
            real_m = 0;
#pragma unroll
            for (int i = 0; i < RPT; ++i)
#pragma unroll
                for (int c = 0; c < CPL; ++c) real_m |= (uint32_t)realc(c) << (i * CPL + c);
        }
        uint32_t empty_m = real_m, cyc_m = 0, old_m = 0, alive_m = 0, doom_m = 0;
        if (__builtin_amdgcn_ballot_w64(occupied != 0u) != 0) {   // wave-uniform; else all EMPTY
            // Environment flags of the thread's sites, from the fields after the
            // sub-steps (x < th  <=>  sign bit of x - th: the difference of two
            // finite floats is zero only when they are equal and otherwise keeps
            // the sign of the exact difference).
            uint32_t nec_m = 0, starv_m = 0;
            {
                const float thOq = s_k.thOq, thGq = s_k.thGq, thOd = s_k.thOd, thGd = s_k.thGd, thHd = s_k.thHd;
#pragma unroll
                for (int i = 0; i < RPT; ++i)
#pragma unroll
                    for (int c = 0; c < CPL; ++c) {
                        const int idx = i * CPL + c;
                        const float O = F[0][i][c], Gl = F[1][i][c], H = F[2][i][c];
                        nec_m |= ((__float_as_uint(Gl - thGd) | __float_as_uint(O - thOd) |
                                   __float_as_uint(H - thHd)) >> 31) << idx;
                        starv_m |= ((__float_as_uint(O - thOq) | __float_as_uint(Gl - thGq)) >> 31) << idx;
                        asm volatile("" : "+v"(nec_m), "+v"(starv_m));   // fold each site in now
                    }
            }
            const int T_lys = s_k.T_lys, T_min = s_k.T_min;
            empty_m = 0;
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                uint32_t w[CPL];
                load_words<CPL>(cellp + i * L, w);
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int idx = i * CPL + c;
                    const uint32_t st = w[c] & 3u, age = EXT ? (w[c] >> 2) & 255u : w[c] >> 2;
                    const uint32_t older = age < 255u ? age + 1u : 255u;
                    const uint32_t nec = (nec_m >> idx) & 1u, starv = (starv_m >> idx) & 1u;
                    const uint32_t live = (0x6u >> st) & 1u;
                    // branch-free selects: x ^ ((y ^ x) & -flag) picks y when flag is 1
                    // a live cell keeps its mitotic-death mark (EXT); dead words carry none
                    const uint32_t kept = (uint32_t)QUIESC | (w[c] & ~3u);
                    const uint32_t grown = (uint32_t)PROLIF | (older << 2) | (EXT ? (w[c] & DOOM_BIT) : 0u);
                    uint32_t nl = grown ^ ((kept ^ grown) & (0u - starv));          // live outcome
                    nl ^= (nl ^ (uint32_t)DEAD) & (0u - nec);
                    const uint32_t decay = (uint32_t)((st == DEAD) & ((int)older < T_lys));
                    const uint32_t nd = ((uint32_t)DEAD | (older << 2)) & (0u - decay);  // DEAD ages or lyses
                    w[c] = nd ^ ((nl ^ nd) & (0u - live));
                    empty_m |= (uint32_t)(st == EMPTY) << idx;
                    cyc_m |= (live & ~(nec | starv) & 1u) << idx;
                    old_m |= (uint32_t)((int)age >= T_min) << idx;
                    alive_m |= (live & ~nec & 1u) << idx;
                    if constexpr (EXT) doom_m |= ((w[c] >> 14) & 1u) << idx;
                    asm volatile("" : "+v"(empty_m), "+v"(cyc_m), "+v"(old_m), "+v"(alive_m));
                }
                store_words<CPL>(cellp + i * L, w);
            }
            if constexpr (PAD) empty_m &= real_m;
        }
        constexpr uint32_t C0 = G::COL_FIRST, CL = G::COL_LAST;
        const uint32_t fN = ((empty_m << CPL) | top) & ALL_SITES;
        const uint32_t fS = (empty_m >> CPL) | (bot << ((RPT - 1) * CPL));
        const uint32_t from_left = lane_from_left_u32(empty_m), from_right = lane_from_right_u32(empty_m);
        const uint32_t fW = (CPL == 1) ? from_left : (((empty_m << 1) & ~C0 & ALL_SITES) | ((from_left >> (CPL - 1)) & C0));
        const uint32_t fE = (CPL == 1) ? from_right : (((empty_m >> 1) & ~CL) | ((from_right << (CPL - 1)) & CL));
        // marked cells never divide: they draw their block whatever their
        // neighbours and die when ready (mitotic death)
        const uint32_t cand = cyc_m & old_m & ~doom_m & (fN | fE | fS | fW);
        if constexpr (EXT) {
            uint32_t m = cyc_m & old_m & doom_m;
            while (m) {
                const int idx = __builtin_ctz(m);
                m &= m - 1;
                const int site = own + (idx / CPL) * L + idx % CPL;
                const Block4 b = philox10(lat_id(site), n, r, p, seed_lo, seed_hi);
                if (b.w3 < s_k.T_div) {
                    cellp[(idx / CPL) * L + idx % CPL] = (uint16_t)DEAD;
                    alive_m &= ~(1u << idx);
                }
            }
        }
        uint32_t prop_m = 0;
        uint64_t dirs = 0;
        {
            uint32_t m = cand;
            while (m) {
                const int idx = __builtin_ctz(m);
                m &= m - 1;
                const int site = own + (idx / CPL) * L + idx % CPL;
                const Block4 b = philox10(lat_id(site), n, r, p, seed_lo, seed_hi);
                if (b.w3 < s_k.T_div) {
                    const uint32_t fm = ((fN >> idx) & 1u) | (((fE >> idx) & 1u) << 1) |
                                        (((fS >> idx) & 1u) << 2) | (((fW >> idx) & 1u) << 3);
                    const uint32_t kth = (uint32_t)(((uint64_t)b.w0 * __builtin_popcount(fm)) >> 32);
                    uint32_t rest = fm;
                    for (uint32_t j = 0; j < kth; ++j) rest &= rest - 1;
                    const uint32_t dir = __builtin_ctz(rest);                 // 0 N, 1 E, 2 S, 3 W
                    const int t = site + (dir == 0 ? -L : dir == 1 ? 1 : dir == 2 ? L : -1);
                    atomicMin(&best[t], ((b.w2 >> 3) << 2) | ((dir + 2) & 3u));
                    atomicOr(&s_claim[t >> 5], 1u << (t & 31));
                    prop_m |= 1u << idx;
                    dirs |= (uint64_t)dir << (2 * idx);
                }
            }
        }
        __syncthreads();   // all claims are in
        uint32_t won_m = 0;
        {
            uint32_t m = prop_m;
            while (m) {
                const int idx = __builtin_ctz(m);
                m &= m - 1;
                const uint32_t dir = (uint32_t)(dirs >> (2 * idx)) & 3u;
                const int site = own + (idx / CPL) * L + idx % CPL;
                const int t = site + (dir == 0 ? -L : dir == 1 ? 1 : dir == 2 ? L : -1);
                if ((best[t] & 3u) == ((dir + 2) & 3u)) won_m |= 1u << idx;
            }
        }
        uint32_t born_m = 0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int wi = (own >> 5) + i * (L / 32);
            if constexpr (32 % CPL == 0) {
                born_m |= ((s_claim[wi] >> (x0 & 31)) & ((1u << CPL) - 1u)) << (i * CPL);
            } else {                             // a lane's bits may run into the next word
                const uint64_t two = (uint64_t)s_claim[wi] | ((uint64_t)s_claim[wi + 1] << 32);
                born_m |= ((uint32_t)(two >> (x0 & 31)) & ((1u << CPL) - 1u)) << (i * CPL);
            }
        }
        born_m &= empty_m;
        {
            uint32_t m = born_m | won_m;             // daughters and winning parents restart at age 0
            while (m) {
                const int idx = __builtin_ctz(m);
                m &= m - 1;
                cellp[(idx / CPL) * L + idx % CPL] = (uint16_t)PROLIF;
            }
        }
        uint32_t counted = alive_m | born_m;
        if constexpr (SLAB) {                      // a slab counts its own rows only
            uint32_t own_rows = 0;
#pragma unroll
            for (int i = 0; i < RPT; ++i)
                own_rows |= (uint32_t)(y0 + i >= iy0 && y0 + i < iy1) * (((1u << CPL) - 1u) << (i * CPL));
            counted &= own_rows;
        }
        int live = __builtin_popcount(counted);
        // (5) live count: wave reduction, one LDS atomic per wave
        live = wave_sum(live);
        if (lane == 0) atomicAdd(&s_count[n & 1], live);
        __syncthreads();
        if (tid == 0) {
            count = s_count[n & 1];
            s_count[(n + 1) & 1] = 0;
            if (!SLAB && a.traj) a.traj[(size_t)inst * a.nsteps + (n - a.n0)] = count;
            // slabs: this slab's share of step n's count
            if (SLAB && a.traj) atomicAdd(&a.traj[(size_t)inst * a.count_at + n], count);
        }
        if constexpr (TEAM) {
            // publish the cell words of the own rows the neighbours hold as
            // halo (their fields went out after the sub-steps), then the step
            // count
            if (n + 1 < a.n0 + nsteps) {
                const int t1 = n + 1 - a.n0;
                uint16_t* cd = ((t1 & 1) ? a.cells_out : a.cells) + (size_t)slot * plane + lat0;
                const int exA = a.slab_exA[slab], exB = a.slab_exB[slab];
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int y = y0 + i;
                    if (real && y >= iy0 && y < iy1 && (y < exA || y >= exB)) {
#pragma unroll
                        for (int c = 0; c < CPL; ++c)
                            if (realc(c)) cd[(size_t)y * LW + x0 + c] = s_cell[y * L + x0 + c];
                    }
                }
                // every wave's rows have reached the cache hierarchy before the
                // barrier; one device-scope release then publishes them all
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
                if (tid == 0)
                    __hip_atomic_store(a.team_flags + (size_t)slot * a.n_slabs + slab, t1, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }

    // The lane and thread index again, from the lane count: keeping them live
    // across the step loop for the uses below would take a register.
    const int lane_end = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const int tid_end = wave * 64 + lane_end;
    if ((!SLAB || TEAM) && nsteps == 0) {
        int live = 0;
#pragma unroll
        for (int i = 0; i < RPT; ++i)
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int st = s_cell[(y0 + i) * L + x0 + c] & 3;
                live += (st == PROLIF || st == QUIESC) && (!SLAB || (y0 + i >= iy0 && y0 + i < iy1));
            }
        live = wave_sum(live);
        if (lane_end == 0) atomicAdd(&s_count[0], live);
        __syncthreads();
        if (tid_end == 0) count = s_count[0];
    }
    if constexpr (TEAM) {
        // the instance's last step (or its initial state): this slab's share
        if (tid_end == 0 && a.live) atomicAdd(&a.live[inst], count);
    } else if constexpr (SLAB) {
        // the instance's last step: add this slab's share of the live count
        if (tid_end == 0 && a.live && a.n0 + 1 == (a.horizon ? a.horizon[p] : a.count_at)) atomicAdd(&a.live[inst], count);
    } else {
        if (tid_end == 0 && a.live) a.live[inst] = count;
    }

    if ((SLAB && !TEAM) || (a.mode & MODE_STORE)) {
        // slabs write their own rows into the other state buffer
        float* dst = (SLAB ? a.fields_out : a.fields) + (size_t)slot * 3 * plane + lat0;
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int i = 0; i < RPT; ++i)
                if (real && (!SLAB || (y0 + i >= iy0 && y0 + i < iy1)))
#pragma unroll
                    for (int c = 0; c < CPL; ++c)
                        if (realc(c)) dst[f * plane + (size_t)(y0 + i) * LW + x0 + c] = F[f][i][c];
        __syncthreads();
        uint16_t* cd = (SLAB ? a.cells_out : a.cells) + (size_t)slot * plane + lat0;
#pragma unroll
        for (int i = 0; i < RPT; ++i)
            if (real && (!SLAB || (y0 + i >= iy0 && y0 + i < iy1)))
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    if (realc(c)) cd[(size_t)(y0 + i) * LW + x0 + c] = s_cell[(y0 + i) * L + x0 + c];
    }
}

}  // namespace
}  // namespace gga
