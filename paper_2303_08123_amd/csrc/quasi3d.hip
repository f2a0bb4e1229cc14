// Quasi-3D variant of the simulation: every lattice site holds C cell slots
// (the paper's model is quasi-three-dimensional, with many cells to a site),
// while oxygen, glucose and acidity stay two-dimensional.
//
// Rules beyond the 2D model (with C = 1 they are the 2D model's):
//   - slot z of site s draws the Philox block of site counter z L^2 + s;
//   - a site's reaction term is the mean over its slots of -kappa_O act[state];
//   - a ready cell's free places are the EMPTY slots of its own site and of its
//     four von Neumann neighbours, in the order own, N, E, S, W and by slot
//     within a site; it proposes the k-th, k = floor(w0 m / 2^32), with the
//     64-bit key ((w2 >> 3) << 8) | (d << 5) | z (d = 4 for its own site,
//     otherwise its direction seen from the target: N 0, E 1, S 2, W 3), and
//     every EMPTY slot takes the smallest key.
//
// Layout and launches.  The state of instance i is fields[i][3][L][L] and
// cells[i][C][L][L]: slot planes, so that for every slot the 64 lanes of a
// wave touch 64 consecutive sites.  An instance on a 128^2 lattice with 8
// slots holds 256 KiB of words plus 192 KiB of fields, more than a compute
// unit's LDS, so the state stays in device memory and a step is a chain of launches
// over all instances at once: fraction, the FTCS sub-steps (fused in LDS
// tiles, two field buffers), a fraction at the half hour, cell update,
// resolution.  The per-site launches have one thread per site; an instance's
// blocks are numbered so that they run on one XCD (blocks are dealt to the 8
// XCDs in turn), keeping the rows a block shares with its neighbours in one L2.
#include "quasi3d.h"
#include "sim_kernel.h"

namespace gga {
namespace {

constexpr int Q3_NT = 256;
constexpr unsigned long long NONE_KEY64 = ~0ull;

__host__ __device__ inline unsigned q3_blocks_per_inst(int L) { return ((unsigned)L * L + Q3_NT - 1) / Q3_NT; }
__host__ __device__ inline unsigned q3_per_xcd(const Q3Args& a) {
    return ((unsigned)a.n_inst * q3_blocks_per_inst(a.L) + 7u) / 8u;
}

// Instance and site of this thread.  Hardware block b runs on XCD b mod 8;
// logical block lb = (b mod 8) * per_xcd + b / 8 puts consecutive logical
// blocks, and so the blocks of one instance, on one XCD.  False (for the whole
// block) past the last logical block.
__device__ __forceinline__ bool q3_place(const Q3Args& a, int& inst, int& site) {
    const unsigned nbx = q3_blocks_per_inst(a.L);
    const unsigned per = q3_per_xcd(a);
    const unsigned b = blockIdx.x;
    const unsigned lb = (b & 7u) * per + (b >> 3);
    if (lb >= (unsigned)a.n_inst * nbx) return false;
    inst = (int)(lb / nbx);
    site = (int)(lb - (unsigned)inst * nbx) * Q3_NT + (int)threadIdx.x;
    return true;
}

__device__ __forceinline__ int sens_class(uint32_t w, const gga_params& P) {
    const int st = w & 3, age = (w >> 2) & 255;
    return st == QUIESC ? 3 : (age < P.class_age[0] ? 0 : (age < P.class_age[1] ? 1 : 2));
}

// Reaction term of a site: the mean of -kappa_O act[state] over its slots
// (the sum alone for one slot, so that C = 1 reproduces the 2D term exactly).
__device__ __forceinline__ float site_react(const float* s_react, const uint16_t* cw, int C, int L2, int site) {
    float acc = s_react[cw[site] & 3];
    for (int z = 1; z < C; ++z) acc += s_react[cw[(size_t)z * L2 + site] & 3];
    return C > 1 ? acc * (1.0f / (float)C) : acc;
}

__device__ __forceinline__ void set_react_table(const gga_params& P, float* s_react) {
    if (threadIdx.x < 4) s_react[threadIdx.x] = -P.kappa[0] * P.activity[threadIdx.x];
}

// Adds the block's live count to *dst (no-op for a null dst).
__device__ __forceinline__ void block_count(int cnt, int32_t* dst, int* s_part) {
    cnt = wave_sum(cnt);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0 && dst) {
        int t = 0;
        for (int w = 0; w < Q3_NT / 64; ++w) t += s_part[w];
        atomicAdd(dst, t);
    }
}

// Initial state: uniform fields, slot 0 the 2D model's seed disc (Philox ages
// from the block at step 0xFFFFFFFF), the other slots EMPTY.
__global__ void __launch_bounds__(Q3_NT) q3_init_kernel(Q3Args a) {
    int inst, site;
    if (!q3_place(a, inst, site)) return;
    const int L = a.L, L2 = L * L;
    if (site >= L2) return;
    const int p = inst / a.R, r = inst - p * a.R;
    float* F = a.fields + (size_t)inst * 3 * L2;
    for (int f = 0; f < 3; ++f) F[(size_t)f * L2 + site] = to_field_units(a.prm, f, a.prm.init[f]);
    uint16_t* cw = a.cells + (size_t)inst * a.C * L2;
    const int y = site / L, x = site - y * L, ctr = L / 2;
    uint16_t w = 0;
    if ((x - ctr) * (x - ctr) + (y - ctr) * (y - ctr) <= a.prm.seed_radius * a.prm.seed_radius) {
        const Block4 b = philox10((uint32_t)site, INIT_STEP, (uint32_t)r, (uint32_t)p, a.seed_lo, a.seed_hi);
        const uint32_t age = (uint32_t)(((uint64_t)b.w0 * (uint32_t)a.prm.A0) >> 32);
        w = (uint16_t)(PROLIF | (age << 2));
    }
    cw[site] = w;
    for (int z = 1; z < a.C; ++z) cw[(size_t)z * L2 + site] = 0;
}

// live[i] = 0 and traj[i][*] = 0 for valid protocols, -1 otherwise; one
// thread per entry of rows [traj[i][0 .. nsteps-1], live[i]] (live alone
// without a trajectory).
__global__ void q3_counts_kernel(Q3Args a, int nsteps) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t row = a.traj ? (size_t)nsteps + 1 : 1;
    if (k >= (size_t)a.n_inst * row) return;
    const int inst = (int)(k / row);
    const size_t j = k - (size_t)inst * row;
    const int v = a.ev_valid[inst / a.R] ? 0 : -1;
    if (j == row - 1) {
        if (a.live) a.live[inst] = v;
    } else {
        a.traj[(size_t)inst * nsteps + j] = v;
    }
}

// Per-site working data from the cells: reaction term, mask of EMPTY slots,
// no key on any slot and no targeted slot; with count set, the live cells into
// live[].
__global__ void __launch_bounds__(Q3_NT) q3_prepare_kernel(Q3Args a, int count) {
    int inst, site;
    if (!q3_place(a, inst, site)) return;
    if (!a.ev_valid[inst / a.R]) return;
    __shared__ float s_react[4];
    __shared__ int s_part[Q3_NT / 64];
    set_react_table(a.prm, s_react);
    __syncthreads();
    const int L2 = a.L * a.L, C = a.C;
    int cnt = 0;
    if (site < L2) {
        const uint16_t* cw = a.cells + (size_t)inst * C * L2;
        unsigned long long* ky = a.keys + (size_t)inst * C * L2;
        uint32_t em = 0;
        for (int z = 0; z < C; ++z) {
            const uint32_t st = cw[(size_t)z * L2 + site] & 3u;
            if (st == EMPTY) em |= 1u << z;
            cnt += (st == PROLIF || st == QUIESC);
            ky[(size_t)z * L2 + site] = NONE_KEY64;
        }
        const size_t at = (size_t)inst * L2 + site, plane = (size_t)a.n_inst * L2;
        a.emask[at] = em;
        a.tmask[at] = 0;
        a.tmask[plane + at] = 0;
        a.react[at] = site_react(s_react, cw, C, L2, site);
    }
    if (count) block_count(cnt, a.live ? a.live + inst : nullptr, s_part);
}

// Index of protocol p's fraction at half-hour tau in its event table, or -1
// (bisection over the increasing times).
__device__ __forceinline__ int find_fraction(const Q3Args& a, int p, int tau) {
    const int32_t* st = a.ev_step + (size_t)p * a.K;
    const int cnt = a.ev_count[p];
    int lo = 0, hi = cnt;
    while (lo < hi) {
        const int md = (lo + hi) >> 1;
        if (st[md] < tau) lo = md + 1; else hi = md;
    }
    return (lo < cnt && st[lo] == tau) ? lo : -1;
}

// Survival thresholds of fraction j of protocol p by class (and oxygen bin
// with the oxygen effect) into s_thr; threads 0 .. 63 of the block.
__device__ __forceinline__ void fraction_thresholds(const Q3Args& a, int p, int j, uint32_t (*s_thr)[GGA_OER_BINS]) {
    const gga_params& P = a.prm;
    const EventFraction ef = a.ev_frac[(size_t)p * a.K + j];
    if (P.oer_max > 1.0) {
        if (threadIdx.x < 4 * GGA_OER_BINS) {
            const int c = threadIdx.x / GGA_OER_BINS, b = threadIdx.x % GGA_OER_BINS;
            const double f = oxygen_modification(P, b);
            s_thr[c][b] = lq_threshold(f * (double)ef.dose, P.m[c], P.alpha, P.beta, f * ef.prior);
        }
    } else if (threadIdx.x < 4) {
        s_thr[threadIdx.x][0] = lq_threshold((double)ef.dose, P.m[threadIdx.x], P.alpha, P.beta, ef.prior);
    }
}

// A fraction at half-hour 2n + mid of the protocol, if there is one: every live
// cell survives iff its w1 < T[class] (with the oxygen effect T[class][bin of
// the site's O in F]); a killed cell becomes DEAD, or is marked with mitotic
// death.  The reaction term is then rebuilt from the surviving cells.
__global__ void __launch_bounds__(Q3_NT) q3_fraction_kernel(Q3Args a, const float* F, int n, int mid) {
    int inst, site;
    if (!q3_place(a, inst, site)) return;
    const int p = inst / a.R, r = inst - p * a.R;
    if (!a.ev_valid[p]) return;
    __shared__ int s_j;
    __shared__ uint32_t s_thr[4][GGA_OER_BINS];
    __shared__ float s_react[4];
    const gga_params& P = a.prm;
    if (threadIdx.x == 0) s_j = find_fraction(a, p, 2 * n + mid);
    __syncthreads();
    const int j = s_j;
    if (j < 0) return;                            // block-uniform
    const bool oer = P.oer_max > 1.0;
    fraction_thresholds(a, p, j, s_thr);
    set_react_table(P, s_react);
    __syncthreads();
    const int L2 = a.L * a.L, C = a.C;
    if (site >= L2) return;
    const int bin = oer ? oxygen_bin(F[(size_t)inst * 3 * L2 + site], P) : 0;
    uint16_t* cw = a.cells + (size_t)inst * C * L2;
    const uint32_t step_word = (uint32_t)n | ((uint32_t)mid << 31);
    for (int z = 0; z < C; ++z) {
        const uint32_t w = cw[(size_t)z * L2 + site];
        const uint32_t st = w & 3u;
        if (st != PROLIF && st != QUIESC) continue;
        const Block4 b = philox10((uint32_t)(z * L2 + site), step_word, (uint32_t)r, (uint32_t)p, a.seed_lo, a.seed_hi);
        if (b.w1 >= s_thr[sens_class(w, P)][bin])
            cw[(size_t)z * L2 + site] = P.mitotic_death ? (uint16_t)(w | DOOM_BIT) : (uint16_t)DEAD;
    }
    a.react[(size_t)inst * L2 + site] = site_react(s_react, cw, C, L2, site);
}

// The FTCS sub-steps of the three fields in field units (boundary 0),
// c' = lam ((N + S) + (W + E)) + (c (1 - 4 lam) + r), O and G clamped at the
// units' zero, fused up to Q3_MAX_HALO per launch: a workgroup loads a
// T x T tile of owned sites with a halo of h sites (the launch's sub-step
// count) of the three fields and the reaction term into LDS, runs h sub-steps
// there (sub-step k updates the region at least k + 1 sites inside the loaded
// square, which its inputs fully determine), and stores the owned sites.
// Sites outside the lattice hold 0, the boundary value in field units, and
// every site's arithmetic is the 2D kernels' (so C = 1 reproduces them).
constexpr int Q3_MAX_HALO = 16;
constexpr int Q3_BIG_TILE_MIN_L = 128;
__host__ __device__ inline unsigned q3_tiles_per_inst(int L, int tile) {
    const unsigned t = ((unsigned)L + tile - 1) / tile;
    return t * t;
}
// rows a thread walks in the widest sub-step (w = EMAX - 2 columns, NT / w threads per column)
constexpr int q3_run(int EMAX, int NT) { return (EMAX - 2 + NT / (EMAX - 2) - 1) / (NT / (EMAX - 2)); }

// Tiles of Q3_TILE x Q3_TILE owned sites, EMAX the loaded side for the
// launch's largest halo, NT threads.
template <int Q3_TILE, int Q3_TILE_NT, int EMAX>
__global__ void __launch_bounds__(Q3_TILE_NT) q3_diffuse_tile_kernel(Q3Args a, const float* src, float* dst, int h) {
    __shared__ float s_f[3][EMAX * EMAX];
    __shared__ float s_r[EMAX * EMAX];
    const int L = a.L, L2 = L * L;
    const int tpr = (L + Q3_TILE - 1) / Q3_TILE;
    const unsigned tiles = q3_tiles_per_inst(L, Q3_TILE);
    const unsigned total = (unsigned)a.n_inst * tiles, per = (total + 7u) / 8u;
    const unsigned lb = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);     // XCD-grouped, as q3_place
    if (lb >= total) return;
    const int inst = (int)(lb / tiles), tile = (int)(lb - (unsigned)inst * tiles);
    if (!a.ev_valid[inst / a.R]) return;
    const int y0 = (tile / tpr) * Q3_TILE - h, x0 = (tile % tpr) * Q3_TILE - h;   // lattice site of LDS (0, 0)
    const int E = Q3_TILE + 2 * h;
    const float* S = src + (size_t)inst * 3 * L2;
    const float* Rg = a.react + (size_t)inst * L2;
    // all of a thread's global loads are issued before its first LDS write
    constexpr int LOADS = (EMAX * EMAX + Q3_TILE_NT - 1) / Q3_TILE_NT;
    float ld[LOADS][4];
#pragma unroll
    for (int j = 0; j < LOADS; ++j) {
        const int i = (int)threadIdx.x + j * Q3_TILE_NT;
        const int ly = i / E, lx = i - ly * E;
        const int gy = y0 + ly, gx = x0 + lx;
        const bool in = i < E * E && gy >= 0 && gy < L && gx >= 0 && gx < L;
        const size_t g = in ? (size_t)gy * L + gx : 0;
#pragma unroll
        for (int f = 0; f < 3; ++f) ld[j][f] = in ? S[(size_t)f * L2 + g] : 0.0f;
        ld[j][3] = in ? Rg[g] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < LOADS; ++j) {
        const int i = (int)threadIdx.x + j * Q3_TILE_NT;
        if (i < E * E) {
            const int ly = i / E, o = ly * EMAX + (i - ly * E);
#pragma unroll
            for (int f = 0; f < 3; ++f) s_f[f][o] = ld[j][f];
            s_r[o] = ld[j][3];
        }
    }
    float lam[3], cen[3], lo[2];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        lam[f] = a.prm.lambda[f];
        cen[f] = 1.0f - 4.0f * a.prm.lambda[f];
    }
    lo[0] = to_field_units(a.prm, 0, 0.0);
    lo[1] = to_field_units(a.prm, 1, 0.0);
    __syncthreads();
    // Sub-step k computes the w x w square starting at (k + 1, k + 1).  Each
    // thread takes one column of it and a run of at most RUN consecutive rows,
    // walking down with the rows above and at the site in registers (three LDS
    // reads per site and field: below, west, east); the new values wait in
    // registers until every thread has read the old ones, so one LDS copy of
    // the fields serves (more workgroups per CU).
    constexpr int RUN = q3_run(EMAX, Q3_TILE_NT);    // ceil(w / (Q3_TILE_NT / w)) for w <= EMAX - 2
    for (int k = 0; k < h; ++k) {
        const int r0 = k + 1, w = E - 2 * (k + 1);
        const int nseg = Q3_TILE_NT / w, rows = (w + nseg - 1) / nseg;
        const int col = (int)threadIdx.x % w, seg = (int)threadIdx.x / w;
        const int ly0 = r0 + seg * rows, ly1 = min(ly0 + rows, r0 + w);
        const bool act = seg < nseg && ly0 < ly1;
        const int lx = r0 + col, gx = x0 + lx;
        float nv[RUN][3];
        if (act) {
            const bool col_in = gx >= 0 && gx < L;
            int o = ly0 * EMAX + lx;
            float up[3] = {s_f[0][o - EMAX], s_f[1][o - EMAX], s_f[2][o - EMAX]};
            float mid[3] = {s_f[0][o], s_f[1][o], s_f[2][o]};
#pragma unroll
            for (int q = 0; q < RUN; ++q, o += EMAX) {
                if (ly0 + q < ly1) {
                    const int gy = y0 + ly0 + q;
                    const bool in = col_in && gy >= 0 && gy < L;
                    const float R = s_r[o];
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        const float below = s_f[f][o + EMAX];
                        const float sum = (up[f] + below) + (s_f[f][o - 1] + s_f[f][o + 1]);
                        float v = fmaf(lam[f], sum, fmaf(mid[f], cen[f], R));
                        if (f < 2) v = fmaxf(v, lo[f]);
                        nv[q][f] = in ? v : 0.0f;
                        up[f] = mid[f];
                        mid[f] = below;
                    }
                }
            }
        }
        __syncthreads();
        if (act) {
#pragma unroll
            for (int q = 0; q < RUN; ++q)
                if (ly0 + q < ly1)
#pragma unroll
                    for (int f = 0; f < 3; ++f) s_f[f][(ly0 + q) * EMAX + lx] = nv[q][f];
        }
        __syncthreads();
    }
    float* D = dst + (size_t)inst * 3 * L2;
    for (int i = threadIdx.x; i < Q3_TILE * Q3_TILE; i += Q3_TILE_NT) {
        const int qy = i / Q3_TILE;
        const int ly = h + qy, lx = h + (i - qy * Q3_TILE);
        const int gy = y0 + ly, gx = x0 + lx;
        if (gy >= L || gx >= L) continue;
        const size_t g = (size_t)gy * L + gx;
#pragma unroll
        for (int f = 0; f < 3; ++f) D[(size_t)f * L2 + g] = s_f[f][ly * EMAX + lx];
    }
}

// Cell update from the snapshot (cells, after the fractions; its EMPTY slots
// in emask) and the fields after the sub-steps, in place: every slot's word
// before births.  A ready proposer takes the minimum of its key into the
// target slot's key, marks the target in this step's targeted mask and keeps
// its target and code (prop, and its bit in pmask).  First the keys of the
// slots targeted in the previous step are cleared (those slots now hold cells,
// so no proposal of this step reaches them) and that mask is zeroed for the
// next step.
__global__ void __launch_bounds__(Q3_NT) q3_update_kernel(Q3Args a, const float* F, int n) {
    int inst, site;
    if (!q3_place(a, inst, site)) return;
    const int p = inst / a.R, r = inst - p * a.R;
    if (!a.ev_valid[p]) return;
    __shared__ CellConst s_k;
    const gga_params& P = a.prm;
    if (threadIdx.x == 0) {
        s_k.thOq = to_field_units(P, 0, P.theta_O_quiesce);
        s_k.thGq = to_field_units(P, 1, P.theta_G_quiesce);
        s_k.thOd = to_field_units(P, 0, P.theta_O_death);
        s_k.thGd = to_field_units(P, 1, P.theta_G_death);
        s_k.thHd = to_field_units(P, 2, P.theta_H_death);
        s_k.T_div = (P.P_div >= 1.0) ? 0xFFFFFFFFu : (uint32_t)floor(P.P_div * 4294967296.0);
    }
    __syncthreads();
    const int L = a.L, L2 = L * L, C = a.C;
    if (site >= L2) return;
    const size_t plane = (size_t)a.n_inst * L2;
    uint32_t* t_now = a.tmask + (n & 1) * plane + (size_t)inst * L2;
    uint32_t* t_prev = a.tmask + ((n + 1) & 1) * plane + (size_t)inst * L2;
    unsigned long long* ky = a.keys + (size_t)inst * C * L2;
    for (uint32_t tp = t_prev[site]; tp; tp &= tp - 1) ky[(size_t)__builtin_ctz(tp) * L2 + site] = NONE_KEY64;
    t_prev[site] = 0;

    const float* Fi = F + (size_t)inst * 3 * L2;
    const float O = Fi[site], Gl = Fi[L2 + site], H = Fi[2 * L2 + site];
    // H's units have a negative scale, so H > theta reads H^ < theta^
    const bool nec = (Gl < s_k.thGd) || (O < s_k.thOd) || (H < s_k.thHd);
    const bool starv = (O < s_k.thOq) || (Gl < s_k.thGq);
    const uint32_t* em = a.emask + (size_t)inst * L2;
    const int y = site / L, x = site - y * L;
    // EMPTY-slot masks by group: own site, N, E, S, W (none outside the lattice)
    const uint32_t gm[5] = {em[site], y > 0 ? em[site - L] : 0u, x < L - 1 ? em[site + 1] : 0u,
                            y < L - 1 ? em[site + L] : 0u, x > 0 ? em[site - 1] : 0u};
    const uint32_t m = (uint32_t)(__builtin_popcount(gm[0]) + __builtin_popcount(gm[1]) + __builtin_popcount(gm[2]) +
                                  __builtin_popcount(gm[3]) + __builtin_popcount(gm[4]));
    uint16_t* cw = a.cells + (size_t)inst * C * L2;
    uint32_t* pr = a.prop + (size_t)inst * C * L2;
    const uint32_t T_div = s_k.T_div;
    // All of the site's words are loaded first (independent loads, issued
    // together; the loop is unrolled to the slot limit so they stay in
    // registers), then the transitions; the Philox blocks are drawn only for the
    // candidates, taken from bit masks.
    uint32_t wv[Q3_MAX_SLOTS];
#pragma unroll
    for (int z = 0; z < Q3_MAX_SLOTS; ++z) wv[z] = z < C ? (uint32_t)cw[(size_t)z * L2 + site] : 0u;
    uint32_t cand = 0, marked = 0;
    unsigned long long states = 0;          // 2 bits per slot, for the resolution
#pragma unroll
    for (int z = 0; z < Q3_MAX_SLOTS; ++z) {
        const uint32_t w = wv[z];
        const uint32_t st = w & 3u, age = (w >> 2) & 255u, doom = w & DOOM_BIT;
        if (z >= C || st == EMPTY) continue;
        const uint32_t older = age < 255u ? age + 1u : 255u;
        uint32_t out;
        if (st == DEAD) {
            out = (int)older >= P.T_lys ? 0u : ((uint32_t)DEAD | (older << 2));
        } else if (nec) {
            out = DEAD;
        } else if (starv) {
            out = (uint32_t)QUIESC | (w & ~3u);
        } else {
            out = (uint32_t)PROLIF | (older << 2) | doom;
            if ((int)age >= P.T_min) {
                if (P.mitotic_death && doom) marked |= 1u << z;     // a marked cell dies when ready
                else if (m >= 1u) cand |= 1u << z;
            }
        }
        if (out != w) cw[(size_t)z * L2 + site] = (uint16_t)out;
        states |= (unsigned long long)(out & 3u) << (2 * z);
    }
    uint32_t proposed = 0;
    for (uint32_t cm = cand | marked; cm; cm &= cm - 1) {
        const int z = __builtin_ctz(cm);
        const size_t at = (size_t)z * L2 + site;
        const Block4 b = philox10((uint32_t)at, (uint32_t)n, (uint32_t)r, (uint32_t)p, a.seed_lo, a.seed_hi);
        if (b.w3 >= T_div) continue;
        if ((marked >> z) & 1u) {
            cw[at] = (uint16_t)DEAD;
            states |= (unsigned long long)DEAD << (2 * z);
            continue;
        }
        uint32_t k = (uint32_t)(((uint64_t)b.w0 * m) >> 32);
        int g = 0;
        while (g < 4 && k >= (uint32_t)__builtin_popcount(gm[g])) k -= (uint32_t)__builtin_popcount(gm[g++]);
        const int t = site + (g == 1 ? -L : g == 2 ? 1 : g == 3 ? L : g == 4 ? -1 : 0);
        uint32_t free_slots = gm[g];
        for (; k; --k) free_slots &= free_slots - 1;      // the k-th EMPTY slot of site t
        const int tz = __builtin_ctz(free_slots);
        const uint32_t code = (g == 0 ? 4u : g == 1 ? 2u : g == 2 ? 3u : g == 3 ? 0u : 1u);
        const uint32_t low = (code << 5) | (uint32_t)z;
        const uint32_t target = (uint32_t)(tz * L2 + t);
        atomicMin(ky + target, ((unsigned long long)(b.w2 >> 3) << 8) | low);
        atomicOr(t_now + t, 1u << tz);
        pr[at] = (target << 8) | low;
        proposed |= 1u << z;
    }
    a.pmask[(size_t)inst * L2 + site] = proposed;
    a.svec[(size_t)inst * L2 + site] = states;
}

// Births and winners: a targeted slot takes the daughter (PROLIF, age 0), a
// proposer whose code holds its target's key is the parent (age 0).  Then,
// from the update's slot states with the births applied (no word is read
// again), the live count added to traj_col[inst * traj_stride] and live[inst]
// (either may be null); with `next` set, the start-of-hour fraction of step
// n + 1 if the protocol has one (as q3_fraction_kernel applies it, from the
// fields F that step starts from); and the next step's reaction term and
// EMPTY mask.
__global__ void __launch_bounds__(Q3_NT) q3_resolve_kernel(Q3Args a, int n, int32_t* traj_col, int traj_stride,
                                                          int32_t* live, const float* F, int next) {
    int inst, site;
    if (!q3_place(a, inst, site)) return;
    const int p = inst / a.R, r = inst - p * a.R;
    if (!a.ev_valid[p]) return;
    __shared__ float s_react[4];
    __shared__ int s_part[Q3_NT / 64];
    __shared__ int s_j;
    __shared__ uint32_t s_thr[4][GGA_OER_BINS];
    set_react_table(a.prm, s_react);
    if (threadIdx.x == 0) s_j = next ? find_fraction(a, p, 2 * (n + 1)) : -1;
    __syncthreads();
    const int j = s_j;                            // step n + 1's fraction at the start of its hour
    if (j >= 0) {
        fraction_thresholds(a, p, j, s_thr);
        __syncthreads();                          // block-uniform
    }
    const int L2 = a.L * a.L, C = a.C;
    int cnt = 0;
    if (site < L2) {
        const size_t plane = (size_t)a.n_inst * L2, at0 = (size_t)inst * L2 + site;
        uint16_t* cw = a.cells + (size_t)inst * C * L2;
        const uint32_t* pr = a.prop + (size_t)inst * C * L2;
        const unsigned long long* ky = a.keys + (size_t)inst * C * L2;
        unsigned long long states = a.svec[at0];
        for (uint32_t tm = a.tmask[(n & 1) * plane + at0]; tm; tm &= tm - 1) {
            cw[(size_t)__builtin_ctz(tm) * L2 + site] = PROLIF;
            states |= (unsigned long long)PROLIF << (2 * __builtin_ctz(tm));    // the slot was EMPTY
        }
        for (uint32_t pm = a.pmask[at0]; pm; pm &= pm - 1) {
            const size_t at = (size_t)__builtin_ctz(pm) * L2 + site;
            const uint32_t pp = pr[at];
            if ((uint32_t)(ky[pp >> 8] & 0xFFu) == (pp & 0xFFu)) cw[at] = (uint16_t)((cw[at] & DOOM_BIT) | PROLIF);
        }
        for (int z = 0; z < C; ++z) {              // winners keep their state: the vector is final
            const uint32_t st = (uint32_t)(states >> (2 * z)) & 3u;
            cnt += (st == PROLIF || st == QUIESC);
        }
        if (j >= 0) {
            // step n + 1's start-of-hour fraction on the counted states: every
            // live cell survives iff its w1 < T[class] (and oxygen bin of the
            // site's O in F, the fields step n + 1 starts from)
            const bool oer = a.prm.oer_max > 1.0;
            const int bin = oer ? oxygen_bin(F[(size_t)inst * 3 * L2 + site], a.prm) : 0;
            for (int z = 0; z < C; ++z) {
                const uint32_t st = (uint32_t)(states >> (2 * z)) & 3u;
                if (st != PROLIF && st != QUIESC) continue;
                const size_t at = (size_t)z * L2 + site;
                const uint32_t w = cw[at];
                const Block4 b = philox10((uint32_t)at, (uint32_t)(n + 1), (uint32_t)r, (uint32_t)p, a.seed_lo,
                                          a.seed_hi);
                if (b.w1 >= s_thr[sens_class(w, a.prm)][bin]) {
                    if (a.prm.mitotic_death) {
                        cw[at] = (uint16_t)(w | DOOM_BIT);
                    } else {
                        cw[at] = (uint16_t)DEAD;
                        states |= (unsigned long long)DEAD << (2 * z);
                    }
                }
            }
        }
        uint32_t em = 0;
        float acc = 0.0f;
        for (int z = 0; z < C; ++z) {
            const uint32_t st = (uint32_t)(states >> (2 * z)) & 3u;
            if (st == EMPTY) em |= 1u << z;
            acc = z == 0 ? s_react[st] : acc + s_react[st];
        }
        a.emask[at0] = em;
        a.react[at0] = C > 1 ? acc * (1.0f / (float)C) : acc;
    }
    block_count(cnt, traj_col ? traj_col + (size_t)inst * traj_stride : nullptr, s_part);
    // the same count once more for the final live count (s_part is unchanged
    // since block_count's barrier and is read by thread 0 only)
    if (threadIdx.x == 0 && live) {
        int t = 0;
        for (int w = 0; w < Q3_NT / 64; ++w) t += s_part[w];
        atomicAdd(live + inst, t);
    }
}

// fields of valid instances: dst <- src (the last sub-step's buffer)
__global__ void __launch_bounds__(Q3_NT) q3_copy_fields_kernel(Q3Args a, const float* src, float* dst) {
    int inst, site;
    if (!q3_place(a, inst, site)) return;
    if (!a.ev_valid[inst / a.R]) return;
    const int L2 = a.L * a.L;
    if (site >= L2) return;
    for (int f = 0; f < 3; ++f) dst[((size_t)inst * 3 + f) * L2 + site] = src[((size_t)inst * 3 + f) * L2 + site];
}

dim3 q3_grid(const Q3Args& a) { return dim3(q3_per_xcd(a) * 8u); }

}  // namespace

hipError_t q3_init(const Q3Args& a, hipStream_t stream) {
    if (a.n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(q3_init_kernel, q3_grid(a), dim3(Q3_NT), 0, stream, a);
    return hipGetLastError();
}

hipError_t q3_run(const Q3Args& a, int n0, int nsteps, hipStream_t stream) {
    if (a.n_inst <= 0) return hipSuccess;
    const dim3 grid = q3_grid(a), block(Q3_NT);
    const size_t nc = (size_t)a.n_inst * (a.traj ? (size_t)nsteps + 1 : 1);
    hipLaunchKernelGGL(q3_counts_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, stream, a, nsteps);
    hipLaunchKernelGGL(q3_prepare_kernel, grid, block, 0, stream, a, nsteps == 0 ? 1 : 0);
    float* cur = a.fields;
    float* oth = a.fields2;
    // 64 x 64 owned sites per workgroup of 1,024 threads (one per CU, 113 KB of
    // LDS at up to 10 sub-steps) once the lattice holds four such tiles, else
    // 32 x 32 per 512 threads (three per CU)
    const bool big = a.L >= Q3_BIG_TILE_MIN_L;
    const dim3 tile_grid(((unsigned)a.n_inst * q3_tiles_per_inst(a.L, big ? 64 : 32) + 7u) / 8u * 8u);
    auto diffuse = [&](int k) {
        while (k > 0) {              // sub-steps fused in LDS tiles, Q3_MAX_HALO at most per launch
            const int h = k < Q3_MAX_HALO ? k : Q3_MAX_HALO;
            if (big && h <= 10)
                hipLaunchKernelGGL((q3_diffuse_tile_kernel<64, 1024, 64 + 20>), tile_grid, dim3(1024), 0, stream, a,
                                   (const float*)cur, oth, h);
            else if (big)
                hipLaunchKernelGGL((q3_diffuse_tile_kernel<64, 1024, 64 + 2 * Q3_MAX_HALO>), tile_grid, dim3(1024), 0,
                                   stream, a, (const float*)cur, oth, h);
            else if (h <= 10)
                hipLaunchKernelGGL((q3_diffuse_tile_kernel<32, 512, 32 + 20>), tile_grid, dim3(512), 0, stream, a,
                                   (const float*)cur, oth, h);
            else
                hipLaunchKernelGGL((q3_diffuse_tile_kernel<32, 512, 32 + 2 * Q3_MAX_HALO>), tile_grid, dim3(512), 0,
                                   stream, a, (const float*)cur, oth, h);
            std::swap(cur, oth);
            k -= h;
        }
    };
    const int first = a.half ? a.substeps / 2 : a.substeps;
    // the start-of-hour fraction of step n0 here; those of later steps are
    // applied by the previous step's resolution
    if (nsteps > 0) hipLaunchKernelGGL(q3_fraction_kernel, grid, block, 0, stream, a, (const float*)cur, n0, 0);
    for (int i = 0; i < nsteps; ++i) {
        const int n = n0 + i;
        diffuse(first);
        if (a.half) {
            hipLaunchKernelGGL(q3_fraction_kernel, grid, block, 0, stream, a, (const float*)cur, n, 1);
            diffuse(a.substeps - first);
        }
        hipLaunchKernelGGL(q3_update_kernel, grid, block, 0, stream, a, (const float*)cur, n);
        hipLaunchKernelGGL(q3_resolve_kernel, grid, block, 0, stream, a, n, a.traj ? a.traj + i : nullptr, nsteps,
                           i == nsteps - 1 ? a.live : nullptr, (const float*)cur, i + 1 < nsteps ? 1 : 0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (cur != a.fields) hipLaunchKernelGGL(q3_copy_fields_kernel, grid, block, 0, stream, a, (const float*)cur, a.fields);
    return hipGetLastError();
}

}  // namespace gga
