// Slab variants of the simulation kernel (see sim_kernel.h) for lattices whose
// state does not fit one compute unit, and the two kernels that prepare them:
// the per-protocol event table and the initial state in device memory.
#include "sim_kernel.h"

namespace gga {
namespace {

// Per protocol: validity (the resident kernel's rules), and the time in
// half-hours (2 t for delays in hours; horizons stay below 2^30), dose and
// unrepaired dose of the earlier fractions of every positive-dose fraction,
// in order (the slab kernels derive the survival thresholds from them).
__global__ void event_table_kernel(SimArgs a, int P, int32_t* valid_out, int32_t* count_out, int32_t* step_out,
                                   EventFraction* frac_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int k = a.nfrac[p];
    int valid = (k >= 0 && k <= a.K);
    int nev = 0;
    double total = 0.0;
    long long t = 0;
    for (int j = 0; valid && j < k; ++j) {
        const float d = a.dose[(size_t)p * a.K + j];
        const int g = a.gap[(size_t)p * a.K + j];
        if (!(d >= 0.0f) || !isfinite(d)) { valid = 0; break; }
        if (g < (j == 0 ? 0 : 1)) { valid = 0; break; }
        total += (double)d;
        t += g;
        if (d > 0.0f) {
            const long long tau = a.half ? t : 2 * t;
            const double D = prior_damage(a.dose + (size_t)p * a.K, a.gap + (size_t)p * a.K, j, t,
                                          a.prm.repair_half_time, a.half ? 0.5 : 1.0);
            step_out[(size_t)p * a.K + nev] = tau > 0x7FFFFFFFll ? 0x7FFFFFFF : (int)tau;
            frac_out[(size_t)p * a.K + nev] = EventFraction{d, 0, D};
            ++nev;
        }
    }
    if (valid && total > a.dose_cap + 1e-6) valid = 0;
    valid_out[p] = valid;
    count_out[p] = valid ? nev : 0;
}

__global__ void slab_live_kernel(SimArgs a, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int inst = a.inst_list ? a.inst_list[k] : k;
    a.live[inst] = a.ev_valid[inst / a.R] ? 0 : -1;
}

// Initial state (seed disc of radius seed_radius at L/2 with Philox ages,
// uniform fields) of state rows 0 .. n-1; one thread per site.
__global__ void slab_init_kernel(SimArgs a, int L, int n, float* fields, uint16_t* cells) {
    const size_t plane = (size_t)L * L;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= plane * n) return;
    const int k = (int)(i / plane);
    const int site = (int)(i - (size_t)k * plane);
    const int inst = a.inst_list ? a.inst_list[k] : k;
    const int p = inst / a.R, r = inst - p * a.R;
    uint32_t k0 = a.seed_lo, k1 = a.seed_hi;
    if (a.generation) {
        const uint64_t key = a.seed + (uint64_t)(uint32_t)*a.generation * 0x9E3779B97F4A7C15ull;
        k0 = (uint32_t)key;
        k1 = (uint32_t)(key >> 32);
    }
    for (int f = 0; f < 3; ++f) fields[(size_t)k * 3 * plane + f * plane + site] = to_field_units(a.prm, f, a.prm.init[f]);
    const int y = site / L, x = site - y * L, ctr = L / 2;
    uint16_t w = 0;
    if ((x - ctr) * (x - ctr) + (y - ctr) * (y - ctr) <= a.prm.seed_radius * a.prm.seed_radius) {
        const Block4 b = philox10((uint32_t)site, INIT_STEP, (uint32_t)r, (uint32_t)p, k0, k1);
        const uint32_t age = (uint32_t)(((uint64_t)b.w0 * (uint32_t)a.prm.A0) >> 32);
        w = (uint16_t)(PROLIF | (age << 2));
        if ((a.horizon ? a.horizon[p] : a.count_at) == 0 && a.ev_valid[p] && a.live) atomicAdd(&a.live[inst], 1);
    }
    cells[(size_t)k * plane + site] = w;
}

template <int CPL, int RPT, int NW, int LW = 64 * CPL>
hipError_t launch_slab(const SimArgs& a, int n_blocks, hipStream_t stream) {
    using G = Geo<CPL, RPT, NW, LW>;
    static_assert(G::SLAB, "resident variants are built in sim.hip");
    if (a.prm.oer_max > 1.0 || a.prm.mitotic_death)   // the extended radiobiology instantiation
        hipLaunchKernelGGL((sim_kernel<CPL, RPT, NW, LW, true>), dim3(n_blocks), dim3(G::NT), 0, stream, a);
    else
        hipLaunchKernelGGL((sim_kernel<CPL, RPT, NW, LW, false>), dim3(n_blocks), dim3(G::NT), 0, stream, a);
    return hipGetLastError();
}

// The team form: every workgroup of the grid resident at once (a cooperative
// launch), so each team's slabs can wait for one another.  With n_blocks = 0,
// returns in *capacity the most workgroups of this kernel the device holds at
// once instead of launching.
template <int CPL, int RPT, int NW, int LW = 64 * CPL>
hipError_t launch_team(const SimArgs& a, int n_blocks, int* capacity, hipStream_t stream) {
    using G = Geo<CPL, RPT, NW, LW>;
    static_assert(G::SLAB, "teams are made of slabs");
    const bool ext = a.prm.oer_max > 1.0 || a.prm.mitotic_death;
    const void* fn = ext ? reinterpret_cast<const void*>(&sim_kernel<CPL, RPT, NW, LW, true, true>)
                         : reinterpret_cast<const void*>(&sim_kernel<CPL, RPT, NW, LW, false, true>);
    if (n_blocks == 0) {
        int dev = 0, per_cu = 0, cus = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, G::NT, 0);
        *capacity = e == hipSuccess ? per_cu * cus : 0;
        return e;
    }
    SimArgs arg = a;
    void* params[] = {&arg};
    return hipLaunchCooperativeKernel(fn, dim3(n_blocks), dim3(G::NT), params, 0, stream);
}

}  // namespace

hipError_t launch_slab_variant(int v, const SimArgs& a, int n_blocks, hipStream_t stream) {
    if (n_blocks <= 0) return hipSuccess;
    switch (v) {
        case 1: return launch_slab<1, 2, 16>(a, n_blocks, stream);
        case 4: return launch_slab<2, 4, 16>(a, n_blocks, stream);
        case 5: return launch_slab<4, 4, 16>(a, n_blocks, stream);
        case 6: return launch_slab<4, 8, 8>(a, n_blocks, stream);
        case 11: return launch_slab<4, 4, 16, 160>(a, n_blocks, stream);
        case 12: return launch_slab<4, 8, 8, 160>(a, n_blocks, stream);
        case 13: return launch_slab<4, 4, 16, 192>(a, n_blocks, stream);
        case 14: return launch_slab<4, 8, 8, 192>(a, n_blocks, stream);
        case 15: return launch_slab<4, 4, 16, 224>(a, n_blocks, stream);
        case 16: return launch_slab<4, 8, 8, 224>(a, n_blocks, stream);
        case 17: return launch_slab<2, 4, 16, 96>(a, n_blocks, stream);
        case 18: return launch_slab<3, 4, 16, 160>(a, n_blocks, stream);
        case 19: return launch_slab<3, 8, 8, 160>(a, n_blocks, stream);
        case 20: return launch_slab<3, 4, 16, 192>(a, n_blocks, stream);
        case 21: return launch_slab<3, 8, 8, 192>(a, n_blocks, stream);
        case 22: return launch_slab<3, 9, 8, 160>(a, n_blocks, stream);
        case 23: return launch_slab<3, 9, 8, 192>(a, n_blocks, stream);
        case 24: return launch_slab<3, 10, 8, 192>(a, n_blocks, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_team_variant(int v, const SimArgs& a, int n_blocks, int* capacity, hipStream_t stream) {
    switch (v) {
        case 1: return launch_team<1, 2, 16>(a, n_blocks, capacity, stream);
        case 4: return launch_team<2, 4, 16>(a, n_blocks, capacity, stream);
        case 5: return launch_team<4, 4, 16>(a, n_blocks, capacity, stream);
        case 6: return launch_team<4, 8, 8>(a, n_blocks, capacity, stream);
        case 11: return launch_team<4, 4, 16, 160>(a, n_blocks, capacity, stream);
        case 12: return launch_team<4, 8, 8, 160>(a, n_blocks, capacity, stream);
        case 13: return launch_team<4, 4, 16, 192>(a, n_blocks, capacity, stream);
        case 14: return launch_team<4, 8, 8, 192>(a, n_blocks, capacity, stream);
        case 15: return launch_team<4, 4, 16, 224>(a, n_blocks, capacity, stream);
        case 16: return launch_team<4, 8, 8, 224>(a, n_blocks, capacity, stream);
        case 17: return launch_team<2, 4, 16, 96>(a, n_blocks, capacity, stream);
        case 18: return launch_team<3, 4, 16, 160>(a, n_blocks, capacity, stream);
        case 19: return launch_team<3, 8, 8, 160>(a, n_blocks, capacity, stream);
        case 20: return launch_team<3, 4, 16, 192>(a, n_blocks, capacity, stream);
        case 21: return launch_team<3, 8, 8, 192>(a, n_blocks, capacity, stream);
        case 22: return launch_team<3, 9, 8, 160>(a, n_blocks, capacity, stream);
        case 23: return launch_team<3, 9, 8, 192>(a, n_blocks, capacity, stream);
        case 24: return launch_team<3, 10, 8, 192>(a, n_blocks, capacity, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_event_table(const SimArgs& a, int P, int32_t* valid, int32_t* count, int32_t* step,
                              EventFraction* frac, hipStream_t stream) {
    if (P <= 0) return hipSuccess;
    hipLaunchKernelGGL(event_table_kernel, dim3((P + 127) / 128), dim3(128), 0, stream, a, P, valid, count, step, frac);
    return hipGetLastError();
}

hipError_t launch_slab_live(const SimArgs& a, int n, hipStream_t stream) {
    if (n <= 0 || !a.live) return hipSuccess;
    hipLaunchKernelGGL(slab_live_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, a, n);
    return hipGetLastError();
}

hipError_t launch_slab_init(const SimArgs& a, int L, int n, float* fields, uint16_t* cells, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const hipError_t e = launch_slab_live(a, n, stream);
    if (e != hipSuccess) return e;
    const size_t sites = (size_t)L * L * n;
    hipLaunchKernelGGL(slab_init_kernel, dim3((unsigned)((sites + 255) / 256)), dim3(256), 0, stream, a, L, n, fields,
                       cells);
    return hipGetLastError();
}

}  // namespace gga
