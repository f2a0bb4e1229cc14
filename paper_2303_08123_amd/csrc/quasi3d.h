// Library-internal interface of the quasi-3D variant (gga_q3_*).
#pragma once
#include "gga_internal.h"

namespace gga {

// Quasi-3D variant (gga_q3_*): C cell slots per site, 2D fields, state in
// device memory, one launch per phase of a step over all instances.
constexpr int Q3_MAX_SLOTS = 32;
constexpr int Q3_MIN_L = 8, Q3_MAX_L = 512;
constexpr long long Q3_MAX_SLOT_SITES = 1ll << 23;   // C L^2: a slot index and an 8-bit code fit 31 bits
struct Q3Args {
    gga_params prm;
    int32_t L, C, R, K, substeps, half, n_inst;
    uint32_t seed_lo, seed_hi;
    const int32_t* ev_valid;                // event table of the protocols (launch_event_table)
    const int32_t* ev_count;
    const int32_t* ev_step;
    const EventFraction* ev_frac;
    float* fields;                          // [inst][3][L][L] state, field units
    float* fields2;                         // second field buffer, same shape
    uint16_t* cells;                        // [inst][C][L][L] state
    float* react;                           // [inst][L][L] reaction term of the site
    uint32_t* emask;                        // [inst][L][L] EMPTY slots of the site (bit z)
    uint32_t* tmask;                        // [2][inst][L][L] slots targeted by a proposal, by step parity
    uint32_t* pmask;                        // [inst][L][L] slots whose cell proposed this step
    unsigned long long* svec;               // [inst][L][L] slot states after the cell update, 2 bits each
    unsigned long long* keys;               // [inst][C][L][L] smallest proposal key of a targeted slot;
                                            // all ones on every other slot
    uint32_t* prop;                         // [inst][C][L][L] a proposer's target slot << 8 | its code
    int32_t* live;                          // [inst] or null
    int32_t* traj;                          // [inst][nsteps] or null
};
// initial state of every instance into a.fields / a.cells
hipError_t q3_init(const Q3Args& a, hipStream_t stream);
// steps n0 .. n0+nsteps-1 in place (a.fields / a.cells); invalid protocols untouched, live -1
hipError_t q3_run(const Q3Args& a, int n0, int nsteps, hipStream_t stream);

}  // namespace gga
