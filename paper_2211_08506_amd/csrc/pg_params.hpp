// pg_params.hpp -- kernel parameter blocks shared by the host runtime and the
// gfx950 kernels (passed by value as kernel arguments).
#pragma once

#include <stdint.h>

#include "../../include/particlegrid.h"

namespace pg {

// Sticky device error word: bit k of flags set <=> pg_status k was raised;
// first = smallest atom (or structure) index involved.
struct DeviceError {
    unsigned int flags;
    unsigned int pad;
    unsigned long long first;
};

// Everything a forward / backward launch needs.  Per-channel constants are
// precomputed on the host: rc = fl32(k * sigma), inv2s2 = fl32(1/(2 sigma^2)),
// invs2 = fl32(1/sigma^2).
struct GridParams {
    const float *xyz;
    const int32_t *types;
    const int32_t *offsets;
    const float *origins;    // per-structure, or nullptr
    const float *spacings;   // per-structure, or nullptr
    void *out;               // forward output, or upstream gradient (backward)
    float *grad_xyz;         // backward output
    void *ws;                // workspace
    DeviceError *err;
    int32_t n_mol;
    int32_t C, D, H, W;
    int32_t periodic;
    int32_t cut;
    int32_t a_cap;           // atoms per structure the LDS layout holds
    int32_t row_stride;      // floats per atom in the LDS factor rows
    int32_t mask_words;      // 64-bit mask words per (channel, z) plane
    int32_t nt_store;        // non-temporal output stores
    int32_t mol_index;       // plain form: the structure of this launch
    int64_t n_atoms;
    float o[3], h[3], L[3];
    float rc[PG_MAX_CHANNELS];
    float inv2s2[PG_MAX_CHANNELS];
    float invs2[PG_MAX_CHANNELS];
};

// Per-atom window table written by the prep kernel (plain form).
struct AtomWindow {
    int32_t type;            // -1: skipped atom
    int32_t n[3];
    int32_t lo[3][3], hi[3][3];
    float bh[3][3], bl[3][3];
};

// Crystal path: per-atom window records and (structure, channel, z) bins.
struct CrystalParams {
    AtomWindow *table;       // n_atoms records
    uint32_t *counts;        // n_mol * C * D bin sizes
    uint32_t *offsets;       // n_mol * C * D + 1 bin starts
    uint32_t *cursor;        // n_mol * C * D fill cursors
    int32_t *list;           // bin contents: global atom indices
    int32_t bin_cap;         // most atoms a plane kernel sorts in LDS (a power of two)
};

}  // namespace pg
