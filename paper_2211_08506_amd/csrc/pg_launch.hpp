// pg_launch.hpp -- host-side launchers of the gfx950 kernels (one per .hip
// translation unit), called by the C-ABI runtime in pg_api.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "pg_params.hpp"

namespace pg {

// Byte layout of the window kernel's dynamic LDS: two buffers (the item
// being stored and the item being prepared), each holding `group` slots of
// factor rows followed by `group` slots of plane masks.
struct WindowLds {
    size_t rows, rows_bytes, masks, masks_bytes, buffer, total;
};

WindowLds window_lds(int a_cap, int row_stride, int C, int D, int mask_words, int group);

// Persistent molecule window kernel (pg_window.hip).
// unroll: runs per lane per pass (1, 2 or 4).
hipError_t launch_window(const GridParams &p, int out_dtype, int vec, int unroll, int block,
                         int grid, size_t lds, hipStream_t s);
int window_occupancy(int out_dtype, int vec, int unroll, int block, size_t lds);

// Per-atom window table into the workspace (pg_plain.hip).
hipError_t launch_prep(const GridParams &p, hipStream_t s);
// One structure (p.mol_index), one thread per output element (pg_plain.hip).
hipError_t launch_plain(const GridParams &p, int out_dtype, hipStream_t s);

// Coordinate adjoint, one wave per atom (pg_adjoint.hip).
hipError_t launch_adjoint(const GridParams &p, int grad_dtype, hipStream_t s);

}  // namespace pg
