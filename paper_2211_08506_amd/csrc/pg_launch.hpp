// pg_launch.hpp -- host-side launchers of the gfx950 kernels (one per .hip
// translation unit), called by the C-ABI runtime in pg_api.cpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "pg_params.hpp"

namespace pg {

// Byte offsets of the window kernel's dynamic LDS regions.
struct WindowLds {
    size_t rows, ranges, masks, types, wts, dsq, total;
};

// weight_ch: channels of per-atom weights held in LDS (0: unweighted);
// sphere: squared-offset rows beside the factor rows
WindowLds window_lds(int a_cap, int row_stride, int C, int D, int mask_words, int weight_ch,
                     bool sphere);

// Persistent molecule window kernel (pg_window.hip); unroll: runs per lane
// per pass (1, 2 or 4).
hipError_t launch_window(const GridParams &p, int out_dtype, int vec, int unroll, int block,
                         int grid, size_t lds, hipStream_t s);

// Per-atom window table into the workspace (pg_plain.hip).
hipError_t launch_prep(const GridParams &p, hipStream_t s);
// One structure (p.mol_index), one thread per output element (pg_plain.hip).
hipError_t launch_plain(const GridParams &p, int out_dtype, hipStream_t s);

// Binned large-structure path (pg_crystal.hip): set-up kernels + the MFMA
// (form PG_FORM_MFMA) or vector-ALU (PG_FORM_WINDOW) plane kernel.
size_t crystal_plane_lds(int form, int H, int W);
int crystal_window_runs(int H, int W);
int crystal_prep_blocks(long long n_atoms);
// Factor slots per atom on one axis of the MFMA form: the 32-voxel tiles
// that a window of at most wmax voxels (periodic: up to 3 images) can meet.
int crystal_axis_slots(int N, int wmax, bool periodic);
size_t crystal_zsort_lds(int D);
// dynamic LDS of the tile-sort workgroup (K = tile columns x D <= 32768 keys)
size_t crystal_tsort_lds(int K);
// planes per wave of the MFMA tile kernels (a workgroup covers two tiles of
// two such plane groups)
int crystal_tile_planes(int out_dtype);
// bytes per factor-slot value of the MFMA form for this output dtype on
// axis 0 (x) or 1 (y)
int crystal_slot_bytes(int out_dtype, int axis);
hipError_t launch_crystal(const GridParams &p, const CrystalParams &q, int form, int out_dtype,
                          size_t lds, hipStream_t s);

// Coordinate adjoint, one wave per atom (pg_adjoint.hip); with p.xyz_upd it
// also writes xyz - p.lr * gradient.
hipError_t launch_adjoint(const GridParams &p, int grad_dtype, hipStream_t s);

// Grid reversal (pg_reversal.hip): the local-maximum peak search, and the
// residual / loss pass over a stored forward grid (p.out, float32) with
// per-chunk float-float partial sums in `partial` (n_mol x residual_chunks
// (hi, lo) pairs).
hipError_t launch_peaks(const PeakParams &p, hipStream_t s);
int residual_chunks(long long per_mol);
hipError_t launch_residual(const GridParams &p, float2 *partial, hipStream_t s);

// Triclinic cells (pg_triclinic.hip): image expansion -- count, scan and
// write of the images that can reach the grid (invalid atoms raise
// PG_E_DEVICE_DATA with their atom index and get no image) -- and the
// image-gradient sum.
hipError_t launch_tri_expand(const TriParams &q, DeviceError *err, hipStream_t s);
hipError_t launch_tri_reduce(const TriParams &q, hipStream_t s);

// Fixed device scratch of the allocation-free forward (pg_scratch.hip):
// scratch_init looks up the current device's copy once (the device must be
// current); scratch_ptr returns it, or nullptr before scratch_init.
hipError_t scratch_init(int device);
void *scratch_ptr(int device);

}  // namespace pg
