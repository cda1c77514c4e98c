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
// invs2 = fl32(1/sigma^2), and for the box form isq2s, inorm.
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
    int32_t box;             // voxel integral (PG_VALUE_BOX) instead of the point sample
    float isq2s[PG_MAX_CHANNELS];   // fl32(1 / (sqrt(2) sigma)), box form
    float inorm[PG_MAX_CHANNELS];   // fl32(1 / (sqrt(2 pi) sigma)), box-form derivative
    // grid reversal: the forward writes 2 (G - target) and the per-structure
    // loss sum (G - target)^2 instead of G; the adjoint may also write
    // xyz - lr * gradient
    const float *target;
    float *loss;
    float *xyz_upd;
    float lr;
    // reversal step without a stored residual: the adjoint forms
    // 2 (G' - target) itself at each window voxel (out is then nullptr)
    int32_t recompute;
    int32_t rec_ntw;         // recompute: bound on an atom's window indices over the 3 axes
    // weighted channels: n_atoms x C weights (nullptr: one channel per type),
    // their gradient (backward, may be nullptr), and the number of entries
    // of the per-type tables (rc, inv2s2, ...) the types index
    const float *weights;
    float *grad_w;
    int32_t n_sig;
    // sphere cutoff: keep a voxel only if the summed squared offsets are at
    // most rc2 = fl32(rc * rc) of the atom's type
    int32_t sphere;
    float rc2[PG_MAX_CHANNELS];
};

// Peak search of grid reversal: local maxima of every channel of a batch of
// float32 grids, written as a CSR batch of voxel-centre positions.
struct PeakParams {
    const float *grid;
    const float *origins;    // per-structure, or nullptr
    const float *spacings;   // per-structure, or nullptr
    float *xyz;              // capacity x 3
    int32_t *types;          // capacity
    int32_t *offsets;        // n_mol + 1: counts, then the clamped CSR bounds
    long long *n_found;
    long long capacity;
    float o[3], h[3];
    float thr;
    int32_t n_mol, C, D, H, W;
};

// Triclinic cells: expansion of every atom into K lattice images (a * K + k)
// and the sum of the images' gradients back onto the atoms.
struct TriParams {
    const float *xyz;
    const int32_t *types;
    const int32_t *offsets;
    float *exp_xyz;          // n_atoms * K x 3 image positions
    int32_t *exp_types;      // n_atoms * K (-1: invalid atom)
    int32_t *exp_offsets;    // n_mol + 1: offsets * K
    const float *grad_img;   // image gradients, in image order
    float *cand;             // K x n_atoms x 3 candidate image positions (NaN: misses the
                             // grid); the same memory as grad_img, used before it
    float *base;             // n_atoms x 3: lattice index of each atom's candidate image 0
    float *grad;             // n_atoms x 3 (may be nullptr)
    int32_t *istart;         // n_atoms + 1: each atom's first image (in its 256-atom block,
                             // then global), istart[n_atoms] = the image count
    uint32_t *bsum;          // per 256-atom block: its images, then their exclusive scan
    const float *origins;    // per-structure grid origins, or nullptr
    float M[9];              // cell, row-major: M[3 * alpha + j] = alpha component of vector j
    float Minv_hi[9], Minv_lo[9];   // its inverse as float-float pairs (hi + lo)
    float o[3], h[3];        // grid origin and spacing (x, y, z)
    float rc[PG_MAX_CHANNELS];
    int32_t N[3];            // grid points along x, y, z
    int32_t klo[3], kdim[3]; // lattice range of the home-cell copy, per cell axis
    int32_t K, n_mol, n_sig;
    long long n_atoms;
    long long bound;         // images the inner request is sized for (n_atoms x most kept)
};

// Per-atom window table written by the prep kernel (plain form).
struct AtomWindow {
    int32_t type;            // -1: skipped atom
    int32_t n[3];
    int32_t lo[3][3], hi[3][3];
    float bh[3][3], bl[3][3];
};

// One entry of the channel partition: the atom, its z ranges packed as
// (lo | hi << 16) with lo, hi as 16-bit signed values (empty: lo 0, hi -1),
// and the float-float base offset o_z - mu_z - n L_z of each range.
struct alignas(16) ListEntry {
    int32_t atom;
    uint32_t z[3];
    float bh[3], bl[3];
};

// One z image of one atom in the z-sorted order of the MFMA form: the atom,
// its z range packed as in ListEntry, and the range's base offset.
struct ZEntry {
    int32_t atom;
    uint32_t range;
    float bh, bl;
};

// One entry of a tile-column list of the MFMA form: a z image of one atom
// (its z range and the range's float-float base offset o_z - mu_z - n L_z)
// with the slots of the column's y and x tiles among the atom's factor
// slots.  zs packs z lo (bits 0-11), z hi (12-23), the y slot (24-27) and
// the x slot (28-31); the lists are sorted by z lo.
struct TileEntry {
    int32_t atom;
    uint32_t zs;
    float bh, bl;
};

// Binned (large-structure) path.  Per atom: its window record; per channel:
// the stable partition of all atoms by channel (atom index order kept),
// which lays out every (structure, channel) pair ("run") as one contiguous
// stretch of the list; per run, the z images sorted by window start and
// each plane's contiguous range of them.  MFMA form: per atom, phi_x and
// phi_y over each 32-voxel tile its windows meet ("slots", 32 values each,
// zero outside the windows); per run and 32 x 32 (y, x) tile column, the
// list of the run's z images whose windows meet the column, in z order.
struct CrystalParams {
    AtomWindow *table;       // n_atoms window records
    uint32_t *bcount;        // C x nblk atoms per (channel, prep block), then their
                             // exclusive scan in channel-major order
    uint32_t *mcount;        // C x n_mol atoms per run (channel-major)
    uint32_t *mstart;        // C x n_mol exclusive scan of mcount
    ListEntry *list;         // n_atoms entries, channel-major, atom order within a channel
    ZEntry *zlist;           // entry capacity: run r starts at entry 32 * run_block(r)
    uint32_t *ecount;        // C x n_mol z images per run
    uint32_t *prange;        // C x n_mol x D x 2: first and end image of each plane
    // MFMA form
    uint32_t *tmask;         // 2 x n_atoms: 32-voxel tiles the x (even) and y (odd) windows
                             // meet, as bit masks (H, W <= 1024)
    void *xval;              // n_atoms x sx_max x 32 phi_x slot values (bf16 bits or float)
    void *yval;              // n_atoms x sy_max x 32 phi_y slot values
    TileEntry *tcl;          // run r's tile-column lists start at entry 32 * run_block(r) * SS
    uint32_t *zstart;        // C x n_mol x ntc x (D + 1): per list, the first entry
                             // whose z lo is >= z, for z = 0 .. D
    int32_t nblk;            // prep blocks (PREP_BLOCK atoms each)
    int32_t sx_max, sy_max;  // factor slots per atom on x and y (<= 16 each)
    int32_t ntx, nty;        // 32-voxel tiles along x and y
    int32_t zwin[PG_MAX_CHANNELS];   // per channel: bound on the length (voxels) of the z
                                     // windows of its runs' images
};
}  // namespace pg
