/*
 * particlegrid.h -- C ABI of the MI355X (gfx950) atoms -> density-grid library.
 *
 * The operation (ParticleGrid, §III-A "Voxel-filling Function", Eq. 1, and
 * the §V programming interface `coord_to_grid`): given atoms (xyz plus an
 * element type), a per-type Gaussian width sigma_t, and a grid (origin,
 * spacing, dimensions), produce a dense multi-channel grid
 *
 *     G[b][c][z][y][x] = sum over atoms a of structure b with type c of
 *                        exp(-|r(z,y,x) - mu_a|^2 / (2 sigma_c^2))
 *
 * (or, with desc->value = PG_VALUE_BOX, the voxel integral of Eq. 2-5),
 *
 * with r the voxel centre origin + (i + 1/2) * spacing on each axis, one
 * channel per element type (§III-A), the squared distance replaced by the
 * nearest-image distance for an orthorhombic periodic cell (§III-A, text
 * after Eq. 1), and each atom truncated to a cube of half-width
 * rc_t = fl32(cutoff_k * sigma_t) (threshold truncation, §VI-B): a voxel
 * is inside iff |r_alpha - mu_alpha| <= rc_t on every axis, decided exactly
 * on the float inputs.
 *
 * Conventions shared by every call:
 *   - Layout: out is B x C x D x H x W, contiguous, x fastest (D = z,
 *     H = y, W = x), i.e. NCDHW as a 3-D convolution consumes it.
 *   - origin / spacing / cell are given in x, y, z order, in the same unit
 *     as the coordinates (Angstrom in the benchmarks).
 *   - Batches are ragged CSR: structure b owns atoms
 *     [offsets[b], offsets[b+1]).
 *   - All array arguments are DEVICE pointers (memory of the device the
 *     context was created on) unless a field says "host".  The caller owns
 *     every buffer; the library keeps no pointer after a call returns.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream).  The library writes every element of `out` (no pre-zeroing
 *     needed); `out` must not alias any input.
 *   - Every function returns a pg_status.  Host-side validation runs before
 *     any launch; on error nothing is launched.  No exception crosses the
 *     ABI.  Errors found in device data (a type outside [0, C), a
 *     non-finite coordinate, a structure larger than the declared
 *     max_atoms) cannot be reported synchronously: the atom is skipped (or
 *     the structure's grid is written as zeros), a sticky device error word
 *     is set, and pg_get_device_error() reports it after the stream is
 *     synchronised.
 */
#ifndef PARTICLEGRID_H
#define PARTICLEGRID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PG_ABI_VERSION 5
#define PG_MAX_CHANNELS 64

typedef enum pg_status {
    PG_OK = 0,
    PG_E_NULL = 1,         /* a required pointer is NULL */
    PG_E_SHAPE = 2,        /* bad dims, channel count, batch sizes */
    PG_E_PARAM = 3,        /* spacing / sigma / cutoff not positive-finite, bad enum */
    PG_E_PERIODIC = 4,     /* periodic cell too small for the cutoff or the grid */
    PG_E_WORKSPACE = 5,    /* workspace smaller than pg_workspace_size() */
    PG_E_UNSUPPORTED = 6,  /* valid request this build does not serve */
    PG_E_HIP = 7,          /* a HIP runtime call failed (see pg_last_hip_error) */
    PG_E_DEVICE_DATA = 8,  /* device data error (pg_get_device_error) */
    PG_E_CAPACITY = 9      /* a structure exceeded the declared max_atoms */
} pg_status;

enum { PG_OUT_F32 = 0, PG_OUT_BF16 = 1 };

/* What a voxel holds.  POINT: the un-normalised Gaussian exp(-|r - mu|^2 /
   (2 sigma^2)) sampled at the voxel centre (§III-A Eq. 1 without the
   prefactor).  BOX: the integral of the normalised Gaussian over the voxel
   box (§III-A Eq. 2-5), the product over axes of
   (1/2)[erf((x_i + h - mu) / (sqrt(2) sigma)) - erf((x_i - mu) / (sqrt(2) sigma))]
   with x_i the lower voxel edge; a channel then sums to its atom count
   (Eq. 6) up to the cutoff.  Both use the same cutoff windows, decided on
   the voxel centres. */
enum { PG_VALUE_POINT = 0, PG_VALUE_BOX = 1 };

/* Kernel form.  AUTO lets the library choose (per-shape rule, refined by
   pg_autotune).  PLAIN: one thread per voxel, one launch per structure (the
   baseline form).  WINDOW: cutoff-window gather in float32.  For structures
   whose atoms fit the window kernel's LDS (max_atoms <= 256 and the staged
   factor rows within the device's LDS) it is one persistent launch per
   batch with each structure's atoms staged in LDS; larger structures take
   the binned path (atoms binned per (structure, channel, z plane), one
   workgroup per plane).  MFMA: binned path whose plane kernels evaluate
   the separable factorisation (§III-A, §IV-C) of each 32 x 32 tile of a
   plane as a matrix-core contraction over the plane's images that meet
   that tile (atoms binned per (structure, channel, 32 x 32 tile column)),
   with float32 accumulation: for bf16 grids on bf16 factors (phi_z phi_y
   formed in float32 and rounded once); for float32 grids on float32
   factors (exact float32 products, rel-L2 about 1e-7 against the FP64
   definition); meant for large, dense structures.  It takes any number of
   atoms per plane (pg_plan_info.atom_capacity 0) but needs at most 32768
   (tile column, z) keys per channel (tiles_x tiles_y D, e.g. 128^3) and
   at most 16 tiles of factor slots per atom and axis; AUTO falls back to
   the binned WINDOW form, then to PLAIN, where it does not apply.  AUTO
   picks WINDOW when the structure fits, else MFMA.  The binned path needs
   a workspace (pg_workspace_size) and does not take per-structure
   spacings; the binned WINDOW form holds at most 32 tiles of 32 x 32
   voxels per (y, x) plane (PG_E_UNSUPPORTED beyond).  The binned path
   needs D <= 4096. */
enum { PG_FORM_AUTO = 0, PG_FORM_PLAIN = 1, PG_FORM_WINDOW = 2, PG_FORM_MFMA = 3 };

/* Grid description (all fields host values). */
typedef struct pg_grid_desc {
    int32_t C, D, H, W;          /* channels (= element types) and grid dims z, y, x; >= 1 */
    float origin[3];             /* lower grid corner, x y z; used when batch->origins == NULL */
    float spacing[3];            /* voxel edge hx hy hz > 0; used when batch->spacings == NULL */
    float cutoff_k;              /* cutoff in units of sigma_t (>= 0); 0 = no cutoff */
    int32_t periodic;            /* PG_CELL_NONE, PG_CELL_ORTHO (cell[]) or
                                    PG_CELL_TRICLINIC (cell_matrix[]) */
    float cell[3];               /* orthorhombic cell edges Lx Ly Lz */
    int32_t out_dtype;           /* PG_OUT_F32 or PG_OUT_BF16 (round-to-nearest-even) */
    int32_t form;                /* PG_FORM_* */
    float sigma[PG_MAX_CHANNELS];/* Gaussian width (standard deviation) per type, > 0 */
    int32_t value;               /* PG_VALUE_POINT or PG_VALUE_BOX */
    int32_t n_types;             /* with batch->weights: entries of sigma[] the types index
                                    (1..64); 0 means C.  Without weights: 0 or C */
    float cell_matrix[9];        /* triclinic cell, row-major: cell_matrix[3 * alpha + j] is
                                    the alpha (x, y, z) component of lattice vector j */
    int32_t cutoff_shape;        /* PG_CUTOFF_CUBE (default) or PG_CUTOFF_SPHERE */
} pg_grid_desc;

/* Cutoff shape.  PG_CUTOFF_CUBE: |r_alpha - mu_alpha| <= rc_t on every axis,
   decided exactly (separable: every form supports it).  PG_CUTOFF_SPHERE:
   inside the cube, also |r - mu|^2 <= rc_t^2 (nearest image per axis when
   periodic), the squared per-axis offsets summed in float32 -- not exact:
   a voxel within about 1e-6 rc_t^2 of the sphere may fall on either side.
   The sphere breaks separability, so it takes the molecule window form or
   the plain form (AUTO picks plain when the window form does not fit); the
   binned forms return PG_E_UNSUPPORTED. */
enum { PG_CUTOFF_CUBE = 0, PG_CUTOFF_SPHERE = 1 };

/* Periodic cells (§III-A: a structure's density sums the lattice
   translations of each atom).
   PG_CELL_ORTHO: an orthorhombic cell; every voxel uses the nearest image
   per axis, decided exactly (rc_t < L/2 and grid extent + 2 rc_t <= 2 L).
   PG_CELL_TRICLINIC: a general cell M = cell_matrix.  Every atom
   contributes through each lattice image mu + M n (n integer) that
   image's Gaussian truncated to its own cutoff cube; the cell must keep
   the cubes of distinct images of one atom apart (for every n != 0 with
   |n_j| <= 4: max_alpha |(M n)_alpha| > 2 rc_max), so a voxel sees at
   most one image of each atom.  An image's position is the exact sum
   mu_alpha + n_0 M[alpha][0] + n_1 M[alpha][1] + n_2 M[alpha][2] rounded
   once to float32 (nearest, ties to even; found on the GPU from error-free
   float32 transforms, no FP64); its windows are then decided exactly as
   for a non-periodic atom.  The library considers for each atom the K images of
   a fixed lattice range (K <= 64, else PG_E_PERIODIC), keeps those whose
   cutoff cube can meet the grid, and runs the non-periodic map on them; the
   workspace is sized for all K.  Invalid atoms are reported by atom index
   and get no image.  Not with per-structure spacings, weighted channels,
   pg_autotune or pg_reversal_step (PG_E_UNSUPPORTED). */
enum { PG_CELL_NONE = 0, PG_CELL_ORTHO = 1, PG_CELL_TRICLINIC = 2 };

/* A ragged batch of structures (device arrays unless noted). */
typedef struct pg_batch {
    const float *xyz;            /* n_atoms x 3 float32 (x, y, z) */
    const int32_t *types;        /* n_atoms int32 channel ids in [0, C) */
    const int32_t *offsets;      /* n_mol + 1 int32 CSR bounds, offsets[0] = 0, non-decreasing */
    const float *origins;        /* n_mol x 3 per-structure grid origins, or NULL */
    const float *spacings;       /* n_mol x 3 per-structure spacings, or NULL (not with periodic) */
    int32_t n_mol;               /* B >= 0 */
    int32_t max_atoms;           /* host: upper bound of atoms in any one structure */
    int64_t n_atoms;             /* host: offsets[n_mol]; 0 allowed */
    const float *weights;        /* n_atoms x C float32 channel weights, or NULL (see below) */
} pg_batch;

/* Weighted channels.  With batch->weights == NULL each atom feeds the one
   channel of its type (one channel per element, §III-A), and types lie in
   [0, C).  With weights, atom a adds weights[a][c] times its Gaussian to
   every channel c (the learned-embedding grids of the paper's Discussion,
   and the weighted grids mentioned after Eq. 6); its width is still
   sigma[types[a]], types lying in [0, n_types), so the number of element
   types is independent of the channel count.  One-hot weights give the
   unweighted grid bit for bit.  Every form takes weights; the binned
   large-structure path lists each atom under every channel with a non-zero
   weight (its workspace grows with C); the MFMA form for bf16 grids rounds
   the weighted phi_y factor to bf16 once.  Not with triclinic cells
   (PG_E_UNSUPPORTED). */

typedef struct pg_ctx pg_ctx;

/* Version of this ABI (PG_ABI_VERSION). */
int pg_abi_version(void);

/* Static description of a status code; never NULL. */
const char *pg_status_str(int status);

/* Create a context bound to HIP device `device`: it owns the sticky device
   error word, the tuning table and the captured-graph cache.  Allocates a
   few bytes of device memory once (not on the hot path).
   device = PG_HOST_ONLY makes a context that touches no device (it needs
   no GPU): it holds a tuning table and options, pg_plan and
   pg_workspace_size consult it as they would a gfx950 device's (256 CUs,
   160 KiB of LDS per workgroup), pg_tuning_load/save work, and every call
   that would launch or synchronise returns PG_E_UNSUPPORTED.
   Errors: PG_E_NULL, PG_E_PARAM (negative device other than PG_HOST_ONLY),
   PG_E_HIP. */
#define PG_HOST_ONLY (-1)
int pg_create(pg_ctx **ctx, int device);

/* Destroy a context (waits for nothing; the caller synchronises first). */
int pg_destroy(pg_ctx *ctx);

/* Host-only validation of a request (no HIP call, no device access).
   Checks dims, channel count, sigma/spacing/cutoff, periodic constraints
   (orthorhombic: rc_t < L/2 and grid extent + 2 rc_t <= 2 L on every axis;
   triclinic: the image-cube separation and the image count; both:
   cutoff_k > 0), batch sizes and non-NULL device pointers.  Returns PG_OK or the first
   error found. */
int pg_validate(const pg_grid_desc *desc, const pg_batch *batch);

/* Bytes of caller-provided device workspace that pg_grid_forward and
   pg_grid_backward need for this request (0 is possible; triclinic cells
   need it in pg_grid_backward too).  Host only.
   The form used is the one pg_grid_forward would pick (desc->form or the
   AUTO rule); ctx may be NULL (then tuned choices are not consulted). */
int pg_workspace_size(const pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch,
                      size_t *bytes);

/* Forward map (§III-A Eq. 1 point-sampled, or the voxel masses of Eq. 2-5
   under PG_VALUE_BOX; §V coord_to_grid): writes every
   element of out (B x C x D x H x W of float32 or bf16 per
   desc->out_dtype, 16-byte aligned for the vector path; any alignment is
   accepted).  ws/ws_bytes: device workspace of at least
   pg_workspace_size() bytes (may be NULL if that is 0).  stream: hipStream_t.
   If the context's graph option is on, the launch sequence is captured
   once per distinct argument set and replayed as a HIP graph.
   Errors: validation codes, PG_E_WORKSPACE, PG_E_UNSUPPORTED, PG_E_HIP. */
int pg_grid_forward(pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch,
                    void *out, void *ws, size_t ws_bytes, void *stream);

/* pg_grid_forward for callers that cannot allocate device memory: code
   under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc.  Same request, output and result as pg_grid_forward (the same
   kernels; bit-identical output), but no workspace argument: the
   workspace is the library's fixed device scratch buffer of
   PG_STATIC_SCRATCH_BYTES, one per device, held from the library's load
   until the process ends (its address is looked up in pg_create).  The
   call allocates nothing (no hipMalloc / hipFree, no graph instantiation:
   the context's graph option is ignored and the kernels are launched
   directly on `stream`).  Every call on one device shares that device's
   buffer and finds the previous call's contents there (the kernels clear
   what must start at zero), so calls that overlap in time on one device --
   on two streams, or from two contexts -- race and must be serialised by
   the caller.
   Errors: as pg_grid_forward; PG_E_WORKSPACE when the request needs more
   than PG_STATIC_SCRATCH_BYTES of workspace (pg_workspace_size tells). */
#define PG_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int pg_grid_forward_static(pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch,
                           void *out, void *stream);

/* Adjoint (§IV-C coordinate gradient): given grad_out = dL/dG (same shape
   and dtype as the forward's out), writes grad_xyz[a][alpha] = sum over
   voxels v in the window of atom a of grad_out[b][t_a][v] * dG_a(v)/dmu_alpha,
   G_a being the product of per-axis factors phi_x phi_y phi_z.  Point form:
   dphi/dmu = phi (r - mu) / sigma_t^2, with nearest-image offsets when
   periodic.  Box form: dphi/dmu = (g(lower edge) - g(upper edge)) /
   (sqrt(2 pi) sigma_t), g(x) = exp(-(x - mu)^2 / (2 sigma_t^2)) -- the erf
   derivative of §IV-C with the minus of its exponent restored.  The cutoff edge contributes
   nothing (derivative almost everywhere).  grad_xyz: n_atoms x 3 float32,
   fully overwritten (skipped atoms get 0).  With weighted channels the
   atom's upstream is sum_c weights[a][c] grad_out[b][c][v], and
   grad_weights (n_atoms x C float32, or NULL) receives
   dL/dweights[a][c] = sum over the window of grad_out[b][c][v] G_a(v)
   (skipped atoms get 0).  grad_xyz may be NULL when grad_weights is not.
   ws/ws_bytes: pg_workspace_size() bytes for a triclinic cell (the image
   expansion and the image gradients); other requests take NULL, 0.
   Errors: as pg_grid_forward. */
int pg_grid_backward(pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch,
                     const void *grad_out, float *grad_xyz, float *grad_weights, void *ws,
                     size_t ws_bytes, void *stream);

/* Time the candidate kernel configurations (and, under AUTO, the forms)
   for this request on `stream`, keep the fastest in the context's tuning
   table (keyed by dims, channels, dtype, periodicity, batch size and atom
   counts) and use it for later matching calls.  `out` is overwritten
   (reps + 2) times per candidate.  Synchronises the stream.
   Errors: as pg_grid_forward. */
int pg_autotune(pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch,
                void *out, void *ws, size_t ws_bytes, void *stream, int reps);

/* Save / load the tuning table as JSON text (host file I/O only).  Loading
   a missing or malformed file leaves the table empty and returns
   PG_E_PARAM. */
int pg_tuning_save(const pg_ctx *ctx, const char *path);
int pg_tuning_load(pg_ctx *ctx, const char *path);

/* Options: PG_OPT_GRAPH (0/1, default 0) -- replay captured HIP graphs for
   repeated identical forward calls whose launch sequence has several
   kernels (a forward on the one-kernel molecule window form is launched
   directly, which costs less than a replay).  PG_OPT_BLOCK, PG_OPT_GRID_PER_CU,
   PG_OPT_UNROLL, PG_OPT_NT_STORE -- override the window form's workgroup
   size (64..1024, a multiple of 64), persistent workgroups per CU (1..64),
   16-byte output runs per lane per pass (1, 2 or 4) and non-temporal
   stores (0/1); -1 restores the tuned/default choice.  Changing an option
   drops the captured graphs.
   Errors: PG_E_NULL, PG_E_PARAM (unknown option or value). */
enum { PG_OPT_GRAPH = 1, PG_OPT_BLOCK = 2, PG_OPT_GRID_PER_CU = 3, PG_OPT_NT_STORE = 4,
       PG_OPT_UNROLL = 5 };
int pg_set_option(pg_ctx *ctx, int option, int64_t value);

/* Read and clear the sticky device error word (synchronises the context's
   device).  code: PG_OK, PG_E_DEVICE_DATA or PG_E_CAPACITY; first_atom:
   smallest global atom index (or structure index for PG_E_CAPACITY)
   involved, -1 if none.  Errors: PG_E_NULL, PG_E_HIP. */
int pg_get_device_error(pg_ctx *ctx, int32_t *code, int64_t *first_atom);

/* The last hipError_t seen by this context (0 if none). */
int pg_last_hip_error(const pg_ctx *ctx);

/* Describe the kernel configuration pg_grid_forward would use for this
   request: form, workgroup size, workgroups launched (per launch; the
   plain form launches one per structure), dynamic LDS bytes, output vector
   width, non-temporal stores, atom capacity (per structure; per plane bin
   on the binned path), runs per lane per pass and persistent workgroups
   per CU (small-structure window form), and binned = 1 when the request
   takes the binned large-structure path.  Host only.
   Errors: validation codes, PG_E_UNSUPPORTED. */
typedef struct pg_plan_info {
    int32_t form, block, grid, lds_bytes, vec, nt_store, atom_capacity, unroll, per_cu, binned;
} pg_plan_info;
int pg_plan(const pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch,
            const void *out, pg_plan_info *info);

/* ---- Grid reversal (§IV): coordinates back from a grid ---------------- */

/* Initial coordinates of grid reversal (§IV-A step 1; §IV-B locates atoms
   as the grid's local maxima).  grid: B x C x D x H x W float32 (device,
   the layout of pg_grid_forward's output); desc supplies C, D, H, W,
   origin and spacing (other fields are not read) and must have out_dtype
   PG_OUT_F32.  Voxel v of channel c is a peak when grid[v] > threshold and,
   among its 26 neighbours inside the grid (same channel, no wrap), grid[v]
   is greater than every neighbour earlier in raster order (z, then y, then
   x) and not less than any later one, so a plateau of equal maxima yields
   its first voxel.  The peaks of structure b are written in raster order
   (channel, z, y, x) from index offsets_out[b] on: xyz_out (capacity x 3
   float32) receives the exact voxel centre o + (i + 1/2) h rounded once to
   float32 (formed from float-float terms; o, h from origins / spacings, B x 3 device
   arrays, when not NULL, else from desc), types_out (capacity int32) the
   channel.  offsets_out (B + 1 int32, device) receives the CSR bounds, each
   clamped to capacity; *n_found (device int64) the total number of peaks,
   which may exceed capacity (peaks past capacity are not written).  The
   outputs form the pg_batch of pg_reversal_step.  Asynchronous on stream;
   no workspace.
   Errors: PG_E_NULL, PG_E_SHAPE (bad dims, capacity outside [0, 2^31), a
   structure of 2^31 or more elements), PG_E_PARAM (non-finite threshold,
   out_dtype not F32, bad origin or spacing), PG_E_HIP. */
int pg_find_peaks(pg_ctx *ctx, const pg_grid_desc *desc, const float *grid, int32_t n_mol,
                  const float *origins, const float *spacings, float threshold, int64_t capacity,
                  float *xyz_out, int32_t *types_out, int32_t *offsets_out, int64_t *n_found,
                  void *stream);

/* Bytes of caller-provided device workspace pg_reversal_step needs for
   this request (0 is possible).  Host only; ctx may be NULL. */
int pg_reversal_workspace_size(const pg_ctx *ctx, const pg_grid_desc *desc,
                               const pg_batch *batch, size_t *bytes);

/* One coordinate step of grid reversal (§IV-A steps 2-4, §IV-C).  With
   G' the forward map of batch under desc (out_dtype must be PG_OUT_F32)
   and T = target (B x C x D x H x W float32, device):
     residual[b]  = 2 (G' - T)                  B x C x D x H x W float32
     loss[b]      = sum over structure b of (G' - T)^2      B float32
     grad_xyz     = the pg_grid_backward of residual        n_atoms x 3
     xyz_update   = xyz - lr * grad_xyz                     n_atoms x 3
   grad_xyz and xyz_update may be NULL (not written); xyz_update may be
   batch->xyz itself (update in place).  On the molecule window form the
   forward kernel forms the residual and the loss as it goes (G' is never
   stored; per-lane FP32 partial sums, float-float sums across a
   workgroup); other forms store G' in residual and then form both in one
   pass (float-float partial sums).  No step uses FP64 on the GPU.
   residual may be NULL on the molecule window form without weights: no
   residual grid is written (half the HBM traffic of the step) and the
   adjoint forms 2 (G' - T) at each voxel of an atom's window, summing G'
   over the structure's atoms of that channel as the forward does, so loss,
   grad_xyz and xyz_update are bit-identical to a step with a residual
   buffer; elsewhere a NULL residual is PG_E_NULL.
   The loss is deterministic for a given launch configuration.  Under
   PG_OPT_GRAPH the whole step is captured once per argument set and
   replayed.  ws: pg_reversal_workspace_size() bytes.
   Errors: as pg_grid_forward; PG_E_PARAM also for out_dtype not F32 or a
   non-finite lr. */
int pg_reversal_step(pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch,
                     const float *target, float *residual, float *loss, float *grad_xyz,
                     float *xyz_update, float lr, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PARTICLEGRID_H */
