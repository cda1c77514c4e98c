// pg_api.cpp -- host runtime and C ABI of the gfx950 density-grid library.
//
// Responsibilities: request validation (host only, before any launch),
// choice of kernel form and launch shape (per-shape rule plus a measured
// tuning table), the captured-HIP-graph cache for repeated identical
// calls, the sticky device error word, and the pg_* exports declared in
// include/particlegrid.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <list>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/particlegrid.h"
#include "pg_launch.hpp"
#include "pg_params.hpp"

using namespace pg;

namespace {

constexpr int kWindowMaxAtoms = 256;   // 4 x 64-bit plane masks
constexpr int kGraphCacheSize = 32;

struct Tuned {
    int block = 0, per_cu = 0, nt = -1, unroll = 0;
    int form = 0;   // large structures: the measured faster form (0 = not tuned)
    double us = 0.0;
};

struct GraphEntry {
    std::string key;
    hipGraphExec_t exec = nullptr;
};

}  // namespace

struct pg_ctx {
    int device = 0;
    int n_cu = 256;
    int max_lds = 65536;
    std::string arch;
    DeviceError *d_err = nullptr;
    hipStream_t cap_stream = nullptr;
    int last_hip = 0;
    // options
    int use_graph = 0;
    int opt_block = -1, opt_per_cu = -1, opt_nt = -1, opt_unroll = -1;
    std::map<std::string, Tuned> tuning;
    std::list<GraphEntry> graphs;   // most recent first
    std::mutex mu;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            changed = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard()
    {
        if (changed)
            hipSetDevice(prev);
    }
};

int hip_fail(pg_ctx *ctx, hipError_t e)
{
    if (ctx)
        ctx->last_hip = (int)e;
    return PG_E_HIP;
}

bool finite_pos(float v) { return std::isfinite(v) && v > 0.f; }

float rc_of(const pg_grid_desc *d, int c)
{
    volatile float r = d->cutoff_k * d->sigma[c];   // fl32(k * sigma)
    return r;
}

// Entries of the per-type tables (sigma and what derives from it): the
// channel count, or with weighted channels the declared number of types.
int n_sig_of(const pg_grid_desc *d, const pg_batch *b)
{
    return (b && b->weights && d->n_types > 0) ? d->n_types : d->C;
}

int tri_check(const pg_grid_desc *d, const pg_batch *b);

int validate(const pg_grid_desc *d, const pg_batch *b)
{
    if (!d || !b)
        return PG_E_NULL;
    if (d->n_types < 0 || d->n_types > PG_MAX_CHANNELS ||
        (!b->weights && d->n_types != 0 && d->n_types != d->C))
        return PG_E_PARAM;
    const int n_sig = n_sig_of(d, b);
    if (d->C < 1 || d->C > PG_MAX_CHANNELS || d->D < 1 || d->H < 1 || d->W < 1)
        return PG_E_SHAPE;
    if (d->D > 32767 || d->H > 32767 || d->W > 32767)
        return PG_E_SHAPE;
    const double vol = (double)d->C * d->D * d->H * d->W;
    if (vol > 2147483647.0)
        return PG_E_SHAPE;
    if (b->n_mol < 0 || b->n_atoms < 0 || b->max_atoms < 0)
        return PG_E_SHAPE;
    if (b->n_atoms > 2147483647LL)
        return PG_E_SHAPE;
    if (b->n_atoms > 0 && b->max_atoms == 0)
        return PG_E_SHAPE;
    if (b->n_atoms > 0 && b->n_mol == 0)
        return PG_E_SHAPE;
    if (b->max_atoms > b->n_atoms)
        return PG_E_SHAPE;
    if (d->out_dtype != PG_OUT_F32 && d->out_dtype != PG_OUT_BF16)
        return PG_E_PARAM;
    if (d->form < PG_FORM_AUTO || d->form > PG_FORM_MFMA)
        return PG_E_PARAM;
    if (d->value != PG_VALUE_POINT && d->value != PG_VALUE_BOX)
        return PG_E_PARAM;
    if (d->cutoff_shape != PG_CUTOFF_CUBE && d->cutoff_shape != PG_CUTOFF_SPHERE)
        return PG_E_PARAM;
    for (int q = 0; q < 3; ++q) {
        if (!finite_pos(d->spacing[q]) || !std::isfinite(d->origin[q]))
            return PG_E_PARAM;
    }
    if (!std::isfinite(d->cutoff_k) || d->cutoff_k < 0.f)
        return PG_E_PARAM;
    for (int t = 0; t < n_sig; ++t)
        if (!finite_pos(d->sigma[t]))
            return PG_E_PARAM;
    if (d->periodic != PG_CELL_NONE && d->periodic != PG_CELL_ORTHO &&
        d->periodic != PG_CELL_TRICLINIC)
        return PG_E_PARAM;
    if (d->periodic == PG_CELL_TRICLINIC) {
        if (d->cutoff_k == 0.f)
            return PG_E_PERIODIC;
        if (b->spacings || b->weights)
            return PG_E_UNSUPPORTED;
        for (int i = 0; i < 9; ++i)
            if (!std::isfinite(d->cell_matrix[i]))
                return PG_E_PERIODIC;
    }
    if (d->periodic == PG_CELL_ORTHO) {
        if (d->cutoff_k == 0.f)
            return PG_E_PERIODIC;
        if (b->spacings)
            return PG_E_UNSUPPORTED;
        const int N[3] = {d->W, d->H, d->D};
        for (int q = 0; q < 3; ++q) {
            if (!finite_pos(d->cell[q]))
                return PG_E_PERIODIC;
            for (int t = 0; t < n_sig; ++t) {
                const double rc = rc_of(d, t);
                if (!(rc < 0.5 * (double)d->cell[q]))
                    return PG_E_PERIODIC;
                if ((double)N[q] * d->spacing[q] + 2.0 * rc > 2.0 * (double)d->cell[q])
                    return PG_E_PERIODIC;
            }
        }
    }
    if (b->n_mol > 0 && !b->offsets)
        return PG_E_NULL;
    if (b->n_atoms > 0 && (!b->xyz || !b->types))
        return PG_E_NULL;
    if (d->periodic == PG_CELL_TRICLINIC)
        return tri_check(d, b);
    return PG_OK;
}

bool weighted(const pg_batch *b) { return b->weights != nullptr && b->n_atoms > 0; }

// Triclinic request: the image expansion (lattice range, K images per atom,
// workspace layout) and the equivalent non-periodic request over images.
struct Tri {
    bool on = false;
    TriParams q;
    pg_grid_desc din;
    pg_batch bin;
    size_t off_types = 0, off_offs = 0, off_grad = 0, off_istart = 0, off_base = 0, off_bsum = 0,
           inner_off = 0;
    int32_t K_keep = 1;      // most images one atom can keep
};

size_t align256(size_t v);

constexpr int kTriMaxImages = 64;
constexpr int kTriCheckReach = 4;

int tri_setup(const pg_grid_desc *d, const pg_batch *b, Tri &T)
{
    T.on = d->periodic == PG_CELL_TRICLINIC;
    if (!T.on)
        return PG_OK;
    std::memset(&T.q, 0, sizeof T.q);
    double M[9], Mi[9];
    for (int i = 0; i < 9; ++i)
        M[i] = d->cell_matrix[i];
    const double det = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                       M[2] * (M[3] * M[7] - M[4] * M[6]);
    if (!std::isfinite(det) || std::fabs(det) < 1e-12)
        return PG_E_PERIODIC;
    Mi[0] = (M[4] * M[8] - M[5] * M[7]) / det;
    Mi[1] = (M[2] * M[7] - M[1] * M[8]) / det;
    Mi[2] = (M[1] * M[5] - M[2] * M[4]) / det;
    Mi[3] = (M[5] * M[6] - M[3] * M[8]) / det;
    Mi[4] = (M[0] * M[8] - M[2] * M[6]) / det;
    Mi[5] = (M[2] * M[3] - M[0] * M[5]) / det;
    Mi[6] = (M[3] * M[7] - M[4] * M[6]) / det;
    Mi[7] = (M[1] * M[6] - M[0] * M[7]) / det;
    Mi[8] = (M[0] * M[4] - M[1] * M[3]) / det;
    // the kernels' copies: the cell as given, its inverse as float-float
    for (int i = 0; i < 9; ++i) {
        T.q.M[i] = d->cell_matrix[i];
        T.q.Minv_hi[i] = (float)Mi[i];
        T.q.Minv_lo[i] = (float)(Mi[i] - (double)T.q.Minv_hi[i]);
    }
    double rc_max = 0.0;
    T.q.n_sig = n_sig_of(d, b);
    for (int t = 0; t < T.q.n_sig; ++t) {
        T.q.rc[t] = rc_of(d, t);
        rc_max = std::max(rc_max, (double)T.q.rc[t]);
    }
    // distinct images of one atom keep their cutoff cubes apart
    const int R = kTriCheckReach;
    for (int n0 = -R; n0 <= R; ++n0)
        for (int n1 = -R; n1 <= R; ++n1)
            for (int n2 = -R; n2 <= R; ++n2) {
                if (!n0 && !n1 && !n2)
                    continue;
                double cheb = 0.0;
                for (int al = 0; al < 3; ++al)
                    cheb = std::max(cheb, std::fabs(n0 * M[3 * al] + n1 * M[3 * al + 1] +
                                                    n2 * M[3 * al + 2]));
                if (!(cheb > 2.0 * rc_max))
                    return PG_E_PERIODIC;
            }
    // lattice range of a home-cell copy (fractional coordinates in [0, 1))
    // whose images can reach the grid box widened by rc_max
    const int N[3] = {d->W, d->H, d->D};
    double gmin[3] = {1e300, 1e300, 1e300}, gmax[3] = {-1e300, -1e300, -1e300};
    for (int c = 0; c < 8; ++c) {
        double x[3];
        for (int al = 0; al < 3; ++al) {
            const double lo = (double)d->origin[al] - rc_max;
            const double hi = (double)d->origin[al] + N[al] * (double)d->spacing[al] + rc_max;
            x[al] = (c >> al) & 1 ? hi : lo;
        }
        for (int j = 0; j < 3; ++j) {
            const double g = Mi[3 * j] * x[0] + Mi[3 * j + 1] * x[1] + Mi[3 * j + 2] * x[2];
            gmin[j] = std::min(gmin[j], g);
            gmax[j] = std::max(gmax[j], g);
        }
    }
    long long K = 1;
    for (int j = 0; j < 3; ++j) {
        const double lo = std::ceil(gmin[j] - 1.0 - 1e-6), hi = std::floor(gmax[j] + 1e-6);
        if (!(hi - lo + 1 <= kTriMaxImages))
            return PG_E_PERIODIC;
        T.q.klo[j] = (int32_t)lo;
        T.q.kdim[j] = (int32_t)std::max(1.0, hi - lo + 1);
        K *= T.q.kdim[j];
    }
    if (K > kTriMaxImages)
        return PG_E_PERIODIC;
    if ((long long)b->n_atoms * K > 2147483647LL)
        return PG_E_SHAPE;
    // images an atom can keep: those inside the grid box widened as the
    // device test widens it (rc_max and a voxel); along cell axis j their
    // fractional coordinates lie in an interval of length l_j, which holds
    // at most floor(l_j) + 1 lattice translates of one atom
    long long K_keep = 1;
    {
        double lmin[3] = {1e300, 1e300, 1e300}, lmax[3] = {-1e300, -1e300, -1e300};
        for (int c = 0; c < 8; ++c) {
            double x[3];
            for (int al = 0; al < 3; ++al) {
                const double w = rc_max + (double)d->spacing[al];
                const double lo = (double)d->origin[al] - w;
                const double hi = (double)d->origin[al] + N[al] * (double)d->spacing[al] + w;
                x[al] = (c >> al) & 1 ? hi : lo;
            }
            for (int j = 0; j < 3; ++j) {
                const double g = Mi[3 * j] * x[0] + Mi[3 * j + 1] * x[1] + Mi[3 * j + 2] * x[2];
                lmin[j] = std::min(lmin[j], g);
                lmax[j] = std::max(lmax[j], g);
            }
        }
        for (int j = 0; j < 3; ++j)
            K_keep *= (long long)std::floor(lmax[j] - lmin[j] + 1e-3) + 1;
        K_keep = std::min(K_keep, K);
    }
    T.K_keep = (int32_t)K_keep;
    T.q.bound = (long long)b->n_atoms * K_keep;
    T.q.K = (int32_t)K;
    T.q.n_mol = b->n_mol;
    T.q.n_atoms = b->n_atoms;
    for (int al = 0; al < 3; ++al) {
        T.q.o[al] = d->origin[al];
        T.q.h[al] = d->spacing[al];
        T.q.N[al] = N[al];
    }
    T.din = *d;
    T.din.periodic = PG_CELL_NONE;
    T.bin = *b;
    T.bin.n_atoms = b->n_atoms * K_keep;
    T.bin.max_atoms = (int32_t)std::min<long long>((long long)b->max_atoms * K_keep, 2147483647LL);
    const size_t nk = (size_t)b->n_atoms * (size_t)K;   // room for every candidate image
    T.off_types = align256(nk * 12);
    T.off_offs = T.off_types + align256(nk * 4);
    T.off_grad = T.off_offs + align256(((size_t)b->n_mol + 1) * 4);
    T.off_istart = T.off_grad + align256(nk * 12);
    T.off_base = T.off_istart + align256(((size_t)b->n_atoms + 1) * 4);
    T.off_bsum = T.off_base + align256((size_t)b->n_atoms * 12);
    T.inner_off = T.off_bsum + align256(((size_t)b->n_atoms / 256 + 2) * 4);
    return PG_OK;
}

int tri_check(const pg_grid_desc *d, const pg_batch *b)
{
    Tri T;
    return tri_setup(d, b, T);
}

// Point the expansion and the inner batch at the workspace.
void tri_bind(Tri &T, const pg_batch *b, void *ws)
{
    unsigned char *w = (unsigned char *)ws;
    T.q.xyz = b->xyz;
    T.q.types = b->types;
    T.q.offsets = b->offsets;
    T.q.exp_xyz = (float *)w;
    T.q.exp_types = (int32_t *)(w + T.off_types);
    T.q.exp_offsets = (int32_t *)(w + T.off_offs);
    T.q.grad_img = (const float *)(w + T.off_grad);
    T.q.cand = (float *)(w + T.off_grad);
    T.q.base = (float *)(w + T.off_base);
    T.q.istart = (int32_t *)(w + T.off_istart);
    T.q.bsum = (uint32_t *)(w + T.off_bsum);
    T.q.origins = b->origins;
    T.bin.xyz = T.q.exp_xyz;
    T.bin.types = T.q.exp_types;
    T.bin.offsets = T.q.exp_offsets;
}

struct Plan {
    int form = PG_FORM_WINDOW;
    bool crystal = false;     // large-structure path (bins + plane kernel)
    int block = 256, grid = 1, per_cu = 0, vec = 1, nt = 1, unroll = 1;
    int a_cap = 8, row_stride = 4, mask_words = 1;
    size_t lds = 0;           // dynamic LDS bytes of one workgroup
    size_t ws = 0;            // workspace bytes
    // binned-path workspace layout (byte offsets) and sizes
    size_t ws_bcount = 0, ws_mcount = 0, ws_mstart = 0, ws_list = 0;
    size_t ws_zlist = 0, ws_ecount = 0, ws_prange = 0;
    size_t ws_tmask = 0, ws_xval = 0, ws_yval = 0, ws_tcl = 0, ws_zstart = 0;
    long long op_blocks = 0;
    int nblk = 0;
    int sx_max = 0, sy_max = 0, ntx = 0, nty = 0;
    int zwin[PG_MAX_CHANNELS] = {};   // per channel: bound on its images' z window lengths
};


size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Most voxels of one axis a window of radius rc can span: floor(2 rc / h) + 1
// centres lie within rc of a point (+2 for rounding), never more than the
// axis holds; the whole axis without a cutoff.
int window_voxels_rc(const pg_grid_desc *d, double rc, int axis, int N)
{
    if (d->cutoff_k == 0.f)
        return N;
    return (int)std::min<double>(N, std::floor(2.0 * rc / (double)d->spacing[axis]) + 3.0);
}

// The same for the widest window of any type.
int window_voxels(const pg_grid_desc *d, const pg_batch *b, int axis, int N)
{
    double rc = 0.0;
    for (int t = 0; t < n_sig_of(d, b); ++t)
        rc = std::max(rc, (double)rc_of(d, t));
    return window_voxels_rc(d, rc, axis, N);
}

// Binned path: workspace layout (window records | per-block channel counts
// | per-structure channel counts | their scan | channel partition | z-sorted
// images | per-run image counts | per-plane image ranges | MFMA form: phi_x
// and phi_y factor slots per atom (bf16, or float for fp32 grids) |
// tile-column lists | their bounds | per-run longest z window and largest
// |weight|) and the plane kernel's LDS.
int crystal_plan(const pg_ctx *ctx, const pg_grid_desc *d, const pg_batch *b, int form, Plan &P)
{
    if (b->spacings)
        return PG_E_UNSUPPORTED;
    if (form == PG_FORM_WINDOW && crystal_window_runs(d->H, d->W) == 0)
        return PG_E_UNSUPPORTED;
    if (d->D > 4096)   // the z sort's LDS counters; z ranges packed as 16-bit values
        return PG_E_UNSUPPORTED;
    P.crystal = true;
    P.form = form;
    P.lds = crystal_plane_lds(form, d->H, d->W);
    const int max_lds = ctx ? ctx->max_lds : 65536;
    if (P.lds > (size_t)max_lds)
        return PG_E_UNSUPPORTED;
    const long long nmc = (long long)b->n_mol * d->C;
    // channel-partition entries: one per atom, or with weighted channels one
    // per (atom, channel with a non-zero weight)
    const long long n_ent = b->n_atoms * (weighted(b) ? d->C : 1);
    if (nmc > 0x7fffffffLL || 3 * n_ent > 0xffffffffLL)
        return PG_E_SHAPE;
    P.nblk = crystal_prep_blocks(b->n_atoms);
    // z images (at most 3 per entry) in 32-image blocks: run r starts at
    // block ceil(3 mstart[r] / 32) + 2 r
    P.op_blocks = (3 * n_ent + 31) / 32 + 2 * nmc + 1;
    size_t off = align256((size_t)b->n_atoms * sizeof(AtomWindow));
    P.ws_bcount = off;
    off += align256((size_t)d->C * P.nblk * 4);
    P.ws_mcount = off;
    off += align256((size_t)nmc * 4);
    P.ws_mstart = off;
    off += align256((size_t)nmc * 4);
    P.ws_list = off;
    off += align256((size_t)std::max<long long>(n_ent, 1) * sizeof(ListEntry));
    P.ws_zlist = off;
    off += align256((size_t)P.op_blocks * 32 * sizeof(ZEntry));
    P.ws_ecount = off;
    off += align256((size_t)nmc * 4);
    P.ws_prange = off;
    off += align256((size_t)nmc * d->D * 8);
    const long long nb = nmc * d->D;
    P.block = 256;
    P.vec = 1;
    long long blocks = nb;
    if (form == PG_FORM_MFMA) {
        P.ntx = (d->W + 31) / 32;
        P.nty = (d->H + 31) / 32;
        if ((long long)P.ntx * P.nty * d->D > 32768)   // the tile sort's LDS key counters
            return PG_E_UNSUPPORTED;
        if (P.ntx > 32 || P.nty > 32)   // tiles met per axis as 32-bit masks
            return PG_E_UNSUPPORTED;
        const bool per = d->periodic == PG_CELL_ORTHO;
        P.sx_max = crystal_axis_slots(d->W, window_voxels(d, b, 0, d->W), per);
        P.sy_max = crystal_axis_slots(d->H, window_voxels(d, b, 1, d->H), per);
        // z window bound per channel: a run of an unweighted channel holds
        // atoms of that type only; weighted channels take any type
        const int zmax = window_voxels(d, b, 2, d->D);
        for (int c = 0; c < d->C; ++c)
            P.zwin[c] = weighted(b) ? zmax : window_voxels_rc(d, rc_of(d, c), 2, d->D);
        // tile-column entries: run r's lists start at entry 32 run_block(r) SS
        const long long ss = (long long)P.sx_max * P.sy_max;
        const long long n_tcl = 32 * P.op_blocks * ss;
        if (P.sx_max > 16 || P.sy_max > 16 || n_tcl > 0xffffffffLL)   // slots packed in 4 bits
            return PG_E_UNSUPPORTED;
        // the tile kernels address slot values by 32-bit byte offsets
        if ((long long)b->n_atoms * std::max(P.sx_max, P.sy_max) * 32 * 4 > 0xffffffffLL)
            return PG_E_UNSUPPORTED;
        // slots: x bf16 for bf16 grids and float for fp32 grids, y float
        P.ws_tmask = off;
        off += align256((size_t)b->n_atoms * 2 * 4);
        P.ws_xval = off;
        off += align256((size_t)b->n_atoms * P.sx_max * 32 * crystal_slot_bytes(d->out_dtype, 0));
        P.ws_yval = off;
        off += align256((size_t)b->n_atoms * P.sy_max * 32 * crystal_slot_bytes(d->out_dtype, 1));
        P.ws_tcl = off;
        off += align256((size_t)n_tcl * sizeof(TileEntry));
        P.ws_zstart = off;   // (D + 1) words per list: 4 bytes per 1024 output voxels
        off += align256((size_t)nmc * P.ntx * P.nty * (d->D + 1) * 4);
        const int zp = crystal_tile_planes(d->out_dtype);
        blocks = nmc * P.nty * ((P.ntx + 1) / 2) * ((d->D + 2 * zp - 1) / (2 * zp));
    }
    P.ws = off;
    if (blocks * P.block > 0xffffffffLL)   // grid size limit of one launch
        return PG_E_UNSUPPORTED;
    P.grid = (int)blocks;
    return PG_OK;
}

std::string tuning_key(const pg_grid_desc *d, const pg_batch *b, int vec)
{
    int nb = 0;
    while ((1 << nb) < std::max(1, b->n_mol))
        ++nb;
    int ma = 8;
    while (ma < b->max_atoms)
        ma <<= 1;
    char buf[160];
    std::snprintf(buf, sizeof buf, "C%d_D%d_H%d_W%d_%s_p%d_v%d_nb%d_ma%d%s", d->C, d->D, d->H,
                  d->W, d->out_dtype == PG_OUT_BF16 ? "bf16" : "f32", d->periodic, vec, nb, ma,
                  d->value == PG_VALUE_BOX ? (b->weights ? "_box_w" : "_box")
                                           : (b->weights ? "_w" : ""));
    if (d->cutoff_shape == PG_CUTOFF_SPHERE)
        std::strncat(buf, "_sph", sizeof buf - std::strlen(buf) - 1);
    return buf;
}

int pick_vec(const pg_grid_desc *d, const void *out)
{
    const int esz = d->out_dtype == PG_OUT_BF16 ? 2 : 4;
    const int maxv = 16 / esz;
    for (int v = maxv; v > 1; v >>= 1) {
        if (d->W % v == 0 && ((uintptr_t)out % (uintptr_t)(v * esz)) == 0)
            return v;
    }
    return 1;
}

// Runs per lane per pass: enough to cover a plane in one pass when it is
// small, at most 4.
int default_unroll(const pg_grid_desc *d, int vec)
{
    const long runs = ((long)d->H * d->W / vec + 63) / 64;
    return runs >= 4 ? 4 : (runs >= 2 ? 2 : 1);
}

int window_grid(const pg_batch *b, const Plan &P, int n_cu)
{
    return std::max(1, std::min(b->n_mol, n_cu * P.per_cu));
}

bool window_fits(const pg_ctx *ctx, const pg_grid_desc *d, const pg_batch *b, Plan &P)
{
    if (b->max_atoms > kWindowMaxAtoms)
        return false;
    P.a_cap = std::max(8, (b->max_atoms + 7) & ~7);
    const int W4 = (d->W + 3) & ~3;
    P.row_stride = (W4 + d->H + d->D + 3) & ~3;
    P.mask_words = (P.a_cap + 63) / 64;
    P.lds = window_lds(P.a_cap, P.row_stride, d->C, d->D, P.mask_words,
                       b->weights ? d->C : 0, d->cutoff_shape == PG_CUTOFF_SPHERE).total;
    P.ws = 0;
    const int max_lds = ctx ? ctx->max_lds : 65536;
    return P.lds <= (size_t)max_lds;
}

int make_plan(const pg_ctx *ctx, const pg_grid_desc *d, const pg_batch *b, const void *out, Plan &P)
{
    int s = validate(d, b);
    if (s != PG_OK)
        return s;
    // a triclinic request is planned over its images (plan_request)
    if (d->periodic == PG_CELL_TRICLINIC)
        return PG_E_UNSUPPORTED;
    P.vec = pick_vec(d, out);
    const bool fits = window_fits(ctx, d, b, P);
    int form = d->form;
    if (form == PG_FORM_AUTO) {
        if (fits) {
            form = PG_FORM_WINDOW;
        } else {
            // large structures: the MFMA contraction (bf16 factors for bf16
            // grids, FP32 factors on the FP32 matrix instruction for fp32
            // grids).  A measured choice (pg_autotune) overrides.
            form = PG_FORM_MFMA;
            if (ctx) {
                auto it = ctx->tuning.find(tuning_key(d, b, P.vec));
                if (it != ctx->tuning.end() && it->second.form > 0)
                    form = it->second.form;
            }
        }
    }
    // the sphere is not separable: molecule window form or plain form
    const bool sphere = d->cutoff_shape == PG_CUTOFF_SPHERE && d->cutoff_k != 0.f;
    if (sphere && d->form == PG_FORM_AUTO && !fits)
        form = PG_FORM_PLAIN;
    if (sphere && (form == PG_FORM_MFMA || (form == PG_FORM_WINDOW && !fits)))
        return PG_E_UNSUPPORTED;
    P.form = form;
    if (form == PG_FORM_MFMA || (form == PG_FORM_WINDOW && !fits)) {
        const int vec = P.vec;
        s = crystal_plan(ctx, d, b, form, P);
        if (s != PG_E_UNSUPPORTED || d->form != PG_FORM_AUTO)
            return s;
        // AUTO on a request the chosen binned form does not serve (plane too
        // large for its tile bookkeeping, per-structure spacings, ...): the
        // other binned form, else the plain form
        P = Plan();
        P.vec = vec;
        s = crystal_plan(ctx, d, b, form == PG_FORM_MFMA ? PG_FORM_WINDOW : PG_FORM_MFMA, P);
        if (s != PG_E_UNSUPPORTED)
            return s;
        P = Plan();
        P.vec = vec;
        form = P.form = PG_FORM_PLAIN;
    }
    if (form == PG_FORM_PLAIN) {
        P.ws = (size_t)b->n_atoms * sizeof(AtomWindow);
        P.ws = (P.ws + 255) & ~(size_t)255;
        P.block = 256;
        P.lds = 0;
        return PG_OK;
    }
    // window form: launch shape from options > tuning table > default
    P.block = 512;
    P.per_cu = 2;
    P.nt = 0;
    P.unroll = default_unroll(d, P.vec);
    if (ctx) {
        auto it = ctx->tuning.find(tuning_key(d, b, P.vec));
        if (it != ctx->tuning.end()) {
            P.block = it->second.block;
            P.per_cu = it->second.per_cu;
            P.nt = it->second.nt;
            P.unroll = it->second.unroll;
        }
        if (ctx->opt_unroll > 0)
            P.unroll = ctx->opt_unroll;
        if (ctx->opt_block > 0)
            P.block = ctx->opt_block;
        if (ctx->opt_per_cu > 0)
            P.per_cu = ctx->opt_per_cu;
        if (ctx->opt_nt >= 0)
            P.nt = ctx->opt_nt;
    }
    if (sphere)
        P.unroll = 1;   // the sphere variant of the window kernel runs one run per lane
    const int n_cu = ctx ? ctx->n_cu : 256;
    P.grid = window_grid(b, P, n_cu);
    return PG_OK;
}

// Validate, then plan the request: for a triclinic cell the plan of the
// non-periodic request over the images (T.on), whose workspace follows
// the expansion's.  total_ws: all workspace bytes.
int plan_request(const pg_ctx *ctx, const pg_grid_desc *d, const pg_batch *b, const void *out,
                 Plan &P, Tri &T, size_t &total_ws)
{
    int s = validate(d, b);
    if (s != PG_OK)
        return s;
    s = tri_setup(d, b, T);
    if (s != PG_OK)
        return s;
    if (!T.on) {
        s = make_plan(ctx, d, b, out, P);
        total_ws = P.ws;
        return s;
    }
    s = make_plan(ctx, &T.din, &T.bin, out, P);
    total_ws = T.inner_off + P.ws;
    return s;
}

void fill_params(GridParams &p, const pg_ctx *ctx, const pg_grid_desc *d, const pg_batch *b,
                 const Plan &P, void *out, void *ws)
{
    std::memset(&p, 0, sizeof p);
    p.xyz = b->xyz;
    p.types = b->types;
    p.offsets = b->offsets;
    p.origins = b->origins;
    p.spacings = b->spacings;
    p.out = out;
    p.ws = ws;
    p.err = ctx->d_err;
    p.n_mol = b->n_mol;
    p.n_atoms = b->n_atoms;
    p.C = d->C;
    p.D = d->D;
    p.H = d->H;
    p.W = d->W;
    p.periodic = d->periodic;
    p.cut = d->cutoff_k != 0.f;
    p.a_cap = P.a_cap;
    p.nt_store = P.nt;
    p.row_stride = P.row_stride;
    p.mask_words = P.mask_words;
    for (int q = 0; q < 3; ++q) {
        p.o[q] = d->origin[q];
        p.h[q] = d->spacing[q];
        p.L[q] = d->periodic ? d->cell[q] : 0.f;
    }
    p.n_sig = n_sig_of(d, b);
    for (int t = 0; t < p.n_sig; ++t) {
        const double s = d->sigma[t];
        p.rc[t] = rc_of(d, t);
        p.inv2s2[t] = (float)(1.0 / (2.0 * s * s));
        p.invs2[t] = (float)(1.0 / (s * s));
        p.isq2s[t] = (float)(1.0 / (std::sqrt(2.0) * s));
        p.inorm[t] = (float)(1.0 / (std::sqrt(2.0 * M_PI) * s));
    }
    p.box = d->value == PG_VALUE_BOX;
    p.weights = weighted(b) ? b->weights : nullptr;
    p.sphere = d->cutoff_shape == PG_CUTOFF_SPHERE && d->cutoff_k != 0.f;
    for (int t = 0; t < p.n_sig; ++t)
        p.rc2[t] = p.rc[t] * p.rc[t];
}

hipError_t launch_forward(pg_ctx *ctx, const pg_grid_desc *d, const Plan &P, GridParams &p,
                          hipStream_t s)
{
    if (p.n_mol == 0)
        return hipSuccess;
    if (P.form == PG_FORM_PLAIN) {
        hipError_t e = launch_prep(p, s);
        if (e != hipSuccess)
            return e;
        for (int m = 0; m < p.n_mol; ++m) {
            p.mol_index = m;
            e = launch_plain(p, d->out_dtype, s);
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    }
    if (P.crystal) {
        unsigned char *ws = (unsigned char *)p.ws;
        CrystalParams q;
        q.table = (AtomWindow *)ws;
        q.bcount = (uint32_t *)(ws + P.ws_bcount);
        q.mcount = (uint32_t *)(ws + P.ws_mcount);
        q.mstart = (uint32_t *)(ws + P.ws_mstart);
        q.list = (ListEntry *)(ws + P.ws_list);
        q.zlist = (ZEntry *)(ws + P.ws_zlist);
        q.ecount = (uint32_t *)(ws + P.ws_ecount);
        q.prange = (uint32_t *)(ws + P.ws_prange);
        q.tmask = P.form == PG_FORM_MFMA ? (uint32_t *)(ws + P.ws_tmask) : nullptr;
        q.xval = ws + P.ws_xval;
        q.yval = ws + P.ws_yval;
        q.tcl = (TileEntry *)(ws + P.ws_tcl);
        q.zstart = (uint32_t *)(ws + P.ws_zstart);
        q.nblk = P.nblk;
        for (int c = 0; c < PG_MAX_CHANNELS; ++c)
            q.zwin[c] = P.zwin[c];
        q.sx_max = P.sx_max;
        q.sy_max = P.sy_max;
        q.ntx = P.ntx;
        q.nty = P.nty;
        return launch_crystal(p, q, P.form, d->out_dtype, P.lds, s);
    }
    return launch_window(p, d->out_dtype, P.vec, P.unroll, P.block, P.grid, P.lds, s);
}

std::string graph_key(const pg_grid_desc *d, const pg_batch *b, const Plan &P, const void *out,
                      const void *ws, size_t ws_bytes)
{
    std::string k;
    k.append((const char *)d, sizeof *d);
    k.append((const char *)b, sizeof *b);
    k.append((const char *)&P, sizeof P);
    k.append((const char *)&out, sizeof out);
    k.append((const char *)&ws, sizeof ws);
    k.append((const char *)&ws_bytes, sizeof ws_bytes);
    return k;
}

// Run a launch sequence directly, or (graph option on) capture it once per
// distinct key on the context's capture stream and replay the cached graph.
template <class F>
int run_launches(pg_ctx *ctx, bool graph, const std::string &key, hipStream_t s, F &&launch)
{
    if (!graph) {
        hipError_t e = launch(s);
        return e == hipSuccess ? PG_OK : hip_fail(ctx, e);
    }
    auto it = std::find_if(ctx->graphs.begin(), ctx->graphs.end(),
                           [&](const GraphEntry &g) { return g.key == key; });
    if (it == ctx->graphs.end()) {
        hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess)
            return hip_fail(ctx, e);
        hipError_t le = launch(ctx->cap_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(ctx->cap_stream, &g);
        if (le != hipSuccess || e != hipSuccess) {
            if (g)
                hipGraphDestroy(g);
            return hip_fail(ctx, le != hipSuccess ? le : e);
        }
        GraphEntry ent;
        ent.key = key;
        e = hipGraphInstantiate(&ent.exec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess)
            return hip_fail(ctx, e);
        ctx->graphs.push_front(std::move(ent));
        if ((int)ctx->graphs.size() > kGraphCacheSize) {
            hipGraphExecDestroy(ctx->graphs.back().exec);
            ctx->graphs.pop_back();
        }
        it = ctx->graphs.begin();
    } else if (it != ctx->graphs.begin()) {
        ctx->graphs.splice(ctx->graphs.begin(), ctx->graphs, it);
        it = ctx->graphs.begin();
    }
    hipError_t e = hipGraphLaunch(it->exec, s);
    return e == hipSuccess ? PG_OK : hip_fail(ctx, e);
}

int forward_impl(pg_ctx *ctx, const pg_grid_desc *d, const pg_batch *b, void *out, void *ws,
                 size_t ws_bytes, hipStream_t s, const Plan &P, bool allow_graph)
{
    if (b->n_mol > 0 && !out)
        return PG_E_NULL;
    if (ws_bytes < P.ws || (P.ws > 0 && !ws))
        return PG_E_WORKSPACE;
    GridParams p;
    fill_params(p, ctx, d, b, P, out, ws);
    // the molecule window form is one kernel: replaying a graph of it costs
    // more than launching it (measured 8 us per call), so it is launched
    // directly under the graph option too
    const bool single = !P.crystal && P.form == PG_FORM_WINDOW;
    const bool graph = allow_graph && ctx->use_graph && b->n_mol > 0 && !single;
    return run_launches(ctx, graph, graph ? graph_key(d, b, P, out, ws, ws_bytes) : std::string(),
                        s, [&](hipStream_t st) {
                            GridParams q = p;
                            return launch_forward(ctx, d, P, q, st);
                        });
}

// Grid reversal step: the forward plan of the residual buffer, whether the
// molecule window kernel forms the residual itself (fused), and the
// workspace (the forward's, then float-float partial loss sums when not fused).
struct RevPlan {
    Plan P;
    bool fused = false;
    size_t partial_off = 0;
    size_t ws = 0;
};

int reversal_plan(const pg_ctx *ctx, const pg_grid_desc *d, const pg_batch *b,
                  const float *residual, const float *target, RevPlan &R)
{
    if (d && d->out_dtype != PG_OUT_F32)
        return PG_E_PARAM;
    int s = make_plan(ctx, d, b, residual, R.P);
    if (s != PG_OK)
        return s;
    const int max_lds = ctx ? ctx->max_lds : 65536;
    // the residual variant adds 128 bytes of static LDS for its loss sums
    R.fused = R.P.form == PG_FORM_WINDOW && !R.P.crystal && R.P.lds + 128 <= (size_t)max_lds;
    if (R.fused && target)
        R.P.vec = std::min(R.P.vec, pick_vec(d, target));
    R.partial_off = align256(R.P.ws);
    R.ws = R.fused ? R.P.ws
                   : R.partial_off + (size_t)b->n_mol *
                                         residual_chunks((long long)d->C * d->D * d->H * d->W) *
                                         sizeof(float2);
    return PG_OK;
}

// Most voxel indices an atom's cube window spans over the three axes: at
// most floor(2 rc / h) + 1 centres lie within rc of the atom on an axis
// (+2 for rounding), and never more than the axis holds; the axis length
// with per-structure spacings, and for periodic cells (a grid wider than
// the cell can hold several images of one window).
int window_index_bound(const GridParams &p)
{
    double rc = 0.0;
    for (int t = 0; t < p.n_sig; ++t)
        rc = std::max(rc, (double)p.rc[t]);
    const int N[3] = {p.W, p.H, p.D};
    int total = 0;
    for (int q = 0; q < 3; ++q) {
        int w = N[q];
        if (!p.spacings && !p.periodic && p.cut)
            w = (int)std::min<double>(N[q], std::floor(2.0 * rc / (double)p.h[q]) + 3.0);
        total += w;
    }
    return total;
}

// Forward request on a given workspace.  allow_graph: the context's graph
// option may capture and replay the launches (the allocation-free entry
// point passes false and always launches directly).  Called with ctx->mu
// held.
int forward_request(pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch, void *out,
                    void *ws, size_t ws_bytes, hipStream_t stream, bool allow_graph)
{
    Plan P;
    Tri T;
    size_t total = 0;
    int s = plan_request(ctx, desc, batch, out, P, T, total);
    if (s != PG_OK)
        return s;
    DeviceGuard g(ctx->device);
    if (!T.on)
        return forward_impl(ctx, desc, batch, out, ws, ws_bytes, stream, P, allow_graph);
    // triclinic: expand the atoms into their lattice images in the
    // workspace, then the non-periodic map over the images
    if (batch->n_mol > 0 && !out)
        return PG_E_NULL;
    if (ws_bytes < total || (total > 0 && !ws))
        return PG_E_WORKSPACE;
    if (batch->n_mol == 0)
        return PG_OK;
    tri_bind(T, batch, ws);
    GridParams p;
    fill_params(p, ctx, &T.din, &T.bin, P, out, (unsigned char *)ws + T.inner_off);
    const bool graph = allow_graph && ctx->use_graph;
    std::string key;
    if (graph) {
        key = graph_key(desc, batch, P, out, ws, ws_bytes);
        key.append("triclinic");
    }
    return run_launches(ctx, graph, key, stream, [&](hipStream_t st) -> hipError_t {
        hipError_t e = launch_tri_expand(T.q, ctx->d_err, st);
        if (e != hipSuccess)
            return e;
        GridParams q = p;
        return launch_forward(ctx, &T.din, P, q, st);
    });
}

void drop_graphs(pg_ctx *ctx)
{
    for (auto &g : ctx->graphs)
        hipGraphExecDestroy(g.exec);
    ctx->graphs.clear();
}

}  // namespace

extern "C" {

int pg_abi_version(void) { return PG_ABI_VERSION; }

const char *pg_status_str(int status)
{
    switch (status) {
    case PG_OK: return "ok";
    case PG_E_NULL: return "required pointer is NULL";
    case PG_E_SHAPE: return "invalid dimensions, channel count or batch sizes";
    case PG_E_PARAM: return "invalid parameter (spacing, sigma, cutoff, dtype or form)";
    case PG_E_PERIODIC: return "periodic cell too small for the cutoff or the grid";
    case PG_E_WORKSPACE: return "workspace too small";
    case PG_E_UNSUPPORTED: return "request not supported by this build";
    case PG_E_HIP: return "HIP runtime error";
    case PG_E_DEVICE_DATA: return "invalid device data (atom type out of range or non-finite coordinate)";
    case PG_E_CAPACITY: return "a structure exceeds the declared max_atoms";
    default: return "unknown status";
    }
}

int pg_create(pg_ctx **out, int device)
{
    if (!out)
        return PG_E_NULL;
    *out = nullptr;
    if (device == PG_HOST_ONLY) {
        // planning and tuning tables only: the shape of a gfx950 device
        pg_ctx *ctx = new pg_ctx();
        ctx->device = PG_HOST_ONLY;
        ctx->n_cu = 256;
        ctx->max_lds = 163840;
        ctx->arch = "gfx950 (host-only context)";
        *out = ctx;
        return PG_OK;
    }
    if (device < 0)
        return PG_E_PARAM;
    pg_ctx *ctx = new pg_ctx();
    ctx->device = device;
    DeviceGuard g(device);
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete ctx;
        return PG_E_HIP;
    }
    ctx->n_cu = prop.multiProcessorCount;
    ctx->arch = prop.gcnArchName;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
        lds > 0)
        ctx->max_lds = lds;
    e = hipMalloc((void **)&ctx->d_err, sizeof(DeviceError));
    if (e == hipSuccess) {
        DeviceError z = {0u, 0u, ~0ull};
        e = hipMemcpy(ctx->d_err, &z, sizeof z, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
    // the device's copy of the fixed scratch buffer (pg_grid_forward_static),
    // looked up once per device with the device current
    if (e == hipSuccess)
        e = scratch_init(device);
    if (e != hipSuccess) {
        if (ctx->cap_stream)
            hipStreamDestroy(ctx->cap_stream);
        if (ctx->d_err)
            hipFree(ctx->d_err);
        delete ctx;
        return PG_E_HIP;
    }
    *out = ctx;
    return PG_OK;
}

int pg_destroy(pg_ctx *ctx)
{
    if (!ctx)
        return PG_E_NULL;
    if (ctx->device != PG_HOST_ONLY) {
        DeviceGuard g(ctx->device);
        drop_graphs(ctx);
        if (ctx->cap_stream)
            hipStreamDestroy(ctx->cap_stream);
        if (ctx->d_err)
            hipFree(ctx->d_err);
    }
    delete ctx;
    return PG_OK;
}

int pg_validate(const pg_grid_desc *desc, const pg_batch *batch) { return validate(desc, batch); }

int pg_workspace_size(const pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch,
                      size_t *bytes)
{
    if (!bytes)
        return PG_E_NULL;
    *bytes = 0;
    Plan P;
    Tri T;
    size_t total = 0;
    int s = plan_request(ctx, desc, batch, nullptr, P, T, total);
    if (s != PG_OK)
        return s;
    *bytes = total;
    return PG_OK;
}

int pg_plan(const pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch, const void *out,
            pg_plan_info *info)
{
    if (!info)
        return PG_E_NULL;
    Plan P;
    Tri T;
    size_t total = 0;
    int s = plan_request(ctx, desc, batch, out, P, T, total);
    if (s != PG_OK)
        return s;
    info->form = P.form;
    info->block = P.block;
    info->grid = P.form == PG_FORM_PLAIN ? batch->n_mol : P.grid;
    info->lds_bytes = (int32_t)P.lds;
    info->vec = P.form == PG_FORM_PLAIN ? 1 : P.vec;
    info->nt_store = P.form == PG_FORM_PLAIN ? 0 : P.nt;
    info->atom_capacity = P.form == PG_FORM_PLAIN ? 0 : P.a_cap;
    const bool mol_window = P.form == PG_FORM_WINDOW && !P.crystal;
    info->unroll = mol_window ? P.unroll : 0;
    info->per_cu = mol_window ? P.per_cu : 0;
    if (P.crystal)
        info->atom_capacity = 0;   // the binned forms take any number of atoms per plane
    info->binned = P.crystal ? 1 : 0;
    return PG_OK;
}

int pg_grid_forward(pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch, void *out,
                    void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx)
        return PG_E_NULL;
    if (ctx->device == PG_HOST_ONLY)
        return PG_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(ctx->mu);
    return forward_request(ctx, desc, batch, out, ws, ws_bytes, (hipStream_t)stream, true);
}

int pg_grid_forward_static(pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch,
                           void *out, void *stream)
{
    if (!ctx)
        return PG_E_NULL;
    if (ctx->device == PG_HOST_ONLY)
        return PG_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(ctx->mu);
    Plan P;
    Tri T;
    size_t total = 0;
    int s = plan_request(ctx, desc, batch, out, P, T, total);
    if (s != PG_OK)
        return s;
    if (total > PG_STATIC_SCRATCH_BYTES)
        return PG_E_WORKSPACE;
    void *ws = total > 0 ? scratch_ptr(ctx->device) : nullptr;
    if (total > 0 && !ws)   // pg_create looks the buffer up; a context always has it
        return PG_E_HIP;
    return forward_request(ctx, desc, batch, out, ws, PG_STATIC_SCRATCH_BYTES,
                           (hipStream_t)stream, false);
}

int pg_grid_backward(pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch,
                     const void *grad_out, float *grad_xyz, float *grad_weights, void *ws,
                     size_t ws_bytes, void *stream)
{
    (void)ws;
    (void)ws_bytes;
    if (!ctx)
        return PG_E_NULL;
    if (ctx->device == PG_HOST_ONLY)
        return PG_E_UNSUPPORTED;
    int s = validate(desc, batch);
    if (s != PG_OK)
        return s;
    if (grad_weights && !batch->weights)
        return PG_E_PARAM;
    if (batch->n_atoms > 0 && (!grad_out || (!grad_xyz && !grad_weights)))
        return PG_E_NULL;
    if (batch->n_atoms == 0)
        return PG_OK;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    Plan P;
    P.a_cap = 0;
    GridParams p;
    Tri T;
    s = tri_setup(desc, batch, T);
    if (s != PG_OK)
        return s;
    if (!T.on) {
        fill_params(p, ctx, desc, batch, P, const_cast<void *>(grad_out), nullptr);
        p.grad_xyz = grad_xyz;
        p.grad_w = grad_weights;
        hipError_t e = launch_adjoint(p, desc->out_dtype, (hipStream_t)stream);
        return e == hipSuccess ? PG_OK : hip_fail(ctx, e);
    }
    // triclinic: the images' gradients into the workspace, then their sum
    // onto each atom
    Plan Pf;
    size_t total = 0;
    s = plan_request(ctx, desc, batch, nullptr, Pf, T, total);
    if (s != PG_OK)
        return s;
    if (ws_bytes < total || !ws)
        return PG_E_WORKSPACE;
    tri_bind(T, batch, ws);
    fill_params(p, ctx, &T.din, &T.bin, P, const_cast<void *>(grad_out), nullptr);
    p.grad_xyz = (float *)((unsigned char *)ws + T.off_grad);
    T.q.grad = grad_xyz;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = launch_tri_expand(T.q, ctx->d_err, st);
    if (e == hipSuccess)
        e = launch_adjoint(p, desc->out_dtype, st);
    if (e == hipSuccess)
        e = launch_tri_reduce(T.q, st);
    return e == hipSuccess ? PG_OK : hip_fail(ctx, e);
}

int pg_find_peaks(pg_ctx *ctx, const pg_grid_desc *desc, const float *grid, int32_t n_mol,
                  const float *origins, const float *spacings, float threshold, int64_t capacity,
                  float *xyz_out, int32_t *types_out, int32_t *offsets_out, int64_t *n_found,
                  void *stream)
{
    if (!ctx || !desc || !offsets_out || !n_found)
        return PG_E_NULL;
    if (ctx->device == PG_HOST_ONLY)
        return PG_E_UNSUPPORTED;
    if (n_mol < 0 || capacity < 0 || capacity > INT32_MAX)
        return PG_E_SHAPE;
    if (desc->C < 1 || desc->C > PG_MAX_CHANNELS || desc->D < 1 || desc->H < 1 || desc->W < 1)
        return PG_E_SHAPE;
    if ((long long)desc->C * desc->D * desc->H * desc->W >= (1ll << 31))
        return PG_E_SHAPE;
    if (desc->out_dtype != PG_OUT_F32 || !std::isfinite(threshold))
        return PG_E_PARAM;
    for (int q = 0; q < 3; ++q) {
        if (!origins && !std::isfinite(desc->origin[q]))
            return PG_E_PARAM;
        if (!spacings && !finite_pos(desc->spacing[q]))
            return PG_E_PARAM;
    }
    if ((n_mol > 0 && !grid) || (capacity > 0 && (!xyz_out || !types_out)))
        return PG_E_NULL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    PeakParams p;
    std::memset(&p, 0, sizeof p);
    p.grid = grid;
    p.origins = origins;
    p.spacings = spacings;
    p.xyz = xyz_out;
    p.types = types_out;
    p.offsets = offsets_out;
    p.n_found = (long long *)n_found;
    p.capacity = capacity;
    for (int q = 0; q < 3; ++q) {
        p.o[q] = desc->origin[q];
        p.h[q] = desc->spacing[q];
    }
    p.thr = threshold;
    p.n_mol = n_mol;
    p.C = desc->C;
    p.D = desc->D;
    p.H = desc->H;
    p.W = desc->W;
    hipError_t e = launch_peaks(p, (hipStream_t)stream);
    return e == hipSuccess ? PG_OK : hip_fail(ctx, e);
}

int pg_reversal_workspace_size(const pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch,
                               size_t *bytes)
{
    if (!bytes)
        return PG_E_NULL;
    *bytes = 0;
    RevPlan R;
    int s = reversal_plan(ctx, desc, batch, nullptr, nullptr, R);
    if (s != PG_OK)
        return s;
    *bytes = R.ws;
    return PG_OK;
}

int pg_reversal_step(pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch,
                     const float *target, float *residual, float *loss, float *grad_xyz,
                     float *xyz_update, float lr, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx)
        return PG_E_NULL;
    if (ctx->device == PG_HOST_ONLY)
        return PG_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(ctx->mu);
    RevPlan R;
    int s = reversal_plan(ctx, desc, batch, residual, target, R);
    if (s != PG_OK)
        return s;
    if (!std::isfinite(lr))
        return PG_E_PARAM;
    // no residual grid: only where the window kernel forms the residual
    // itself (the adjoint then recomputes it at the window voxels)
    const bool keep_residual = residual != nullptr;
    if (batch->n_mol > 0 && (!target || !loss || (!keep_residual && (!R.fused || weighted(batch)))))
        return PG_E_NULL;
    if (ws_bytes < R.ws || (R.ws > 0 && !ws))
        return PG_E_WORKSPACE;
    if (batch->n_mol == 0)
        return PG_OK;
    DeviceGuard g(ctx->device);
    GridParams p;
    fill_params(p, ctx, desc, batch, R.P, residual, ws);
    float2 *partial = (float2 *)((unsigned char *)ws + R.partial_off);
    auto launch = [&](hipStream_t st) -> hipError_t {
        GridParams q = p;
        if (R.fused) {
            q.target = target;
            q.loss = loss;
        }
        hipError_t e = launch_forward(ctx, desc, R.P, q, st);
        if (e != hipSuccess)
            return e;
        if (!R.fused) {
            q = p;
            q.target = target;
            q.loss = loss;
            e = launch_residual(q, partial, st);
            if (e != hipSuccess)
                return e;
        }
        if (batch->n_atoms > 0 && (grad_xyz || xyz_update)) {
            q = p;
            q.grad_xyz = grad_xyz;
            q.xyz_upd = xyz_update;
            q.lr = lr;
            if (!keep_residual) {
                q.target = target;
                q.recompute = 1;
                q.rec_ntw = window_index_bound(q);
            }
            e = launch_adjoint(q, PG_OUT_F32, st);
        }
        return e;
    };
    std::string key;
    if (ctx->use_graph) {
        key = graph_key(desc, batch, R.P, residual, ws, ws_bytes);
        const void *ptrs[] = {target, loss, grad_xyz, xyz_update};
        key.append("reversal");
        key.append((const char *)ptrs, sizeof ptrs);
        key.append((const char *)&lr, sizeof lr);
    }
    return run_launches(ctx, ctx->use_graph != 0, key, (hipStream_t)stream, launch);
}

int pg_autotune(pg_ctx *ctx, const pg_grid_desc *desc, const pg_batch *batch, void *out, void *ws,
                size_t ws_bytes, void *stream, int reps)
{
    if (!ctx)
        return PG_E_NULL;
    if (ctx->device == PG_HOST_ONLY)
        return PG_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(ctx->mu);
    Plan base;
    int s = make_plan(ctx, desc, batch, out, base);
    if (s != PG_OK)
        return s;
    if (batch->n_mol == 0 || base.form == PG_FORM_PLAIN)
        return PG_OK;   // nothing tunable for this request
    if (base.crystal && desc->form != PG_FORM_AUTO)
        return PG_OK;   // a single admissible large-structure form
    if (reps < 1)
        reps = 1;
    const char *venv = std::getenv("PG_AUTOTUNE_VERBOSE");
    const bool verbose = venv && venv[0] == '1';
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return PG_E_HIP;
    auto time_plan = [&](const Plan &P, double &us) -> hipError_t {
        GridParams p;
        fill_params(p, ctx, desc, batch, P, out, ws);
        hipError_t e = hipSuccess;
        for (int w = 0; w < 2 && e == hipSuccess; ++w)
            e = launch_forward(ctx, desc, P, p, st);
        if (e == hipSuccess)
            e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
            e = launch_forward(ctx, desc, P, p, st);
        if (e == hipSuccess)
            e = hipEventRecord(e1, st);
        if (e == hipSuccess)
            e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, e0, e1);
        us = 1000.0 * ms / reps;
        return e;
    };
    if (base.crystal) {
        // large structures: measure both binned forms
        int best_form = 0;
        double best_us = 1e30;
        int rc = PG_OK;
        for (int f : {PG_FORM_MFMA, PG_FORM_WINDOW}) {
            Plan P;
            P.vec = base.vec;
            if (crystal_plan(ctx, desc, batch, f, P) != PG_OK || ws_bytes < P.ws || !ws)
                continue;
            double us = 0;
            hipError_t e = time_plan(P, us);
            if (e != hipSuccess) {
                rc = hip_fail(ctx, e);
                break;
            }
            if (verbose)
                std::fprintf(stderr, "pg_autotune %s form %d: %.2f us\n",
                             tuning_key(desc, batch, base.vec).c_str(), f, us);
            if (us < best_us) {
                best_us = us;
                best_form = f;
            }
        }
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        if (rc == PG_OK && best_form > 0) {
            Tuned &t = ctx->tuning[tuning_key(desc, batch, base.vec)];
            t.form = best_form;
            t.us = best_us;
            if (t.block == 0) {
                t.block = 256;
                t.per_cu = 1;
                t.nt = 0;
                t.unroll = 1;
            }
            drop_graphs(ctx);
        }
        return rc;
    }
    Tuned best;
    best.us = 1e30;
    int rc = PG_OK;
    // candidates: workgroup size, resident workgroups per CU (up to one
    // workgroup per structure), runs per lane per pass, store mode
    std::vector<int> pcs;
    const int per_cu_all = (batch->n_mol + ctx->n_cu - 1) / ctx->n_cu;
    for (int v = 1; v <= 64; v *= 2) {
        if (v >= per_cu_all) {
            pcs.push_back(std::max(1, per_cu_all));
            break;
        }
        pcs.push_back(v);
    }
    for (int blk : {256, 512, 1024})
        for (int pc : pcs)
            for (int un : {1, 2, 4})
                for (int nt : {0, 1}) {
                    if (rc != PG_OK)
                        break;
                    Plan P = base;
                    P.block = blk;
                    P.per_cu = pc;
                    P.unroll = un;
                    P.nt = nt;
                    P.grid = window_grid(batch, P, ctx->n_cu);
                    double us = 0;
                    hipError_t e = time_plan(P, us);
                    if (e != hipSuccess) {
                        rc = hip_fail(ctx, e);
                        break;
                    }
                    if (verbose)
                        std::fprintf(stderr,
                                     "pg_autotune %s block %d per_cu %d grid %d unroll %d nt %d: %.2f us\n",
                                     tuning_key(desc, batch, base.vec).c_str(), blk, pc, P.grid, un,
                                     nt, us);
                    if (us < best.us) {
                        best.us = us;
                        best.block = blk;
                        best.per_cu = pc;
                        best.nt = nt;
                        best.unroll = un;
                    }
                }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc == PG_OK && best.block > 0) {
        ctx->tuning[tuning_key(desc, batch, base.vec)] = best;
        drop_graphs(ctx);
    }
    return rc;
}

int pg_tuning_save(const pg_ctx *ctx, const char *path)
{
    if (!ctx || !path)
        return PG_E_NULL;
    std::ofstream f(path);
    if (!f)
        return PG_E_PARAM;
    f << "{\"version\": 1, \"arch\": \"" << ctx->arch << "\", \"entries\": [";
    bool first = true;
    for (const auto &kv : ctx->tuning) {
        f << (first ? "\n" : ",\n") << "  {\"key\": \"" << kv.first << "\", \"block\": "
          << kv.second.block << ", \"per_cu\": " << kv.second.per_cu << ", \"unroll\": "
          << kv.second.unroll << ", \"nt\": " << kv.second.nt << ", \"form\": " << kv.second.form
          << ", \"us\": " << kv.second.us << "}";
        first = false;
    }
    f << "\n]}\n";
    return f.good() ? PG_OK : PG_E_PARAM;
}

int pg_tuning_load(pg_ctx *ctx, const char *path)
{
    if (!ctx || !path)
        return PG_E_NULL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tuning.clear();
    drop_graphs(ctx);
    std::ifstream f(path);
    if (!f)
        return PG_E_PARAM;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string txt = ss.str();
    if (txt.find("\"version\": 1") == std::string::npos)
        return PG_E_PARAM;
    std::map<std::string, Tuned> tab;
    size_t pos = 0;
    auto field = [](const std::string &obj, const char *name, double &v) {
        const std::string k = std::string("\"") + name + "\": ";
        const size_t at = obj.find(k);
        if (at == std::string::npos)
            return false;
        return std::sscanf(obj.c_str() + at + k.size(), "%lf", &v) == 1;
    };
    while ((pos = txt.find("{\"key\": \"", pos)) != std::string::npos) {
        pos += 9;
        const size_t q = txt.find('"', pos);
        const size_t end = txt.find('}', pos);
        if (q == std::string::npos || end == std::string::npos || end < q)
            return PG_E_PARAM;
        const std::string key = txt.substr(pos, q - pos);
        const std::string obj = txt.substr(q, end - q);
        double blk, pc, un, nt, us, form = 0;
        if (!field(obj, "block", blk) || !field(obj, "per_cu", pc) || !field(obj, "unroll", un) ||
            !field(obj, "nt", nt) || !field(obj, "us", us))
            return PG_E_PARAM;
        field(obj, "form", form);
        Tuned t;
        t.block = (int)blk;
        t.per_cu = (int)pc;
        t.unroll = (int)un;
        t.nt = (int)nt;
        t.us = us;
        t.form = (int)form;
        if (t.block < 64 || t.block > 1024 || t.block % 64 || t.nt < 0 || t.nt > 1 ||
            (t.unroll != 1 && t.unroll != 2 && t.unroll != 4) || t.per_cu < 1 || t.per_cu > 64 ||
            (t.form != 0 && t.form != PG_FORM_WINDOW && t.form != PG_FORM_MFMA))
            return PG_E_PARAM;
        tab[key] = t;
        pos = end;
    }
    ctx->tuning = std::move(tab);
    return PG_OK;
}

int pg_set_option(pg_ctx *ctx, int option, int64_t value)
{
    if (!ctx)
        return PG_E_NULL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    switch (option) {
    case PG_OPT_GRAPH:
        if (value != 0 && value != 1)
            return PG_E_PARAM;
        ctx->use_graph = (int)value;
        if (!value)
            drop_graphs(ctx);
        return PG_OK;
    case PG_OPT_BLOCK:
        if (value != -1 && (value < 64 || value > 1024 || value % 64))
            return PG_E_PARAM;
        ctx->opt_block = (int)value;
        break;
    case PG_OPT_NT_STORE:
        if (value < -1 || value > 1)
            return PG_E_PARAM;
        ctx->opt_nt = (int)value;
        break;
    case PG_OPT_GRID_PER_CU:
        if (value != -1 && (value < 1 || value > 64))
            return PG_E_PARAM;
        ctx->opt_per_cu = (int)value;
        break;
    case PG_OPT_UNROLL:
        if (value != -1 && value != 1 && value != 2 && value != 4)
            return PG_E_PARAM;
        ctx->opt_unroll = (int)value;
        break;
    default:
        return PG_E_PARAM;
    }
    drop_graphs(ctx);
    return PG_OK;
}

int pg_get_device_error(pg_ctx *ctx, int32_t *code, int64_t *first_atom)
{
    if (!ctx || !code || !first_atom)
        return PG_E_NULL;
    if (ctx->device == PG_HOST_ONLY)
        return PG_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    DeviceError h;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(&h, ctx->d_err, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_fail(ctx, e);
    DeviceError z = {0u, 0u, ~0ull};
    e = hipMemcpy(ctx->d_err, &z, sizeof z, hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return hip_fail(ctx, e);
    *code = PG_OK;
    if (h.flags & (1u << PG_E_DEVICE_DATA))
        *code = PG_E_DEVICE_DATA;
    else if (h.flags & (1u << PG_E_CAPACITY))
        *code = PG_E_CAPACITY;
    *first_atom = h.flags ? (int64_t)h.first : -1;
    return PG_OK;
}

int pg_last_hip_error(const pg_ctx *ctx) { return ctx ? ctx->last_hip : 0; }

}  // extern "C"
