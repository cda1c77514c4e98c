// pg_window.hip -- persistent cutoff-window kernel for ragged batches of
// molecules (gfx950).
//
// One workgroup owns one structure at a time (persistent grid, structures
// strided by gridDim.x).  For its structure it
//   1. computes every atom's exact per-axis window ranges (one thread per
//      atom and axis) -- the per-axis search of §VI-B, done exactly;
//   2. fills dense 1-D factor rows phi_x[W] | phi_y[H] | phi_z[D] per atom in
//      LDS (zeros outside the window; the separable per-axis tables of
//      §VI-A) and, per (channel, z) plane, a bit mask of the atoms of that
//      channel whose z-window contains the plane (with weighted channels:
//      of the atoms with a non-zero weight for the channel, the weights
//      being staged in LDS too and folded into phi_z);
//   3. streams the structure's C x D x H x W output: each wave takes whole
//      (c, z) planes, pass by pass (a pass: U runs of VEC consecutive x, 16
//      bytes each, per lane; its run indices serve all the wave's planes),
//      accumulates sum_a phi_z[a][z] phi_y[a][y] phi_x[a][x..]
//      over the plane's mask in FP32 registers and writes each run once --
//      zeros included -- with a 16-byte store, so one store instruction of a
//      wave covers 1 KiB of contiguous output.
// Steps 1-2 run once per structure out of LDS-resident data, so the store
// stream of step 3 needs no global loads.  In the residual mode of a grid
// reversal step (§IV-A, §IV-C) step 3 also reads the target run, writes
// 2 (G - target) in place of G and sums (G - target)^2 per structure
// (per-lane FP32 partial sums, float-float sums across the workgroup).
// Every output element is written exactly once, with no atomics on the
// output; each voxel's sum runs over
// atoms in index order, so results are bitwise reproducible for every
// launch shape.
#include "pg_device.hpp"
#include "pg_launch.hpp"

namespace pg {

__host__ __device__ inline WindowLds window_lds_layout(int a_cap, int row_stride, int C, int D,
                                                      int mask_words, int weight_ch, bool sphere)
{
    WindowLds L;
    size_t off = 0;
    L.rows = off;
    off += (size_t)a_cap * row_stride * sizeof(float);
    off = (off + 15) & ~(size_t)15;
    L.ranges = off;
    off += (size_t)a_cap * 3 * sizeof(RangeRec);
    off = (off + 15) & ~(size_t)15;
    L.masks = off;
    off += (size_t)C * D * mask_words * sizeof(unsigned long long);
    L.types = off;
    off += (size_t)a_cap * sizeof(int32_t);
    L.wts = off;
    off += (size_t)a_cap * weight_ch * sizeof(float);
    off = (off + 15) & ~(size_t)15;
    L.dsq = off;
    if (sphere)
        off += (size_t)a_cap * row_stride * sizeof(float);
    L.total = (off + 15) & ~(size_t)15;
    return L;
}

WindowLds window_lds(int a_cap, int row_stride, int C, int D, int mask_words, int weight_ch,
                     bool sphere)
{
    return window_lds_layout(a_cap, row_stride, C, D, mask_words, weight_ch, sphere);
}

__device__ __forceinline__ unsigned long long uniform64(unsigned long long v)
{
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(v & 0xffffffffu));
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

template <int VEC>
__device__ __forceinline__ void load_row(const float *r, float (&v)[VEC])
{
    if constexpr (VEC == 8) {
        float4 a = *(const float4 *)r, b = *(const float4 *)(r + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else if constexpr (VEC == 4) {
        float4 a = *(const float4 *)r;
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    } else if constexpr (VEC == 2) {
        float2 a = *(const float2 *)r;
        v[0] = a.x; v[1] = a.y;
    } else {
        v[0] = r[0];
    }
}

// One structure's LDS-resident state (steps 1-2).
struct MolBuf {
    float *rows;                  // factor rows phi_x | phi_y | phi_z per atom
    RangeRec *rr;                 // window ranges per (atom, axis)
    unsigned long long *masks;    // per (channel, z) plane: atoms with a factor there
    int32_t *atype;               // type per atom, -1 for an invalid atom
    float *wl;                    // per-atom channel weights (weighted channels)
    float *dsq;                   // sphere: squared centre offsets beside the rows
};

__device__ __forceinline__ MolBuf mol_buf(unsigned char *base, const WindowLds &lay)
{
    MolBuf B;
    B.rows = (float *)(base + lay.rows);
    B.rr = (RangeRec *)(base + lay.ranges);
    B.masks = (unsigned long long *)(base + lay.masks);
    B.atype = (int32_t *)(base + lay.types);
    B.wl = (float *)(base + lay.wts);
    B.dsq = (float *)(base + lay.dsq);
    return B;
}

// Steps 1-2 for structure m into B, run by the workgroup's threads
// t = 0 .. n-1; the caller synchronises before the state is read.
template <bool SPH>
__device__ void mol_setup(const GridParams &p, const MolBuf &B, int m, int t, int n)
{
    const int C = p.C, D = p.D, H = p.H, W = p.W;
    const int RS = p.row_stride;
    const int W4 = (W + 3) & ~3;
    const int MW = p.mask_words;
    const int WC = p.weights ? C : 0;
    const int planes = C * D;
    const int a0 = p.offsets[m];
    int na = p.offsets[m + 1] - a0;
    if (na > p.a_cap || na < 0 || a0 < 0 || (long long)a0 + na > p.n_atoms) {
        // more atoms than the declared capacity (or bad offsets): no atoms,
        // so the structure's grid is written as zeros; sticky error
        if (t == 0)
            raise_error(p.err, na > p.a_cap ? PG_E_CAPACITY : PG_E_DEVICE_DATA, m);
        na = 0;
    }
    float o[3], h[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        o[q] = p.origins ? p.origins[3 * (size_t)m + q] : p.o[q];
        h[q] = p.spacings ? p.spacings[3 * (size_t)m + q] : p.h[q];
    }

    // ---- 1. window ranges per (atom, axis); clear plane masks and rows
    for (int i = t; i < planes * MW; i += n)
        B.masks[i] = 0ull;
    for (int i = t; i < na * RS; i += n) {
        B.rows[i] = 0.f;
        if constexpr (SPH)
            B.dsq[i] = __builtin_huge_valf();
    }
    for (int i = t; i < na * WC; i += n)
        B.wl[i] = p.weights[(size_t)a0 * C + i];
    for (int i = t; i < na * 3; i += n) {
        const int a = i / 3, ax = i - 3 * a;
        const size_t ga = (size_t)a0 + a;
        const float x = p.xyz[3 * ga + 0], y = p.xyz[3 * ga + 1], zc = p.xyz[3 * ga + 2];
        const int ty = p.types[ga];
        const bool ok = atom_valid(x, y, zc, ty, p.n_sig);
        RangeRec R;
        R.n = 0;
        if (ok) {
            const float mu = ax == 0 ? x : (ax == 1 ? y : zc);
            const int N = ax == 0 ? W : (ax == 1 ? H : D);
            const float oq = ax == 0 ? o[0] : (ax == 1 ? o[1] : o[2]);
            const float hq = ax == 0 ? h[0] : (ax == 1 ? h[1] : h[2]);
            const float Lq = ax == 0 ? p.L[0] : (ax == 1 ? p.L[1] : p.L[2]);
            AxisRanges ar;
            axis_ranges(oq, hq, N, mu, p.periodic != 0, Lq, p.rc[ty], p.cut != 0, ar);
            R.n = ar.n;
#pragma unroll
            for (int r = 0; r < MAX_IMAGES; ++r) {
                R.lo[r] = (int16_t)(r < ar.n ? ar.lo[r] : 0);
                R.hi[r] = (int16_t)(r < ar.n ? ar.hi[r] : -1);
                R.bh[r] = r < ar.n ? ar.bh[r] : 0.f;
                R.bl[r] = r < ar.n ? ar.bl[r] : 0.f;
            }
        }
        B.rr[i] = R;
        if (ax == 0) {
            B.atype[a] = ok ? ty : -1;
            if (!ok)
                raise_error(p.err, PG_E_DEVICE_DATA, (long long)ga);
        }
    }
    __syncthreads();

    // ---- 2. the 1-D factor rows inside the windows (zero elsewhere), eight
    // consecutive voxels of one atom and axis per item (the box form walks
    // their edges once), and the (channel, z) atom masks
    const int nx = (W + 7) >> 3, ny = (H + 7) >> 3, nz = (D + 7) >> 3, nc = nx + ny + nz;
    for (int it = t; it < na * nc; it += n) {
        const int a = it / nc;
        int c = it - a * nc, ax, N, base;
        float hq;
        if (c < nx) {
            ax = 0; N = W; base = 0; hq = h[0];
        } else if (c < nx + ny) {
            ax = 1; c -= nx; N = H; base = W4; hq = h[1];
        } else {
            ax = 2; c -= nx + ny; N = D; base = W4 + H; hq = h[2];
        }
        const int ty = B.atype[a];
        if (ty < 0)
            continue;
        const RangeRec &R = B.rr[3 * a + ax];
        const int v0 = 8 * c, v1 = min(v0 + 7, N - 1);
        float *row = B.rows + a * RS + base;
        for (int r = 0; r < R.n; ++r) {
            const int lo = max((int)R.lo[r], v0), hi = min((int)R.hi[r], v1);
            if (lo > hi)
                continue;
            const float bh = R.bh[r], bl = R.bl[r];
            if (p.box != 0) {
                box_walk<false>(bh, bl, hq, lo, hi, p.isq2s[ty], 1.f, row);
            } else {
                for (int i = lo; i <= hi; ++i)
                    row[i] = gauss1d(offset_at(bh, bl, hq, i), p.inv2s2[ty]);
            }
            for (int i = lo; i <= hi; ++i) {
                if constexpr (SPH) {
                    const float d = offset_at(bh, bl, hq, i);
                    B.dsq[a * RS + base + i] = d * d;
                }
                if (ax == 2) {
                    if (WC == 0) {
                        atomicOr(&B.masks[(size_t)(ty * D + i) * MW + (a >> 6)], 1ull << (a & 63));
                    } else {
                        for (int ch = 0; ch < C; ++ch)
                            if (B.wl[a * WC + ch] != 0.f)
                                atomicOr(&B.masks[(size_t)(ch * D + i) * MW + (a >> 6)],
                                         1ull << (a & 63));
                    }
                }
            }
        }
    }
}

// Plane geometry of step 3.
struct PlaneGeom {
    int D, H, W, RS, W4, MW, WC, CW, chunks;
    float inv_cw;
    size_t plane_elems;
    bool nt;
};

template <int VEC>
__device__ __forceinline__ PlaneGeom plane_geom(const GridParams &p)
{
    PlaneGeom g;
    g.D = p.D;
    g.H = p.H;
    g.W = p.W;
    g.RS = p.row_stride;
    g.W4 = (p.W + 3) & ~3;
    g.MW = p.mask_words;
    g.WC = p.weights ? p.C : 0;
    g.plane_elems = (size_t)p.H * p.W;
    g.chunks = (int)(g.plane_elems / VEC);
    g.nt = p.nt_store != 0;
    // runs (VEC consecutive x) per row.  A run's row is floor(j / CW); the
    // float estimate (j + 1/2) / CW is within one row of it for every plane
    // the validation admits (fewer than 2^15 rows: three roundings of
    // relative size 2^-24 move a value below 2^15 by less than 2^-8), and
    // one integer comparison on each side makes it exact.
    g.CW = p.W / VEC;
    g.inv_cw = 1.0f / (float)g.CW;
    return g;
}

// The lane's U runs j0 + 64 u of one pass over a plane: row, first column,
// and whether the run exists.  The same for every plane, so computed once
// per pass and structure.
template <int U>
struct PassRuns {
    int yq[U], xq[U];
    bool ok[U];
};

template <int VEC, int U>
__device__ __forceinline__ PassRuns<U> pass_runs(const PlaneGeom &g, int j0)
{
    PassRuns<U> R;
    const int CW = g.CW;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = j0 + 64 * u;
        R.ok[u] = j < g.chunks;
        // run j starts at element j*VEC: row j / CW, column (j % CW) * VEC
        int yy = (int)(((float)j + 0.5f) * g.inv_cw);
        yy -= yy * CW > j ? 1 : 0;
        yy += (yy + 1) * CW <= j ? 1 : 0;
        R.yq[u] = R.ok[u] ? yy : 0;
        R.xq[u] = R.ok[u] ? (j - yy * CW) * VEC : 0;
    }
    return R;
}

// acc (+)= gy * phi_x over the runs of one atom; FIRST: the plane's first
// atom initialises the sums (a product, exactly what an FMA onto zero gives)
template <int VEC, int U, bool SPH, bool FIRST>
__device__ __forceinline__ void add_atom(const GridParams &p, const MolBuf &B, const PlaneGeom &g,
                                         int a, int z, int pc, const PassRuns<U> &R,
                                         float (&acc)[U][VEC])
{
    const float *row = B.rows + a * g.RS;
    float gz = row[g.W4 + g.H + z];
    if (g.WC)
        gz *= B.wl[a * g.WC + pc];
    float r2z = 0.f;
    if constexpr (SPH)
        r2z = p.rc2[B.atype[a]] - B.dsq[a * g.RS + g.W4 + g.H + z];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const float gy = row[g.W4 + R.yq[u]] * gz;
        float fx[VEC];
        load_row<VEC>(row + R.xq[u], fx);
        if constexpr (SPH) {
            // keep x only inside the ball: dx^2 <= rc^2 - dz^2 - dy^2
            const float r2 = r2z - B.dsq[a * g.RS + g.W4 + R.yq[u]];
            float dx2[VEC];
            load_row<VEC>(B.dsq + a * g.RS + R.xq[u], dx2);
#pragma unroll
            for (int k = 0; k < VEC; ++k)
                fx[k] = dx2[k] <= r2 ? fx[k] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < VEC; ++k)
            acc[u][k] = FIRST ? gy * fx[k] : __builtin_fmaf(gy, fx[k], acc[u][k]);
    }
}

// ---- 3. one wave writes one pass (the lane's U runs R, starting at run j0)
// of plane pl = (channel, z): sum_a phi_z[a][z] phi_y[a][y] phi_x[a][x..]
// over the plane's mask in index order, U back-to-back 16-byte stores per
// lane.  out / tgt: the structure's grid and target (or null); sq: the
// lane's running sum of squared residuals (residual mode).
template <typename T, int VEC, int U, bool RES, bool SPH>
__device__ __forceinline__ void stream_pass(const GridParams &p, const MolBuf &B,
                                            const PlaneGeom &g, int pl, int j0,
                                            const PassRuns<U> &R, T *out, const float *tgt,
                                            float &sq)
{
    const int z = pl % g.D;
    const int pc = pl / g.D;
    unsigned long long mk[4];
#pragma unroll
    for (int w = 0; w < 4; ++w)
        mk[w] = (w < g.MW) ? uniform64(B.masks[(size_t)pl * g.MW + w]) : 0ull;
    // residual mode: the target runs are loaded before the accumulation, so
    // their latency overlaps it
    float tv[RES ? U : 1][VEC];
    if constexpr (RES) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (R.ok[u])
                load_row<VEC>(tgt + (size_t)pl * g.plane_elems + (size_t)(j0 + 64 * u) * VEC, tv[u]);
            else
#pragma unroll
                for (int k = 0; k < VEC; ++k)
                    tv[u][k] = 0.f;
        }
    }
    // the first atom of the plane (in index order), taken out of its word
    int a0 = -1;
#pragma unroll
    for (int w = 0; w < 4; ++w)
        if (a0 < 0 && mk[w]) {
            a0 = w * 64 + __builtin_ctzll(mk[w]);
            mk[w] &= mk[w] - 1;
        }
    float acc[U][VEC];
    if (a0 >= 0) {
        add_atom<VEC, U, SPH, true>(p, B, g, a0, z, pc, R, acc);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            unsigned long long bits = mk[w];
            while (bits) {
                const int a = w * 64 + __builtin_ctzll(bits);
                bits &= bits - 1;
                add_atom<VEC, U, SPH, false>(p, B, g, a, z, pc, R, acc);
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < VEC; ++k)
                acc[u][k] = 0.f;
    }
    T *op = out ? out + (size_t)pl * g.plane_elems : nullptr;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (R.ok[u]) {
            if constexpr (RES) {
#pragma unroll
                for (int k = 0; k < VEC; ++k) {
                    const float r = acc[u][k] - tv[u][k];
                    sq = __builtin_fmaf(r, r, sq);
                    acc[u][k] = 2.f * r;
                }
            }
            if (!RES || op)
                store_vec<T, VEC>(op + (size_t)(j0 + 64 * u) * VEC, acc[u], g.nt);
        }
}

// Set-up, then stream, structure by structure.  Each wave takes the planes
// pl = wave (mod waves) pass by pass (the run indices of a pass serve all
// of its planes); the fixed assignment keeps the residual mode's
// per-structure sums in a fixed order.
template <typename T, int VEC, int U, bool RES, bool SPH>
__global__ void __launch_bounds__(1024) window_mol_kernel(GridParams p)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const WindowLds lay = window_lds_layout(p.a_cap, p.row_stride, p.C, p.D, p.mask_words,
                                            p.weights ? p.C : 0, SPH);
    const MolBuf B = mol_buf(smem, lay);
    const PlaneGeom g = plane_geom<VEC>(p);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, nwaves = nthr >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int planes = p.C * p.D;
    const size_t mol_elems = (size_t)planes * g.plane_elems;

    for (int m = blockIdx.x; m < p.n_mol; m += gridDim.x) {
        mol_setup<SPH>(p, B, m, tid, nthr);
        __syncthreads();
        // a reversal step may keep no residual grid (out == nullptr)
        T *out = p.out ? (T *)p.out + (size_t)m * mol_elems : nullptr;
        const float *tgt = RES ? p.target + (size_t)m * mol_elems : nullptr;
        float sq = 0.f;
        for (int j0 = lane; j0 < g.chunks; j0 += 64 * U) {
            const PassRuns<U> R = pass_runs<VEC, U>(g, j0);
            for (int pl = wave; pl < planes; pl += nwaves)
                stream_pass<T, VEC, U, RES, SPH>(p, B, g, pl, j0, R, out, tgt, sq);
        }
        if constexpr (RES) {
            // per-lane FP32 partial sums, combined as float-float sums (a
            // wave butterfly, then the waves in order): no FP64 on the GPU
            __shared__ float red[2][16];
            float dh, dl;
            ff_wave_sum(sq, dh, dl);
            if (lane == 0) {
                red[0][wave] = dh;
                red[1][wave] = dl;
            }
            __syncthreads();
            if (tid == 0) {
                float ah = 0.f, alo = 0.f;
                for (int w = 0; w < nwaves; ++w)
                    ff_add(ah, alo, red[0][w], red[1][w]);
                p.loss[m] = ah + alo;
            }
        }
        __syncthreads();
    }
}

template <typename T, int VEC, int U, bool RES, bool SPH = false>
static const void *window_fn()
{
    return (const void *)window_mol_kernel<T, VEC, U, RES, SPH>;
}

template <typename T, int VEC, bool RES = false>
static const void *window_fn_u(int unroll)
{
    switch (unroll) {
    case 1: return window_fn<T, VEC, 1, RES>();
    case 2: return window_fn<T, VEC, 2, RES>();
    case 4: return window_fn<T, VEC, 4, RES>();
    }
    return nullptr;
}

// sphere cutoff: one run per lane only (unroll 1)
template <bool RES>
static const void *window_fn_sphere(int out_dtype, int vec)
{
    if (out_dtype == PG_OUT_F32) {
        switch (vec) {
        case 4: return window_fn<float, 4, 1, RES, true>();
        case 2: return window_fn<float, 2, 1, RES, true>();
        case 1: return window_fn<float, 1, 1, RES, true>();
        }
    } else if (!RES) {
        switch (vec) {
        case 8: return window_fn<__bf16, 8, 1, false, true>();
        case 4: return window_fn<__bf16, 4, 1, false, true>();
        case 2: return window_fn<__bf16, 2, 1, false, true>();
        case 1: return window_fn<__bf16, 1, 1, false, true>();
        }
    }
    return nullptr;
}

static const void *window_kernel_fn(int out_dtype, int vec, int unroll, bool residual, bool sphere)
{
    if (sphere)
        return unroll == 1 ? (residual ? window_fn_sphere<true>(out_dtype, vec)
                                       : window_fn_sphere<false>(out_dtype, vec))
                           : nullptr;
    if (residual) {
        if (out_dtype != PG_OUT_F32)
            return nullptr;
        switch (vec) {
        case 4: return window_fn_u<float, 4, true>(unroll);
        case 2: return window_fn_u<float, 2, true>(unroll);
        case 1: return window_fn_u<float, 1, true>(unroll);
        }
        return nullptr;
    }
    if (out_dtype == PG_OUT_F32) {
        switch (vec) {
        case 4: return window_fn_u<float, 4>(unroll);
        case 2: return window_fn_u<float, 2>(unroll);
        case 1: return window_fn_u<float, 1>(unroll);
        }
    } else {
        switch (vec) {
        case 8: return window_fn_u<__bf16, 8>(unroll);
        case 4: return window_fn_u<__bf16, 4>(unroll);
        case 2: return window_fn_u<__bf16, 2>(unroll);
        case 1: return window_fn_u<__bf16, 1>(unroll);
        }
    }
    return nullptr;
}

hipError_t launch_window(const GridParams &p, int out_dtype, int vec, int unroll, int block,
                         int grid, size_t lds, hipStream_t s)
{
    const void *k = window_kernel_fn(out_dtype, vec, unroll, p.target != nullptr, p.sphere != 0);
    if (!k)
        return hipErrorInvalidValue;
    if (p.n_mol == 0)
        return hipSuccess;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    GridParams pc = p;
    void *args[] = {&pc};
    return hipLaunchKernel(k, dim3(grid), dim3(block), args, lds, s);
}

}  // namespace pg
