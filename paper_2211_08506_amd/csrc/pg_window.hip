// pg_window.hip -- persistent cutoff-window kernel for ragged molecule batches
// (gfx950).
//
// One workgroup owns one structure at a time (persistent grid, structures
// strided by gridDim.x).  For its structure it
//   1. computes every atom's exact per-axis window ranges (one thread per
//      atom and axis) -- the per-axis search of §VI-B, done exactly;
//   2. fills dense 1-D factor rows phi_x[W] | phi_y[H] | phi_z[D] per atom in
//      LDS (zeros outside the window; the separable tables of §VI-A) and,
//      per (channel, z) plane, a bit mask of the atoms whose z-window
//      contains that plane;
//   3. streams the structure's C x D x H x W output plane by plane: each
//      wave takes whole (c, z) planes, each lane a run of VEC consecutive x
//      (16 bytes), accumulates sum_a phi_z[a][z] phi_y[a][y] phi_x[a][x..]
//      over the plane's mask in FP32 registers (only atoms of that channel
//      whose z-window holds the plane), and writes the run once -- zeros
//      included -- with one 16-byte (optionally non-temporal) store, so a
//      wave's store instruction covers 1 KiB of contiguous output.
// Every output element is written exactly once and no atomics touch the
// output, so the result is bitwise reproducible for any launch shape; the
// per-voxel sum runs over atoms in index order.
#include "pg_device.hpp"
#include "pg_launch.hpp"

namespace pg {

struct RangeRec {
    int32_t n;
    int16_t lo[MAX_IMAGES], hi[MAX_IMAGES];
    float bh[MAX_IMAGES], bl[MAX_IMAGES];
};

__host__ __device__ inline WindowLds window_lds_layout(int a_cap, int row_stride, int C, int D,
                                                      int mask_words)
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
    L.total = (off + 15) & ~(size_t)15;
    return L;
}

WindowLds window_lds(int a_cap, int row_stride, int C, int D, int mask_words)
{
    return window_lds_layout(a_cap, row_stride, C, D, mask_words);
}

__device__ __forceinline__ unsigned long long uniform64(unsigned long long v)
{
    unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(v & 0xffffffffu));
    unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
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

template <typename T, int VEC>
__global__ void __launch_bounds__(1024) window_mol_kernel(GridParams p)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int C = p.C, D = p.D, H = p.H, W = p.W;
    const int RS = p.row_stride;
    const int W4 = (W + 3) & ~3;
    const int MW = p.mask_words;
    const WindowLds lay = window_lds_layout(p.a_cap, RS, C, D, MW);
    float *rows = (float *)(smem + lay.rows);
    RangeRec *rr = (RangeRec *)(smem + lay.ranges);
    unsigned long long *masks = (unsigned long long *)(smem + lay.masks);
    int32_t *atype = (int32_t *)(smem + lay.types);

    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
    const int planes = C * D;
    const size_t plane_elems = (size_t)H * W;
    const size_t mol_elems = (size_t)planes * plane_elems;
    const int chunks = (int)(plane_elems / VEC);
    const bool nt = p.nt_store != 0;
    // per-lane run position inside a plane, and its step per 64 runs
    const int step = 64 * VEC;
    const int dy = step / W, dx = step - dy * W;
    const int y_init = (lane * VEC) / W, x_init = lane * VEC - y_init * W;

    for (int m = blockIdx.x; m < p.n_mol; m += gridDim.x) {
        const int a0 = p.offsets[m];
        const int na = p.offsets[m + 1] - a0;
        T *out = (T *)p.out + (size_t)m * mol_elems;

        if (na > p.a_cap || na < 0 || a0 < 0 || (long long)a0 + na > p.n_atoms) {
            // structure larger than declared (or offsets out of range):
            // zeros, and a sticky error
            if (tid == 0)
                raise_error(p.err, na > p.a_cap ? PG_E_CAPACITY : PG_E_DEVICE_DATA, m);
            const float z[VEC] = {};
            for (size_t j = tid; j < mol_elems / VEC; j += nthr)
                store_vec<T, VEC>(out + j * VEC, z, nt);
            continue;
        }
        float o[3], h[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            o[q] = p.origins ? p.origins[3 * m + q] : p.o[q];
            h[q] = p.spacings ? p.spacings[3 * m + q] : p.h[q];
        }

        // ---- 1. window ranges per (atom, axis); clear plane masks
        for (int i = tid; i < planes * MW; i += nthr)
            masks[i] = 0ull;
        for (int i = tid; i < na * 3; i += nthr) {
            const int a = i / 3, ax = i - 3 * a;
            const float x = p.xyz[3 * (size_t)(a0 + a) + 0];
            const float y = p.xyz[3 * (size_t)(a0 + a) + 1];
            const float zc = p.xyz[3 * (size_t)(a0 + a) + 2];
            const int t = p.types[a0 + a];
            const bool ok = atom_valid(x, y, zc, t, C);
            RangeRec R;
            R.n = 0;
            if (ok) {
                const float mu = ax == 0 ? x : (ax == 1 ? y : zc);
                const int N = ax == 0 ? W : (ax == 1 ? H : D);
                AxisRanges ar;
                axis_ranges(o[ax], h[ax], N, mu, p.periodic != 0, p.L[ax], p.rc[t], p.cut != 0, ar);
                R.n = ar.n;
#pragma unroll
                for (int r = 0; r < MAX_IMAGES; ++r) {
                    R.lo[r] = (int16_t)(r < ar.n ? ar.lo[r] : 0);
                    R.hi[r] = (int16_t)(r < ar.n ? ar.hi[r] : -1);
                    R.bh[r] = r < ar.n ? ar.bh[r] : 0.f;
                    R.bl[r] = r < ar.n ? ar.bl[r] : 0.f;
                }
            }
            rr[i] = R;
            if (ax == 0) {
                atype[a] = ok ? t : -1;
                if (!ok)
                    raise_error(p.err, PG_E_DEVICE_DATA, (long long)(a0 + a));
            }
        }
        __syncthreads();

        // ---- 2. dense 1-D factor rows and (channel, z) atom masks
        for (int e = tid; e < na * RS; e += nthr) {
            const int a = e / RS, j = e - a * RS;
            int ax, i, N;
            if (j < W4) {
                ax = 0; i = j; N = W;
            } else if (j < W4 + H) {
                ax = 1; i = j - W4; N = H;
            } else {
                ax = 2; i = j - W4 - H; N = D;
            }
            const int t = atype[a];
            float v = 0.f;
            if (t >= 0 && i < N) {
                const RangeRec &R = rr[3 * a + ax];
                for (int r = 0; r < R.n; ++r) {
                    if (i >= R.lo[r] && i <= R.hi[r]) {
                        v = gauss1d(offset_at(R.bh[r], R.bl[r], h[ax], i), p.inv2s2[t]);
                        if (ax == 2)
                            atomicOr(&masks[(size_t)(t * D + i) * MW + (a >> 6)], 1ull << (a & 63));
                    }
                }
            }
            rows[e] = v;
        }
        __syncthreads();

        // ---- 3. stream the planes
        for (int pl = wave; pl < planes; pl += nwaves) {
            const int z = pl % D;
            unsigned long long mk[4];
#pragma unroll
            for (int w = 0; w < 4; ++w)
                mk[w] = (w < MW) ? uniform64(masks[(size_t)pl * MW + w]) : 0ull;
            T *op = out + (size_t)pl * plane_elems;
            int y = y_init, x0 = x_init;
            for (int j = lane; j < chunks; j += 64) {
                float acc[VEC];
#pragma unroll
                for (int k = 0; k < VEC; ++k)
                    acc[k] = 0.f;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    unsigned long long bits = mk[w];
                    while (bits) {
                        const int a = w * 64 + __builtin_ctzll(bits);
                        bits &= bits - 1;
                        const float *row = rows + a * RS;
                        const float gz = row[W4 + H + z];
                        const float gy = row[W4 + y] * gz;
                        float fx[VEC];
                        load_row<VEC>(row + x0, fx);
#pragma unroll
                        for (int k = 0; k < VEC; ++k)
                            acc[k] = __builtin_fmaf(gy, fx[k], acc[k]);
                    }
                }
                store_vec<T, VEC>(op + (size_t)j * VEC, acc, nt);
                x0 += dx;
                y += dy;
                if (x0 >= W) {
                    x0 -= W;
                    ++y;
                }
            }
        }
        __syncthreads();
    }
}

template <typename T, int VEC>
static hipError_t launch_window_t(const GridParams &p, int block, int grid, size_t lds, hipStream_t s)
{
    auto kern = window_mol_kernel<T, VEC>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, p);
    return hipGetLastError();
}

hipError_t launch_window(const GridParams &p, int out_dtype, int vec, int block, int grid,
                         size_t lds, hipStream_t s)
{
    if (out_dtype == PG_OUT_F32) {
        switch (vec) {
        case 4: return launch_window_t<float, 4>(p, block, grid, lds, s);
        case 2: return launch_window_t<float, 2>(p, block, grid, lds, s);
        case 1: return launch_window_t<float, 1>(p, block, grid, lds, s);
        }
    } else {
        switch (vec) {
        case 8: return launch_window_t<__bf16, 8>(p, block, grid, lds, s);
        case 4: return launch_window_t<__bf16, 4>(p, block, grid, lds, s);
        case 2: return launch_window_t<__bf16, 2>(p, block, grid, lds, s);
        case 1: return launch_window_t<__bf16, 1>(p, block, grid, lds, s);
        }
    }
    return hipErrorInvalidValue;
}

int window_occupancy(int out_dtype, int vec, int block, size_t lds)
{
    int n = 0;
    const void *k = nullptr;
    if (out_dtype == PG_OUT_F32)
        k = vec == 4 ? (const void *)window_mol_kernel<float, 4>
                     : vec == 2 ? (const void *)window_mol_kernel<float, 2>
                                : (const void *)window_mol_kernel<float, 1>;
    else
        k = vec == 8 ? (const void *)window_mol_kernel<__bf16, 8>
                     : vec == 4 ? (const void *)window_mol_kernel<__bf16, 4>
                                : vec == 2 ? (const void *)window_mol_kernel<__bf16, 2>
                                           : (const void *)window_mol_kernel<__bf16, 1>;
    if (lds > 65536)
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, block, lds) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace pg
