// pg_crystal.hip -- large / dense structures (periodic crystal cells) on gfx950.
//
// Structures with more atoms than the molecule window kernel stages in LDS
// take this path.  Set-up, all on the GPU:
//   prep:  one thread per atom: exact per-axis window ranges (nearest
//          periodic images included) into a per-atom record, and a count of
//          the atom in every (structure, channel, z) plane bin its z-window
//          covers;
//   scan:  exclusive prefix sum of the bin counts (one workgroup);
//   fill:  one thread per atom appends the atom index to each of its bins.
// Then one of two plane kernels, one workgroup per (structure, channel, z
// plane[, 128 x 128 super-tile]); each first sorts its bin by atom index so
// that every voxel's sum runs over atoms in index order (bitwise
// reproducible results whatever order the fill's atomics produced):
//   mfma:   the plane is a contraction over the bin's atoms of two factor
//           matrices (separability of the Gaussian and of the cube cutoff,
//           §III-A / §IV-C):  G[y][x] = sum_k A[y][k] B[k][x] with
//           A[y][k] = phi_z^k(z) phi_y^k(y) built in FP32 and rounded once
//           to bf16, B[k][x] = phi_x^k(x) in bf16; 32 atoms per step on
//           v_mfma_f32_32x32x16_bf16 with FP32 accumulation;
//   window: the same sum in FP32 on the vector ALUs -- per 32-atom step the
//           atoms' dense factor rows go to LDS, and each lane accumulates
//           its four 16-voxel row runs over the atoms whose y-window holds
//           the row.
#include "pg_device.hpp"
#include "pg_launch.hpp"

namespace pg {

constexpr int KC = 32;          // atoms per contraction step
constexpr int ST = 128;         // MFMA super-tile edge (y and x)
constexpr int KPAD = KC + 8;    // bf16 row pitch of the LDS operand tiles

__global__ void cr_clear_kernel(uint32_t *a, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        a[i] = 0u;
}

// z planes of one record: calls f(z) once per plane of the window(s)
template <typename F>
__device__ __forceinline__ void for_each_z(const AtomWindow &w, F f)
{
    for (int r = 0; r < w.n[2]; ++r)
        for (int z = w.lo[2][r]; z <= w.hi[2][r]; ++z)
            f(z);
}

__global__ void __launch_bounds__(256) cr_prep_kernel(GridParams p, CrystalParams q)
{
    const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= p.n_atoms)
        return;
    const int m = write_atom_window(p, a, q.table + a);
    const AtomWindow &w = q.table[a];
    if (w.type < 0)
        return;
    const size_t base = ((size_t)m * p.C + w.type) * p.D;
    for_each_z(w, [&](int z) { atomicAdd(&q.counts[base + z], 1u); });
}

// Exclusive scan of n counts into offsets[0..n]; cursor[] cleared.  One
// workgroup of 1024 threads, each owning a contiguous segment.
__global__ void __launch_bounds__(1024) cr_scan_kernel(CrystalParams q, long long n)
{
    __shared__ unsigned long long part[1024];
    const int t = threadIdx.x;
    const long long seg = (n + 1023) / 1024;
    const long long b = (long long)t * seg, e = min(n, b + seg);
    unsigned long long s = 0;
    for (long long i = b; i < e; ++i)
        s += q.counts[i];
    part[t] = s;
    __syncthreads();
    // inclusive Hillis-Steele scan of the 1024 segment sums
    for (int d = 1; d < 1024; d <<= 1) {
        const unsigned long long v = t >= d ? part[t - d] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned long long run = part[t] - s;
    for (long long i = b; i < e; ++i) {
        q.offsets[i] = (uint32_t)run;
        run += q.counts[i];
        q.cursor[i] = 0u;
    }
    if (t == 1023)
        q.offsets[n] = (uint32_t)part[1023];
}

__global__ void __launch_bounds__(256) cr_fill_kernel(GridParams p, CrystalParams q)
{
    const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= p.n_atoms)
        return;
    const AtomWindow &w = q.table[a];
    if (w.type < 0)
        return;
    const int m = structure_of(p.offsets, p.n_mol, a);
    const size_t base = ((size_t)m * p.C + w.type) * p.D;
    for_each_z(w, [&](int z) {
        const size_t bin = base + z;
        const uint32_t pos = atomicAdd(&q.cursor[bin], 1u);
        q.list[q.offsets[bin] + pos] = (int32_t)a;
    });
}

// Load a plane's bin into LDS and sort it ascending (bitonic, padded to a
// power of two with INT_MAX).  Returns the count, or -1 if it exceeds cap.
__device__ int load_sorted_bin(const CrystalParams &q, size_t bin, int32_t *ids, int cap)
{
    const uint32_t start = q.offsets[bin];
    const int cnt = (int)(q.offsets[bin + 1] - start);
    if (cnt > cap)
        return -1;
    int np = 1;
    while (np < cnt)
        np <<= 1;
    for (int i = threadIdx.x; i < np; i += blockDim.x)
        ids[i] = i < cnt ? q.list[start + i] : 0x7fffffff;
    __syncthreads();
    for (int k = 2; k <= np; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < np; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const int32_t x = ids[i], y = ids[l];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        ids[i] = y;
                        ids[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    return cnt;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// One workgroup (4 waves) per (structure, channel, z, super-tile); wave w
// owns the 64 x 64 quadrant (w / 2, w % 2) of the 128 x 128 super-tile as
// 2 x 2 MFMA tiles of 32 x 32.
template <typename T>
__global__ void __launch_bounds__(256) cr_mfma_kernel(GridParams p, CrystalParams q)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    __bf16 *At = (__bf16 *)smem;                          // [ST][KPAD]: A[y][k]
    __bf16 *Bt = At + ST * KPAD;                          // [ST][KPAD]: B[k][x] stored by x
    AtomWindow *recs = (AtomWindow *)(Bt + ST * KPAD);    // [KC] records of the step
    int32_t *ids = (int32_t *)(recs + KC);                // sorted bin
    const int C = p.C, D = p.D, H = p.H, W = p.W;
    const int nsx = (W + ST - 1) / ST, nsy = (H + ST - 1) / ST;
    long long b = blockIdx.x;
    const int sx = (int)(b % nsx);
    b /= nsx;
    const int sy = (int)(b % nsy);
    b /= nsy;
    const int z = (int)(b % D);
    b /= D;
    const int c = (int)(b % C);
    const int m = (int)(b / C);
    const int y0 = sy * ST, x0 = sx * ST;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const size_t bin = ((size_t)m * C + c) * D + z;

    const int cnt = load_sorted_bin(q, bin, ids, q.bin_cap);
    if (cnt < 0 && tid == 0 && sx == 0 && sy == 0)
        raise_error(p.err, PG_E_CAPACITY, m);
    const int nk = cnt < 0 ? 0 : cnt;

    const float hx = p.h[0], hy = p.h[1], hz = p.h[2];
    const float inv2s2 = p.inv2s2[c];
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e)
                acc[i][j][e] = 0.f;
    const int qy = (wave >> 1) * 64, qx = (wave & 1) * 64;

    for (int k0 = 0; k0 < nk; k0 += KC) {
        // ---- the step's atom records into LDS
        {
            const int words = (int)(sizeof(AtomWindow) / 4);
            for (int e = tid; e < KC * words; e += blockDim.x) {
                const int k = e / words, wd = e - k * words;
                ((int32_t *)recs)[e] = k0 + k < nk ? ((const int32_t *)(q.table + ids[k0 + k]))[wd] : 0;
            }
        }
        __syncthreads();
        // ---- operand columns of 32 atoms: 8 threads per atom, each 16 rows
        // of A and 16 rows of B^T (every entry written, zeros included)
        {
            const int k = tid >> 3, part = tid & 7;
            const bool live = k0 + k < nk;
            const AtomWindow &w = recs[k];
            const float gz = live ? record_factor(w, 2, z, hz, inv2s2) : 0.f;
            for (int i = part; i < ST; i += 8) {
                const int y = y0 + i, x = x0 + i;
                const float fy = (live && y < H) ? record_factor(w, 1, y, hy, inv2s2) : 0.f;
                const float fx = (live && x < W) ? record_factor(w, 0, x, hx, inv2s2) : 0.f;
                At[i * KPAD + k] = (__bf16)(gz * fy);
                Bt[i * KPAD + k] = (__bf16)fx;
            }
        }
        __syncthreads();
        // ---- 2 k-steps of 16 on the wave's 2 x 2 tiles
#pragma unroll
        for (int ks = 0; ks < KC; ks += 16) {
            const int kk = ks + 8 * (lane >> 5);
            bf16x8 av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                av[i] = *(const bf16x8 *)(At + (qy + 32 * i + (lane & 31)) * KPAD + kk);
                bv[i] = *(const bf16x8 *)(Bt + (qx + 32 * i + (lane & 31)) * KPAD + kk);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }

    // ---- store the quadrant: lane holds column (lane & 31) of rows
    // 8 (e / 4) + 4 (lane / 32) + e % 4 of each tile
    T *out = (T *)p.out + (((size_t)m * C + c) * D + z) * (size_t)H * W;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int y = y0 + qy + 32 * i + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                const int x = x0 + qx + 32 * j + (lane & 31);
                if (y < H && x < W) {
                    const float v[1] = {acc[i][j][e]};
                    store_vec<T, 1>(out + (size_t)y * W + x, v, p.nt_store != 0);
                }
            }
}

// FP32 vector-ALU form: one workgroup (256 threads) per (structure,
// channel, z); lane t owns 16-voxel row runs p = t + 256 r of the plane.
template <typename T, int RMAX>
__global__ void __launch_bounds__(256) cr_window_kernel(GridParams p, CrystalParams q)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int C = p.C, D = p.D, H = p.H, W = p.W;
    const int W16 = (W + 15) & ~15;
    float *gx = (float *)smem;                    // [KC][W16] phi_x
    float *gy = gx + KC * W16;                    // [KC][H]   phi_z(z) phi_y
    int32_t *ids = (int32_t *)(gy + KC * H);
    long long b = blockIdx.x;
    const int z = (int)(b % D);
    b /= D;
    const int c = (int)(b % C);
    const int m = (int)(b / C);
    const int tid = threadIdx.x;
    const size_t bin = ((size_t)m * C + c) * D + z;
    const int cnt = load_sorted_bin(q, bin, ids, q.bin_cap);
    if (cnt < 0 && tid == 0)
        raise_error(p.err, PG_E_CAPACITY, m);
    const int nk = cnt < 0 ? 0 : cnt;
    const float hx = p.h[0], hy = p.h[1], hz = p.h[2];
    const float inv2s2 = p.inv2s2[c];
    const int runs_x = W16 / 16;
    const int n_runs = H * runs_x;
    float acc[RMAX][16];
#pragma unroll
    for (int r = 0; r < RMAX; ++r)
#pragma unroll
        for (int e = 0; e < 16; ++e)
            acc[r][e] = 0.f;

    for (int k0 = 0; k0 < nk; k0 += KC) {
        const int kn = min(KC, nk - k0);
        // dense factor rows of the step's atoms
        for (int e = tid; e < kn * (W16 + H); e += blockDim.x) {
            const int k = e / (W16 + H), j = e - k * (W16 + H);
            const AtomWindow &w = q.table[ids[k0 + k]];
            if (j < W16) {
                gx[k * W16 + j] = j < W ? record_factor(w, 0, j, hx, inv2s2) : 0.f;
            } else {
                const int y = j - W16;
                gy[k * H + y] = record_factor(w, 2, z, hz, inv2s2) * record_factor(w, 1, y, hy, inv2s2);
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
            const int run = tid + 256 * r;
            if (run < n_runs) {
                const int y = run / runs_x, xr = (run - y * runs_x) * 16;
                for (int k = 0; k < kn; ++k) {
                    const float g = gy[k * H + y];
                    if (g == 0.f)
                        continue;
                    const float4 *f = (const float4 *)(gx + k * W16 + xr);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const float4 fv = f[v];
                        acc[r][4 * v + 0] = __builtin_fmaf(g, fv.x, acc[r][4 * v + 0]);
                        acc[r][4 * v + 1] = __builtin_fmaf(g, fv.y, acc[r][4 * v + 1]);
                        acc[r][4 * v + 2] = __builtin_fmaf(g, fv.z, acc[r][4 * v + 2]);
                        acc[r][4 * v + 3] = __builtin_fmaf(g, fv.w, acc[r][4 * v + 3]);
                    }
                }
            }
        }
        __syncthreads();
    }
    T *out = (T *)p.out + (((size_t)m * C + c) * D + z) * (size_t)H * W;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
        const int run = tid + 256 * r;
        if (run < n_runs) {
            const int y = run / runs_x, xr = (run - y * runs_x) * 16;
            for (int e = 0; e < 16; ++e) {
                if (xr + e < W) {
                    const float v[1] = {acc[r][e]};
                    store_vec<T, 1>(out + (size_t)y * W + xr + e, v, p.nt_store != 0);
                }
            }
        }
    }
}

size_t crystal_plane_lds(int form, int H, int W, int bin_cap)
{
    if (form == PG_FORM_MFMA)
        return (size_t)2 * ST * KPAD * sizeof(__bf16) + (size_t)KC * sizeof(AtomWindow) +
               (size_t)bin_cap * sizeof(int32_t);
    const int W16 = (W + 15) & ~15;
    return (size_t)KC * (W16 + H) * sizeof(float) + (size_t)bin_cap * sizeof(int32_t);
}

// runs of 16 voxels per lane of the vector form (0: plane too large)
int crystal_window_runs(int H, int W)
{
    const long long runs = (long long)H * (((W + 15) & ~15) / 16);
    for (int r = 1; r <= 8; r <<= 1)
        if (runs <= 256LL * r)
            return r;
    return 0;
}

hipError_t launch_crystal(const GridParams &p, const CrystalParams &q, int form, int out_dtype,
                          size_t lds, hipStream_t s)
{
    if (p.n_mol == 0)
        return hipSuccess;
    const long long nb = (long long)p.n_mol * p.C * p.D;
    hipLaunchKernelGGL(cr_clear_kernel, dim3((unsigned)std::min<long long>((nb + 255) / 256, 65535)),
                       dim3(256), 0, s, q.counts, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (p.n_atoms > 0) {
        const unsigned ga = (unsigned)((p.n_atoms + 255) / 256);
        hipLaunchKernelGGL(cr_prep_kernel, dim3(ga), dim3(256), 0, s, p, q);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(cr_scan_kernel, dim3(1), dim3(1024), 0, s, q, nb);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if (p.n_atoms > 0) {
        const unsigned ga = (unsigned)((p.n_atoms + 255) / 256);
        hipLaunchKernelGGL(cr_fill_kernel, dim3(ga), dim3(256), 0, s, p, q);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    const void *k;
    long long grid;
    if (form == PG_FORM_MFMA) {
        k = out_dtype == PG_OUT_F32 ? (const void *)cr_mfma_kernel<float>
                                    : (const void *)cr_mfma_kernel<__bf16>;
        grid = nb * ((p.H + ST - 1) / ST) * ((p.W + ST - 1) / ST);
    } else {
        const int r = crystal_window_runs(p.H, p.W);
        if (out_dtype == PG_OUT_F32)
            k = r == 1 ? (const void *)cr_window_kernel<float, 1>
              : r == 2 ? (const void *)cr_window_kernel<float, 2>
              : r == 4 ? (const void *)cr_window_kernel<float, 4>
              : r == 8 ? (const void *)cr_window_kernel<float, 8> : nullptr;
        else
            k = r == 1 ? (const void *)cr_window_kernel<__bf16, 1>
              : r == 2 ? (const void *)cr_window_kernel<__bf16, 2>
              : r == 4 ? (const void *)cr_window_kernel<__bf16, 4>
              : r == 8 ? (const void *)cr_window_kernel<__bf16, 8> : nullptr;
        if (!k)
            return hipErrorInvalidValue;
        grid = nb;
    }
    if (lds > 65536) {
        e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    GridParams pc = p;
    CrystalParams qc = q;
    void *args[] = {&pc, &qc};
    return hipLaunchKernel(k, dim3((unsigned)grid), dim3(256), args, lds, s);
}

}  // namespace pg
