// pg_crystal.hip -- large / dense structures (periodic crystal cells, big
// clusters) on gfx950.
//
// Structures with more atoms than the molecule window kernel stages in LDS
// take this path.  Set-up, all on the GPU and free of order-dependent
// atomics in anything that reaches the output:
//   prep:   one thread per atom: exact per-axis window ranges (nearest
//           periodic images included) into the atom's record, the 1-D
//           factors of every voxel index inside them (once per atom, ranges
//           concatenated), and counts of the atom per (channel, structure)
//           and per (channel, prep block);
//   scan:   exclusive scans of both count arrays in channel-major order;
//   place:  a stable partition of all atoms by channel (ballot ranks within
//           a block): channel c's atoms in index order, so each (structure,
//           channel) pair is one contiguous run of the list.
// Then one plane kernel, one workgroup per (structure, channel, z plane
// [, 128 x 128 super-tile]).  It compacts, in list order, the atoms of its
// run whose z window holds the plane, so every voxel sums its atoms in
// atom-index order (bitwise reproducible), then contracts over them:
//   mfma:   the plane is a product of two factor matrices (separability of
//           the Gaussian and of the cube cutoff, Sec. III-A / IV-C):
//           G[y][x] = sum_k A[y][k] B[k][x], A[y][k] = phi_z^k(z) phi_y^k(y)
//           formed in FP32 and rounded once to bf16, B[k][x] = phi_x^k(x) in
//           bf16; 32 atoms per step on v_mfma_f32_32x32x16_bf16, FP32
//           accumulation;
//   window: the same sum in FP32 on the vector ALUs -- per 32-atom step the
//           atoms' dense factor rows go to LDS, and each lane accumulates
//           its 16-voxel row runs over the atoms whose y window holds the row.
#include "pg_device.hpp"
#include "pg_launch.hpp"

namespace pg {

constexpr int PREP_BLOCK = 256; // atoms per prep / place block (4 waves)
constexpr int KC = 32;          // atoms per contraction step
constexpr int ST = 128;         // MFMA super-tile edge (y and x)
constexpr int KPAD = KC + 8;    // bf16 row pitch of the LDS operand tiles

__global__ void cr_clear_kernel(uint32_t *a, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        a[i] = 0u;
}

__global__ void __launch_bounds__(PREP_BLOCK) cr_prep_kernel(GridParams p, CrystalParams q)
{
    __shared__ uint32_t cnt[PG_MAX_CHANNELS];
    const int tid = threadIdx.x;
    for (int c = tid; c < p.C; c += PREP_BLOCK)
        cnt[c] = 0u;
    __syncthreads();
    const long long a = (long long)blockIdx.x * PREP_BLOCK + tid;
    if (a < p.n_atoms) {
        AtomWindow *w = q.table + a;
        const int m = write_atom_window(p, a, w);
        const int t = w->type;
        if (t >= 0) {
            const float inv2s2 = p.inv2s2[t];
            const int S = q.fstride;
            for (int ax = 0; ax < 3; ++ax) {
                float *f = q.fac + ((size_t)a * 3 + ax) * S;
                const float h = p.h[ax];
                int j = 0;
                for (int r = 0; r < w->n[ax]; ++r) {
                    const float bh = w->bh[ax][r], bl = w->bl[ax][r];
                    for (int i = w->lo[ax][r]; i <= w->hi[ax][r] && j < S; ++i, ++j)
                        f[j] = gauss1d(offset_at(bh, bl, h, i), inv2s2);
                }
            }
            atomicAdd(&cnt[t], 1u);
            atomicAdd(&q.mcount[(size_t)t * p.n_mol + m], 1u);
        }
    }
    __syncthreads();
    for (int c = tid; c < p.C; c += PREP_BLOCK)
        q.bcount[(size_t)c * q.nblk + blockIdx.x] = cnt[c];
}

// Exclusive scan of n counts, in place (workgroup 0: the per-block counts)
// or into mstart (workgroup 1: the per-structure counts).  One workgroup
// of 1024 threads per array, each thread owning a contiguous segment.
__global__ void __launch_bounds__(1024) cr_scan_kernel(CrystalParams q, long long n_blk,
                                                       long long n_mol)
{
    __shared__ unsigned long long part[1024];
    const uint32_t *in = blockIdx.x == 0 ? q.bcount : q.mcount;
    uint32_t *out = blockIdx.x == 0 ? q.bcount : q.mstart;
    const long long n = blockIdx.x == 0 ? n_blk : n_mol;
    const int t = threadIdx.x;
    const long long seg = (n + 1023) / 1024;
    const long long b = (long long)t * seg, e = min(n, b + seg);
    unsigned long long s = 0;
    for (long long i = b; i < e; ++i)
        s += in[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const unsigned long long v = t >= d ? part[t - d] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned long long run = part[t] - s;
    for (long long i = b; i < e; ++i) {
        const uint32_t v = in[i];
        out[i] = (uint32_t)run;
        run += v;
    }
}

__device__ __forceinline__ uint32_t pack_range(int lo, int hi)
{
    return (uint32_t)(uint16_t)(int16_t)lo | ((uint32_t)(uint16_t)(int16_t)hi << 16);
}

__global__ void __launch_bounds__(PREP_BLOCK) cr_place_kernel(GridParams p, CrystalParams q)
{
    __shared__ uint32_t wc[PREP_BLOCK / 64][PG_MAX_CHANNELS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long a = (long long)blockIdx.x * PREP_BLOCK + tid;
    const int t = a < p.n_atoms ? q.table[a].type : -1;
    const unsigned long long below = (1ull << lane) - 1ull;
    uint32_t rank = 0;
    for (int c = 0; c < p.C; ++c) {
        const unsigned long long mask = __ballot(t == c);
        if (t == c)
            rank = (uint32_t)__popcll(mask & below);
        if (lane == 0)
            wc[wave][c] = (uint32_t)__popcll(mask);
    }
    __syncthreads();
    if (t >= 0) {
        uint32_t pos = q.bcount[(size_t)t * q.nblk + blockIdx.x] + rank;
        for (int w = 0; w < wave; ++w)
            pos += wc[w][t];
        const AtomWindow &w = q.table[a];
        ListEntry e;
        e.atom = (int32_t)a;
#pragma unroll
        for (int r = 0; r < 3; ++r)
            e.z[r] = r < w.n[2] ? pack_range(w.lo[2][r], w.hi[2][r]) : pack_range(0, -1);
        q.list[pos] = e;
    }
}

// XCD-aware workgroup order: the hardware deals consecutive workgroups to
// the 8 XCDs in turn; remap so that each XCD runs a contiguous stretch of
// planes (consecutive z of one structure and channel share their atoms'
// factor rows in that XCD's L2).  A bijection on [0, gridDim.x).
__device__ __forceinline__ long long xcd_block()
{
    const unsigned G = gridDim.x, full = G & ~7u, b = blockIdx.x;
    return b < full ? (long long)(b & 7u) * (full >> 3) + (b >> 3) : (long long)b;
}

// Ordered compaction of the plane's atoms: the (m, c) run of the channel
// partition filtered by "z window holds z", in list order, into ids[] with
// each atom's z factor in gz[].  Returns the count, or -1 above cap (then
// ids / gz hold a prefix only).  Uniform across the workgroup; contains
// barriers (all threads must call it).
__device__ int gather_plane(const GridParams &p, const CrystalParams &q, int m, int c, int z,
                            int32_t *ids, float *gz, uint32_t *wsum)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const size_t mc = (size_t)c * p.n_mol + m;
    const uint32_t start = q.mstart[mc], n = q.mcount[mc];
    const int S = q.fstride, cap = q.bin_cap;
    const unsigned long long below = (1ull << lane) - 1ull;
    int cnt = 0;
    for (uint32_t base = 0; base < n; base += blockDim.x) {
        const uint32_t e = base + tid;
        bool live = false;
        int a = 0, jz = 0;
        if (e < n) {
            const ListEntry le = q.list[start + e];
            a = le.atom;
            int s = 0;
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int lo = (int16_t)(le.z[r] & 0xffffu), hi = (int16_t)(le.z[r] >> 16);
                if (z >= lo && z <= hi) {
                    live = true;
                    jz = s + z - lo;
                }
                s += hi >= lo ? hi - lo + 1 : 0;
            }
        }
        const unsigned long long mask = __ballot(live);
        if (lane == 0)
            wsum[wave] = (uint32_t)__popcll(mask);
        __syncthreads();
        int off = cnt, total = 0;
        for (int w = 0; w < nw; ++w) {
            off += w < wave ? (int)wsum[w] : 0;
            total += (int)wsum[w];
        }
        const int pos = off + __popcll(mask & below);
        if (live && pos < cap) {
            ids[pos] = a;
            gz[pos] = jz < S ? q.fac[((size_t)a * 3 + 2) * S + jz] : 0.f;
        }
        cnt += total;
        __syncthreads();
    }
    return cnt > cap ? -1 : cnt;
}

// x / y ranges of one step's atoms, staged in LDS: lo, hi, and the start of
// each range in the atom's concatenated factor values.
struct StepRec {
    int32_t atom;
    int32_t lo[2][3], hi[2][3], st[2][3];
};

__device__ __forceinline__ void stage_records(const CrystalParams &q, const int32_t *ids, int k0,
                                              int kn, StepRec *recs)
{
    const int k = threadIdx.x;
    if (k < KC) {
        StepRec r;
        r.atom = k < kn ? ids[k0 + k] : -1;
#pragma unroll
        for (int ax = 0; ax < 2; ++ax) {
            int s = 0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                int lo = 0, hi = -1;
                if (r.atom >= 0) {
                    const AtomWindow &w = q.table[r.atom];
                    if (i < w.n[ax]) {
                        lo = w.lo[ax][i];
                        hi = w.hi[ax][i];
                    }
                }
                r.lo[ax][i] = lo;
                r.hi[ax][i] = hi;
                r.st[ax][i] = s - lo;
                s += hi - lo + 1;
            }
        }
        recs[k] = r;
    }
}

// Factor of the staged atom on axis ax at index v (0 outside its window).
__device__ __forceinline__ float step_factor(const CrystalParams &q, const StepRec &r, int ax,
                                             int v)
{
    int j = -1;
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (v >= r.lo[ax][i] && v <= r.hi[ax][i])
            j = r.st[ax][i] + v;
    return (j >= 0 && j < q.fstride) ? q.fac[((size_t)r.atom * 3 + ax) * q.fstride + j] : 0.f;
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
    StepRec *recs = (StepRec *)(Bt + ST * KPAD);          // [KC]
    uint32_t *wsum = (uint32_t *)(recs + KC);             // [4]
    int32_t *ids = (int32_t *)(wsum + 4);                 // [bin_cap]
    float *gzs = (float *)(ids + q.bin_cap);              // [bin_cap]
    const int C = p.C, D = p.D, H = p.H, W = p.W;
    const int nsx = (W + ST - 1) / ST, nsy = (H + ST - 1) / ST;
    long long b = xcd_block();
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

    const int cnt = gather_plane(p, q, m, c, z, ids, gzs, wsum);
    if (cnt < 0 && tid == 0 && sx == 0 && sy == 0)
        raise_error(p.err, PG_E_CAPACITY, m);
    const int nk = cnt < 0 ? 0 : cnt;

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
        stage_records(q, ids, k0, min(KC, nk - k0), recs);
        __syncthreads();
        // operand columns of 32 atoms: 8 threads per atom, each 16 rows of A
        // and 16 rows of B^T (every entry written, zeros included)
        {
            const int k = tid >> 3, part = tid & 7;
            const StepRec r = recs[k];
            const float g = r.atom >= 0 ? gzs[k0 + k] : 0.f;
#pragma unroll 4
            for (int i = part; i < ST; i += 8) {
                const float fy = r.atom >= 0 ? step_factor(q, r, 1, y0 + i) : 0.f;
                const float fx = r.atom >= 0 ? step_factor(q, r, 0, x0 + i) : 0.f;
                At[i * KPAD + k] = (__bf16)(g * fy);
                Bt[i * KPAD + k] = (__bf16)fx;
            }
        }
        __syncthreads();
        // 2 k-steps of 16 on the wave's 2 x 2 tiles
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

    // store the quadrant: lane holds column (lane & 31) of rows
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
    StepRec *recs = (StepRec *)(gy + KC * ((H + 3) & ~3));
    uint32_t *wsum = (uint32_t *)(recs + KC);
    int32_t *ids = (int32_t *)(wsum + 4);
    float *gzs = (float *)(ids + q.bin_cap);
    long long b = xcd_block();
    const int z = (int)(b % D);
    b /= D;
    const int c = (int)(b % C);
    const int m = (int)(b / C);
    const int tid = threadIdx.x;
    const int cnt = gather_plane(p, q, m, c, z, ids, gzs, wsum);
    if (cnt < 0 && tid == 0)
        raise_error(p.err, PG_E_CAPACITY, m);
    const int nk = cnt < 0 ? 0 : cnt;
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
        stage_records(q, ids, k0, kn, recs);
        __syncthreads();
        // dense factor rows of the step's atoms
        for (int e = tid; e < kn * (W16 + H); e += blockDim.x) {
            const int k = e / (W16 + H), j = e - k * (W16 + H);
            const StepRec &r = recs[k];
            if (j < W16) {
                gx[k * W16 + j] = j < W ? step_factor(q, r, 0, j) : 0.f;
            } else {
                const int y = j - W16;
                gy[k * H + y] = gzs[k0 + k] * step_factor(q, r, 1, y);
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
    const size_t tail = (size_t)KC * sizeof(StepRec) + 4 * sizeof(uint32_t) +
                        (size_t)bin_cap * (sizeof(int32_t) + sizeof(float));
    if (form == PG_FORM_MFMA)
        return (size_t)2 * ST * KPAD * sizeof(__bf16) + tail;
    const int W16 = (W + 15) & ~15;
    return (size_t)KC * (W16 + ((H + 3) & ~3)) * sizeof(float) + tail;
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

int crystal_prep_blocks(long long n_atoms)
{
    return (int)((n_atoms + PREP_BLOCK - 1) / PREP_BLOCK);
}

hipError_t launch_crystal(const GridParams &p, const CrystalParams &q, int form, int out_dtype,
                          size_t lds, hipStream_t s)
{
    if (p.n_mol == 0)
        return hipSuccess;
    const long long nmc = (long long)p.n_mol * p.C;
    hipLaunchKernelGGL(cr_clear_kernel, dim3((unsigned)std::min<long long>((nmc + 255) / 256, 65535)),
                       dim3(256), 0, s, q.mcount, nmc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (p.n_atoms > 0) {
        hipLaunchKernelGGL(cr_prep_kernel, dim3((unsigned)q.nblk), dim3(PREP_BLOCK), 0, s, p, q);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        hipLaunchKernelGGL(cr_scan_kernel, dim3(2), dim3(1024), 0, s, q, (long long)p.C * q.nblk,
                           nmc);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        hipLaunchKernelGGL(cr_place_kernel, dim3((unsigned)q.nblk), dim3(PREP_BLOCK), 0, s, p, q);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    } else {
        // no atoms: every run is empty; mstart only has to be readable
        hipLaunchKernelGGL(cr_clear_kernel, dim3((unsigned)std::min<long long>((nmc + 255) / 256, 65535)),
                           dim3(256), 0, s, q.mstart, nmc);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    const void *k;
    long long grid;
    if (form == PG_FORM_MFMA) {
        k = out_dtype == PG_OUT_F32 ? (const void *)cr_mfma_kernel<float>
                                    : (const void *)cr_mfma_kernel<__bf16>;
        grid = nmc * p.D * ((p.H + ST - 1) / ST) * ((p.W + ST - 1) / ST);
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
        grid = nmc * p.D;
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
