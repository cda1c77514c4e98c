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

// LDS buffer of one work item (a group of `group` structures): per slot, the
// dense factor rows [a_cap][row_stride] and the plane masks
// [C*D][mask_words].  The kernel holds two such buffers.
__host__ __device__ inline WindowLds window_lds_layout(int a_cap, int row_stride, int C, int D,
                                                      int mask_words, int group)
{
    WindowLds L;
    L.rows = 0;
    L.rows_bytes = ((size_t)a_cap * row_stride * sizeof(float) + 15) & ~(size_t)15;
    L.masks = (size_t)group * L.rows_bytes;
    L.masks_bytes = (size_t)C * D * mask_words * sizeof(unsigned long long);
    L.buffer = (L.masks + (size_t)group * L.masks_bytes + 15) & ~(size_t)15;
    L.total = 2 * L.buffer;
    return L;
}

WindowLds window_lds(int a_cap, int row_stride, int C, int D, int mask_words, int group)
{
    return window_lds_layout(a_cap, row_stride, C, D, mask_words, group);
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

// Prep role: build the factor rows and plane masks of work item `item` into
// LDS buffer `buf` (whose masks the store role left zeroed).  One thread per
// (slot, atom, axis): exact window ranges, then the thread fills that
// atom's dense row for the axis and, for z, sets the atom's bit in the
// (type, z) plane masks.  Only these waves touch global memory for inputs.
__device__ void prep_item(const GridParams &p, const WindowLds &lay, unsigned char *buf, int item,
                          int tp, int ntp)
{
    const int C = p.C, D = p.D, H = p.H, W = p.W;
    const int RS = p.row_stride, W4 = (W + 3) & ~3, MW = p.mask_words, K = p.group;
    const int m0 = item * K;
    const int ns = min(K, p.n_mol - m0);
    // total (slot, atom, axis) entries; slots with bad offsets or too many
    // atoms get none (their grids are written as zeros) and raise an error
    int total = 0;
    for (int s = 0; s < ns; ++s) {
        const int m = m0 + s;
        const int a0 = p.offsets[m], na = p.offsets[m + 1] - a0;
        const bool bad = na > p.a_cap || na < 0 || a0 < 0 || (long long)a0 + na > p.n_atoms;
        if (bad && tp == 0)
            raise_error(p.err, na > p.a_cap ? PG_E_CAPACITY : PG_E_DEVICE_DATA, m);
        total += bad ? 0 : 3 * na;
    }
    for (int i = tp; i < total; i += ntp) {
        // locate the slot of entry i: the first slot whose entries extend
        // past i (entries of slot q are [base_q, base_q + cnt_q))
        int s = 0, base = 0, a0 = 0;
        for (int q = 0; q < ns; ++q) {
            const int m = m0 + q;
            const int qa0 = p.offsets[m], qna = p.offsets[m + 1] - qa0;
            const bool bad = qna > p.a_cap || qna < 0 || qa0 < 0 || (long long)qa0 + qna > p.n_atoms;
            const int cnt = bad ? 0 : 3 * qna;
            if (i < base + cnt) {
                s = q;
                a0 = qa0;
                break;
            }
            base += cnt;
        }
        const int li = i - base;
        const int a = li / 3, ax = li - 3 * a;
        const int m = m0 + s;
        const size_t ga = (size_t)a0 + a;
        const float x = p.xyz[3 * ga + 0], y = p.xyz[3 * ga + 1], z = p.xyz[3 * ga + 2];
        const int t = p.types[ga];
        if (!atom_valid(x, y, z, t, C)) {
            if (ax == 0)
                raise_error(p.err, PG_E_DEVICE_DATA, (long long)ga);
            continue;
        }
        const float mu = ax == 0 ? x : (ax == 1 ? y : z);
        const int N = ax == 0 ? W : (ax == 1 ? H : D);
        const int off = ax == 0 ? 0 : (ax == 1 ? W4 : W4 + H);
        const float o = p.origins ? p.origins[3 * (size_t)m + ax] : (ax == 0 ? p.o[0] : (ax == 1 ? p.o[1] : p.o[2]));
        const float h = p.spacings ? p.spacings[3 * (size_t)m + ax] : (ax == 0 ? p.h[0] : (ax == 1 ? p.h[1] : p.h[2]));
        const float L = ax == 0 ? p.L[0] : (ax == 1 ? p.L[1] : p.L[2]);
        AxisRanges R;
        axis_ranges(o, h, N, mu, p.periodic != 0, L, p.rc[t], p.cut != 0, R);
        float *row = (float *)(buf + lay.rows + (size_t)s * lay.rows_bytes) + (size_t)a * RS + off;
        unsigned long long *masks =
            (unsigned long long *)(buf + lay.masks + (size_t)s * lay.masks_bytes);
        const float inv2s2 = p.inv2s2[t];
        int r = 0;
        for (int idx = 0; idx < N; ++idx) {
            // ranges are disjoint and ascending
            while (r < R.n && idx > (r == 0 ? R.hi[0] : (r == 1 ? R.hi[1] : R.hi[2])))
                ++r;
            float v = 0.f;
            if (r < R.n) {
                const int lo = r == 0 ? R.lo[0] : (r == 1 ? R.lo[1] : R.lo[2]);
                if (idx >= lo) {
                    const float bh = r == 0 ? R.bh[0] : (r == 1 ? R.bh[1] : R.bh[2]);
                    const float bl = r == 0 ? R.bl[0] : (r == 1 ? R.bl[1] : R.bl[2]);
                    v = gauss1d(offset_at(bh, bl, h, idx), inv2s2);
                    if (ax == 2)
                        atomicOr(&masks[(size_t)(t * D + idx) * MW + (a >> 6)], 1ull << (a & 63));
                }
            }
            row[idx] = v;
        }
    }
}

template <typename T, int VEC, int U>
__global__ void __launch_bounds__(1024) window_mol_kernel(GridParams p)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int C = p.C, D = p.D, H = p.H, W = p.W;
    const int RS = p.row_stride;
    const int W4 = (W + 3) & ~3;
    const int MW = p.mask_words;
    const int K = p.group;
    const WindowLds lay = window_lds_layout(p.a_cap, RS, C, D, MW, K);

    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
    const int n_store = nwaves - p.prep_waves;      // store-role waves
    const bool prep_role = wave >= n_store;
    const int tp = tid - n_store * 64, ntp = p.prep_waves * 64;
    const int planes = C * D;
    const size_t plane_elems = (size_t)H * W;
    const size_t mol_elems = (size_t)planes * plane_elems;
    const int chunks = (int)(plane_elems / VEC);
    const bool nt = p.nt_store != 0;
    // runs (VEC consecutive x) per row; floor((j + 1/2) / CW) in float is
    // exact for run indices below 2^20
    const int CW = W / VEC;
    const float inv_cw = 1.0f / (float)CW;
    const int n_items = (p.n_mol + K - 1) / K;

    // both buffers' masks start cleared; afterwards the store role clears
    // each plane mask right after reading it
    for (size_t i = tid; i < lay.total / sizeof(unsigned long long); i += nthr)
        ((unsigned long long *)smem)[i] = 0ull;
    __syncthreads();
    if (prep_role && (int)blockIdx.x < n_items)
        prep_item(p, lay, smem, blockIdx.x, tp, ntp);
    __syncthreads();

    int cur = 0;
    for (int item = blockIdx.x; item < n_items; item += gridDim.x, cur ^= 1) {
        unsigned char *bcur = smem + (size_t)cur * lay.buffer;
        if (prep_role) {
            // the next item of this workgroup, into the other buffer
            const int nxt = item + gridDim.x;
            if (nxt < n_items)
                prep_item(p, lay, smem + (size_t)(cur ^ 1) * lay.buffer, nxt, tp, ntp);
        } else {
            // store role: stream the planes of every slot of this item; each
            // lane owns U runs per pass (U back-to-back 16-byte stores)
            const int m0 = item * K;
            const int ns = min(K, p.n_mol - m0);
            for (int gp = wave; gp < ns * planes; gp += n_store) {
                const int s = gp / planes;
                const int pl = gp - s * planes;
                const int z = pl % D;
                const float *rows = (const float *)(bcur + lay.rows + (size_t)s * lay.rows_bytes);
                unsigned long long *masks =
                    (unsigned long long *)(bcur + lay.masks + (size_t)s * lay.masks_bytes);
                unsigned long long mk[4];
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    mk[w] = (w < MW) ? uniform64(masks[(size_t)pl * MW + w]) : 0ull;
                // this wave is the only reader of the plane's mask: clear it
                // for the item that will reuse the buffer
                if (lane < MW)
                    masks[(size_t)pl * MW + lane] = 0ull;
                T *op = (T *)p.out + (size_t)(m0 + s) * mol_elems + (size_t)pl * plane_elems;
                for (int j0 = lane; j0 < chunks; j0 += 64 * U) {
                    int yq[U], xq[U];
                    bool ok[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int j = j0 + 64 * u;
                        ok[u] = j < chunks;
                        // run j starts at element j*VEC: row j / CW, column (j % CW) * VEC
                        const int yy = (int)(((float)j + 0.5f) * inv_cw);
                        yq[u] = ok[u] ? yy : 0;
                        xq[u] = ok[u] ? (j - yy * CW) * VEC : 0;
                    }
                    float acc[U][VEC];
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int k = 0; k < VEC; ++k)
                            acc[u][k] = 0.f;
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        unsigned long long bits = mk[w];
                        while (bits) {
                            const int a = w * 64 + __builtin_ctzll(bits);
                            bits &= bits - 1;
                            const float *row = rows + a * RS;
                            const float gz = row[W4 + H + z];
#pragma unroll
                            for (int u = 0; u < U; ++u) {
                                const float gy = row[W4 + yq[u]] * gz;
                                float fx[VEC];
                                load_row<VEC>(row + xq[u], fx);
#pragma unroll
                                for (int k = 0; k < VEC; ++k)
                                    acc[u][k] = __builtin_fmaf(gy, fx[k], acc[u][k]);
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (ok[u])
                            store_vec<T, VEC>(op + (size_t)(j0 + 64 * u) * VEC, acc[u], nt);
                }
            }
        }
        __syncthreads();
    }
}

template <typename T, int VEC, int U>
static const void *window_fn()
{
    return (const void *)window_mol_kernel<T, VEC, U>;
}

template <typename T, int VEC>
static const void *window_fn_u(int unroll)
{
    return unroll >= 4 ? window_fn<T, VEC, 4>() : unroll == 2 ? window_fn<T, VEC, 2>()
                                                              : window_fn<T, VEC, 1>();
}

static const void *window_kernel_fn(int out_dtype, int vec, int unroll)
{
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
    const void *k = window_kernel_fn(out_dtype, vec, unroll);
    if (!k)
        return hipErrorInvalidValue;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    GridParams pc = p;
    void *args[] = {&pc};
    return hipLaunchKernel(k, dim3(grid), dim3(block), args, lds, s);
}

int window_occupancy(int out_dtype, int vec, int unroll, int block, size_t lds)
{
    int n = 0;
    const void *k = window_kernel_fn(out_dtype, vec, unroll);
    if (!k)
        return 1;
    if (lds > 65536)
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, block, lds) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace pg
