// pg_reversal.hip -- grid reversal (§IV) kernels on gfx950: the local-maximum
// peak search that gives the initial coordinates (§IV-A step 1, §IV-B), and
// the residual / loss pass of a coordinate step for the forms whose forward
// kernel does not form the residual itself.
//
// Peak rule.  Voxel v of channel c is a peak when G[v] > threshold and, for
// each of its 26 neighbours u inside the grid (same channel, no wrap),
// G[v] > G[u] when u precedes v in raster order (z, y, x) and G[v] >= G[u]
// when u follows it, so a plateau of equal maxima gives its first voxel.
// Three launches, no atomics, output in raster order per structure:
//   peak_count  one workgroup per structure counts its peaks;
//   peak_scan   one workgroup turns the counts into CSR bounds clamped to
//               the output capacity, and the total;
//   peak_write  one workgroup per structure walks its voxels in raster order
//               in blocks of blockDim, ranks the peaks of each block with
//               wave ballots, and writes position and channel.
#include "pg_device.hpp"
#include "pg_launch.hpp"

namespace pg {

namespace {

constexpr int PEAK_BLOCK = 256;
constexpr int RES_BLOCK = 256;
constexpr int RES_PER_THREAD = 16;

// The floats adjacent to a finite r.
__device__ __forceinline__ float next_up(float r)
{
    if (r == 0.f)
        return __builtin_bit_cast(float, 1u);   // the smallest positive subnormal
    const uint32_t u = __builtin_bit_cast(uint32_t, r);
    return __builtin_bit_cast(float, r > 0.f ? u + 1u : u - 1u);
}

__device__ __forceinline__ float next_down(float r) { return -next_up(-r); }

// o + (i + 1/2) h rounded once to float32 (round to nearest, ties to even).
// (i + 1/2) h = ph + pl exactly (TwoProd); r is the float sum of o + ph + pl
// within an ulp, and the exact sign of (o + ph + pl) - r -/+ half an ulp of
// r (expansion arithmetic) moves it to the correctly rounded value.
__device__ __forceinline__ float centre_rounded(float o, int i, float h)
{
    float ph, pl;
    two_prod((float)i + 0.5f, h, ph, pl);
    float s, e;
    two_sum(o, ph, s, e);
    float r = s + (e + pl);
    const float up = next_up(r), dn = next_down(r);
    const float hu = 0.5f * (up - r), hd = 0.5f * (r - dn);   // exact halves of the gaps
    const float tu[5] = {o, ph, pl, -r, -hu};
    const int su = exact_sign(tu);
    if (su > 0 || (su == 0 && (__builtin_bit_cast(uint32_t, up) & 1u) == 0u))
        return up;
    const float td[5] = {o, ph, pl, -r, hd};
    const int sd = exact_sign(td);
    if (sd < 0 || (sd == 0 && (__builtin_bit_cast(uint32_t, dn) & 1u) == 0u))
        return dn;
    return r;
}

__device__ __forceinline__ bool peak_at(const float *g, int z, int y, int x, int D, int H, int W,
                                        float thr)
{
    const size_t plane = (size_t)H * W;
    const float v = g[(size_t)z * plane + (size_t)y * W + x];
    if (!(v > thr))
        return false;
    for (int dz = -1; dz <= 1; ++dz) {
        const int zz = z + dz;
        if (zz < 0 || zz >= D)
            continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = y + dy;
            if (yy < 0 || yy >= H)
                continue;
            for (int dx = -1; dx <= 1; ++dx) {
                const int xx = x + dx;
                if (xx < 0 || xx >= W || (dz == 0 && dy == 0 && dx == 0))
                    continue;
                const float u = g[(size_t)zz * plane + (size_t)yy * W + xx];
                const bool earlier = dz < 0 || (dz == 0 && (dy < 0 || (dy == 0 && dx < 0)));
                if (earlier ? !(v > u) : !(v >= u))
                    return false;
            }
        }
    }
    return true;
}

// voxel e of a structure (raster order over channel, z, y, x) is a peak
__device__ __forceinline__ bool peak_voxel(const PeakParams &p, const float *gm, long long e,
                                           int &c, int &z, int &y, int &x)
{
    const long long vol = (long long)p.D * p.H * p.W;
    c = (int)(e / vol);
    long long r = e - (long long)c * vol;
    z = (int)(r / ((long long)p.H * p.W));
    r -= (long long)z * p.H * p.W;
    y = (int)(r / p.W);
    x = (int)(r - (long long)y * p.W);
    return peak_at(gm + (size_t)c * vol, z, y, x, p.D, p.H, p.W, p.thr);
}

__global__ void __launch_bounds__(PEAK_BLOCK) peak_count_kernel(PeakParams p)
{
    __shared__ int part[PEAK_BLOCK / 64];
    const int m = blockIdx.x;
    const long long E = (long long)p.C * p.D * p.H * p.W;
    const float *gm = p.grid + (size_t)m * E;
    int n = 0;
    for (long long e = threadIdx.x; e < E; e += blockDim.x) {
        int c, z, y, x;
        n += peak_voxel(p, gm, e, c, z, y, x) ? 1 : 0;
    }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
        n += __shfl_xor(n, s, 64);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
            t += part[w];
        p.offsets[m + 1] = t;
    }
}

// one workgroup: offsets[1..n] hold counts on entry, clamped inclusive
// bounds on exit; offsets[0] = 0; *n_found = the unclamped total
__global__ void __launch_bounds__(1024) peak_scan_kernel(PeakParams p)
{
    __shared__ long long buf[1024];
    __shared__ long long carry;
    if (threadIdx.x == 0) {
        carry = 0;
        p.offsets[0] = 0;
    }
    __syncthreads();
    for (int base = 0; base < p.n_mol; base += blockDim.x) {
        const int i = base + threadIdx.x;
        buf[threadIdx.x] = i < p.n_mol ? (long long)p.offsets[i + 1] : 0;
        __syncthreads();
        for (int s = 1; s < (int)blockDim.x; s <<= 1) {
            const long long add = threadIdx.x >= (unsigned)s ? buf[threadIdx.x - s] : 0;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        const long long incl = carry + buf[threadIdx.x];
        if (i < p.n_mol)
            p.offsets[i + 1] = (int32_t)(incl < p.capacity ? incl : p.capacity);
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1)
            carry = incl;
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *p.n_found = carry;
}

__global__ void __launch_bounds__(PEAK_BLOCK) peak_write_kernel(PeakParams p)
{
    __shared__ int wcount[PEAK_BLOCK / 64];
    const int m = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long E = (long long)p.C * p.D * p.H * p.W;
    const float *gm = p.grid + (size_t)m * E;
    float o[3], h[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        o[q] = p.origins ? p.origins[3 * (size_t)m + q] : p.o[q];
        h[q] = p.spacings ? p.spacings[3 * (size_t)m + q] : p.h[q];
    }
    long long next = p.offsets[m];   // clamped: below capacity it is exact
    for (long long e0 = 0; e0 < E; e0 += blockDim.x) {
        const long long e = e0 + threadIdx.x;
        int c = 0, z = 0, y = 0, x = 0;
        const bool pk = e < E && peak_voxel(p, gm, e, c, z, y, x);
        const unsigned long long bal = __ballot(pk);
        if (lane == 0)
            wcount[wave] = __popcll(bal);
        __syncthreads();
        long long before = next;
        int total = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            if (w < wave)
                before += wcount[w];
            total += wcount[w];
        }
        const unsigned long long below = lane ? (bal & (~0ull >> (64 - lane))) : 0ull;
        const long long pos = before + __popcll(below);
        if (pk && pos < p.capacity) {
            const int idx[3] = {x, y, z};
#pragma unroll
            for (int q = 0; q < 3; ++q)
                p.xyz[3 * pos + q] = centre_rounded(o[q], idx[q], h[q]);
            p.types[pos] = c;
        }
        next += total;
        __syncthreads();
    }
}

// residual = 2 (G - target) in place over G, per-chunk partial sums of
// (G - target)^2 as float-float pairs (chunk = RES_BLOCK * RES_PER_THREAD
// elements of one structure; lanes' FP32 sums combined in a fixed order)
__global__ void __launch_bounds__(RES_BLOCK) residual_kernel(GridParams p, long long per_mol,
                                                            int nchunk, float2 *partial)
{
    __shared__ float part[2][RES_BLOCK / 64];
    const long long chunk = blockIdx.x;
    const int m = (int)(chunk / nchunk);
    const long long k = chunk - (long long)m * nchunk;
    float *g = (float *)p.out + (size_t)m * per_mol;
    const float *t = p.target + (size_t)m * per_mol;
    const long long base = k * (RES_BLOCK * RES_PER_THREAD);
    float sq = 0.f;
#pragma unroll 4
    for (int j = 0; j < RES_PER_THREAD; ++j) {
        const long long e = base + (long long)j * RES_BLOCK + threadIdx.x;
        if (e < per_mol) {
            const float r = g[e] - t[e];
            sq = __builtin_fmaf(r, r, sq);
            g[e] = 2.f * r;
        }
    }
    float sh, sl;
    ff_wave_sum(sq, sh, sl);
    if ((threadIdx.x & 63) == 0) {
        part[0][threadIdx.x >> 6] = sh;
        part[1][threadIdx.x >> 6] = sl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float ah = 0.f, al = 0.f;
        for (int w = 0; w < RES_BLOCK / 64; ++w)
            ff_add(ah, al, part[0][w], part[1][w]);
        partial[chunk] = make_float2(ah, al);
    }
}

__global__ void loss_finish_kernel(GridParams p, int nchunk, const float2 *partial)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= p.n_mol)
        return;
    float ah = 0.f, al = 0.f;
    for (int k = 0; k < nchunk; ++k) {
        const float2 v = partial[(size_t)m * nchunk + k];
        ff_add(ah, al, v.x, v.y);
    }
    p.loss[m] = ah + al;
}

}  // namespace

hipError_t launch_peaks(const PeakParams &p, hipStream_t s)
{
    if (p.n_mol == 0) {
        // an empty batch still gets offsets[0] = 0 and a zero total
        hipLaunchKernelGGL(peak_scan_kernel, dim3(1), dim3(1024), 0, s, p);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(peak_count_kernel, dim3(p.n_mol), dim3(PEAK_BLOCK), 0, s, p);
    hipLaunchKernelGGL(peak_scan_kernel, dim3(1), dim3(1024), 0, s, p);
    hipLaunchKernelGGL(peak_write_kernel, dim3(p.n_mol), dim3(PEAK_BLOCK), 0, s, p);
    return hipGetLastError();
}

int residual_chunks(long long per_mol)
{
    const long long ch = (long long)RES_BLOCK * RES_PER_THREAD;
    return (int)((per_mol + ch - 1) / ch);
}

hipError_t launch_residual(const GridParams &p, float2 *partial, hipStream_t s)
{
    if (p.n_mol == 0)
        return hipSuccess;
    const long long per_mol = (long long)p.C * p.D * p.H * p.W;
    const int nchunk = residual_chunks(per_mol);
    const long long blocks = (long long)p.n_mol * nchunk;
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)blocks), dim3(RES_BLOCK), 0, s, p, per_mol,
                       nchunk, partial);
    hipLaunchKernelGGL(loss_finish_kernel, dim3((p.n_mol + 255) / 256), dim3(256), 0, s, p, nchunk,
                       (const float2 *)partial);
    return hipGetLastError();
}

}  // namespace pg
