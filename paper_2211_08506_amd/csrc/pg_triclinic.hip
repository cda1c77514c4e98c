// pg_triclinic.hip -- triclinic periodic cells on gfx950 (§III-A lattice
// translations for a general cell).
//
// A triclinic request is turned into a non-periodic one over lattice
// images.  Atom a has the K candidate images mu + M n, n = k - floor(M^-1 mu)
// for the host's fixed range of k (the images of the home-cell copy that
// can reach the grid); their positions are the exact sums
// mu_alpha + n_0 M[alpha][0] + n_1 M[alpha][1] + n_2 M[alpha][2] rounded
// once to float32 (no FP64 on the GPU).  The cell keeps the cutoff cubes of distinct
// images of one atom apart, so each voxel sees at most one image of an atom
// and the non-periodic map over the images is the periodic map.
//
// Only the images whose cutoff cube can meet the grid box (a conservative
// test, widened by one voxel) are kept, in atom order and then k order:
//   tri_base    one thread per atom: the lattice index of its first candidate;
//   tri_pos     one thread per (atom, candidate image): the position, or NaN
//               for an image that misses the grid, in a candidate buffer;
//   tri_count   one thread per atom counts its kept images; each 256-atom
//               block scans its counts (the atoms' starts within the block)
//               and writes its total;
//   tri_scan    one workgroup: exclusive scan of the block totals and the
//               image batch's CSR bounds;
//   tri_write   one thread per atom: its global start (block start + start
//               within the block, kept for the gradient pass) and its kept
//               images.
// Images a test keeps but that miss the grid just have empty windows.  The
// coordinate gradient of an atom is the sum of its images' gradients (each
// image is a translate of the atom), summed in image order.
#include <algorithm>

#include "pg_device.hpp"
#include "pg_launch.hpp"

namespace pg {

namespace {

// The exact lattice sum mu + n_0 m_0 + n_1 m_1 + n_2 m_2 (n_j integers held
// exactly as floats, m_j the cell's float entries) rounded once to float32,
// to nearest, ties to even.  A float-float sum of the seven exact terms
// decides whenever it lies farther than its error bound from a rounding
// midpoint (or is exact); otherwise the exact expansion of the terms decides: its largest
// component is within one ulp of the sum, and the exact sign of the sum
// minus the midpoint on the side of the remainder picks the neighbour.
__device__ float lattice_coord(float mu, const float (&nf)[3], const float (&m)[3])
{
    float t[7];
    t[0] = mu;
#pragma unroll
    for (int j = 0; j < 3; ++j)
        two_prod(nf[j], m[j], t[1 + 2 * j], t[2 + 2 * j]);
    float hi = t[0], lo = 0.f, mag = fabsf(t[0]);
    bool inexact = false;   // some rounding of the low part lost bits
#pragma unroll
    for (int k = 1; k < 7; ++k) {
        float s, e, l, e2;
        two_sum(hi, t[k], s, e);
        hi = s;
        two_sum(lo, e, l, e2);
        lo = l;
        inexact = inexact || e2 != 0.f;
        mag += fabsf(t[k]);
    }
    // hi + lo is then the exact sum, and its float addition rounds it once
    // (ties to even): the common case, ties included (lattice sums of
    // dyadic entries that cross a binade are ties)
    if (!inexact)
        return hi + lo;
    // hi + lo is the sum to within 2^-43 mag; c its rounding, r the rest;
    // halfw: half the gap from c to its neighbour on the side of r (the
    // neighbour one bit pattern away from or towards zero)
    const float c = hi + lo;
    const float r = (hi - c) + lo;
    const float bound = mag * 0x1p-40f;
    const uint32_t cb = __float_as_uint(c) & 0x7fffffffu;
    const bool away = (r >= 0.f) == (c >= 0.f);
    const float halfw = cb == 0u || cb >= 0x7f800000u
                            ? 0.f
                            : 0.5f * (away ? __uint_as_float(cb + 1u) - fabsf(c)
                                           : fabsf(c) - __uint_as_float(cb - 1u));
    if (halfw > 4.f * bound && fabsf(r) < halfw - bound)
        return c;
    // exact: the terms as a non-overlapping expansion of increasing
    // magnitude (grow-expansion); its top component ct is within one ulp
    float e[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        float q = t[k];
#pragma unroll
        for (int j = 0; j < k; ++j) {
            float s, h;
            two_sum(q, e[j], s, h);
            e[j] = h;
            q = s;
        }
        e[k] = q;
    }
    float ct = 0.f, below = 0.f;   // top component and the next non-zero one
#pragma unroll
    for (int k = 0; k < 7; ++k)
        if (e[k] != 0.f) {
            below = ct;
            ct = e[k];
        }
    if (below == 0.f)
        return ct;                   // the sum is a float
    const float nb = nextafterf(ct, below > 0.f ? __builtin_huge_valf() : -__builtin_huge_valf());
    const float mid = 0.5f * (nb - ct);   // the midpoint is ct + mid
    const float u[9] = {t[0], t[1], t[2], t[3], t[4], t[5], t[6], -ct, -mid};
    const int sg = exact_sign(u);
    if (sg == 0)
        return (__float_as_uint(ct) & 1u) ? nb : ct;
    return (sg > 0) == (mid > 0.f) ? nb : ct;
}

// The lattice index of candidate image 0 of an atom at mu: klo - floor(M^-1
// mu), the floor of the home-cell copy taken from a float-float evaluation
// of M^-1 mu (the host's lattice range has a margin, so an off-by-one floor
// next to an integer loses no image that reaches the grid).
__device__ __forceinline__ void tri_base(const TriParams &q, const float mu[3], float nb[3])
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        float fh = 0.f, fl = 0.f;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            float p, pe, p2, pe2;
            two_prod(q.Minv_hi[3 * j + i], mu[i], p, pe);
            two_prod(q.Minv_lo[3 * j + i], mu[i], p2, pe2);
            ff_add(fh, fl, p, pe);
            ff_add(fh, fl, p2, pe2);
        }
        float fi = floorf(fh);
        if (fi == fh && fl < 0.f)
            fi -= 1.f;
        nb[j] = (float)q.klo[j] - fi;
    }
}

// Position of candidate image k of an atom at mu (lattice index nb + the
// digits of k); true when its cutoff cube (half-width rc) can meet the grid
// box [o, o + N h] of its structure.  The position is exact
// (lattice_coord).  No FP64 on the GPU.
__device__ __forceinline__ bool tri_image(const TriParams &q, const float mu[3], const float nb[3],
                                          int k, float rc, const float o[3], float pos[3])
{
    const float nf[3] = {nb[0] + (float)(k % q.kdim[0]),
                         nb[1] + (float)((k / q.kdim[0]) % q.kdim[1]),
                         nb[2] + (float)(k / (q.kdim[0] * q.kdim[1]))};
    bool reach = true;
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        const float m[3] = {q.M[3 * al], q.M[3 * al + 1], q.M[3 * al + 2]};
        pos[al] = lattice_coord(mu[al], nf, m);
        const float lo = o[al] - rc - q.h[al], hi = o[al] + (float)q.N[al] * q.h[al] + rc + q.h[al];
        reach = reach && pos[al] >= lo && pos[al] <= hi;
    }
    return reach;
}

struct AtomIn {
    float mu[3], o[3], rc;
    int t;
    bool ok;
};

__device__ __forceinline__ AtomIn tri_atom(const TriParams &q, long long a)
{
    AtomIn A;
    A.mu[0] = q.xyz[3 * a];
    A.mu[1] = q.xyz[3 * a + 1];
    A.mu[2] = q.xyz[3 * a + 2];
    A.t = q.types[a];
    A.ok = atom_valid(A.mu[0], A.mu[1], A.mu[2], A.t, q.n_sig);
    A.rc = A.ok ? q.rc[A.t] : 0.f;
    const int m = q.origins ? structure_of(q.offsets, q.n_mol, a) : 0;
#pragma unroll
    for (int al = 0; al < 3; ++al)
        A.o[al] = q.origins ? q.origins[3 * (size_t)m + al] : q.o[al];
    return A;
}

// One thread per atom: the lattice index of its candidate image 0.
__global__ void __launch_bounds__(256) tri_base_kernel(TriParams q)
{
    const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= q.n_atoms)
        return;
    const float mu[3] = {q.xyz[3 * a], q.xyz[3 * a + 1], q.xyz[3 * a + 2]};
    float nb[3];
    tri_base(q, mu, nb);
#pragma unroll
    for (int j = 0; j < 3; ++j)
        q.base[3 * a + j] = nb[j];
}

// One thread per (atom, candidate image k): the image's position, or NaN
// when its cutoff cube cannot meet the grid (or the atom is invalid), into
// cand[k][a] (consecutive atoms contiguous).
__global__ void __launch_bounds__(256) tri_pos_kernel(TriParams q, DeviceError *err)
{
    const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (a >= q.n_atoms)
        return;
    const AtomIn A = tri_atom(q, a);
    float pos[3];
    bool keep = false;
    if (!A.ok) {
        if (k == 0)
            raise_error(err, PG_E_DEVICE_DATA, a);
    } else {
        const float nb[3] = {q.base[3 * a], q.base[3 * a + 1], q.base[3 * a + 2]};
        keep = tri_image(q, A.mu, nb, k, A.rc, A.o, pos);
    }
    float *c = q.cand + 3 * ((size_t)k * q.n_atoms + a);
    c[0] = keep ? pos[0] : __builtin_nanf("");
    c[1] = keep ? pos[1] : 0.f;
    c[2] = keep ? pos[2] : 0.f;
}

// One thread per atom: its kept images, counted from the candidates, and
// their exclusive scan within the 256-atom block (wave scans by shuffles,
// then the waves' totals); the block's total goes to bsum.
__global__ void __launch_bounds__(256) tri_count_kernel(TriParams q)
{
    __shared__ uint32_t wsum[4];
    const long long a = (long long)blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t n = 0;
    if (a < q.n_atoms)
        for (int k = 0; k < q.K; ++k)
            n += __builtin_isnan(q.cand[3 * ((size_t)k * q.n_atoms + a)]) ? 0u : 1u;
    uint32_t inc = n;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)inc, d, 64);
        if (lane >= d)
            inc += v;
    }
    if (lane == 63)
        wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0u;
    for (int i = 0; i < w; ++i)
        before += wsum[i];
    if (a < q.n_atoms)
        q.istart[a] = (int32_t)(before + inc - n);
    if (threadIdx.x == 255)
        q.bsum[blockIdx.x] = before + inc;
}

// one workgroup: the block totals -> their exclusive scan (each block's
// first image), istart[n] = total; exp_offsets[m] = the global start of
// atom offsets[m] (its start within its block + the block's start)
__global__ void __launch_bounds__(1024) tri_scan_kernel(TriParams q, DeviceError *err)
{
    __shared__ unsigned long long part[1024];
    const int t = threadIdx.x;
    const long long n = q.n_atoms, nb = (n + 255) / 256;
    const unsigned long long total = workgroup_exclusive_scan(q.bsum, q.bsum, nb, part);
    if (t == 1023) {
        q.istart[n] = (int32_t)total;
        // more kept images than the host bound (not expected: the bound is
        // the most lattice translates the widened box holds): report it
        if (total > (unsigned long long)q.bound)
            raise_error(err, PG_E_CAPACITY, 0);
    }
    __syncthreads();
    for (long long m = t; m <= (long long)q.n_mol; m += 1024) {
        long long om = q.offsets[m];       // device data: clamp into [0, n]
        om = om < 0 ? 0 : (om > n ? n : om);
        q.exp_offsets[m] = om == n ? q.istart[n] : (int32_t)(q.istart[om] + q.bsum[om >> 8]);
    }
}

// One thread per atom: its kept images, in k order, from its global start on.
__global__ void __launch_bounds__(256) tri_write_kernel(TriParams q)
{
    const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= q.n_atoms)
        return;
    long long j = (long long)q.istart[a] + q.bsum[a >> 8];
    q.istart[a] = (int32_t)j;   // the global start, for the gradient pass
    const int t = q.types[a];
    for (int k = 0; k < q.K; ++k) {
        const float *c = q.cand + 3 * ((size_t)k * q.n_atoms + a);
        if (!__builtin_isnan(c[0])) {
            q.exp_xyz[3 * j + 0] = c[0];
            q.exp_xyz[3 * j + 1] = c[1];
            q.exp_xyz[3 * j + 2] = c[2];
            q.exp_types[j] = t;
            ++j;
        }
    }
}

__global__ void __launch_bounds__(256) tri_reduce_kernel(TriParams q)
{
    const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= q.n_atoms || !q.grad)
        return;
    float g[3] = {0.f, 0.f, 0.f};
    for (long long i = q.istart[a]; i < q.istart[a + 1]; ++i) {
        g[0] += q.grad_img[3 * i + 0];
        g[1] += q.grad_img[3 * i + 1];
        g[2] += q.grad_img[3 * i + 2];
    }
#pragma unroll
    for (int al = 0; al < 3; ++al)
        q.grad[3 * a + al] = g[al];
}

}  // namespace

hipError_t launch_tri_expand(const TriParams &q, DeviceError *err, hipStream_t s)
{
    const long long grid = std::max<long long>((q.n_atoms + 255) / 256, 1);
    hipLaunchKernelGGL(tri_base_kernel, dim3((unsigned)grid), dim3(256), 0, s, q);
    hipLaunchKernelGGL(tri_pos_kernel, dim3((unsigned)grid, (unsigned)q.K), dim3(256), 0, s, q, err);
    hipLaunchKernelGGL(tri_count_kernel, dim3((unsigned)grid), dim3(256), 0, s, q);
    hipLaunchKernelGGL(tri_scan_kernel, dim3(1), dim3(1024), 0, s, q, err);
    hipLaunchKernelGGL(tri_write_kernel, dim3((unsigned)grid), dim3(256), 0, s, q);
    return hipGetLastError();
}

hipError_t launch_tri_reduce(const TriParams &q, hipStream_t s)
{
    if (q.n_atoms == 0)
        return hipSuccess;
    const long long grid = (q.n_atoms + 255) / 256;
    hipLaunchKernelGGL(tri_reduce_kernel, dim3((unsigned)grid), dim3(256), 0, s, q);
    return hipGetLastError();
}

}  // namespace pg
