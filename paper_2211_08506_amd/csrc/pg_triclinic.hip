// pg_triclinic.hip -- triclinic periodic cells on gfx950 (§III-A lattice
// translations for a general cell).
//
// A triclinic request is turned into a non-periodic one over lattice
// images.  Atom a has the K candidate images mu + M n, n = k - floor(M^-1 mu)
// for the host's fixed range of k (the images of the home-cell copy that
// can reach the grid); their positions are
// fl32(mu_alpha + ((n_0 M[alpha][0] + n_1 M[alpha][1]) + n_2 M[alpha][2]))
// in double, in that order.  The cell keeps the cutoff cubes of distinct
// images of one atom apart, so each voxel sees at most one image of an atom
// and the non-periodic map over the images is the periodic map.
//
// Only the images whose cutoff cube can meet the grid box (a conservative
// test, widened by one voxel) are kept, in atom order and then k order:
//   tri_count   one thread per atom counts its kept images;
//   tri_scan    one workgroup: exclusive scan of the counts (image start of
//               each atom) and the image batch's CSR bounds;
//   tri_write   one thread per atom writes its kept images.
// Images a test keeps but that miss the grid just have empty windows.  The
// coordinate gradient of an atom is the sum of its images' gradients (each
// image is a translate of the atom), summed in image order.
#include <algorithm>

#include "pg_device.hpp"
#include "pg_launch.hpp"

namespace pg {

namespace {

// Position of candidate image k of an atom at mu; true when its cutoff
// cube (half-width rc) can meet the grid box [o, o + N h] of its structure.
__device__ __forceinline__ bool tri_image(const TriParams &q, const float mu[3], int k, float rc,
                                          const float o[3], float pos[3])
{
    int kk[3];
    kk[0] = k % q.kdim[0];
    kk[1] = (k / q.kdim[0]) % q.kdim[1];
    kk[2] = k / (q.kdim[0] * q.kdim[1]);
    double n[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double f = q.Minv[3 * j + 0] * (double)mu[0] + q.Minv[3 * j + 1] * (double)mu[1] +
                         q.Minv[3 * j + 2] * (double)mu[2];
        n[j] = (double)(q.klo[j] + kk[j]) - floor(f);
    }
    bool reach = true;
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        double s = n[0] * q.M[3 * al + 0];
        s = s + n[1] * q.M[3 * al + 1];
        s = s + n[2] * q.M[3 * al + 2];
        pos[al] = (float)((double)mu[al] + s);
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
    const int m = structure_of(q.offsets, q.n_mol, a);
#pragma unroll
    for (int al = 0; al < 3; ++al)
        A.o[al] = q.origins ? q.origins[3 * (size_t)m + al] : q.o[al];
    return A;
}

__global__ void __launch_bounds__(256) tri_count_kernel(TriParams q, DeviceError *err)
{
    const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= q.n_atoms)
        return;
    const AtomIn A = tri_atom(q, a);
    int n = 0;
    if (!A.ok) {
        raise_error(err, PG_E_DEVICE_DATA, a);
    } else {
        for (int k = 0; k < q.K; ++k) {
            float pos[3];
            n += tri_image(q, A.mu, k, A.rc, A.o, pos) ? 1 : 0;
        }
    }
    q.istart[a] = n;
}

// one workgroup: istart[0..n) counts -> exclusive scan, istart[n] = total;
// exp_offsets[m] = istart[offsets[m]]
__global__ void __launch_bounds__(1024) tri_scan_kernel(TriParams q, DeviceError *err)
{
    __shared__ unsigned long long part[1024];
    const int t = threadIdx.x;
    const long long n = q.n_atoms;
    const unsigned long long total =
        workgroup_exclusive_scan((const uint32_t *)q.istart, (uint32_t *)q.istart, n, part);
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
        q.exp_offsets[m] = q.istart[om];
    }
}

__global__ void __launch_bounds__(256) tri_write_kernel(TriParams q)
{
    const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= q.n_atoms)
        return;
    const AtomIn A = tri_atom(q, a);
    if (!A.ok)
        return;
    long long j = q.istart[a];
    const long long j_end = q.istart[a + 1];
    for (int k = 0; k < q.K && j < j_end; ++k) {
        float pos[3];
        if (tri_image(q, A.mu, k, A.rc, A.o, pos)) {
            q.exp_xyz[3 * j + 0] = pos[0];
            q.exp_xyz[3 * j + 1] = pos[1];
            q.exp_xyz[3 * j + 2] = pos[2];
            q.exp_types[j] = A.t;
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
    hipLaunchKernelGGL(tri_count_kernel, dim3((unsigned)grid), dim3(256), 0, s, q, err);
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
