// pg_triclinic.hip -- triclinic periodic cells on gfx950 (§III-A lattice
// translations for a general cell).
//
// A triclinic request is turned into a non-periodic one over lattice
// images: every atom a becomes the K images mu + M n, n = k - floor(M^-1 mu)
// for the host's fixed range of k (the images of the home-cell copy that
// can reach the grid), stored at index a * K + k.  Image positions are
// fl32(mu_alpha + ((n_0 M[alpha][0] + n_1 M[alpha][1]) + n_2 M[alpha][2]))
// in double, in that order; images that cannot reach the grid simply get
// empty windows downstream.  The cell keeps the cutoff cubes of distinct
// images of one atom apart, so each voxel sees at most one image of an
// atom and the non-periodic map over the images is the periodic map.
//
// The coordinate gradient of an atom is the sum of its images' gradients
// (each image is a translate of the atom), summed in k order.
#include <algorithm>

#include "pg_device.hpp"
#include "pg_launch.hpp"

namespace pg {

namespace {

__global__ void __launch_bounds__(256) tri_expand_kernel(TriParams q, DeviceError *err,
                                                          int n_sig)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = q.n_atoms * q.K;
    if (i < (long long)q.n_mol + 1)
        q.exp_offsets[i] = q.offsets[i] * q.K;
    if (i >= total)
        return;
    const long long a = i / q.K;
    const int k = (int)(i - a * q.K);
    const float mu[3] = {q.xyz[3 * a], q.xyz[3 * a + 1], q.xyz[3 * a + 2]};
    const int t = q.types[a];
    const bool ok = atom_valid(mu[0], mu[1], mu[2], t, n_sig);
    if (!ok) {
        if (k == 0)
            raise_error(err, PG_E_DEVICE_DATA, a);
        q.exp_types[i] = -1;
        q.exp_xyz[3 * i + 0] = q.exp_xyz[3 * i + 1] = q.exp_xyz[3 * i + 2] = 0.f;
        return;
    }
    // lattice offset of the home-cell copy, then this image's n
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
#pragma unroll
    for (int al = 0; al < 3; ++al) {
        double s = n[0] * q.M[3 * al + 0];
        s = s + n[1] * q.M[3 * al + 1];
        s = s + n[2] * q.M[3 * al + 2];
        q.exp_xyz[3 * i + al] = (float)((double)mu[al] + s);
    }
    q.exp_types[i] = t;
}

__global__ void __launch_bounds__(256) tri_reduce_kernel(TriParams q)
{
    const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= q.n_atoms)
        return;
    float g[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < q.K; ++k) {
        const float *gi = q.grad_img + 3 * (a * q.K + k);
        g[0] += gi[0];
        g[1] += gi[1];
        g[2] += gi[2];
    }
#pragma unroll
    for (int al = 0; al < 3; ++al)
        if (q.grad)
            q.grad[3 * a + al] = g[al];
}

}  // namespace

hipError_t launch_tri_expand(const TriParams &q, DeviceError *err, int n_sig, hipStream_t s)
{
    const long long total = std::max<long long>(q.n_atoms * q.K, (long long)q.n_mol + 1);
    const long long grid = (total + 255) / 256;
    hipLaunchKernelGGL(tri_expand_kernel, dim3((unsigned)grid), dim3(256), 0, s, q, err, n_sig);
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
