// pg_plain.hip -- the baseline ("plain") form on gfx950.
//
// prep:  one thread per atom computes the atom's exact per-axis window
//        ranges (and nearest-image bases) into the workspace.
// plain: one launch per structure, one thread per output element; each
//        thread visits every atom of its structure, tests the three axis
//        windows and adds the 3-D Gaussian exp(-|r - mu|^2 / (2 sigma^2))
//        (§III-A Eq. 1, point-sampled, without the prefactor), or for the box
//        form the product of the three per-axis voxel masses (with weighted
//        channels: every atom, times its weight for the channel; with the
//        sphere cutoff, only voxels whose summed squared offsets are within
//        rc^2).  This is the
//        straightforward GPU transcription of the definition; the batched
//        window kernel is measured against it.
#include "pg_device.hpp"
#include "pg_launch.hpp"

namespace pg {

__global__ void __launch_bounds__(256) prep_kernel(GridParams p)
{
    const long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= live_atoms(p))
        return;
    write_atom_window(p, a, (AtomWindow *)p.ws + a);
}

template <typename T>
__global__ void __launch_bounds__(256) plain_kernel(GridParams p)
{
    const int m = p.mol_index;
    const size_t plane = (size_t)p.H * p.W, vol = (size_t)p.D * plane;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)p.C * vol)
        return;
    const int c = (int)(e / vol);
    const size_t r0 = e - (size_t)c * vol;
    const int iz = (int)(r0 / plane);
    const size_t r1 = r0 - (size_t)iz * plane;
    const int iy = (int)(r1 / p.W);
    const int ix = (int)(r1 - (size_t)iy * p.W);
    const int idx[3] = {ix, iy, iz};
    float h[3];
    for (int q = 0; q < 3; ++q)
        h[q] = p.spacings ? p.spacings[3 * m + q] : p.h[q];
    const AtomWindow *tab = (const AtomWindow *)p.ws;
    int a0 = p.offsets[m], a1 = p.offsets[m + 1];
    if (a0 < 0 || a1 < a0 || (long long)a1 > p.n_atoms)
        a0 = a1 = 0;   // malformed offsets: nothing is read
    const bool box = p.box != 0;
    const float *wts = p.weights;
    float acc = 0.f;
    for (int a = a0; a < a1; ++a) {
        const int t = tab[a].type;
        float wgt = 1.f;
        if (wts) {
            // weighted channels: every valid atom, scaled by its weight
            if (t < 0)
                continue;
            wgt = wts[(size_t)a * p.C + c];
            if (wgt == 0.f)
                continue;
        } else if (t != c) {
            continue;
        }
        const float inv2s2 = p.inv2s2[t], isq2s = p.isq2s[t];
        float d2 = 0.f, mass = 1.f;
        bool inside = true;
        for (int q = 0; q < 3 && inside; ++q) {
            bool hit = false;
            for (int r = 0; r < tab[a].n[q]; ++r) {
                if (idx[q] >= tab[a].lo[q][r] && idx[q] <= tab[a].hi[q][r]) {
                    const float bh = tab[a].bh[q][r], bl = tab[a].bl[q][r];
                    if (box)
                        mass *= box1d(edge_at(bh, bl, h[q], idx[q]), edge_at(bh, bl, h[q], idx[q] + 1),
                                      isq2s);
                    if (!box || p.sphere) {
                        const float d = offset_at(bh, bl, h[q], idx[q]);
                        d2 = __builtin_fmaf(d, d, d2);
                    }
                    hit = true;
                }
            }
            inside = hit;
        }
        if (inside && p.sphere && !(d2 <= p.rc2[t]))
            inside = false;
        if (inside) {
            const float v = box ? mass : expf(-d2 * inv2s2);
            acc += wts ? wgt * v : v;
        }
    }
    const float v[1] = {acc};
    store_vec<T, 1>((T *)p.out + (size_t)m * p.C * vol + e, v, false);
}

hipError_t launch_prep(const GridParams &p, hipStream_t s)
{
    if (p.n_atoms == 0)
        return hipSuccess;
    const int block = 256;
    const long long grid = (p.n_atoms + block - 1) / block;
    hipLaunchKernelGGL(prep_kernel, dim3((unsigned)grid), dim3(block), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_plain(const GridParams &p, int out_dtype, hipStream_t s)
{
    const size_t n = (size_t)p.C * p.D * p.H * p.W;
    const int block = 256;
    const size_t grid = (n + block - 1) / block;
    if (out_dtype == PG_OUT_F32)
        hipLaunchKernelGGL(plain_kernel<float>, dim3((unsigned)grid), dim3(block), 0, s, p);
    else
        hipLaunchKernelGGL(plain_kernel<__bf16>, dim3((unsigned)grid), dim3(block), 0, s, p);
    return hipGetLastError();
}

}  // namespace pg
