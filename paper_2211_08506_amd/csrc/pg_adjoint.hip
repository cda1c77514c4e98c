// pg_adjoint.hip -- coordinate adjoint of the density grid on gfx950.
//
// For L = sum_v U[v] G[v] with G the product of per-axis factors
// phi_x phi_y phi_z (the point-sampled Gaussian of §III-A Eq. 1, or the
// voxel masses of Eq. 2-5),
//   dL/dmu_{a,x} = sum_{v in window(a)} U[b, t_a, v] phi_x'(v) phi_y(v) phi_z(v),
// and likewise for y and z -- the separable coordinate gradient of §IV-C.
// With weighted channels the atom's upstream is sum_c w_c U[b, c, v], and
// dL/dw_{a,c} = sum_v U[b, c, v] phi_x phi_y phi_z.
// For the point sample phi' = phi d / sigma^2 (d = r - mu, nearest image
// when periodic); for the box, phi' = (g(lower edge) - g(upper edge)) /
// (sqrt(2 pi) sigma).  The cutoff edge contributes nothing (the map is
// differentiable almost everywhere).
//
// One wave per atom, any structure size: the wave builds its atom's 1-D
// factor and offset lists over the window (per-wave LDS), then its lanes
// sweep the window with x fastest -- lanes of one window row read
// consecutive addresses -- and the three partial sums are reduced across
// the wave.  No atomics; each atom's gradient is written by one lane, which
// in a grid-reversal step also writes the updated coordinates
// xyz - lr * gradient.
#include "pg_device.hpp"
#include "pg_launch.hpp"

namespace pg {

constexpr int ADJ_UNROLL = 4;   // window elements per lane whose loads are in flight together

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
        v += __shfl_xor(v, s, 64);
    return v;
}

template <typename T>
__global__ void __launch_bounds__(256) adjoint_kernel(GridParams p)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const long long a = (long long)blockIdx.x * waves + wave;
    const bool active = a < live_atoms(p);
    const int NT = p.W + p.H + p.D;
    // per-wave slice: idx[NT] (int) | phi[NT] | dphi[NT] | dsq[NT] | 3 range records
    int *idx = (int *)(smem + (size_t)wave * (NT * 16 + 3 * sizeof(AxisRanges)));
    float *phi = (float *)(idx + NT);
    float *dphi = phi + NT;
    float *dsq = dphi + NT;      // sphere cutoff: squared centre offsets
    AxisRanges *rg = (AxisRanges *)(dsq + NT);
    const int base[3] = {0, p.W, p.W + p.H};
    const int N[3] = {p.W, p.H, p.D};   // indexed by the compile-time axis only

    float mu[3] = {0.f, 0.f, 0.f};
    int t = -1, m = 0;
    float o[3] = {0.f, 0.f, 0.f}, h[3] = {1.f, 1.f, 1.f};
    if (active) {   // uniform across the wave
        mu[0] = p.xyz[3 * a];
        mu[1] = p.xyz[3 * a + 1];
        mu[2] = p.xyz[3 * a + 2];
        t = p.types[a];
        m = structure_of_wave(p.offsets, p.n_mol, a);
        if (!atom_valid(mu[0], mu[1], mu[2], t, p.n_sig)) {
            if (lane == 0)
                raise_error(p.err, PG_E_DEVICE_DATA, a);
            t = -1;
        } else {
            for (int q = 0; q < 3; ++q) {
                o[q] = p.origins ? p.origins[3 * m + q] : p.o[q];
                h[q] = p.spacings ? p.spacings[3 * m + q] : p.h[q];
            }
        }
    }
    // lanes 0..2: window ranges of the three axes
    if (t >= 0 && lane < 3) {
        const int q = lane;
        const float oq = q == 0 ? o[0] : (q == 1 ? o[1] : o[2]);
        const float hq = q == 0 ? h[0] : (q == 1 ? h[1] : h[2]);
        const float mq = q == 0 ? mu[0] : (q == 1 ? mu[1] : mu[2]);
        const float Lq = q == 0 ? p.L[0] : (q == 1 ? p.L[1] : p.L[2]);
        axis_ranges(oq, hq, N[q], mq, p.periodic != 0, Lq, p.rc[t], p.cut != 0, rg[q]);
    }
    __syncthreads();
    int n[3] = {0, 0, 0};
    if (t >= 0) {
        for (int q = 0; q < 3; ++q) {
            const AxisRanges &R = rg[q];
            int k0 = 0;
            for (int r = 0; r < R.n; ++r) {
                const int len = R.hi[r] - R.lo[r] + 1;
                for (int k = lane; k < len; k += 64) {
                    const int i = R.lo[r] + k;
                    idx[base[q] + k0 + k] = i;
                    phi[base[q] + k0 + k] = factor1d(p.box != 0, R.bh[r], R.bl[r], h[q], i,
                                                     p.inv2s2[t], p.isq2s[t]);
                    dphi[base[q] + k0 + k] = dfactor1d(p.box != 0, R.bh[r], R.bl[r], h[q], i,
                                                       p.inv2s2[t], p.invs2[t], p.inorm[t]);
                    if (p.sphere) {
                        const float d = offset_at(R.bh[r], R.bl[r], h[q], i);
                        dsq[base[q] + k0 + k] = d * d;
                    }
                }
                k0 += len;
            }
            n[q] = k0;
        }
    }
    __syncthreads();
    float gx = 0.f, gy = 0.f, gz = 0.f;
    const bool wtd = p.weights != nullptr;
    if (t >= 0) {
        const size_t plane = (size_t)p.H * p.W;
        const int nx = n[0], ny = n[1], nz = n[2];
        const int total = nx * ny * nz;
        // unweighted: the atom's own channel; weighted: every channel, each
        // swept with its weight (and its weight gradient when asked for)
        const int c0 = wtd ? 0 : t, c1 = wtd ? p.C : t + 1;
        const bool want_gw = wtd && p.grad_w != nullptr;
        for (int c = c0; c < c1; ++c) {
            const float wc = wtd ? p.weights[(size_t)a * p.C + c] : 1.f;
            if (wc == 0.f && !want_gw)
                continue;
            const T *U = (const T *)p.out + ((size_t)m * p.C + c) * (size_t)p.D * plane;
            float sx = 0.f, sy = 0.f, sz = 0.f, sw = 0.f;
            // ADJ_UNROLL window elements per lane per round: their upstream
            // loads are issued together, then consumed in element order
            for (int e0 = 0; e0 < total; e0 += 64 * ADJ_UNROLL) {
                float u[ADJ_UNROLL];
                int ke[ADJ_UNROLL][3];
#pragma unroll
                for (int j = 0; j < ADJ_UNROLL; ++j) {
                    const int e = e0 + 64 * j + lane;
                    const int kx = e % nx;
                    const int r = e / nx;
                    const int ky = r % ny;
                    const int kz = r / ny;
                    ke[j][0] = kx;
                    ke[j][1] = ky;
                    ke[j][2] = kz;
                    bool in = e < total;
                    if (in && p.sphere)
                        in = dsq[kx] <= (p.rc2[t] - dsq[base[2] + kz]) - dsq[base[1] + ky];
                    u[j] = 0.f;
                    if (in) {
                        const int ix = idx[kx], iy = idx[base[1] + ky], iz = idx[base[2] + kz];
                        u[j] = load_as_float<T>(U + (size_t)iz * plane + (size_t)iy * p.W + ix);
                    } else {
                        ke[j][0] = -1;
                    }
                }
#pragma unroll
                for (int j = 0; j < ADJ_UNROLL; ++j) {
                    if (ke[j][0] < 0)
                        continue;
                    const int kx = ke[j][0], ky = ke[j][1], kz = ke[j][2];
                    const float fx = phi[kx], fy = phi[base[1] + ky], fz = phi[base[2] + kz];
                    const float dx = dphi[kx], dy = dphi[base[1] + ky], dz = dphi[base[2] + kz];
                    sx = __builtin_fmaf(u[j], dx * (fy * fz), sx);
                    sy = __builtin_fmaf(u[j], fx * (dy * fz), sy);
                    sz = __builtin_fmaf(u[j], (fx * fy) * dz, sz);
                    if (want_gw)
                        sw = __builtin_fmaf(u[j], (fx * fy) * fz, sw);
                }
            }
            if (want_gw) {
                sw = wave_sum(sw);
                if (lane == 0)
                    p.grad_w[(size_t)a * p.C + c] = sw;
            }
            if (wtd) {
                gx = __builtin_fmaf(wc, sx, gx);
                gy = __builtin_fmaf(wc, sy, gy);
                gz = __builtin_fmaf(wc, sz, gz);
            } else {
                gx = sx;
                gy = sy;
                gz = sz;
            }
        }
    }
    gx = wave_sum(gx);
    gy = wave_sum(gy);
    gz = wave_sum(gz);
    if (active && lane == 0 && t < 0 && wtd && p.grad_w) {
        for (int c = 0; c < p.C; ++c)
            p.grad_w[(size_t)a * p.C + c] = 0.f;
    }
    if (active && lane == 0) {
        const float g[3] = {t >= 0 ? gx : 0.f, t >= 0 ? gy : 0.f, t >= 0 ? gz : 0.f};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (p.grad_xyz)
                p.grad_xyz[3 * a + q] = g[q];
            // a grid-reversal step: the coordinate update (only this wave
            // reads or writes atom a, so xyz_upd may alias xyz)
            if (p.xyz_upd)
                p.xyz_upd[3 * a + q] = __builtin_fmaf(-p.lr, g[q], mu[q]);
        }
    }
}

hipError_t launch_adjoint(const GridParams &p, int grad_dtype, hipStream_t s)
{
    if (p.n_atoms == 0)
        return hipSuccess;
    const int block = 256, waves = block / 64;
    const size_t lds = (size_t)waves * ((size_t)(p.W + p.H + p.D) * 16 + 3 * sizeof(AxisRanges));
    const long long grid = (p.n_atoms + waves - 1) / waves;
    if (grad_dtype == PG_OUT_F32) {
        if (lds > 65536)
            hipFuncSetAttribute((const void *)adjoint_kernel<float>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(adjoint_kernel<float>, dim3((unsigned)grid), dim3(block), lds, s, p);
    } else {
        if (lds > 65536)
            hipFuncSetAttribute((const void *)adjoint_kernel<__bf16>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(adjoint_kernel<__bf16>, dim3((unsigned)grid), dim3(block), lds, s, p);
    }
    return hipGetLastError();
}

}  // namespace pg
