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
// In a grid-reversal step that keeps no residual grid, the upstream value
// 2 (G'(v) - T(v)) is formed at each window voxel: G'(v) is summed over the
// structure's atoms of the same channel exactly as the window kernel sums
// it (index order, the same factors and fused multiply-adds, the same
// sphere test), so the gradient is bit-identical to the one read from a
// stored residual.
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

// Per-wave LDS bytes of the adjoint: the atom's lists over the NT = W + H + D
// indices and its ranges, plus, when recomputing the residual, for up to
// a_cap same-channel atoms their index, flags, order, range records and
// factor rows (and squared offsets for the sphere) over this atom's window
// lists of at most ntw indices.
__host__ __device__ inline size_t adjoint_wave_lds(int NT, int a_cap, int ntw, bool sphere)
{
    return (size_t)NT * 16 + 3 * sizeof(AxisRanges) +
           (size_t)a_cap * (3 * sizeof(int) + 3 * sizeof(RangeRec) +
                            (size_t)ntw * sizeof(float) * (sphere ? 2 : 1));
}

// G'(v) of the atom's channel at window element (kx, ky, kz): the window
// kernel's sum over the same-channel atoms in index order,
// acc = fma(phi_y phi_z, phi_x, acc), from their factor rows over this
// atom's window lists (0 outside an atom's window, where the window kernel
// adds an exact zero), keeping under the sphere cutoff phi_x only where
// dx^2 <= (rc^2 - dz^2) - dy^2.
__device__ __forceinline__ float recompute_density(const float *srow, const float *sd2, int nrel,
                                                   int ntw, int by, int bz, int kx, int ky,
                                                   int kz, bool sph, float rc2)
{
    float acc = 0.f;
    for (int r = 0; r < nrel; ++r) {
        const int o = r * ntw;
        const float fz = srow[o + bz + kz];
        const float fy = srow[o + by + ky];
        const float fx = srow[o + kx];
        if (fz == 0.f || fy == 0.f || fx == 0.f)
            continue;
        if (sph && !(sd2[o + kx] <= (rc2 - sd2[o + bz + kz]) - sd2[o + by + ky]))
            continue;
        acc = __builtin_fmaf(fy * fz, fx, acc);
    }
    return acc;
}

template <typename T, bool RECOMP>
__global__ void __launch_bounds__(256) adjoint_kernel(GridParams p)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const long long a = (long long)blockIdx.x * waves + wave;
    const bool active = a < live_atoms(p);
    const int NT = p.W + p.H + p.D;
    // per-wave slice: idx[NT] (int) | phi[NT] | dphi[NT] | dsq[NT] | 3 range
    // records | recompute: same[a_cap] | flags[a_cap] | rel[a_cap] |
    // range records[a_cap][3] | rows[a_cap][ntw] | (sphere) squared
    // offsets[a_cap][ntw]
    constexpr bool recomp = RECOMP;
    const int rcap = recomp ? p.a_cap : 0, ntw = recomp ? p.rec_ntw : 0;
    unsigned char *slice =
        smem + (size_t)wave * adjoint_wave_lds(p.W + p.H + p.D, rcap, ntw, p.sphere != 0);
    int *idx = (int *)slice;
    float *phi = (float *)(idx + NT);
    float *dphi = phi + NT;
    float *dsq = dphi + NT;      // sphere cutoff: squared centre offsets
    AxisRanges *rg = (AxisRanges *)(dsq + NT);
    int *same = (int *)(rg + 3);
    int *sflag = same + rcap;
    int *rel = sflag + rcap;
    RangeRec *srr = (RangeRec *)(rel + rcap);
    float *srow = (float *)(srr + 3 * rcap);
    float *sd2 = srow + (size_t)rcap * ntw;
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
    // recompute: the structure's first 64 atoms are requested before the
    // range search below, so that latency overlaps it
    long long s0 = 0, s1 = 0;
    int tk = -1;
    float kx = 0.f, ky = 0.f, kz = 0.f;
    if (recomp && t >= 0) {
        s0 = p.offsets[m];
        s1 = p.offsets[m + 1];
        const long long k = s0 + lane;
        if (k < s1) {
            tk = p.types[k];
            kx = p.xyz[3 * k];
            ky = p.xyz[3 * k + 1];
            kz = p.xyz[3 * k + 2];
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
    // recompute: the structure's valid atoms of channel t in index order
    int nsame = 0, nrel = 0;
    if (recomp && t >= 0) {
        for (long long k0 = s0; k0 < s1; k0 += 64) {
            const long long k = k0 + lane;
            if (k0 != s0) {
                tk = -1;
                if (k < s1) {
                    tk = p.types[k];
                    kx = p.xyz[3 * k];
                    ky = p.xyz[3 * k + 1];
                    kz = p.xyz[3 * k + 2];
                }
            }
            const bool hit = k < s1 && tk == t && atom_valid(kx, ky, kz, tk, p.n_sig);
            const unsigned long long bal = __ballot(hit);
            const int rank = nsame + __popcll(bal & ((1ull << lane) - 1ull));
            if (hit && rank < rcap) {
                same[rank] = (int)k;
                sflag[rank] = 0;
            }
            nsame += __popcll(bal);
        }
        nsame = min(nsame, rcap);   // the window plan holds every atom of a structure
    }
    __syncthreads();
    // the window's index, factor and derivative lists of the three axes,
    // built in one pass over their concatenation (lane e takes element e)
    int n[3] = {0, 0, 0};
    if (t >= 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const AxisRanges &R = rg[q];
            int len = 0;
            for (int r = 0; r < R.n; ++r)
                len += R.hi[r] - R.lo[r] + 1;
            n[q] = len;
        }
        const int n01 = n[0] + n[1], nall = n01 + n[2];
        for (int e = lane; e < nall; e += 64) {
            const int q = e < n[0] ? 0 : (e < n01 ? 1 : 2);
            const int eq = e - (q == 0 ? 0 : (q == 1 ? n[0] : n01));   // position in axis q
            const AxisRanges &R = rg[q];
            int r = 0, k = eq;
            while (r + 1 < R.n && k > R.hi[r] - R.lo[r]) {
                k -= R.hi[r] - R.lo[r] + 1;
                ++r;
            }
            const int i = R.lo[r] + k;
            const float hq = q == 0 ? h[0] : (q == 1 ? h[1] : h[2]);
            const int slot = base[q] + eq;
            idx[slot] = i;
            phi[slot] = factor1d(p.box != 0, R.bh[r], R.bl[r], hq, i, p.inv2s2[t], p.isq2s[t]);
            dphi[slot] = dfactor1d(p.box != 0, R.bh[r], R.bl[r], hq, i, p.inv2s2[t], p.invs2[t],
                                   p.inorm[t]);
            if (p.sphere) {
                const float d = offset_at(R.bh[r], R.bl[r], hq, i);
                dsq[slot] = d * d;
            }
        }
    }
    const int wtot = n[0] + n[1] + n[2];
    const bool rec_ok = recomp && t >= 0 && wtot <= ntw;
    if (recomp && t >= 0 && wtot > ntw && lane == 0)
        raise_error(p.err, PG_E_CAPACITY, a);   // not expected: the host bounds every window
    // ranges of every listed atom, and whether they meet this atom's window
    // ranges on each axis (then the atom adds to some window voxel); the
    // same phase as the atom's own lists (both need only its ranges)
    if (rec_ok) {
        for (int j = lane; j < 3 * nsame; j += 64) {
            const int sa = j / 3, q = j - 3 * (j / 3), k = same[sa];
            const float oq = q == 0 ? o[0] : (q == 1 ? o[1] : o[2]);
            const float hq = q == 0 ? h[0] : (q == 1 ? h[1] : h[2]);
            const float Lq = q == 0 ? p.L[0] : (q == 1 ? p.L[1] : p.L[2]);
            const int Nq = q == 0 ? p.W : (q == 1 ? p.H : p.D);
            AxisRanges ar;
            axis_ranges(oq, hq, Nq, p.xyz[3 * (size_t)k + q], p.periodic != 0, Lq, p.rc[t],
                        p.cut != 0, ar);
            const RangeRec rr = range_rec(ar);
            srr[j] = rr;
            const AxisRanges &mine = rg[q];
            bool meet = false;
#pragma unroll
            for (int r = 0; r < MAX_IMAGES; ++r)
                for (int r2 = 0; r2 < mine.n; ++r2)
                    meet = meet || (r < rr.n && rr.lo[r] <= mine.hi[r2] && mine.lo[r2] <= rr.hi[r]);
            if (meet)
                atomicOr(&sflag[sa], 1 << q);
        }
    }
    __syncthreads();
    // the atoms that meet the window on all three axes, in index order
    if (rec_ok) {
        for (int s0 = 0; s0 < nsame; s0 += 64) {
            const int sa = s0 + lane;
            const bool hit = sa < nsame && sflag[sa] == 7;
            const unsigned long long bal = __ballot(hit);
            if (hit)
                rel[nrel + __popcll(bal & ((1ull << lane) - 1ull))] = sa;
            nrel += __popcll(bal);
        }
    }
    if constexpr (RECOMP)
        __syncthreads();
    // their factor rows over this atom's window lists, one element per lane
    if (rec_ok) {
        const bool box = p.box != 0, sph = p.sphere != 0;
        for (int j = lane; j < nrel * wtot; j += 64) {
            const int r0 = j / wtot, e0 = j - r0 * wtot;
            const int q = e0 < n[0] ? 0 : (e0 < n[0] + n[1] ? 1 : 2);
            const int i = idx[base[q] + e0 - (q == 0 ? 0 : (q == 1 ? n[0] : n[0] + n[1]))];
            const RangeRec &rr = srr[3 * rel[r0] + q];
            const float hq = q == 0 ? h[0] : (q == 1 ? h[1] : h[2]);
            float f = 0.f, d2 = __builtin_huge_valf();
#pragma unroll
            for (int r = 0; r < MAX_IMAGES; ++r) {
                if (r < rr.n && i >= rr.lo[r] && i <= rr.hi[r]) {
                    f = factor1d(box, rr.bh[r], rr.bl[r], hq, i, p.inv2s2[t], p.isq2s[t]);
                    if (sph) {
                        const float d = offset_at(rr.bh[r], rr.bl[r], hq, i);
                        d2 = d * d;
                    }
                }
            }
            srow[(size_t)r0 * ntw + e0] = f;
            if (sph)
                sd2[(size_t)r0 * ntw + e0] = d2;
        }
    }
    if constexpr (RECOMP)
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
            const size_t cbase = ((size_t)m * p.C + c) * (size_t)p.D * plane;
            const T *U = recomp ? nullptr : (const T *)p.out + cbase;
            const float *TG = recomp ? p.target + cbase : nullptr;
            float sx = 0.f, sy = 0.f, sz = 0.f, sw = 0.f;
            // the lane's window element e = lane, lane + 64, ... as digits
            // (kx, ky, kz) of the mixed radix (nx, ny, nz), stepped by 64 =
            // (dx, dy, dz) per element with one carry at most per digit
            int cx = 0, cy = 0, cz = 0, dx = 0, dy = 0, dz = 0;
            if (total > 0) {
                cx = lane % nx;
                cy = (lane / nx) % ny;
                cz = (lane / nx) / ny;
                dx = 64 % nx;
                dy = (64 / nx) % ny;
                dz = (64 / nx) / ny;
            }
            // ADJ_UNROLL window elements per lane per round: their upstream
            // loads are issued together, then consumed in element order
            for (int e0 = 0; e0 < total; e0 += 64 * ADJ_UNROLL) {
                float u[ADJ_UNROLL];
                int ke[ADJ_UNROLL][3];
#pragma unroll
                for (int j = 0; j < ADJ_UNROLL; ++j) {
                    const int e = e0 + 64 * j + lane;
                    const int kx = cx, ky = cy, kz = cz;
                    cx += dx;
                    const int carry_x = cx >= nx ? 1 : 0;
                    cx -= carry_x * nx;
                    cy += dy + carry_x;
                    const int carry_y = cy >= ny ? 1 : 0;
                    cy -= carry_y * ny;
                    cz += dz + carry_y;
                    ke[j][0] = kx;
                    ke[j][1] = ky;
                    ke[j][2] = kz;
                    bool in = e < total;
                    if (in && p.sphere)
                        in = dsq[kx] <= (p.rc2[t] - dsq[base[2] + kz]) - dsq[base[1] + ky];
                    u[j] = 0.f;
                    if (in) {
                        const int ix = idx[kx], iy = idx[base[1] + ky], iz = idx[base[2] + kz];
                        const size_t v = (size_t)iz * plane + (size_t)iy * p.W + ix;
                        u[j] = recomp ? TG[v] : load_as_float<T>(U + v);
                    } else {
                        ke[j][0] = -1;
                    }
                }
                if (recomp) {
                    // u = 2 (G'(v) - T(v)), G'(v) summed as the window kernel does
#pragma unroll
                    for (int j = 0; j < ADJ_UNROLL; ++j) {
                        if (ke[j][0] < 0)
                            continue;
                        const float gp = recompute_density(srow, sd2, nrel, ntw, nx,
                                                           nx + ny, ke[j][0], ke[j][1], ke[j][2],
                                                           p.sphere != 0, p.rc2[t]);
                        u[j] = 2.f * (gp - u[j]);
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
    const size_t per_wave = adjoint_wave_lds(p.W + p.H + p.D, p.recompute ? p.a_cap : 0,
                                             p.recompute ? p.rec_ntw : 0, p.sphere != 0);
    // one wave per workgroup: the waves share nothing, so a workgroup of
    // several would only make each wait for the slowest at the barriers
    const int waves = 1;
    const int block = 64 * waves;
    const size_t lds = (size_t)waves * per_wave;
    const long long grid = (p.n_atoms + waves - 1) / waves;
    const void *k = grad_dtype == PG_OUT_F32
                        ? (p.recompute ? (const void *)adjoint_kernel<float, true>
                                       : (const void *)adjoint_kernel<float, false>)
                        : (const void *)adjoint_kernel<__bf16, false>;
    if (grad_dtype != PG_OUT_F32 && p.recompute)
        return hipErrorInvalidValue;   // the residual is recomputed only in float32
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    GridParams pc = p;
    void *args[] = {&pc};
    const hipError_t e = hipLaunchKernel(k, dim3((unsigned)grid), dim3(block), args, lds, s);
    if (e != hipSuccess)
        return e;
    return hipGetLastError();
}

}  // namespace pg
