// pg_device.hpp -- device-side building blocks shared by the gfx950 kernels.
//
//  * exact cutoff-window bounds per atom and axis, from error-free FP32
//    transforms (no FP64 on the GPU);
//  * nearest-image ranges for orthorhombic periodic cells;
//  * accurate per-axis offsets and 1-D Gaussian factors;
//  * bf16 conversion and vector stores.
//
// The voxel value is the point-sampled Gaussian of §III-A Eq. 1 (without
// its normalising prefactor), truncated per axis at rc_t = fl32(k sigma_t)
// (the threshold truncation suggested in §VI-B).  Because the Gaussian and
// the cube cutoff are both separable (§III-A; §IV-C relies on the same
// property), one atom's grid is the outer product of three 1-D factors
// phi_x(ix) phi_y(iy) phi_z(iz), which is what every kernel here evaluates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pg_params.hpp"

namespace pg {

// ---------------------------------------------------------------------------
// Error-free transforms (Knuth TwoSum, FMA-based TwoProd).  The library is
// compiled with -ffp-contract=off so these are evaluated as written.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void two_prod(float a, float b, float &p, float &e)
{
    p = a * b;
    e = __builtin_fmaf(a, b, -p);
}

// Float-float accumulation (a value held as hi + lo, |lo| <= ulp(hi) / 2):
// (hi, lo) += (bhi, blo), Dekker's addition -- TwoSum of the high parts,
// the low parts added to its error, renormalised.  For sums of non-negative
// terms the relative error stays near 2^-44 per addition, far below the
// float32 rounding of the final hi + lo.
__device__ __forceinline__ void ff_add(float &hi, float &lo, float bhi, float blo)
{
    float s, e;
    two_sum(hi, bhi, s, e);
    e += lo + blo;
    hi = s + e;
    lo = e - (hi - s);
}

// Wave-wide float-float sum of one float per lane (butterfly over the 64
// lanes, a fixed order); every lane receives the total.
__device__ __forceinline__ void ff_wave_sum(float v, float &hi, float &lo)
{
    hi = v;
    lo = 0.f;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const float oh = __shfl_xor(hi, w, 64), ol = __shfl_xor(lo, w, 64);
        ff_add(hi, lo, oh, ol);
    }
}

// Sign (-1, 0, +1) of the exact real sum of N float terms.  Grow-expansion
// (Shewchuk 1997): the running sum is kept as a non-overlapping expansion
// of increasing magnitude, so the sign is that of its largest non-zero
// component.
template <int N>
__device__ __forceinline__ int exact_sign(const float (&t)[N])
{
    float e[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
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
    int sgn = 0;
#pragma unroll
    for (int j = 0; j < N; ++j)
        sgn = (e[j] > 0.f) ? 1 : ((e[j] < 0.f) ? -1 : sgn);
    return sgn;
}

// Exact sign of o + fi h - mu - n L + r by expansion arithmetic.  Reached
// only for offsets within ~2^-20 of the cutoff edge (inlined: measured
// faster than a call in the window kernel's set-up phase).
__device__ __forceinline__ int side_exact(float o, float h, float fi, float mu, int n, float L, float r)
{
    float pp, pe, qq = 0.f, qe = 0.f;
    two_prod(fi, h, pp, pe);
    if (n != 0)
        two_prod((float)n, L, qq, qe);
    const float t[7] = {o, pp, pe, -mu, -qq, -qe, r};
    return exact_sign(t);
}

// sign(o + (i + 1/2) h - mu - n L + r), exactly.  A plain FP32 evaluation
// decides when it is far from zero: with M the sum of the terms' magnitudes,
// the five roundings below move the result by at most 5 * 2^-24 * M (plus
// the same again for the rounding of M itself), so |s| > 2^-20 M fixes the
// sign.  Otherwise the exact expansion decides.
__device__ __forceinline__ int side(float o, float h, int i, float mu, int n, float L, float r)
{
    const float fi = (float)i + 0.5f;
    const float p = fi * h;
    const float q = (float)n * L;
    const float s = (((o - mu) + p) - q) + r;
    const float M = (((fabsf(o) + fabsf(mu)) + fabsf(p)) + fabsf(q)) + fabsf(r);
    if (fabsf(s) > M * 0x1p-20f)
        return s > 0.f ? 1 : -1;
    return side_exact(o, h, fi, mu, n, L, r);
}

// Inside indices of one atom along one axis: up to MAX_IMAGES disjoint
// ranges [lo, hi] (one per periodic image that reaches the grid), each with
// the float-float base offset o - mu - n L.
constexpr int MAX_IMAGES = 3;

struct AxisRanges {
    int n;
    int lo[MAX_IMAGES], hi[MAX_IMAGES];
    float bh[MAX_IMAGES], bl[MAX_IMAGES];
};

// Bounds for image n: smallest i with offset >= -rc, largest with
// offset <= rc, clipped to [0, N).  The FP32 estimate is corrected with the
// exact sign test; for coordinates within 2^20 voxels of the grid the
// estimate is already within one index, so the correction loops run at
// most a couple of times (they are bounded regardless).
__device__ __forceinline__ void image_range(float o, float h, int N, float mu, int n, float L,
                                            float rc, bool cut, int &lo_out, int &hi_out)
{
    if (!cut) {
        lo_out = 0;
        hi_out = N - 1;
        return;
    }
    const float c = (n != 0) ? __builtin_fmaf((float)n, L, mu) : mu;
    const float f = (c - o) / h - 0.5f;
    const float r = rc / h;
    const float lim_lo = -4.f, lim_hi = (float)N + 4.f;
    float flo = fminf(fmaxf(ceilf(f - r), lim_lo), lim_hi);
    float fhi = fminf(fmaxf(floorf(f + r), lim_lo), lim_hi);
    // an image whose estimated window lies two or more indices outside the
    // grid is empty (the estimate of an image that can reach the grid is
    // within one index): no exact test needed -- most periodic images
    if (fhi <= -2.f || flo >= (float)N + 1.f) {
        lo_out = 0;
        hi_out = -1;
        return;
    }
    int lo = (int)flo, hi = (int)fhi;
    const int ilo = -4, ihi = N + 4;
    for (int it = 0; it < 8 && lo > ilo && side(o, h, lo - 1, mu, n, L, rc) >= 0; ++it)
        --lo;
    for (int it = 0; it < 8 && lo < ihi && side(o, h, lo, mu, n, L, rc) < 0; ++it)
        ++lo;
    for (int it = 0; it < 8 && hi < ihi && side(o, h, hi + 1, mu, n, L, -rc) <= 0; ++it)
        ++hi;
    for (int it = 0; it < 8 && hi > ilo && side(o, h, hi, mu, n, L, -rc) > 0; ++it)
        --hi;
    lo_out = lo < 0 ? 0 : lo;
    hi_out = hi > N - 1 ? N - 1 : hi;
}

__device__ __forceinline__ void base_offset(float o, float mu, int n, float L, float &bh, float &bl)
{
    float s1, e1;
    two_sum(o, -mu, s1, e1);
    if (n == 0) {
        bh = s1;
        bl = e1;
        return;
    }
    float q, qe, s2, e2;
    two_prod((float)n, L, q, qe);
    two_sum(s1, -q, s2, e2);
    bh = s2;
    bl = (e1 + e2) - qe;
}

// Compact copy of AxisRanges kept in LDS (16-bit window bounds).
struct RangeRec {
    int32_t n;
    int16_t lo[MAX_IMAGES], hi[MAX_IMAGES];
    float bh[MAX_IMAGES], bl[MAX_IMAGES];
};

__device__ __forceinline__ RangeRec range_rec(const AxisRanges &ar)
{
    RangeRec R;
    R.n = ar.n;
#pragma unroll
    for (int r = 0; r < MAX_IMAGES; ++r) {
        R.lo[r] = (int16_t)(r < ar.n ? ar.lo[r] : 0);
        R.hi[r] = (int16_t)(r < ar.n ? ar.hi[r] : -1);
        R.bh[r] = r < ar.n ? ar.bh[r] : 0.f;
        R.bl[r] = r < ar.n ? ar.bl[r] : 0.f;
    }
    return R;
}

// All ranges of one atom on one axis.  Far-away coordinates give n = 0.
// Set-up work: runs once per atom and axis, before any output is written.
__device__ __forceinline__ void axis_ranges(float o, float h, int N, float mu, bool periodic,
                                            float L, float rc, bool cut, AxisRanges &R)
{
    R.n = 0;
    // an atom more than 2^20 voxels away cannot reach the grid
    const float span = 1048576.f * h;
    if (!(fabsf(mu - o) < span))
        return;
    if (!periodic) {
        int lo, hi;
        image_range(o, h, N, mu, 0, L, rc, cut, lo, hi);
        if (lo <= hi) {
            R.lo[0] = lo;
            R.hi[0] = hi;
            base_offset(o, mu, 0, L, R.bh[0], R.bl[0]);
            R.n = 1;
        }
        return;
    }
    // images n whose cutoff interval can reach the voxel centres of the grid
    const float ext = (float)N * h;
    const int n_min = (int)floorf((o - rc - mu) / L) - 1;
    const int n_max = (int)ceilf((o + ext + rc - mu) / L) + 1;
    for (int n = n_min; n <= n_max && R.n < MAX_IMAGES; ++n) {
        int lo, hi;
        image_range(o, h, N, mu, n, L, rc, cut, lo, hi);
        if (lo <= hi) {
            float bh, bl;
            base_offset(o, mu, n, L, bh, bl);
            // insert at slot R.n without dynamic register indexing
#pragma unroll
            for (int s = 0; s < MAX_IMAGES; ++s) {
                if (s == R.n) {
                    R.lo[s] = lo;
                    R.hi[s] = hi;
                    R.bh[s] = bh;
                    R.bl[s] = bl;
                }
            }
            R.n++;
        }
    }
}

// Offset r_i - mu (nearest image via the range's base), rounded once from
// a float-float sum: |error| <= ulp(offset)/2 + 2^-48 |base|.
__device__ __forceinline__ float offset_at(float bh, float bl, float h, int i)
{
    float p, pe;
    two_prod((float)i + 0.5f, h, p, pe);
    float s, e;
    two_sum(bh, p, s, e);
    return s + ((e + pe) + bl);
}

// exp(-d^2 / (2 sigma^2)) with inv2s2 = fl32(1 / (2 sigma^2)).
__device__ __forceinline__ float gauss1d(float d, float inv2s2)
{
    return expf(-(d * d) * inv2s2);
}

// Offset of the lower edge of voxel i from the atom, o + i h - mu (- n L),
// from the float-float base, rounded once.
__device__ __forceinline__ float edge_at(float bh, float bl, float h, int i)
{
    float p, pe;
    two_prod((float)i, h, p, pe);
    float s, e;
    two_sum(bh, p, s, e);
    return s + ((e + pe) + bl);
}

// Mass of the normalised 1-D Gaussian between edge offsets l < r:
// (1/2)[erf(r s) - erf(l s)], s = 1 / (sqrt(2) sigma); on a tail the
// complementary form, so the difference does not cancel.
__device__ __forceinline__ float box1d(float l, float r, float isq2s)
{
    const float a = l * isq2s, b = r * isq2s;
    if (a >= 0.f)
        return 0.5f * (erfcf(a) - erfcf(b));
    if (b <= 0.f)
        return 0.5f * (erfcf(-b) - erfcf(-a));
    return 0.5f * (erff(b) - erff(a));
}

// Box form with each edge's error function shared by the two voxels that
// meet there (N + 1 evaluations for a window of N voxels instead of 2N,
// §VI-A).  box_edge(e) = erfc(|e| s) is the tail term of edge offset e; a
// voxel's mass is half the difference of its edges' terms when both edges
// lie on one side of the atom (from the nearer tail), the direct difference
// of erf values for the one voxel that holds the centre: bitwise what box1d
// returns.
__device__ __forceinline__ float box_edge(float e, float isq2s)
{
    return erfcf(fabsf(e * isq2s));
}

// Box-form masses of the N voxels v0 .. v0+N-1 of one image (the caller
// keeps those inside its window): N + 1 edge terms, and the direct erf
// difference once, for the voxel holding the centre, after the walk (so a
// wave runs that branch once, not once per voxel).
template <int N>
__device__ __forceinline__ void box_fixed(float bh, float bl, float h, int v0, float isq2s,
                                          float (&out)[N])
{
    float el = edge_at(bh, bl, h, v0), ql = box_edge(el, isq2s);
    int ks = -1;
    float as = 0.f, bs = 0.f;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const float er = edge_at(bh, bl, h, v0 + k + 1), qr = box_edge(er, isq2s);
        const float a = el * isq2s, b = er * isq2s;
        out[k] = a >= 0.f ? 0.5f * (ql - qr) : 0.5f * (qr - ql);
        if (a < 0.f && b > 0.f) {
            ks = k;
            as = a;
            bs = b;
        }
        el = er;
        ql = qr;
    }
    if (ks >= 0) {
        const float v = 0.5f * (erff(bs) - erff(as));
#pragma unroll
        for (int k = 0; k < N; ++k)
            if (k == ks)
                out[k] = v;
    }
}

// The same along voxels lo .. hi of one image's window into dst[lo .. hi]
// (times scale), for runs of any length.
template <bool SCALE>
__device__ __forceinline__ void box_walk(float bh, float bl, float h, int lo, int hi, float isq2s,
                                         float scale, float *dst)
{
    if (lo > hi)
        return;
    float el = edge_at(bh, bl, h, lo), ql = box_edge(el, isq2s);
    int vs = -1;
    float as = 0.f, bs = 0.f;
    for (int v = lo; v <= hi; ++v) {
        const float er = edge_at(bh, bl, h, v + 1), qr = box_edge(er, isq2s);
        const float a = el * isq2s, b = er * isq2s;
        const float f = a >= 0.f ? 0.5f * (ql - qr) : 0.5f * (qr - ql);
        dst[v] = SCALE ? scale * f : f;
        if (a < 0.f && b > 0.f) {
            vs = v;
            as = a;
            bs = b;
        }
        el = er;
        ql = qr;
    }
    if (vs >= 0) {
        const float f = 0.5f * (erff(bs) - erff(as));
        dst[vs] = SCALE ? scale * f : f;
    }
}

// The value of window element i on one axis: the point sample at the voxel
// centre, or (box) the voxel's Gaussian mass.
__device__ __forceinline__ float factor1d(bool box, float bh, float bl, float h, int i,
                                          float inv2s2, float isq2s)
{
    if (box)
        return box1d(edge_at(bh, bl, h, i), edge_at(bh, bl, h, i + 1), isq2s);
    return gauss1d(offset_at(bh, bl, h, i), inv2s2);
}

// d/dmu of factor1d: point, g(d) d / sigma^2; box, (g(l) - g(r)) / (sqrt(2 pi) sigma).
__device__ __forceinline__ float dfactor1d(bool box, float bh, float bl, float h, int i,
                                           float inv2s2, float invs2, float inorm)
{
    if (box) {
        const float l = edge_at(bh, bl, h, i), r = edge_at(bh, bl, h, i + 1);
        return (gauss1d(l, inv2s2) - gauss1d(r, inv2s2)) * inorm;
    }
    const float d = offset_at(bh, bl, h, i);
    return gauss1d(d, inv2s2) * d * invs2;
}

// ---------------------------------------------------------------------------
// Output conversion and vector stores
// ---------------------------------------------------------------------------
template <typename T> struct OutTraits;
template <> struct OutTraits<float> {
    static constexpr int bytes = 4;
};
template <> struct OutTraits<__bf16> {
    static constexpr int bytes = 2;
};

// Store VEC accumulated values (float) to p as T (bf16: round to nearest
// even via the gfx950 conversion instruction).
template <typename T, int VEC>
__device__ __forceinline__ void store_vec(T *p, const float (&v)[VEC], bool nt)
{
    constexpr int BYTES = VEC * OutTraits<T>::bytes;
    uint32_t w[(BYTES + 3) / 4];
    if constexpr (OutTraits<T>::bytes == 4) {
#pragma unroll
        for (int k = 0; k < VEC; ++k)
            w[k] = __builtin_bit_cast(uint32_t, v[k]);
    } else {
        if constexpr (VEC == 1) {
            __bf16 b = (__bf16)v[0];
            unsigned short s = __builtin_bit_cast(unsigned short, b);
            if (nt)
                __builtin_nontemporal_store(s, (unsigned short *)p);
            else
                *(unsigned short *)p = s;
            return;
        } else {
            // pairs rounded in one conversion (element 0 in the low half)
            typedef float f2v __attribute__((ext_vector_type(2)));
            typedef __bf16 b2v __attribute__((ext_vector_type(2)));
#pragma unroll
            for (int k = 0; k < VEC / 2; ++k) {
                const f2v pr = {v[2 * k], v[2 * k + 1]};
                w[k] = __builtin_bit_cast(uint32_t, __builtin_convertvector(pr, b2v));
            }
        }
    }
    if constexpr (BYTES == 16) {
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
        u4 x = {w[0], w[1], w[2], w[3]};
        if (nt)
            __builtin_nontemporal_store(x, (u4 *)p);
        else
            *(u4 *)p = x;
    } else if constexpr (BYTES == 8) {
        typedef uint32_t u2 __attribute__((ext_vector_type(2)));
        u2 x = {w[0], w[1]};
        if (nt)
            __builtin_nontemporal_store(x, (u2 *)p);
        else
            *(u2 *)p = x;
    } else if constexpr (BYTES == 4) {
        if (nt)
            __builtin_nontemporal_store(w[0], (uint32_t *)p);
        else
            *(uint32_t *)p = w[0];
    }
}

template <typename T>
__device__ __forceinline__ float load_as_float(const T *p);
template <>
__device__ __forceinline__ float load_as_float<float>(const float *p) { return *p; }
template <>
__device__ __forceinline__ float load_as_float<__bf16>(const __bf16 *p)
{
    unsigned short s = *(const unsigned short *)p;
    return __builtin_bit_cast(float, (uint32_t)s << 16);
}

// ---------------------------------------------------------------------------
// One-workgroup exclusive scan
// ---------------------------------------------------------------------------
// out[i] = in[0] + ... + in[i - 1] for the n 32-bit counts in[0..n) (out may
// be in; both 16-byte aligned), by one workgroup of 1024 threads with a
// 1024-entry LDS array part; returns the total to every thread.  Each
// thread owns a contiguous segment whose length is a multiple of 4, read
// and written in 16-byte pieces, so its loads are independent and stay in
// flight together instead of one dependent round trip per count.
__device__ inline unsigned long long workgroup_exclusive_scan(const uint32_t *in, uint32_t *out,
                                                              long long n,
                                                              unsigned long long *part)
{
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    const int t = threadIdx.x;
    const long long seg = (((n + 1023) / 1024) + 3) & ~3ll;
    const long long b = min(n, (long long)t * seg), e = min(n, b + seg);
    const long long e4 = b + ((e - b) & ~3ll);
    unsigned long long s = 0;
#pragma unroll 4
    for (long long i = b; i < e4; i += 4) {
        const u4 v = *(const u4 *)(in + i);
        s += (unsigned long long)v.x + v.y + v.z + v.w;
    }
    for (long long i = e4; i < e; ++i)
        s += in[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const unsigned long long v = t >= d ? part[t - d] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const unsigned long long total = part[1023];
    unsigned long long run = part[t] - s;
#pragma unroll 4
    for (long long i = b; i < e4; i += 4) {
        const u4 v = *(const u4 *)(in + i);
        u4 o;
        o.x = (uint32_t)run;
        run += v.x;
        o.y = (uint32_t)run;
        run += v.y;
        o.z = (uint32_t)run;
        run += v.z;
        o.w = (uint32_t)run;
        run += v.w;
        *(u4 *)(out + i) = o;
    }
    for (long long i = e4; i < e; ++i) {
        const uint32_t v = in[i];
        out[i] = (uint32_t)run;
        run += v;
    }
    return total;
}

// ---------------------------------------------------------------------------
// Sticky device error word
// ---------------------------------------------------------------------------
__device__ __forceinline__ void raise_error(DeviceError *err, int code, long long index)
{
    atomicOr(&err->flags, 1u << code);
    atomicMin(&err->first, (unsigned long long)index);
}

__device__ __forceinline__ bool atom_valid(float x, float y, float z, int t, int C)
{
    return t >= 0 && t < C && isfinite(x) && isfinite(y) && isfinite(z);
}

// Atoms the batch holds on the device, offsets[n_mol], capped by the host
// bound n_atoms: atoms past the CSR belong to no structure (and the image
// batch of a triclinic request fills only part of its bound).
__device__ __forceinline__ long long live_atoms(const GridParams &p)
{
    const long long n = p.n_mol > 0 ? (long long)p.offsets[p.n_mol] : 0;
    return n < 0 ? 0 : (n < p.n_atoms ? n : p.n_atoms);
}

// ---------------------------------------------------------------------------
// Per-atom window records (plain and crystal paths)
// ---------------------------------------------------------------------------
// Structure holding global atom a: the last m with offsets[m] <= a (that
// structure is non-empty and owns a).
__device__ __forceinline__ int structure_of(const int32_t *offsets, int n_mol, long long a)
{
    int lo = 0, hi = n_mol;   // invariant: offsets[lo] <= a < offsets[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((long long)offsets[mid] <= a)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// structure_of within a known bracket: the last m in [lo, hi] with
// offsets[m] <= a, given offsets[lo] <= a (the atoms of one prep block span
// a few structures).
__device__ __forceinline__ int structure_in(const int32_t *offsets, int lo, int hi, long long a)
{
    int h = hi + 1;   // invariant: offsets[lo] <= a < offsets[h] (h past the bracket: unknown)
    while (h - lo > 1) {
        const int mid = (lo + h) >> 1;
        if ((long long)offsets[mid] <= a)
            lo = mid;
        else
            h = mid;
    }
    return lo;
}

// structure_of for an atom index a that is uniform across the calling wave:
// each round the 64 lanes probe 63 evenly spaced offsets of the bracket at
// once, so a batch of n structures takes ceil(log64 n) dependent loads
// instead of log2 n.  Every lane of the wave must call it.
__device__ __forceinline__ int structure_of_wave(const int32_t *offsets, int n_mol, long long a)
{
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = n_mol;   // invariant: offsets[lo] <= a < offsets[hi]
    while (hi - lo > 1) {
        const int step = (hi - lo + 63) / 64;
        const int q = lo + lane * step;
        const bool le = lane > 0 && q < hi && (long long)offsets[q] <= a;
        // offsets are non-decreasing: the probes at or below a form a prefix
        const int below = __popcll(__ballot(le));
        lo += below * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// Exact window ranges of atom a on axis q into its record (axis 0 also
// writes the type: -1 for a skipped atom, which also raises the device
// error).  Returns the atom's structure; n_out = the axis's range count.
// m_known: the atom's structure when the caller knows it, else -1.
__device__ inline int write_atom_axis(const GridParams &p, long long a, int q, AtomWindow *w,
                                      int &n_out, int m_known = -1)
{
    const float mu[3] = {p.xyz[3 * a], p.xyz[3 * a + 1], p.xyz[3 * a + 2]};
    const int t = p.types[a];
    const bool ok = atom_valid(mu[0], mu[1], mu[2], t, p.n_sig);
    if (!ok && q == 0)
        raise_error(p.err, PG_E_DEVICE_DATA, a);
    const int m = m_known >= 0 ? m_known : structure_of(p.offsets, p.n_mol, a);
    if (q == 0)
        w->type = ok ? t : -1;
    AxisRanges R;
    R.n = 0;
    if (ok) {
        const float o = p.origins ? p.origins[3 * (size_t)m + q] : p.o[q];
        const float h = p.spacings ? p.spacings[3 * (size_t)m + q] : p.h[q];
        const int N = q == 0 ? p.W : (q == 1 ? p.H : p.D);
        axis_ranges(o, h, N, mu[q], p.periodic != 0, p.L[q], p.rc[t], p.cut != 0, R);
    }
    w->n[q] = R.n;
#pragma unroll
    for (int r = 0; r < MAX_IMAGES; ++r) {
        const bool u = r < R.n;
        w->lo[q][r] = u ? R.lo[r] : 0;
        w->hi[q][r] = u ? R.hi[r] : -1;
        w->bh[q][r] = u ? R.bh[r] : 0.f;
        w->bl[q][r] = u ? R.bl[r] : 0.f;
    }
    n_out = R.n;
    return m;
}

// Exact window ranges of atom a on the three axes.  Returns the atom's
// structure.
__device__ inline int write_atom_window(const GridParams &p, long long a, AtomWindow *w)
{
    int n, m = 0;
#pragma unroll
    for (int q = 0; q < 3; ++q)
        m = write_atom_axis(p, a, q, w, n);
    return m;
}

}  // namespace pg
