// pg_crystal.hip -- large / dense structures (periodic crystal cells, big
// clusters) on gfx950.
//
// Structures with more atoms than the molecule window kernel stages in LDS
// take this path.  Set-up, all on the GPU and free of order-dependent
// atomics in anything that reaches the output:
//   prep:    three threads per atom (one per axis): exact window ranges
//            (nearest periodic images included) into the atom's record,
//            counts of the atom per (channel, structure) and per (channel,
//            prep block), and (MFMA form) the 32-voxel tiles its x and y
//            windows meet;
//   scan:    exclusive scans of both count arrays in channel-major order;
//   place:   a stable partition of all atoms by channel (ballot ranks within
//            a block): channel c's atoms in index order, so each (structure,
//            channel) pair -- a "run" -- is one contiguous stretch of the list.
// Then one of two plane forms:
//   mfma:    the plane is a product of two factor matrices (separability of
//            the Gaussian and of the cube cutoff, Sec. III-A / IV-C):
//            G[y][x] = sum_k phi_z^k(z) phi_y^k(y) phi_x^k(x).  One launch
//            sorts every run's z images into per-32 x 32-tile-column lists
//            (ordered by z start) and, beside it, writes each atom's phi_x
//            and phi_y over the 32-voxel tiles its windows meet ("factor
//            slots"); the tile kernels then contract, per 32 x 32 tile and 4
//            planes, the entries of the tile column's list (block-sparse K):
//            bf16 grids on v_mfma_f32_32x32x16_bf16 (A = phi_z phi_y formed in
//            FP32 and rounded to bf16 once), fp32 grids on
//            v_mfma_f32_32x32x2_f32 with FP32 operands; FP32 accumulation;
//   window:  per run, the atoms' z images sorted stably by window start (each
//            plane's images one contiguous range), then the same sum in FP32
//            on the vector ALUs, one workgroup per (structure, channel, z):
//            per 32-image step the images' dense factor rows go to LDS with a
//            bit mask of the images meeting each 32 x 32 tile, and each lane
//            accumulates a 4 x 4 block of voxels over its tile's images.
// Both forms sum each voxel's atoms in an order fixed by the input alone
// (z-window start, then list order), so results are bitwise reproducible.
#include <type_traits>

#include "pg_device.hpp"
#include "pg_launch.hpp"

namespace pg {

constexpr int PREP_BLOCK = 256; // atoms per prep / place block
constexpr int KC = 32;          // images per step of the vector form

__global__ void cr_clear_kernel(uint32_t *a, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        a[i] = 0u;
}

// Per-structure counts are aggregated in LDS when the block's atoms span
// few structures (large structures: one global atomic per channel and
// structure per block instead of one per atom).
constexpr int PREP_SPAN = 4;

// The type of an atom that enters the channel partition, or -1: skipped
// atoms, and atoms whose window misses the grid on some axis (they add
// nothing -- e.g. the lattice images of a triclinic cell that do not reach
// the grid).
__device__ __forceinline__ int listed_type(const AtomWindow &w)
{
    return (w.type >= 0 && w.n[0] > 0 && w.n[1] > 0 && w.n[2] > 0) ? w.type : -1;
}

// Listed atom a of type t is entered in channel c: c is its type, or with
// weighted channels its weight for c is non-zero.
__device__ __forceinline__ bool listed_in(const GridParams &p, long long a, int t, int c)
{
    return p.weights ? p.weights[(size_t)a * p.C + c] != 0.f : t == c;
}

// Per image of channel c: the atom's type (its sigma) and weight.
__device__ __forceinline__ int image_type(const GridParams &p, const CrystalParams &q, int atom,
                                          int c)
{
    return p.weights ? q.table[atom].type : c;
}

__device__ __forceinline__ float image_weight(const GridParams &p, int atom, int c)
{
    return p.weights ? p.weights[(size_t)atom * p.C + c] : 1.f;
}

__device__ __forceinline__ uint16_t bf16_bits(float v)
{
    return __builtin_bit_cast(uint16_t, (__bf16)v);
}

// Slot value storage: bf16 bits (x slots of the bf16 contraction) or float
// (y slots, and x slots of the fp32 contraction).
__device__ __forceinline__ void op_store(uint16_t *p, float v) { *p = bf16_bits(v); }
__device__ __forceinline__ void op_store(float *p, float v) { *p = v; }
// four consecutive slot values (p aligned to four elements)
__device__ __forceinline__ void op_store4(uint16_t *p, const float (&v)[4])
{
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef __bf16 b2v __attribute__((ext_vector_type(2)));
    const f2v lo = {v[0], v[1]}, hi = {v[2], v[3]};
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    *(u2 *)p = u2{__builtin_bit_cast(uint32_t, __builtin_convertvector(lo, b2v)),
                  __builtin_bit_cast(uint32_t, __builtin_convertvector(hi, b2v))};
}
__device__ __forceinline__ void op_store4(float *p, const float (&v)[4])
{
    *(float4 *)p = float4{v[0], v[1], v[2], v[3]};
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// The window ranges of one atom on axis ax (0 = x, 1 = y), ascending and
// disjoint (images in increasing lattice order).
struct AxisWin {
    int n;
    int lo[MAX_IMAGES], hi[MAX_IMAGES];
};

__device__ __forceinline__ AxisWin axis_win(const AtomWindow &w, int ax)
{
    AxisWin a;
    a.n = ax == 0 ? w.n[0] : w.n[1];
#pragma unroll
    for (int r = 0; r < MAX_IMAGES; ++r) {
        a.lo[r] = ax == 0 ? w.lo[0][r] : w.lo[1][r];
        a.hi[r] = ax == 0 ? w.hi[0][r] : w.hi[1][r];
    }
    return a;
}

// Factor slots of the MFMA form: per listed atom and axis x or y, per
// 32-voxel tile its windows meet (ascending: the set bits of its tile mask),
// the 32 values phi(32 tile + j), zero outside the windows and past the grid
// edge.  Eight lanes per (atom, axis), four consecutive values each per slot
// (the box form walks their five edges once), so one wave fills eight
// atom-axes; the atoms' records are read once.  wv: the global index of
// the calling wave among the pass's waves.
template <typename YT, typename XT>
__device__ __forceinline__ void slot_wave(const GridParams &p, const CrystalParams &q, long long wv)
{
    const int lane = threadIdx.x & 63, grp = lane >> 3, j8 = lane & 7;
    const long long id = wv * 8 + grp;
    const long long a = id >> 1;
    const int ax = (int)(id & 1);
    if (a >= live_atoms(p))
        return;
    const AtomWindow &w = q.table[a];
    if (listed_type(w) < 0)
        return;
    const AxisWin aw = axis_win(w, ax);
    float bh[MAX_IMAGES], bl[MAX_IMAGES];
#pragma unroll
    for (int r = 0; r < MAX_IMAGES; ++r) {
        bh[r] = ax == 0 ? w.bh[0][r] : w.bh[1][r];
        bl[r] = ax == 0 ? w.bl[0][r] : w.bl[1][r];
    }
    const int t = w.type;
    const float inv2s2 = p.inv2s2[t], isq2s = p.isq2s[t], h = p.h[ax];
    const int S = ax == 0 ? q.sx_max : q.sy_max;
    XT *outx = (XT *)q.xval + (size_t)a * S * 32;
    YT *outy = (YT *)q.yval + (size_t)a * S * 32;
    const bool box = p.box != 0;
    uint32_t mk = q.tmask[2 * a + ax];
    for (int s = 0; s < S && mk != 0u; ++s, mk &= mk - 1u) {
        const int tile = __builtin_ctz(mk);
        const int v0 = 32 * tile + 4 * j8;
        float val[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < MAX_IMAGES; ++r) {
            if (r >= aw.n || aw.hi[r] < v0 || aw.lo[r] > v0 + 3)
                continue;
            float f[4];
            if (box) {
                box_fixed<4>(bh[r], bl[r], h, v0, isq2s, f);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    f[k] = gauss1d(offset_at(bh[r], bl[r], h, v0 + k), inv2s2);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (v0 + k >= aw.lo[r] && v0 + k <= aw.hi[r])
                    val[k] = f[k];
        }
        if (ax == 0)
            op_store4(outx + (size_t)s * 32 + 4 * j8, val);
        else
            op_store4(outy + (size_t)s * 32 + 4 * j8, val);
    }
}

// Three threads per atom (wave group q of the block finds axis q of the
// block's PREP_BLOCK atoms: the exact window search is the long part) build
// the block's window records in LDS; the block then writes them out as one
// contiguous 16-byte-store copy, and the first group counts the listed atoms.
__global__ void __launch_bounds__(3 * PREP_BLOCK) cr_prep_kernel(GridParams p, CrystalParams q)
{
    __shared__ uint32_t cnt[PG_MAX_CHANNELS];
    __shared__ uint32_t cntm[PG_MAX_CHANNELS][PREP_SPAN];
    __shared__ int32_t sn[3][PREP_BLOCK];   // ranges per axis
    __shared__ int32_t sm[PREP_BLOCK];      // structure
    __shared__ __attribute__((aligned(16))) AtomWindow srec[PREP_BLOCK];
    const int tid = threadIdx.x;
    for (int c = tid; c < p.C; c += blockDim.x) {
        cnt[c] = 0u;
#pragma unroll
        for (int j = 0; j < PREP_SPAN; ++j)
            cntm[c][j] = 0u;
    }
    const long long a0 = (long long)blockIdx.x * PREP_BLOCK;
    const long long a1 = (a0 + PREP_BLOCK < p.n_atoms ? a0 + PREP_BLOCK : p.n_atoms) - 1;
    // every wave finds the block's first and last structures (64-ary search)
    const int m_first = structure_of_wave(p.offsets, p.n_mol, a0);
    const int m_last = structure_of_wave(p.offsets, p.n_mol, a1);
    const bool local = m_last - m_first < PREP_SPAN;
    const int ax = tid / PREP_BLOCK, al = tid - ax * PREP_BLOCK;
    const long long a = a0 + al;
    const bool live = a < live_atoms(p);
    if (live) {
        int n;
        const int m = write_atom_axis(p, a, ax, srec + al, n,
                                      structure_in(p.offsets, m_first, m_last, a));
        sn[ax][al] = n;
        if (ax == 0)
            sm[al] = m;
    }
    __syncthreads();
    // MFMA form: the 32-voxel tiles each listed atom's x and y windows meet
    if (q.tmask && live && ax < 2) {
        uint32_t mk = 0u;
        const AtomWindow &w = srec[al];
#pragma unroll
        for (int r = 0; r < MAX_IMAGES; ++r)
            if (r < w.n[ax] && w.hi[ax][r] >= w.lo[ax][r])
                mk |= (uint32_t)((2ull << (w.hi[ax][r] >> 5)) - (1ull << (w.lo[ax][r] >> 5)));
        q.tmask[2 * a + ax] = mk;
    }
    const long long n_live = live_atoms(p) - a0;
    const int nrec = (int)(n_live < PREP_BLOCK ? (n_live > 0 ? n_live : 0) : PREP_BLOCK);
    {
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
        constexpr int R16 = (int)(sizeof(AtomWindow) / 16);
        static_assert(sizeof(AtomWindow) % 16 == 0, "record copy in 16-byte pieces");
        const u4 *src = (const u4 *)srec;
        u4 *dst = (u4 *)(q.table + a0);
        for (int i = tid; i < nrec * R16; i += blockDim.x)
            dst[i] = src[i];
    }
    if (ax == 0 && live) {
        const int m = sm[al];
        // listed: a valid atom whose windows meet the grid on every axis
        const int t = (srec[al].type >= 0 && sn[0][al] > 0 && sn[1][al] > 0 && sn[2][al] > 0)
                          ? srec[al].type : -1;
        // the channels the atom is listed under: its type, or with weighted
        // channels every channel with a non-zero weight
        for (int c = 0; c < p.C && t >= 0; ++c) {
            if (!listed_in(p, a, t, c))
                continue;
            atomicAdd(&cnt[c], 1u);
            if (local)
                atomicAdd(&cntm[c][m - m_first], 1u);
            else
                atomicAdd(&q.mcount[(size_t)c * p.n_mol + m], 1u);
        }
    }
    __syncthreads();
    for (int c = tid; c < p.C; c += blockDim.x)
        q.bcount[(size_t)c * q.nblk + blockIdx.x] = cnt[c];
    if (local)
        for (int i = tid; i < p.C * PREP_SPAN; i += blockDim.x) {
            const int c = i / PREP_SPAN, j = i - c * PREP_SPAN;
            if (cntm[c][j] != 0u)
                atomicAdd(&q.mcount[(size_t)c * p.n_mol + m_first + j], cntm[c][j]);
        }
}

// Exclusive scan of n counts, in place (workgroup 0: the per-block counts)
// or into mstart (workgroup 1: the per-structure counts).  One workgroup
// of 1024 threads per array.
__global__ void __launch_bounds__(1024) cr_scan_kernel(CrystalParams q, long long n_blk,
                                                       long long n_mol)
{
    __shared__ unsigned long long part[1024];
    const uint32_t *in = blockIdx.x == 0 ? q.bcount : q.mcount;
    uint32_t *out = blockIdx.x == 0 ? q.bcount : q.mstart;
    const long long n = blockIdx.x == 0 ? n_blk : n_mol;
    (void)workgroup_exclusive_scan(in, out, n, part);
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
    const int t = a < live_atoms(p) ? listed_type(q.table[a]) : -1;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int c = 0; c < p.C; ++c) {
        const unsigned long long mask = __ballot(t >= 0 && listed_in(p, a, t, c));
        if (lane == 0)
            wc[wave][c] = (uint32_t)__popcll(mask);
    }
    __syncthreads();
    if (t < 0)
        return;
    const AtomWindow &w = q.table[a];
    ListEntry e;
    e.atom = (int32_t)a;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const bool u = r < w.n[2];
        e.z[r] = u ? pack_range(w.lo[2][r], w.hi[2][r]) : pack_range(0, -1);
        e.bh[r] = u ? w.bh[2][r] : 0.f;
        e.bl[r] = u ? w.bl[2][r] : 0.f;
    }
    // one entry per channel the atom is listed under, at its stable rank
    for (int c = 0; c < p.C; ++c) {
        const bool in = listed_in(p, a, t, c);
        const unsigned long long mask = __ballot(in);
        if (!in)
            continue;
        uint32_t pos = q.bcount[(size_t)c * q.nblk + blockIdx.x] +
                       (uint32_t)__popcll(mask & below);
        for (int v = 0; v < wave; ++v)
            pos += wc[v][c];
        q.list[pos] = e;
    }
}

// XCD-aware workgroup order: the hardware deals consecutive workgroups to
// the 8 XCDs in turn; remap so that each XCD runs a contiguous stretch of
// planes (consecutive z of one structure and channel share their atoms'
// factor rows in that XCD's L2).  A bijection on [0, gridDim.x).
__device__ __forceinline__ unsigned xcd_block()
{
    const unsigned G = gridDim.x, full = G & ~7u, b = blockIdx.x;
    return b < full ? (b & 7u) * (full >> 3) + (b >> 3) : b;
}

// ---------------------------------------------------------------------------
// MFMA form
// ---------------------------------------------------------------------------

// First 32-image operand block of run mc.  Runs are spaced so that run mc
// owns at least ceil(3 count / 32) blocks (an atom has at most 3 z images):
// block(mc) = ceil(3 mstart[mc] / 32) + 2 mc.
__device__ __forceinline__ long long run_block(const CrystalParams &q, size_t mc)
{
    return (long long)((3ull * q.mstart[mc] + 31ull) / 32ull) + 2ll * (long long)mc;
}

__device__ __forceinline__ int range_lo(uint32_t v) { return (int16_t)(v & 0xffffu); }
__device__ __forceinline__ int range_hi(uint32_t v) { return (int16_t)(v >> 16); }

// One workgroup per run: the run's z images (one per z range of each
// atom), sorted stably by window start, into zlist -- a counting sort over z
// in LDS.  The run's list is split into one contiguous part per wave; each
// wave counts its part (per-wave histograms), the counts are scanned over
// (z, wave) so that every wave gets its own cursors, and each wave places its
// part in list order, ranks of equal keys from ballots over the key bits.
// Per plane z it writes a range [first, end) of that order holding every
// image whose window holds z (end: images starting at or before z; first:
// the start of the images starting at z - Lmax + 1, Lmax the run's longest
// z window, as no earlier image reaches z), the run's image count and the
// map of its operand blocks.  Dynamic LDS: (waves + 1) x D words.
__global__ void __launch_bounds__(1024) cr_zsort_kernel(GridParams p, CrystalParams q)
{
    extern __shared__ uint32_t zs[];
    __shared__ uint32_t wtot[16];
    __shared__ int lmax_s;
    const int D = p.D, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nw = blockDim.x >> 6, nt = blockDim.x;
    uint32_t *zst = zs, *hist = zs + D;          // hist[w * D + z]: counts, then cursors
    const size_t mc = blockIdx.x;
    const uint32_t start = q.mstart[mc], n = q.mcount[mc];
    for (int i = tid; i < (nw + 1) * D; i += nt)
        zs[i] = 0u;
    if (tid == 0)
        lmax_s = 1;
    __syncthreads();
    const uint32_t part = (n + nw - 1) / nw;
    const uint32_t pb = min(n, part * wave), pe = min(n, pb + part);
    uint32_t *hw = hist + (size_t)wave * D;
    int lmax = 1;
    for (uint32_t base = pb; base < pe; base += 256) {
        uint32_t zr[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t e = base + 64 * u + lane;
#pragma unroll
            for (int r = 0; r < 3; ++r)
                zr[u][r] = e < pe ? q.list[start + e].z[r] : 0xffff0000u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int lo = range_lo(zr[u][r]), hi = range_hi(zr[u][r]);
                if (hi >= lo) {
                    atomicAdd(&hw[lo], 1u);
                    lmax = max(lmax, hi - lo + 1);
                }
            }
    }
    atomicMax(&lmax_s, lmax);
    __syncthreads();
    // exclusive scan over z of the per-z totals: a segment of z per thread
    const int seg = (D + nt - 1) / nt, zb = min(D, tid * seg), ze = min(D, zb + seg);
    uint32_t sum = 0;
    for (int z = zb; z < ze; ++z)
        for (int w = 0; w < nw; ++w)
            sum += hist[(size_t)w * D + z];
    uint32_t incl = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t v = __shfl_up(incl, d, 64);
        if (lane >= d)
            incl += v;
    }
    if (lane == 63)
        wtot[wave] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (int w = 0; w < wave; ++w)
        run += wtot[w];
    uint32_t n_img = 0;
    for (int w = 0; w < nw; ++w)
        n_img += wtot[w];
    for (int z = zb; z < ze; ++z) {
        zst[z] = run;
        for (int w = 0; w < nw; ++w) {   // counts -> per-wave cursors
            const uint32_t c = hist[(size_t)w * D + z];
            hist[(size_t)w * D + z] = run;
            run += c;
        }
    }
    __syncthreads();
    const int lmx = lmax_s;
    for (int z = tid; z < D; z += nt) {
        const uint32_t first = zst[max(0, z - lmx + 1)];
        const uint32_t end = z + 1 < D ? zst[z + 1] : n_img;
        q.prange[((size_t)mc * D + z) * 2] = first;
        q.prange[((size_t)mc * D + z) * 2 + 1] = end;
    }
    int bits = 0;
    while ((1 << bits) < D)
        ++bits;
    const long long eb = 32ll * run_block(q, mc);
    const unsigned long long below = (1ull << lane) - 1ull;
    auto fetch = [&](uint32_t e, ListEntry &le) {
        le.atom = -1;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            le.z[r] = 0xffff0000u;   // empty range
            le.bh[r] = le.bl[r] = 0.f;
        }
        if (e < pe)
            le = q.list[start + e];
    };
    ListEntry nxt;
    fetch(pb + lane, nxt);
    for (uint32_t base = pb; base < pe; base += 64) {
        const ListEntry le = nxt;
        fetch(base + 64 + lane, nxt);   // the next chunk's entry, in flight meanwhile
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int lo = range_lo(le.z[r]), hi = range_hi(le.z[r]);
            const bool valid = hi >= lo;
            // lanes of this wave holding an image with the same start
            unsigned long long match = __ballot(valid);
            for (int bb = 0; bb < bits; ++bb) {
                const bool bit = valid && ((lo >> bb) & 1);
                const unsigned long long m1 = __ballot(bit);
                match &= bit ? m1 : ~m1;
            }
            if (valid) {
                const uint32_t rank = (uint32_t)__popcll(match & below);
                const uint32_t pos = hw[lo] + rank;
                if (rank == 0)
                    hw[lo] = pos + (uint32_t)__popcll(match);
                ZEntry zent;
                zent.atom = le.atom;
                zent.range = le.z[r];
                zent.bh = le.bh[r];
                zent.bl = le.bl[r];
                q.zlist[eb + pos] = zent;
            }
        }
    }
    if (tid == 0)
        q.ecount[mc] = n_img;
}


// Items of one channel-partition entry for the tile-column lists: each z
// range r of the atom (a z image) with each (y tile, x tile) pair its
// windows meet, enumerated r-major, then y, then x, over the atom's tile
// bit masks; sy and sx count the set bits passed (the factor slots).
struct MaskWalk {
    uint32_t my, mx, cy, cx;
    uint32_t z[MAX_IMAGES];
    int r, sy, sx, sy0;
    bool live;
    __device__ __forceinline__ int next_range(int from) const
    {
        int nr = MAX_IMAGES;
#pragma unroll
        for (int k = MAX_IMAGES - 1; k >= 0; --k)
            if (k >= from && range_hi(z[k]) >= range_lo(z[k]))
                nr = k;
        return nr;
    }
    // my_: the y tiles walked (a band of the atom's y mask), sy0_: the atom's
    // y slots below the band
    __device__ __forceinline__ void start(const ListEntry &e, uint32_t mx_, uint32_t my_, int sy0_)
    {
        mx = cx = mx_;
        my = cy = my_;
#pragma unroll
        for (int k = 0; k < MAX_IMAGES; ++k)
            z[k] = e.z[k];
        sy0 = sy = sy0_;
        sx = 0;
        r = next_range(0);
        live = r < MAX_IMAGES && mx != 0u && my != 0u;
    }
    __device__ __forceinline__ int ty() const { return __builtin_ctz(cy); }
    __device__ __forceinline__ int tx() const { return __builtin_ctz(cx); }
    __device__ __forceinline__ void next()
    {
        cx &= cx - 1u;
        ++sx;
        if (cx == 0u) {
            cx = mx;
            sx = 0;
            cy &= cy - 1u;
            ++sy;
            if (cy == 0u) {
                cy = my;
                sy = sy0;
                r = next_range(r + 1);
            }
        }
        live = r < MAX_IMAGES;
    }
    // z images (non-empty z ranges) of the entry
    __device__ __forceinline__ int ranges() const
    {
        int n = 0;
#pragma unroll
        for (int k = 0; k < MAX_IMAGES; ++k)
            n += range_hi(z[k]) >= range_lo(z[k]) ? 1 : 0;
        return n;
    }
    __device__ __forceinline__ uint32_t zs() const
    {
        uint32_t v = 0u;
#pragma unroll
        for (int k = 0; k < MAX_IMAGES; ++k)
            if (k == r)
                v = z[k];
        return v;
    }
};

// One workgroup per run (its stretch of the channel partition): every z
// image of the run goes into the list of each 32 x 32 (y, x) tile column
// its windows meet, the lists sorted by the image's z start -- a counting
// sort on the key (tile column, z start), D keys per column: per-wave key
// counts, a scan over (key, wave), then each wave places its part, equal
// keys within 64 entries ranked by a match over the key bits.  The scan
// gives each list's z boundaries directly: zstart[tc][z] = the first entry
// of key (tc, z), zstart[tc][D] = the list's end.
//
// A run's tile rows are dealt to G workgroups in bands (G > 1 when runs are
// few, to spread the sort over the chip): each walks all of the run's
// entries with the same split over its waves but counts and places only the
// items of its band's tile columns, after the items of the rows above it
// (counted from the tile masks), so the lists are the same for any G.
// Dynamic LDS: waves x (band rows x ntx) x D words.  blk: the sort's
// workgroup index (run x G + band).
__device__ void tsort_block(const GridParams &p, const CrystalParams &q, int G, unsigned blk, uint32_t *tls)
{
    __shared__ uint32_t tsum[1024];
    __shared__ uint32_t nabove;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nw = blockDim.x >> 6, nt = blockDim.x;
    const size_t mc = blk / (unsigned)G;
    const int g = (int)(blk % (unsigned)G);
    // the band's tile rows [ty0, ty1) and its keys ((ty - ty0) ntx + tx) D + z
    const int ty0 = g * q.nty / G, ty1 = (g + 1) * q.nty / G;
    const uint32_t rows_above = (uint32_t)((1ull << ty0) - 1ull);
    const uint32_t band = (uint32_t)((1ull << ty1) - 1ull) & ~rows_above;
    const int D = p.D, ntc = q.ntx * q.nty, K = (ty1 - ty0) * q.ntx * D;
    uint32_t *cnt = tls;   // [wave][K]: counts, then cursors
    const uint32_t start = q.mstart[mc], n = q.mcount[mc];
    const uint32_t base = (uint32_t)(32ll * run_block(q, mc) * (long long)(q.sx_max * q.sy_max));
    for (int i = tid; i < nw * K; i += nt)
        cnt[i] = 0u;
    if (tid == 0)
        nabove = 0u;
    __syncthreads();
    const uint32_t part = (n + nw - 1) / nw;
    const uint32_t pb = min(n, part * wave), pe = min(n, pb + part);
    uint32_t *cw = cnt + (size_t)wave * K;
    const int ntx = q.ntx;
    // the wave's first CHC chunks of 64 entries (and their atoms' tile masks)
    // stay in registers for both passes; later chunks are read again
    constexpr int CHC = 1;
    const int nch = (int)((pe - pb + 63) / 64);
    ListEntry lec[CHC];
    uint32_t mxc[CHC], myc[CHC];
#pragma unroll
    for (int ch = 0; ch < CHC; ++ch) {
        const uint32_t i = pb + 64 * ch + lane;
        lec[ch].atom = -1;
        if (ch < nch && i < pe)
            lec[ch] = q.list[start + i];
    }
#pragma unroll
    for (int ch = 0; ch < CHC; ++ch) {
        mxc[ch] = myc[ch] = 0u;
        if (lec[ch].atom >= 0) {
            mxc[ch] = q.tmask[2 * (size_t)lec[ch].atom];
            myc[ch] = q.tmask[2 * (size_t)lec[ch].atom + 1];
        }
    }
    // chunk ch of the wave's part: the lane's entry (atom -1: none) and masks
    auto chunk = [&](int ch, ListEntry &le, uint32_t &mx, uint32_t &my) {
#pragma unroll
        for (int k = 0; k < CHC; ++k)
            if (k == ch) {
                le = lec[k];
                mx = mxc[k];
                my = myc[k];
            }
        if (ch >= CHC) {
            const uint32_t i = pb + 64 * ch + lane;
            le.atom = -1;
            mx = my = 0u;
            if (i < pe) {
                le = q.list[start + i];
                mx = q.tmask[2 * (size_t)le.atom];
                my = q.tmask[2 * (size_t)le.atom + 1];
            }
        }
    };
    uint32_t above = 0u;   // the thread's items in rows above the band
    for (int ch = 0; ch < nch; ++ch) {
        ListEntry le;
        uint32_t mx, my;
        chunk(ch, le, mx, my);
        if (le.atom < 0)
            continue;
        MaskWalk iw;
        iw.start(le, mx, my & band, __popc(my & rows_above));
        above += (uint32_t)(iw.ranges() * __popc(mx) * __popc(my & rows_above));
        while (iw.live) {
            atomicAdd(&cw[((iw.ty() - ty0) * ntx + iw.tx()) * D + range_lo(iw.zs())], 1u);
            iw.next();
        }
    }
    if (above)
        atomicAdd(&nabove, above);
    __syncthreads();
    // key totals and their exclusive scan: a contiguous segment of keys per
    // thread, the segment sums scanned across the workgroup
    const int seg = (K + nt - 1) / nt, kb = min(K, tid * seg), ke = min(K, kb + seg);
    uint32_t ssum = 0;
    for (int k = kb; k < ke; ++k)
        for (int w = 0; w < nw; ++w)
            ssum += cnt[(size_t)w * K + k];
    tsum[tid] = ssum;
    __syncthreads();
    for (int d = 1; d < nt; d <<= 1) {
        const uint32_t v = tid >= d ? tsum[tid - d] : 0u;
        __syncthreads();
        tsum[tid] += v;
        __syncthreads();
    }
    uint32_t run = base + nabove + tsum[tid] - ssum;
    for (int k = kb; k < ke; ++k) {
        const int tc = ty0 * ntx + k / D, z = k % D;
        uint32_t *zs = q.zstart + (mc * ntc + tc) * (size_t)(D + 1);
        zs[z] = run;
        for (int w = 0; w < nw; ++w) {   // counts -> per-wave cursors
            const uint32_t v = cnt[(size_t)w * K + k];
            cnt[(size_t)w * K + k] = run;
            run += v;
        }
        if (z == D - 1)
            zs[D] = run;
    }
    __syncthreads();
    int kbits = 0;
    while ((1 << kbits) < K)
        ++kbits;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int ch = 0; ch < nch; ++ch) {
        ListEntry le;
        uint32_t mx, my;
        chunk(ch, le, mx, my);
        MaskWalk iw;
        iw.live = false;
        if (le.atom >= 0)
            iw.start(le, mx, my & band, __popc(my & rows_above));
        // one item per lane per round; equal keys ranked by lane
        while (__ballot(iw.live) != 0ull) {
            const uint32_t key =
                iw.live ? (uint32_t)(((iw.ty() - ty0) * ntx + iw.tx()) * D + range_lo(iw.zs())) : 0u;
            unsigned long long m = __ballot(iw.live);
            for (int b = 0; b < kbits; ++b) {
                const unsigned long long mb = __ballot(iw.live && ((key >> b) & 1u));
                m &= ((key >> b) & 1u) ? mb : ~mb;
            }
            if (iw.live) {
                const uint32_t rank = (uint32_t)__popcll(m & below);
                const uint32_t cur = cw[key];
                TileEntry te;
                te.atom = le.atom;
                const uint32_t zr = iw.zs();
                te.zs = (uint32_t)range_lo(zr) | ((uint32_t)range_hi(zr) << 12) |
                        ((uint32_t)iw.sy << 24) | ((uint32_t)iw.sx << 28);
                te.bh = 0.f;
                te.bl = 0.f;
#pragma unroll
                for (int k = 0; k < MAX_IMAGES; ++k)
                    if (k == iw.r) {
                        te.bh = le.bh[k];
                        te.bl = le.bl[k];
                    }
                q.tcl[cur + rank] = te;
                if (rank == 0)
                    cw[key] = cur + (uint32_t)__popcll(m);
                iw.next();
            }
        }
    }
}

// The tile sort and the factor-slot pass in one launch: the first n_sort
// workgroups sort (one per run and band; latency-bound, one per CU), the
// rest fill factor slots (8 atom-axes per wave) on the capacity the sort
// leaves free.  The two read only what the prep and partition passes wrote
// and write disjoint arrays.
// (At most 64 VGPRs: two 1024-thread workgroups share a CU, so slot
// workgroups run beside the sort's.)
template <typename YT, typename XT>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
cr_sort_slot_kernel(GridParams p, CrystalParams q, int G,
                                                            unsigned n_sort)
{
    extern __shared__ uint32_t tls[];
    if (blockIdx.x < n_sort) {
        tsort_block(p, q, G, blockIdx.x, tls);
        return;
    }
    slot_wave<YT, XT>(p, q, (long long)(blockIdx.x - n_sort) * (blockDim.x >> 6) + (threadIdx.x >> 6));
}

// ---------------------------------------------------------------------------
// MFMA plane tiles
// ---------------------------------------------------------------------------
// Workgroup (4 waves) = (run, tile row ty, tile pair tp, plane group zq);
// wave w owns the 32 x 32 tile (ty, 2 tp + w % 2) of the ZP planes from
// z0 = ZP (2 zq + w / 2) on (two neighbouring tiles make full 128-byte rows
// of a bf16 plane; neighbouring planes share their images, so one wave
// contracts the images of its ZP planes together).  The wave's entries are
// those of its tile column's list whose z start lies in
// [z0 - zwin + 1, z0 + ZP - 1] (zwin bounds the z windows of the channel's
// images: one type's windows for an unweighted channel; an entry whose
// window misses a plane gets phi_z = 0 there), taken 64 at a time, one per
// lane; their factor-slot rows are loaded before the first MFMA step.
// Every entry is taken in list order, so each voxel's sum has a fixed order.
constexpr int KS = 16;    // entries per bf16 MFMA step

__device__ __forceinline__ int entry_zlo(uint32_t zs) { return (int)(zs & 0xfffu); }
__device__ __forceinline__ int entry_zhi(uint32_t zs) { return (int)((zs >> 12) & 0xfffu); }

struct TileItem {
    size_t mc;
    int c, m, z0, ty, tx;
};

template <int ZP>
__device__ __forceinline__ TileItem tile_item(const GridParams &p, const CrystalParams &q)
{
    const unsigned ntp = (unsigned)(q.ntx + 1) / 2, nzq = (unsigned)(p.D + 2 * ZP - 1) / (2 * ZP);
    // the run is the fastest index: every stretch of items mixes the runs
    // (structures of very different density), so no XCD ends on a run of
    // heavy tiles
    unsigned b = xcd_block();
    TileItem it;
    const unsigned nmc = (unsigned)p.n_mol * (unsigned)p.C;
    const unsigned mc = b % nmc;
    b /= nmc;
    const int zq = (int)(b % nzq);
    b /= nzq;
    const int tp = (int)(b % ntp);
    b /= ntp;
    it.ty = (int)b;
    it.mc = (size_t)mc;
    it.c = (int)(mc / (unsigned)p.n_mol);
    it.m = (int)(mc % (unsigned)p.n_mol);
    const int w = (int)(threadIdx.x >> 6);
    it.tx = 2 * tp + (w & 1);
    it.z0 = ZP * (2 * zq + (w >> 1));
    return it;
}

// The wave's range [first, end) of its tile column's list.
template <int ZP>
__device__ __forceinline__ void tile_range(const GridParams &p, const CrystalParams &q,
                                           const TileItem &it, uint32_t &first, uint32_t &end)
{
    first = end = 0u;
    if (it.tx >= q.ntx || it.z0 >= p.D)
        return;
    const uint32_t *zs =
        q.zstart + (it.mc * (size_t)(q.ntx * q.nty) + it.ty * q.ntx + it.tx) * (size_t)(p.D + 1);
    first = zs[max(0, it.z0 - q.zwin[it.c] + 1)];
    end = zs[min(it.z0 + ZP, p.D)];
}

// One list entry per lane: phi_z of its image at each of the wave's planes
// (times the channel weight; 0 where its z window misses the plane, or past
// the range) and the indices of its y and x factor slots.  inv2s2_c,
// isq2s_c: the channel's constants, used when channels are not weighted
// (the image's type is then the channel).
template <int ZP>
struct LaneImage {
    float gz[ZP];
    uint32_t yslot, xslot;
};

// List entry e, or an empty one (atom -1) past the range.
__device__ __forceinline__ TileEntry tile_entry(const CrystalParams &q, uint32_t e, uint32_t end)
{
    TileEntry te;
    te.atom = -1;
    te.zs = 0u;
    te.bh = te.bl = 0.f;
    if (e < end)
        te = q.tcl[e];
    return te;
}

template <int ZP>
__device__ __forceinline__ LaneImage<ZP> lane_image(const GridParams &p, const CrystalParams &q,
                                                    const TileEntry &te, int z0, int c,
                                                    float inv2s2_c, float isq2s_c)
{
    LaneImage<ZP> li;
#pragma unroll
    for (int k = 0; k < ZP; ++k)
        li.gz[k] = 0.f;
    li.yslot = li.xslot = 0u;
    if (te.atom >= 0) {
        const int zlo = entry_zlo(te.zs), zhi = min(entry_zhi(te.zs), p.D - 1);
        float inv2s2 = inv2s2_c, isq2s = isq2s_c, wgt = 1.f;
        if (p.weights) {
            const int ti = q.table[te.atom].type;
            inv2s2 = p.inv2s2[ti];
            isq2s = p.isq2s[ti];
            wgt = p.weights[(size_t)te.atom * p.C + c];
        }
        if (p.box != 0) {
            // the ZP planes' masses from ZP + 1 shared edges
            float f[ZP];
            box_fixed<ZP>(te.bh, te.bl, p.h[2], z0, isq2s, f);
#pragma unroll
            for (int k = 0; k < ZP; ++k)
                if (z0 + k >= zlo && z0 + k <= zhi)
                    li.gz[k] = f[k] * wgt;
        } else {
#pragma unroll
            for (int k = 0; k < ZP; ++k) {
                const int z = z0 + k;
                if (z >= zlo && z <= zhi)
                    li.gz[k] = gauss1d(offset_at(te.bh, te.bl, p.h[2], z), inv2s2) * wgt;
            }
        }
        li.yslot = (uint32_t)te.atom * (uint32_t)q.sy_max + ((te.zs >> 24) & 15u);
        li.xslot = (uint32_t)te.atom * (uint32_t)q.sx_max + (te.zs >> 28);
    }
    return li;
}

// A wave's 32 x 32 tiles (accumulators: lane l holds column l % 32 of rows
// 8 (e / 4) + 4 (l / 32) + e % 4) go through the wave's LDS buffer as T, one
// plane at a time, then out in 16-byte pieces, whole 32-element row
// segments (no bounds tests when the tile lies inside the plane).  Rows and
// columns past the plane edge are not written; unaligned rows fall back to
// element stores.
template <typename T>
constexpr int tile_lrow() { return 32 + 16 / (int)sizeof(T); }   // padded LDS row (elements)

template <typename T>
__device__ __forceinline__ void tile_to_lds(const f32x16 &acc, T *ls)
{
    constexpr int LROW = tile_lrow<T>();
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int e = 0; e < 16; ++e)
        ls[(8 * (e >> 2) + 4 * (lane >> 5) + (e & 3)) * LROW + (lane & 31)] = (T)acc[e];
}

template <typename T>
__device__ __forceinline__ void lds_to_global(T *out, int H, int W, int y0, int x0, bool nt, const T *ls)
{
    constexpr int LROW = tile_lrow<T>();
    constexpr int EPL = 16 / (int)sizeof(T);         // elements per 16-byte piece
    constexpr int LPR = 32 / EPL;                    // lanes per row
    constexpr int RPI = 64 / LPR;                    // rows per store instruction
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63;
    const bool vec = ((size_t)W * sizeof(T)) % 16 == 0 && ((uintptr_t)out & 15) == 0;
    if (vec && y0 + 32 <= H && x0 + 32 <= W) {
        // the whole tile lies inside the plane: every piece is a 16-byte store
        const int r0 = lane / LPR, cs = EPL * (lane % LPR);
        const T *src = ls + r0 * LROW + cs;
        T *dst = out + (size_t)(y0 + r0) * W + x0 + cs;
#pragma unroll
        for (int k = 0; k < 32 / RPI; ++k) {
            const u4 v = *(const u4 *)(src + RPI * k * LROW);
            if (nt)
                __builtin_nontemporal_store(v, (u4 *)(dst + (size_t)(RPI * k) * W));
            else
                *(u4 *)(dst + (size_t)(RPI * k) * W) = v;
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < 32 / RPI; ++k) {
        const int r = RPI * k + lane / LPR, cs = EPL * (lane % LPR);
        const int y = y0 + r, x = x0 + cs;
        if (y >= H || x >= W)
            continue;
        const T *src = ls + r * LROW + cs;
        T *dst = out + (size_t)y * W + x;
        if (vec && x + EPL <= W) {
            const u4 v = *(const u4 *)src;
            if (nt)
                __builtin_nontemporal_store(v, (u4 *)dst);
            else
                *(u4 *)dst = v;
        } else {
            for (int u = 0; u < EPL && x + u < W; ++u)
                dst[u] = src[u];
        }
    }
}

// The wave's ZP planes from z0 on (those below D) through ls (32 x
// tile_lrow<T>() elements).
template <typename T, int ZP>
__device__ __forceinline__ void store_tiles(const GridParams &p, const TileItem &it, const f32x16 (&acc)[ZP],
                                            T *ls)
{
#pragma unroll
    for (int k = 0; k < ZP; ++k) {
        const int z = it.z0 + k;
        if (z >= p.D)
            break;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");   // the buffer's last reads are done
        tile_to_lds<T>(acc[k], ls);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        T *out = (T *)p.out + (((size_t)it.m * p.C + it.c) * p.D + z) * (size_t)p.H * p.W;
        lds_to_global<T>(out, p.H, p.W, 32 * it.ty, 32 * it.tx, p.nt_store != 0, ls);
    }
}

// bf16 grids: per 16-entry step, lane l stages the image pair 2 (l / 8),
// 2 (l / 8) + 1 of the step on rows (columns) 4 (l % 8) .. + 3: per plane the
// four rows of phi_z phi_y (FP32 products, each pair of images rounded to
// bf16 by one conversion) and, once per step, of phi_x go into the wave's
// LDS buffer as [row][16 entries] (4 bytes per row and pair); the wave then
// reads its fragments and each plane takes one v_mfma_f32_32x32x16_bf16.
// The y slots are float, the x slots bf16.  Each lane publishes its entry's
// phi_z and slot indices in the wave's LDS once per 64 entries; the slot
// rows of the next step are loaded while the current step is staged and
// contracted.
constexpr int AST = 24;   // staged row: 16 entries + 8 bf16 of padding (48 B)

template <int ZP, int KCH>
__global__ void __launch_bounds__(256) cr_tile_bf16_kernel(GridParams p, CrystalParams q)
{
    static_assert(KCH == KS, "one step of entries per load group");
    static_assert(ZP == 4, "phi_z of the wave's planes is published as one float4 per entry");
    // bf16 per wave: staging 2 x 32 x AST (phi_x, then one plane's A at a
    // time) >= one output tile 32 x tile_lrow
    constexpr int WBUF = 2 * 32 * AST;
    static_assert(WBUF >= 32 * tile_lrow<__bf16>(), "the output tile fits the staging buffer");
    __shared__ __attribute__((aligned(16))) __bf16 lds[4][WBUF];
    __shared__ float4 gzs[4][64];   // per wave: phi_z of its 64 entries at its planes
    __shared__ uint2 sls[4][64];    // per wave: their (y slot, x slot)
    const TileItem it = tile_item<ZP>(p, q);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t first, end;
    tile_range<ZP>(p, q, it, first, end);
    if (it.tx >= q.ntx || it.z0 >= p.D)
        return;
    const float inv2s2_c = p.inv2s2[it.c], isq2s_c = p.isq2s[it.c];
    __bf16 *Bs = lds[wave], *As = lds[wave] + 32 * AST;
    const int ip = lane >> 3, g = lane & 7;   // image pair, row group
    const int wo = 4 * g * AST + 2 * ip;      // the lane's staged pair, row 4 g
    const int fo = (lane & 31) * AST + 8 * (lane >> 5);
    // slot rows by 32-bit byte offsets (the plan keeps each slot array below 4 GiB)
    const char *ybase = (const char *)q.yval, *xbase = (const char *)q.xval;
    f32x16 acc[ZP];
#pragma unroll
    for (int k = 0; k < ZP; ++k)
#pragma unroll
        for (int e = 0; e < 16; ++e)
            acc[k][e] = 0.f;
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b4 __attribute__((ext_vector_type(4)));
    for (uint32_t c64 = first; c64 < end; c64 += 64) {
        const LaneImage<ZP> li =
            lane_image<ZP>(p, q, tile_entry(q, c64 + lane, end), it.z0, it.c, inv2s2_c, isq2s_c);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");   // the last chunk's reads are done
        gzs[wave][lane] = make_float4(li.gz[0], li.gz[1], li.gz[2], li.gz[3]);
        sls[wave][lane] = make_uint2(li.yslot, li.xslot);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        const int nv = (int)min(64u, end - c64);   // entries of this chunk
        const int nst = (nv + KS - 1) / KS;
        // slot rows of the lane's pair in step st, loaded without branches
        // (entries past the chunk's have slot indices 0, an allocated slot;
        // they are zeroed where used)
        auto load_step = [&](int st, float4 (&ya)[2], b4 (&xb)[2]) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const uint2 sl = sls[wave][min(KS * st + 2 * ip + u, 63)];
                ya[u] = *(const float4 *)(ybase + (sl.x * 128u + 16u * g));
                xb[u] = *(const b4 *)(xbase + (sl.y * 64u + 8u * g));
            }
        };
        auto mma_step = [&](int st, const float4 (&ya)[2], const b4 (&xb)[2]) {
            const int e0 = KS * st + 2 * ip;
            const bool v0 = e0 < nv, v1 = e0 + 1 < nv;
            const b4 z4 = {(__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
            const b4 x0 = v0 ? xb[0] : z4, x1 = v1 ? xb[1] : z4;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const b2 pb = {x0[r], x1[r]};
                *(uint32_t *)(Bs + r * AST + wo) = __builtin_bit_cast(uint32_t, pb);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            const bf16x8 bf = *(const bf16x8 *)(Bs + fo);
            const float4 ya0 = v0 ? ya[0] : make_float4(0.f, 0.f, 0.f, 0.f);
            const float4 ya1 = v1 ? ya[1] : make_float4(0.f, 0.f, 0.f, 0.f);
            const float y0[4] = {ya0.x, ya0.y, ya0.z, ya0.w};
            const float y1[4] = {ya1.x, ya1.y, ya1.z, ya1.w};
            const float4 g0 = gzs[wave][e0], g1 = gzs[wave][e0 + 1];   // e0 + 1 < 64
            const float gz0[4] = {g0.x, g0.y, g0.z, g0.w}, gz1[4] = {g1.x, g1.y, g1.z, g1.w};
#pragma unroll
            for (int k = 0; k < ZP; ++k) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const f2 pr = {y0[r] * gz0[k], y1[r] * gz1[k]};
                    *(uint32_t *)(As + r * AST + wo) = __builtin_bit_cast(uint32_t, __builtin_convertvector(pr, b2));
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                const bf16x8 af = *(const bf16x8 *)(As + fo);
                acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bf, acc[k], 0, 0, 0);
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            }
        };
        // the next step's loads are issued unconditionally (in bounds past the
        // chunk too), so the wait before each step covers only its own loads
        float4 ya0[2], ya1[2];
        b4 xb0[2], xb1[2];
        load_step(0, ya0, xb0);
        for (int st = 0; st < nst; st += 2) {
            load_step(st + 1, ya1, xb1);
            mma_step(st, ya0, xb0);
            if (st + 1 >= nst)
                break;
            load_step(st + 2, ya0, xb0);
            mma_step(st + 1, ya1, xb1);
        }
    }
    store_tiles<__bf16, ZP>(p, it, acc, lds[wave]);
}

// fp32 grids: v_mfma_f32_32x32x2_f32 takes one value of A and one of B per
// lane -- lane l: entry l / 32 of a pair of entries, row (A) or column (B)
// l % 32 -- which is one float of that entry's y or x slot: the slots are
// read straight into the operands (no transposition), A scaled by phi_z of
// each plane in FP32.  Exact FP32 products, FP32 accumulation; per pair of
// entries one MFMA per plane.  Each lane publishes its entry's phi_z and slot
// indices in the wave's LDS once per 64 entries; the slot values of the next
// PB pairs are loaded while the current PB pairs are contracted.
template <int ZP, int KCH>
__global__ void __launch_bounds__(256) cr_tile_f32_kernel(GridParams p, CrystalParams q)
{
    static_assert(KCH == 64, "one list entry per lane");
    static_assert(ZP == 4, "phi_z of the wave's planes is published as one float4 per entry");
    constexpr int PB = 8;   // entry pairs per load group
    __shared__ __attribute__((aligned(16))) float lds[4][32 * tile_lrow<float>()];
    __shared__ float4 gzs[4][64];   // per wave: phi_z of its 64 entries at its planes
    __shared__ uint2 sls[4][64];    // per wave: their (y slot, x slot)
    const TileItem it = tile_item<ZP>(p, q);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t first, end;
    tile_range<ZP>(p, q, it, first, end);
    if (it.tx >= q.ntx || it.z0 >= p.D)
        return;
    const float inv2s2_c = p.inv2s2[it.c], isq2s_c = p.isq2s[it.c];
    const uint32_t j = lane & 31;
    const int hi = lane >> 5;
    // slot rows by 32-bit byte offsets (the plan keeps each slot array below 4 GiB)
    const char *yb = (const char *)q.yval, *xb = (const char *)q.xval;
    f32x16 acc[ZP];
#pragma unroll
    for (int k = 0; k < ZP; ++k)
#pragma unroll
        for (int e = 0; e < 16; ++e)
            acc[k][e] = 0.f;
    for (uint32_t c0 = first; c0 < end; c0 += KCH) {
        const LaneImage<ZP> li =
            lane_image<ZP>(p, q, tile_entry(q, c0 + lane, end), it.z0, it.c, inv2s2_c, isq2s_c);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");   // the last chunk's reads are done
        gzs[wave][lane] = make_float4(li.gz[0], li.gz[1], li.gz[2], li.gz[3]);
        sls[wave][lane] = make_uint2(li.yslot, li.xslot);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        const int nv = (int)min((uint32_t)KCH, end - c0);   // entries of this chunk
        const int npair = (nv + 1) / 2;
        // slot values of pairs p0 .. p0 + PB - 1, loaded without branches (the
        // entry index is clamped to the wave's 64; entries past the chunk's
        // have slot indices 0, an allocated slot) and zeroed where used
        auto load_group = [&](int p0, float (&av)[PB], float (&bv)[PB]) {
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const uint2 sl = sls[wave][min(2 * (p0 + u) + hi, 63)];
                av[u] = *(const float *)(yb + (sl.x * 128u + 4u * j));
                bv[u] = *(const float *)(xb + (sl.y * 128u + 4u * j));
            }
        };
        auto mma_group = [&](int p0, const float (&av)[PB], const float (&bv)[PB]) {
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                if (p0 + u >= npair)
                    break;
                const int src = 2 * (p0 + u) + hi;   // < 64 as p0 + u < 32
                const float4 g = gzs[wave][src];
                const float a = src < nv ? av[u] : 0.f, b = src < nv ? bv[u] : 0.f;
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a * g.x, b, acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a * g.y, b, acc[1], 0, 0, 0);
                acc[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a * g.z, b, acc[2], 0, 0, 0);
                acc[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a * g.w, b, acc[3], 0, 0, 0);
            }
        };
        // the next group's loads are issued unconditionally (in bounds past
        // the chunk too), so the waits of a group cover only its own loads
        float a0[PB], b0[PB], a1[PB], b1[PB];
        load_group(0, a0, b0);
        for (int p0 = 0; p0 < npair; p0 += 2 * PB) {
            load_group(p0 + PB, a1, b1);
            mma_group(p0, a0, b0);
            if (p0 + PB >= npair)
                break;
            load_group(p0 + 2 * PB, a0, b0);
            mma_group(p0 + PB, a1, b1);
        }
    }
    store_tiles<float, ZP>(p, it, acc, lds[wave]);
}

constexpr int ZP_BF16 = 4;    // planes per wave of the bf16 tile kernel
constexpr int KCH_BF16 = 16;  // entries per load group of the bf16 tile kernel (one step)
constexpr int ZP_F32 = 4;     // planes per wave of the fp32 tile kernel
constexpr int KCH_F32 = 64;   // entries per chunk of the fp32 tile kernel

// FP32 vector-ALU form: one workgroup (256 threads) per (structure, channel,
// z); the plane's images are the range [first, end) of the run's z order.
// Per 32-image step the images' dense factor rows go to LDS -- phi_x, and
// phi_z(z) phi_y -- evaluated where the windows are (8 threads per image),
// and, per 32 x 32 output tile, a bit mask of the step's images whose
// window meets the tile.  Wave w owns tiles w, w + 4, ...; lane l owns the
// 4 x 4 voxels at rows 4 (l / 8), columns 4 (l % 8) of each: for every
// image in the tile's mask (lowest bit first) it reads 4 phi_y and 4 phi_x
// values and does 16 FMAs.  Each voxel sums its images in z order, in FP32.
template <typename T, int TMAX, bool BOX>
__global__ void __launch_bounds__(256) cr_window_kernel(GridParams p, CrystalParams q)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int C = p.C, D = p.D, H = p.H, W = p.W;
    const int W32 = (W + 31) & ~31, H32 = (H + 31) & ~31;
    const int ntx = W32 / 32, nty = H32 / 32, ntiles = ntx * nty;
    float *gx = (float *)smem;                    // [KC][W32] phi_x
    float *gy = gx + KC * W32;                    // [KC][H32] phi_z(z) phi_y
    uint32_t *tmask = (uint32_t *)(gy + KC * H32);   // [ntiles] images meeting each tile
    // the run is the fastest index (every stretch of planes mixes structures
    // of very different density), then z
    const unsigned b = xcd_block(), nmc = (unsigned)p.n_mol * (unsigned)C;
    const int z = (int)(b / nmc);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const size_t mc = b % nmc;
    const int c = (int)(mc / (unsigned)p.n_mol), m = (int)(mc % (unsigned)p.n_mol);
    const uint32_t first = q.prange[((size_t)mc * D + z) * 2];
    const uint32_t end = q.prange[((size_t)mc * D + z) * 2 + 1];
    const long long eb = 32ll * run_block(q, mc);
    constexpr bool box = BOX;   // the value form (a separate instance: its
                                // registers stay out of the point form's)
    const int ly = 4 * (lane >> 3), lx = 4 * (lane & 7);
    float acc[TMAX][4][4];
#pragma unroll
    for (int i = 0; i < TMAX; ++i)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                acc[i][rr][e] = 0.f;

    // The thread's image of each step (image tid / 8 of the step, an eighth
    // of its windows per thread).  Point form: its z-list entry is loaded one
    // step ahead, at the start of the previous step's factor pass, and the
    // first two x and y window ranges of its atom (an atom has a second
    // range near a periodic boundary) during the previous step's
    // accumulation, so a factor pass waits on global memory only for a
    // third range.  The loads take indices clamped into the plane's range,
    // so they need no branch.  The box form, whose edge walk needs more
    // registers, loads them at the start of each factor pass.
    constexpr bool PRE = !BOX;
    const int kimg = tid >> 3, part = tid & 7;
    struct Ranges2 {
        int n[2], lo[2][2], hi[2][2];   // [axis][range]
        float bh[2][2], bl[2][2];
    };
    auto entry_at = [&](uint32_t k0n) -> ZEntry {
        return q.zlist[eb + min(k0n + (uint32_t)kimg, end - 1u)];
    };
    auto ranges2 = [&](const ZEntry &ze) -> Ranges2 {
        const AtomWindow &w = q.table[ze.atom];
        Ranges2 r;
#pragma unroll
        for (int ax = 0; ax < 2; ++ax) {
            r.n[ax] = w.n[ax];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                r.lo[ax][j] = w.lo[ax][j];
                r.hi[ax][j] = w.hi[ax][j];
                r.bh[ax][j] = w.bh[ax][j];
                r.bl[ax][j] = w.bl[ax][j];
            }
        }
        return r;
    };
    ZEntry ze{};
    Ranges2 rg{};
    if (PRE && first < end) {
        ze = entry_at(first);
        rg = ranges2(ze);
    }
    for (uint32_t k0 = first; k0 < end; k0 += KC) {
        const int kn = (int)min((uint32_t)KC, end - k0);
        ZEntry ze_next{};
        if (PRE)
            ze_next = entry_at(k0 + KC);   // in flight through this factor pass
        else
            ze = entry_at(k0);
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
        for (int i = tid; i < 8 * (W32 + H32); i += blockDim.x)
            ((u4 *)gx)[i] = u4{0u, 0u, 0u, 0u};
        for (int i = tid; i < ntiles; i += blockDim.x)
            tmask[i] = 0u;
        __syncthreads();
        if (kimg < kn && z >= range_lo(ze.range) && z <= range_hi(ze.range)) {
            const int k = kimg;
            const int ti = image_type(p, q, ze.atom, c);
            const float inv2s2 = p.inv2s2[ti], isq2s = p.isq2s[ti];
            const float g = factor1d(box, ze.bh, ze.bl, p.h[2], z, inv2s2, isq2s) *
                            image_weight(p, ze.atom, c);
            const AtomWindow &w = q.table[ze.atom];
            uint32_t tx = 0u, ty = 0u;   // tile columns / rows the windows meet
            // each of the image's 8 threads takes a contiguous eighth of
            // each window (the box form walks its edges once)
            auto row_x = [&](int wlo, int whi, float bh, float bl) {
                for (int t = wlo >> 5; t <= (whi >> 5); ++t)
                    tx |= 1u << t;
                const int L8 = (whi - wlo + 8) >> 3;
                const int lo = wlo + part * L8, hi = min(whi, lo + L8 - 1);
                if (box)
                    box_walk<false>(bh, bl, p.h[0], lo, hi, isq2s, 1.f, gx + k * W32);
                else
                    for (int v = lo; v <= hi; ++v)
                        gx[k * W32 + v] = gauss1d(offset_at(bh, bl, p.h[0], v), inv2s2);
            };
            auto row_y = [&](int wlo, int whi, float bh, float bl) {
                for (int t = wlo >> 5; t <= (whi >> 5); ++t)
                    ty |= 1u << t;
                const int L8 = (whi - wlo + 8) >> 3;
                const int lo = wlo + part * L8, hi = min(whi, lo + L8 - 1);
                if (box)
                    box_walk<true>(bh, bl, p.h[1], lo, hi, isq2s, g, gy + k * H32);
                else
                    for (int v = lo; v <= hi; ++v)
                        gy[k * H32 + v] = g * gauss1d(offset_at(bh, bl, p.h[1], v), inv2s2);
            };
            if (PRE) {
                // a listed image meets the grid on every axis: at least one range each
                row_x(rg.lo[0][0], rg.hi[0][0], rg.bh[0][0], rg.bl[0][0]);
                if (rg.n[0] > 1)
                    row_x(rg.lo[0][1], rg.hi[0][1], rg.bh[0][1], rg.bl[0][1]);
                for (int r = 2; r < rg.n[0]; ++r)
                    row_x(w.lo[0][r], w.hi[0][r], w.bh[0][r], w.bl[0][r]);
                row_y(rg.lo[1][0], rg.hi[1][0], rg.bh[1][0], rg.bl[1][0]);
                if (rg.n[1] > 1)
                    row_y(rg.lo[1][1], rg.hi[1][1], rg.bh[1][1], rg.bl[1][1]);
                for (int r = 2; r < rg.n[1]; ++r)
                    row_y(w.lo[1][r], w.hi[1][r], w.bh[1][r], w.bl[1][r]);
            } else {
                for (int r = 0; r < w.n[0]; ++r)
                    row_x(w.lo[0][r], w.hi[0][r], w.bh[0][r], w.bl[0][r]);
                for (int r = 0; r < w.n[1]; ++r)
                    row_y(w.lo[1][r], w.hi[1][r], w.bh[1][r], w.bl[1][r]);
            }
            if (part == 0)
                for (int tr = 0; tr < nty; ++tr)
                    if ((ty >> tr) & 1u)
                        for (int tc = 0; tc < ntx; ++tc)
                            if ((tx >> tc) & 1u)
                                atomicOr(&tmask[tr * ntx + tc], 1u << k);
        }
        __syncthreads();
        // the next step's ranges, in flight through the accumulation
        if (PRE) {
            ze = ze_next;
            rg = ranges2(ze);
        }
#pragma unroll
        for (int i = 0; i < TMAX; ++i) {
            const int t = wave + 4 * i;
            if (t >= ntiles)
                break;
            const int y = 32 * (t / ntx) + ly, x = 32 * (t % ntx) + lx;
            // the tile's mask is the same for the whole wave: its walk and the
            // rows' offsets run on the scalar unit
            uint32_t mk = (uint32_t)__builtin_amdgcn_readfirstlane((int)tmask[t]);
            const float *gyl = gy + y, *gxl = gx + x;
            while (mk) {
                const int k = __builtin_ctz(mk);
                mk &= mk - 1u;
                const float4 g4 = *(const float4 *)(gyl + k * H32);
                const float4 f4 = *(const float4 *)(gxl + k * W32);
                const float gr[4] = {g4.x, g4.y, g4.z, g4.w}, fr[4] = {f4.x, f4.y, f4.z, f4.w};
#pragma unroll
                for (int rr = 0; rr < 4; ++rr)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc[i][rr][e] = __builtin_fmaf(gr[rr], fr[e], acc[i][rr][e]);
            }
        }
        __syncthreads();
    }
    T *out = (T *)p.out + (((size_t)m * C + c) * D + z) * (size_t)H * W;
    const bool vec_ok = (W & 3) == 0 && ((uintptr_t)p.out & 15) == 0;
#pragma unroll
    for (int i = 0; i < TMAX; ++i) {
        const int t = wave + 4 * i;
        if (t >= ntiles)
            break;
        const int y0 = 32 * (t / ntx) + ly, x0 = 32 * (t % ntx) + lx;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int y = y0 + rr;
            if (y >= H)
                continue;
            T *o = out + (size_t)y * W + x0;
            if (vec_ok && x0 + 3 < W) {
                store_vec<T, 4>(o, acc[i][rr], p.nt_store != 0);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (x0 + e < W) {
                        const float v[1] = {acc[i][rr][e]};
                        store_vec<T, 1>(o + e, v, p.nt_store != 0);
                    }
            }
        }
    }
}

size_t crystal_plane_lds(int form, int H, int W)
{
    if (form == PG_FORM_MFMA)   // all static: the waves' staging and store buffers
        return 0;
    const int W32 = (W + 31) & ~31, H32 = (H + 31) & ~31;
    return (size_t)KC * (W32 + H32) * sizeof(float) + (size_t)(W32 / 32) * (H32 / 32) * 4;
}

int crystal_axis_slots(int N, int wmax, bool periodic)
{
    const int tiles = (N + 31) / 32;
    const int per_range = std::min(tiles, (std::max(wmax, 1) - 1 + 31) / 32 + 1);
    return std::min(tiles, (periodic ? MAX_IMAGES : 1) * per_range);
}

// waves of the z-sort workgroup: up to 16, within 64 KB of LDS counters
int crystal_zsort_waves(int D)
{
    return std::max(1, std::min(16, 16000 / D - 1));
}

size_t crystal_zsort_lds(int D)
{
    return (size_t)(crystal_zsort_waves(D) + 1) * D * sizeof(uint32_t);
}

// 32 x 32 tiles per wave of the vector form (0: plane too large; tile masks
// are 32-bit per axis)
int crystal_window_runs(int H, int W)
{
    const int ty = (H + 31) / 32, tx = (W + 31) / 32;
    if (ty > 32 || tx > 32)
        return 0;
    const int tiles = tx * ty;
    for (int r = 1; r <= 8; r <<= 1)
        if (tiles <= 4 * r)
            return r;
    return 0;
}

// waves of the tile-sort workgroup: up to 16, within 128 KB of LDS key
// counters (K = tile columns x D keys, at most 32768)
int crystal_tsort_waves(int K)
{
    return std::max(1, std::min(16, 32768 / std::max(K, 1)));
}

size_t crystal_tsort_lds(int K)
{
    return (size_t)crystal_tsort_waves(K) * K * sizeof(uint32_t);
}

int crystal_slot_bytes(int out_dtype, int axis)
{
    return (out_dtype == PG_OUT_F32 || axis == 1) ? 4 : 2;
}

int crystal_tile_planes(int out_dtype)
{
    return out_dtype == PG_OUT_F32 ? ZP_F32 : ZP_BF16;
}

int crystal_prep_blocks(long long n_atoms)
{
    return (int)((n_atoms + PREP_BLOCK - 1) / PREP_BLOCK);
}

// The vector-form instance for a grid type, tiles per wave and value form.
template <bool BOX>
static const void *window_kernel_for(int out_dtype, int r)
{
    if (out_dtype == PG_OUT_F32)
        return r == 1 ? (const void *)cr_window_kernel<float, 1, BOX>
             : r == 2 ? (const void *)cr_window_kernel<float, 2, BOX>
             : r == 4 ? (const void *)cr_window_kernel<float, 4, BOX>
             : r == 8 ? (const void *)cr_window_kernel<float, 8, BOX> : nullptr;
    return r == 1 ? (const void *)cr_window_kernel<__bf16, 1, BOX>
         : r == 2 ? (const void *)cr_window_kernel<__bf16, 2, BOX>
         : r == 4 ? (const void *)cr_window_kernel<__bf16, 4, BOX>
         : r == 8 ? (const void *)cr_window_kernel<__bf16, 8, BOX> : nullptr;
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
        hipLaunchKernelGGL(cr_prep_kernel, dim3((unsigned)q.nblk), dim3(3 * PREP_BLOCK), 0, s, p, q);
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
        // the tile-column lists of every run (tile-row bands per run: enough
        // workgroups to spread the sort over the chip when runs are few) and,
        // in the same launch, the factor slots of every atom (8 atom-axes per
        // wave).  y slots are float in both forms (phi_z phi_y is formed in
        // FP32); x slots bf16 for bf16 grids, float for fp32 grids.
        const int G = (int)std::max<long long>(1, std::min<long long>(q.nty, (256 + nmc - 1) / nmc));
        const int K = ((q.nty + G - 1) / G) * q.ntx * p.D;   // keys of the widest band
        const size_t tl = crystal_tsort_lds(K);
        const int tw = crystal_tsort_waves(K);
        const long long slot_waves = (2 * p.n_atoms + 7) / 8;
        const long long blocks = nmc * G + (slot_waves + tw - 1) / tw;
        if (blocks > 0x7fffffffLL)
            return hipErrorInvalidValue;
        const void *ks = out_dtype == PG_OUT_F32 ? (const void *)cr_sort_slot_kernel<float, float>
                                                 : (const void *)cr_sort_slot_kernel<float, uint16_t>;
        if (tl > 65536) {
            e = hipFuncSetAttribute(ks, hipFuncAttributeMaxDynamicSharedMemorySize, (int)tl);
            if (e != hipSuccess)
                return e;
        }
        GridParams ps = p;
        CrystalParams qs = q;
        int Gs = G;
        unsigned n_sort = (unsigned)(nmc * G);
        void *sargs[] = {&ps, &qs, &Gs, &n_sort};
        if ((e = hipLaunchKernel(ks, dim3((unsigned)blocks), dim3(64 * tw), sargs, tl, s)) != hipSuccess)
            return e;
        const int zp = out_dtype == PG_OUT_F32 ? ZP_F32 : ZP_BF16;
        k = out_dtype == PG_OUT_F32 ? (const void *)cr_tile_f32_kernel<ZP_F32, KCH_F32>
                                    : (const void *)cr_tile_bf16_kernel<ZP_BF16, KCH_BF16>;
        grid = nmc * q.nty * ((q.ntx + 1) / 2) * ((p.D + 2 * zp - 1) / (2 * zp));
    } else {
        const size_t zl = crystal_zsort_lds(p.D);
        if (zl > 65536) {
            e = hipFuncSetAttribute((const void *)cr_zsort_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)zl);
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(cr_zsort_kernel, dim3((unsigned)nmc), dim3(64 * crystal_zsort_waves(p.D)), zl,
                           s, p, q);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        const int r = crystal_window_runs(p.H, p.W);
        k = p.box ? window_kernel_for<true>(out_dtype, r) : window_kernel_for<false>(out_dtype, r);
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
