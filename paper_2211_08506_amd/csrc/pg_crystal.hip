// pg_crystal.hip -- large / dense structures (periodic crystal cells, big
// clusters) on gfx950.
//
// Structures with more atoms than the molecule window kernel stages in LDS
// take this path.  Set-up, all on the GPU and free of order-dependent
// atomics in anything that reaches the output:
//   prep:    three threads per atom (one per axis): exact window ranges
//            (nearest periodic images included) into the atom's record, and
//            counts of the atom per (channel, structure) and per (channel,
//            prep block);
//   scan:    exclusive scans of both count arrays in channel-major order;
//   place:   a stable partition of all atoms by channel (ballot ranks within
//            a block): channel c's atoms in index order, so each (structure,
//            channel) pair -- a "run" -- is one contiguous stretch of the list;
//   zsort:   per run, the atoms' z images sorted stably by window start, so
//            each plane's images are one contiguous range of that order.
// Then one of two plane forms, one workgroup per (structure, channel, z
// plane[, 128 x 128 super-tile]):
//   mfma:    the plane is a product of two factor matrices (separability of
//            the Gaussian and of the cube cutoff, Sec. III-A / IV-C):
//            G[y][x] = sum_k phi_z^k(z) phi_y^k(y) phi_x^k(x).  An operand
//            kernel writes phi_y and phi_x of every image once, in 32-image
//            blocks laid out as the matrix cores read them; the plane kernel
//            stages each block's rows of its super-tile in LDS once per
//            workgroup (phi_y scaled by phi_z of the plane on the way), two
//            blocks ahead of the contraction.  bf16 grids contract bf16
//            operands on v_mfma_f32_32x32x16_bf16; fp32 grids split the
//            operands into fp16 hi/lo pairs and take three
//            v_mfma_f32_32x32x16_f16 per step (FP32 accuracy); FP32
//            accumulation in both;
//   window:  the same sum in FP32 on the vector ALUs -- per 32-image step the
//            images' dense factor rows go to LDS with a bit mask of the
//            images meeting each 32 x 32 tile, and each lane accumulates a
//            4 x 4 block of voxels over its tile's images.
// Both forms sum each voxel's atoms in an order fixed by the input alone
// (z-window start, then list order), so results are bitwise reproducible.
#include "pg_device.hpp"
#include "pg_launch.hpp"

namespace pg {

constexpr int PREP_BLOCK = 256; // atoms per prep / place block
constexpr int KC = 32;          // atoms per contraction step
constexpr int ST = 128;         // MFMA super-tile edge (y and x)
constexpr int OPROW = 40;       // staged operand row: 32 images + 8 bf16 of padding

__global__ void cr_clear_kernel(uint32_t *a, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        a[i] = 0u;
}

// Two arrays in one launch: [0, na) of a, then [0, nb) of b.
__global__ void cr_clear2_kernel(uint32_t *a, long long na, uint32_t *b, long long nb)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb;
         i += (long long)gridDim.x * blockDim.x) {
        if (i < na)
            a[i] = 0u;
        else
            b[i - na] = 0u;
    }
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
    const long long a1 = min(p.n_atoms, a0 + PREP_BLOCK) - 1;
    const int m_first = structure_of(p.offsets, p.n_mol, a0);
    const int m_last = structure_of(p.offsets, p.n_mol, a1);
    const bool local = m_last - m_first < PREP_SPAN;
    const int ax = tid / PREP_BLOCK, al = tid - ax * PREP_BLOCK;
    const long long a = a0 + al;
    const bool live = a < live_atoms(p);
    if (live) {
        int n;
        const int m = write_atom_axis(p, a, ax, srec + al, n);
        sn[ax][al] = n;
        if (ax == 0)
            sm[al] = m;
    }
    __syncthreads();
    {
        const long long n_live = live_atoms(p) - a0;
        const int nrec = (int)(n_live < PREP_BLOCK ? (n_live > 0 ? n_live : 0) : PREP_BLOCK);
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
__device__ __forceinline__ long long xcd_block()
{
    const unsigned G = gridDim.x, full = G & ~7u, b = blockIdx.x;
    return b < full ? (long long)(b & 7u) * (full >> 3) + (b >> 3) : (long long)b;
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
    const long long b0 = run_block(q, mc), nb = (n_img + 31) / 32;
    for (long long i = tid; i < nb; i += nt)
        q.bmap[b0 + i] = (uint32_t)mc + 1u;
}

__device__ __forceinline__ uint16_t bf16_bits(float v)
{
    return __builtin_bit_cast(uint16_t, (__bf16)v);
}

// Operand element storage: bf16 bits (the bf16 contraction; the image's
// weight folded into phi_y) or float (the split-fp16 contraction; the weight
// is applied with phi_z in the plane kernel).
__device__ __forceinline__ void op_store(uint16_t *p, float v) { *p = bf16_bits(v); }
__device__ __forceinline__ void op_store(float *p, float v) { *p = v; }

// One workgroup per operand block: phi_x and phi_y of its 32 images over
// the whole x and y axes, laid out [block][row][32 images] so that a
// 16-byte load is one MFMA operand fragment (bf16) or one staging piece
// (float).  The block is first cleared with 16-byte stores; then 8 threads
// per image write the image's window elements only (zeros elsewhere;
// images past the run's end stay zero).
template <typename OT>
__global__ void __launch_bounds__(256) cr_operand_kernel(GridParams p, CrystalParams q)
{
    const long long gb = blockIdx.x;
    const uint32_t tag = q.bmap[gb];
    if (tag == 0u)
        return;
    const size_t mc = tag - 1u;
    const int c = (int)(mc / (size_t)p.n_mol);
    const long long b0 = run_block(q, mc);
    const int tid = threadIdx.x, kl = tid & 31, rg = tid >> 5;
    const long long k = (gb - b0) * 32 + kl;
    const int W = p.W, H = p.H;
    constexpr int CH = 32 * (int)sizeof(OT) / 16;   // 16-byte pieces per row
    OT *xop = (OT *)q.xop, *yop = (OT *)q.yop;
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    u4 *xz = (u4 *)(xop + (size_t)gb * W * 32);
    u4 *yz = (u4 *)(yop + (size_t)gb * H * 32);
    for (int i = tid; i < W * CH; i += 256)
        xz[i] = u4{0u, 0u, 0u, 0u};
    for (int i = tid; i < H * CH; i += 256)
        yz[i] = u4{0u, 0u, 0u, 0u};
    __threadfence_block();
    __syncthreads();
    if (k >= (long long)q.ecount[mc])
        return;
    const int atom = q.zlist[32 * b0 + k].atom;
    const AtomWindow &w = q.table[atom];
    const int ti = image_type(p, q, atom, c);
    const float inv2s2 = p.inv2s2[ti], isq2s = p.isq2s[ti];
    const float wgt = sizeof(OT) == 2 ? image_weight(p, atom, c) : 1.f;
    const bool box = p.box != 0;
    OT *xo = xop + (size_t)gb * W * 32 + kl;
    OT *yo = yop + (size_t)gb * H * 32 + kl;
    for (int r = 0; r < w.n[0]; ++r) {
        const float bh = w.bh[0][r], bl = w.bl[0][r];
        for (int v = w.lo[0][r] + rg; v <= w.hi[0][r]; v += 8)
            op_store(xo + (size_t)v * 32, factor1d(box, bh, bl, p.h[0], v, inv2s2, isq2s));
    }
    for (int r = 0; r < w.n[1]; ++r) {
        const float bh = w.bh[1][r], bl = w.bl[1][r];
        for (int v = w.lo[1][r] + rg; v <= w.hi[1][r]; v += 8)
            op_store(yo + (size_t)v * 32, factor1d(box, bh, bl, p.h[1], v, inv2s2, isq2s) * wgt);
    }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// One workgroup (4 waves) per (structure, channel, z, super-tile); wave w
// owns the 64 x 64 quadrant (w / 2, w % 2) of the 128 x 128 super-tile as
// 2 x 2 MFMA tiles of 32 x 32.  The plane's images are the contiguous range
// [first, end) of its run's z order, taken in whole 32-image operand blocks
// (images of a block outside the plane get phi_z = 0).
// The plane of this workgroup: its coordinates, its run's operand blocks
// [kb0, kb0 + nkb) and phi_z of its images in gzs (with weighted channels
// times the image's weight when fold_weight), ending with a barrier.
struct PlaneItem {
    int sx, sy, z, c, m, kb0, nkb;
    long long rb;
};

__device__ __forceinline__ PlaneItem mfma_plane_begin(const GridParams &p, const CrystalParams &q,
                                                      float *gzs, bool fold_weight)
{
    const int C = p.C, D = p.D, H = p.H, W = p.W;
    const int nsx = (W + ST - 1) / ST, nsy = (H + ST - 1) / ST;
    PlaneItem P;
    long long b = xcd_block();
    P.sx = (int)(b % nsx);
    b /= nsx;
    P.sy = (int)(b % nsy);
    b /= nsy;
    P.z = (int)(b % D);
    b /= D;
    P.c = (int)(b % C);
    P.m = (int)(b / C);
    const int tid = threadIdx.x;
    const size_t mc = (size_t)P.c * p.n_mol + P.m;
    const uint32_t first = q.prange[((size_t)mc * D + P.z) * 2];
    const uint32_t end = q.prange[((size_t)mc * D + P.z) * 2 + 1];
    const uint32_t n_img = q.ecount[mc];
    P.kb0 = (int)(first / 32);
    P.nkb = first < end ? (int)((end + 31) / 32) - P.kb0 : 0;
    if (P.nkb * 32 > min(q.bin_cap, MFMA_BIN_CAP)) {
        if (tid == 0 && P.sx == 0 && P.sy == 0)
            raise_error(p.err, PG_E_CAPACITY, P.m);
        P.nkb = 0;
    }
    P.rb = run_block(q, mc);
    const float hz = p.h[2];
    for (int i = tid; i < P.nkb * 32; i += blockDim.x) {
        const uint32_t k = (uint32_t)P.kb0 * 32 + i;
        float g = 0.f;
        if (k < n_img) {
            const ZEntry ze = q.zlist[32 * P.rb + k];
            if (P.z >= range_lo(ze.range) && P.z <= range_hi(ze.range)) {
                const int ti = image_type(p, q, ze.atom, P.c);
                g = factor1d(p.box != 0, ze.bh, ze.bl, hz, P.z, p.inv2s2[ti], p.isq2s[ti]);
                if (fold_weight)
                    g *= image_weight(p, ze.atom, P.c);
            }
        }
        gzs[i] = g;
    }
    __syncthreads();
    return P;
}

// Store a wave's 64 x 64 quadrant -- 2 x 2 MFMA tiles of 32 x 32, element
// (i, j, e) given by val -- at rows yq.., columns xq.. of an H x W plane.
// Lane l holds column l % 32 of rows 8 (e / 4) + 4 (l / 32) + e % 4 of each
// tile, so one store instruction writes 32 contiguous elements per
// half-wave.  A quadrant that lies inside the plane takes no bounds tests.
template <typename T, typename F>
__device__ __forceinline__ void store_quadrant(T *out, int H, int W, int yq, int xq, bool nt, F val)
{
    const int lane = threadIdx.x & 63;
    if (yq + 64 <= H && xq + 64 <= W) {
        T *o = out + (size_t)(yq + 4 * (lane >> 5)) * W + xq + (lane & 31);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const float v[1] = {val(i, j, e)};
                    store_vec<T, 1>(o + (size_t)(32 * i + 8 * (e >> 2) + (e & 3)) * W + 32 * j, v, nt);
                }
        return;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int y = yq + 32 * i + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                const int x = xq + 32 * j + (lane & 31);
                if (y < H && x < W) {
                    const float v[1] = {val(i, j, e)};
                    store_vec<T, 1>(out + (size_t)y * W + x, v, nt);
                }
            }
}

__global__ void __launch_bounds__(256) cr_mfma_kernel(GridParams p, CrystalParams q)
{
    using T = __bf16;
    __shared__ __attribute__((aligned(16))) float gzs[MFMA_BIN_CAP];   // phi_z per image
    // two staging buffers of [phi_z phi_y, phi_x][super-tile row][32 images],
    // rows padded to OPROW elements so that the fragment reads (lanes on
    // consecutive rows) fall in distinct banks
    __shared__ __attribute__((aligned(16))) __bf16 ops[2][2][ST * OPROW];
    const int C = p.C, D = p.D, H = p.H, W = p.W;
    const PlaneItem PI = mfma_plane_begin(p, q, gzs, false);
    const int z = PI.z, c = PI.c, m = PI.m, kb0 = PI.kb0, nkb = PI.nkb;
    const long long rb = PI.rb;
    const int y0 = PI.sy * ST, x0 = PI.sx * ST;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e)
                acc[i][j][e] = 0.f;
    const int qy = (wave >> 1) * 64, qx = (wave & 1) * 64;
    const int ko = 8 * (lane >> 5);
    const __bf16 *yop = (const __bf16 *)q.yop, *xop = (const __bf16 *)q.xop;
    // Staging: the workgroup copies each 32-image operand block's rows of
    // the super-tile to LDS once -- phi_y scaled by phi_z of the plane
    // (rounded once to bf16), and phi_x -- so every operand element is
    // fetched and scaled once per workgroup instead of once per wave that
    // uses it.  Thread t moves the 16-byte chunk (t % 4) of local rows t / 4
    // and t / 4 + 64 of both operands; rows past the plane edge copy the last
    // row instead (they only feed outputs that are never stored).
    const int srow = tid >> 2, skq = 8 * (tid & 3);
    int sy_[2], sx_[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        sy_[r] = min(y0 + srow + 64 * r, H - 1);
        sx_[r] = min(x0 + srow + 64 * r, W - 1);
    }
    // two register sets: block kb + 2 is fetched while block kb is
    // contracted and block kb + 1 (fetched one step earlier) is staged
    bf16x8 ga[2][2], gb[2][2];
    auto fetch = [&](int kb, bf16x8 (&fa)[2], bf16x8 (&fb)[2]) {
        const size_t blk = (size_t)(rb + kb0 + kb);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            fa[r] = *(const bf16x8 *)(yop + (blk * H + sy_[r]) * 32 + skq);
            fb[r] = *(const bf16x8 *)(xop + (blk * W + sx_[r]) * 32 + skq);
        }
    };
    auto stage = [&](int kb, int buf, const bf16x8 (&fa)[2], const bf16x8 (&fb)[2]) {
        const float4 g0 = *(const float4 *)(gzs + kb * 32 + skq);
        const float4 g1 = *(const float4 *)(gzs + kb * 32 + skq + 4);
        const float g[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            bf16x8 av;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                av[e] = (__bf16)((float)fa[r][e] * g[e]);
            *(bf16x8 *)(ops[buf][0] + (srow + 64 * r) * OPROW + skq) = av;
            *(bf16x8 *)(ops[buf][1] + (srow + 64 * r) * OPROW + skq) = fb[r];
        }
    };
    auto contract = [&](int buf) {
        const __bf16 *As = ops[buf][0], *Bs = ops[buf][1];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int kk = 16 * h + ko;
            bf16x8 af[2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                af[i] = *(const bf16x8 *)(As + (qy + 32 * i + (lane & 31)) * OPROW + kk);
                bf[i] = *(const bf16x8 *)(Bs + (qx + 32 * i + (lane & 31)) * OPROW + kk);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
    };
    // one step: fetch kb + 2 (clamped: past the end it refetches the last
    // block), contract kb, stage kb + 1 into the other buffer (last read
    // before the previous barrier), barrier
    auto step = [&](int kb, bf16x8 (&fa_next)[2], bf16x8 (&fb_next)[2],
                    const bf16x8 (&fa_stage)[2], const bf16x8 (&fb_stage)[2]) {
        fetch(min(kb + 2, nkb - 1), fa_next, fb_next);
        contract(kb & 1);
        if (kb + 1 < nkb)
            stage(kb + 1, (kb + 1) & 1, fa_stage, fb_stage);
        __syncthreads();
    };
    if (nkb > 0) {
        fetch(0, ga[0], gb[0]);
        fetch(min(1, nkb - 1), ga[1], gb[1]);
        stage(0, 0, ga[0], gb[0]);
    }
    __syncthreads();
    int kb = 0;
    for (; kb + 1 < nkb; kb += 2) {
        step(kb, ga[0], gb[0], ga[1], gb[1]);
        step(kb + 1, ga[1], gb[1], ga[0], gb[0]);
    }
    if (kb < nkb)
        step(kb, ga[0], gb[0], ga[1], gb[1]);

    T *out = (T *)p.out + (((size_t)m * C + c) * D + z) * (size_t)H * W;
    store_quadrant(out, H, W, y0 + qy, x0 + qx, p.nt_store != 0,
                   [&](int i, int j, int e) { return acc[i][j][e]; });
}

// ---------------------------------------------------------------------------
// Split-fp16 MFMA form (fp32 grids at FP32 accuracy)
// ---------------------------------------------------------------------------
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
constexpr int SPROW = 24;             // staged row: 16 images + 8 halves of padding
constexpr float SPLIT_UP = 4096.f;    // scale of the low parts (2^12)

// v = hi + lo / 2^12 to about 2^-22 |v|: hi = fp16(v), lo = fp16((v - hi) 2^12)
// (v - hi is exact in FP32; the scaled low part stays in the fp16 normal
// range for every v the plane kernel splits).
__device__ __forceinline__ void split16(float v, _Float16 &hi, _Float16 &lo)
{
    hi = (_Float16)v;
    lo = (_Float16)((v - (float)hi) * SPLIT_UP);
}

// One workgroup (4 waves) per (structure, channel, z, super-tile), as the
// bf16 form, on FP32 operands (phi_x, and phi_y without the weight).  Per
// 16-image step the workgroup stages A = s phi_z w phi_y and B = phi_x in
// LDS, each split as hi + lo / 2^12 into fp16 pairs; s = 2^e is chosen per
// plane from the largest |phi_z w| so that every A stays within the fp16
// range.  Each 32 x 32 tile takes three v_mfma_f32_32x32x16_f16 per step:
// P += Ahi Bhi, Q += Ahi Blo + Alo Bhi; the plane is (P + Q / 2^12) / s.  The
// dropped Alo Blo and the splits leave about 2^-21 relative error per
// product, against 2^-8 for the bf16 operands.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) cr_mfma_split_kernel(GridParams p, CrystalParams q)
{
    __shared__ __attribute__((aligned(16))) float gzs[MFMA_BIN_CAP];   // phi_z w per image
    __shared__ float wmax[4];
    // two staging buffers of [Ahi, Alo, Bhi, Blo][super-tile row][16 images]
    __shared__ __attribute__((aligned(16))) _Float16 sops[2][4][ST * SPROW];
    const int H = p.H, W = p.W, C = p.C, D = p.D;
    const PlaneItem PI = mfma_plane_begin(p, q, gzs, true);
    const int z = PI.z, c = PI.c, m = PI.m, kb0 = PI.kb0;
    const long long rb = PI.rb;
    const int nst = 2 * PI.nkb;   // 16-image steps
    const int y0 = PI.sy * ST, x0 = PI.sx * ST;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // plane scale: s = 2^(14 - e) for the largest |phi_z w| = f 2^e, f in [0.5, 1)
    float mx = 0.f;
    for (int i = tid; i < nst * 16; i += blockDim.x)
        mx = fmaxf(mx, fabsf(gzs[i]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        mx = fmaxf(mx, __shfl_xor(mx, off));
    if (lane == 0)
        wmax[wave] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    int ex = 0;
    if (mx > 0.f)
        (void)frexpf(mx, &ex);
    ex = max(ex, -110);   // s and 1 / s stay normal floats for the tiniest weights
    const float sc = ldexpf(1.f, 14 - ex), unsc = ldexpf(1.f, ex - 14);

    f32x16 accp[2][2], accq[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                accp[i][j][e] = 0.f;
                accq[i][j][e] = 0.f;
            }
    const int qy = (wave >> 1) * 64, qx = (wave & 1) * 64;
    const int ko = 8 * (lane >> 5);
    const float *yop = (const float *)q.yop, *xop = (const float *)q.xop;
    // staging: thread t moves images 4 (t % 4) .. + 3 of the step for local
    // rows t / 4 and t / 4 + 64 of both operands; rows past the plane edge
    // copy the last row (they only feed outputs that are never stored)
    const int srow = tid >> 2, skq = 4 * (tid & 3);
    int sy_[2], sx_[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        sy_[r] = min(y0 + srow + 64 * r, H - 1);
        sx_[r] = min(x0 + srow + 64 * r, W - 1);
    }
    float4 ga[2][2], gb[2][2];
    auto fetch = [&](int st, float4 (&fa)[2], float4 (&fb)[2]) {
        const size_t blk = (size_t)(rb + kb0 + (st >> 1));
        const int off = 16 * (st & 1) + skq;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            fa[r] = *(const float4 *)(yop + (blk * H + sy_[r]) * 32 + off);
            fb[r] = *(const float4 *)(xop + (blk * W + sx_[r]) * 32 + off);
        }
    };
    auto stage = [&](int st, int buf, const float4 (&fa)[2], const float4 (&fb)[2]) {
        const float4 g4 = *(const float4 *)(gzs + st * 16 + skq);
        const float g[4] = {g4.x * sc, g4.y * sc, g4.z * sc, g4.w * sc};
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const float av[4] = {fa[r].x * g[0], fa[r].y * g[1], fa[r].z * g[2], fa[r].w * g[3]};
            const float bv[4] = {fb[r].x, fb[r].y, fb[r].z, fb[r].w};
            f16x4 ah, al, bh, bl;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                _Float16 h, l;
                split16(av[e], h, l);
                ah[e] = h;
                al[e] = l;
                split16(bv[e], h, l);
                bh[e] = h;
                bl[e] = l;
            }
            const int o = (srow + 64 * r) * SPROW + skq;
            *(f16x4 *)(sops[buf][0] + o) = ah;
            *(f16x4 *)(sops[buf][1] + o) = al;
            *(f16x4 *)(sops[buf][2] + o) = bh;
            *(f16x4 *)(sops[buf][3] + o) = bl;
        }
    };
    auto contract = [&](int buf) {
        f16x8 ahf[2], alf[2], bhf[2], blf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int ra = (qy + 32 * i + (lane & 31)) * SPROW + ko;
            const int rbx = (qx + 32 * i + (lane & 31)) * SPROW + ko;
            ahf[i] = *(const f16x8 *)(sops[buf][0] + ra);
            alf[i] = *(const f16x8 *)(sops[buf][1] + ra);
            bhf[i] = *(const f16x8 *)(sops[buf][2] + rbx);
            blf[i] = *(const f16x8 *)(sops[buf][3] + rbx);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                accp[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahf[i], bhf[j], accp[i][j], 0, 0, 0);
                accq[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahf[i], blf[j], accq[i][j], 0, 0, 0);
                accq[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(alf[i], bhf[j], accq[i][j], 0, 0, 0);
            }
    };
    // as the bf16 form: fetch step st + 2 (clamped), contract st, stage
    // st + 1 into the other buffer, barrier
    auto step = [&](int st, float4 (&fa_next)[2], float4 (&fb_next)[2],
                    const float4 (&fa_stage)[2], const float4 (&fb_stage)[2]) {
        fetch(min(st + 2, nst - 1), fa_next, fb_next);
        contract(st & 1);
        if (st + 1 < nst)
            stage(st + 1, (st + 1) & 1, fa_stage, fb_stage);
        __syncthreads();
    };
    if (nst > 0) {
        fetch(0, ga[0], gb[0]);
        fetch(min(1, nst - 1), ga[1], gb[1]);
        stage(0, 0, ga[0], gb[0]);
    }
    __syncthreads();
    int st = 0;
    for (; st + 1 < nst; st += 2) {
        step(st, ga[0], gb[0], ga[1], gb[1]);
        step(st + 1, ga[1], gb[1], ga[0], gb[0]);
    }
    if (st < nst)
        step(st, ga[0], gb[0], ga[1], gb[1]);

    float *out = (float *)p.out + (((size_t)m * C + c) * D + z) * (size_t)H * W;
    store_quadrant(out, H, W, y0 + qy, x0 + qx, p.nt_store != 0, [&](int i, int j, int e) {
        return (accp[i][j][e] + accq[i][j][e] * (1.f / SPLIT_UP)) * unsc;
    });
}

// FP32 vector-ALU form: one workgroup (256 threads) per (structure, channel,
// z); the plane's images are the range [first, end) of the run's z order.
// Per 32-image step the images' dense factor rows go to LDS -- phi_x, and
// phi_z(z) phi_y -- evaluated where the windows are (8 threads per image),
// and, per 32 x 32 output tile, a bit mask of the step's images whose
// window meets the tile.  Wave w owns tiles w, w + 4, ...; lane l owns the
// 4 x 4 voxels at rows 4 (l / 8), columns 4 (l % 8) of each: for every
// image in the tile's mask (lowest bit first) it reads 4 phi_y and 4 phi_x
// values and does 16 FMAs.  Each voxel sums its images in z order, in FP32.
template <typename T, int TMAX>
__global__ void __launch_bounds__(256) cr_window_kernel(GridParams p, CrystalParams q)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int C = p.C, D = p.D, H = p.H, W = p.W;
    const int W32 = (W + 31) & ~31, H32 = (H + 31) & ~31;
    const int ntx = W32 / 32, nty = H32 / 32, ntiles = ntx * nty;
    float *gx = (float *)smem;                    // [KC][W32] phi_x
    float *gy = gx + KC * W32;                    // [KC][H32] phi_z(z) phi_y
    uint32_t *tmask = (uint32_t *)(gy + KC * H32);   // [ntiles] images meeting each tile
    long long b = xcd_block();
    const int z = (int)(b % D);
    b /= D;
    const int c = (int)(b % C);
    const int m = (int)(b / C);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const size_t mc = (size_t)c * p.n_mol + m;
    const uint32_t first = q.prange[((size_t)mc * D + z) * 2];
    const uint32_t end = q.prange[((size_t)mc * D + z) * 2 + 1];
    const long long eb = 32ll * run_block(q, mc);
    const bool box = p.box != 0;
    const int ly = 4 * (lane >> 3), lx = 4 * (lane & 7);
    float acc[TMAX][4][4];
#pragma unroll
    for (int i = 0; i < TMAX; ++i)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                acc[i][rr][e] = 0.f;

    for (uint32_t k0 = first; k0 < end; k0 += KC) {
        const int kn = (int)min((uint32_t)KC, end - k0);
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
        for (int i = tid; i < 8 * (W32 + H32); i += blockDim.x)
            ((u4 *)gx)[i] = u4{0u, 0u, 0u, 0u};
        for (int i = tid; i < ntiles; i += blockDim.x)
            tmask[i] = 0u;
        __syncthreads();
        {
            const int k = tid >> 3, part = tid & 7;
            if (k < kn) {
                const ZEntry ze = q.zlist[eb + k0 + k];
                if (z >= range_lo(ze.range) && z <= range_hi(ze.range)) {
                    const int ti = image_type(p, q, ze.atom, c);
                    const float inv2s2 = p.inv2s2[ti], isq2s = p.isq2s[ti];
                    const float g = factor1d(box, ze.bh, ze.bl, p.h[2], z, inv2s2, isq2s) *
                                    image_weight(p, ze.atom, c);
                    const AtomWindow &w = q.table[ze.atom];
                    uint32_t tx = 0u, ty = 0u;   // tile columns / rows the windows meet
                    for (int r = 0; r < w.n[0]; ++r) {
                        const float bh = w.bh[0][r], bl = w.bl[0][r];
                        for (int t = w.lo[0][r] >> 5; t <= (w.hi[0][r] >> 5); ++t)
                            tx |= 1u << t;
                        for (int v = w.lo[0][r] + part; v <= w.hi[0][r]; v += 8)
                            gx[k * W32 + v] = factor1d(box, bh, bl, p.h[0], v, inv2s2, isq2s);
                    }
                    for (int r = 0; r < w.n[1]; ++r) {
                        const float bh = w.bh[1][r], bl = w.bl[1][r];
                        for (int t = w.lo[1][r] >> 5; t <= (w.hi[1][r] >> 5); ++t)
                            ty |= 1u << t;
                        for (int v = w.lo[1][r] + part; v <= w.hi[1][r]; v += 8)
                            gy[k * H32 + v] = g * factor1d(box, bh, bl, p.h[1], v, inv2s2, isq2s);
                    }
                    if (part == 0)
                        for (int tr = 0; tr < nty; ++tr)
                            if ((ty >> tr) & 1u)
                                for (int tc = 0; tc < ntx; ++tc)
                                    if ((tx >> tc) & 1u)
                                        atomicOr(&tmask[tr * ntx + tc], 1u << k);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < TMAX; ++i) {
            const int t = wave + 4 * i;
            if (t >= ntiles)
                break;
            const int y = 32 * (t / ntx) + ly, x = 32 * (t % ntx) + lx;
            uint32_t mk = tmask[t];
            while (mk) {
                const int k = __builtin_ctz(mk);
                mk &= mk - 1u;
                const float4 g4 = *(const float4 *)(gy + k * H32 + y);
                const float4 f4 = *(const float4 *)(gx + k * W32 + x);
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
    if (form == PG_FORM_MFMA)   // all static: phi_z per image
        return 0;
    const int W32 = (W + 31) & ~31, H32 = (H + 31) & ~31;
    return (size_t)KC * (W32 + H32) * sizeof(float) + (size_t)(W32 / 32) * (H32 / 32) * 4;
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

int crystal_prep_blocks(long long n_atoms)
{
    return (int)((n_atoms + PREP_BLOCK - 1) / PREP_BLOCK);
}

hipError_t launch_crystal(const GridParams &p, const CrystalParams &q, int form, int out_dtype,
                          size_t lds, hipStream_t s)
{
    if (p.n_mol == 0)
        return hipSuccess;
    const long long nmc = (long long)p.n_mol * p.C;
    const unsigned clear_grid = (unsigned)std::min<long long>((nmc + q.op_blocks + 255) / 256, 65535);
    hipLaunchKernelGGL(cr_clear2_kernel, dim3(clear_grid), dim3(256), 0, s, q.mcount, nmc, q.bmap,
                       (long long)q.op_blocks);
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
    if (form == PG_FORM_MFMA) {
        if (out_dtype == PG_OUT_F32)
            hipLaunchKernelGGL(cr_operand_kernel<float>, dim3((unsigned)q.op_blocks), dim3(256), 0, s, p, q);
        else
            hipLaunchKernelGGL(cr_operand_kernel<uint16_t>, dim3((unsigned)q.op_blocks), dim3(256), 0, s,
                               p, q);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    const void *k;
    long long grid;
    if (form == PG_FORM_MFMA) {
        k = out_dtype == PG_OUT_F32 ? (const void *)cr_mfma_split_kernel
                                    : (const void *)cr_mfma_kernel;
        grid = nmc * p.D * ((p.H + ST - 1) / ST) * ((p.W + ST - 1) / ST);
    } else {
        const int r = crystal_window_runs(p.H, p.W);
        if (out_dtype == PG_OUT_F32)
            k = r == 1 ? (const void *)cr_window_kernel<float, 1>
              : r == 2 ? (const void *)cr_window_kernel<float, 2>
              : r == 4 ? (const void *)cr_window_kernel<float, 4>
              : r == 8 ? (const void *)cr_window_kernel<float, 8> : nullptr;
        else
            k = r == 1 ? (const void *)cr_window_kernel<__bf16, 1>
              : r == 2 ? (const void *)cr_window_kernel<__bf16, 2>
              : r == 4 ? (const void *)cr_window_kernel<__bf16, 4>
              : r == 8 ? (const void *)cr_window_kernel<__bf16, 8> : nullptr;
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
