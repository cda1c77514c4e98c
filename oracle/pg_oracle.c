/*
 * pg_oracle.c -- plain FP64 CPU reference of the atoms -> density-grid map.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; the product path never
 * calls it.
 *
 * What it computes (the plain definition, written out):
 *
 *   Each atom a with position mu_a and element type t_a owns the channel
 *   c = t_a (one channel per element, §III-A).  The grid holds, at every
 *   voxel centre r = origin + (i + 1/2) * h (per axis), the sum over atoms
 *   of that channel of the un-normalised 3-D Gaussian of Eq. 1,
 *
 *       exp( -|r - mu_a|^2 / (2 sigma_t^2) ),
 *
 *   where |r - mu|^2 is the squared Euclidean distance, or for a periodic
 *   cell the nearest-image distance (§III-A, text after Eq. 1: minimum
 *   over lattice translations; here an orthorhombic cell, per axis).
 *
 *   Truncation (§VI-B: the paper suggests a threshold instead of relying on
 *   FP underflow): an atom contributes only to voxels inside its cutoff
 *   cube, |r_alpha - mu_alpha| <= rc_t on every axis, with
 *   rc_t = fl32(k * sigma_t) (the single-precision product of the two
 *   float inputs) and an inclusive comparison.  k == 0 means no cutoff.
 *   The decision is made in exact arithmetic on the inputs: a double
 *   evaluation decides when it is far from the edge; near the edge the
 *   offset is recomputed in binary128 with every addition checked to be
 *   exact (abort otherwise), so no voxel is ever misclassified.
 *
 *   The value itself is the 3-D exponential of the summed squared offsets
 *   in double -- NOT the separable product of 1-D factors (separability,
 *   §III-A and §IV-C, is checked by the tests, not assumed here).
 *
 *   Box form (value = 1): the voxel holds the integral of the normalised
 *   Gaussian over the voxel box (§III-A Eq. 2-5), i.e. the product over
 *   axes of (1/2)[erf((x_i + h - mu) / (sqrt(2) sigma)) - erf((x_i - mu) /
 *   (sqrt(2) sigma))] with x_i the lower voxel edge (the sign read so that
 *   the value is positive), inside the same cutoff windows (decided on the
 *   voxel centres).  Tails are evaluated through erfc to avoid cancellation.
 *   Its coordinate gradient uses d/dmu of each axis factor,
 *   (g(x_i - mu) - g(x_i + h - mu)) / (sqrt(2 pi) sigma), g = exp(-d^2 / (2 sigma^2)).
 *
 *   Adjoint: for L = sum_v U[v] G[v], dL/dmu_{a,alpha} =
 *   sum_{v inside} U[t_a, v] * g_a(v) * (r_alpha - mu_alpha) / sigma_t^2,
 *   the derivative of the point-sampled Gaussian (the point-sample analogue
 *   of the separable coordinate gradient of §IV-C), cutoff-edge jumps
 *   excluded (derivative almost everywhere).
 *
 *   Sphere cutoff (sphere = 1, with a cutoff): a voxel inside an atom's
 *   cube is kept only if also |r - mu|^2 <= rc_t^2, the squared offsets
 *   (nearest image per axis when periodic) summed in double.  This decision
 *   is not made exactly: voxels within a relative 1e-6 of the sphere are
 *   left to the tests to treat as either side.
 *
 *   Weighted channels (weights != NULL; the learned-embedding grids the
 *   Discussion proposes, and the weighted grids mentioned after Eq. 6): atom
 *   a adds weights[a][c] times its Gaussian to every channel c, the
 *   Gaussian's width still being sigma of its type t_a, which then indexes
 *   a table of n_sig widths independent of the channel count.  One-hot
 *   weights (weights[a][c] = [c == t_a]) give the unweighted grid.  The
 *   adjoint then also yields dL/dweights[a][c] = sum_v U[c, v] g_a(v).
 *
 *   Atoms with a type outside [0, C) (weighted: [0, n_sig)) or a non-finite
 *   coordinate are skipped and counted.
 *
 * Layout: out[b][c][z][y][x], x fastest; dims (D, H, W) = (z, y, x);
 * origin / spacing / cell given in x, y, z order.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 quad;

/* ---- exact offset evaluation near a cutoff edge ------------------------- */

/* a + b in binary128, aborting unless the sum is exact (Knuth's TwoSum error
   term must vanish).  Inputs here are float32 / float64 values and exact
   products of them, so the sums fit 113 bits for any sane coordinates. */
static quad qadd_exact(quad a, quad b)
{
    quad s = a + b;
    quad bb = s - a;
    quad err = (a - (s - bb)) + (b - bb);
    if (err != 0) {
        fprintf(stderr, "pg_oracle: inexact binary128 sum (input span too wide)\n");
        abort();
    }
    return s;
}

/* Exact r_i - mu - n*L with r_i = o + (i + 1/2) h. */
static quad offset_exact(double o, double h, int i, double mu, double n, double L)
{
    quad p = (quad)((double)i + 0.5) * (quad)h;   /* exact: 53 x 53 bits */
    quad q = (quad)n * (quad)L;                   /* exact */
    quad s = qadd_exact((quad)o, p);
    s = qadd_exact(s, -(quad)mu);
    s = qadd_exact(s, -q);
    return s;
}

/*
 * Offset of axis index i from the atom (nearest image if periodic) and
 * whether it lies inside the cutoff.  Returns 1 if inside.
 */
static int axis_offset(double o, double h, int i, double mu,
                       int periodic, double L, int cut, double rc, double *delta)
{
    double d = o + ((double)i + 0.5) * h - mu;
    double n = 0.0;
    if (periodic) {
        n = nearbyint(d / L);
        d -= n * L;
    }
    *delta = d;
    if (!cut)
        return 1;
    double margin = fabs(fabs(d) - rc);
    if (margin > 1e-9 * (1.0 + fabs(o) + fabs(mu) + fabs(n * L) + fabs(((double)i + 0.5) * h)))
        return fabs(d) <= rc;
    /* near the edge: decide exactly */
    quad e = offset_exact(o, h, i, mu, n, L);
    if (e < 0)
        e = -e;
    return e <= (quad)rc;
}

static int atom_ok(const double *mu, int32_t t, int C)
{
    if (t < 0 || t >= C)
        return 0;
    return isfinite(mu[0]) && isfinite(mu[1]) && isfinite(mu[2]);
}

static double cutoff_radius(float k, float sigma)
{
    volatile float r = k * sigma;   /* single-precision product, RNE */
    return (double)r;
}

/* (1/2)[erf(r / (sqrt 2 sigma)) - erf(l / (sqrt 2 sigma))] for l < r: the mass
   of the normalised 1-D Gaussian between offsets l and r. */
static double box1d(double l, double r, double sigma)
{
    const double s = 1.0 / (sqrt(2.0) * sigma);
    const double a = l * s, b = r * s;
    if (a >= 0.0)
        return 0.5 * (erfc(a) - erfc(b));
    if (b <= 0.0)
        return 0.5 * (erfc(-b) - erfc(-a));
    return 0.5 * (erf(b) - erf(a));
}

/* d/dmu of box1d(x_lo - mu, x_hi - mu). */
static double dbox1d(double l, double r, double sigma)
{
    const double s2 = sigma * sigma;
    return (exp(-l * l / (2.0 * s2)) - exp(-r * r / (2.0 * s2))) / (sqrt(2.0 * M_PI) * sigma);
}

typedef struct {
    int D, H, W, C;
    double o[3], h[3];
    int periodic;
    double L[3];
    int cut;
    double rc;
} geom_t;

static void geom_for(geom_t *g, int b, int C, int D, int H, int W,
                     const double *origin3, const double *spacing3,
                     const double *origins, const double *spacings,
                     int periodic, const double *cell3)
{
    g->C = C; g->D = D; g->H = H; g->W = W;
    for (int a = 0; a < 3; ++a) {
        g->o[a] = origins ? origins[3 * (size_t)b + a] : origin3[a];
        g->h[a] = spacings ? spacings[3 * (size_t)b + a] : spacing3[a];
        g->L[a] = periodic ? cell3[a] : 0.0;
    }
    g->periodic = periodic;
}

/* Per-axis window of one atom: lists of inside indices and their offsets. */
typedef struct {
    int n[3];
    int *idx[3];
    double *del[3];
} window_t;

static void window_build(window_t *w, const geom_t *g, const double *mu)
{
    const int N[3] = {g->W, g->H, g->D};
    for (int a = 0; a < 3; ++a) {
        w->n[a] = 0;
        for (int i = 0; i < N[a]; ++i) {
            double d;
            if (axis_offset(g->o[a], g->h[a], i, mu[a], g->periodic, g->L[a],
                            g->cut, g->rc, &d)) {
                w->idx[a][w->n[a]] = i;
                w->del[a][w->n[a]] = d;
                w->n[a]++;
            }
        }
    }
}

static int window_alloc(window_t *w, int D, int H, int W)
{
    const int N[3] = {W, H, D};
    for (int a = 0; a < 3; ++a) {
        w->idx[a] = (int *)malloc(sizeof(int) * (size_t)(N[a] > 0 ? N[a] : 1));
        w->del[a] = (double *)malloc(sizeof(double) * (size_t)(N[a] > 0 ? N[a] : 1));
        if (!w->idx[a] || !w->del[a])
            return -1;
    }
    return 0;
}

static void window_free(window_t *w)
{
    for (int a = 0; a < 3; ++a) {
        free(w->idx[a]);
        free(w->del[a]);
    }
}

/*
 * Dense grids for a batch.  out has B*C*D*H*W doubles and is overwritten.
 * evals (may be NULL) receives the number of atom-voxel pairs evaluated;
 * skipped (may be NULL) the number of atoms skipped as invalid.
 * Returns 0, or -1 on allocation failure.
 */
int pgo_grid(int B, const int64_t *offsets, const double *xyz, const int32_t *types,
             int C, int D, int H, int W,
             const double *origin3, const double *spacing3,
             const double *origins, const double *spacings,
             const float *sigma, float cutoff_k,
             int periodic, const double *cell3, int value, int sphere,
             const double *weights, int n_sig,
             double *out, int64_t *evals, int64_t *skipped)
{
    const size_t plane = (size_t)H * W, vol = (size_t)D * plane;
    memset(out, 0, sizeof(double) * (size_t)B * C * vol);
    int64_t ev = 0, sk = 0;
    window_t w;
    if (window_alloc(&w, D, H, W))
        return -1;
    for (int b = 0; b < B; ++b) {
        geom_t g;
        geom_for(&g, b, C, D, H, W, origin3, spacing3, origins, spacings, periodic, cell3);
        for (int64_t a = offsets[b]; a < offsets[b + 1]; ++a) {
            const double *mu = xyz + 3 * a;
            int32_t t = types[a];
            if (!atom_ok(mu, t, weights ? n_sig : C)) {
                ++sk;
                continue;
            }
            g.cut = cutoff_k != 0.0f;
            g.rc = cutoff_radius(cutoff_k, sigma[t]);
            window_build(&w, &g, mu);
            const double s2 = (double)sigma[t] * (double)sigma[t];
            double *grid = out + ((size_t)b * C + t) * vol;
            const double *wa = weights ? weights + (size_t)a * C : NULL;
            for (int kz = 0; kz < w.n[2]; ++kz)
                for (int ky = 0; ky < w.n[1]; ++ky)
                    for (int kx = 0; kx < w.n[0]; ++kx) {
                        double dx = w.del[0][kx], dy = w.del[1][ky], dz = w.del[2][kz];
                        if (sphere && g.cut && dx * dx + dy * dy + dz * dz > g.rc * g.rc)
                            continue;
                        double v;
                        if (value == 1)
                            v = box1d(dx - 0.5 * g.h[0], dx + 0.5 * g.h[0], sigma[t]) *
                                box1d(dy - 0.5 * g.h[1], dy + 0.5 * g.h[1], sigma[t]) *
                                box1d(dz - 0.5 * g.h[2], dz + 0.5 * g.h[2], sigma[t]);
                        else
                            v = exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * s2));
                        const size_t vox = (size_t)w.idx[2][kz] * plane +
                                           (size_t)w.idx[1][ky] * W + w.idx[0][kx];
                        if (!wa) {
                            grid[vox] += v;
                        } else {
                            for (int c = 0; c < C; ++c)
                                if (wa[c] != 0.0)
                                    out[((size_t)b * C + c) * vol + vox] += wa[c] * v;
                        }
                    }
            ev += (int64_t)w.n[0] * w.n[1] * w.n[2];
        }
    }
    window_free(&w);
    if (evals)
        *evals = ev;
    if (skipped)
        *skipped = sk;
    return 0;
}

/*
 * Coordinate gradient of L = sum U * G.  U has B*C*D*H*W doubles; grad has
 * n_atoms*3 doubles (x, y, z) and is overwritten (skipped atoms get 0).
 * Weighted channels: grad_w (may be NULL) receives dL/dweights, n_atoms*C.
 */
int pgo_grad(int B, const int64_t *offsets, const double *xyz, const int32_t *types,
             int C, int D, int H, int W,
             const double *origin3, const double *spacing3,
             const double *origins, const double *spacings,
             const float *sigma, float cutoff_k,
             int periodic, const double *cell3, int value, int sphere,
             const double *weights, int n_sig,
             const double *U, double *grad, double *grad_w)
{
    const size_t plane = (size_t)H * W, vol = (size_t)D * plane;
    window_t w;
    if (window_alloc(&w, D, H, W))
        return -1;
    for (int b = 0; b < B; ++b) {
        geom_t g;
        geom_for(&g, b, C, D, H, W, origin3, spacing3, origins, spacings, periodic, cell3);
        for (int64_t a = offsets[b]; a < offsets[b + 1]; ++a) {
            const double *mu = xyz + 3 * a;
            int32_t t = types[a];
            grad[3 * a + 0] = grad[3 * a + 1] = grad[3 * a + 2] = 0.0;
            const double *wa = weights ? weights + (size_t)a * C : NULL;
            double *gwa = (weights && grad_w) ? grad_w + (size_t)a * C : NULL;
            if (gwa)
                for (int c = 0; c < C; ++c)
                    gwa[c] = 0.0;
            if (!atom_ok(mu, t, weights ? n_sig : C))
                continue;
            g.cut = cutoff_k != 0.0f;
            g.rc = cutoff_radius(cutoff_k, sigma[t]);
            window_build(&w, &g, mu);
            const double s2 = (double)sigma[t] * (double)sigma[t];
            const double *u = U + ((size_t)b * C + t) * vol;
            const double *ub = U + (size_t)b * C * vol;
            double gx = 0, gy = 0, gz = 0;
            for (int kz = 0; kz < w.n[2]; ++kz)
                for (int ky = 0; ky < w.n[1]; ++ky)
                    for (int kx = 0; kx < w.n[0]; ++kx) {
                        double dx = w.del[0][kx], dy = w.del[1][ky], dz = w.del[2][kz];
                        if (sphere && g.cut && dx * dx + dy * dy + dz * dz > g.rc * g.rc)
                            continue;
                        const size_t vox = (size_t)w.idx[2][kz] * plane +
                                           (size_t)w.idx[1][ky] * W + w.idx[0][kx];
                        double uv;
                        if (!wa) {
                            uv = u[vox];
                        } else {
                            /* sum_c w_c U[c, v]: the upstream seen by this atom */
                            uv = 0.0;
                            for (int c = 0; c < C; ++c)
                                uv += wa[c] * ub[(size_t)c * vol + vox];
                        }
                        if (gwa) {
                            double gval;
                            if (value == 1)
                                gval = box1d(dx - 0.5 * g.h[0], dx + 0.5 * g.h[0], sigma[t]) *
                                       box1d(dy - 0.5 * g.h[1], dy + 0.5 * g.h[1], sigma[t]) *
                                       box1d(dz - 0.5 * g.h[2], dz + 0.5 * g.h[2], sigma[t]);
                            else
                                gval = exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * s2));
                            for (int c = 0; c < C; ++c)
                                gwa[c] += ub[(size_t)c * vol + vox] * gval;
                        }
                        if (value == 1) {
                            const double sg = sigma[t];
                            const double lx = dx - 0.5 * g.h[0], rx = dx + 0.5 * g.h[0];
                            const double ly = dy - 0.5 * g.h[1], ry = dy + 0.5 * g.h[1];
                            const double lz = dz - 0.5 * g.h[2], rz = dz + 0.5 * g.h[2];
                            const double bx = box1d(lx, rx, sg), by = box1d(ly, ry, sg),
                                         bz = box1d(lz, rz, sg);
                            gx += uv * dbox1d(lx, rx, sg) * by * bz;
                            gy += uv * bx * dbox1d(ly, ry, sg) * bz;
                            gz += uv * bx * by * dbox1d(lz, rz, sg);
                        } else {
                            double gval = exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * s2));
                            double f = uv * gval / s2;
                            gx += f * dx;
                            gy += f * dy;
                            gz += f * dz;
                        }
                    }
            grad[3 * a + 0] = gx;
            grad[3 * a + 1] = gy;
            grad[3 * a + 2] = gz;
        }
    }
    window_free(&w);
    return 0;
}

/*
 * Individual voxels, one at a time: sample s is (b, c, z, y, x) =
 * idx[5s .. 5s+4]; val[s] receives the grid value there.  Every atom of the
 * structure is visited (no window bookkeeping at all), so this is the most
 * literal form of the definition; it serves the sampled checks at sizes
 * where a dense FP64 grid would not fit.
 */
int pgo_voxels(int B, const int64_t *offsets, const double *xyz, const int32_t *types,
               int C, int D, int H, int W,
               const double *origin3, const double *spacing3,
               const double *origins, const double *spacings,
               const float *sigma, float cutoff_k,
               int periodic, const double *cell3, int value, int sphere,
               const double *weights, int n_sig,
               int64_t n_samples, const int64_t *idx, double *val)
{
    for (int64_t s = 0; s < n_samples; ++s) {
        const int64_t *q = idx + 5 * s;
        int b = (int)q[0], c = (int)q[1];
        const int vi[3] = {(int)q[4], (int)q[3], (int)q[2]};   /* x, y, z */
        val[s] = 0.0;
        if (b < 0 || b >= B || c < 0 || c >= C || vi[2] < 0 || vi[2] >= D ||
            vi[1] < 0 || vi[1] >= H || vi[0] < 0 || vi[0] >= W)
            return -1;
        geom_t g;
        geom_for(&g, b, C, D, H, W, origin3, spacing3, origins, spacings, periodic, cell3);
        g.cut = cutoff_k != 0.0f;
        double acc = 0.0;
        for (int64_t a = offsets[b]; a < offsets[b + 1]; ++a) {
            const double *mu = xyz + 3 * a;
            const int32_t t = types[a];
            double wt = 1.0;
            if (weights) {
                if (!atom_ok(mu, t, n_sig))
                    continue;
                wt = weights[(size_t)a * C + c];
                if (wt == 0.0)
                    continue;
            } else if (t != c || !atom_ok(mu, t, C)) {
                continue;
            }
            g.rc = cutoff_radius(cutoff_k, sigma[t]);
            const double s2 = (double)sigma[t] * (double)sigma[t];
            double d[3];
            int inside = 1;
            for (int ax = 0; ax < 3 && inside; ++ax)
                inside = axis_offset(g.o[ax], g.h[ax], vi[ax], mu[ax], g.periodic,
                                     g.L[ax], g.cut, g.rc, &d[ax]);
            if (inside && sphere && g.cut &&
                d[0] * d[0] + d[1] * d[1] + d[2] * d[2] > g.rc * g.rc)
                inside = 0;
            if (inside) {
                double v;
                if (value == 1)
                    v = box1d(d[0] - 0.5 * g.h[0], d[0] + 0.5 * g.h[0], sigma[t]) *
                        box1d(d[1] - 0.5 * g.h[1], d[1] + 0.5 * g.h[1], sigma[t]) *
                        box1d(d[2] - 0.5 * g.h[2], d[2] + 0.5 * g.h[2], sigma[t]);
                else
                    v = exp(-(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) / (2.0 * s2));
                acc += weights ? wt * v : v;
            }
        }
        val[s] = acc;
    }
    return 0;
}

/* Number of atom-voxel pairs inside the cutoff windows (the algorithmic
   work count), without building a grid. */
int64_t pgo_count_evals(int B, const int64_t *offsets, const double *xyz, const int32_t *types,
                        int C, int D, int H, int W,
                        const double *origin3, const double *spacing3,
                        const double *origins, const double *spacings,
                        const float *sigma, float cutoff_k,
                        int periodic, const double *cell3)
{
    int64_t ev = 0;
    window_t w;
    if (window_alloc(&w, D, H, W))
        return -1;
    for (int b = 0; b < B; ++b) {
        geom_t g;
        geom_for(&g, b, C, D, H, W, origin3, spacing3, origins, spacings, periodic, cell3);
        for (int64_t a = offsets[b]; a < offsets[b + 1]; ++a) {
            const double *mu = xyz + 3 * a;
            if (!atom_ok(mu, types[a], C))
                continue;
            g.cut = cutoff_k != 0.0f;
            g.rc = cutoff_radius(cutoff_k, sigma[types[a]]);
            window_build(&w, &g, mu);
            ev += (int64_t)w.n[0] * w.n[1] * w.n[2];
        }
    }
    window_free(&w);
    return ev;
}

int pgo_version(void) { return 4; }
