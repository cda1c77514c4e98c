"""Pins of the FP64 oracle to facts the paper and the mathematics fix.

None of these compares the oracle with a retyped copy of itself: each one
checks it against a closed form (Poisson summation of a sampled Gaussian),
an exact invariant (translation, permutation, periodic images), an exact
rational brute force, finite differences, or hand-derived values with
dyadic inputs, chosen so that a plausible slip -- a dropped 1/2 in the
voxel centre, sigma read as a variance, swapped axes, an exclusive cutoff
edge, a wrong nearest image, a flipped gradient sign -- fails one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one_atom(mu, t=0, C=1):
    return (np.asarray([mu], np.float64), np.asarray([t], np.int32), np.asarray([0, 1]))


# ---------------------------------------------------------------- closed forms

def poisson_axis_sum(mu, o, h, sigma, m_max=40):
    """sum_{i in Z} exp(-(o + (i+1/2) h - mu)^2 / (2 sigma^2)) by Poisson
    summation: (sqrt(2 pi) sigma / h) * sum_m exp(-2 pi^2 m^2 sigma^2 / h^2)
    cos(2 pi m (mu - o - h/2) / h)."""
    a = mu - o - 0.5 * h
    s = 1.0
    for m in range(1, m_max):
        s += 2.0 * math.exp(-2.0 * math.pi ** 2 * m * m * sigma * sigma / (h * h)) * \
            math.cos(2.0 * math.pi * m * a / h)
    return math.sqrt(2.0 * math.pi) * sigma / h * s


@pytest.mark.parametrize("sigma,h", [(0.2, 0.5), (0.25, 0.5), (0.3, 0.35), (0.4, 0.5)])
def test_P3_lattice_sum_poisson(sigma, h):
    """No cutoff, atom >= 8 sigma from every face: the grid sum equals the
    product of three Poisson-summed 1-D lattice sums.  At sigma/h = 0.4 the
    m = 1 term is ~4%, so the voxel-centre convention and sigma's meaning
    (a standard deviation) are both pinned at 1e-12."""
    rng = np.random.default_rng(11)
    n = 40
    o = (-0.5 * n * h,) * 3
    mu = rng.uniform(-1.0, 1.0, size=3)
    sig = np.float32(sigma)
    xyz, t, off = one_atom(mu)
    g = oracle.grid_fp64(xyz, t, off, [sig], (n, n, n), h, o, cutoff_k=0.0)
    # the geometry enters as float32 values (h = 0.35 is not exact)
    h32 = float(np.float32(h))
    o32 = [float(np.float32(v)) for v in o]
    expect = np.prod([poisson_axis_sum(mu[q], o32[q], h32, float(sig)) for q in range(3)])
    assert abs(g.sum() / expect - 1.0) < 1e-12


@pytest.mark.parametrize("sigma", [0.4, 0.475, 0.55, 0.625, 0.7])
def test_P4_channel_integral(sigma):
    """Sum over a channel ~ N (2 pi sigma^2)^{3/2} / h^3 with relative error
    bounded by (1 + 2 exp(-2 pi^2 sigma^2 / h^2))^3 - 1 (no cutoff, atoms
    well inside)."""
    h = 0.5
    n = 48
    o = (-0.5 * n * h,) * 3
    rng = np.random.default_rng(5)
    N = 3
    mu = rng.uniform(-2.0, 2.0, size=(N, 3))
    sig = np.float32(sigma)
    g = oracle.grid_fp64(mu, np.zeros(N, np.int32), [0, N], [sig], (n, n, n), h, o, cutoff_k=0.0)
    s = float(sig)
    expect = N * (2 * math.pi * s * s) ** 1.5 / h ** 3
    bound = (1 + 2 * math.exp(-2 * math.pi ** 2 * s * s / h ** 2)) ** 3 - 1
    assert abs(g.sum() / expect - 1.0) <= bound + 1e-13


def test_P4_hydrogen_example():
    """One H atom (sigma 0.4) at 0.5 A spacing sums to ~8.064."""
    h, n = 0.5, 40
    g = oracle.grid_fp64([[0.1, -0.2, 0.3]], [0], [0, 1], [np.float32(0.4)], (n, n, n), h,
                         (-10.0, -10.0, -10.0), cutoff_k=0.0)
    assert abs(g.sum() - (2 * math.pi * float(np.float32(0.4)) ** 2) ** 1.5 / h ** 3) < 2e-4
    assert abs(g.sum() - 8.064) < 1e-3


def test_P1_voxel_centre_peak_and_layout():
    """Dyadic inputs: an atom exactly on the centre of voxel (ix, iy, iz) =
    (3, 9, 14) gives exactly 1.0 there, at out[c, 14, 9, 3] (x fastest);
    the neighbour one voxel along x holds exp(-h^2 / (2 sigma^2))."""
    h = 0.5
    o = (-4.0, -8.0, -2.0)
    ix, iy, iz = 3, 9, 14
    mu = [o[0] + (ix + 0.5) * h, o[1] + (iy + 0.5) * h, o[2] + (iz + 0.5) * h]
    sig = np.float32(0.5)
    g = oracle.grid_fp64([mu], [1], [0, 1], [np.float32(0.4), sig], (16, 20, 24), h, o)
    assert g.shape == (1, 2, 16, 20, 24)
    assert g[0, 0].max() == 0.0                       # other channel untouched
    assert g[0, 1, iz, iy, ix] == 1.0
    assert np.unravel_index(np.argmax(g[0, 1]), g[0, 1].shape) == (iz, iy, ix)
    s = float(sig)
    assert abs(g[0, 1, iz, iy, ix + 1] - math.exp(-h * h / (2 * s * s))) < 1e-16
    assert abs(g[0, 1, iz + 1, iy + 1, ix] - math.exp(-2 * h * h / (2 * s * s))) < 1e-16


def test_P1_window_width_and_inclusive_edge():
    """rc = k sigma = 3 * 0.5 = 1.5 = 3 h exactly: an atom on a voxel centre
    keeps 2*3+1 = 7 voxels per axis, the edge voxels (|d| == rc) included
    with value exp(-4.5); moving the atom by one float32 ulp along +x drops
    the low-x face (|d| just above rc) and keeps the high-x face."""
    h = 0.5
    o = (-8.0, -8.0, -8.0)
    mu = np.array([o[0] + 16.5 * h, o[1] + 16.5 * h, o[2] + 16.5 * h])
    sig = np.float32(0.5)
    g = oracle.grid_fp64([mu], [0], [0, 1], [sig], (32, 32, 32), h, o, cutoff_k=3.0)[0, 0]
    nz = np.argwhere(g > 0)
    assert nz.min(axis=0).tolist() == [13, 13, 13]
    assert nz.max(axis=0).tolist() == [19, 19, 19]
    assert len(nz) == 7 ** 3
    assert abs(g[16, 16, 13] - math.exp(-4.5)) < 1e-16
    mu2 = mu.copy()
    mu2[0] = float(np.nextafter(np.float32(mu[0]), np.float32(100.0)))
    g2 = oracle.grid_fp64([mu2], [0], [0, 1], [sig], (32, 32, 32), h, o, cutoff_k=3.0)[0, 0]
    nz2 = np.argwhere(g2 > 0)
    assert nz2[:, 2].min() == 14 and nz2[:, 2].max() == 19
    assert len(nz2) == 6 * 7 * 7


def test_P1_cutoff_radius_is_single_precision_product():
    """rc = fl32(k * sigma): k = 3, sigma = 0.55 (float32) gives
    rc = 1.6500000953674316 (the float32 product), not 3 * 0.55 in double.
    A voxel at offset exactly equal to that float is inside; at the next
    float above it is outside."""
    sig = np.float32(0.55)
    rc = np.float32(3.0) * sig
    assert float(rc) != 3.0 * float(sig)
    h = 0.5
    o = (0.0, 0.0, 0.0)
    centre = o[0] + 4.5 * h                 # voxel 4
    for mu0, inside in ((centre - float(rc), True),
                        (centre - float(np.nextafter(rc, np.float32(9))), False)):
        assert float(np.float32(mu0)) == mu0     # exactly representable coordinate
        g = oracle.grid_fp64([[mu0, 1.25, 1.25]], [0], [0, 1], [sig], (8, 8, 8), h, o)[0, 0]
        assert (g[2, 2, 4] > 0) == inside


def test_P5_cube_cutoff_mass_separable():
    """With k = 3 the per-atom mass equals the product of the three
    truncated 1-D sums (rank-1 separability of one atom, §III-A / §IV-C),
    computed here in 1-D with the cutoff applied per axis; and it is within
    edge discretisation of erf(3/sqrt 2)^3 (2 pi sigma^2)^{3/2} / h^3."""
    rng = np.random.default_rng(8)
    h = float(np.float32(0.35))             # geometry enters as float32 values
    n = 48
    o = (float(np.float32(-8.4)),) * 3
    sig = np.float32(0.55)
    s = float(sig)
    rc = float(np.float32(3.0) * sig)
    mu = rng.uniform(-3, 3, size=3)
    g = oracle.grid_fp64([mu], [0], [0, 1], [sig], (n, n, n), h, o)[0, 0]
    one_d = []
    for q in range(3):
        d = o[q] + (np.arange(n) + 0.5) * h - mu[q]
        one_d.append(np.where(np.abs(d) <= rc, np.exp(-d * d / (2 * s * s)), 0.0))
    outer = np.einsum("z,y,x->zyx", one_d[2], one_d[1], one_d[0])
    assert np.max(np.abs(g - outer)) < 1e-15
    mass = np.prod([v.sum() for v in one_d])
    assert abs(g.sum() / mass - 1) < 1e-13
    ref = math.erf(3 / math.sqrt(2)) ** 3 * (2 * math.pi * s * s) ** 1.5 / h ** 3
    assert abs(g.sum() / ref - 1) < 0.03


def test_P6_permutation_invariance():
    wl = synth.WORKLOADS["single20"]
    b = wl.batch()
    perm = np.random.default_rng(3).permutation(b.n_atoms)
    kw = dict(dims=wl.dims, spacing=wl.spacing, origin=wl.origin)
    g1 = oracle.grid_fp64(b.xyz, b.types, b.offsets, wl.sigma(), **kw)
    g2 = oracle.grid_fp64(b.xyz[perm], b.types[perm], b.offsets, wl.sigma(), **kw)
    assert np.max(np.abs(g1 - g2)) <= 1e-14 * np.max(g1)


def test_P7_integer_voxel_translation():
    """Coordinates on a 2^-12 lattice and h = 0.5: translating every atom by
    n voxels shifts the grid by n voxels, bit for bit."""
    rng = np.random.default_rng(9)
    h = 0.5
    o = (-8.0, -8.0, -8.0)
    mu = np.round(rng.uniform(-2, 2, size=(6, 3)) * 4096) / 4096
    t = rng.integers(0, 3, size=6).astype(np.int32)
    sig = synth.sigma_table(3)
    n = np.array([2, -1, 3])
    g1 = oracle.grid_fp64(mu, t, [0, 6], sig, (32, 32, 32), h, o)[0]
    g2 = oracle.grid_fp64(mu + n * h, t, [0, 6], sig, (32, 32, 32), h, o)[0]
    a = g1[:, 4:24, 4:24, 4:24]
    b = g2[:, 4 + n[2]:24 + n[2], 4 + n[1]:24 + n[1], 4 + n[0]:24 + n[0]]
    assert np.array_equal(a, b)


def test_P8_periodic_images_and_roll():
    """Periodic cell L = N h = 8 (dyadic): mu and mu + L e_alpha give the same
    grid; translating by one voxel is an exact cyclic roll; an atom at a
    cell face feeds the opposite face."""
    h = 0.5
    L = 8.0
    o = (0.0, 0.0, 0.0)
    sig = np.float32(0.5)
    mu = np.array([0.125, 3.0, 7.875])
    kw = dict(dims=(16, 16, 16), spacing=h, origin=o, cell=L)
    g = oracle.grid_fp64([mu], [0], [0, 1], [sig], **kw)[0, 0]
    for q in range(3):
        e = np.zeros(3)
        e[q] = L
        assert np.array_equal(g, oracle.grid_fp64([mu + e], [0], [0, 1], [sig], **kw)[0, 0])
        assert np.array_equal(g, oracle.grid_fp64([mu - 2 * e], [0], [0, 1], [sig], **kw)[0, 0])
    g_roll = oracle.grid_fp64([mu + [h, 0, 0]], [0], [0, 1], [sig], **kw)[0, 0]
    assert np.array_equal(np.roll(g, 1, axis=2), g_roll)
    assert g[:, :, 15].max() > 0.3 and g[:, :, 0].max() > 0.3   # x face wraps
    assert g[:, :, 8].max() == 0.0


def test_P8_periodic_grid_larger_than_cell():
    """Grid extent 20.48 A over a 20 A cell: voxels beyond the cell see the
    nearest image, so an atom near x = 0 also appears near x = 20."""
    h = 0.16
    sig = np.float32(0.4)
    g = oracle.grid_fp64([[0.05, 10.0, 10.0]], [0], [0, 1], [sig], (128, 128, 128), h,
                         (0.0, 0.0, 0.0), cell=20.0)[0, 0]
    row = g[62, 62]
    assert row[0] > 0.5
    i_img = int((20.05 - 0.0) / h)
    assert row[i_img] > 0.5
    assert row[64] == 0.0


@pytest.mark.parametrize("seed", range(12))
def test_P9_brute_force_tiny(seed):
    """The window-iterating C oracle equals the all-pairs exact-rational
    brute force on tiny grids, random k, periodic on and off."""
    rng = np.random.default_rng(100 + seed)
    D, H, W = (int(v) for v in rng.integers(2, 9, size=3))
    C = int(rng.integers(1, 4))
    n_mol = int(rng.integers(1, 3))
    counts = rng.integers(0, 6, size=n_mol)
    off = np.concatenate([[0], np.cumsum(counts)])
    h = float(rng.choice([0.25, 0.5, 0.35, 0.3]))
    o = tuple(float(np.float32(v)) for v in rng.uniform(-1.5, 0.0, size=3))
    periodic = bool(seed % 3 == 0)
    cell = None
    if periodic:
        cell = float(np.float32(rng.uniform(2.5, 3.0)))
    hi = np.array([W, H, D]) * h
    xyz = (rng.uniform(-0.5, 1.0, size=(off[-1], 3)) * hi + np.array(o)).astype(np.float32)
    types = rng.integers(0, C, size=off[-1]).astype(np.int32)
    sig = rng.uniform(0.2, 0.45, size=C).astype(np.float32)
    k = float(rng.choice([0.0, 1.0, 2.0, 3.0])) if not periodic else float(rng.choice([1.0, 2.0]))
    g = oracle.grid_fp64(xyz, types, off, sig, (D, H, W), h, o, cutoff_k=k, cell=cell)
    b = oracle.brute_fp64(xyz, types, off, sig, (D, H, W), h, o, cutoff_k=k, cell=cell)
    assert np.max(np.abs(g - b)) <= 1e-14 * max(1.0, np.max(b))
    assert np.array_equal(g > 0, b > 0)


def test_P9_brute_force_edge_hits():
    """Atoms placed so that voxel centres sit exactly on the cutoff edge
    (dyadic rc = 0.75 = 1.5 h): the exact brute force and the oracle agree
    on every edge voxel."""
    h = 0.5
    o = (0.0, 0.0, 0.0)
    sig = np.float32(0.25)                  # rc = 3 * 0.25 = 0.75
    xyz = np.array([[1.0, 1.0, 1.0], [2.0, 0.5, 1.5]], np.float32)
    g = oracle.grid_fp64(xyz, [0, 0], [0, 2], [sig], (6, 6, 6), h, o)
    b = oracle.brute_fp64(xyz, [0, 0], [0, 2], [sig], (6, 6, 6), h, o)
    assert np.max(np.abs(g - b)) < 1e-15
    # voxel centre 0.25 is 0.75 from 1.0: inside (inclusive edge)
    assert g[0, 0, 0, 0, 0] > 0


def test_invalid_atoms_skipped():
    xyz = np.array([[0, 0, 0], [np.nan, 0, 0], [0.5, 0.5, 0.5], [0, 0, 0]], np.float64)
    t = np.array([0, 0, 5, -1], np.int32)
    g, st = oracle.grid_fp64(xyz, t, [0, 4], [np.float32(0.4)], (8, 8, 8), 0.5, (-2, -2, -2),
                             return_stats=True)
    g0 = oracle.grid_fp64(xyz[:1], t[:1], [0, 1], [np.float32(0.4)], (8, 8, 8), 0.5, (-2, -2, -2))
    assert st["skipped"] == 3
    assert np.array_equal(g, g0)


def test_empty_molecules_and_batch():
    g = oracle.grid_fp64(np.zeros((0, 3)), np.zeros(0, np.int32), [0, 0, 0], [np.float32(0.4)],
                         (4, 4, 4), 0.5, (0, 0, 0))
    assert g.shape == (2, 1, 4, 4, 4) and not g.any()
    g = oracle.grid_fp64(np.zeros((0, 3)), np.zeros(0, np.int32), [0], [np.float32(0.4)],
                         (4, 4, 4), 0.5, (0, 0, 0))
    assert g.shape == (0, 1, 4, 4, 4)


def test_per_molecule_origin_and_spacing():
    """Per-structure origins/spacings equal separate calls (§III-A: the
    bounding box and resolution may differ per molecule)."""
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(3)
    org = np.array([[-8, -8, -8], [-7.5, -8.25, -6.0], [-4, -4, -4]], np.float64)
    spc = np.array([[0.5, 0.5, 0.5], [0.45, 0.5, 0.55], [0.25, 0.25, 0.25]], np.float64)
    g = oracle.grid_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, 0.5,
                         origins=org, spacings=spc)
    for m in range(3):
        s = b.subset([m])
        gm = oracle.grid_fp64(s.xyz, s.types, s.offsets, wl.sigma(), wl.dims, spc[m], org[m])
        assert np.array_equal(g[m], gm[0])


def test_voxels_match_dense():
    """The per-voxel all-atoms form equals the dense window form."""
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(4)
    kw = dict(dims=wl.dims, spacing=wl.spacing, origin=wl.origin)
    g = oracle.grid_fp64(b.xyz, b.types, b.offsets, wl.sigma(), **kw)
    rng = np.random.default_rng(1)
    nzi = np.argwhere(g > 0)
    pick = nzi[rng.choice(len(nzi), 200, replace=False)]
    rnd = np.stack([rng.integers(0, s, 300) for s in g.shape], axis=1)
    idx = np.concatenate([pick, rnd])
    v = oracle.voxels_fp64(b.xyz, b.types, b.offsets, wl.sigma(), idx=idx, **kw)
    assert np.max(np.abs(v - g[tuple(idx.T)])) < 1e-14


def test_count_evals_matches_nonzeros():
    wl = synth.WORKLOADS["single20"]
    b = wl.batch()
    kw = dict(dims=wl.dims, spacing=wl.spacing, origin=wl.origin)
    n = 0
    for a in range(b.n_atoms):
        g = oracle.grid_fp64(b.xyz[a:a + 1], b.types[a:a + 1], [0, 1], wl.sigma(), **kw)
        n += int((g > 0).sum())
    assert oracle.count_evals(b.xyz, b.types, b.offsets, wl.sigma(), **kw) == n


# ------------------------------------------------------------------- gradient

def _edge_safe(mu, o, h, rc, n, eps):
    """True if no voxel centre is within eps of the cutoff edge on any axis
    (there the windowed map is not differentiable)."""
    for q in range(3):
        d = o[q] + (np.arange(n) + 0.5) * h - mu[q]
        if np.any(np.abs(np.abs(d) - rc) < eps):
            return False
    return True


def test_P10_gradient_vs_finite_differences():
    wl = synth.WORKLOADS["single20"]
    b = wl.batch()
    kw = dict(dims=wl.dims, spacing=wl.spacing, origin=wl.origin)
    sig = wl.sigma()
    U = synth.upstream(7, wl.grid_shape()).astype(np.float64)
    g = oracle.grad_fp64(b.xyz, b.types, b.offsets, sig, U=U, **kw)
    xyz = b.xyz.astype(np.float64)
    hfd = 1e-4
    checked = 0
    for a in range(0, b.n_atoms, 3):
        rc = float(np.float32(3.0) * sig[b.types[a]])
        if not _edge_safe(xyz[a], wl.origin, wl.spacing, rc, 32, 3 * hfd):
            continue
        for q in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[a, q] += hfd
            xm[a, q] -= hfd
            lp = np.sum(U * oracle.grid_fp64(xp, b.types, b.offsets, sig, **kw))
            lm = np.sum(U * oracle.grid_fp64(xm, b.types, b.offsets, sig, **kw))
            fd = (lp - lm) / (2 * hfd)
            assert abs(fd - g[a, q]) <= 1e-6 * max(1.0, abs(fd))
            checked += 1
    assert checked >= 9


def test_P11_gradient_symmetry():
    """Atom on a voxel centre, U == 1, window inside: the gradient is 0
    (mirror-symmetric window), up to summation rounding."""
    h = 0.5
    o = (-8.0, -8.0, -8.0)
    mu = [o[0] + 15.5 * h, o[1] + 16.5 * h, o[2] + 14.5 * h]
    U = np.ones((1, 1, 32, 32, 32))
    g = oracle.grad_fp64([mu], [0], [0, 1], [np.float32(0.55)], (32, 32, 32), h, U=U, origin=o)
    # terms of size ~1 cancel in pairs; allow summation rounding only
    assert np.max(np.abs(g)) <= 1e-13


def test_P12_uniform_upstream_gradient_no_cutoff():
    """k = 0, U == 1: dL/dmu_alpha is the derivative of the Poisson lattice
    sum, bounded by (4 pi / h) e^{-2 pi^2 sigma^2 / h^2} prod S."""
    h = 0.5
    n = 40
    o = (-10.0, -10.0, -10.0)
    for s32, mu in ((np.float32(0.4), [0.13, -0.21, 0.07]), (np.float32(0.55), [0.3, 0.1, -0.2])):
        s = float(s32)
        U = np.ones((1, 1, n, n, n))
        g = oracle.grad_fp64([mu], [0], [0, 1], [s32], (n, n, n), h, U=U, origin=o, cutoff_k=0.0)
        S = np.prod([poisson_axis_sum(mu[q], o[q], h, s) for q in range(3)])
        bound = 4 * math.pi / h * math.exp(-2 * math.pi ** 2 * s * s / h ** 2) * S
        assert np.max(np.abs(g)) <= bound * 1.0001 + 1e-13
        # and the sign/magnitude of the m = 1 Poisson term is right: compare
        # with the analytic derivative of the truncated Poisson series
        for q in range(3):
            Sq = [poisson_axis_sum(mu[r], o[r], h, s) for r in range(3)]
            eps = 1e-6
            dq = (poisson_axis_sum(mu[q] + eps, o[q], h, s) - poisson_axis_sum(mu[q] - eps, o[q], h, s)) / (2 * eps)
            other = np.prod([Sq[r] for r in range(3) if r != q])
            assert abs(g[0, q] - dq * other) <= 1e-7 * S + 1e-12


# ------------------------------------------------------------ paper's example

def test_listing2_shape_golden():
    """§V Listing 2: two points (channel, x, y, z), a unit box, 2 channels,
    grid_size 32, 'variance' 0.05 -> a (2, 32, 32, 32) grid.  The paper
    prints only the shape.  Reading: box [0, 1]^3, spacing 1/32, sigma 0.05."""
    with open(os.path.join(GOLDEN, "listing2_shape.json")) as f:
        gold = json.load(f)
    pts = np.asarray(gold["points"], np.float64)
    n = gold["grid_size"]
    h = gold["width"] / n
    g = oracle.grid_fp64(pts[:, 1:], pts[:, 0].astype(np.int32), [0, len(pts)],
                         [np.float32(gold["variance"])] * gold["num_channels"],
                         (n, n, n), h, (0.0, 0.0, 0.0))
    assert list(g.shape[1:]) == gold["shape"]
    # each point lands in its own channel; its maximum sits on the voxel
    # whose centre is nearest (either voxel on an exact tie)
    for c, x, y, z in pts:
        gc = g[0, int(c)]
        m = gc.max()
        near = [{int(np.floor(v / h - 0.5)), int(np.ceil(v / h - 0.5))} for v in (z, y, x)]
        near = [{min(max(i, 0), n - 1) for i in s} for s in near]
        hits = {tuple(int(i) for i in ix) for ix in np.argwhere(gc == m)}
        assert hits and all(hz in near[0] and hy in near[1] and hx in near[2] for hz, hy, hx in hits)
        assert g[0, 1 - int(c)][tuple(next(iter(hits)))] < m
