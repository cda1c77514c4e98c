"""Pins of the oracle's box form (the integral of the normalised Gaussian
over each voxel, §III-A Eq. 2-5) to facts the paper and the mathematics fix.

Each check uses something other than the oracle's own arithmetic: the
telescoping of per-voxel erf differences into a closed form for the whole
grid (the paper's Eq. 6: a channel sums to its atom count), numerical
quadrature of the 1-D Gaussian in the far tail, the midpoint rule for small
voxels (against the separately pinned point form), finite differences,
reflection symmetry and periodic images.  A plausible slip -- a reversed
erf difference, the voxel centre taken as the lower edge, sigma read as a
variance, a missing 1/2, an erf difference that cancels in the tails, a
gradient of the wrong sign -- fails one of them.
"""
import math

import numpy as np
import pytest

import oracle
import synth


def one(mu, t=0):
    return (np.asarray([mu], np.float64), np.asarray([t], np.int32), np.asarray([0, 1]))


def f32(v):
    """The float32 value of v: sigma and the grid geometry are float32 inputs."""
    return float(np.float32(v))


def axis_mass(lo_edge, hi_edge, mu, sigma):
    """Mass of the normalised 1-D Gaussian between two edges (math.erf)."""
    s = math.sqrt(2.0) * sigma
    return 0.5 * (math.erf((hi_edge - mu) / s) - math.erf((lo_edge - mu) / s))


@pytest.mark.parametrize("mu", [(0.1, -0.3, 0.45), (3.9, -3.2, 0.0), (-6.3, 5.1, 7.7)])
def test_box_grid_mass_telescopes(mu):
    """No cutoff: the grid sum telescopes to the product over axes of the mass
    between the outer grid faces (Eq. 6 before truncation)."""
    sig, h, N, o = f32(0.55), 0.5, 32, -8.0
    x, t, off = one(mu)
    g = oracle.grid_fp64(x, t, off, [sig], (N, N, N), h, (o, o, o), cutoff_k=0.0, value="box")
    want = 1.0
    for q in range(3):
        want *= axis_mass(o, o + N * h, mu[q], sig)
    assert g.sum() == pytest.approx(want, rel=1e-12)
    if all(abs(m) < 6 for m in mu):
        assert g.sum() == pytest.approx(1.0, abs=1e-12)


def test_box_channel_sums_count_atoms():
    """Eq. 6: each channel sums to the number of atoms of its type, the grid
    to the number of atoms (atoms well inside, no cutoff)."""
    wl = synth.WORKLOADS["single20"]
    b = wl.batch()
    g = oracle.grid_fp64(b.xyz, b.types, b.offsets, wl.sigma(), (48, 48, 48), 0.5,
                         (-12, -12, -12), cutoff_k=0.0, value="box")
    counts = np.bincount(b.types, minlength=5)
    np.testing.assert_allclose(g[0].sum(axis=(1, 2, 3)), counts, rtol=1e-10, atol=1e-10)
    assert g.sum() == pytest.approx(b.n_atoms, rel=1e-11)


@pytest.mark.parametrize("mu,k", [((0.25, -0.125, 0.0625), 3.0), ((1.3, 0.7, -2.2), 2.0)])
def test_box_window_mass_closed_form(mu, k):
    """With the cube cutoff the sum over one atom's window telescopes to the
    mass between the window's outer edges on each axis; the window is found
    here by brute force on the voxel centres."""
    sig, h, N, o = 0.5, 0.25, 40, -5.0
    x, t, off = one(mu)
    g = oracle.grid_fp64(x, t, off, [sig], (N, N, N), h, (o, o, o), cutoff_k=k, value="box")
    rc = float(np.float32(k) * np.float32(sig))
    want = 1.0
    for q in range(3):
        inside = [i for i in range(N) if abs(o + (i + 0.5) * h - mu[q]) <= rc]
        want *= axis_mass(o + inside[0] * h, o + (inside[-1] + 1) * h, mu[q], sig)
    assert g.sum() == pytest.approx(want, rel=1e-12)


def test_box_far_tail_matches_quadrature():
    """Far in the tail the voxel mass is ~1e-12 of the peak; it must match
    numerical quadrature of the Gaussian to 1e-9 relative (an erf difference
    there would lose all but a few digits to cancellation)."""
    from scipy.integrate import quad
    sig, h = f32(0.4), 0.25
    W = 32
    # y and z voxels so wide (40 sigma, centred) that their mass is 1.0
    mu = (0.0, 0.0, 0.0)
    x, t, off = one(mu)
    wide = f32(40 * sig)
    g = oracle.grid_fp64(x, t, off, [sig], (1, 1, W), (h, wide, wide), (0.0, -wide / 2, -wide / 2),
                         cutoff_k=0.0, value="box")
    pdf = lambda u: math.exp(-u * u / (2 * sig * sig)) / (math.sqrt(2 * math.pi) * sig)
    for i in (10, 14, 17, 20):
        lo, hi = i * h, (i + 1) * h
        ref, _ = quad(pdf, lo, hi, epsabs=0, epsrel=1e-13)
        assert g[0, 0, 0, 0, i] == pytest.approx(ref, rel=1e-9), i


def test_box_small_voxels_approach_scaled_point_samples():
    """Midpoint rule: for h << sigma each axis mass is h * pdf(centre) with a
    relative correction of h^2/24 * (d^2/sigma^4 - 1/sigma^2); the box grid
    equals (h / (sqrt(2 pi) sigma))^3 times the (separately pinned) point
    grid within that bound."""
    sig, h, N = 0.5, f32(0.02), 40
    mu = (0.013, -0.007, 0.021)
    x, t, off = one(mu)
    o = -N * h / 2
    box = oracle.grid_fp64(x, t, off, [sig], (N, N, N), h, (o, o, o), cutoff_k=0.0, value="box")
    pt = oracle.grid_fp64(x, t, off, [sig], (N, N, N), h, (o, o, o), cutoff_k=0.0)
    scale = (h / (math.sqrt(2 * math.pi) * sig)) ** 3
    ratio = box / (scale * pt)
    bound = 3 * (h * h / 24) * (((N * h) ** 2 / sig ** 4) + 1 / sig ** 2) * 1.1
    assert np.max(np.abs(ratio - 1)) <= bound
    # and the correction has the predicted sign at the centre (negative curvature)
    c = N // 2
    assert ratio[0, 0, c, c, c] < 1.0


def test_box_gradient_matches_finite_differences():
    wl = synth.WORKLOADS["single20"]
    b = wl.batch()
    dims, h, o = (24, 24, 24), 0.5, (-6, -6, -6)
    U = np.random.default_rng(3).standard_normal((1, 5) + dims)
    grad = oracle.grad_fp64(b.xyz, b.types, b.offsets, wl.sigma(), dims, h, U, o, cutoff_k=0.0,
                            value="box")
    eps = 1e-6
    fd = np.zeros_like(grad)
    for a in range(b.n_atoms):
        for q in range(3):
            xp = b.xyz.astype(np.float64).copy()
            xm = xp.copy()
            xp[a, q] += eps
            xm[a, q] -= eps
            gp = oracle.grid_fp64(xp, b.types, b.offsets, wl.sigma(), dims, h, o, cutoff_k=0.0,
                                  value="box")
            gm = oracle.grid_fp64(xm, b.types, b.offsets, wl.sigma(), dims, h, o, cutoff_k=0.0,
                                  value="box")
            fd[a, q] = ((gp - gm) * U).sum() / (2 * eps)
    rel = np.linalg.norm(grad - fd) / np.linalg.norm(fd)
    assert rel < 1e-7


def test_box_reflection_symmetry_and_gradient_zero():
    """An atom at a voxel centre: the box grid is symmetric under reflection
    of each axis through that centre, and with a symmetric upstream the
    gradient vanishes."""
    sig, h, N = 0.45, 0.5, 21
    o = -N * h / 2   # voxel 10 is centred at 0
    x, t, off = one((0.0, 0.0, 0.0))
    g = oracle.grid_fp64(x, t, off, [sig], (N, N, N), h, (o, o, o), value="box")[0, 0]
    for axis in range(3):
        np.testing.assert_array_equal(g, np.flip(g, axis=axis))
    grad = oracle.grad_fp64(x, t, off, [sig], (N, N, N), h, np.ones((1, 1, N, N, N)), (o, o, o),
                            value="box")
    assert np.max(np.abs(grad)) < 1e-15


def test_box_periodic_image_is_the_same_atom():
    sig, h, L = 0.5, 0.25, 8.0
    dims = (32, 32, 32)
    mu = np.array([0.3, 7.9, 4.0])
    g0 = oracle.grid_fp64(mu[None], [0], [0, 1], [sig], dims, h, (0, 0, 0), cell=L, value="box")
    g1 = oracle.grid_fp64((mu + [L, -L, 2 * L])[None], [0], [0, 1], [sig], dims, h, (0, 0, 0),
                          cell=L, value="box")
    np.testing.assert_allclose(g0, g1, rtol=0, atol=1e-15)
    # the atom at the x face feeds both faces
    assert g0[0, 0, :, :, 0].sum() > 0 and g0[0, 0, :, :, -1].sum() > 0
