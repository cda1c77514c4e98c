"""Pins of the oracle's triclinic cells (§III-A lattice translations for a
general cell), against things other than its image expansion: the
orthorhombic nearest-image path for a diagonal cell, the invariance of the
grid under a unimodular change of cell basis (the same lattice) and under
lattice translations of the atoms, a per-voxel brute force that searches
every lattice image, finite differences of the gradient, and the overlap
test of the cell check.

Coordinates and cell entries are dyadic where a pin is bitwise, so that
every image position is exact in float32 and the image rounding of the
reading plays no part.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import triclinic

SHEAR = np.array([[8.0, 2.5, 1.0], [0.0, 7.5, -1.5], [0.0, 0.0, 8.5]])
UNIMOD = np.array([[1, 1, 0], [0, 1, 0], [-1, 0, 1]])    # det 1


def dyadic_atoms(seed, n, lo, hi, types=3, step=2.0 ** -8):
    rng = np.random.default_rng(seed)
    xyz = (np.round(rng.uniform(lo, hi, size=(n, 3)) / step) * step).astype(np.float32)
    return xyz, rng.integers(0, types, n).astype(np.int32)


@pytest.mark.parametrize("value", ["point", "box"])
def test_diagonal_cell_is_the_orthorhombic_path(value):
    xyz, t = dyadic_atoms(1, 12, 0.0, 8.0)
    sig = [0.4, 0.5, 0.6]
    dims, h = (32, 32, 32), 0.25
    ref = oracle.grid_fp64(xyz, t, [0, 5, 12], sig, dims, h, (0, 0, 0), cell=8.0, value=value)
    got = triclinic.grid_triclinic_fp64(xyz, t, [0, 5, 12], sig, dims, h, np.diag([8.0] * 3),
                                        (0, 0, 0), value=value)
    np.testing.assert_array_equal(got, ref)


def test_diagonal_cell_random_coordinates():
    """Arbitrary float32 coordinates: image positions are rounded to float32
    (the reading), the orthorhombic path decides exactly -- they agree to
    the rounding of the image positions."""
    rng = np.random.default_rng(2)
    xyz = rng.uniform(0, 8, size=(10, 3)).astype(np.float32)
    t = rng.integers(0, 3, 10).astype(np.int32)
    sig = [0.4, 0.5, 0.6]
    ref = oracle.grid_fp64(xyz, t, [0, 10], sig, (30, 30, 30), 0.3, (-0.5, -0.5, -0.5), cell=8.0)
    got = triclinic.grid_triclinic_fp64(xyz, t, [0, 10], sig, (30, 30, 30), 0.3,
                                        np.diag([8.0] * 3), (-0.5, -0.5, -0.5))
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5


@pytest.mark.parametrize("M", [np.diag([8.0] * 3), SHEAR])
def test_unimodular_basis_gives_the_same_grid(M):
    xyz, t = dyadic_atoms(3, 10, -1.0, 9.0)
    sig = [0.4, 0.5, 0.6]
    dims, h, o = (28, 30, 32), 0.3125, (-0.5, 0.25, -1.0)
    g0 = triclinic.grid_triclinic_fp64(xyz, t, [0, 10], sig, dims, h, M, o)
    g1 = triclinic.grid_triclinic_fp64(xyz, t, [0, 10], sig, dims, h, M @ UNIMOD, o)
    np.testing.assert_array_equal(g0, g1)
    assert g0.sum() > 0


def test_lattice_translation_invariance():
    xyz, t = dyadic_atoms(4, 8, 0.0, 8.0)
    sig = [0.4, 0.5, 0.6]
    dims, h = (30, 30, 30), 0.3
    shift = (SHEAR @ np.array([1, -2, 1])).astype(np.float32)
    g0 = triclinic.grid_triclinic_fp64(xyz, t, [0, 8], sig, dims, h, SHEAR, (0, 0, 0))
    g1 = triclinic.grid_triclinic_fp64(xyz + shift, t, [0, 8], sig, dims, h, SHEAR, (0, 0, 0))
    np.testing.assert_array_equal(g0, g1)


def test_per_voxel_brute_force_over_lattice_images():
    """Every voxel centre against every image within a wide lattice range:
    at most one image of an atom lies within the cube, and the grid holds
    its Gaussian."""
    rng = np.random.default_rng(5)
    xyz = rng.uniform(0, 8, size=(4, 3)).astype(np.float32)
    t = np.array([0, 1, 1, 0], np.int32)
    sig = np.array([0.45, 0.6], np.float32)
    dims, h, o = (9, 10, 11), np.float32(0.9), np.array([-1.3, -0.7, 0.4], np.float32)
    got = triclinic.grid_triclinic_fp64(xyz, t, [0, 4], sig, dims, float(h), SHEAR, o)
    rc = (np.float32(3.0) * sig).astype(np.float64)
    want = np.zeros_like(got)
    D, H, W = dims
    images = [[triclinic.image_position(xyz[a], SHEAR, n)
               for n in itertools.product(range(-3, 4), repeat=3)] for a in range(4)]
    for z, y, x in itertools.product(range(D), range(H), range(W)):
        r = o.astype(np.float64) + (np.array([x, y, z]) + 0.5) * np.float64(h)
        for a in range(4):
            inside = [p for p in images[a]
                      if np.all(np.abs(r - p.astype(np.float64)) <= rc[t[a]])]
            assert len(inside) <= 1
            if inside:
                d = r - inside[0].astype(np.float64)
                want[0, t[a], z, y, x] += np.exp(-(d @ d) / (2.0 * np.float64(sig[t[a]]) ** 2))
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-15)
    assert (got > 0).sum() > 100


def test_gradient_matches_finite_differences():
    """Dyadic coordinates and a dyadic step keep every image position exact."""
    xyz, t = dyadic_atoms(6, 5, 0.5, 7.5, step=2.0 ** -12)
    sig = [0.4, 0.5, 0.6]
    dims, h = (28, 28, 30), 0.3
    U = np.random.default_rng(7).standard_normal((1, 3) + dims)
    g = triclinic.grad_triclinic_fp64(xyz, t, [0, 5], sig, dims, h, U, SHEAR, (0, 0, 0))
    eps = 2.0 ** -10
    fd = np.zeros_like(g)
    for a in range(5):
        for q in range(3):
            xp = xyz.astype(np.float64).copy()
            xm = xp.copy()
            xp[a, q] += eps
            xm[a, q] -= eps
            lp = (triclinic.grid_triclinic_fp64(xp, t, [0, 5], sig, dims, h, SHEAR, (0, 0, 0)) * U).sum()
            lm = (triclinic.grid_triclinic_fp64(xm, t, [0, 5], sig, dims, h, SHEAR, (0, 0, 0)) * U).sum()
            fd[a, q] = (lp - lm) / (2 * eps)
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-4


def test_cell_check_rejects_overlapping_image_cubes():
    assert triclinic.check_cell(SHEAR, 2.1)
    thin = np.array([[8.0, 7.0, 0.0], [0.0, 1.5, 0.0], [0.0, 0.0, 8.0]])
    # n = (-1, 1, 0) gives (-1, 1.5, 0): Chebyshev norm 1.5 <= 2 rc for rc = 0.9
    assert not triclinic.check_cell(thin, 0.9)
    assert triclinic.check_cell(thin, 0.7)


# -- image positions: the exact lattice sum rounded once to float32 --------

EDGE = np.array([[2.0 ** -24, 2.0 ** -80, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


@pytest.mark.parametrize("n,want", [
    ((1, 0, 0), 1.0),                         # 1 + 2^-24: a tie, to the even 1
    ((3, 0, 0), 1.0 + 2.0 ** -22),            # 1 + 3 2^-24: a tie, to the even neighbour above
    ((1, 1, 0), 1.0 + 2.0 ** -23),            # just past the tie: up (double arithmetic
                                              # would round 1 + 2^-24 + 2^-80 to the tie, then down)
    ((-1, 0, 0), 1.0 - 2.0 ** -24),           # below 1 the step is 2^-24: exact
    ((0, 0, 0), 1.0),
])
def test_image_position_rounds_the_exact_sum_once(n, want):
    got = triclinic.image_position(np.array([1.0, 0.0, 0.0], np.float32), EDGE, n)
    assert got[0] == np.float32(want)


def test_image_position_exact_when_representable():
    """Integer-valued coordinates and cell entries below 2^20 with small n:
    every exact sum is an integer below 2^24, a float32, so rounding is the
    identity."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        mu = rng.integers(-2 ** 19, 2 ** 19, 3).astype(np.float32)
        M = rng.integers(-2 ** 19, 2 ** 19, (3, 3)).astype(np.float64)
        n = rng.integers(-4, 5, 3)
        want = mu.astype(np.int64) + M.astype(np.int64) @ n
        got = triclinic.image_position(mu, M, n)
        np.testing.assert_array_equal(got.astype(np.int64), want)


def test_round_f32_is_nearest_with_ties_to_even():
    """round_f32 against its definition on rationals: no float32 neighbour
    of the result is nearer, and at a tie the result's significand is even."""
    from fractions import Fraction
    rng = np.random.default_rng(8)
    for _ in range(300):
        x = Fraction(int(rng.integers(-10 ** 12, 10 ** 12)), int(rng.integers(1, 10 ** 6)))
        r = triclinic.round_f32(x)
        d = abs(Fraction(float(r)) - x)
        for nb in (np.nextafter(r, np.float32(np.inf)), np.nextafter(r, np.float32(-np.inf))):
            dn = abs(Fraction(float(nb)) - x)
            assert d <= dn
            if d == dn:
                assert int(np.float32(r).view(np.uint32)) & 1 == 0
