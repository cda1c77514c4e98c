"""Pins of the oracle's grid reversal (§IV): the local-maximum peak finder
against an independent pure-Python brute force and against grids whose
maxima are known, the exact rounding of peak positions, and the reversal
step against the facts the method fixes -- zero loss and zero gradient at
the generating coordinates, the loss gradient against finite differences
(the factor 2 and the sign of the residual), and gradient descent from the
peaks recovering the generating coordinates (§IV-A) for both voxel values.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import reversal


def brute_peaks(g, thr):
    """Independent statement of the rule: loops over voxels and neighbours,
    raster order compared as index tuples."""
    B, C, D, H, W = g.shape
    out = np.zeros(g.shape, bool)
    for b, c, z, y, x in itertools.product(range(B), range(C), range(D), range(H), range(W)):
        v = g[b, c, z, y, x]
        if not v > thr:
            continue
        ok = True
        for zz in range(max(0, z - 1), min(D, z + 2)):
            for yy in range(max(0, y - 1), min(H, y + 2)):
                for xx in range(max(0, x - 1), min(W, x + 2)):
                    if (zz, yy, xx) == (z, y, x):
                        continue
                    u = g[b, c, zz, yy, xx]
                    if (zz, yy, xx) < (z, y, x):
                        ok = ok and v > u
                    else:
                        ok = ok and v >= u
        out[b, c, z, y, x] = ok
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_peaks_match_brute_force_with_plateaus(seed):
    rng = np.random.default_rng(seed)
    g = rng.integers(0, 4, size=(2, 2, 4, 5, 6)).astype(np.float32)   # many ties
    np.testing.assert_array_equal(reversal.peak_mask(g, 0.5), brute_peaks(g, 0.5))
    g = rng.standard_normal((1, 3, 5, 4, 7)).astype(np.float32)
    np.testing.assert_array_equal(reversal.peak_mask(g, -0.3), brute_peaks(g, -0.3))


def test_plateau_keeps_only_its_first_voxel():
    g = np.zeros((1, 1, 3, 3, 3), np.float32)
    g[0, 0, 1, 1, 1] = g[0, 0, 1, 1, 2] = 2.0
    m = reversal.peak_mask(g, 0.0)
    assert m.sum() == 1 and m[0, 0, 1, 1, 1]
    g[:] = 1.0
    m = reversal.peak_mask(g, 0.5)
    assert m.sum() == 1 and m[0, 0, 0, 0, 0]
    assert reversal.peak_mask(g, 1.0).sum() == 0          # strictly above threshold


def test_isolated_atoms_at_voxel_centres_are_the_peaks():
    """Atoms at voxel centres, far apart or in different channels: the peaks
    are exactly the atoms, positions bit-equal, in raster order."""
    h, o = 0.5, -8.0
    xyz = np.array([[-4.25, 2.75, 0.25], [3.25, -3.75, -5.25], [0.75, 0.75, 0.75],
                    [1.25, 0.75, 0.75]], np.float32)
    types = np.array([1, 1, 0, 2], np.int32)
    sig = [0.4, 0.5, 0.6]
    g = oracle.grid_fp64(xyz, types, [0, 2, 4], sig, (32, 32, 32), h, (o, o, o))
    p_xyz, p_t, p_off = reversal.find_peaks(g.astype(np.float32), 1e-3, (o, o, o), h)
    np.testing.assert_array_equal(p_off, [0, 2, 4])
    # structure 0: both type 1, raster order puts smaller z first
    np.testing.assert_array_equal(p_xyz[:2], xyz[[1, 0]])
    np.testing.assert_array_equal(p_t[:2], [1, 1])
    np.testing.assert_array_equal(p_xyz[2:], xyz[[2, 3]])
    np.testing.assert_array_equal(p_t[2:], [0, 2])


def nearest_f32(x: Fraction) -> np.float32:
    """Nearest float32 to x by bisection over the float32 bit patterns of
    its sign (ties to even): an independent rounding for the pins."""
    if x == 0:
        return np.float32(0.0)
    neg = x < 0
    a = -x if neg else x
    lo, hi = 0, 0x7F7FFFFF                  # non-negative finite float32 patterns
    while hi - lo > 1:                      # largest pattern whose value <= a
        mid = (lo + hi) // 2
        if Fraction(float(np.uint32(mid).view(np.float32))) <= a:
            lo = mid
        else:
            hi = mid
    v_lo = Fraction(float(np.uint32(lo).view(np.float32)))
    v_hi = Fraction(float(np.uint32(lo + 1).view(np.float32)))
    pick = lo if (a - v_lo < v_hi - a or (a - v_lo == v_hi - a and lo % 2 == 0)) else lo + 1
    v = np.uint32(pick).view(np.float32)
    return np.float32(-v if neg else v)


def test_peak_centre_rounded_once_where_double_would_round_twice():
    """o = 1, h = 16773121 * 2^-59, voxel 2048: the exact centre is
    1 + 2^-24 + 2^-60, just above the float32 midpoint 1 + 2^-24.  A double
    evaluation rounds it to the midpoint and then to 1.0 (ties to even); the
    single rounding gives 1 + 2^-23."""
    h = np.float32(16773121 * 2.0 ** -59)
    assert Fraction(float(h)) == Fraction(16773121, 2 ** 59)
    g = np.zeros((1, 1, 1, 1, 2049), np.float32)
    g[0, 0, 0, 0, 2048] = 1.0
    p_xyz, _, _ = reversal.find_peaks(g, 0.5, (1.0, 0.0, 0.0), (h, 1.0, 1.0))
    assert p_xyz.shape == (1, 3)
    assert p_xyz[0, 0] == np.float32(1.0 + 2.0 ** -23)
    assert np.float32(1.0 + (2048.5 * float(h))) == np.float32(1.0)   # the double route
    exact = Fraction(1) + Fraction(4097, 2) * Fraction(float(h))
    assert p_xyz[0, 0] == nearest_f32(exact)


def test_peak_positions_are_rounded_once_from_the_exact_centre():
    o = np.array([-7.3, 1.9, -0.11], np.float32)
    h = np.array([0.37, 0.29, 0.53], np.float32)
    g = np.zeros((1, 1, 6, 7, 9), np.float32)
    spots = [(0, 0, 0), (5, 6, 8), (2, 3, 4)]
    for z, y, x in spots:
        g[0, 0, z, y, x] = 1.0
    p_xyz, _, _ = reversal.find_peaks(g, 0.5, o, h)
    for (z, y, x), got in zip(sorted(spots), p_xyz):
        for q, i in enumerate((x, y, z)):
            exact = Fraction(float(o[q])) + (Fraction(i) + Fraction(1, 2)) * Fraction(float(h[q]))
            assert got[q] == nearest_f32(exact), (q, i)


def small_case(value="point"):
    h, o = 0.5, (-6.0, -6.0, -6.0)
    true = np.array([[-2.13, 1.07, 0.31], [2.41, -1.86, 1.53], [0.22, 2.94, -2.47]], np.float32)
    types = np.array([0, 1, 2], np.int32)
    sig = [0.5, 0.5, 0.5] if value == "box" else [0.4, 0.55, 0.7]
    return h, o, true, types, sig


@pytest.mark.parametrize("value", ["point", "box"])
def test_loss_and_gradient_vanish_at_the_generating_coordinates(value):
    h, o, true, types, sig = small_case(value)
    T = oracle.grid_fp64(true, types, [0, 3], sig, (24, 24, 24), h, o, value=value)
    loss, U, grad, new = reversal.reversal_step(true, types, [0, 3], sig, (24, 24, 24), h, T,
                                                0.1, o, value=value)
    assert loss[0] == 0.0 and not U.any() and not grad.any()
    np.testing.assert_array_equal(new, true.astype(np.float64))


@pytest.mark.parametrize("value", ["point", "box"])
def test_loss_gradient_matches_finite_differences(value):
    h, o, true, types, sig = small_case(value)
    dims = (24, 24, 24)
    T = oracle.grid_fp64(true, types, [0, 3], sig, dims, h, o, value=value)
    x0 = true.astype(np.float64) + np.array([[0.11, -0.07, 0.05], [-0.04, 0.09, 0.02],
                                             [0.06, 0.03, -0.12]])
    _, _, grad, _ = reversal.reversal_step(x0, types, [0, 3], sig, dims, h, T, 0.0, o,
                                           value=value)
    eps = 1e-6
    fd = np.zeros_like(grad)
    for a in range(3):
        for q in range(3):
            xp, xm = x0.copy(), x0.copy()
            xp[a, q] += eps
            xm[a, q] -= eps
            lp, _ = reversal.reversal_loss(xp, types, [0, 3], sig, dims, h, T, o, value=value)
            lm, _ = reversal.reversal_loss(xm, types, [0, 3], sig, dims, h, T, o, value=value)
            fd[a, q] = (lp[0] - lm[0]) / (2 * eps)
    assert np.linalg.norm(grad - fd) / np.linalg.norm(fd) < 1e-6


@pytest.mark.parametrize("value,lr", [("point", 0.02), ("box", 5.0)])
def test_descent_from_the_peaks_recovers_the_coordinates(value, lr):
    """§IV-A: peaks of the target grid, then gradient steps, converge to the
    coordinates that generated it; the loss never rises."""
    h, o, true, types, sig = small_case(value)
    dims = (24, 24, 24)
    T = oracle.grid_fp64(true, types, [0, 3], sig, dims, h, o, value=value)
    x, t, off = reversal.find_peaks(T, 1e-4 if value == "box" else 0.05, o, h)
    np.testing.assert_array_equal(off, [0, 3])
    np.testing.assert_array_equal(t, types)
    assert np.max(np.abs(x - true)) <= h / 2 + 1e-6        # the voxel of each atom
    x = x.astype(np.float64)
    last = np.inf
    for _ in range(80):
        loss, _, _, x = reversal.reversal_step(x, t, off, sig, dims, h, T, lr, o, value=value)
        assert loss[0] <= last * (1 + 1e-12)
        last = loss[0]
    assert np.max(np.abs(x - true)) < 1e-6
