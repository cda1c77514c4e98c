"""Pins of the oracle's sphere cutoff: a single atom against a numpy brute
force over voxel centres, a batch (periodic too) against the superposition
of the separately pinned cube grids restricted to each atom's ball, and the
gradient against finite differences.  Inputs are random, so no voxel sits
on a sphere edge (the edge band is checked to be empty)."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import sphere


@pytest.mark.parametrize("value", ["point", "box"])
def test_single_atom_brute_force(value):
    sig, h, N, o = np.float32(0.5), 0.25, 28, -3.5
    mu = np.array([[0.123, -0.271, 0.0517]])
    g = oracle.grid_fp64(mu, [0], [0, 1], [sig], (N, N, N), h, (o, o, o), value=value,
                         cutoff_shape="sphere")[0, 0]
    cube = oracle.grid_fp64(mu, [0], [0, 1], [sig], (N, N, N), h, (o, o, o), value=value)[0, 0]
    c = o + (np.arange(N) + 0.5) * h
    d2 = ((c[:, None, None] - mu[0, 2]) ** 2 + (c[None, :, None] - mu[0, 1]) ** 2 +
          (c[None, None, :] - mu[0, 0]) ** 2)
    rc = float(np.float32(3.0) * sig)
    inside = d2 <= rc * rc
    assert not sphere.edge_band(mu, [0], [0, 1], [sig], (N, N, N), h, (o, o, o)).any()
    if value == "point":
        want = np.where(inside, np.exp(-d2 / (2.0 * float(sig) ** 2)), 0.0)
        np.testing.assert_allclose(g, want, rtol=1e-14, atol=0)
    np.testing.assert_array_equal(g, np.where(inside, cube, 0.0))
    assert 0.4 < inside.sum() / (cube > 0).sum() < 0.6     # ball / cube = pi / 6


@pytest.mark.parametrize("cell", [None, 8.0])
def test_batch_is_the_ball_restricted_superposition(cell):
    rng = np.random.default_rng(8)
    n = 7
    xyz = rng.uniform(0.2, 7.8, size=(n, 3)).astype(np.float32)
    t = rng.integers(0, 3, n).astype(np.int32)
    sig = [0.4, 0.5, 0.6]
    dims, h, o = (26, 28, 30), 0.3, (0.1, -0.2, 0.05)
    got = oracle.grid_fp64(xyz, t, [0, 3, n], sig, dims, h, o, cell=cell, cutoff_shape="sphere")
    band = sphere.edge_band(xyz, t, [0, 3, n], sig, dims, h, o, cell=cell)
    assert not band.any()
    want = np.zeros_like(got)
    D, H, W = dims
    cz, cy, cx = (np.float32(o[2]) + (np.arange(D) + 0.5) * np.float32(h),
                  np.float32(o[1]) + (np.arange(H) + 0.5) * np.float32(h),
                  np.float32(o[0]) + (np.arange(W) + 0.5) * np.float32(h))
    for m, a in [(0, 0), (0, 1), (0, 2), (1, 3), (1, 4), (1, 5), (1, 6)]:
        single = oracle.grid_fp64(xyz[a:a + 1], t[a:a + 1], [0, 1], sig, dims, h, o, cell=cell,
                                  n_types=3)[0, t[a]]
        d = [cx - xyz[a, 0], cy - xyz[a, 1], cz - xyz[a, 2]]
        if cell is not None:
            d = [v - cell * np.round(v / cell) for v in d]
        d2 = d[2][:, None, None] ** 2 + d[1][None, :, None] ** 2 + d[0][None, None, :] ** 2
        rc = float(np.float32(3.0) * np.float32(sig[t[a]]))
        want[m, t[a]] += np.where(d2 <= rc * rc, single, 0.0)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-300)


def test_sphere_gradient_matches_finite_differences():
    rng = np.random.default_rng(9)
    n = 5
    xyz = rng.uniform(-2, 2, size=(n, 3))
    t = rng.integers(0, 3, n).astype(np.int32)
    sig = [0.4, 0.5, 0.6]
    dims, h, o = (22, 22, 22), 0.4, (-4.4, -4.4, -4.4)
    U = rng.standard_normal((1, 3) + dims)
    g = oracle.grad_fp64(xyz, t, [0, n], sig, dims, h, U, o, cutoff_shape="sphere")
    eps = 1e-6
    fd = np.zeros_like(g)
    for a, q in itertools.product(range(n), range(3)):
        xp, xm = xyz.copy(), xyz.copy()
        xp[a, q] += eps
        xm[a, q] -= eps
        lp = (oracle.grid_fp64(xp, t, [0, n], sig, dims, h, o, cutoff_shape="sphere") * U).sum()
        lm = (oracle.grid_fp64(xm, t, [0, n], sig, dims, h, o, cutoff_shape="sphere") * U).sum()
        fd[a, q] = (lp - lm) / (2 * eps)
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-7
