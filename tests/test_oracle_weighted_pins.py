"""Pins of the oracle's weighted channels (each atom adds weights[a, c] times
its Gaussian to every channel c; the learned-embedding grids proposed in the
paper's Discussion, the weighted grids mentioned after §III-A Eq. 6).

Checked against things other than the weighted code path: one-hot weights
against the (separately pinned) unweighted grid, bit for bit; superposition
of single-atom unweighted grids combined with the weights by numpy; the box
form's channel sums (Eq. 6 with weights); finite differences of the loss in
the coordinates; and the exact linearity of the loss in the weights.
"""
import numpy as np
import pytest

import oracle
import synth


def one_hot(types, C):
    E = np.zeros((len(types), C))
    E[np.arange(len(types)), types] = 1.0
    return E


def single_atom_grids(b, sig, dims, h, o, value="point", cell=None, n_channels=None):
    """Per atom, its unweighted grid alone, taken from its own channel."""
    C = n_channels or len(sig)
    out = []
    for a in range(b.n_atoms):
        g = oracle.grid_fp64(b.xyz[a:a + 1], b.types[a:a + 1], [0, 1], sig, dims, h, o,
                             cell=cell, value=value, n_types=C)
        out.append(g[0, b.types[a]])
    return np.stack(out)


@pytest.mark.parametrize("value,cell", [("point", None), ("box", None), ("point", 8.0)])
def test_one_hot_weights_reproduce_the_unweighted_grid(value, cell):
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(6)
    sig = wl.sigma()
    dims, h = (24, 24, 24), 0.5
    o = (-6.0, -6.0, -6.0) if cell is None else (0.0, 0.0, 0.0)
    xyz = b.xyz if cell is None else np.mod(b.xyz, 8.0)
    plain = oracle.grid_fp64(xyz, b.types, b.offsets, sig, dims, h, o, cell=cell, value=value)
    w = oracle.grid_fp64(xyz, b.types, b.offsets, sig, dims, h, o, cell=cell, value=value,
                         weights=one_hot(b.types, len(sig)))
    np.testing.assert_array_equal(w, plain)


@pytest.mark.parametrize("value", ["point", "box"])
def test_weighted_grid_is_the_superposition_of_single_atom_grids(value):
    """More types (8 widths) than channels (3), dense signed weights."""
    rng = np.random.default_rng(4)
    n = 9
    xyz = rng.uniform(-3, 3, size=(n, 3)).astype(np.float32)
    types = rng.integers(0, 8, n).astype(np.int32)
    sig = synth.sigma_table(8, 0.35, 0.7)
    E = rng.standard_normal((n, 3))
    dims, h, o = (20, 20, 20), 0.5, (-5.0, -5.0, -5.0)
    b = synth.Batch(xyz, types, np.array([0, 4, n], np.int32))
    got = oracle.grid_fp64(xyz, types, b.offsets, sig, dims, h, o, value=value, weights=E)
    singles = single_atom_grids(b, sig, dims, h, o, value, n_channels=8)
    for m in range(2):
        a0, a1 = b.offsets[m], b.offsets[m + 1]
        want = np.einsum("ac,azyx->czyx", E[a0:a1], singles[a0:a1])
        np.testing.assert_allclose(got[m], want, rtol=1e-13, atol=1e-14)
    # the sampled-voxel entry point agrees with the dense grid
    idx = np.stack([rng.integers(0, s, 300) for s in (2, 3) + dims], axis=1)
    v = oracle.voxels_fp64(xyz, types, b.offsets, sig, dims, h, idx, o, value=value, weights=E)
    np.testing.assert_allclose(v, got[tuple(idx.T)], rtol=1e-13, atol=1e-14)


def test_box_channel_sums_are_the_weight_sums():
    """Eq. 6 with weights: without a cutoff each channel sums to the sum of
    its weights over the atoms."""
    wl = synth.WORKLOADS["single20"]
    b = wl.batch()
    E = np.random.default_rng(2).uniform(-1, 2, size=(b.n_atoms, 4))
    g = oracle.grid_fp64(b.xyz, b.types, b.offsets, wl.sigma(), (48, 48, 48), 0.5,
                         (-12, -12, -12), cutoff_k=0.0, value="box", weights=E)
    np.testing.assert_allclose(g[0].sum(axis=(1, 2, 3)), E.sum(axis=0), rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("value", ["point", "box"])
def test_weighted_gradients(value):
    rng = np.random.default_rng(6)
    n = 6
    xyz = rng.uniform(-2.5, 2.5, size=(n, 3))
    types = rng.integers(0, 5, n).astype(np.int32)
    sig = synth.sigma_table(5)
    E = rng.standard_normal((n, 3))
    dims, h, o = (20, 20, 20), 0.5, (-5.0, -5.0, -5.0)
    off = [0, n]
    U = rng.standard_normal((1, 3) + dims)
    gx, gw = oracle.grad_fp64(xyz, types, off, sig, dims, h, U, o, cutoff_k=0.0, value=value,
                              weights=E, return_weight_grad=True)

    def L(x, e):
        return (oracle.grid_fp64(x, types, off, sig, dims, h, o, cutoff_k=0.0, value=value,
                                 weights=e) * U).sum()

    eps = 1e-6
    fd = np.zeros_like(gx)
    for a in range(n):
        for q in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[a, q] += eps
            xm[a, q] -= eps
            fd[a, q] = (L(xp, E) - L(xm, E)) / (2 * eps)
    assert np.linalg.norm(gx - fd) / np.linalg.norm(fd) < 1e-7
    # the loss is linear in the weights: unit steps give the gradient exactly
    base = L(xyz, E)
    for a in range(n):
        for c in range(3):
            e = E.copy()
            e[a, c] += 1.0
            assert L(xyz, e) - base == pytest.approx(gw[a, c], rel=1e-9, abs=1e-12)


def test_weighted_atoms_with_types_past_the_table_are_skipped():
    xyz = np.array([[0.1, 0.2, 0.3], [1.0, 1.0, 1.0]], np.float32)
    sig = [0.4, 0.5]
    E = np.ones((2, 3))
    dims, h, o = (12, 12, 12), 0.5, (-3.0, -3.0, -3.0)
    g, st = oracle.grid_fp64(xyz, [1, 2], [0, 2], sig, dims, h, o, weights=E,
                             return_stats=True)
    ref = oracle.grid_fp64(xyz[:1], [1], [0, 1], sig, dims, h, o, weights=E[:1])
    assert st["skipped"] == 1
    np.testing.assert_array_equal(g, ref)
