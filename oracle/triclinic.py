"""Triclinic periodic cells, FP64 (test infrastructure, like the rest of oracle/).

§III-A makes a periodic structure's density the sum over lattice
translations T(mu) of each atom.  For a general (triclinic) cell with
matrix M -- column j is lattice vector j in x, y, z -- the reading used on
both sides is:

  * every atom contributes, through each lattice image mu + M n (n integer),
    that image's Gaussian truncated to its own cutoff cube;
  * the cell must keep the cubes of distinct images of one atom apart,
    max_alpha |(M n)_alpha| > 2 rc for every n != 0 (check_cell), so each
    voxel sees at most one image of each atom (for an orthorhombic cell this
    is the nearest-image map of the orthorhombic path);
  * an image's position is the exact real sum mu_alpha + n0 M[alpha,0] +
    n1 M[alpha,1] + n2 M[alpha,2] of the float32 inputs, rounded once to
    the nearest float32 (ties to even); its cutoff windows are then decided
    exactly on that float32 position, as for any non-periodic atom.

The functions expand every atom into the images that can reach the grid
(a generous range, found per atom from its fractional coordinates) and pass
them to the non-periodic oracle; coordinate gradients of the images are
summed back onto their atom.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np

from . import grad_fp64, grid_fp64


def _cell(M) -> np.ndarray:
    """The cell matrix as float32 values in float64."""
    return np.asarray(M, np.float64).reshape(3, 3).astype(np.float32).astype(np.float64)


def round_f32(x: Fraction) -> np.float32:
    """The float32 nearest to the rational x, ties to the even significand."""
    c = np.float32(float(x))          # within one float32 step of the answer
    best = None
    for cand in (np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))):
        key = (abs(Fraction(float(cand)) - x), int(np.float32(cand).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, cand)
    return np.float32(best[1])


def image_position(mu, M, n) -> np.ndarray:
    """fl32(mu + M n): the exact lattice sum, rounded once to float32."""
    M = _cell(M)
    mu = np.asarray(mu, np.float32)
    out = np.empty(3, np.float32)
    for a in range(3):
        x = Fraction(float(mu[a]))
        for j in range(3):
            x += int(n[j]) * Fraction(float(M[a, j]))
        out[a] = round_f32(x)
    return out


def check_cell(M, rc_max: float, reach: int = 3) -> bool:
    """True when the cutoff cubes of distinct images never overlap."""
    M = _cell(M)
    for n in itertools.product(range(-reach, reach + 1), repeat=3):
        if n == (0, 0, 0):
            continue
        if np.max(np.abs(M @ np.asarray(n, np.float64))) <= 2.0 * rc_max:
            return False
    return True


def expand(xyz, types, offsets, M, dims, spacing, origin, rc_max):
    """Images of every atom that can reach the grid box widened by rc_max:
    (xyz float32 (m, 3), types (m,), offsets (B + 1,), source atom (m,))."""
    M = _cell(M)
    Minv = np.linalg.inv(M)
    D, H, W = dims
    h = np.broadcast_to(np.asarray(spacing, np.float64), (3,))
    o = np.broadcast_to(np.asarray(origin, np.float64), (3,))
    lo = o - rc_max - 1e-3
    hi = o + np.array([W, H, D]) * h + rc_max + 1e-3
    corners = np.array([[lo[0] if i == 0 else hi[0], lo[1] if j == 0 else hi[1],
                         lo[2] if k == 0 else hi[2]] for i in (0, 1) for j in (0, 1)
                        for k in (0, 1)])
    cf = corners @ Minv.T                  # fractional coordinates of the box corners
    fmin, fmax = cf.min(axis=0), cf.max(axis=0)
    xyz = np.asarray(xyz, np.float64)
    out_x, out_t, out_s, offs = [], [], [], [0]
    for m in range(len(offsets) - 1):
        for a in range(int(offsets[m]), int(offsets[m + 1])):
            f = Minv @ xyz[a]
            rng = [range(int(np.floor(fmin[j] - f[j])) - 1, int(np.ceil(fmax[j] - f[j])) + 2)
                   for j in range(3)]
            for n in itertools.product(*rng):
                p = image_position(xyz[a], M, n)
                if np.all(p >= lo) and np.all(p <= hi):
                    out_x.append(p)
                    out_t.append(types[a])
                    out_s.append(a)
        offs.append(len(out_s))
    return (np.asarray(out_x, np.float32).reshape(-1, 3), np.asarray(out_t, np.int32),
            np.asarray(offs, np.int64), np.asarray(out_s, np.int64))


def grid_triclinic_fp64(xyz, types, offsets, sigma, dims, spacing, M, origin, cutoff_k=3.0,
                        value="point", cutoff_shape="cube"):
    """Dense FP64 grids (B, C, D, H, W) of a batch of triclinic cells."""
    sig = np.asarray(sigma, np.float32)
    rc_max = float(np.max(np.float32(cutoff_k) * sig))
    assert check_cell(M, rc_max), "image cutoff cubes overlap"
    xi, ti, oi, _ = expand(xyz, types, offsets, M, dims, spacing, origin, rc_max)
    return grid_fp64(xi, ti, oi, sigma, dims, spacing, origin, cutoff_k=cutoff_k, value=value,
                     cutoff_shape=cutoff_shape)


def grad_triclinic_fp64(xyz, types, offsets, sigma, dims, spacing, U, M, origin, cutoff_k=3.0,
                        value="point", cutoff_shape="cube"):
    """dL/dxyz (n_atoms, 3) for L = sum(U * G) over triclinic cells: each
    image is a translate of its atom, so the image gradients add up."""
    sig = np.asarray(sigma, np.float32)
    rc_max = float(np.max(np.float32(cutoff_k) * sig))
    xi, ti, oi, src = expand(xyz, types, offsets, M, dims, spacing, origin, rc_max)
    gi = grad_fp64(xi, ti, oi, sigma, dims, spacing, U, origin, cutoff_k=cutoff_k, value=value,
                   cutoff_shape=cutoff_shape)
    g = np.zeros((np.asarray(xyz).reshape(-1, 3).shape[0], 3))
    np.add.at(g, src, gi)
    return g
