"""Grid reversal of §IV, FP64 (test infrastructure, like the rest of oracle/).

Recovers atom coordinates from a grid in the two stages of §IV-A:

  find_peaks     the initial coordinates: every local maximum of each channel
                 above a threshold (§IV-B locates the atoms as the grid's
                 local maxima; the persistent-homology search it uses is
                 replaced by the plain local-maximum test below);
  reversal_step  one gradient step on the coordinates (§IV-A steps 2-4,
                 §IV-C): G' = grid(xyz), L_b = sum over structure b of
                 (G' - T)^2, dL/dG' = 2 (G' - T), the coordinate gradient of
                 that upstream, and xyz - lr * gradient.

Local maximum (the reading used on both sides).  Voxel v of channel c is a
peak when T[v] > threshold and, for each of its 26 neighbours u inside the
grid (same channel, no wrap), T[v] > T[u] when u comes before v in raster
order (z, then y, then x) and T[v] >= T[u] when u comes after v.  On a
plateau of equal maxima only the first voxel in raster order is a peak.
Comparisons are made in the precision of the array passed in, so the same
float32 grid gives the same peaks on both sides.

Peaks of a structure come out in raster order (channel, z, y, x); the
position is the exact voxel centre o + (i + 1/2) h (o, h float32) rounded
once to float32, to nearest with ties to even, and the type is the channel.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np

from . import grad_fp64, grid_fp64

# the 26 neighbour offsets (dz, dy, dx) and whether each comes earlier in
# raster order than the centre
_NEIGHBOURS = [(d, d < (0, 0, 0)) for d in itertools.product((-1, 0, 1), repeat=3)
               if d != (0, 0, 0)]


def peak_mask(grid: np.ndarray, threshold: float) -> np.ndarray:
    """Boolean mask of the local maxima of a (..., D, H, W) array."""
    g = np.asarray(grid)
    D, H, W = g.shape[-3:]
    lead = g.shape[:-3]
    pad = np.full(lead + (D + 2, H + 2, W + 2), -np.inf, dtype=g.dtype)
    pad[..., 1:-1, 1:-1, 1:-1] = g
    mask = g > g.dtype.type(threshold)
    for (dz, dy, dx), earlier in _NEIGHBOURS:
        nb = pad[..., 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
        mask &= (g > nb) if earlier else (g >= nb)
    return mask


def round_f32(x: Fraction) -> np.float32:
    """The float32 nearest to the rational x (ties to the even significand)."""
    c = np.float32(float(x))
    cands = [np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))]
    best = None
    for v in cands:
        if not np.isfinite(v):
            continue
        d = abs(Fraction(float(v)) - x)
        even = (int(np.asarray(v).view(np.uint32)) & 1) == 0
        if best is None or d < best[0] or (d == best[0] and even):
            best = (d, v)
    return np.float32(best[1])


def voxel_centres_f32(o: np.ndarray, idx: np.ndarray, h: np.ndarray) -> np.ndarray:
    """o + (idx + 1/2) h rounded once to float32, for float32 o, h (per
    column) and integer idx: in double where both operations are exact (the
    product always is for idx < 2^28; the sum is checked with TwoSum), else
    in rationals."""
    o64 = np.broadcast_to(np.asarray(o, np.float32).astype(np.float64), idx.shape)
    h64 = np.broadcast_to(np.asarray(h, np.float32).astype(np.float64), idx.shape)
    p = (idx.astype(np.float64) + 0.5) * h64
    s = o64 + p
    bb = s - o64
    err = (o64 - (s - bb)) + (p - bb)
    out = s.astype(np.float32)
    for k in zip(*np.nonzero(err != 0.0)):
        exact = Fraction(float(o64[k])) + (Fraction(int(idx[k])) + Fraction(1, 2)) * \
            Fraction(float(h64[k]))
        out[k] = round_f32(exact)
    return out


def find_peaks(grid, threshold, origin, spacing, origins=None, spacings=None):
    """Peaks of a batch of grids (B, C, D, H, W) -> (xyz float32 (n, 3),
    types int32 (n,), offsets int64 (B + 1,))."""
    g = np.asarray(grid)
    assert g.ndim == 5
    B = g.shape[0]
    m = peak_mask(g, threshold)
    xyz, types, offsets = [], [], [0]
    o32 = np.asarray(np.broadcast_to(np.asarray(origin, np.float32), (3,)), np.float32)
    h32 = np.asarray(np.broadcast_to(np.asarray(spacing, np.float32), (3,)), np.float32)
    for b in range(B):
        c, z, y, x = np.nonzero(m[b])          # row-major order = raster order
        o = o32 if origins is None else np.asarray(origins, np.float32)[b]
        h = h32 if spacings is None else np.asarray(spacings, np.float32)[b]
        idx = np.stack([x, y, z], axis=1).astype(np.int64)
        xyz.append(voxel_centres_f32(o, idx, h))
        types.append(c.astype(np.int32))
        offsets.append(offsets[-1] + len(c))
    return (np.concatenate(xyz).reshape(-1, 3) if xyz else np.zeros((0, 3), np.float32),
            np.concatenate(types) if types else np.zeros(0, np.int32),
            np.asarray(offsets, np.int64))


def reversal_loss(xyz, types, offsets, sigma, dims, spacing, target, origin=None, **kw):
    """Per-structure L_b = sum (G'(xyz) - T)^2 and the residual G' - T."""
    gp = grid_fp64(xyz, types, offsets, sigma, dims, spacing, origin, **kw)
    r = gp - np.asarray(target, np.float64).reshape(gp.shape)
    return (r * r).reshape(r.shape[0], -1).sum(axis=1), r


def reversal_step(xyz, types, offsets, sigma, dims, spacing, target, lr, origin=None, **kw):
    """One coordinate step of §IV-A: returns (loss (B,), residual 2 (G' - T),
    gradient (n, 3), updated xyz (n, 3) float64)."""
    loss, r = reversal_loss(xyz, types, offsets, sigma, dims, spacing, target, origin, **kw)
    U = 2.0 * r
    grad = grad_fp64(xyz, types, offsets, sigma, dims, spacing, U, origin, **kw)
    return loss, U, grad, np.asarray(xyz, np.float64) - lr * grad
