"""All-voxels x all-atoms brute force for tiny grids (test infrastructure).

Independent of `pg_oracle.c`: the cutoff decision |r_i - mu| <= rc is taken
in exact rational arithmetic (`fractions.Fraction` of the binary inputs, so
no rounding at all), the nearest periodic image is chosen by exact rational
comparison over a range of lattice translations (§III-A: minimum over
translations), and every (voxel, atom) pair is visited with no window
bookkeeping.  Values are FP64 exponentials of the summed squared offsets
(§III-A, Eq. 1 without its normalising prefactor).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _rc(k: float, sigma: float) -> Fraction:
    # single-precision product of the two float inputs (numpy float32 * float32)
    return Fraction(float(np.float32(k) * np.float32(sigma)))


def _axis(o, h, n_vox, mu, cut, rc, cell):
    """For one atom and axis: list of (inside, offset as Fraction)."""
    o, h, mu = Fraction(o), Fraction(h), Fraction(mu)
    res = []
    for i in range(n_vox):
        r = o + (Fraction(2 * i + 1, 2)) * h
        d = r - mu
        if cell is not None:
            L = Fraction(cell)
            # nearest image: the translation n minimising |d - n L|
            n0 = int(np.floor(float(d / L)))
            best = min((abs(d - n * L), n) for n in range(n0 - 2, n0 + 3))
            d = d - best[1] * L
        inside = (not cut) or abs(d) <= rc
        res.append((inside, d))
    return res


def brute_fp64(xyz, types, offsets, sigma, dims, spacing, origin, cutoff_k=3.0,
               cell=None, n_types=None):
    """Dense FP64 grid (B, C, D, H, W) by visiting every voxel for every atom."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    types = np.asarray(types).reshape(-1)
    offsets = np.asarray(offsets).reshape(-1)
    sigma = np.asarray(sigma, dtype=np.float32).reshape(-1)
    C = int(n_types if n_types is not None else sigma.shape[0])
    D, H, W = (int(d) for d in dims)
    # grid geometry is single precision (rounded once), coordinates as given
    sp = np.broadcast_to(np.asarray(spacing, dtype=np.float32).astype(np.float64), (3,))
    og = np.broadcast_to(np.asarray(origin, dtype=np.float32).astype(np.float64), (3,))
    cl = None if cell is None else np.broadcast_to(
        np.asarray(cell, dtype=np.float32).astype(np.float64), (3,))
    B = offsets.shape[0] - 1
    out = np.zeros((B, C, D, H, W), dtype=np.float64)
    cut = float(np.float32(cutoff_k)) != 0.0
    N = (W, H, D)
    for b in range(B):
        for a in range(int(offsets[b]), int(offsets[b + 1])):
            t = int(types[a])
            if t < 0 or t >= C or not np.all(np.isfinite(xyz[a])):
                continue
            rc = _rc(cutoff_k, sigma[t])
            ax = [_axis(og[q], sp[q], N[q], xyz[a, q], cut,
                        rc, None if cl is None else cl[q]) for q in range(3)]
            s2 = float(sigma[t]) ** 2
            for z in range(D):
                for y in range(H):
                    for x in range(W):
                        ix, iy, iz = ax[0][x], ax[1][y], ax[2][z]
                        if ix[0] and iy[0] and iz[0]:
                            d2 = float(ix[1]) ** 2 + float(iy[1]) ** 2 + float(iz[1]) ** 2
                            out[b, t, z, y, x] += np.exp(-d2 / (2.0 * s2))
    return out
