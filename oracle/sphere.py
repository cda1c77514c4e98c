"""Sphere cutoff helpers (test infrastructure, like the rest of oracle/).

With cutoff_shape="sphere" an atom's voxel is kept when the squared
distance to the voxel centre (nearest image per axis when periodic) is at
most rc_t^2.  Unlike the cube's per-axis edges this decision is not made
exactly on either side: the oracle sums the squares in double, the GPU in
float32.  edge_band() marks the voxels where some atom of the voxel's
channel lies within a relative `eps` of its sphere, the voxels a comparison
accepts on either side.
"""
from __future__ import annotations

import numpy as np


def edge_band(xyz, types, offsets, sigma, dims, spacing, origin, cutoff_k=3.0, cell=None,
              eps=1e-6, n_channels=None):
    """Boolean (B, C, D, H, W) mask of the voxels near a sphere edge."""
    xyz = np.asarray(xyz, np.float64).reshape(-1, 3)
    sig = np.asarray(sigma, np.float32)
    C = int(n_channels or len(sig))
    D, H, W = dims
    B = len(offsets) - 1
    h = np.broadcast_to(np.asarray(spacing, np.float32).astype(np.float64), (3,))
    o = np.broadcast_to(np.asarray(origin, np.float32).astype(np.float64), (3,))
    L = None if cell is None else np.broadcast_to(
        np.asarray(cell, np.float32).astype(np.float64), (3,))
    centres = [o[q] + (np.arange(n) + 0.5) * h[q] for q, n in enumerate((W, H, D))]
    mask = np.zeros((B, C, D, H, W), bool)
    for b in range(B):
        for a in range(int(offsets[b]), int(offsets[b + 1])):
            t = int(types[a])
            rc = float(np.float32(cutoff_k) * sig[t])
            d2 = []
            for q in range(3):
                d = centres[q] - xyz[a, q]
                if L is not None:
                    d = d - L[q] * np.round(d / L[q])
                d2.append(d * d)
            r2 = d2[2][:, None, None] + d2[1][None, :, None] + d2[0][None, None, :]
            mask[b, t] |= np.abs(r2 - rc * rc) <= eps * rc * rc
    return mask
