"""Shared helpers of the GPU parity tests (imported only by tests)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def say(*a):
    print(*a, flush=True)


def to_device(batch: "synth.Batch", dev):
    import torch
    return (torch.tensor(batch.xyz, device=dev), torch.tensor(batch.types, device=dev),
            torch.tensor(batch.offsets, device=dev))


def errors(got: np.ndarray, ref: np.ndarray):
    """(rel-L2, max-abs) of got against ref (float64)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    rel = np.linalg.norm(got - ref) / den if den > 0 else np.linalg.norm(got - ref)
    return float(rel), float(np.max(np.abs(got - ref))) if got.size else 0.0


def worst_molecule(got: np.ndarray, ref: np.ndarray):
    """Largest per-structure rel-L2 over the batch axis."""
    w = 0.0
    for m in range(ref.shape[0]):
        r, _ = errors(got[m], ref[m])
        w = max(w, r)
    return w


def sample_voxels(rng, batch, shape, wl_origin, spacing, n_random, n_near):
    """Sample (b, c, z, y, x) rows: uniform random voxels plus voxels next to
    atoms (where values are non-zero)."""
    B, C, D, H, W = shape
    rnd = np.stack([rng.integers(0, s, n_random) for s in shape], axis=1)
    a = rng.integers(0, batch.n_atoms, n_near)
    b = np.searchsorted(batch.offsets, a, side="right") - 1
    o = np.asarray(wl_origin)
    idx = np.floor((batch.xyz[a].astype(np.float64) - o) / spacing).astype(np.int64)
    idx += rng.integers(-3, 4, size=idx.shape)
    near = np.stack([b, batch.types[a], np.clip(idx[:, 2], 0, D - 1),
                     np.clip(idx[:, 1], 0, H - 1), np.clip(idx[:, 0], 0, W - 1)], axis=1)
    return np.concatenate([rnd, near]).astype(np.int64)
