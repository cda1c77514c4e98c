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


sample_voxels = synth.sample_voxel_indices
