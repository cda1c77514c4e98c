"""Seeded synthetic inputs for the atoms -> density-grid path.

This module only *draws inputs*: molecules (xyz + element type) packed as a
ragged CSR batch, periodic crystal cells and upstream gradients.  It holds
none of the method's arithmetic (no Gaussians, no windows, no grids), so both
the GPU library and the FP64 oracle can be fed from it without sharing any
code with each other.

Workloads stand in for the paper's datasets (MOSES conformers for the
throughput study and PCQM4Mv2 for training, §VI-D and §VII-A), which are not
available here: the shapes, type mix, box sizes and grid geometries below are
the ones the molecule/crystal benchmark configurations name, drawn from
seeded `numpy.random.Generator(PCG64(seed))` streams.

Conventions (shared with the library's ABI, not arithmetic of the method):
  * coordinates are float32, shape (n_atoms, 3), columns x, y, z in Angstrom;
  * types are int32 element ids 0..C-1 (molecules: H, C, N, O, F);
  * offsets are int32 CSR bounds, shape (n_mol + 1,), offsets[0] == 0;
  * grid dims are (D, H, W) = (z, y, x); origin/spacing are given x, y, z.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence, Tuple

import numpy as np

ELEMENTS = ("H", "C", "N", "O", "F")
# Element mix of the molecule workloads (H, C, N, O, F).
TYPE_P = (0.5, 0.3, 0.1, 0.08, 0.02)
MIN_SEPARATION = 0.9  # Angstrom, molecule workloads only


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def sigma_table(n_types: int, lo: float = 0.4, hi: float = 0.7) -> np.ndarray:
    """Per-type Gaussian width sigma_t (Angstrom, a standard deviation),
    evenly spread over [lo, hi]; float32 as the library consumes it."""
    if n_types == 1:
        return np.array([lo], dtype=np.float32)
    return np.linspace(lo, hi, n_types).astype(np.float32)


@dataclasses.dataclass
class Batch:
    """A ragged batch of structures in CSR form (host numpy arrays)."""
    xyz: np.ndarray       # (n_atoms, 3) float32
    types: np.ndarray     # (n_atoms,) int32
    offsets: np.ndarray   # (n_mol + 1,) int32

    @property
    def n_mol(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_atoms(self) -> int:
        return int(self.xyz.shape[0])

    def counts(self) -> np.ndarray:
        return np.diff(self.offsets)

    def subset(self, idx: Sequence[int]) -> "Batch":
        """Structures idx (in that order) as a new batch."""
        xs, ts, offs = [], [], [0]
        for m in idx:
            a, b = int(self.offsets[m]), int(self.offsets[m + 1])
            xs.append(self.xyz[a:b])
            ts.append(self.types[a:b])
            offs.append(offs[-1] + (b - a))
        xyz = np.concatenate(xs) if xs else np.zeros((0, 3), np.float32)
        types = np.concatenate(ts) if ts else np.zeros((0,), np.int32)
        return Batch(np.ascontiguousarray(xyz, np.float32),
                     np.ascontiguousarray(types, np.int32),
                     np.asarray(offs, np.int32))


def molecule(rng: np.random.Generator, n_atoms: int, box: float,
             min_sep: float = MIN_SEPARATION, p=TYPE_P,
             max_tries: int = 10000) -> Tuple[np.ndarray, np.ndarray]:
    """One molecule: types drawn categorically with probabilities p, positions
    uniform in [-box/2, box/2]^3 by sequential rejection to a minimum pairwise
    separation, then recentred on the bounding-box midpoint."""
    pos = np.zeros((n_atoms, 3), dtype=np.float64)
    half = 0.5 * box
    for i in range(n_atoms):
        for _ in range(max_tries):
            cand = rng.uniform(-half, half, size=3)
            if i == 0 or np.min(np.sum((pos[:i] - cand) ** 2, axis=1)) >= min_sep * min_sep:
                pos[i] = cand
                break
        else:
            raise RuntimeError("rejection sampling did not converge")
    if n_atoms:
        mid = 0.5 * (pos.min(axis=0) + pos.max(axis=0))
        pos -= mid
    types = rng.choice(len(p), size=n_atoms, p=np.asarray(p, dtype=np.float64))
    return pos.astype(np.float32), types.astype(np.int32)


def molecule_batch(seed: int, n_mol: int, n_min: int, n_max: int, box: float,
                   p=TYPE_P, min_sep: float = MIN_SEPARATION) -> Batch:
    """n_mol molecules with atom counts uniform on {n_min..n_max}."""
    rng = rng_for(seed)
    counts = rng.integers(n_min, n_max + 1, size=n_mol)
    xs, ts = [], []
    for n in counts:
        x, t = molecule(rng, int(n), box, min_sep, p)
        xs.append(x)
        ts.append(t)
    offsets = np.zeros(n_mol + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    xyz = np.concatenate(xs) if xs else np.zeros((0, 3), np.float32)
    types = np.concatenate(ts) if ts else np.zeros((0,), np.int32)
    return Batch(np.ascontiguousarray(xyz, np.float32),
                 np.ascontiguousarray(types, np.int32),
                 offsets.astype(np.int32))


def crystal_batch(seed: int, counts: Sequence[int], cell: float,
                  n_types: int) -> Batch:
    """Periodic cubic cells: positions uniform in [0, cell)^3, types uniform
    over n_types.  No minimum separation (20k atoms in a 20 A cell exceeds
    random close packing at 0.9 A)."""
    rng = rng_for(seed)
    xs, ts = [], []
    for n in counts:
        x = rng.uniform(0.0, cell, size=(int(n), 3)).astype(np.float32)
        # float32 rounding can land exactly on `cell`; keep the half-open range
        x[x >= np.float32(cell)] = np.float32(0.0)
        xs.append(x)
        ts.append(rng.integers(0, n_types, size=int(n)).astype(np.int32))
    offsets = np.zeros(len(counts) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(np.asarray(counts, dtype=np.int64))
    return Batch(np.ascontiguousarray(np.concatenate(xs), np.float32),
                 np.ascontiguousarray(np.concatenate(ts), np.int32),
                 offsets.astype(np.int32))


def upstream(seed: int, shape: Sequence[int]) -> np.ndarray:
    """Upstream gradient dL/dG, i.i.d. N(0, 1) per voxel, float32."""
    return rng_for(seed).standard_normal(size=tuple(shape), dtype=np.float32)


def embedding(seed: int, n_types: int, n_channels: int) -> np.ndarray:
    """A dense channel-embedding table of the element types, i.i.d.
    U(0.1, 1) per entry, float32 (n_types x n_channels)."""
    return rng_for(seed).uniform(0.1, 1.0, size=(n_types, n_channels)).astype(np.float32)


def perturbation(seed: int, n_atoms: int, amp: float) -> np.ndarray:
    """Coordinate displacements, i.i.d. uniform in [-amp, amp] A per axis,
    float32 (the starting point of a grid-reversal workload)."""
    return rng_for(seed).uniform(-amp, amp, size=(n_atoms, 3)).astype(np.float32)


@dataclasses.dataclass
class Workload:
    """A named workload: the batch recipe plus the grid geometry."""
    name: str
    seed: int
    n_mol: int
    dims: Tuple[int, int, int]          # (D, H, W) = (z, y, x)
    n_types: int
    spacing: float                      # Angstrom, same on all axes
    origin: Tuple[float, float, float]  # x, y, z lower corner
    cutoff_k: float = 3.0
    kind: str = "molecule"              # "molecule" | "crystal"
    atoms: Tuple[int, int] = (5, 29)    # molecule atom-count range
    box: float = 12.0                   # molecule sampling box edge
    crystal_counts: Optional[Tuple[int, ...]] = None
    cell: Optional[float] = None        # periodic cubic cell edge
    out_dtype: str = "f32"
    upstream_seed: Optional[int] = None

    @property
    def periodic(self) -> bool:
        return self.cell is not None

    def sigma(self) -> np.ndarray:
        return sigma_table(self.n_types)

    def batch(self, n_mol: Optional[int] = None) -> Batch:
        if self.kind == "crystal":
            counts = self.crystal_counts
            if n_mol is not None:
                counts = counts[:n_mol]
            return crystal_batch(self.seed, counts, self.cell, self.n_types)
        n = self.n_mol if n_mol is None else n_mol
        return molecule_batch(self.seed, n, self.atoms[0], self.atoms[1], self.box)

    def grid_shape(self, n_mol: Optional[int] = None) -> Tuple[int, ...]:
        n = self.n_mol if n_mol is None else n_mol
        return (n, self.n_types) + tuple(self.dims)


def sample_voxel_indices(rng: np.random.Generator, batch: Batch, shape, origin, spacing,
                         n_random: int, n_near: int) -> np.ndarray:
    """Voxel sample rows (b, c, z, y, x) for spot checks of a batch of grids
    of `shape` (B, C, D, H, W): n_random uniform voxels plus n_near voxels
    within 3 voxels of randomly chosen atoms, in the atom's channel."""
    B, C, D, H, W = shape
    rnd = np.stack([rng.integers(0, s, n_random) for s in shape], axis=1)
    if batch.n_atoms == 0 or n_near == 0:
        return rnd.astype(np.int64)
    a = rng.integers(0, batch.n_atoms, n_near)
    b = np.searchsorted(batch.offsets, a, side="right") - 1
    o = np.asarray(origin, dtype=np.float64)
    idx = np.floor((batch.xyz[a].astype(np.float64) - o) / spacing).astype(np.int64)
    idx += rng.integers(-3, 4, size=idx.shape)
    near = np.stack([b, batch.types[a], np.clip(idx[:, 2], 0, D - 1),
                     np.clip(idx[:, 1], 0, H - 1), np.clip(idx[:, 0], 0, W - 1)], axis=1)
    return np.concatenate([rnd, near]).astype(np.int64)


def _centered_origin(n: int, h: float) -> Tuple[float, float, float]:
    e = -0.5 * n * h
    return (e, e, e)


WORKLOADS = {
    # single molecule, 20 atoms, 32^3 x 5 ch at 0.5 A
    "single20": Workload("single20", 1, 1, (32, 32, 32), 5, 0.5,
                         _centered_origin(32, 0.5), atoms=(20, 20), box=12.0),
    # 256 molecules of 5..29 atoms, 32^3 x 5 ch, one plain launch each
    "mol256": Workload("mol256", 2, 256, (32, 32, 32), 5, 0.5,
                       _centered_origin(32, 0.5), atoms=(5, 29), box=12.0),
    # headline: 4096 molecules of 5..29 atoms on 32^3 x 5 ch, bf16 batched
    "mol4096": Workload("mol4096", 3, 4096, (32, 32, 32), 5, 0.5,
                        _centered_origin(32, 0.5), atoms=(5, 29), box=12.0,
                        out_dtype="bf16"),
    # ragged 4096 molecules of 5..60 atoms, 16 A box, 48^3 x 5 ch at 0.35 A
    "mol4096x48": Workload("mol4096x48", 4, 4096, (48, 48, 48), 5, 0.35,
                           _centered_origin(48, 0.35), atoms=(5, 60), box=16.0,
                           out_dtype="bf16"),
    # 8 periodic cells of 2000..20000 atoms, 20 A, 8 ch, 128^3 at 0.16 A
    "crystal8": Workload("crystal8", 5, 8, (128, 128, 128), 8, 0.16,
                         (0.0, 0.0, 0.0), kind="crystal",
                         crystal_counts=tuple(int(round(v)) for v in
                                              np.linspace(2000, 20000, 8)),
                         cell=20.0),
    # adjoint: 1024 molecules of 5..29 atoms, 32^3 x 5 ch, N(0,1) upstream
    "adjoint1024": Workload("adjoint1024", 6, 1024, (32, 32, 32), 5, 0.5,
                            _centered_origin(32, 0.5), atoms=(5, 29), box=12.0,
                            upstream_seed=7),
    # grid reversal: 1024 molecules of 5..29 atoms, 32^3 x 5 ch float32
    # targets, coordinates displaced by up to 0.15 A per axis (seed 9)
    "reversal1024": Workload("reversal1024", 8, 1024, (32, 32, 32), 5, 0.5,
                             _centered_origin(32, 0.5), atoms=(5, 29), box=12.0,
                             upstream_seed=9),
}
