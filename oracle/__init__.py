"""FP64 CPU oracle of the atoms -> density-grid map (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library (the C source is
`pg_oracle.c`, built by `oracle/build.py` with gcc) and never imports it.

Functions:
  grid_fp64   dense B x C x D x H x W float64 grids (pg_oracle.c)
  grad_fp64   coordinate gradient of sum(U * G) (pg_oracle.c)
  voxels_fp64 individual voxels by visiting every atom (pg_oracle.c)
  count_evals number of atom-voxel pairs inside the cutoff windows
  brute_fp64  all-voxels x all-atoms NumPy form with exact rational edge
              decisions, for tiny grids (brute.py)
  reversal    grid reversal of §IV: local-maximum peaks and the coordinate
              descent step on the squared grid error (reversal.py)
  triclinic   triclinic periodic cells: lattice images passed to the
              non-periodic map (triclinic.py)
  sphere      the voxels near a sphere-cutoff edge, which comparisons accept
              on either side (sphere.py)

cutoff_shape="sphere" keeps, inside each atom's cube, only the voxels with
|r - mu|^2 <= rc_t^2 (squares summed in double).

What is computed is the point-sampled, un-normalised Gaussian of §III-A
Eq. 1 at voxel centres (value="point"), or the integral of the normalised
Gaussian over each voxel box, a product of per-axis erf differences (§III-A
Eq. 2-5; value="box"), one channel per element type, truncated to a cube of
half-width rc_t = fl32(k * sigma_t) around the atom, decided on the voxel
centres (§VI-B threshold truncation), with the nearest-image offset for
periodic orthorhombic cells (§III-A).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from .brute import brute_fp64  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# PGORACLE_LIB selects another build of the same source (the sanitizer
# build of oracle/build.py --sanitize)
_LIB_PATH = os.environ.get("PGORACLE_LIB") or os.path.join(_HERE, "libpgoracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f32p = ctypes.POINTER(ctypes.c_float)

_COMMON = [ctypes.c_int, _i64p, _dp, _i32p,
           ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
           _dp, _dp, _dp, _dp, _f32p, ctypes.c_float, ctypes.c_int, _dp]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from .build import build
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.pgo_grid.argtypes = _COMMON + [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp, _i64p,
                                       _i64p]
    lib.pgo_grid.restype = ctypes.c_int
    lib.pgo_grad.argtypes = _COMMON + [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp, _dp,
                                       _dp]
    lib.pgo_grad.restype = ctypes.c_int
    lib.pgo_voxels.argtypes = _COMMON + [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int,
                                         ctypes.c_int64, _i64p, _dp]
    lib.pgo_voxels.restype = ctypes.c_int
    lib.pgo_count_evals.argtypes = _COMMON
    lib.pgo_count_evals.restype = ctypes.c_int64
    lib.pgo_version.restype = ctypes.c_int
    if lib.pgo_version() != 4:
        raise ImportError(f"{_LIB_PATH} is stale: rebuild it with oracle/build.py")
    _lib = lib
    return lib


def _f32(v) -> np.ndarray:
    """float32-rounded values as float64."""
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


VALUES = {"point": 0, "box": 1}
SHAPES = {"cube": 0, "sphere": 1}


def _ptr(a: Optional[np.ndarray], t):
    if a is None:
        return ctypes.cast(None, t)
    return a.ctypes.data_as(t)


class _Args:
    """Marshals one call's inputs into contiguous arrays of the C types."""

    def __init__(self, xyz, types, offsets, sigma, dims, spacing, origin,
                 cutoff_k, cell, origins, spacings, n_types, weights=None):
        self.xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
        self.types = np.ascontiguousarray(np.asarray(types, dtype=np.int32).reshape(-1))
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64).reshape(-1))
        self.sigma = np.ascontiguousarray(np.asarray(sigma, dtype=np.float32).reshape(-1))
        self.n_sig = int(self.sigma.shape[0])
        if weights is not None:
            # weighted channels: C comes from the weights, sigma is per type
            self.weights = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
            if self.weights.ndim != 2 or self.weights.shape[0] != self.xyz.shape[0]:
                raise ValueError("weights must have shape (n_atoms, C)")
            self.C = int(self.weights.shape[1])
        else:
            self.weights = None
            self.C = int(n_types if n_types is not None else self.sigma.shape[0])
            if self.sigma.shape[0] < self.C:
                raise ValueError("sigma must have one entry per channel")
        self.D, self.H, self.W = (int(d) for d in dims)
        self.B = int(self.offsets.shape[0] - 1)
        # Grid geometry (origin, spacing, cell) is single precision in the
        # problem statement: the values are rounded to float32 once, then
        # used exactly in FP64.  Coordinates stay as given (FP64 allowed, so
        # that finite differences can perturb them).
        sp = np.broadcast_to(_f32(spacing), (3,))
        self.spacing = np.ascontiguousarray(sp, dtype=np.float64)
        og = np.zeros(3) if origin is None else np.broadcast_to(_f32(origin), (3,))
        self.origin = np.ascontiguousarray(og, dtype=np.float64)
        self.origins = None if origins is None else np.ascontiguousarray(
            _f32(origins).reshape(self.B, 3))
        self.spacings = None if spacings is None else np.ascontiguousarray(
            _f32(spacings).reshape(self.B, 3))
        self.periodic = cell is not None
        self.cell = np.ascontiguousarray(
            np.broadcast_to(_f32(cell if cell is not None else 0.0), (3,)), dtype=np.float64)
        self.k = float(np.float32(cutoff_k))
        if self.offsets[0] != 0 or self.offsets[-1] != self.xyz.shape[0]:
            raise ValueError("offsets must start at 0 and end at n_atoms")

    def common(self):
        return [self.B, _ptr(self.offsets, _i64p), _ptr(self.xyz, _dp), _ptr(self.types, _i32p),
                self.C, self.D, self.H, self.W,
                _ptr(self.origin, _dp), _ptr(self.spacing, _dp),
                _ptr(self.origins, _dp), _ptr(self.spacings, _dp),
                _ptr(self.sigma, _f32p), ctypes.c_float(self.k), int(self.periodic),
                _ptr(self.cell, _dp)]

    def weighting(self):
        return [_ptr(self.weights, _dp), self.n_sig]

    @property
    def shape(self):
        return (self.B, self.C, self.D, self.H, self.W)


def grid_fp64(xyz, types, offsets, sigma, dims, spacing, origin=None, cutoff_k=3.0,
              cell=None, origins=None, spacings=None, n_types=None, return_stats=False,
              value="point", weights=None, cutoff_shape="cube"):
    """Dense FP64 grids, shape (B, C, D, H, W), x fastest.  With weights
    (n_atoms, C), atom a adds weights[a, c] times its Gaussian (width
    sigma[types[a]]) to every channel c."""
    a = _Args(xyz, types, offsets, sigma, dims, spacing, origin, cutoff_k, cell,
              origins, spacings, n_types, weights)
    out = np.empty(a.shape, dtype=np.float64)
    ev = ctypes.c_int64(0)
    sk = ctypes.c_int64(0)
    rc = _load().pgo_grid(*a.common(), VALUES[value], SHAPES[cutoff_shape], *a.weighting(),
                          _ptr(out, _dp), ctypes.byref(ev), ctypes.byref(sk))
    if rc != 0:
        raise MemoryError("pgo_grid failed")
    if return_stats:
        return out, {"evals": ev.value, "skipped": sk.value}
    return out


def grad_fp64(xyz, types, offsets, sigma, dims, spacing, U, origin=None, cutoff_k=3.0,
              cell=None, origins=None, spacings=None, n_types=None, value="point",
              weights=None, return_weight_grad=False, cutoff_shape="cube"):
    """dL/dxyz for L = sum(U * G), shape (n_atoms, 3) float64; with weights
    and return_weight_grad, also dL/dweights (n_atoms, C)."""
    a = _Args(xyz, types, offsets, sigma, dims, spacing, origin, cutoff_k, cell,
              origins, spacings, n_types, weights)
    u = np.ascontiguousarray(np.asarray(U, dtype=np.float64).reshape(a.shape))
    g = np.empty((a.xyz.shape[0], 3), dtype=np.float64)
    gw = np.empty((a.xyz.shape[0], a.C), dtype=np.float64) if weights is not None else None
    rc = _load().pgo_grad(*a.common(), VALUES[value], SHAPES[cutoff_shape], *a.weighting(),
                          _ptr(u, _dp), _ptr(g, _dp), _ptr(gw, _dp))
    if rc != 0:
        raise MemoryError("pgo_grad failed")
    return (g, gw) if return_weight_grad else g


def voxels_fp64(xyz, types, offsets, sigma, dims, spacing, idx, origin=None, cutoff_k=3.0,
                cell=None, origins=None, spacings=None, n_types=None, value="point",
                weights=None, cutoff_shape="cube"):
    """Grid values at sampled voxels; idx is (S, 5) rows of (b, c, z, y, x)."""
    a = _Args(xyz, types, offsets, sigma, dims, spacing, origin, cutoff_k, cell,
              origins, spacings, n_types, weights)
    q = np.ascontiguousarray(np.asarray(idx, dtype=np.int64).reshape(-1, 5))
    v = np.empty(q.shape[0], dtype=np.float64)
    rc = _load().pgo_voxels(*a.common(), VALUES[value], SHAPES[cutoff_shape], *a.weighting(),
                            ctypes.c_int64(q.shape[0]), _ptr(q, _i64p), _ptr(v, _dp))
    if rc != 0:
        raise ValueError("sample index out of range")
    return v


def count_evals(xyz, types, offsets, sigma, dims, spacing, origin=None, cutoff_k=3.0,
                cell=None, origins=None, spacings=None, n_types=None) -> int:
    """Sum over atoms of the number of voxels inside each atom's window."""
    a = _Args(xyz, types, offsets, sigma, dims, spacing, origin, cutoff_k, cell,
              origins, spacings, n_types)
    return int(_load().pgo_count_evals(*a.common()))
