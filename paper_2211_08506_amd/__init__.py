"""MI355X (gfx950) density-grid generation: atoms -> C x D x H x W Gaussian grids.

Thin Python binding of the C-ABI library `libparticlegrid.so`
(include/particlegrid.h).  It only marshals arguments: every step of the
computation runs in the library's HIP kernels; PyTorch provides device
memory and the stream.  Importing this package on a machine without the
built library raises immediately -- there is no fallback path.

    import torch, paper_2211_08506_amd as pg
    g = pg.grid(xyz, types, offsets, sigma, dims=(32, 32, 32), spacing=0.5,
                origin=(-8, -8, -8), out_dtype=torch.bfloat16)

What is computed (ParticleGrid §III-A Eq. 1, point-sampled at voxel centres,
one channel per element type, truncated per axis at fl32(k sigma_t) as in
the threshold variant of §VI-B, nearest image for periodic cells): see the
header for the exact definition.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional, Sequence, Tuple, Union

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
# PARTICLEGRID_LIB selects another build of the same sources (the host
# sanitizer build of build.py --sanitize, for CPU test runs)
LIB_PATH = os.environ.get("PARTICLEGRID_LIB") or os.path.join(_HERE, "libparticlegrid.so")
# launch shapes measured by pg_autotune on an MI355X, loaded by every Context
SHIPPED_TUNING = os.path.join(_HERE, "tuning_gfx950.json")

PG_OK = 0
PG_E_NULL, PG_E_SHAPE, PG_E_PARAM, PG_E_PERIODIC = 1, 2, 3, 4
PG_E_WORKSPACE, PG_E_UNSUPPORTED, PG_E_HIP, PG_E_DEVICE_DATA, PG_E_CAPACITY = 5, 6, 7, 8, 9
PG_OUT_F32, PG_OUT_BF16 = 0, 1
FORMS = {"auto": 0, "plain": 1, "window": 2, "mfma": 3}
FORM_NAMES = {v: k for k, v in FORMS.items()}
VALUES = {"point": 0, "box": 1}
PG_CELL_NONE, PG_CELL_ORTHO, PG_CELL_TRICLINIC = 0, 1, 2
SHAPES = {"cube": 0, "sphere": 1}
PG_OPT_GRAPH, PG_OPT_BLOCK, PG_OPT_GRID_PER_CU, PG_OPT_NT_STORE, PG_OPT_UNROLL = 1, 2, 3, 4, 5
PG_HOST_ONLY = -1          # pg_create device of a context that touches no GPU
MAX_CHANNELS = 64


class PGError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = _lib().pg_status_str(status).decode() if _LIB is not None else str(status)
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)


class GridDesc(ctypes.Structure):
    _fields_ = [("C", ctypes.c_int32), ("D", ctypes.c_int32), ("H", ctypes.c_int32),
                ("W", ctypes.c_int32),
                ("origin", ctypes.c_float * 3), ("spacing", ctypes.c_float * 3),
                ("cutoff_k", ctypes.c_float), ("periodic", ctypes.c_int32),
                ("cell", ctypes.c_float * 3), ("out_dtype", ctypes.c_int32),
                ("form", ctypes.c_int32), ("sigma", ctypes.c_float * MAX_CHANNELS),
                ("value", ctypes.c_int32), ("n_types", ctypes.c_int32),
                ("cell_matrix", ctypes.c_float * 9), ("cutoff_shape", ctypes.c_int32)]


class Batch(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("types", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p), ("origins", ctypes.c_void_p),
                ("spacings", ctypes.c_void_p), ("n_mol", ctypes.c_int32),
                ("max_atoms", ctypes.c_int32), ("n_atoms", ctypes.c_int64),
                ("weights", ctypes.c_void_p)]


class PlanInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("form", "block", "grid", "lds_bytes", "vec", "nt_store", "atom_capacity",
                 "unroll", "per_cu", "binned")]


_LIB = None
_LIB_LOCK = threading.Lock()

EXPORTS = ("pg_abi_version", "pg_status_str", "pg_create", "pg_destroy", "pg_validate",
           "pg_workspace_size", "pg_grid_forward", "pg_grid_backward", "pg_autotune",
           "pg_tuning_save", "pg_tuning_load", "pg_set_option", "pg_get_device_error",
           "pg_last_hip_error", "pg_plan", "pg_find_peaks", "pg_reversal_workspace_size",
           "pg_reversal_step", "pg_grid_forward_static")
# fixed device scratch of pg_grid_forward_static (PG_STATIC_SCRATCH_BYTES)
STATIC_SCRATCH_BYTES = 64 << 20


def _lib():
    """Load libparticlegrid.so (raises if it was not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    with _LIB_LOCK:
        if _LIB is not None:
            return _LIB
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python paper_2211_08506_amd/build.py` (or __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        vp, P = ctypes.c_void_p, ctypes.POINTER
        lib.pg_abi_version.restype = ctypes.c_int
        lib.pg_status_str.restype = ctypes.c_char_p
        lib.pg_status_str.argtypes = [ctypes.c_int]
        lib.pg_create.argtypes = [P(vp), ctypes.c_int]
        lib.pg_destroy.argtypes = [vp]
        lib.pg_validate.argtypes = [P(GridDesc), P(Batch)]
        lib.pg_workspace_size.argtypes = [vp, P(GridDesc), P(Batch), P(ctypes.c_size_t)]
        lib.pg_grid_forward.argtypes = [vp, P(GridDesc), P(Batch), vp, vp, ctypes.c_size_t, vp]
        lib.pg_grid_forward_static.argtypes = [vp, P(GridDesc), P(Batch), vp, vp]
        lib.pg_grid_backward.argtypes = [vp, P(GridDesc), P(Batch), vp, vp, vp, vp,
                                         ctypes.c_size_t, vp]
        lib.pg_autotune.argtypes = [vp, P(GridDesc), P(Batch), vp, vp, ctypes.c_size_t, vp,
                                    ctypes.c_int]
        lib.pg_tuning_save.argtypes = [vp, ctypes.c_char_p]
        lib.pg_tuning_load.argtypes = [vp, ctypes.c_char_p]
        lib.pg_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_int64]
        lib.pg_get_device_error.argtypes = [vp, P(ctypes.c_int32), P(ctypes.c_int64)]
        lib.pg_last_hip_error.argtypes = [vp]
        lib.pg_plan.argtypes = [vp, P(GridDesc), P(Batch), vp, P(PlanInfo)]
        lib.pg_find_peaks.argtypes = [vp, P(GridDesc), vp, ctypes.c_int32, vp, vp, ctypes.c_float,
                                      ctypes.c_int64, vp, vp, vp, vp, vp]
        lib.pg_reversal_workspace_size.argtypes = [vp, P(GridDesc), P(Batch), P(ctypes.c_size_t)]
        lib.pg_reversal_step.argtypes = [vp, P(GridDesc), P(Batch), vp, vp, vp, vp, vp,
                                         ctypes.c_float, vp, ctypes.c_size_t, vp]
        for name in EXPORTS:
            getattr(lib, name).restype = ctypes.c_int if name != "pg_status_str" else ctypes.c_char_p
        _LIB = lib
        return lib


def _check(status: int, what: str):
    if status != PG_OK:
        raise PGError(status, what)


def _f3(v) -> Tuple[float, float, float]:
    if isinstance(v, (int, float)):
        return (float(v),) * 3
    v = tuple(float(x) for x in v)
    if len(v) != 3:
        raise ValueError("expected a scalar or 3 values (x, y, z)")
    return v


def make_desc(C: int, dims: Sequence[int], spacing, origin=(0.0, 0.0, 0.0), sigma=(),
              cutoff_k: float = 3.0, cell=None, out_dtype=torch.float32,
              form: Union[str, int] = "auto", value: Union[str, int] = "point",
              n_types: int = 0, cutoff_shape: Union[str, int] = "cube") -> GridDesc:
    """Build a pg_grid_desc (host struct).  dims = (D, H, W) = (z, y, x);
    origin / spacing in x, y, z order; cell: None, a scalar or 3 edges
    (orthorhombic), or a 3 x 3 matrix whose column j is lattice vector j
    (triclinic); sigma one width per type
    (= per channel unless weighted); value "point" (the Gaussian at voxel
    centres) or "box" (the normalised Gaussian's mass in each voxel);
    n_types: with weighted channels, how many widths the types index;
    cutoff_shape "cube" (exact, separable) or "sphere"."""
    d = GridDesc()
    d.C = int(C)
    d.D, d.H, d.W = (int(x) for x in dims)
    d.origin[:] = _f3(origin)
    d.spacing[:] = _f3(spacing)
    d.cutoff_k = float(cutoff_k)
    if cell is None:
        d.periodic = PG_CELL_NONE
        d.cell[:] = (0.0, 0.0, 0.0)
    elif np.asarray(cell).size == 9:
        d.periodic = PG_CELL_TRICLINIC
        d.cell_matrix[:] = [float(x) for x in np.asarray(cell, np.float64).reshape(3, 3).ravel()]
    else:
        d.periodic = PG_CELL_ORTHO
        d.cell[:] = _f3(cell)
    if out_dtype in (torch.float32, "f32", PG_OUT_F32):
        d.out_dtype = PG_OUT_F32
    elif out_dtype in (torch.bfloat16, "bf16", PG_OUT_BF16):
        d.out_dtype = PG_OUT_BF16
    else:
        raise ValueError(f"unsupported out_dtype {out_dtype}")
    d.form = FORMS[form] if isinstance(form, str) else int(form)
    d.value = VALUES[value] if isinstance(value, str) else int(value)
    d.n_types = int(n_types)
    d.cutoff_shape = SHAPES[cutoff_shape] if isinstance(cutoff_shape, str) else int(cutoff_shape)
    sig = [float(s) for s in sigma]
    if len(sig) > MAX_CHANNELS:
        raise ValueError(f"at most {MAX_CHANNELS} channels")
    for i, s in enumerate(sig):
        d.sigma[i] = s
    return d


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


class BatchView:
    """Device-resident CSR batch plus the host facts the ABI needs.  Keeps
    the tensors alive while the library may use them."""

    def __init__(self, xyz: torch.Tensor, types: torch.Tensor, offsets: torch.Tensor,
                 origins: Optional[torch.Tensor] = None, spacings: Optional[torch.Tensor] = None,
                 max_atoms: Optional[int] = None, offsets_host=None,
                 weights: Optional[torch.Tensor] = None):
        dev = xyz.device
        if dev.type != "cuda":
            raise ValueError("xyz must be a device (cuda/hip) tensor")
        self.xyz = xyz.to(torch.float32).contiguous()
        if self.xyz.dim() != 2 or self.xyz.shape[1] != 3:
            raise ValueError("xyz must have shape (n_atoms, 3)")
        self.types = types.to(device=dev, dtype=torch.int32).contiguous()
        self.offsets = offsets.to(device=dev, dtype=torch.int32).contiguous()
        self.origins = None if origins is None else origins.to(device=dev, dtype=torch.float32).contiguous()
        self.spacings = None if spacings is None else spacings.to(device=dev, dtype=torch.float32).contiguous()
        self.n_mol = int(self.offsets.shape[0]) - 1
        self.n_atoms = int(self.xyz.shape[0])
        if self.types.shape[0] != self.n_atoms:
            raise ValueError("types must have one entry per atom")
        if max_atoms is None:
            oh = offsets_host if offsets_host is not None else offsets.detach().to("cpu")
            oh = torch.as_tensor(oh, dtype=torch.int64)
            max_atoms = int((oh[1:] - oh[:-1]).max().item()) if self.n_mol > 0 else 0
        self.max_atoms = int(max_atoms)
        b = Batch()
        b.xyz = _ptr(self.xyz)
        b.types = _ptr(self.types)
        b.offsets = _ptr(self.offsets)
        b.origins = _ptr(self.origins)
        b.spacings = _ptr(self.spacings)
        b.n_mol = self.n_mol
        b.max_atoms = self.max_atoms
        b.n_atoms = self.n_atoms
        self.weights = None
        if weights is not None:
            self.weights = weights.to(device=dev, dtype=torch.float32).contiguous()
            if self.weights.dim() != 2 or self.weights.shape[0] != self.n_atoms:
                raise ValueError("weights must have shape (n_atoms, C)")
        b.weights = _ptr(self.weights)
        self.c = b


class Context:
    """A library context on one device (error word, tuning table, graph
    cache) plus a cached torch workspace buffer."""

    def __init__(self, device: Union[int, torch.device, None] = None,
                 tuning: Optional[str] = "shipped"):
        if device is None:
            device = torch.cuda.current_device()
        if isinstance(device, torch.device):
            device = device.index if device.index is not None else torch.cuda.current_device()
        self.device = int(device)
        h = ctypes.c_void_p()
        _check(_lib().pg_create(ctypes.byref(h), self.device), "pg_create")
        self.handle = h
        self._ws = None
        if tuning == "shipped":
            tuning = SHIPPED_TUNING if os.path.exists(SHIPPED_TUNING) else None
        if tuning:
            self.tuning_load(tuning)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _LIB is not None:
            try:
                _LIB.pg_destroy(h)
            except Exception:
                pass
            self.handle = None

    def workspace(self, nbytes: int) -> Optional[torch.Tensor]:
        if nbytes == 0:
            return None
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def set_option(self, option: int, value: int):
        _check(_lib().pg_set_option(self.handle, option, int(value)), "pg_set_option")

    def device_error(self) -> Tuple[int, int]:
        code = ctypes.c_int32()
        first = ctypes.c_int64()
        _check(_lib().pg_get_device_error(self.handle, ctypes.byref(code), ctypes.byref(first)),
               "pg_get_device_error")
        return code.value, first.value

    def plan(self, desc: GridDesc, batch: BatchView, out: Optional[torch.Tensor] = None) -> dict:
        info = PlanInfo()
        _check(_lib().pg_plan(self.handle, ctypes.byref(desc), ctypes.byref(batch.c),
                              _ptr(out), ctypes.byref(info)), "pg_plan")
        d = {n: getattr(info, n) for n, _ in PlanInfo._fields_}
        d["form"] = FORM_NAMES.get(d["form"], d["form"])
        return d

    def workspace_size(self, desc: GridDesc, batch: BatchView) -> int:
        n = ctypes.c_size_t()
        _check(_lib().pg_workspace_size(self.handle, ctypes.byref(desc), ctypes.byref(batch.c),
                                        ctypes.byref(n)), "pg_workspace_size")
        return int(n.value)

    def forward(self, desc: GridDesc, batch: BatchView, out: torch.Tensor,
                stream: Optional[torch.cuda.Stream] = None):
        nbytes = self.workspace_size(desc, batch)
        ws = self.workspace(nbytes)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(_lib().pg_grid_forward(self.handle, ctypes.byref(desc), ctypes.byref(batch.c),
                                      _ptr(out), _ptr(ws), nbytes, s.cuda_stream),
               "pg_grid_forward")
        return out

    def forward_static(self, desc: GridDesc, batch: BatchView, out: torch.Tensor,
                       stream: Optional[torch.cuda.Stream] = None):
        """pg_grid_forward_static: the forward on the library's fixed device
        scratch buffer -- no workspace is allocated here or in the library."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(_lib().pg_grid_forward_static(self.handle, ctypes.byref(desc),
                                             ctypes.byref(batch.c), _ptr(out), s.cuda_stream),
               "pg_grid_forward_static")
        return out

    def backward(self, desc: GridDesc, batch: BatchView, grad_out: torch.Tensor,
                 grad_xyz: Optional[torch.Tensor], stream: Optional[torch.cuda.Stream] = None,
                 grad_weights: Optional[torch.Tensor] = None):
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = self.workspace_size(desc, batch) if desc.periodic == PG_CELL_TRICLINIC else 0
        ws = self.workspace(nbytes)
        _check(_lib().pg_grid_backward(self.handle, ctypes.byref(desc), ctypes.byref(batch.c),
                                       _ptr(grad_out), _ptr(grad_xyz), _ptr(grad_weights),
                                       _ptr(ws), nbytes, s.cuda_stream), "pg_grid_backward")
        return grad_xyz

    def autotune(self, desc: GridDesc, batch: BatchView, out: torch.Tensor, reps: int = 5,
                 stream: Optional[torch.cuda.Stream] = None):
        nbytes = self.workspace_size(desc, batch)
        ws = self.workspace(nbytes)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(_lib().pg_autotune(self.handle, ctypes.byref(desc), ctypes.byref(batch.c),
                                  _ptr(out), _ptr(ws), nbytes, s.cuda_stream, int(reps)),
               "pg_autotune")

    def find_peaks(self, desc: GridDesc, grid: torch.Tensor, threshold: float,
                   origins: Optional[torch.Tensor] = None, spacings: Optional[torch.Tensor] = None,
                   capacity: Optional[int] = None, stream: Optional[torch.cuda.Stream] = None):
        """Local maxima of every channel of a float32 grid batch (pg_find_peaks)
        -> (xyz (n, 3), types (n,), offsets (B + 1,)) device tensors.  Reads
        the peak count back to the host; with capacity None the output is
        sized to hold every peak."""
        if grid.dtype != torch.float32 or not grid.is_contiguous() or grid.dim() != 5:
            raise ValueError("grid must be a contiguous (B, C, D, H, W) float32 tensor")
        dev = grid.device
        B = int(grid.shape[0])
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        cap = int(capacity) if capacity is not None else max(1024, 64 * B)
        o_t = None if origins is None else origins.to(dev, torch.float32).contiguous()
        s_t = None if spacings is None else spacings.to(dev, torch.float32).contiguous()
        n_found = torch.zeros(1, dtype=torch.int64, device=dev)
        while True:
            xyz = torch.empty((cap, 3), dtype=torch.float32, device=dev)
            types = torch.empty(cap, dtype=torch.int32, device=dev)
            offsets = torch.empty(B + 1, dtype=torch.int32, device=dev)
            _check(_lib().pg_find_peaks(self.handle, ctypes.byref(desc), _ptr(grid), B,
                                        _ptr(o_t), _ptr(s_t), float(threshold), cap, _ptr(xyz),
                                        _ptr(types), _ptr(offsets), _ptr(n_found),
                                        s.cuda_stream), "pg_find_peaks")
            s.synchronize()
            n = int(n_found.item())
            if n <= cap or capacity is not None:
                n = min(n, cap)
                return xyz[:n], types[:n], offsets
            cap = n

    def reversal_workspace_size(self, desc: GridDesc, batch: BatchView) -> int:
        n = ctypes.c_size_t()
        _check(_lib().pg_reversal_workspace_size(self.handle, ctypes.byref(desc),
                                                 ctypes.byref(batch.c), ctypes.byref(n)),
               "pg_reversal_workspace_size")
        return int(n.value)

    def reversal_step(self, desc: GridDesc, batch: BatchView, target: torch.Tensor,
                      residual: Optional[torch.Tensor], loss: torch.Tensor,
                      grad_xyz: Optional[torch.Tensor] = None,
                      xyz_update: Optional[torch.Tensor] = None, lr: float = 0.0,
                      stream: Optional[torch.cuda.Stream] = None):
        """One grid-reversal step (pg_reversal_step): residual = 2 (G' - T),
        loss per structure, and optionally the gradient and xyz - lr * grad
        (xyz_update may be batch.xyz for an in-place step).  residual may be
        None on the molecule window form without weights: no residual grid
        is stored and the adjoint forms it where it reads it."""
        for name, t in (("target", target), ("residual", residual), ("loss", loss)):
            if t is None and name == "residual":
                continue
            if t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float32 tensor")
        nbytes = self.reversal_workspace_size(desc, batch)
        ws = self.workspace(nbytes)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _check(_lib().pg_reversal_step(self.handle, ctypes.byref(desc), ctypes.byref(batch.c),
                                       _ptr(target), _ptr(residual), _ptr(loss), _ptr(grad_xyz),
                                       _ptr(xyz_update), float(lr), _ptr(ws), nbytes,
                                       s.cuda_stream), "pg_reversal_step")
        return loss

    def tuning_save(self, path: str):
        _check(_lib().pg_tuning_save(self.handle, path.encode()), "pg_tuning_save")

    def tuning_load(self, path: str):
        _check(_lib().pg_tuning_load(self.handle, path.encode()), "pg_tuning_load")


_CTX = {}


def default_context(device=None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    if isinstance(device, torch.device):
        device = device.index if device.index is not None else torch.cuda.current_device()
    if device not in _CTX:
        _CTX[device] = Context(device)
    return _CTX[device]


def empty_grid(desc: GridDesc, n_mol: int, device) -> torch.Tensor:
    dt = torch.bfloat16 if desc.out_dtype == PG_OUT_BF16 else torch.float32
    return torch.empty((n_mol, desc.C, desc.D, desc.H, desc.W), dtype=dt, device=device)


class GridFn(torch.autograd.Function):
    """Differentiable w.r.t. xyz and the channel weights: forward ->
    pg_grid_forward, backward -> pg_grid_backward (the coordinate adjoint
    and, for weighted channels, the weight gradient)."""

    @staticmethod
    def forward(ctx_, xyz, types, offsets, origins, spacings, weights, desc, max_atoms, pgctx):
        batch = BatchView(xyz.detach(), types, offsets, origins, spacings, max_atoms=max_atoms,
                          weights=None if weights is None else weights.detach())
        out = empty_grid(desc, batch.n_mol, xyz.device)
        pgctx.forward(desc, batch, out)
        ctx_.batch = batch
        ctx_.desc = desc
        ctx_.pgctx = pgctx
        return out

    @staticmethod
    def backward(ctx_, grad_out):
        batch = ctx_.batch
        g = grad_out.contiguous()
        want = torch.bfloat16 if ctx_.desc.out_dtype == PG_OUT_BF16 else torch.float32
        if g.dtype != want:
            g = g.to(want)
        need_xyz, need_w = ctx_.needs_input_grad[0], ctx_.needs_input_grad[5]
        grad_xyz = torch.empty_like(batch.xyz) if (need_xyz or not need_w) else None
        grad_w = torch.empty_like(batch.weights) if need_w else None
        ctx_.pgctx.backward(ctx_.desc, batch, g, grad_xyz, grad_weights=grad_w)
        return (grad_xyz if need_xyz else None, None, None, None, None, grad_w, None, None,
                None)


def grid(xyz: torch.Tensor, types: torch.Tensor, offsets: torch.Tensor, sigma: Sequence[float], *,
         dims: Sequence[int], spacing=0.5, origin=(0.0, 0.0, 0.0), origins=None, spacings=None,
         cutoff_k: float = 3.0, cell=None, out_dtype=torch.float32, form: str = "auto",
         value: str = "point", weights: Optional[torch.Tensor] = None,
         cutoff_shape: str = "cube", n_channels: Optional[int] = None,
         max_atoms: Optional[int] = None, ctx: Optional[Context] = None) -> torch.Tensor:
    """Density grids (B, C, D, H, W) for a ragged batch (differentiable in
    xyz, and in weights when given).

    xyz (n_atoms, 3) float32, types (n_atoms,) int, offsets (B+1,) int CSR,
    all on the same device; sigma: one width per type; value "point" or
    "box" as in make_desc.  Without weights each type is one channel
    (C = len(sigma) unless n_channels is given).  With weights (n_atoms, C)
    atom a adds weights[a, c] times its Gaussian to every channel c --
    e.g. weights = embedding[types] for a learned (T x C) embedding table,
    whose gradient then flows through torch's indexing."""
    if weights is not None:
        C = int(weights.shape[1])
        n_types = len(sigma)
    else:
        C = int(n_channels if n_channels is not None else len(sigma))
        n_types = 0
    desc = make_desc(C, dims, spacing, origin, sigma, cutoff_k, cell, out_dtype, form, value,
                     n_types, cutoff_shape)
    pgctx = ctx if ctx is not None else default_context(xyz.device)
    return GridFn.apply(xyz, types, offsets, origins, spacings, weights, desc, max_atoms, pgctx)


def reverse(target: torch.Tensor, sigma: Sequence[float], *, spacing=0.5,
            origin=(0.0, 0.0, 0.0), threshold: float = 0.05, lr: float = 0.02, steps: int = 100,
            tol: float = 0.0, check_every: int = 10, cutoff_k: float = 3.0, cell=None,
            value: str = "point", ctx: Optional[Context] = None):
    """Grid reversal (§IV-A): atoms back from a batch of float32 grids
    (B, C, D, H, W).  Starts from the local maxima above `threshold`, then
    takes gradient steps xyz <- xyz - lr * dL/dxyz on L = sum (G' - T)^2
    until every structure's loss is below tol (checked every check_every
    steps) or `steps` steps are done.  Returns (xyz, types, offsets, loss)."""
    if target.dtype != torch.float32:
        raise ValueError("target must be float32")
    target = target.contiguous()
    B, C, D, H, W = (int(x) for x in target.shape)
    pgctx = ctx if ctx is not None else default_context(target.device)
    desc = make_desc(C, (D, H, W), spacing, origin, sigma, cutoff_k, cell, torch.float32, "auto",
                     value)
    xyz, types, offsets = pgctx.find_peaks(desc, target, threshold)
    xyz = xyz.clone()
    batch = BatchView(xyz, types, offsets)
    # the molecule window form keeps no residual grid; the binned path
    # needs one
    plan = pgctx.plan(desc, batch)
    residual = None if (plan["form"] == "window" and not plan["binned"]) else \
        torch.empty_like(target)
    loss = torch.empty(B, dtype=torch.float32, device=target.device)
    for k in range(steps):
        pgctx.reversal_step(desc, batch, target, residual, loss, None, batch.xyz, lr)
        if tol > 0 and (k + 1) % check_every == 0 and float(loss.max().item()) < tol:
            break
    # the loss at the final coordinates
    pgctx.reversal_step(desc, batch, target, residual, loss)
    return batch.xyz, types, offsets, loss


def lib_path() -> str:
    return LIB_PATH


def abi_version() -> int:
    return int(_lib().pg_abi_version())


# fail loudly at import if the library is missing
_lib()
