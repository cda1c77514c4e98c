"""GPU check of pg_grid_forward_static, the forward entry point that
allocates nothing: called through the C ABI, its output must equal
pg_grid_forward's (same kernels; bit for bit) on two calls in a row, the
second with a smaller input, and match the FP64 oracle to the bar of the
output dtype.  Requests whose workspace exceeds the fixed scratch buffer
are refused with PG_E_WORKSPACE before anything is launched."""
import ctypes

import numpy as np
import pytest

from gpu_util import errors, oracle, say, synth, to_device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F32_TOL = 1e-5
BF16_TOL = 1e-2


@pytest.fixture(scope="module")
def pg():
    import paper_2211_08506_amd as pg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pg


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def cell_batch(seed, counts, cell, n_types):
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    xyz = rng.uniform(0.0, cell, size=(int(off[-1]), 3)).astype(np.float32)
    return synth.Batch(xyz, rng.integers(0, n_types, int(off[-1])).astype(np.int32), off)


def both(pg, dev, ctx, b, sig, dims, h, dtype, form, cell):
    """(pg_grid_forward output, pg_grid_forward_static output, workspace bytes)."""
    xyz, types, offs = to_device(b, dev)
    desc = pg.make_desc(len(sig), dims, h, (0.0, 0.0, 0.0), sig, 3.0, cell, dtype, form)
    bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets)
    ws = ctx.workspace_size(desc, bv)
    ref = pg.empty_grid(desc, b.n_mol, dev).fill_(float("nan"))
    got = pg.empty_grid(desc, b.n_mol, dev).fill_(float("nan"))
    ctx.forward(desc, bv, ref)
    torch.cuda.synchronize()
    ctx.forward_static(desc, bv, got)
    torch.cuda.synchronize()
    assert ctx.device_error() == (0, -1)
    return ref, got, ws


# two calls in a row on one context, the second on a smaller batch and grid:
# (counts, cell edge, grid dims, spacing)
SEQUENCE = [([520, 430, 380], 8.0, (40, 40, 40), 0.21),
            ([300, 260], 6.0, (28, 28, 28), 0.225)]


@pytest.mark.parametrize("form,dtype,tol", [("mfma", torch.bfloat16, BF16_TOL),
                                            ("mfma", torch.float32, F32_TOL),
                                            ("window", torch.float32, F32_TOL)])
def test_static_matches_forward_binned(pg, dev, form, dtype, tol):
    ctx = pg.Context(dev)
    sig = synth.sigma_table(4, 0.3, 0.45)
    for i, (counts, cell, dims, h) in enumerate(SEQUENCE):
        say(f"[no-alloc] call {i}: {form} {dtype} counts {counts} dims {dims}")
        b = cell_batch(90 + i, counts, cell, 4)
        ref, got, ws = both(pg, dev, ctx, b, sig, dims, h, dtype, form, cell)
        assert 0 < ws <= pg.STATIC_SCRATCH_BYTES
        assert torch.equal(got.view(torch.int16 if dtype == torch.bfloat16 else torch.int32),
                           ref.view(torch.int16 if dtype == torch.bfloat16 else torch.int32))
        want = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, dims, h, (0, 0, 0), cell=cell)
        rel, mx = errors(got.double().cpu().numpy(), want)
        say(f"[no-alloc] call {i}: workspace {ws} B, rel-L2 {rel:.3e}, max-abs {mx:.3e}")
        assert rel <= tol


def test_static_matches_forward_molecules(pg, dev):
    """A molecule batch (window form, no workspace) then a smaller one."""
    ctx = pg.Context(dev)
    wl = synth.WORKLOADS["mol256"]
    sig = list(wl.sigma())
    full = wl.batch()
    for i, n in enumerate((200, 37)):
        off = full.offsets[:n + 1]
        b = synth.Batch(full.xyz[:off[-1]], full.types[:off[-1]], off)
        xyz, types, offs = to_device(b, dev)
        desc = pg.make_desc(len(sig), wl.dims, wl.spacing, wl.origin, sig, wl.cutoff_k, None,
                            torch.float32, "auto")
        bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets)
        ref = pg.empty_grid(desc, b.n_mol, dev).fill_(float("nan"))
        got = pg.empty_grid(desc, b.n_mol, dev).fill_(float("nan"))
        ctx.forward(desc, bv, ref)
        ctx.forward_static(desc, bv, got)
        torch.cuda.synchronize()
        assert torch.equal(got.view(torch.int32), ref.view(torch.int32)), i
        want = oracle.grid_fp64(b.xyz, b.types, b.offsets, np.asarray(sig), wl.dims, wl.spacing,
                                wl.origin, cutoff_k=wl.cutoff_k)
        rel, _ = errors(got.double().cpu().numpy(), want)
        say(f"[no-alloc] molecules call {i}: {b.n_mol} structures, rel-L2 {rel:.3e}")
        assert rel <= F32_TOL


def test_static_refuses_oversized_workspace(pg, dev):
    """600k atoms in one structure: the binned path's window records alone
    exceed the scratch buffer, so the call returns PG_E_WORKSPACE and
    launches nothing (the inputs are real, so nothing could be misread)."""
    ctx = pg.Context(dev)
    n = 600_000
    b = cell_batch(97, [n], 20.0, 2)
    xyz, types, offs = to_device(b, dev)
    sig = synth.sigma_table(2, 0.4, 0.5)
    desc = pg.make_desc(2, (16, 16, 16), 1.25, (0.0, 0.0, 0.0), sig, 3.0, 20.0, torch.float32,
                        "mfma")
    bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets)
    assert ctx.workspace_size(desc, bv) > pg.STATIC_SCRATCH_BYTES
    out = pg.empty_grid(desc, 1, dev)
    st = pg._lib().pg_grid_forward_static(ctx.handle, ctypes.byref(desc), ctypes.byref(bv.c),
                                          out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert st == pg.PG_E_WORKSPACE
