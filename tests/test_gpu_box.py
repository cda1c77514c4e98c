"""GPU parity of the box form -- each voxel holds the mass of the normalised
Gaussian inside it (§III-A Eq. 2-5) -- against the FP64 oracle's box form,
through the C ABI: the molecule window kernel, the plain kernel, both forms
of the binned large-structure path, and the coordinate adjoint.

Bars as for the point form: FP32 rel-L2 <= 1e-5, BF16 (and the MFMA form,
whose separable factors are bf16) rel-L2 <= 1e-2, adjoint rel-L2 <= 1e-4.
The cutoff windows are decided on the voxel centres exactly as for the
point form, so the support must match the oracle's voxel for voxel.
"""
import numpy as np
import pytest

from gpu_util import errors, oracle, sample_voxels, say, synth, to_device, worst_molecule

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F32_TOL = 1e-5
BF16_TOL = 1e-2
ADJ_TOL = 1e-4


@pytest.fixture(scope="module")
def pg():
    import paper_2211_08506_amd as pg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pg


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def run(pg, dev, b, sig, dims, h, origin, dtype=torch.float32, form="auto", cell=None,
        cutoff_k=3.0):
    xyz, types, offs = to_device(b, dev)
    g = pg.grid(xyz, types, offs, list(sig), dims=dims, spacing=h, origin=origin, cell=cell,
                out_dtype=dtype, form=form, cutoff_k=cutoff_k, value="box")
    torch.cuda.synchronize()
    return g


def check(name, g, ref, tol):
    got = g.double().cpu().numpy()
    rel, mx = errors(got, ref)
    wm = worst_molecule(got, ref) if ref.shape[0] > 1 else rel
    say(f"[box {name}] rel-L2 {rel:.3e}  max-abs {mx:.3e}  worst-structure rel-L2 {wm:.3e}")
    assert rel <= tol and wm <= tol, name
    assert np.array_equal(got > 0, ref > 0), name
    return got


@pytest.mark.parametrize("form", ["window", "plain"])
@pytest.mark.parametrize("dtype,tol", [(torch.float32, F32_TOL), (torch.bfloat16, BF16_TOL)])
def test_box_molecule_batch(pg, dev, form, dtype, tol):
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(48)
    say(f"case box molecules form={form} dtype={dtype}")
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing,
                           wl.origin, value="box")
    g = run(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, dtype, form)
    check(f"mol256x48/{form}/{dtype}", g, ref, tol)


@pytest.mark.parametrize("dims", [(8, 12, 30), (5, 7, 33), (1, 1, 1)])
def test_box_odd_shapes(pg, dev, dims):
    rng = np.random.default_rng(sum(dims) + 7)
    counts = [0, 3, 7, 1, 0, 5]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    h = 0.3
    ext = np.array([dims[2], dims[1], dims[0]]) * h
    xyz = (rng.uniform(-0.2, 1.2, size=(off[-1], 3)) * ext).astype(np.float32)
    b = synth.Batch(xyz, rng.integers(0, 3, off[-1]).astype(np.int32), off)
    sig = synth.sigma_table(3, 0.25, 0.4)
    say(f"case box odd shape {dims}")
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, dims, h, (0, 0, 0), value="box")
    for form in ("window", "plain"):
        g = run(pg, dev, b, sig, dims, h, (0.0, 0.0, 0.0), torch.float32, form)
        check(f"odd{dims}/{form}", g, ref, F32_TOL)


def test_box_channel_sums_count_atoms(pg, dev):
    """Eq. 6 on the device: without a cutoff each channel of a molecule well
    inside the grid sums to its number of atoms of that type."""
    wl = synth.WORKLOADS["single20"]
    b = wl.batch()
    dims, h, o = (48, 48, 48), 0.5, (-12.0, -12.0, -12.0)
    say("case box channel sums, no cutoff")
    for form in ("window", "plain"):
        g = run(pg, dev, b, wl.sigma(), dims, h, o, torch.float32, form, cutoff_k=0.0)
        sums = g[0].double().sum(dim=(1, 2, 3)).cpu().numpy()
        counts = np.bincount(b.types, minlength=len(wl.sigma()))
        say(f"[box sums/{form}] {sums} vs {counts}")
        np.testing.assert_allclose(sums, counts, rtol=1e-5, atol=1e-5)


def test_box_binned_path(pg, dev):
    """Periodic cells above the window kernel's capacity: the binned FP32
    vector form and the MFMA form, with images through the faces."""
    sig = synth.sigma_table(3, 0.3, 0.45)
    rng = np.random.default_rng(41)
    counts = [400, 300]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    xyz = rng.uniform(0, 8.0, size=(off[-1], 3)).astype(np.float32)
    xyz[0] = [0.01, 7.99, 4.0]
    b = synth.Batch(xyz, rng.integers(0, 3, off[-1]).astype(np.int32), off)
    dims, h = (40, 40, 40), 0.21
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, dims, h, (0, 0, 0), cell=8.0,
                           value="box")
    for form, dt, tol in [("window", torch.float32, F32_TOL), ("window", torch.bfloat16, BF16_TOL),
                          ("mfma", torch.bfloat16, BF16_TOL), ("mfma", torch.float32, F32_TOL)]:
        say(f"case box binned form={form} dtype={dt}")
        g = run(pg, dev, b, sig, dims, h, (0, 0, 0), dt, form, cell=8.0)
        check(f"cells/{form}/{dt}", g, ref, tol)


def test_box_full_size_sampled(pg, dev):
    """The 4096-molecule 32^3 batch in bf16, sampled voxels against the
    oracle evaluated one by one."""
    wl = synth.WORKLOADS["mol4096"]
    b = wl.batch()
    say("case box full-size mol4096 bf16")
    g = run(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, torch.bfloat16)
    rng = np.random.default_rng(23)
    idx = sample_voxels(rng, b, tuple(g.shape), wl.origin, wl.spacing, 20000, 20000)
    ref = oracle.voxels_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing, idx,
                             wl.origin, value="box")
    it = torch.tensor(idx, device=dev)
    got = g[it[:, 0], it[:, 1], it[:, 2], it[:, 3], it[:, 4]].double().cpu().numpy()
    rel, mx = errors(got, ref)
    say(f"[box mol4096/bf16 sampled {len(idx)}] rel-L2 {rel:.3e} max-abs {mx:.3e}")
    assert rel <= BF16_TOL
    assert np.array_equal(got > 0, ref > 0)


@pytest.mark.parametrize("cell", [None, 8.0])
def test_box_adjoint(pg, dev, cell):
    """dL/dxyz of the box form against the oracle's analytic gradient:
    molecules, then periodic cells above the window kernel's capacity."""
    if cell is None:
        wl = synth.WORKLOADS["adjoint1024"]
        b = wl.batch(32)
        sig, dims, h, o = wl.sigma(), wl.dims, wl.spacing, wl.origin
    else:
        sig = synth.sigma_table(3, 0.3, 0.45)
        rng = np.random.default_rng(43)
        off = np.array([0, 400, 700], np.int32)
        xyz = rng.uniform(0, cell, size=(700, 3)).astype(np.float32)
        b = synth.Batch(xyz, rng.integers(0, 3, 700).astype(np.int32), off)
        dims, h, o = (40, 40, 40), 0.21, (0.0, 0.0, 0.0)
    say(f"case box adjoint cell={cell}")
    U = synth.upstream(44, (b.n_mol, len(sig)) + tuple(dims))
    xyz, types, offs = to_device(b, dev)
    xyz.requires_grad_(True)
    g = pg.grid(xyz, types, offs, list(sig), dims=dims, spacing=h, origin=o, cell=cell,
                value="box")
    g.backward(torch.tensor(U, device=dev))
    torch.cuda.synchronize()
    got = xyz.grad.double().cpu().numpy()
    ref = oracle.grad_fp64(b.xyz, b.types, b.offsets, sig, dims, h, U, o, cell=cell,
                           value="box")
    rel, mx = errors(got, ref)
    say(f"[box adjoint cell={cell}] rel-L2 {rel:.3e} max-abs {mx:.3e}")
    assert rel <= ADJ_TOL
