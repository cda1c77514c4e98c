"""GPU parity of the sphere cutoff through the C ABI, against the oracle's
sphere: the molecule window form and the plain form (point and box values,
FP32 and BF16, periodic cells), large structures (AUTO takes the plain
form), the coordinate adjoint and the reversal step.

The sphere edge is decided in float32 on the GPU and in double in the
oracle, so voxels within a relative 1e-6 of some atom's sphere (the edge
band) are left out of the element-wise comparison and counted; everywhere
else the bars are the usual ones and the support matches voxel for voxel.
"""
import numpy as np
import pytest

from gpu_util import errors, oracle, say, synth, to_device, worst_molecule
from oracle import reversal, sphere

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


def compare(name, g, ref, band, tol):
    got = g.double().cpu().numpy()
    keep = ~band
    rel, mx = errors(got[keep], ref[keep])
    say(f"[sphere {name}] rel-L2 {rel:.3e} max-abs {mx:.3e} (edge band: {int(band.sum())} "
        f"voxels of {band.size})")
    assert rel <= tol, name
    assert np.array_equal(got[keep] > 0, ref[keep] > 0), name
    # in the band a voxel holds the oracle's value with or without the
    # edge atom's term, whose size is at most exp(-k^2/2) (point form)
    if band.any():
        assert np.max(np.abs(got[band] - ref[band])) <= 0.0112 + 1e-2 * np.max(ref[band])


@pytest.mark.parametrize("form", ["window", "plain"])
@pytest.mark.parametrize("value", ["point", "box"])
def test_sphere_molecules(pg, dev, form, value):
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(48)
    say(f"case sphere molecules form={form} value={value}")
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing,
                           wl.origin, value=value, cutoff_shape="sphere")
    band = sphere.edge_band(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing,
                            wl.origin)
    xyz, types, offs = to_device(b, dev)
    for dt, tol in ((torch.float32, F32_TOL), (torch.bfloat16, BF16_TOL)):
        g = pg.grid(xyz, types, offs, list(wl.sigma()), dims=wl.dims, spacing=wl.spacing,
                    origin=wl.origin, out_dtype=dt, form=form, value=value,
                    cutoff_shape="sphere")
        torch.cuda.synchronize()
        compare(f"mol/{form}/{value}/{dt}", g, ref, band, tol)


def test_sphere_periodic_cells_and_auto_plain(pg, dev):
    sig = synth.sigma_table(3, 0.3, 0.45)
    rng = np.random.default_rng(71)
    # small cells: the window form; a 300-atom cell: AUTO takes the plain form
    for counts, form_want in (([12, 20], "window"), ([300], "plain")):
        off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
        xyz = rng.uniform(0, 8.0, size=(int(off[-1]), 3)).astype(np.float32)
        b = synth.Batch(xyz, rng.integers(0, 3, int(off[-1])).astype(np.int32), off)
        dims, h = (28, 30, 32), 0.27
        x, t, o = to_device(b, dev)
        desc = pg.make_desc(3, dims, h, (0, 0, 0), sig, 3.0, 8.0, cutoff_shape="sphere")
        plan = pg.default_context(dev).plan(desc, pg.BatchView(x, t, o))
        assert plan["form"] == form_want and plan["binned"] == 0, plan
        say(f"case sphere periodic cells {counts} form={form_want}")
        ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, dims, h, (0, 0, 0), cell=8.0,
                               cutoff_shape="sphere")
        band = sphere.edge_band(b.xyz, b.types, b.offsets, sig, dims, h, (0, 0, 0), cell=8.0)
        g = pg.grid(x, t, o, list(sig), dims=dims, spacing=h, cell=8.0, cutoff_shape="sphere")
        torch.cuda.synchronize()
        compare(f"cells/{form_want}", g, ref, band, F32_TOL)


@pytest.mark.parametrize("value", ["point", "box"])
def test_sphere_adjoint(pg, dev, value):
    wl = synth.WORKLOADS["adjoint1024"]
    b = wl.batch(32)
    U = synth.upstream(72, wl.grid_shape(32))
    say(f"case sphere adjoint value={value}")
    ref = oracle.grad_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing, U,
                           wl.origin, value=value, cutoff_shape="sphere")
    xyz, types, offs = to_device(b, dev)
    xyz.requires_grad_(True)
    g = pg.grid(xyz, types, offs, list(wl.sigma()), dims=wl.dims, spacing=wl.spacing,
                origin=wl.origin, value=value, cutoff_shape="sphere")
    g.backward(torch.tensor(U, device=dev))
    torch.cuda.synchronize()
    rel, mx = errors(xyz.grad.cpu().numpy(), ref)
    say(f"[sphere adjoint {value}] rel-L2 {rel:.3e} max-abs {mx:.3e}")
    assert rel <= ADJ_TOL


def test_sphere_reversal_step(pg, dev):
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(16)
    rng = np.random.default_rng(73)
    T = oracle.grid_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing, wl.origin,
                         cutoff_shape="sphere").astype(np.float32)
    x0 = (b.xyz + rng.uniform(-0.1, 0.1, size=b.xyz.shape)).astype(np.float32)
    say("case sphere reversal step")
    loss_o, U_o, grad_o, _ = reversal.reversal_step(x0, b.types, b.offsets, wl.sigma(), wl.dims,
                                                    wl.spacing, T, 0.01, wl.origin,
                                                    cutoff_shape="sphere")
    band = sphere.edge_band(x0, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing, wl.origin)
    ctx = pg.Context(0)
    desc = pg.make_desc(5, wl.dims, wl.spacing, wl.origin, wl.sigma(), 3.0, None,
                        cutoff_shape="sphere")
    xyz, types, offs = to_device(synth.Batch(x0, b.types, b.offsets), dev)
    bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets)
    assert ctx.plan(desc, bv)["form"] == "window"
    Tt = torch.tensor(T, device=dev)
    res, loss = torch.empty_like(Tt), torch.empty(b.n_mol, device=dev)
    grad = torch.empty_like(xyz)
    ctx.reversal_step(desc, bv, Tt, res, loss, grad, None, 0.0)
    torch.cuda.synchronize()
    keep = ~band
    rel_r, _ = errors(res.cpu().numpy()[keep], U_o[keep])
    rel_l = float(np.max(np.abs(loss.cpu().numpy() - loss_o) / loss_o))
    rel_g, _ = errors(grad.cpu().numpy(), grad_o)
    say(f"[sphere reversal] residual rel-L2 {rel_r:.3e} (band {int(band.sum())}), loss "
        f"max-rel {rel_l:.3e}, grad rel-L2 {rel_g:.3e}")
    assert rel_r <= F32_TOL and rel_g <= ADJ_TOL
    if not band.any():
        assert rel_l <= F32_TOL
