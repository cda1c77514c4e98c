"""GPU parity of the request options in combination, through the C ABI,
against the oracle: each option (voxel value, cutoff shape, cell, weighted
channels) is tested on its own elsewhere; here they meet -- sphere with
weights, box with weights in a periodic cell, triclinic cells with the box
value and with the sphere, and a reversal step on a weighted box request.
"""
import numpy as np
import pytest

from gpu_util import errors, oracle, say, synth, to_device
from oracle import reversal, sphere, triclinic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F32_TOL = 1e-5
ADJ_TOL = 1e-4
SHEAR = np.array([[8.0, 2.5, 1.0], [0.0, 7.5, -1.5], [0.0, 0.0, 8.5]])


@pytest.fixture(scope="module")
def pg():
    import paper_2211_08506_amd as pg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pg


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def check(name, got, ref, keep=None, tol=F32_TOL):
    got = got.double().cpu().numpy()
    if keep is not None:
        got, ref = got[keep], ref[keep]
    rel, mx = errors(got, ref)
    say(f"[{name}] rel-L2 {rel:.3e} max-abs {mx:.3e}")
    assert rel <= tol and np.array_equal(got > 0, ref > 0), name


@pytest.mark.parametrize("form", ["window", "plain"])
def test_sphere_with_weights(pg, dev, form):
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(24)
    rng = np.random.default_rng(81)
    E = rng.uniform(0.1, 1.0, size=(b.n_atoms, 3)).astype(np.float32)
    say(f"case sphere + weights form={form}")
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing, wl.origin,
                           weights=E, cutoff_shape="sphere")
    band = sphere.edge_band(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing,
                            wl.origin).any(axis=1, keepdims=True)
    band = np.broadcast_to(band, ref.shape)
    xyz, types, offs = to_device(b, dev)
    g = pg.grid(xyz, types, offs, list(wl.sigma()), dims=wl.dims, spacing=wl.spacing,
                origin=wl.origin, form=form, weights=torch.tensor(E, device=dev),
                cutoff_shape="sphere")
    torch.cuda.synchronize()
    check(f"sphere+weights/{form}", g, ref, ~band)


def test_box_weights_periodic_with_gradients(pg, dev):
    sig = synth.sigma_table(4, 0.3, 0.5)
    rng = np.random.default_rng(82)
    off = np.array([0, 14, 30], np.int32)
    xyz = rng.uniform(0, 8.0, size=(30, 3)).astype(np.float32)
    types = rng.integers(0, 4, 30).astype(np.int32)
    E = rng.standard_normal((30, 2)).astype(np.float32)
    dims, h = (30, 28, 32), 0.27
    say("case box + weights + periodic cell, forward and gradients")
    ref = oracle.grid_fp64(xyz, types, off, sig, dims, h, (0, 0, 0), cell=8.0, value="box",
                           weights=E)
    U = synth.upstream(83, (2, 2) + dims)
    gx_o, gw_o = oracle.grad_fp64(xyz, types, off, sig, dims, h, U, (0, 0, 0), cell=8.0,
                                  value="box", weights=E, return_weight_grad=True)
    x = torch.tensor(xyz, device=dev, requires_grad=True)
    Et = torch.tensor(E, device=dev, requires_grad=True)
    g = pg.grid(x, torch.tensor(types, device=dev), torch.tensor(off, device=dev), list(sig),
                dims=dims, spacing=h, cell=8.0, value="box", weights=Et)
    g.backward(torch.tensor(U, device=dev))
    torch.cuda.synchronize()
    check("box+weights+cell", g.detach(), ref)
    rx, _ = errors(x.grad.cpu().numpy(), gx_o)
    rw, _ = errors(Et.grad.cpu().numpy(), gw_o)
    say(f"[box+weights+cell grads] xyz rel-L2 {rx:.3e}, weights rel-L2 {rw:.3e}")
    assert rx <= ADJ_TOL and rw <= ADJ_TOL


@pytest.mark.parametrize("value,shape", [("box", "cube"), ("point", "sphere")])
def test_triclinic_with_value_and_shape(pg, dev, value, shape):
    sig = synth.sigma_table(3, 0.35, 0.55)
    rng = np.random.default_rng(84)
    f = rng.uniform(0, 1, size=(9, 3))
    xyz = (f @ SHEAR.T).astype(np.float32)
    types = rng.integers(0, 3, 9).astype(np.int32)
    off = np.array([0, 4, 9], np.int32)
    dims, h, o = (32, 30, 34), 0.28, (-0.5, 0.0, -1.0)
    say(f"case triclinic value={value} shape={shape}")
    ref = triclinic.grid_triclinic_fp64(xyz, types, off, sig, dims, h, SHEAR, o, value=value,
                                        cutoff_shape=shape)
    keep = None
    if shape == "sphere":
        # the edge band of every image the oracle expands
        rc = float(np.max(np.float32(3.0) * sig))
        xi, ti, oi, _ = triclinic.expand(xyz, types, off, SHEAR, dims, h, o, rc)
        keep = ~sphere.edge_band(xi, ti, oi, sig, dims, h, o)
    x = torch.tensor(xyz, device=dev, requires_grad=True)
    g = pg.grid(x, torch.tensor(types, device=dev), torch.tensor(off, device=dev), list(sig),
                dims=dims, spacing=h, origin=o, cell=SHEAR, value=value, cutoff_shape=shape)
    torch.cuda.synchronize()
    check(f"triclinic/{value}/{shape}", g.detach(), ref, keep)
    U = synth.upstream(85, (2, 3) + dims)
    g.backward(torch.tensor(U, device=dev))
    torch.cuda.synchronize()
    gref = triclinic.grad_triclinic_fp64(xyz, types, off, sig, dims, h, U, SHEAR, o, value=value,
                                         cutoff_shape=shape)
    rel, _ = errors(x.grad.cpu().numpy(), gref)
    say(f"[triclinic/{value}/{shape} gradient] rel-L2 {rel:.3e}")
    assert rel <= ADJ_TOL


def test_reversal_step_weighted_box(pg, dev):
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(12)
    rng = np.random.default_rng(86)
    E = rng.uniform(0.2, 1.0, size=(b.n_atoms, 5)).astype(np.float32)
    T = oracle.grid_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing, wl.origin,
                         value="box", weights=E).astype(np.float32)
    x0 = (b.xyz + rng.uniform(-0.1, 0.1, size=b.xyz.shape)).astype(np.float32)
    say("case reversal step, weighted box request")
    loss_o, U_o, grad_o, _ = reversal.reversal_step(x0, b.types, b.offsets, wl.sigma(), wl.dims,
                                                    wl.spacing, T, 1.0, wl.origin, value="box",
                                                    weights=E)
    ctx = pg.Context(0)
    desc = pg.make_desc(5, wl.dims, wl.spacing, wl.origin, wl.sigma(), 3.0, None, value="box",
                        n_types=5)
    xyz, types, offs = to_device(synth.Batch(x0, b.types, b.offsets), dev)
    bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets,
                      weights=torch.tensor(E, device=dev))
    Tt = torch.tensor(T, device=dev)
    res, loss = torch.empty_like(Tt), torch.empty(b.n_mol, device=dev)
    grad = torch.empty_like(xyz)
    ctx.reversal_step(desc, bv, Tt, res, loss, grad, None, 0.0)
    torch.cuda.synchronize()
    rel_r, _ = errors(res.cpu().numpy(), U_o)
    rel_l = float(np.max(np.abs(loss.cpu().numpy() - loss_o) / loss_o))
    rel_g, _ = errors(grad.cpu().numpy(), grad_o)
    say(f"[reversal weighted box] residual {rel_r:.3e}, loss {rel_l:.3e}, grad {rel_g:.3e}")
    assert rel_r <= F32_TOL and rel_l <= F32_TOL and rel_g <= ADJ_TOL
