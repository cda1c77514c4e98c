"""GPU parity of weighted channels (atom a adds weights[a, c] times its
Gaussian to every channel c; the learned-embedding grids of the paper's
Discussion) through the C ABI: one-hot weights against the unweighted path
bit for bit, dense signed weights with more types than channels against the
oracle, the weight and coordinate gradients against the oracle's, a learned
embedding table trained through torch autograd, and a sampled full-size
batch.

Bars: FP32 rel-L2 <= 1e-5, BF16 <= 1e-2, gradients <= 1e-4.
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


def one_hot(types, C):
    E = np.zeros((len(types), C), np.float32)
    E[np.arange(len(types)), types] = 1.0
    return E


@pytest.mark.parametrize("form", ["window", "plain"])
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("value", ["point", "box"])
def test_one_hot_weights_are_bitwise_the_unweighted_grid(pg, dev, form, dtype, value):
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(32)
    say(f"case one-hot weights form={form} dtype={dtype} value={value}")
    xyz, types, offs = to_device(b, dev)
    kw = dict(dims=wl.dims, spacing=wl.spacing, origin=wl.origin, out_dtype=dtype, form=form,
              value=value)
    g0 = pg.grid(xyz, types, offs, list(wl.sigma()), **kw)
    E = torch.tensor(one_hot(b.types, 5), device=dev)
    g1 = pg.grid(xyz, types, offs, list(wl.sigma()), weights=E, **kw)
    torch.cuda.synchronize()
    assert torch.equal(g0, g1)


@pytest.mark.parametrize("form", ["window", "plain"])
@pytest.mark.parametrize("value", ["point", "box"])
def test_dense_weights_more_types_than_channels(pg, dev, form, value):
    rng = np.random.default_rng(21)
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(40)
    types = rng.integers(0, 8, b.n_atoms).astype(np.int32)
    sig = synth.sigma_table(8, 0.35, 0.7)
    E = rng.standard_normal((b.n_atoms, 3)).astype(np.float32)
    E[rng.random(E.shape) < 0.3] = 0.0            # some exact zeros
    say(f"case dense weights 8 types -> 3 channels form={form} value={value}")
    ref = oracle.grid_fp64(b.xyz, types, b.offsets, sig, wl.dims, wl.spacing, wl.origin,
                           value=value, weights=E)
    xyz = torch.tensor(b.xyz, device=dev)
    offs = torch.tensor(b.offsets, device=dev)
    tt = torch.tensor(types, device=dev)
    Et = torch.tensor(E, device=dev)
    for dt, tol in ((torch.float32, F32_TOL), (torch.bfloat16, BF16_TOL)):
        g = pg.grid(xyz, tt, offs, list(sig), dims=wl.dims, spacing=wl.spacing, origin=wl.origin,
                    out_dtype=dt, form=form, value=value, weights=Et)
        torch.cuda.synchronize()
        got = g.double().cpu().numpy()
        rel, mx = errors(got, ref)
        wm = worst_molecule(got, ref)
        say(f"[weighted {form}/{value}/{dt}] rel-L2 {rel:.3e} max-abs {mx:.3e} worst {wm:.3e}")
        assert rel <= tol and wm <= tol


@pytest.mark.parametrize("value", ["point", "box"])
def test_weighted_gradients_against_oracle(pg, dev, value):
    rng = np.random.default_rng(22)
    wl = synth.WORKLOADS["adjoint1024"]
    b = wl.batch(24)
    types = rng.integers(0, 6, b.n_atoms).astype(np.int32)
    sig = synth.sigma_table(6)
    E = rng.standard_normal((b.n_atoms, 4)).astype(np.float32)
    U = synth.upstream(23, (b.n_mol, 4) + tuple(wl.dims))
    say(f"case weighted gradients value={value}")
    gx_o, gw_o = oracle.grad_fp64(b.xyz, types, b.offsets, sig, wl.dims, wl.spacing, U,
                                  wl.origin, value=value, weights=E, return_weight_grad=True)
    xyz = torch.tensor(b.xyz, device=dev, requires_grad=True)
    Et = torch.tensor(E, device=dev, requires_grad=True)
    g = pg.grid(xyz, torch.tensor(types, device=dev), torch.tensor(b.offsets, device=dev),
                list(sig), dims=wl.dims, spacing=wl.spacing, origin=wl.origin, value=value,
                weights=Et)
    g.backward(torch.tensor(U, device=dev))
    torch.cuda.synchronize()
    rx, _ = errors(xyz.grad.cpu().numpy(), gx_o)
    rw, mw = errors(Et.grad.cpu().numpy(), gw_o)
    say(f"[weighted grads {value}] xyz rel-L2 {rx:.3e}, weights rel-L2 {rw:.3e} (max-abs {mw:.3e})")
    assert rx <= ADJ_TOL and rw <= ADJ_TOL


def test_learned_embedding_table_through_autograd(pg, dev):
    """weights = table[types] for a (T x C) table: its gradient is the
    oracle's weight gradient summed by type."""
    rng = np.random.default_rng(24)
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(16)
    T, C = 5, 4
    table = rng.standard_normal((T, C)).astype(np.float32)
    U = synth.upstream(25, (b.n_mol, C) + tuple(wl.dims))
    say("case learned embedding table")
    _, gw_o = oracle.grad_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing, U,
                               wl.origin, weights=table[b.types], return_weight_grad=True)
    want = np.zeros((T, C))
    np.add.at(want, b.types, gw_o)
    xyz, types, offs = to_device(b, dev)
    tab = torch.tensor(table, device=dev, requires_grad=True)
    g = pg.grid(xyz, types, offs, list(wl.sigma()), dims=wl.dims, spacing=wl.spacing,
                origin=wl.origin, weights=tab[types.long()])
    (g * torch.tensor(U, device=dev)).sum().backward()
    torch.cuda.synchronize()
    rel, _ = errors(tab.grad.cpu().numpy(), want)
    say(f"[embedding table grad] rel-L2 {rel:.3e}")
    assert rel <= ADJ_TOL


def test_weighted_full_size_sampled(pg, dev):
    """The 4096-molecule 32^3 x 5 batch in bf16 with an embedding of the 5
    types into 5 channels, sampled voxels against the oracle."""
    wl = synth.WORKLOADS["mol4096"]
    b = wl.batch()
    rng = np.random.default_rng(26)
    table = rng.uniform(-0.5, 1.5, size=(5, 5)).astype(np.float32)
    E = table[b.types]
    say("case weighted full-size mol4096 bf16")
    xyz, types, offs = to_device(b, dev)
    g = pg.grid(xyz, types, offs, list(wl.sigma()), dims=wl.dims, spacing=wl.spacing,
                origin=wl.origin, out_dtype=torch.bfloat16, weights=torch.tensor(E, device=dev))
    torch.cuda.synchronize()
    idx = sample_voxels(rng, b, tuple(g.shape), wl.origin, wl.spacing, 20000, 20000)
    ref = oracle.voxels_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing, idx,
                             wl.origin, weights=E)
    it = torch.tensor(idx, device=dev)
    got = g[it[:, 0], it[:, 1], it[:, 2], it[:, 3], it[:, 4]].double().cpu().numpy()
    rel, mx = errors(got, ref)
    say(f"[weighted mol4096 sampled {len(idx)}] rel-L2 {rel:.3e} max-abs {mx:.3e}")
    assert rel <= BF16_TOL


@pytest.mark.parametrize("form,dtype,tol", [("window", torch.float32, F32_TOL),
                                            ("mfma", torch.bfloat16, BF16_TOL),
                                            ("mfma", torch.float32, F32_TOL)])
def test_weighted_binned_path(pg, dev, form, dtype, tol):
    """Periodic cells above the window kernel's capacity, 6 types into 3
    channels with signed weights (some exactly zero): the binned path lists
    each atom under every channel it weighs into, with the width of its
    type; the MFMA form folds the weight into its phi_y operand."""
    rng = np.random.default_rng(27)
    off = np.array([0, 400, 700], np.int32)
    xyz = rng.uniform(0, 8, size=(700, 3)).astype(np.float32)
    types = rng.integers(0, 6, 700).astype(np.int32)
    sig = synth.sigma_table(6, 0.3, 0.45)
    E = rng.standard_normal((700, 3)).astype(np.float32)
    E[rng.random(E.shape) < 0.3] = 0.0
    dims, h = (40, 40, 40), 0.21
    say(f"case weighted binned path form={form} dtype={dtype}")
    ref = oracle.grid_fp64(xyz, types, off, sig, dims, h, (0, 0, 0), cell=8.0, weights=E)
    x = torch.tensor(xyz, device=dev, requires_grad=True)
    Et = torch.tensor(E, device=dev, requires_grad=True)
    t, o = torch.tensor(types, device=dev), torch.tensor(off, device=dev)
    desc = pg.make_desc(3, dims, h, (0, 0, 0), sig, 3.0, 8.0, dtype, form, n_types=6)
    plan = pg.default_context(dev).plan(desc, pg.BatchView(x.detach(), t, o, weights=Et.detach()))
    assert plan["binned"] == 1 and plan["form"] == form, plan
    g = pg.grid(x, t, o, list(sig), dims=dims, spacing=h, cell=8.0, out_dtype=dtype, form=form,
                weights=Et)
    torch.cuda.synchronize()
    got = g.detach().double().cpu().numpy()
    rel, mx = errors(got, ref)
    wm = worst_molecule(got, ref)
    say(f"[weighted binned {form}/{dtype}] rel-L2 {rel:.3e} max-abs {mx:.3e} worst {wm:.3e}")
    assert rel <= tol and wm <= tol
    # gradients through the (one wave per atom) adjoint
    U = synth.upstream(28, (2, 3) + dims)
    g.backward(torch.tensor(U, device=dev).to(g.dtype))
    torch.cuda.synchronize()
    Uused = torch.tensor(U, device=dev).to(g.dtype).double().cpu().numpy()
    gx_o, gw_o = oracle.grad_fp64(xyz, types, off, sig, dims, h, Uused, (0, 0, 0), cell=8.0,
                                  weights=E, return_weight_grad=True)
    rx, _ = errors(x.grad.cpu().numpy(), gx_o)
    rw, _ = errors(Et.grad.cpu().numpy(), gw_o)
    say(f"[weighted binned grads] xyz {rx:.3e}, weights {rw:.3e}")
    assert rx <= ADJ_TOL and rw <= ADJ_TOL


@pytest.mark.parametrize("scale", [1e-6, 1e5])
def test_weighted_split_mfma_weight_range(pg, dev, scale):
    """The MFMA form for float32 grids with weights of 1e-6 or 1e5 (far from
    1 once multiplied into phi_z), mixed in sign and spread over three
    decades within a channel: FP32 operands and accumulation keep the
    result at the FP32 bar (a check kept from an earlier fp16-split operand
    form, whose per-plane power-of-two scaling it guarded)."""
    rng = np.random.default_rng(29)
    off = np.array([0, 400, 700], np.int32)
    xyz = rng.uniform(0, 8, size=(700, 3)).astype(np.float32)
    types = rng.integers(0, 4, 700).astype(np.int32)
    sig = synth.sigma_table(4, 0.3, 0.45)
    E = (rng.standard_normal((700, 3)) * 10.0 ** rng.uniform(-1.5, 1.5, (700, 3)) * scale)
    E = E.astype(np.float32)
    dims, h = (40, 40, 40), 0.21
    say(f"case split MFMA weight range scale={scale:g}")
    ref = oracle.grid_fp64(xyz, types, off, sig, dims, h, (0, 0, 0), cell=8.0, weights=E)
    g = pg.grid(torch.tensor(xyz, device=dev), torch.tensor(types, device=dev),
                torch.tensor(off, device=dev), list(sig), dims=dims, spacing=h, cell=8.0,
                out_dtype=torch.float32, form="mfma", weights=torch.tensor(E, device=dev))
    torch.cuda.synchronize()
    got = g.double().cpu().numpy()
    assert np.isfinite(got).all()
    rel, mx = errors(got, ref)
    wm = worst_molecule(got, ref)
    say(f"[split MFMA weights x{scale:g}] rel-L2 {rel:.3e} max-abs {mx:.3e} worst {wm:.3e}")
    assert rel <= F32_TOL and wm <= F32_TOL
