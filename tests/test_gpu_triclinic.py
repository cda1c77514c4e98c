"""GPU parity of triclinic periodic cells (§III-A lattice translations for a
general cell) through the C ABI, against the oracle's triclinic map: small
cells on the molecule window form, large cells on both binned forms, a
diagonal cell against the orthorhombic path, the coordinate gradient, and
graph replay.

Image positions are computed identically on both sides (the reading), so the
support matches voxel for voxel; bars as elsewhere: FP32 rel-L2 <= 1e-5,
BF16 / MFMA <= 1e-2, gradient <= 1e-4.
"""
import numpy as np
import pytest

from gpu_util import errors, oracle, say, synth, to_device, worst_molecule
from oracle import triclinic

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F32_TOL = 1e-5
BF16_TOL = 1e-2
ADJ_TOL = 1e-4
SHEAR = np.array([[8.0, 2.5, 1.0], [0.0, 7.5, -1.5], [0.0, 0.0, 8.5]])
SKEW = np.array([[9.1, -2.3, 1.7], [0.4, 8.2, -2.9], [-0.6, 1.1, 8.8]])


@pytest.fixture(scope="module")
def pg():
    import paper_2211_08506_amd as pg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pg


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def cells(seed, counts, M, n_types):
    """Atoms uniform in the cell (fractional coordinates in [0, 1)), some
    moved by lattice vectors so that they sit outside the home cell."""
    rng = np.random.default_rng(seed)
    n = int(sum(counts))
    f = rng.uniform(0, 1, size=(n, 3))
    f[::7] += rng.integers(-2, 3, size=(len(f[::7]), 3))
    xyz = (f @ np.asarray(M, np.float64).T).astype(np.float32)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    return synth.Batch(xyz, rng.integers(0, n_types, n).astype(np.int32), off)


def run(pg, dev, b, sig, dims, h, origin, M, dtype=torch.float32, form="auto"):
    xyz, types, offs = to_device(b, dev)
    g = pg.grid(xyz, types, offs, list(sig), dims=dims, spacing=h, origin=origin, cell=M,
                out_dtype=dtype, form=form)
    torch.cuda.synchronize()
    return g


def check(name, g, ref, tol):
    got = g.double().cpu().numpy()
    rel, mx = errors(got, ref)
    wm = worst_molecule(got, ref)
    say(f"[triclinic {name}] rel-L2 {rel:.3e} max-abs {mx:.3e} worst-structure {wm:.3e}")
    assert rel <= tol and wm <= tol, name
    assert np.array_equal(got > 0, ref > 0), name


@pytest.mark.parametrize("M", [SHEAR, SKEW], ids=["shear", "skew"])
def test_small_cells_window_form(pg, dev, M):
    sig = synth.sigma_table(3, 0.35, 0.55)
    b = cells(61, [3, 5, 0, 4], M, 3)
    dims, h, o = (36, 34, 40), 0.27, (-1.0, -0.5, -1.5)
    say(f"case triclinic small cells {dims}")
    plan = pg.default_context(dev).plan(
        pg.make_desc(3, dims, h, o, sig, 3.0, M), pg.BatchView(*to_device(b, dev)))
    assert plan["binned"] == 0 and plan["form"] == "window", plan
    ref = triclinic.grid_triclinic_fp64(b.xyz, b.types, b.offsets, sig, dims, h, M, o)
    for dt, tol in ((torch.float32, F32_TOL), (torch.bfloat16, BF16_TOL)):
        check(f"small/{dt}", run(pg, dev, b, sig, dims, h, o, M, dt), ref, tol)
    check("small/plain", run(pg, dev, b, sig, dims, h, o, M, torch.float32, "plain"), ref,
          F32_TOL)


def test_large_cells_binned_forms(pg, dev):
    sig = synth.sigma_table(3, 0.3, 0.45)
    b = cells(62, [300, 180], SHEAR, 3)
    dims, h, o = (40, 44, 48), 0.21, (0.0, -0.3, 0.2)
    ref = triclinic.grid_triclinic_fp64(b.xyz, b.types, b.offsets, sig, dims, h, SHEAR, o)
    for form, dt, tol in (("window", torch.float32, F32_TOL), ("mfma", torch.bfloat16, BF16_TOL),
                          ("mfma", torch.float32, F32_TOL)):
        say(f"case triclinic large cells form={form}")
        check(f"large/{form}", run(pg, dev, b, sig, dims, h, o, SHEAR, dt, form), ref, tol)


def test_diagonal_cell_matches_the_orthorhombic_path(pg, dev):
    sig = synth.sigma_table(3, 0.35, 0.55)
    rng = np.random.default_rng(63)
    xyz = rng.uniform(0, 8, size=(9, 3)).astype(np.float32)
    b = synth.Batch(xyz, rng.integers(0, 3, 9).astype(np.int32), np.array([0, 4, 9], np.int32))
    dims, h = (32, 32, 32), 0.25
    say("case triclinic diagonal cell vs orthorhombic")
    g_tri = run(pg, dev, b, sig, dims, h, (0, 0, 0), np.diag([8.0] * 3))
    g_ort = run(pg, dev, b, sig, dims, h, (0, 0, 0), 8.0)
    rel, _ = errors(g_tri.double().cpu().numpy(), g_ort.double().cpu().numpy())
    say(f"[triclinic diagonal vs orthorhombic] rel-L2 {rel:.3e}")
    assert rel <= F32_TOL


def test_triclinic_gradient(pg, dev):
    sig = synth.sigma_table(3, 0.35, 0.55)
    b = cells(64, [4, 6], SKEW, 3)
    dims, h, o = (30, 30, 32), 0.3, (-0.5, -0.5, -0.5)
    U = synth.upstream(65, (2, 3) + dims)
    say("case triclinic gradient")
    ref = triclinic.grad_triclinic_fp64(b.xyz, b.types, b.offsets, sig, dims, h, U, SKEW, o)
    xyz, types, offs = to_device(b, dev)
    xyz.requires_grad_(True)
    g = pg.grid(xyz, types, offs, list(sig), dims=dims, spacing=h, origin=o, cell=SKEW)
    g.backward(torch.tensor(U, device=dev))
    torch.cuda.synchronize()
    rel, mx = errors(xyz.grad.cpu().numpy(), ref)
    say(f"[triclinic gradient] rel-L2 {rel:.3e} max-abs {mx:.3e}")
    assert rel <= ADJ_TOL


def test_triclinic_graph_replay(pg, dev):
    sig = synth.sigma_table(3, 0.35, 0.55)
    b = cells(66, [5, 3], SHEAR, 3)
    dims, h, o = (32, 32, 32), 0.28, (0.0, 0.0, 0.0)
    ref = triclinic.grid_triclinic_fp64(b.xyz, b.types, b.offsets, sig, dims, h, SHEAR, o)
    xyz, types, offs = to_device(b, dev)
    ctx = pg.Context(0)
    desc = pg.make_desc(3, dims, h, o, sig, 3.0, SHEAR)
    bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets)
    out = pg.empty_grid(desc, b.n_mol, dev)
    ctx.set_option(pg.PG_OPT_GRAPH, 1)
    say("case triclinic graph replay")
    for r in range(3):
        out.fill_(float("nan"))
        ctx.forward(desc, bv, out)
        torch.cuda.synchronize()
        check(f"graph rep {r}", out, ref, F32_TOL)
    assert ctx.device_error()[0] == 0


@pytest.mark.parametrize("M", [SHEAR, SKEW], ids=["shear-dyadic", "skew"])
def test_image_positions_are_the_oracles_bit_for_bit(pg, dev, M):
    """Image positions are the exact lattice sums rounded once to float32 on
    both sides.  With one atom per structure a voxel sees at most one image,
    so the triclinic grid must equal, bit for bit, the non-periodic grid over
    the oracle's images: a position one ulp off moves its window or its
    values.  The dyadic shear cell makes exact ties frequent (sums crossing
    a binade); the skew cell's entries are not dyadic."""
    rng = np.random.default_rng(64)
    n = 96
    f = rng.uniform(-0.3, 1.3, size=(n, 3))
    xyz = (f @ np.asarray(M, np.float64).T).astype(np.float32)
    b = synth.Batch(xyz, rng.integers(0, 3, n).astype(np.int32), np.arange(n + 1, dtype=np.int32))
    sig = synth.sigma_table(3, 0.35, 0.55)
    dims, h, o = (20, 24, 28), 0.3, (0.5, -0.25, 1.0)
    rc_max = float(np.max(np.float32(3.0) * np.asarray(sig, np.float32)))
    xi, ti, oi, _ = triclinic.expand(b.xyz, b.types, b.offsets, M, dims, h, o, rc_max)
    imgs = synth.Batch(xi, ti, oi.astype(np.int32))
    say(f"case triclinic image positions {M[0, 1]} ({len(xi)} oracle images)")
    g_tri = run(pg, dev, b, sig, dims, h, o, M, form="window")
    g_img = run(pg, dev, imgs, sig, dims, h, o, None, form="window")
    assert torch.equal(g_tri, g_img)
