"""GPU parity of the binned large-structure path (structures above the
window kernel's LDS capacity: periodic crystal cells, large clusters)
against the FP64 oracle, through the C ABI.

Bars: the FP32 vector form (form="window" on large structures) to the FP32
bar rel-L2 <= 1e-5; the MFMA form contracts bf16 factors for bf16 grids (BF16
bar rel-L2 <= 1e-2) and FP32 factors on the FP32 matrix instruction for
float32 grids (FP32 bar).
"""
import numpy as np
import pytest

from gpu_util import errors, oracle, sample_voxels, say, synth, to_device, worst_molecule

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F32_TOL = 1e-5
BF16_TOL = 1e-2
# (form, output dtype, tolerance)
CASES = [("window", torch.float32, F32_TOL), ("window", torch.bfloat16, BF16_TOL),
         ("mfma", torch.bfloat16, BF16_TOL), ("mfma", torch.float32, F32_TOL)]


@pytest.fixture(scope="module")
def pg():
    import paper_2211_08506_amd as pg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pg


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def cell_batch(seed, counts, cell, n_types, lo=0.0):
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    xyz = rng.uniform(lo, lo + cell, size=(int(off[-1]), 3)).astype(np.float32)
    return synth.Batch(xyz, rng.integers(0, n_types, int(off[-1])).astype(np.int32), off)


def run(pg, dev, b, sig, dims, h, origin, dtype, form, cell=None, ctx=None):
    xyz, types, offs = to_device(b, dev)
    g = pg.grid(xyz, types, offs, list(sig), dims=dims, spacing=h, origin=origin, cell=cell,
                out_dtype=dtype, form=form, ctx=ctx)
    torch.cuda.synchronize()
    return g


def plan_of(pg, dev, b, sig, dims, h, origin, dtype, form, cell=None, ctx=None):
    xyz, types, offs = to_device(b, dev)
    ctx = ctx or pg.default_context(dev)
    desc = pg.make_desc(len(sig), dims, h, origin, sig, 3.0, cell, dtype, form)
    bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets)
    return ctx.plan(desc, bv, pg.empty_grid(desc, b.n_mol, dev))


def check(name, g, ref, tol):
    got = g.double().cpu().numpy()
    rel, mx = errors(got, ref)
    wm = worst_molecule(got, ref)
    say(f"[{name}] rel-L2 {rel:.3e}  max-abs {mx:.3e}  worst-structure rel-L2 {wm:.3e}")
    assert rel <= tol and wm <= tol, name
    # the cube cutoff is decided exactly: the support matches voxel for voxel
    assert np.array_equal(got > 0, ref > 0), name
    return got


@pytest.mark.parametrize("dims,h", [((24, 24, 24), 1.0 / 3.0), ((40, 40, 40), 0.21)])
def test_periodic_cells(pg, dev, dims, h):
    """Cells of 400 and 300 atoms (above the window kernel's capacity) with
    the grid equal to the cell and larger than the cell (atoms near a face
    seen through two images per axis; a third needs a grid exactly
    2L - 2rc wide)."""
    sig = synth.sigma_table(3, 0.3, 0.45)
    b = cell_batch(31, [400, 300], 8.0, 3)
    b.xyz[0] = [0.01, 7.99, 4.0]               # atoms at the faces
    b.xyz[1] = [7.999, 0.0, 0.0]
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, dims, h, (0, 0, 0), cell=8.0)
    for form, dt, tol in CASES:
        say(f"case periodic {dims} h={h:.4f} form={form} dtype={dt}")
        plan = plan_of(pg, dev, b, sig, dims, h, (0, 0, 0), dt, form, cell=8.0)
        assert plan["binned"] == 1 and plan["form"] == form, plan
        g = run(pg, dev, b, sig, dims, h, (0, 0, 0), dt, form, cell=8.0)
        check(f"periodic{dims}/{form}/{dt}", g, ref, tol)


def test_periodic_small_grid_in_large_cell(pg, dev):
    """A 28 x 24 x 20 grid at 0.41 A inside 24 A periodic cells, its origin
    offset so that it crosses the cell faces on y and z: most of an atom's
    candidate lattice images lie far outside the grid and are dropped by the
    window search's float estimate before its exact tests.  Every form
    matches the oracle, support voxel for voxel."""
    sig = synth.sigma_table(3, 0.3, 0.45)
    b = cell_batch(37, [500, 350], 24.0, 3)
    dims, h, origin = (20, 24, 28), 0.41, (7.0, -3.0, 20.5)
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, dims, h, origin, cell=24.0)
    assert ref[:, :, :, :3].sum() > 0 and ref[:, :, -3:].sum() > 0   # images across the faces
    for form, dt, tol in CASES:
        say(f"case small grid in large cell form={form} dtype={dt}")
        g = run(pg, dev, b, sig, dims, h, origin, dt, form, cell=24.0)
        check(f"subgrid/{form}/{dt}", g, ref, tol)


@pytest.mark.parametrize("dims", [(20, 37, 45), (6, 150, 140), (9, 16, 200), (4, 300, 320)])
def test_ragged_planes_large_cluster(pg, dev, dims):
    """Non-periodic clusters of 300-700 atoms on planes that are not whole
    32 x 32 tiles: ragged tile rows and columns (partial tiles stored with
    bounds tests, partial factor slots), many tiles per plane, an empty
    structure in the batch; planes wider than 32 tiles are refused by the
    vector form and served by the MFMA form."""
    sig = synth.sigma_table(4, 0.35, 0.6)
    b = cell_batch(32, [300, 0, 700], 6.0, 4, lo=-3.0)
    h = 0.17
    D, H, W = dims
    origin = (-0.5 * W * h, -0.5 * H * h, -0.5 * D * h)
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, dims, h, origin)
    wide = ((H + 31) // 32) * ((W + 31) // 32) > 32
    for form, dt, tol in CASES:
        if wide and form == "window":
            # the binned vector form holds at most 32 tiles of 32 x 32 per plane
            with pytest.raises(pg.PGError) as ei:
                plan_of(pg, dev, b, sig, dims, h, origin, dt, form)
            assert ei.value.status == pg.PG_E_UNSUPPORTED
            continue
        say(f"case cluster {dims} form={form} dtype={dt}")
        g = run(pg, dev, b, sig, dims, h, origin, dt, form)
        got = check(f"cluster{dims}/{form}/{dt}", g, ref, tol)
        assert not got[1].any()


@pytest.mark.parametrize("dtype,tol", [(torch.bfloat16, BF16_TOL), (torch.float32, F32_TOL)])
def test_mfma_many_and_few_runs(pg, dev, dtype, tol):
    """The MFMA form on many runs (40 periodic cells x 8 channels = 320
    (structure, channel) runs, more than the chip has CUs) and on few (the
    first 5 cells: 40 runs): both match the oracle, voxel support included,
    and are bitwise reproducible."""
    sig = synth.sigma_table(8, 0.3, 0.5)
    counts = [300 + 7 * i for i in range(40)]
    b = cell_batch(35, counts, 8.0, 8)
    dims, h = (16, 24, 32), 0.25
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, dims, h, (0, 0, 0), cell=8.0)
    m5 = int(b.offsets[5])
    few = synth.Batch(b.xyz[:m5], b.types[:m5], b.offsets[:6])
    for name, bb, rr in (("many", b, ref), ("few", few, ref[:5])):
        say(f"case mfma {name} runs dtype={dtype}")
        g = run(pg, dev, bb, sig, dims, h, (0, 0, 0), dtype, "mfma", cell=8.0)
        check(f"runs-{name}/{dtype}", g, rr, tol)
        again = run(pg, dev, bb, sig, dims, h, (0, 0, 0), dtype, "mfma", cell=8.0)
        assert torch.equal(g, again), name


@pytest.mark.parametrize("dtype,tol", [(torch.bfloat16, BF16_TOL), (torch.float32, F32_TOL)])
def test_mfma_other_stream_and_graph_replay(pg, dev, dtype, tol):
    """The MFMA form's launch sequence (prep, scans, partition, factor
    slots, tile sort, tile kernel): the eager result matches the oracle, and
    a run on another caller stream and replays of the captured graph (eager
    work and synchronisation between them) reproduce it bit for bit."""
    say(f"case mfma other stream and graph replay dtype={dtype}")
    sig = synth.sigma_table(3, 0.3, 0.45)
    b = cell_batch(41, [900, 1500, 600], 10.0, 3)
    dims, h = (48, 48, 48), 10.0 / 48
    xyz, types, offs = to_device(b, dev)
    ctx = pg.Context(0)
    desc = pg.make_desc(3, dims, h, (0, 0, 0), sig, 3.0, 10.0, dtype, "mfma")
    bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets)
    eager = pg.empty_grid(desc, b.n_mol, dev)
    ctx.forward(desc, bv, eager)
    torch.cuda.synchronize()
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, dims, h, (0, 0, 0), cell=10.0)
    check(f"mfma eager/{dtype}", eager, ref, tol)
    s = torch.cuda.Stream(dev)
    other = pg.empty_grid(desc, b.n_mol, dev)
    other.fill_(float("nan"))
    s.wait_stream(torch.cuda.current_stream(dev))
    ctx.forward(desc, bv, other, stream=s)
    s.synchronize()
    assert torch.equal(other, eager)
    ctx.set_option(pg.PG_OPT_GRAPH, 1)
    try:
        out = pg.empty_grid(desc, b.n_mol, dev)
        for rep in range(4):
            out.fill_(float("nan"))
            ctx.forward(desc, bv, out)
            torch.cuda.synchronize()
            junk = torch.randn(1 << 20, device=dev).sum()      # eager work between replays
            torch.cuda.synchronize()
            assert torch.equal(out, eager), f"replay {rep}"
            del junk
    finally:
        ctx.set_option(pg.PG_OPT_GRAPH, 0)
    assert ctx.device_error()[0] == 0


def test_auto_form_rule(pg, dev):
    """AUTO on large structures: the MFMA form for bf16 and float32 grids;
    small structures keep the one-launch window form."""
    sig = synth.sigma_table(3, 0.3, 0.45)
    big = cell_batch(33, [400], 8.0, 3)
    p = plan_of(pg, dev, big, sig, (24, 24, 24), 1 / 3, (0, 0, 0), torch.bfloat16, "auto", 8.0)
    assert p["binned"] == 1 and p["form"] == "mfma"
    p = plan_of(pg, dev, big, sig, (24, 24, 24), 1 / 3, (0, 0, 0), torch.float32, "auto", 8.0)
    assert p["binned"] == 1 and p["form"] == "mfma"
    small = cell_batch(33, [40], 8.0, 3)
    p = plan_of(pg, dev, small, sig, (24, 24, 24), 1 / 3, (0, 0, 0), torch.float32, "auto", 8.0)
    assert p["binned"] == 0 and p["form"] == "window"


def test_binned_path_agrees_with_small_structure_path(pg, dev):
    """Forced through the binned path, structures the window kernel could
    also take give the same grids within FP32 rounding."""
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(24)
    sig = wl.sigma()
    xyz, types, offs = to_device(b, dev)
    ctx = pg.default_context(dev)
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, wl.dims, wl.spacing, wl.origin)
    desc = pg.make_desc(wl.n_types, wl.dims, wl.spacing, wl.origin, sig, 3.0, None,
                        torch.float32, "window")
    for max_atoms, binned in ((None, 0), (300, 1)):
        bv = pg.BatchView(xyz, types, offs, max_atoms=max_atoms, offsets_host=b.offsets)
        assert ctx.plan(desc, bv)["binned"] == binned
    outs = {}
    for label, max_atoms in (("window", None), ("binned", 300)):
        g = pg.grid(xyz, types, offs, list(sig), dims=wl.dims, spacing=wl.spacing,
                    origin=wl.origin, form="window", max_atoms=max_atoms, ctx=ctx)
        torch.cuda.synchronize()
        outs[label] = check(f"mol256[:24]/{label}", g, ref, F32_TOL)
    rel, _ = errors(outs["binned"], outs["window"])
    assert rel <= 1e-6


def test_determinism(pg, dev):
    """The set-up fixes each plane's image order from the input alone (a
    stable partition by channel, then a stable sort by z-window start), so
    repeated calls are bitwise identical."""
    sig = synth.sigma_table(3, 0.3, 0.45)
    b = cell_batch(34, [900, 500], 8.0, 3)
    for form, dt, _ in CASES:
        say(f"case determinism form={form} dtype={dt}")
        g0 = run(pg, dev, b, sig, (40, 40, 40), 0.21, (0, 0, 0), dt, form, cell=8.0)
        for _ in range(3):
            g1 = run(pg, dev, b, sig, (40, 40, 40), 0.21, (0, 0, 0), dt, form, cell=8.0)
            assert torch.equal(g0, g1), form


@pytest.mark.parametrize("form,dtype,tol", [("window", torch.float32, F32_TOL),
                                            ("mfma", torch.float32, F32_TOL),
                                            ("mfma", torch.bfloat16, BF16_TOL)])
def test_dense_plane_takes_every_image(pg, dev, form, dtype, tol):
    """5000 atoms of one channel within 1 A (about 5000 z images in each of
    their planes, one 32 x 32 tile column): every form takes every image of a
    plane -- no capacity limit, no device error, oracle parity everywhere."""
    rng = np.random.default_rng(35)
    sig = [0.5, 0.5]
    xyz = np.concatenate([rng.uniform(-0.5, 0.5, size=(5000, 3)),
                          rng.uniform(-2, 2, size=(300, 3))]).astype(np.float32)
    types = np.concatenate([np.zeros(5000, np.int32), rng.integers(0, 2, 300).astype(np.int32)])
    b = synth.Batch(xyz, types, np.array([0, 5000, 5300], np.int32))
    dims, h, origin = (24, 24, 24), 0.25, (-3, -3, -3)
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, dims, h, origin)
    say(f"case dense plane form={form} dtype={dtype}")
    ctx = pg.Context(0)
    g = run(pg, dev, b, sig, dims, h, origin, dtype, form, ctx=ctx)
    assert ctx.device_error() == (0, -1)
    check(f"dense/{form}/{dtype}", g, ref, tol)


@pytest.mark.parametrize("dtype,tol", [(torch.bfloat16, BF16_TOL), (torch.float32, F32_TOL)])
def test_full_size_single_channel_cell(pg, dev, dtype, tol):
    """One periodic 20 A cell of 20000 atoms of a single type at 128^3,
    0.16 A, under AUTO (the MFMA form): about 3200 z images per plane, all
    of them in one channel.  Sampled voxels against the oracle, exact
    support, no device error."""
    rng = np.random.default_rng(41)
    n, cell = 20000, 20.0
    xyz = rng.uniform(0.0, cell, size=(n, 3)).astype(np.float32)
    xyz[xyz >= np.float32(cell)] = np.float32(0.0)
    b = synth.Batch(xyz, np.zeros(n, np.int32), np.array([0, n], np.int32))
    sig = [0.55]
    dims, h = (128, 128, 128), 0.16
    say(f"case full-size single-channel cell dtype={dtype}")
    xyz_d, types_d, offs_d = to_device(b, dev)
    ctx = pg.Context(0)
    desc = pg.make_desc(1, dims, h, (0, 0, 0), sig, 3.0, cell, dtype, "auto")
    bv = pg.BatchView(xyz_d, types_d, offs_d, offsets_host=b.offsets)
    out = pg.empty_grid(desc, 1, dev)
    plan = ctx.plan(desc, bv, out)
    say(f"plan {plan}")
    assert plan["form"] == "mfma" and plan["binned"] == 1
    ctx.forward(desc, bv, out)
    torch.cuda.synchronize()
    assert ctx.device_error() == (0, -1)
    idx = sample_voxels(np.random.default_rng(42), b, tuple(out.shape), (0, 0, 0), h, 6000, 6000)
    ref = oracle.voxels_fp64(b.xyz, b.types, b.offsets, sig, dims, h, idx, (0, 0, 0), cell=cell)
    it = torch.tensor(idx, device=dev)
    got = out[it[:, 0], it[:, 1], it[:, 2], it[:, 3], it[:, 4]].double().cpu().numpy()
    rel, mx = errors(got, ref)
    say(f"[single-channel cell/{dtype} sampled {len(idx)}] rel-L2 {rel:.3e} max-abs {mx:.3e}")
    assert rel <= tol
    assert np.array_equal(got > 0, ref > 0)
    assert out.float().sum().item() > 0


def test_adjoint_large_structures(pg, dev):
    """The adjoint kernel has no per-structure capacity: coordinate
    gradients of periodic cells of 400 and 300 atoms against the oracle."""
    sig = synth.sigma_table(3, 0.3, 0.45)
    b = cell_batch(36, [400, 300], 8.0, 3)
    dims, h = (40, 40, 40), 0.21
    U = synth.upstream(37, (2, 3) + dims)
    ref = oracle.grad_fp64(b.xyz, b.types, b.offsets, sig, dims, h, U, (0, 0, 0), cell=8.0)
    xyz, types, offs = to_device(b, dev)
    xyz.requires_grad_(True)
    g = pg.grid(xyz, types, offs, list(sig), dims=dims, spacing=h, origin=(0, 0, 0), cell=8.0)
    g.backward(torch.tensor(U, device=dev))
    torch.cuda.synchronize()
    got = xyz.grad.double().cpu().numpy()
    rel, mx = errors(got, ref)
    say(f"[adjoint cells] rel-L2 {rel:.3e} max-abs {mx:.3e}")
    assert rel <= 1e-4


def test_autotune_picks_a_form_and_persists(pg, dev, tmp_path):
    sig = synth.sigma_table(3, 0.3, 0.45)
    b = cell_batch(38, [900, 500], 8.0, 3)
    xyz, types, offs = to_device(b, dev)
    ctx = pg.Context(0)
    desc = pg.make_desc(3, (40, 40, 40), 0.21, (0, 0, 0), sig, 3.0, 8.0, torch.bfloat16, "auto")
    bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets)
    out = pg.empty_grid(desc, b.n_mol, dev)
    ctx.autotune(desc, bv, out, reps=3)
    plan = ctx.plan(desc, bv, out)
    say(f"tuned large-structure plan {plan}")
    assert plan["binned"] == 1 and plan["form"] in ("mfma", "window")
    ctx.forward(desc, bv, out)
    torch.cuda.synchronize()
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, (40, 40, 40), 0.21, (0, 0, 0),
                           cell=8.0)
    check("autotuned cells", out, ref, BF16_TOL)
    path = str(tmp_path / "tune.json")
    ctx.tuning_save(path)
    ctx2 = pg.Context(0)
    ctx2.tuning_load(path)
    assert ctx2.plan(desc, bv, out) == plan


@pytest.mark.parametrize("form,dtype,tol", [("auto", torch.bfloat16, BF16_TOL),
                                            ("auto", torch.float32, F32_TOL),
                                            ("mfma", torch.float32, F32_TOL),
                                            ("window", torch.float32, F32_TOL),
                                            ("window", torch.bfloat16, BF16_TOL)])
def test_full_size_crystal8_sampled(pg, dev, form, dtype, tol):
    """Eight 20 A cells of 2000-20000 atoms, 8 channels, 128^3 at 0.16 A,
    in the launch configuration the benchmark times (HIP graph): the MFMA
    forms and the FP32 vector ("window") form the crystal comparison is
    made against, at the plane shape it is timed on."""
    wl = synth.WORKLOADS["crystal8"]
    b = wl.batch()
    say(f"case full-size crystal8 form={form} dtype={dtype}")
    xyz, types, offs = to_device(b, dev)
    ctx = pg.default_context(dev)
    desc = pg.make_desc(wl.n_types, wl.dims, wl.spacing, wl.origin, wl.sigma(), wl.cutoff_k,
                        wl.cell, dtype, form)
    bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets)
    out = pg.empty_grid(desc, b.n_mol, dev)
    say(f"plan {ctx.plan(desc, bv, out)}")
    ctx.set_option(pg.PG_OPT_GRAPH, 1)
    try:
        ctx.forward(desc, bv, out)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(pg.PG_OPT_GRAPH, 0)
    assert ctx.device_error()[0] == 0
    rng = np.random.default_rng(19)
    idx = sample_voxels(rng, b, tuple(out.shape), wl.origin, wl.spacing, 20000, 20000)
    ref = oracle.voxels_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing, idx,
                             wl.origin, cutoff_k=wl.cutoff_k, cell=wl.cell)
    it = torch.tensor(idx, device=dev)
    got = out[it[:, 0], it[:, 1], it[:, 2], it[:, 3], it[:, 4]].double().cpu().numpy()
    rel, mx = errors(got, ref)
    say(f"[crystal8/{dtype} sampled {len(idx)}] rel-L2 {rel:.3e} max-abs {mx:.3e}")
    assert rel <= tol
    assert np.array_equal(got > 0, ref > 0)
    # mass per channel: every channel of every cell holds atoms, and the
    # grid's channel sum matches the oracle's lattice sum of sampled planes
    sums = out.float().sum(dim=(2, 3, 4)).cpu().numpy()
    assert np.all(sums > 0)
