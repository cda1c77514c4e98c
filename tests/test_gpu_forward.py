"""GPU parity of the forward map against the FP64 oracle, through the C ABI.

Bars (per spec targets): FP32 output rel-L2 <= 1e-5, BF16 output
rel-L2 <= 1e-2, against the oracle on the same seeded inputs; max-abs and
rel-L2 are printed for every case.  Full-size workloads are checked on
sampled voxels that the oracle evaluates one by one.
"""
import math

import numpy as np
import pytest

from gpu_util import errors, oracle, sample_voxels, say, synth, to_device, worst_molecule

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


def run(pg, dev, batch, sigma, dims, spacing, origin, out_dtype=torch.float32, form="auto",
        cutoff_k=3.0, cell=None, origins=None, spacings=None, ctx=None, max_atoms=None):
    xyz, types, offs = to_device(batch, dev)
    o_t = None if origins is None else torch.tensor(np.asarray(origins, np.float32), device=dev)
    s_t = None if spacings is None else torch.tensor(np.asarray(spacings, np.float32), device=dev)
    g = pg.grid(xyz, types, offs, list(sigma), dims=dims, spacing=spacing, origin=origin,
                origins=o_t, spacings=s_t, cutoff_k=cutoff_k, cell=cell, out_dtype=out_dtype,
                form=form, ctx=ctx, max_atoms=max_atoms)
    torch.cuda.synchronize()
    return g


def ref_grid(batch, sigma, dims, spacing, origin, cutoff_k=3.0, cell=None, origins=None,
             spacings=None):
    return oracle.grid_fp64(batch.xyz, batch.types, batch.offsets, sigma, dims, spacing, origin,
                            cutoff_k=cutoff_k, cell=cell, origins=origins, spacings=spacings)


def check(name, g, ref, tol):
    got = g.double().cpu().numpy()
    rel, mx = errors(got, ref)
    wm = worst_molecule(got, ref) if ref.shape[0] > 1 else rel
    say(f"[{name}] rel-L2 {rel:.3e}  max-abs {mx:.3e}  worst-molecule rel-L2 {wm:.3e}")
    assert rel <= tol and wm <= tol, name
    return got


@pytest.mark.parametrize("form", ["window", "plain"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_single_molecule(pg, dev, form, dtype):
    wl = synth.WORKLOADS["single20"]
    b = wl.batch()
    say(f"case single20 form={form} dtype={dtype}")
    g = run(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin,
            torch.float32 if dtype == "f32" else torch.bfloat16, form)
    ref = ref_grid(b, wl.sigma(), wl.dims, wl.spacing, wl.origin)
    check(f"single20/{form}/{dtype}", g, ref, F32_TOL if dtype == "f32" else BF16_TOL)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batch_window_vs_oracle_and_plain(pg, dev, dtype):
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(48)
    say(f"case mol256[:48] dtype={dtype}")
    dt = torch.float32 if dtype == "f32" else torch.bfloat16
    ref = ref_grid(b, wl.sigma(), wl.dims, wl.spacing, wl.origin)
    gw = run(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, dt, "window")
    check(f"mol256[:48]/window/{dtype}", gw, ref, F32_TOL if dtype == "f32" else BF16_TOL)
    gp = run(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, dt, "plain")
    check(f"mol256[:48]/plain/{dtype}", gp, ref, F32_TOL if dtype == "f32" else BF16_TOL)
    # the two forms agree far more tightly than either vs the oracle
    rel, _ = errors(gw.double().cpu().numpy(), gp.double().cpu().numpy())
    say(f"[window vs plain/{dtype}] rel-L2 {rel:.3e}")
    assert rel <= (1e-6 if dtype == "f32" else 1e-2)
    # the non-zero pattern (the exact cutoff windows) is identical
    assert torch.equal(gw != 0, gp != 0)


def test_larger_grid_ragged_48(pg, dev):
    wl = synth.WORKLOADS["mol4096x48"]
    b = wl.batch(24)
    say("case mol4096x48[:24] f32 + bf16")
    ref = ref_grid(b, wl.sigma(), wl.dims, wl.spacing, wl.origin)
    g = run(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, torch.float32)
    check("mol4096x48[:24]/f32", g, ref, F32_TOL)
    g = run(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, torch.bfloat16)
    check("mol4096x48[:24]/bf16", g, ref, BF16_TOL)


@pytest.mark.parametrize("dims", [(8, 12, 30), (5, 7, 33), (16, 16, 16), (3, 40, 18), (1, 1, 1)])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_odd_shapes(pg, dev, dims, dtype):
    """Dims that are not multiples of the 16-byte store width, single voxel,
    and a ragged tail of runs in the last plane."""
    rng = np.random.default_rng(sum(dims))
    counts = [0, 3, 7, 1, 0, 5]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    h = 0.3
    ext = np.array([dims[2], dims[1], dims[0]]) * h
    xyz = (rng.uniform(-0.2, 1.2, size=(off[-1], 3)) * ext).astype(np.float32)
    b = synth.Batch(xyz, rng.integers(0, 3, off[-1]).astype(np.int32), off)
    sig = synth.sigma_table(3, 0.25, 0.4)
    say(f"case odd dims={dims} dtype={dtype}")
    dt = torch.float32 if dtype == "f32" else torch.bfloat16
    ref = ref_grid(b, sig, dims, h, (0.0, 0.0, 0.0))
    for form in ("window", "plain"):
        g = run(pg, dev, b, sig, dims, h, (0.0, 0.0, 0.0), dt, form)
        check(f"odd{dims}/{form}/{dtype}", g, ref, F32_TOL if dtype == "f32" else BF16_TOL)


def test_empty_structures_and_empty_batch(pg, dev):
    say("case empty")
    sig = [0.4, 0.5]
    b = synth.Batch(np.zeros((0, 3), np.float32), np.zeros(0, np.int32),
                    np.zeros(4, np.int32))
    g = run(pg, dev, b, sig, (4, 8, 8), 0.5, (0, 0, 0), max_atoms=0)
    assert g.shape == (3, 2, 4, 8, 8) and not g.any()
    b = synth.Batch(np.zeros((0, 3), np.float32), np.zeros(0, np.int32), np.zeros(1, np.int32))
    g = run(pg, dev, b, sig, (4, 8, 8), 0.5, (0, 0, 0), max_atoms=0)
    assert g.shape == (0, 2, 4, 8, 8)
    # a batch whose middle structure is empty and whose others sit outside the grid
    xyz = np.array([[100, 100, 100], [-50, 0, 0], [1.0, 1.0, 1.0]], np.float32)
    b = synth.Batch(xyz, np.array([0, 1, 1], np.int32), np.array([0, 2, 2, 3], np.int32))
    ref = ref_grid(b, sig, (4, 8, 8), 0.5, (0, 0, 0))
    g = run(pg, dev, b, sig, (4, 8, 8), 0.5, (0, 0, 0))
    check("empty-middle", g, ref, F32_TOL)
    assert not g[0].any() and not g[1].any() and g[2].any()


def test_exact_cutoff_edges(pg, dev):
    """Dyadic atoms with voxel centres exactly at distance rc: the GPU keeps
    exactly the voxels the oracle keeps (inclusive edge), and drops them one
    float32 ulp further away."""
    say("case exact edges")
    h = 0.5
    sig = [0.5, 0.25]                       # rc = 1.5 = 3 h, 0.75 = 1.5 h
    base = np.array([[4.25, 4.25, 4.25], [2.0, 3.0, 1.5], [6.25, 1.25, 3.75]], np.float32)
    nudged = base.copy()
    nudged[:, 0] = np.nextafter(nudged[:, 0], np.float32(100))
    nudged[:, 2] = np.nextafter(nudged[:, 2], np.float32(-100))
    for xyz in (base, nudged):
        b = synth.Batch(xyz, np.array([0, 1, 0], np.int32), np.array([0, 3], np.int32))
        ref = ref_grid(b, sig, (16, 16, 16), h, (0, 0, 0))
        for form in ("window", "plain"):
            g = run(pg, dev, b, sig, (16, 16, 16), h, (0, 0, 0), form=form)
            got = check(f"edges/{form}", g, ref, F32_TOL)
            assert np.array_equal(got > 0, ref > 0), "cutoff window differs from the oracle"


def test_periodic_cells(pg, dev):
    say("case periodic")
    rng = np.random.default_rng(21)
    sig = synth.sigma_table(3, 0.3, 0.45)
    # grid == cell (L = 16 * 0.5) and grid larger than the cell (40 * 0.21 = 8.4 > 8)
    for dims, h in (((16, 16, 16), 0.5), ((40, 40, 40), 0.21)):
        counts = [60, 17, 1]
        off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
        xyz = rng.uniform(0, 8.0, size=(off[-1], 3)).astype(np.float32)
        xyz[0] = [0.01, 7.99, 4.0]          # atoms at the faces
        b = synth.Batch(xyz, rng.integers(0, 3, off[-1]).astype(np.int32), off)
        ref = ref_grid(b, sig, dims, h, (0, 0, 0), cell=8.0)
        for form in ("window", "plain"):
            for dt, tol in ((torch.float32, F32_TOL), (torch.bfloat16, BF16_TOL)):
                g = run(pg, dev, b, sig, dims, h, (0, 0, 0), dt, form, cell=8.0)
                got = check(f"periodic{dims}/{form}/{dt}", g, ref, tol)
                assert np.array_equal(got > 0, ref > 0)


def test_per_structure_origins_spacings_and_no_cutoff(pg, dev):
    say("case origins/spacings/k=0")
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(5)
    org = np.array([[-8, -8, -8], [-7.5, -8.25, -6.0], [-4, -4, -4], [-9, -9, -9], [0, 0, 0]],
                   np.float32)
    spc = np.array([[0.5] * 3, [0.45, 0.5, 0.55], [0.25] * 3, [0.6] * 3, [0.5] * 3], np.float32)
    ref = ref_grid(b, wl.sigma(), (20, 24, 28), 0.5, (0, 0, 0), origins=org, spacings=spc)
    for form in ("window", "plain"):
        g = run(pg, dev, b, wl.sigma(), (20, 24, 28), 0.5, (0, 0, 0), form=form, origins=org,
                spacings=spc)
        check(f"origins+spacings/{form}", g, ref, F32_TOL)
    ref = ref_grid(b, wl.sigma(), (20, 20, 20), 0.6, (-6, -6, -6), cutoff_k=0.0)
    for form in ("window", "plain"):
        g = run(pg, dev, b, wl.sigma(), (20, 20, 20), 0.6, (-6, -6, -6), form=form, cutoff_k=0.0)
        check(f"no-cutoff/{form}", g, ref, F32_TOL)


def test_invalid_atoms_flagged_and_skipped(pg, dev):
    say("case invalid atoms")
    sig = [0.4, 0.5]
    xyz = np.array([[1, 1, 1], [np.nan, 1, 1], [2, 2, 2], [1.5, 1.5, 1.5]], np.float32)
    types = np.array([0, 1, 7, 1], np.int32)
    b = synth.Batch(xyz, types, np.array([0, 4], np.int32))
    good = synth.Batch(xyz[[0, 3]], types[[0, 3]], np.array([0, 2], np.int32))
    ref = ref_grid(good, sig, (8, 8, 8), 0.5, (0, 0, 0))
    for form in ("window", "plain"):
        ctx = pg.Context(0)
        g = run(pg, dev, b, sig, (8, 8, 8), 0.5, (0, 0, 0), form=form, ctx=ctx)
        check(f"invalid/{form}", g, ref, F32_TOL)
        code, first = ctx.device_error()
        assert code == pg.PG_E_DEVICE_DATA and first == 1
        assert ctx.device_error() == (0, -1)      # read clears it


def test_capacity_overflow_reports_and_zeroes(pg, dev):
    """A structure larger than the declared max_atoms is written as zeros and
    flagged, never read past the LDS capacity."""
    say("case capacity")
    rng = np.random.default_rng(2)
    counts = [3, 20, 5, 9]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    xyz = rng.uniform(-3, 3, size=(off[-1], 3)).astype(np.float32)
    b = synth.Batch(xyz, rng.integers(0, 5, off[-1]).astype(np.int32), off)
    wl = synth.WORKLOADS["mol256"]
    ref = ref_grid(b, wl.sigma(), wl.dims, wl.spacing, wl.origin)
    for block in (64, 512):
        ctx = pg.Context(0)
        ctx.set_option(pg.PG_OPT_BLOCK, block)
        g = run(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, form="window", ctx=ctx,
                max_atoms=8)                   # capacity rounds to 8 atoms
        code, first = ctx.device_error()
        assert code == pg.PG_E_CAPACITY and first == 1
        for m in range(4):
            if counts[m] > 8:
                assert not g[m].any()
            else:
                rel, _ = errors(g[m].double().cpu().numpy(), ref[m])
                assert rel <= F32_TOL


def test_determinism_across_launch_shapes(pg, dev):
    """Gather-only, no atomics on the output: bitwise identical across runs
    and across workgroup sizes / persistent grid sizes / store modes."""
    say("case determinism")
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(64)
    ctx = pg.Context(0)
    base = run(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, torch.bfloat16, ctx=ctx)
    again = run(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, torch.bfloat16, ctx=ctx)
    assert torch.equal(base, again)
    for blk, pc, un, nt in ((64, 1, 1, 0), (256, 2, 2, 1), (512, 4, 4, 1), (128, 8, 2, 0),
                            (1024, 1, 1, 1), (192, 3, 4, 0)):
        ctx.set_option(pg.PG_OPT_BLOCK, blk)
        ctx.set_option(pg.PG_OPT_GRID_PER_CU, pc)
        ctx.set_option(pg.PG_OPT_UNROLL, un)
        ctx.set_option(pg.PG_OPT_NT_STORE, nt)
        g = run(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, torch.bfloat16, ctx=ctx)
        assert torch.equal(base, g), (blk, pc, un, nt)


def _drop_atoms(b, m):
    """b with structure m emptied (its atoms removed)."""
    off = b.offsets.astype(np.int64)
    lo, hi = int(off[m]), int(off[m + 1])
    keep = np.r_[0:lo, hi:len(b.types)]
    noff = off.copy()
    noff[m + 1:] -= hi - lo
    return synth.Batch(b.xyz[keep].copy(), b.types[keep].copy(), noff.astype(np.int32))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_many_structures_per_workgroup(pg, dev, dtype):
    """Persistent workgroups that take several structures each (700 > one
    per CU), across empty structures, invalid atoms and structures over the
    declared capacity: grids and reported errors are bitwise the same for
    every workgroup size (one wave streams alone) and persistent grid size,
    and match the oracle."""
    say(f"case many structures per workgroup {dtype}")
    wl = synth.WORKLOADS["mol4096"]
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    tol = F32_TOL if dtype == "f32" else BF16_TOL
    b = _drop_atoms(wl.batch(700), 261)
    bad = synth.Batch(b.xyz.copy(), b.types.copy(), b.offsets)
    bad.xyz[b.offsets[300] + 1, 1] = np.nan      # an invalid atom in a later structure
    for name, bb, cap in (("plain", b, None), ("invalid", bad, None), ("capacity", b, 24)):
        grids, errs = [], []
        for blk, pc in ((512, 1), (1024, 1), (64, 1), (256, 3), (192, 2)):
            ctx = pg.Context(0)
            ctx.set_option(pg.PG_OPT_BLOCK, blk)
            ctx.set_option(pg.PG_OPT_GRID_PER_CU, pc)
            say(f"  {name}: block {blk} per_cu {pc}")
            grids.append(run(pg, dev, bb, wl.sigma(), wl.dims, wl.spacing, wl.origin, tdt,
                             form="window", ctx=ctx, max_atoms=cap))
            errs.append(ctx.device_error())
        for g, e in zip(grids[1:], errs[1:]):
            assert torch.equal(grids[0], g), name
            assert e == errs[0], name
        counts = np.diff(bb.offsets)
        if name == "plain":
            assert errs[0] == (0, -1)
        elif name == "invalid":
            assert errs[0] == (pg.PG_E_DEVICE_DATA, int(b.offsets[300]) + 1)
        else:
            assert errs[0] == (pg.PG_E_CAPACITY, int(np.argmax(counts > 24)))
        g = grids[1]
        assert not g[261].any()
        for m in (0, 255, 256, 260, 262, 300, 511, 512, 699):
            lo, hi = int(bb.offsets[m]), int(bb.offsets[m + 1])
            if cap is not None and hi - lo > cap:
                assert not g[m].any()
                continue
            keep = np.isfinite(bb.xyz[lo:hi]).all(axis=1)
            one = synth.Batch(bb.xyz[lo:hi][keep], bb.types[lo:hi][keep],
                              np.array([0, int(keep.sum())], np.int32))
            ref = ref_grid(one, wl.sigma(), wl.dims, wl.spacing, wl.origin)
            rel, mx = errors(g[m:m + 1].double().cpu().numpy(), ref)
            assert rel <= tol, (name, m, rel, mx)


def test_permutation_invariance(pg, dev):
    say("case permutation")
    wl = synth.WORKLOADS["single20"]
    b = wl.batch()
    perm = np.random.default_rng(4).permutation(b.n_atoms)
    bp = synth.Batch(b.xyz[perm].copy(), b.types[perm].copy(), b.offsets)
    g1 = run(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin)
    g2 = run(pg, dev, bp, wl.sigma(), wl.dims, wl.spacing, wl.origin)
    rel, _ = errors(g2.double().cpu().numpy(), g1.double().cpu().numpy())
    assert rel <= 1e-6


def test_integer_translation_shifts_grid_bitwise(pg, dev):
    """Coordinates on a 2^-12 lattice, h = 0.5: translating by whole voxels
    shifts the window-form grid bit for bit (same offsets, same order)."""
    say("case translation")
    rng = np.random.default_rng(9)
    mu = (np.round(rng.uniform(-2, 2, size=(9, 3)) * 4096) / 4096).astype(np.float32)
    t = rng.integers(0, 3, size=9).astype(np.int32)
    sig = synth.sigma_table(3)
    n = np.array([2, -1, 3])
    b1 = synth.Batch(mu, t, np.array([0, 9], np.int32))
    b2 = synth.Batch((mu + n * 0.5).astype(np.float32), t, np.array([0, 9], np.int32))
    g1 = run(pg, dev, b1, sig, (32, 32, 32), 0.5, (-8, -8, -8))[0]
    g2 = run(pg, dev, b2, sig, (32, 32, 32), 0.5, (-8, -8, -8))[0]
    a = g1[:, 4:24, 4:24, 4:24]
    c = g2[:, 4 + n[2]:24 + n[2], 4 + n[1]:24 + n[1], 4 + n[0]:24 + n[0]]
    assert torch.equal(a, c)


@pytest.mark.parametrize("form", ["window", "plain"])
def test_graph_replay_matches_eager(pg, dev, form):
    """With the graph option on, repeated calls -- the one-kernel window form
    launched directly, the multi-kernel plain form replayed from its captured
    graph -- with eager work and synchronisation between them each reproduce
    the eager result bit for bit."""
    say(f"case graph replay form={form}")
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(128)
    xyz, types, offs = to_device(b, dev)
    ctx = pg.Context(0)
    desc = pg.make_desc(5, wl.dims, wl.spacing, wl.origin, wl.sigma(), 3.0, None, torch.bfloat16, form)
    bv = pg.BatchView(xyz, types, offs)
    eager = pg.empty_grid(desc, b.n_mol, dev)
    ctx.forward(desc, bv, eager)
    torch.cuda.synchronize()
    ctx.set_option(pg.PG_OPT_GRAPH, 1)
    out = pg.empty_grid(desc, b.n_mol, dev)
    for rep in range(4):
        out.fill_(float("nan"))
        ctx.forward(desc, bv, out)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device=dev).sum()      # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {rep}"
        del junk


def test_autotune_keeps_result_identical(pg, dev, tmp_path):
    say("case autotune")
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(256)
    xyz, types, offs = to_device(b, dev)
    ctx = pg.Context(0)
    desc = pg.make_desc(5, wl.dims, wl.spacing, wl.origin, wl.sigma(), 3.0, None, torch.bfloat16)
    bv = pg.BatchView(xyz, types, offs)
    before = pg.empty_grid(desc, b.n_mol, dev)
    ctx.forward(desc, bv, before)
    out = pg.empty_grid(desc, b.n_mol, dev)
    ctx.autotune(desc, bv, out, reps=2)
    plan = ctx.plan(desc, bv, out)
    say(f"tuned plan {plan}")
    after = pg.empty_grid(desc, b.n_mol, dev)
    ctx.forward(desc, bv, after)
    torch.cuda.synchronize()
    assert torch.equal(before, after)
    path = str(tmp_path / "tune.json")
    ctx.tuning_save(path)
    ctx2 = pg.Context(0)
    ctx2.tuning_load(path)
    assert ctx2.plan(desc, bv, out) == plan


def _full_size_sampled(pg, dev, name, dtype, tol, n_mol=None):
    wl = synth.WORKLOADS[name]
    b = wl.batch(n_mol)
    say(f"case full-size {name} B={b.n_mol} dtype={dtype}")
    xyz, types, offs = to_device(b, dev)
    ctx = pg.default_context(dev)
    desc = pg.make_desc(wl.n_types, wl.dims, wl.spacing, wl.origin, wl.sigma(), wl.cutoff_k,
                        None, dtype)
    bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets)
    out = pg.empty_grid(desc, b.n_mol, dev)
    ctx.set_option(pg.PG_OPT_GRAPH, 1)        # the launch configuration the bench times
    try:
        ctx.forward(desc, bv, out)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(pg.PG_OPT_GRAPH, 0)
    rng = np.random.default_rng(17)
    idx = sample_voxels(rng, b, tuple(out.shape), wl.origin, wl.spacing, 20000, 20000)
    ref = oracle.voxels_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing, idx,
                             wl.origin, cutoff_k=wl.cutoff_k)
    it = torch.tensor(idx, device=dev)
    got = out[it[:, 0], it[:, 1], it[:, 2], it[:, 3], it[:, 4]].double().cpu().numpy()
    rel, mx = errors(got, ref)
    say(f"[{name}/{dtype} sampled {len(idx)}] rel-L2 {rel:.3e} max-abs {mx:.3e}")
    assert rel <= tol
    assert np.array_equal(got > 0, ref > 0)
    # zero-structure invariant at full size: every grid holds mass only in
    # the channels of its atoms
    sums = out.float().sum(dim=(2, 3, 4)).cpu().numpy()
    has = np.zeros_like(sums, dtype=bool)
    for m in range(b.n_mol):
        has[m, np.unique(b.types[b.offsets[m]:b.offsets[m + 1]])] = True
    assert np.all(sums[~has] == 0) and np.all(sums[has] > 0)


def test_full_size_headline_bf16(pg, dev):
    _full_size_sampled(pg, dev, "mol4096", torch.bfloat16, BF16_TOL)


def test_full_size_headline_f32(pg, dev):
    _full_size_sampled(pg, dev, "mol4096", torch.float32, F32_TOL)


def test_full_size_48_bf16(pg, dev):
    _full_size_sampled(pg, dev, "mol4096x48", torch.bfloat16, BF16_TOL)


def test_wide_plane_window_rows(pg, dev):
    """A 3296 x 1783 plane (one z layer, one-element runs, 160 KB of LDS per
    workgroup): the molecule window kernel must place every run in its row
    (a float estimate alone is one row off for 187 runs of this plane, in
    the last column).  No cutoff and a wide Gaussian make every voxel
    non-zero and row-dependent, so a run read from the wrong row is seen."""
    D, H, W = 1, 3296, 1783
    h = 0.5
    rng = np.random.default_rng(77)
    off = np.array([0, 8, 16], np.int32)
    ext = np.array([W, H, D], np.float64) * h
    xyz = (rng.uniform(0.1, 0.9, size=(16, 3)) * ext).astype(np.float32)
    b = synth.Batch(xyz, np.zeros(16, np.int32), off)
    sig = np.array([300.0])
    say("case wide plane 1 x 3296 x 1783, window form")
    xyz_d, types, offs = to_device(b, dev)
    ctx = pg.default_context(dev)
    desc = pg.make_desc(1, (D, H, W), h, (0.0, 0.0, 0.0), sig, 0.0, None, torch.float32, "auto")
    bv = pg.BatchView(xyz_d, types, offs, offsets_host=b.offsets)
    out = pg.empty_grid(desc, b.n_mol, dev)
    plan = ctx.plan(desc, bv, out)
    say(f"plan {plan}")
    assert plan["form"] == "window" and plan["binned"] == 0 and plan["vec"] == 1
    assert plan["lds_bytes"] > 65536
    ctx.forward(desc, bv, out)
    torch.cuda.synchronize()
    assert ctx.device_error()[0] == 0
    ref = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, (D, H, W), h, (0.0, 0.0, 0.0),
                           cutoff_k=0.0)
    got = out.double().cpu().numpy()
    rel, mx = errors(got, ref)
    elem = float(np.max(np.abs(got - ref) / ref))
    say(f"[wide plane] rel-L2 {rel:.3e} max-abs {mx:.3e} max elementwise rel {elem:.3e}")
    assert ref.min() > 0
    assert rel <= F32_TOL and elem <= 1e-5
