"""GPU parity of grid reversal (§IV) through the C ABI: the local-maximum
peak search against the oracle's peak finder on the same float32 grids
(index work: bit-exact positions, types and CSR bounds), the reversal step
(residual, per-structure loss, coordinate gradient, updated coordinates)
against the oracle's FP64 step on every forward form, graph replay of the
step, and the whole loop recovering known coordinates.

Bars: residual and loss rel <= 1e-5 (FP32), gradient and coordinate
displacement rel-L2 <= 1e-4 (the adjoint bar).
"""
import numpy as np
import pytest

from gpu_util import errors, oracle, say, synth, to_device
from oracle import reversal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F32_TOL = 1e-5
ADJ_TOL = 1e-4


@pytest.fixture(scope="module")
def pg():
    import paper_2211_08506_amd as pg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pg


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def gpu_peaks(pg, dev, grid_np, thr, origin, spacing, origins=None, spacings=None, capacity=None):
    g = torch.tensor(np.ascontiguousarray(grid_np, np.float32), device=dev)
    B, C, D, H, W = g.shape
    desc = pg.make_desc(C, (D, H, W), spacing, origin, [0.5] * C)
    ctx = pg.default_context(dev)
    o_t = None if origins is None else torch.tensor(origins, device=dev)
    s_t = None if spacings is None else torch.tensor(spacings, device=dev)
    xyz, t, off = ctx.find_peaks(desc, g, thr, o_t, s_t, capacity=capacity)
    return xyz.cpu().numpy(), t.cpu().numpy(), off.cpu().numpy()


def check_peaks(name, got, want):
    gx, gt, go = got
    wx, wt, wo = want
    say(f"[peaks {name}] {len(wt)} peaks over {len(wo) - 1} structures")
    np.testing.assert_array_equal(go, wo)
    np.testing.assert_array_equal(gt, wt)
    np.testing.assert_array_equal(gx, wx)      # bit-exact positions


def test_peak_centre_rounded_once(pg, dev):
    """The exact centre 1 + 2^-24 + 2^-60 (o = 1, h = 16773121 * 2^-59, voxel
    2048) lies just above a float32 midpoint: rounded once it is 1 + 2^-23
    (rounding through double would give 1.0).  The GPU forms it from
    float-float terms with an exact sign test; it must match the oracle."""
    h = float(np.float32(16773121 * 2.0 ** -59))
    G = np.zeros((1, 1, 1, 1, 2049), np.float32)
    G[0, 0, 0, 0, 2048] = 1.0
    got = gpu_peaks(pg, dev, G, 0.5, (1.0, 0.0, 0.0), (h, 1.0, 1.0))
    want = reversal.find_peaks(G, 0.5, (1.0, 0.0, 0.0), (h, 1.0, 1.0))
    assert want[0][0, 0] == np.float32(1.0 + 2.0 ** -23)
    check_peaks("rounded once", got, want)
    # and a spread of origins and spacings, every centre of a long axis
    rng = np.random.default_rng(23)
    G = np.zeros((3, 1, 1, 1, 4099), np.float32)
    G[:, 0, 0, 0, ::2] = 1.0
    origins = rng.uniform(-50, 50, (3, 3)).astype(np.float32)
    spacings = rng.uniform(1e-4, 2.0, (3, 3)).astype(np.float32)
    check_peaks("centres of a long axis",
                gpu_peaks(pg, dev, G, 0.5, (0, 0, 0), 1.0, origins, spacings),
                reversal.find_peaks(G, 0.5, (0, 0, 0), 1.0, origins, spacings))


@pytest.mark.parametrize("value,thr", [("point", 0.05), ("box", 1e-4)])
def test_peaks_of_molecule_grids(pg, dev, value, thr):
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(48)
    say(f"case peaks of mol256x48 grids value={value}")
    xyz, types, offs = to_device(b, dev)
    g = pg.grid(xyz, types, offs, list(wl.sigma()), dims=wl.dims, spacing=wl.spacing,
                origin=wl.origin, value=value)
    torch.cuda.synchronize()
    G = g.cpu().numpy()
    want = reversal.find_peaks(G, thr, wl.origin, wl.spacing)
    check_peaks(f"mol/{value}", gpu_peaks(pg, dev, G, thr, wl.origin, wl.spacing), want)
    assert len(want[1]) > b.n_atoms // 2


@pytest.mark.parametrize("seed", [0, 1])
def test_peaks_tie_rule_and_ragged_shapes(pg, dev, seed):
    """Integer-valued grids (many plateaus) on shapes that are not multiples
    of the workgroup, with per-structure origins and spacings."""
    rng = np.random.default_rng(seed)
    G = rng.integers(0, 4, size=(3, 2, 7, 9, 11)).astype(np.float32)
    origins = rng.uniform(-5, 5, size=(3, 3)).astype(np.float32)
    spacings = rng.uniform(0.2, 0.7, size=(3, 3)).astype(np.float32)
    say(f"case peaks tie rule seed={seed}")
    want = reversal.find_peaks(G, 0.5, (0, 0, 0), 1.0, origins, spacings)
    check_peaks("ties", gpu_peaks(pg, dev, G, 0.5, (0, 0, 0), 1.0, origins, spacings), want)


def test_peaks_capacity_clamp_and_empty(pg, dev):
    rng = np.random.default_rng(5)
    G = rng.standard_normal((4, 1, 6, 6, 6)).astype(np.float32)
    wx, wt, wo = reversal.find_peaks(G, 0.0, (0, 0, 0), 0.5)
    cap = int(wo[2]) + 1                      # cuts structure 2 after one peak
    say(f"case peaks capacity {cap} of {len(wt)}")
    g = torch.tensor(G, device=dev)
    desc = pg.make_desc(1, (6, 6, 6), 0.5, (0, 0, 0), [0.5])
    ctx = pg.default_context(dev)
    xyz = torch.empty((cap, 3), device=dev)
    ty = torch.empty(cap, dtype=torch.int32, device=dev)
    off = torch.empty(5, dtype=torch.int32, device=dev)
    nf = torch.zeros(1, dtype=torch.int64, device=dev)
    lib = pg._lib()
    import ctypes
    st = lib.pg_find_peaks(ctx.handle, ctypes.byref(desc), g.data_ptr(), 4, None, None,
                           ctypes.c_float(0.0), cap, xyz.data_ptr(), ty.data_ptr(),
                           off.data_ptr(), nf.data_ptr(), None)
    assert st == pg.PG_OK
    torch.cuda.synchronize()
    assert int(nf.item()) == len(wt)
    np.testing.assert_array_equal(off.cpu().numpy(), np.minimum(wo, cap))
    np.testing.assert_array_equal(xyz.cpu().numpy(), wx[:cap])
    np.testing.assert_array_equal(ty.cpu().numpy(), wt[:cap])
    # an empty batch: offsets [0], no peaks
    off1 = torch.full((1,), 7, dtype=torch.int32, device=dev)
    st = lib.pg_find_peaks(ctx.handle, ctypes.byref(desc), None, 0, None, None,
                           ctypes.c_float(0.0), 0, None, None, off1.data_ptr(), nf.data_ptr(),
                           None)
    assert st == pg.PG_OK
    torch.cuda.synchronize()
    assert int(off1.item()) == 0 and int(nf.item()) == 0
    assert lib.pg_find_peaks(ctx.handle, ctypes.byref(desc), g.data_ptr(), 4, None, None,
                             ctypes.c_float(float("nan")), cap, xyz.data_ptr(), ty.data_ptr(),
                             off.data_ptr(), nf.data_ptr(), None) == pg.PG_E_PARAM


def step_case(pg, dev, b, sig, dims, h, origin, form, value="point", cell=None, lr=0.01,
              graph=False, seed=11):
    """GPU reversal step from perturbed coordinates vs the oracle's step."""
    rng = np.random.default_rng(seed)
    T = oracle.grid_fp64(b.xyz, b.types, b.offsets, sig, dims, h, origin, cell=cell,
                         value=value).astype(np.float32)
    x0 = (b.xyz + rng.uniform(-0.15, 0.15, size=b.xyz.shape)).astype(np.float32)
    if cell is not None:
        x0 = np.mod(x0, np.float32(cell)).astype(np.float32)
    loss_o, U_o, grad_o, new_o = reversal.reversal_step(x0, b.types, b.offsets, sig, dims, h, T,
                                                        lr, origin, cell=cell, value=value)
    pert = synth.Batch(x0, b.types, b.offsets)
    xyz, types, offs = to_device(pert, dev)
    ctx = pg.Context(0)
    desc = pg.make_desc(len(sig), dims, h, origin, sig, 3.0, cell, torch.float32, form, value)
    bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets)
    Tt = torch.tensor(T, device=dev)
    res = torch.empty_like(Tt)
    loss = torch.empty(b.n_mol, device=dev)
    grad = torch.empty_like(xyz)
    upd = torch.empty_like(xyz)
    if graph:
        ctx.set_option(pg.PG_OPT_GRAPH, 1)
    reps = 3 if graph else 1
    for r in range(reps):
        res.fill_(float("nan"))
        loss.fill_(float("nan"))
        ctx.reversal_step(desc, bv, Tt, res, loss, grad, upd, lr)
        torch.cuda.synchronize()
        rel_r, mx = errors(res.cpu().numpy(), U_o)
        ln = loss.cpu().numpy().astype(np.float64)
        rel_l = float(np.max(np.abs(ln - loss_o) / np.maximum(loss_o, 1e-30)))
        rel_g, _ = errors(grad.cpu().numpy(), grad_o)
        rel_d, _ = errors(upd.cpu().numpy().astype(np.float64) - x0, new_o - x0)
        say(f"[step {form}/{value} rep {r}] residual rel-L2 {rel_r:.3e} (max-abs {mx:.3e}), "
            f"loss max-rel {rel_l:.3e}, grad rel-L2 {rel_g:.3e}, step rel-L2 {rel_d:.3e}")
        assert rel_r <= F32_TOL and rel_l <= F32_TOL
        assert rel_g <= ADJ_TOL and rel_d <= ADJ_TOL
    assert ctx.device_error()[0] == 0
    return ctx


@pytest.mark.parametrize("form", ["window", "plain"])
@pytest.mark.parametrize("value", ["point", "box"])
def test_step_molecules(pg, dev, form, value):
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(24)
    say(f"case reversal step molecules form={form} value={value}")
    step_case(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, form, value,
              lr=0.01 if value == "point" else 2.0)


def test_step_binned_cells(pg, dev):
    sig = synth.sigma_table(3, 0.3, 0.45)
    rng = np.random.default_rng(51)
    off = np.array([0, 400, 700], np.int32)
    xyz = rng.uniform(0, 8.0, size=(700, 3)).astype(np.float32)
    b = synth.Batch(xyz, rng.integers(0, 3, 700).astype(np.int32), off)
    # the binned FP32 window form: the residual is held to the FP32 bar on
    # the vector form (a residual much smaller than G' magnifies any
    # relative error in G')
    say("case reversal step periodic cells, binned window form")
    step_case(pg, dev, b, sig, (40, 40, 40), 0.21, (0, 0, 0), "window", cell=8.0, lr=0.005)


def test_step_graph_replay(pg, dev):
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(16)
    say("case reversal step under graph replay")
    step_case(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, "auto", graph=True)


@pytest.mark.parametrize("case", ["point", "box", "periodic", "periodic_wide", "sphere", "graph"])
def test_step_without_residual_grid_is_bitwise(pg, dev, case):
    """residual = NULL on the molecule window form: the adjoint forms
    2 (G' - T) in each window from the target, summing G' as the forward
    does, so loss, gradient and update equal a step with a residual buffer
    bit for bit (and the oracle's step within the bars)."""
    wl = synth.WORKLOADS["mol256"]
    b = wl.batch(24)
    rng = np.random.default_rng(52)
    value = "box" if case == "box" else "point"
    # periodic_wide: a 16 A grid over a 12 A cell, so one atom's window
    # can appear twice along an axis
    cell = {"periodic": 16.0, "periodic_wide": 12.0}.get(case)
    shape = "sphere" if case == "sphere" else "cube"
    origin = (0.0, 0.0, 0.0) if cell else wl.origin
    xyz0 = np.mod(b.xyz, np.float32(cell)).astype(np.float32) if cell else b.xyz
    bb = synth.Batch(xyz0, b.types, b.offsets)
    T = oracle.grid_fp64(bb.xyz, bb.types, bb.offsets, wl.sigma(), wl.dims, wl.spacing, origin,
                         cell=cell, value=value, cutoff_shape=shape).astype(np.float32)
    x0 = (bb.xyz + rng.uniform(-0.15, 0.15, size=bb.xyz.shape)).astype(np.float32)
    if cell:
        x0 = np.mod(x0, np.float32(cell)).astype(np.float32)
    lr = 0.01 if value == "point" else 2.0
    loss_o, _, grad_o, _ = reversal.reversal_step(x0, bb.types, bb.offsets, wl.sigma(), wl.dims,
                                                  wl.spacing, T, lr, origin, cell=cell,
                                                  value=value, cutoff_shape=shape)
    say(f"case reversal step without residual grid: {case}")
    ctx = pg.Context(0)
    desc = pg.make_desc(wl.n_types, wl.dims, wl.spacing, origin, wl.sigma(), 3.0, cell,
                        torch.float32, "window", value, cutoff_shape=shape)
    xyz = torch.tensor(x0, device=dev)
    types, offs = torch.tensor(bb.types, device=dev), torch.tensor(bb.offsets, device=dev)
    bv = pg.BatchView(xyz, types, offs, offsets_host=bb.offsets)
    assert ctx.plan(desc, bv)["form"] == "window"
    Tt = torch.tensor(T, device=dev)
    if case == "graph":
        ctx.set_option(pg.PG_OPT_GRAPH, 1)
    outs = {}
    for keep in (True, False, True, False):
        res = torch.full_like(Tt, float("nan")) if keep else None
        loss = torch.full((bb.n_mol,), float("nan"), device=dev)
        grad = torch.full_like(xyz, float("nan"))
        upd = torch.full_like(xyz, float("nan"))
        ctx.reversal_step(desc, bv, Tt, res, loss, grad, upd, lr)
        torch.cuda.synchronize()
        got = (loss.cpu().numpy(), grad.cpu().numpy(), upd.cpu().numpy())
        if keep in outs:
            for a, c in zip(outs[keep], got):
                np.testing.assert_array_equal(a, c)   # replays repeat exactly
        outs[keep] = got
    for a, c in zip(outs[True], outs[False]):
        np.testing.assert_array_equal(a, c)
    ln, gr, _ = outs[False]
    rel_l = float(np.max(np.abs(ln.astype(np.float64) - loss_o) / np.maximum(loss_o, 1e-30)))
    rel_g, _ = errors(gr, grad_o)
    say(f"[no residual grid {case}] bitwise equal to the stored-residual step; "
        f"loss max-rel {rel_l:.3e}, grad rel-L2 {rel_g:.3e}")
    assert rel_l <= F32_TOL and rel_g <= ADJ_TOL
    assert ctx.device_error()[0] == 0


def test_step_without_residual_grid_refused_elsewhere(pg, dev):
    """A NULL residual needs the molecule window form without weights."""
    import ctypes
    lib = pg._lib()
    ctx = pg.Context(0)
    sig = synth.sigma_table(3, 0.3, 0.45)
    rng = np.random.default_rng(53)
    off = np.array([0, 400, 700], np.int32)
    xyz = torch.tensor(rng.uniform(0, 8.0, size=(700, 3)).astype(np.float32), device=dev)
    types = torch.tensor(rng.integers(0, 3, 700).astype(np.int32), device=dev)
    offs = torch.tensor(off, device=dev)
    desc = pg.make_desc(3, (40, 40, 40), 0.21, (0, 0, 0), sig, 3.0, 8.0, torch.float32, "window")
    bv = pg.BatchView(xyz, types, offs, offsets_host=off)
    assert ctx.plan(desc, bv)["binned"] == 1
    T = torch.zeros((2, 3, 40, 40, 40), device=dev)
    loss = torch.empty(2, device=dev)
    ws = ctx.workspace(ctx.reversal_workspace_size(desc, bv))
    st = lib.pg_reversal_step(ctx.handle, ctypes.byref(desc), ctypes.byref(bv.c), T.data_ptr(),
                              None, loss.data_ptr(), None, None, ctypes.c_float(0.0),
                              ws.data_ptr() if ws is not None and ws.numel() else None,
                              ctx.reversal_workspace_size(desc, bv), None)
    assert st == pg.PG_E_NULL


def separated_batch(seed, n_mol, n_atoms, box=9.0, min_sep=2.6, n_types=5):
    rng = np.random.default_rng(seed)
    xyz, types, offs = [], [], [0]
    for _ in range(n_mol):
        pts = []
        while len(pts) < n_atoms:
            p = rng.uniform(-box / 2, box / 2, size=3)
            if all(np.linalg.norm(p - q) >= min_sep for q in pts):
                pts.append(p)
        xyz.append(np.array(pts, np.float32))
        types.append(rng.integers(0, n_types, n_atoms).astype(np.int32))
        offs.append(offs[-1] + n_atoms)
    return synth.Batch(np.concatenate(xyz), np.concatenate(types), np.array(offs, np.int32))


def test_reverse_recovers_coordinates(pg, dev):
    """§IV-A end to end on the GPU: peaks of the grids of well-separated
    atoms, then coordinate steps, give back every atom to well under 1e-3 A."""
    wl = synth.WORKLOADS["mol256"]
    sig = wl.sigma()
    b = separated_batch(3, 32, 8)
    say("case reverse() end to end, 32 molecules of 8 separated atoms")
    xyz, types, offs = to_device(b, dev)
    T = pg.grid(xyz, types, offs, list(sig), dims=wl.dims, spacing=wl.spacing, origin=wl.origin)
    rx, rt, ro, loss = pg.reverse(T, list(sig), spacing=wl.spacing, origin=wl.origin,
                                  threshold=0.05, lr=0.02, steps=150)
    torch.cuda.synchronize()
    rx, rt, ro = rx.cpu().numpy(), rt.cpu().numpy(), ro.cpu().numpy()
    np.testing.assert_array_equal(ro, b.offsets)
    worst = 0.0
    for m in range(b.n_mol):
        a0, a1 = b.offsets[m], b.offsets[m + 1]
        for a in range(a0, a1):
            d = np.linalg.norm(rx[a0:a1] - b.xyz[a], axis=1)
            d[rt[a0:a1] != b.types[a]] = np.inf
            worst = max(worst, float(d.min()))
    say(f"[reverse] worst coordinate error {worst:.3e} A, max final loss "
        f"{float(loss.max()):.3e}")
    assert worst < 1e-3
