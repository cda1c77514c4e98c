"""CPU-only checks of the C-ABI library: it loads, exports every function
declared in include/particlegrid.h, and its host-side validation, workspace
sizing and planning behave as documented.  No call here touches a GPU."""
import ctypes
import os
import re

import pytest

import paper_2211_08506_amd as pg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "particlegrid.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pg_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(pg.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), f"{n} declared in particlegrid.h but not exported"
    assert set(names) == set(pg.EXPORTS)


def test_abi_version_and_status_strings():
    assert pg.abi_version() == 5
    lib = pg._lib()
    for s in range(0, 10):
        assert lib.pg_status_str(s)
    assert lib.pg_status_str(12345) == b"unknown status"


def desc_ok(**kw):
    d = pg.make_desc(kw.pop("C", 5), kw.pop("dims", (32, 32, 32)), kw.pop("spacing", 0.5),
                     kw.pop("origin", (-8, -8, -8)), kw.pop("sigma", [0.4, 0.475, 0.55, 0.625, 0.7]),
                     kw.pop("cutoff_k", 3.0), kw.pop("cell", None), kw.pop("out_dtype", "f32"),
                     kw.pop("form", "auto"), kw.pop("value", "point"))
    assert not kw
    return d


def batch_ok(n_mol=4, n_atoms=40, max_atoms=12, fake=0x1000):
    b = pg.Batch()
    b.xyz = fake
    b.types = fake
    b.offsets = fake
    b.origins = None
    b.spacings = None
    b.n_mol = n_mol
    b.n_atoms = n_atoms
    b.max_atoms = max_atoms
    return b


def validate(d, b):
    return pg._lib().pg_validate(ctypes.byref(d), ctypes.byref(b))


def test_validate_accepts_good_request():
    assert validate(desc_ok(), batch_ok()) == pg.PG_OK
    assert validate(desc_ok(out_dtype="bf16"), batch_ok()) == pg.PG_OK
    assert validate(desc_ok(cutoff_k=0.0), batch_ok()) == pg.PG_OK
    assert validate(desc_ok(value="box"), batch_ok()) == pg.PG_OK
    assert validate(desc_ok(), batch_ok(n_mol=0, n_atoms=0, max_atoms=0)) == pg.PG_OK


@pytest.mark.parametrize("field,value,code", [
    ("C", 0, pg.PG_E_SHAPE), ("C", 65, pg.PG_E_SHAPE), ("D", 0, pg.PG_E_SHAPE),
    ("W", -3, pg.PG_E_SHAPE), ("cutoff_k", -1.0, pg.PG_E_PARAM),
    ("cutoff_k", float("nan"), pg.PG_E_PARAM), ("out_dtype", 7, pg.PG_E_PARAM),
    ("form", 9, pg.PG_E_PARAM), ("value", 2, pg.PG_E_PARAM), ("value", -1, pg.PG_E_PARAM),
])
def test_validate_rejects_bad_desc(field, value, code):
    d = desc_ok()
    setattr(d, field, value)
    assert validate(d, batch_ok()) == code


def test_validate_rejects_bad_params():
    d = desc_ok()
    d.spacing[1] = 0.0
    assert validate(d, batch_ok()) == pg.PG_E_PARAM
    d = desc_ok()
    d.sigma[3] = -0.1
    assert validate(d, batch_ok()) == pg.PG_E_PARAM
    d = desc_ok()
    d.origin[0] = float("inf")
    assert validate(d, batch_ok()) == pg.PG_E_PARAM


def test_validate_batch_sizes_and_nulls():
    d = desc_ok()
    assert validate(d, batch_ok(n_mol=-1)) == pg.PG_E_SHAPE
    assert validate(d, batch_ok(max_atoms=0)) == pg.PG_E_SHAPE      # atoms but no bound
    assert validate(d, batch_ok(max_atoms=41)) == pg.PG_E_SHAPE     # bound above n_atoms
    assert validate(d, batch_ok(n_mol=0)) == pg.PG_E_SHAPE          # atoms without structures
    b = batch_ok()
    b.offsets = None
    assert validate(d, b) == pg.PG_E_NULL
    b = batch_ok()
    b.xyz = None
    assert validate(d, b) == pg.PG_E_NULL
    assert pg._lib().pg_validate(None, ctypes.byref(batch_ok())) == pg.PG_E_NULL


def test_validate_periodic_constraints():
    sig = [0.4 + 0.3 * i / 7 for i in range(8)]
    ok = desc_ok(C=8, dims=(128, 128, 128), spacing=0.16, origin=(0, 0, 0), sigma=sig,
                 cell=20.0)
    assert validate(ok, batch_ok()) == pg.PG_OK
    small = desc_ok(C=8, dims=(16, 16, 16), spacing=0.16, origin=(0, 0, 0), sigma=sig, cell=4.0)
    assert validate(small, batch_ok()) == pg.PG_E_PERIODIC        # rc = 2.1 >= L/2
    wide = desc_ok(C=8, dims=(300, 128, 128), spacing=0.16, origin=(0, 0, 0), sigma=sig,
                   cell=20.0)
    assert validate(wide, batch_ok()) == pg.PG_E_PERIODIC         # extent 48 > 2 L - 2 rc
    nocut = desc_ok(C=8, dims=(128, 128, 128), spacing=0.16, origin=(0, 0, 0), sigma=sig,
                    cell=20.0, cutoff_k=0.0)
    assert validate(nocut, batch_ok()) == pg.PG_E_PERIODIC
    b = batch_ok()
    b.spacings = 0x2000
    assert validate(ok, b) == pg.PG_E_UNSUPPORTED


def test_workspace_and_plan_host_only():
    lib = pg._lib()
    n = ctypes.c_size_t(123)
    d = desc_ok(form="window")
    assert lib.pg_workspace_size(None, ctypes.byref(d), ctypes.byref(batch_ok()), ctypes.byref(n)) == 0
    assert n.value == 0                  # the window form needs no workspace
    d = desc_ok(form="plain")
    assert lib.pg_workspace_size(None, ctypes.byref(d), ctypes.byref(batch_ok()), ctypes.byref(n)) == 0
    assert n.value >= 40 * 100 and n.value % 256 == 0
    info = pg.PlanInfo()
    d = desc_ok(out_dtype="bf16")
    assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(batch_ok()), 0x10000, ctypes.byref(info)) == 0
    assert info.form == pg.FORMS["window"] and info.vec == 8 and info.atom_capacity == 16
    # misaligned output pointer falls back to narrower stores
    assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(batch_ok()), 0x10002, ctypes.byref(info)) == 0
    assert info.vec == 1
    # structures larger than the window kernel's LDS capacity take the
    # large-structure (binned plane) path, which needs a workspace
    big = batch_ok(n_atoms=4000, max_atoms=1000)
    for form, dtype in (("window", "f32"), ("mfma", "bf16"), ("auto", "bf16"), ("auto", "f32")):
        d = desc_ok(form=form, out_dtype=dtype)
        assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(big), 0x10000, ctypes.byref(info)) == 0
        want = "mfma" if form in ("mfma", "auto") else "window"
        assert info.form == pg.FORMS[want] and info.binned == 1
        assert info.atom_capacity == 0   # 0: no limit on the images of a plane
        assert lib.pg_workspace_size(None, ctypes.byref(d), ctypes.byref(big), ctypes.byref(n)) == 0
        # per-atom records + 3 counters per (structure, channel, z plane) + bin lists
        assert n.value >= 4000 * 160 + 3 * 4 * 5 * 32 * 4 and n.value % 256 == 0
    # the MFMA form keeps float phi_x factor slots for float32 grids and bf16
    # ones for bf16 grids (phi_y slots are float in both): at least one
    # 32-value slot per atom on x
    ws = {}
    for dtype in ("bf16", "f32"):
        d = desc_ok(form="mfma", out_dtype=dtype)
        assert lib.pg_workspace_size(None, ctypes.byref(d), ctypes.byref(big), ctypes.byref(n)) == 0
        ws[dtype] = n.value
    assert ws["f32"] >= ws["bf16"] + 4000 * 32 * 2
    # per-structure spacings are not supported on the large-structure path
    big.spacings = 0x2000
    assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(big), 0x10000,
                       ctypes.byref(info)) == pg.PG_E_UNSUPPORTED
    # the small-structure window plan reports no large-structure flag
    d = desc_ok(form="window")
    assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(batch_ok()), 0x10000, ctypes.byref(info)) == 0
    assert info.binned == 0


def test_weighted_channels_validation_and_plans():
    """Weighted channels: types index n_types widths independent of C; every
    form takes them; the window form stages the weights in LDS, the binned
    path lists each atom under every channel it weighs into."""
    lib = pg._lib()
    info = pg.PlanInfo()
    sig8 = [0.4 + 0.3 * i / 7 for i in range(8)]
    bw = batch_ok()
    bw.weights = 0x3000
    d = desc_ok(C=3, sigma=sig8)
    d.n_types = 8                      # 8 types into 3 channels
    assert validate(d, bw) == pg.PG_OK
    d.sigma[7] = 0.0                   # every width the types index is checked
    assert validate(d, bw) == pg.PG_E_PARAM
    d = desc_ok(C=3, sigma=sig8)
    d.n_types = 65
    assert validate(d, bw) == pg.PG_E_PARAM
    d.n_types = 8
    assert validate(d, batch_ok()) == pg.PG_E_PARAM     # n_types without weights must be C
    d = desc_ok()
    d.n_types = 5
    assert validate(d, batch_ok()) == pg.PG_OK
    # plans: window holds the weights in LDS; binned path refuses them
    d = desc_ok()
    assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(batch_ok()), 0x10000,
                       ctypes.byref(info)) == 0
    lds0 = info.lds_bytes
    assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(bw), 0x10000, ctypes.byref(info)) == 0
    assert info.form == pg.FORMS["window"] and info.lds_bytes == lds0 + 16 * 5 * 4
    big = batch_ok(n_atoms=4000, max_atoms=1000)
    n = ctypes.c_size_t()
    for form in ("window", "mfma"):
        d = desc_ok(form=form, out_dtype="bf16")
        assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(big), 0x10000,
                           ctypes.byref(info)) == 0 and info.binned == 1
        assert lib.pg_workspace_size(None, ctypes.byref(d), ctypes.byref(big), ctypes.byref(n)) == 0
        ws_one = n.value
        big.weights = 0x3000       # one channel-partition entry per (atom, channel)
        assert lib.pg_workspace_size(None, ctypes.byref(d), ctypes.byref(big), ctypes.byref(n)) == 0
        assert n.value > ws_one + 4000 * 4 * 48
        big.weights = None
    d = desc_ok(form="plain")
    assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(big), 0x10000, ctypes.byref(info)) == 0


SHEAR = [[8.0, 2.5, 1.0], [0.0, 7.5, -1.5], [0.0, 0.0, 8.5]]


def test_triclinic_validation_and_plans():
    """Triclinic cells: the cell check (image cubes apart, non-singular,
    bounded image count), the unsupported combinations, and the plan of the
    non-periodic request over the images (the workspace holds the images)."""
    lib = pg._lib()
    info = pg.PlanInfo()
    n = ctypes.c_size_t()
    sig = [0.3, 0.35, 0.4, 0.45, 0.5]
    tri = lambda cell, **kw: desc_ok(sigma=sig, dims=(32, 32, 32), spacing=0.25,
                                    origin=(0, 0, 0), cell=cell, **kw)
    d = tri(SHEAR)
    assert d.periodic == pg.PG_CELL_TRICLINIC
    small = batch_ok(n_mol=2, n_atoms=6, max_atoms=3)
    assert validate(d, small) == pg.PG_OK
    assert validate(tri([[8, 0, 0], [0, 8, 0], [0, 0, 0]]), small) == pg.PG_E_PERIODIC   # singular
    thin = [[8.0, 7.0, 0.0], [0.0, 1.5, 0.0], [0.0, 0.0, 8.0]]   # (-1, 1.5, 0) is a lattice vector
    assert validate(tri(thin), small) == pg.PG_E_PERIODIC
    assert validate(tri(SHEAR, cutoff_k=0.0), small) == pg.PG_E_PERIODIC
    b = batch_ok(n_mol=2, n_atoms=6, max_atoms=3)
    b.spacings = 0x2000
    assert validate(d, b) == pg.PG_E_UNSUPPORTED
    b = batch_ok(n_mol=2, n_atoms=6, max_atoms=3)
    b.weights = 0x2000
    assert validate(d, b) == pg.PG_E_UNSUPPORTED
    # a grid far larger than the cell needs too many images
    big_grid = desc_ok(sigma=sig, dims=(256, 256, 256), spacing=0.25, origin=(0, 0, 0),
                       cell=SHEAR)
    assert validate(big_grid, small) == pg.PG_E_PERIODIC
    # plans: 3 atoms x 27 images fit the window form; 40 x 27 take the binned path
    assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(small), 0x10000, ctypes.byref(info)) == 0
    assert info.form == pg.FORMS["window"] and info.binned == 0
    assert lib.pg_workspace_size(None, ctypes.byref(d), ctypes.byref(small), ctypes.byref(n)) == 0
    assert n.value >= 6 * 27 * (12 + 4 + 12)
    mid = batch_ok(n_mol=2, n_atoms=80, max_atoms=40)
    assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(mid), 0x10000, ctypes.byref(info)) == 0
    assert info.binned == 1
    # not with the autotuner's or the reversal step's plans
    assert lib.pg_reversal_workspace_size(None, ctypes.byref(d), ctypes.byref(small),
                                          ctypes.byref(n)) == pg.PG_E_UNSUPPORTED


def test_sphere_cutoff_validation_and_plans():
    """The sphere cutoff: a valid shape code; molecule window or plain form
    (AUTO falls back to plain for structures past the window kernel); the
    binned forms refuse it; the window form stages squared offsets in LDS."""
    lib = pg._lib()
    info = pg.PlanInfo()
    d = desc_ok()
    d.cutoff_shape = 2
    assert validate(d, batch_ok()) == pg.PG_E_PARAM
    cube = desc_ok()
    assert lib.pg_plan(None, ctypes.byref(cube), ctypes.byref(batch_ok()), 0x10000,
                       ctypes.byref(info)) == 0
    lds_cube = info.lds_bytes
    sph = desc_ok()
    sph.cutoff_shape = pg.SHAPES["sphere"]
    assert lib.pg_plan(None, ctypes.byref(sph), ctypes.byref(batch_ok()), 0x10000,
                       ctypes.byref(info)) == 0
    assert info.form == pg.FORMS["window"] and info.unroll == 1
    assert info.lds_bytes > lds_cube
    big = batch_ok(n_atoms=4000, max_atoms=1000)
    assert lib.pg_plan(None, ctypes.byref(sph), ctypes.byref(big), 0x10000, ctypes.byref(info)) == 0
    assert info.form == pg.FORMS["plain"] and info.binned == 0
    for form in ("window", "mfma"):
        d = desc_ok(form=form)
        d.cutoff_shape = pg.SHAPES["sphere"]
        assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(big), 0x10000,
                           ctypes.byref(info)) == pg.PG_E_UNSUPPORTED


def test_reversal_workspace_host_only():
    """The molecule window form forms the residual in its forward kernel (no
    workspace); other forms need FP64 partial loss sums (one per 4096
    elements of each structure) after their own workspace; bf16 grids are
    refused (the residual and the loss are float32)."""
    lib = pg._lib()
    n = ctypes.c_size_t(123)
    ws = lambda d, b: (lib.pg_reversal_workspace_size(None, ctypes.byref(d), ctypes.byref(b),
                                                       ctypes.byref(n)), n.value)
    assert ws(desc_ok(form="window"), batch_ok()) == (0, 0)
    per_mol = 5 * 32 * 32 * 32
    chunks = -(-per_mol // 4096)
    st, plain = ws(desc_ok(form="plain"), batch_ok())
    assert st == 0 and plain >= 4 * chunks * 8 + 40 * 100
    big = batch_ok(n_atoms=4000, max_atoms=1000)
    _, fwd = (lib.pg_workspace_size(None, ctypes.byref(desc_ok(form="window")), ctypes.byref(big),
                                    ctypes.byref(n)), n.value)
    st, rev = ws(desc_ok(form="window"), big)
    assert st == 0 and rev == -(-fwd // 256) * 256 + 4 * chunks * 8
    assert ws(desc_ok(out_dtype="bf16"), batch_ok())[0] == pg.PG_E_PARAM
    assert lib.pg_reversal_workspace_size(None, ctypes.byref(desc_ok()), ctypes.byref(batch_ok()),
                                          None) == pg.PG_E_NULL


def test_null_context_calls_fail_cleanly():
    lib = pg._lib()
    d = desc_ok()
    b = batch_ok()
    assert lib.pg_grid_forward(None, ctypes.byref(d), ctypes.byref(b), 0x1000, None, 0, None) == pg.PG_E_NULL
    assert lib.pg_grid_backward(None, ctypes.byref(d), ctypes.byref(b), 0x1000, 0x1000, None, None,
                                0, None) == pg.PG_E_NULL
    assert lib.pg_set_option(None, 1, 1) == pg.PG_E_NULL
    assert lib.pg_find_peaks(None, ctypes.byref(d), 0x1000, 4, None, None, 0.1, 16, 0x1000,
                             0x1000, 0x1000, 0x1000, None) == pg.PG_E_NULL
    assert lib.pg_reversal_step(None, ctypes.byref(d), ctypes.byref(b), 0x1000, 0x1000, 0x1000,
                                None, None, 0.1, None, 0, None) == pg.PG_E_NULL
    assert lib.pg_destroy(None) == pg.PG_E_NULL
    assert lib.pg_create(None, 0) == pg.PG_E_NULL


# ---- host-only contexts: planning with a tuning table, no GPU -------------

def host_ctx():
    lib = pg._lib()
    h = ctypes.c_void_p()
    assert lib.pg_create(ctypes.byref(h), pg.PG_HOST_ONLY) == pg.PG_OK
    assert h.value
    return lib, h


def test_host_only_context_refuses_device_calls():
    lib, h = host_ctx()
    try:
        d = desc_ok()
        b = batch_ok()
        assert lib.pg_grid_forward(h, ctypes.byref(d), ctypes.byref(b), 0x1000, None, 0,
                                   None) == pg.PG_E_UNSUPPORTED
        assert lib.pg_grid_backward(h, ctypes.byref(d), ctypes.byref(b), 0x1000, 0x1000, None,
                                    None, 0, None) == pg.PG_E_UNSUPPORTED
        assert lib.pg_autotune(h, ctypes.byref(d), ctypes.byref(b), 0x1000, None, 0, None,
                               3) == pg.PG_E_UNSUPPORTED
        code, first = ctypes.c_int32(), ctypes.c_int64()
        assert lib.pg_get_device_error(h, ctypes.byref(code),
                                       ctypes.byref(first)) == pg.PG_E_UNSUPPORTED
        assert lib.pg_set_option(h, pg.PG_OPT_GRAPH, 1) == pg.PG_OK
        assert lib.pg_last_hip_error(h) == 0
        bad = ctypes.c_void_p()
        assert lib.pg_create(ctypes.byref(bad), -7) == pg.PG_E_PARAM
    finally:
        assert lib.pg_destroy(h) == pg.PG_OK


def plan_info(lib, h, d, b, out=0x10000):
    info = pg.PlanInfo()
    st = lib.pg_plan(h, ctypes.byref(d), ctypes.byref(b), out, ctypes.byref(info))
    return st, {n: getattr(info, n) for n, _ in pg.PlanInfo._fields_}


def test_host_only_plan_wide_plane_takes_window_form():
    """A 1 x 3296 x 1783 plane with 8-atom structures fits gfx950's 160 KiB
    of LDS per workgroup, so it takes the molecule window form (whose run
    rows are exact for every admitted plane), not the binned path."""
    lib, h = host_ctx()
    try:
        d = pg.make_desc(1, (1, 3296, 1783), 0.5, (0, 0, 0), [300.0], 0.0)
        b = batch_ok(n_mol=2, n_atoms=16, max_atoms=8)
        st, info = plan_info(lib, h, d, b)
        assert st == pg.PG_OK
        assert info["binned"] == 0 and info["form"] == pg.FORMS["window"]
        assert info["vec"] == 1 and 65536 < info["lds_bytes"] <= 163840
        # without a context the plan assumes 64 KiB of LDS: not the molecule
        # window form; without a cutoff the plane is too wide for the binned
        # forms' tile bookkeeping, so AUTO takes the plain form
        info0 = pg.PlanInfo()
        assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(b), 0x10000,
                           ctypes.byref(info0)) == pg.PG_OK
        assert info0.binned == 0 and info0.form == pg.FORMS["plain"]
    finally:
        lib.pg_destroy(h)


def test_plan_mfma_slot_arrays_below_4gib():
    """The MFMA tile kernels address factor-slot values by 32-bit byte
    offsets: a batch whose slot array would reach 4 GiB is refused by the
    MFMA form, and AUTO takes the binned vector form instead."""
    lib = pg._lib()
    d = desc_ok(form="mfma", out_dtype="bf16")
    # 32^3 grid: one 32-voxel slot per atom and axis, 128 bytes per float slot
    ok = batch_ok(n_mol=4, n_atoms=(1 << 25) - 1024, max_atoms=1000)
    huge = batch_ok(n_mol=4, n_atoms=(1 << 25) + 1024, max_atoms=1000)
    info = pg.PlanInfo()
    assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(ok), 0x10000, ctypes.byref(info)) == pg.PG_OK
    assert info.form == pg.FORMS["mfma"] and info.binned == 1
    assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(huge), 0x10000,
                       ctypes.byref(info)) == pg.PG_E_UNSUPPORTED
    d = desc_ok(form="auto", out_dtype="bf16")
    assert lib.pg_plan(None, ctypes.byref(d), ctypes.byref(huge), 0x10000, ctypes.byref(info)) == pg.PG_OK
    assert info.form == pg.FORMS["window"] and info.binned == 1


def test_tuning_table_round_trip_and_plan(tmp_path):
    lib, h = host_ctx()
    try:
        d = desc_ok(out_dtype="bf16")
        b = batch_ok(n_mol=4096, n_atoms=60000, max_atoms=29)
        st, base = plan_info(lib, h, d, b)
        assert st == pg.PG_OK and base["form"] == pg.FORMS["window"]
        key = "C5_D32_H32_W32_bf16_p0_v8_nb12_ma32"
        path = tmp_path / "t.json"
        path.write_text('{"version": 1, "arch": "x", "entries": [\n  {"key": "%s", "block": 256, '
                        '"per_cu": 3, "unroll": 4, "nt": 1, "form": 0, "us": 12.5}\n]}\n' % key)
        assert lib.pg_tuning_load(h, str(path).encode()) == pg.PG_OK
        st, tuned = plan_info(lib, h, d, b)
        assert (tuned["block"], tuned["per_cu"], tuned["unroll"], tuned["nt_store"]) == (256, 3, 4, 1)
        assert tuned["grid"] == 256 * 3
        out = tmp_path / "saved.json"
        assert lib.pg_tuning_save(h, str(out).encode()) == pg.PG_OK
        assert key in out.read_text()
        assert lib.pg_tuning_load(h, str(out).encode()) == pg.PG_OK
        assert plan_info(lib, h, d, b)[1] == tuned
    finally:
        lib.pg_destroy(h)


@pytest.mark.parametrize("text", [
    "", "{", '{"version": 2, "entries": []}', '{"version": 1, "entries": [{"key": "k"',
    '{"version": 1, "entries": [{"key": "k", "block": 256}]}',
    '{"version": 1, "entries": [{"key": "k", "block": 7, "per_cu": 1, "unroll": 1, "nt": 0, "us": 1}]}',
    '{"version": 1, "entries": [{"key": "k", "block": 256, "per_cu": 1, "unroll": 3, "nt": 0, "us": 1}]}',
    '{"version": 1, "entries": [{"key": "k", "block": 256, "per_cu": 1, "unroll": 1, "nt": 0, "us": 1, "form": 9}]}',
    '{"version": 1, "entries": [{"key": "k", "block": ', '{"version": 1, "entries": [{"key": "',
    '{"version": 1, "entries": [{"key": "k}", "block": 256, "per_cu": 1, "unroll": 1, "nt": 0}',
    "\x00\xff" * 64])
def test_tuning_load_rejects_malformed_and_truncated(tmp_path, text):
    """Malformed or truncated tables are refused and leave the table empty
    (the plan falls back to the default shape)."""
    lib, h = host_ctx()
    try:
        d = desc_ok(out_dtype="bf16")
        b = batch_ok(n_mol=4096, n_atoms=60000, max_atoms=29)
        default = plan_info(lib, h, d, b)[1]
        good = tmp_path / "good.json"
        good.write_text('{"version": 1, "entries": [{"key": "C5_D32_H32_W32_bf16_p0_v8_nb12_ma32", '
                        '"block": 256, "per_cu": 3, "unroll": 4, "nt": 1, "us": 1}]}')
        assert lib.pg_tuning_load(h, str(good).encode()) == pg.PG_OK
        assert plan_info(lib, h, d, b)[1] != default
        bad = tmp_path / "bad.json"
        bad.write_bytes(text.encode("latin-1"))
        assert lib.pg_tuning_load(h, str(bad).encode()) == pg.PG_E_PARAM
        assert plan_info(lib, h, d, b)[1] == default
        assert lib.pg_tuning_load(h, str(tmp_path / "missing.json").encode()) == pg.PG_E_PARAM
    finally:
        lib.pg_destroy(h)
