"""Every output element is written, by every form, and twice the same.

The library promises to write every element of `out` (zeros included), so
callers need not clear it.  Each case fills the output with NaN, runs the
forward map through the C ABI, and requires no NaN to remain and a second
run to give the same bits.  Shapes are ragged (not multiples of the vector
width, the wave or the 32 x 32 MFMA tile) and include structures
without atoms.  That each element is written exactly once is what the HBM
write counters show for the headline kernel (WRITE_SIZE equals the output
size), not something an output can reveal.
"""
import numpy as np
import pytest

from gpu_util import say, synth, to_device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHEAR = np.array([[8.0, 2.5, 1.0], [0.0, 7.5, -1.5], [0.0, 0.0, 8.5]])


@pytest.fixture(scope="module")
def pg():
    import paper_2211_08506_amd as pg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pg


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def batch(seed, counts, lo, hi, n_types):
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    xyz = rng.uniform(lo, hi, size=(int(off[-1]), 3)).astype(np.float32)
    return synth.Batch(xyz, rng.integers(0, n_types, int(off[-1])).astype(np.int32), off)


def covered(pg, dev, b, sig, dims, h, origin, dtype, form, **kw):
    xyz, types, offs = to_device(b, dev)
    ctx = pg.Context(0)
    desc = pg.make_desc(len(sig), dims, h, origin, sig, 3.0, kw.pop("cell", None), dtype, form,
                        kw.pop("value", "point"), cutoff_shape=kw.pop("cutoff_shape", "cube"))
    assert not kw
    bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets)
    outs = []
    for _ in range(2):
        out = pg.empty_grid(desc, b.n_mol, dev)
        out.fill_(float("nan"))
        ctx.forward(desc, bv, out)
        torch.cuda.synchronize()
        assert not torch.isnan(out).any(), (form, dtype, dims)
        outs.append(out)
    assert torch.equal(outs[0].view(torch.int16 if dtype == torch.bfloat16 else torch.int32),
                       outs[1].view(torch.int16 if dtype == torch.bfloat16 else torch.int32))
    plan = ctx.plan(desc, bv, outs[0])
    say(f"[coverage] {plan['form']}{' binned' if plan['binned'] else ''} {dtype} {dims}: "
        f"every element written, runs bitwise equal")
    return plan


@pytest.mark.parametrize("dims", [(5, 7, 33), (8, 12, 30), (3, 40, 18), (1, 1, 1)])
@pytest.mark.parametrize("form", ["window", "plain"])
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_molecule_forms(pg, dev, dims, form, dtype):
    ext = 0.3 * max(dims)
    b = batch(91, [0, 4, 9, 0, 2], -0.2 * ext, 1.2 * ext, 3)
    covered(pg, dev, b, synth.sigma_table(3, 0.25, 0.4), dims, 0.3, (0, 0, 0), dtype, form)


@pytest.mark.parametrize("dims", [(20, 37, 45), (9, 16, 200), (6, 150, 140)])
@pytest.mark.parametrize("form,dtype", [("window", torch.float32), ("window", torch.bfloat16),
                                        ("mfma", torch.bfloat16), ("mfma", torch.float32)])
def test_binned_forms(pg, dev, dims, form, dtype):
    b = batch(92, [300, 0, 450], -3.0, 3.0, 4)
    D, H, W = dims
    h = 0.17
    plan = covered(pg, dev, b, synth.sigma_table(4, 0.35, 0.6), dims, h,
                   (-0.5 * W * h, -0.5 * H * h, -0.5 * D * h), dtype, form)
    assert plan["binned"] == 1


@pytest.mark.parametrize("opts", [dict(cutoff_shape="sphere"), dict(value="box"),
                                  dict(cell=8.0), dict(cell=SHEAR)],
                         ids=["sphere", "box", "orthorhombic", "triclinic"])
@pytest.mark.parametrize("form", ["auto", "plain"])
def test_options(pg, dev, opts, form):
    b = batch(93, [6, 0, 11], 0.0, 8.0, 3)
    covered(pg, dev, b, synth.sigma_table(3, 0.3, 0.45), (26, 29, 31), 0.29, (0, 0, 0),
            torch.float32, form, **dict(opts))
