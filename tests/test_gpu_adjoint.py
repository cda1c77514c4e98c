"""GPU parity of the coordinate adjoint (dL/dxyz for L = sum(U * G)).

Checked against the FP64 oracle's analytic gradient and against FP64
central finite differences of the oracle's grid (h = 1e-4 A), per molecule
relative L2 <= 1e-4; coordinates whose cutoff window edge lies within a
few h of a voxel centre (where the windowed map is not differentiable) are
excluded from the FD comparison and counted.
"""
import numpy as np
import pytest

from gpu_util import errors, oracle, say, synth, to_device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ADJ_TOL = 1e-4


@pytest.fixture(scope="module")
def pg():
    import paper_2211_08506_amd as pg
    assert torch.cuda.is_available()
    return pg


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def gpu_grad(pg, dev, b, sigma, dims, spacing, origin, U, out_dtype=torch.float32, cell=None,
             cutoff_k=3.0, form="auto"):
    xyz, types, offs = to_device(b, dev)
    xyz.requires_grad_(True)
    g = pg.grid(xyz, types, offs, list(sigma), dims=dims, spacing=spacing, origin=origin,
                cell=cell, out_dtype=out_dtype, cutoff_k=cutoff_k, form=form)
    Ut = torch.tensor(U, device=dev).to(g.dtype)
    g.backward(Ut)
    torch.cuda.synchronize()
    return xyz.grad.double().cpu().numpy(), Ut.double().cpu().numpy()


def per_molecule_rel(got, ref, offsets):
    worst = 0.0
    for m in range(len(offsets) - 1):
        a, b = offsets[m], offsets[m + 1]
        if b > a:
            r, _ = errors(got[a:b], ref[a:b])
            worst = max(worst, r)
    return worst


def test_adjoint_vs_oracle_gradient(pg, dev):
    wl = synth.WORKLOADS["adjoint1024"]
    b = wl.batch(64)
    say("case adjoint vs oracle, 64 molecules")
    U = synth.upstream(wl.upstream_seed, wl.grid_shape(64))
    got, Uused = gpu_grad(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, U)
    ref = oracle.grad_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing, Uused,
                           wl.origin)
    rel, mx = errors(got, ref)
    wm = per_molecule_rel(got, ref, b.offsets)
    say(f"[adjoint/f32] rel-L2 {rel:.3e} max-abs {mx:.3e} worst-molecule {wm:.3e}")
    assert rel <= ADJ_TOL and wm <= ADJ_TOL


def test_adjoint_bf16_upstream(pg, dev):
    """A bf16 grid's gradient arrives in bf16; the oracle takes the same
    (rounded) upstream values, so the bar is still the FP32 one."""
    wl = synth.WORKLOADS["adjoint1024"]
    b = wl.batch(16)
    say("case adjoint bf16 upstream")
    U = synth.upstream(wl.upstream_seed, wl.grid_shape(16))
    got, Uused = gpu_grad(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, U,
                          out_dtype=torch.bfloat16)
    ref = oracle.grad_fp64(b.xyz, b.types, b.offsets, wl.sigma(), wl.dims, wl.spacing, Uused,
                           wl.origin)
    rel, mx = errors(got, ref)
    say(f"[adjoint/bf16-upstream] rel-L2 {rel:.3e} max-abs {mx:.3e}")
    assert rel <= ADJ_TOL


def test_adjoint_periodic(pg, dev):
    say("case adjoint periodic")
    rng = np.random.default_rng(31)
    sig = synth.sigma_table(3, 0.3, 0.45)
    counts = [40, 9]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    xyz = rng.uniform(0, 8.0, size=(off[-1], 3)).astype(np.float32)
    xyz[0] = [0.02, 7.97, 4.0]
    b = synth.Batch(xyz, rng.integers(0, 3, off[-1]).astype(np.int32), off)
    dims, h = (40, 40, 40), 0.21
    U = synth.upstream(3, (2, 3) + dims)
    got, Uused = gpu_grad(pg, dev, b, sig, dims, h, (0, 0, 0), U, cell=8.0)
    ref = oracle.grad_fp64(b.xyz, b.types, b.offsets, sig, dims, h, Uused, (0, 0, 0), cell=8.0)
    rel, mx = errors(got, ref)
    say(f"[adjoint/periodic] rel-L2 {rel:.3e} max-abs {mx:.3e}")
    assert rel <= ADJ_TOL


def _differentiable(mu, o, h, n, rc, eps):
    for q in range(3):
        d = o[q] + (np.arange(n) + 0.5) * h - mu[q]
        if np.any(np.abs(np.abs(d) - rc) < eps):
            return False
    return True


def test_adjoint_vs_finite_differences(pg, dev):
    """16 molecules of the adjoint workload: GPU dL/dxyz vs FP64 central
    differences of the oracle's grid, h = 1e-4 A."""
    wl = synth.WORKLOADS["adjoint1024"]
    nm = 16
    b = wl.batch(nm)
    say("case adjoint vs FD, 16 molecules")
    U = synth.upstream(wl.upstream_seed, wl.grid_shape(nm))
    got, Uused = gpu_grad(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, U)
    sig = wl.sigma()
    hfd = 1e-4
    excluded = 0
    worst = 0.0
    for m in range(nm):
        s = b.subset([m])
        Um = Uused[m:m + 1]
        xyz = s.xyz.astype(np.float64)
        fd = np.zeros_like(xyz)
        keep = np.ones(xyz.shape, dtype=bool)
        for a in range(s.n_atoms):
            rc = float(np.float32(wl.cutoff_k) * sig[s.types[a]])
            if not _differentiable(xyz[a], wl.origin, wl.spacing, wl.dims[0], rc, 2 * hfd):
                keep[a] = False
                excluded += 3
                continue
            for q in range(3):
                xp, xm = xyz.copy(), xyz.copy()
                xp[a, q] += hfd
                xm[a, q] -= hfd
                lp = np.sum(Um * oracle.grid_fp64(xp, s.types, s.offsets, sig, wl.dims, wl.spacing,
                                                  wl.origin))
                lm = np.sum(Um * oracle.grid_fp64(xm, s.types, s.offsets, sig, wl.dims, wl.spacing,
                                                  wl.origin))
                fd[a, q] = (lp - lm) / (2 * hfd)
        g = got[b.offsets[m]:b.offsets[m + 1]]
        rel, _ = errors(g[keep], fd[keep])
        worst = max(worst, rel)
    say(f"[adjoint vs FD] worst per-molecule rel-L2 {worst:.3e}; excluded coords {excluded}")
    assert worst <= ADJ_TOL


def test_adjoint_full_size_1024(pg, dev):
    """All 1024 molecules of the adjoint workload vs the oracle gradient."""
    wl = synth.WORKLOADS["adjoint1024"]
    b = wl.batch()
    say("case adjoint full size 1024")
    U = synth.upstream(wl.upstream_seed, wl.grid_shape())
    got, _ = gpu_grad(pg, dev, b, wl.sigma(), wl.dims, wl.spacing, wl.origin, U)
    worst = 0.0
    num = den = 0.0
    for c0 in range(0, b.n_mol, 128):
        idx = list(range(c0, min(b.n_mol, c0 + 128)))
        s = b.subset(idx)
        ref = oracle.grad_fp64(s.xyz, s.types, s.offsets, wl.sigma(), wl.dims, wl.spacing,
                               U[c0:c0 + len(idx)].astype(np.float64), wl.origin)
        g = got[b.offsets[c0]:b.offsets[c0 + len(idx)]]
        num += np.sum((g - ref) ** 2)
        den += np.sum(ref ** 2)
        worst = max(worst, per_molecule_rel(g, ref, s.offsets))
    rel = float(np.sqrt(num / den))
    say(f"[adjoint 1024] rel-L2 {rel:.3e} worst-molecule {worst:.3e}")
    assert rel <= ADJ_TOL and worst <= ADJ_TOL


@pytest.mark.parametrize("dims", [(5, 7, 90), (6, 20, 9), (12, 10, 1)],
                         ids=["x_wider_than_a_wave", "y_carries", "single_x_column"])
def test_adjoint_whole_grid_windows(pg, dev, dims):
    """No cutoff (k = 0): every window is the whole grid, so a lane's window
    elements run over many rounds and the lane's (x, y, z) position in the
    window is stepped by 64 with carries in every digit: x rows longer than
    a wave (90), carries from x into y and from y into z (9 x 20), and a
    single x column (nx = 1)."""
    D, H, W = dims
    h = 0.3
    rng = np.random.default_rng(sum(dims))
    counts = [3, 0, 5]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    ext = np.array([W, H, D]) * h
    xyz = (rng.uniform(0.1, 0.9, size=(int(off[-1]), 3)) * ext).astype(np.float32)
    types = rng.integers(0, 3, int(off[-1])).astype(np.int32)
    b = synth.Batch(xyz, types, off)
    sig = synth.sigma_table(3, 0.45, 0.8)
    say(f"case adjoint whole-grid windows, dims {dims}")
    U = synth.upstream(41, (len(counts), 3) + dims)
    got, Uused = gpu_grad(pg, dev, b, sig, dims, h, (0, 0, 0), U, cutoff_k=0.0)
    ref = oracle.grad_fp64(b.xyz, b.types, b.offsets, sig, dims, h, Uused, (0, 0, 0),
                           cutoff_k=0.0)
    rel, mx = errors(got, ref)
    wm = per_molecule_rel(got, ref, b.offsets)
    say(f"[adjoint/whole grid {dims}] rel-L2 {rel:.3e} max-abs {mx:.3e} worst-molecule {wm:.3e}")
    assert rel <= ADJ_TOL and wm <= ADJ_TOL
