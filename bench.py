"""Benchmark of the atoms -> density-grid hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload mol4096]
                    [--value point|box] [--no-cpu] [--no-baseline]

A step is one pass of the forward hot path over one batch: inputs are
staged in HBM once, then each step runs the per-atom window bounds and 1-D
factors, the accumulation and the dense write of the whole B x C x D x H x W
grid (for molecules one persistent window-kernel launch; for large periodic
cells the binned path's set-up kernels and its plane kernel), launched
directly: replaying captured HIP graphs (--graph) measured slower on MI355X
for every sequence here.  Rank 0 prints
one JSON line on stdout; progress goes to stderr.

Workloads (synth.WORKLOADS):
  mol4096      (default, headline) 4096 molecules of 5-29 atoms, 32^3 x 5
               channels at 0.5 A, bf16 output, beside the plain per-molecule
               fp32 baseline (one launch per molecule), the batched fp32
               form and a torch fill of the same byte count;
  mol4096x48   4096 molecules of 5-60 atoms, 48^3 x 5 at 0.35 A, bf16;
  crystal8     8 periodic 20 A cells of 2000-20000 atoms, 128^3 x 8 at
               0.16 A: bf16 (MFMA plane kernel) beside the fp32 vector form;
  adjoint1024  the coordinate gradient of 1024 molecules, 32^3 x 5 fp32
               upstream;
  reversal1024 one grid-reversal step (residual, loss, coordinate gradient
               and update) of 1024 molecules against fp32 32^3 x 5 targets.
--value box measures the box form (each voxel holds the normalised
Gaussian's mass inside it) instead of the point-sampled Gaussian.
The FP64 CPU oracle is timed on a bounded sample of the same workload, one
thread and a thread pool (the oracle releases the GIL).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HEADLINE_METRIC = ("grids/sec + HBM GB/s (32³×5ch, batch 4096): batched BF16 vs plain FP32")
METRICS = {
    "mol4096": HEADLINE_METRIC,
    "mol4096x48": "grids/sec + HBM GB/s (48³×5ch, batch 4096, 5-60 atoms): batched BF16",
    "crystal8": "grids/sec + HBM GB/s (128³×8ch periodic cells, batch 8): BF16 MFMA vs FP32 window",
    "adjoint1024": "grids/sec (adjoint dL/dxyz, 32³×5ch FP32 upstream, batch 1024)",
    "reversal1024": "grids/sec (grid-reversal step: residual + loss + dL/dxyz + update, "
                    "32³×5ch FP32, batch 1024)",
}
PEAK_HBM_GBS = 8000.0
WINDOW_SOURCES = ("paper_2211_08506_amd/csrc/pg_window.hip", "paper_2211_08506_amd/csrc/pg_device.hpp",
                  "paper_2211_08506_amd/csrc/pg_params.hpp")
CPU_THREADS_MAX = 16


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key: str, digest: str):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, only if
    they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            tab = json.load(f)
    except (OSError, ValueError):
        return None
    ent = tab.get(kernel_key)
    if not ent or ent.get("source_digest") != digest:
        return None
    return ent.get("bytes_per_launch")


def timed_steps(fn, steps, warmup, torch, stream):
    """Run warmup + timed steps bracketed by synchronisations; each step is
    also bracketed by events on the launch stream.  Returns wall ms/step and
    event statistics (mean, median, p10, p90 in ms)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    per = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    return wall, {"mean": float(per.mean()), "median": float(np.median(per)),
                  "p10": float(np.percentile(per, 10)), "p90": float(np.percentile(per, 90))}


def axis_windows(b, wl):
    """Per atom and axis, the voxel index ranges of the cutoff window
    (nearest images included when periodic), evaluated in float64: a
    measurement aid for eval counts and dense-contraction sizes (edge voxels
    may differ from the exact decision the kernels take)."""
    o = np.asarray(wl.origin, np.float64)
    h = float(wl.spacing)
    dims_xyz = (wl.dims[2], wl.dims[1], wl.dims[0])
    rc = (np.float32(wl.cutoff_k) * wl.sigma().astype(np.float32)).astype(np.float64)[b.types]
    mu = b.xyz.astype(np.float64)
    images = (-1, 0, 1) if wl.periodic else (0,)
    ranges = []
    for q in range(3):
        rq = []
        for n in images:
            c = mu[:, q] + n * (wl.cell or 0.0) - o[q]
            lo = np.maximum(np.ceil((c - rc) / h - 0.5), 0).astype(np.int64)
            hi = np.minimum(np.floor((c + rc) / h - 0.5), dims_xyz[q] - 1).astype(np.int64)
            rq.append((lo, hi))
        ranges.append(rq)
    return ranges


def window_evals(b, wl) -> int:
    """Atom-voxel evaluations of one pass: sum over atoms of window sizes."""
    cnt = []
    for rq in axis_windows(b, wl):
        cnt.append(sum(np.maximum(hi - lo + 1, 0) for lo, hi in rq))
    return int(np.sum(cnt[0] * cnt[1] * cnt[2]))


def parity_stats(got, ref, what):
    """Error of the GPU result against the FP64 oracle on the same structures:
    whole-sample rel-L2 and max-abs, and the worst structure's rel-L2 (axis 0
    indexes structures)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    rel = float(np.linalg.norm(got - ref) / den) if den > 0 else float(np.linalg.norm(got - ref))
    worst = 0.0
    for m in range(ref.shape[0]):
        d = np.linalg.norm(ref[m])
        e = np.linalg.norm(got[m] - ref[m])
        worst = max(worst, float(e / d) if d > 0 else float(e))
    out = {"of": what, "rel_l2": rel, "max_abs": float(np.max(np.abs(got - ref))) if got.size else 0.0,
           "worst_structure_rel_l2": worst, "n_structures": int(ref.shape[0])}
    log(f"[bench] parity vs FP64 oracle ({what}): rel-L2 {rel:.3e}, max-abs {out['max_abs']:.3e}, "
        f"worst structure rel-L2 {worst:.3e} over {ref.shape[0]} structures")
    return out


# The paper's own CPU figures (context, not targets: the paper computes
# the normalised erf voxel integral on one CPU core with AVX, and prints
# mostly relative speedups; its absolute molecules/s are in a figure).
PAPER_CPU_CONTEXT = [
    {"figure": "truncation (zero-range skipping) over the base C++ grid code", "value": "~7x average",
     "hardware": "Intel Xeon Silver 4114 @ 2.2 GHz, GCC 7.5, FP32", "section": "VI-B"},
    {"figure": "AVX on top of truncation", "value": "< 2% for grids of 64^3 and up",
     "hardware": "Xeon Silver 4114 (256-bit AVX)", "section": "VI-C, VI-D"},
    {"figure": "optimised vs base C++", "value": "over 15x (14x in the conclusion)",
     "hardware": "Xeon Silver 4114", "section": "VI-D, IX"},
    {"figure": "optimised vs NumPy / Numba", "value": "up to 9000x / 79.5x",
     "hardware": "Xeon Silver 4114", "section": "VI-D"},
    {"figure": "training with grids made on the fly (PCQM4Mv2, 1 channel, 32^3, batch 256)",
     "value": "166 s per epoch, i.e. >= ~17.9k grids/s sustained including the CNN",
     "hardware": "AMD EPYC 7F52 (16 cores) + 4x NVIDIA A100 40 GB", "section": "VII-C, VII-D"},
]


def _oracle_call(spec):
    """One FP64 oracle call of the CPU baseline leg, in this process or in a
    pool worker: spec = (entry, args, kwargs, grids); returns the grids."""
    name, a, kw, n = spec
    import oracle as cpu_oracle
    if name == "grid":
        cpu_oracle.grid_fp64(*a, **kw)
    elif name == "grid_tri":
        from oracle import triclinic as cpu_triclinic
        cpu_triclinic.grid_triclinic_fp64(*a, **kw)
    elif name == "grad":
        cpu_oracle.grad_fp64(*a, **kw)
    elif name == "rev":
        from oracle import reversal as cpu_reversal
        cpu_reversal.reversal_step(*a, **kw)
    return n


def cpu_oracle_baseline(units, make_spec, seconds, describe, max_procs=None, pool_units=None):
    """Time the FP64 oracle on a bounded sample: make_spec(unit) describes
    one oracle call (_oracle_call) over the unit's structures; units are
    taken cycling through the list, first in this process, then on P worker
    processes (spawned, so they share nothing with this process's GPU state)
    with one task per unit of pool_units (a molecule's grid takes about a
    tenth of a millisecond, so tasks of 16 molecules keep the inter-process
    traffic small; a crystal cell is a task).  P is the process's CPU affinity,
    capped at the host share of one GPU (16 cores); the pool is started and
    its workers have imported the oracle before the clock starts."""
    import multiprocessing
    t0 = time.perf_counter()
    n1 = i = 0
    while time.perf_counter() - t0 < seconds * 0.6 or i < 1:
        n1 += _oracle_call(make_spec(units[i % len(units)]))
        i += 1
    dt1 = time.perf_counter() - t0
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    P = max(1, min(max_procs or CPU_THREADS_MAX, avail))
    pool_units = pool_units or units
    nP = i = 0
    with cf.ProcessPoolExecutor(P, mp_context=multiprocessing.get_context("spawn")) as ex:
        warm = make_spec(pool_units[0])
        list(ex.map(_oracle_call, [warm] * P))   # worker start-up and imports, untimed
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds * 0.4 or i < P:
            nP += sum(ex.map(_oracle_call, [make_spec(pool_units[(i + j) % len(pool_units)])
                                            for j in range(4 * P)], chunksize=2))
            i += 4 * P
        dtP = time.perf_counter() - t0
    log(f"[bench] oracle: 1 process {n1} grids in {dt1:.1f} s; {P} processes {nP} in {dtP:.1f} s")
    return {"value": n1 / dt1, "unit": "grids/s", "cores": 1, "kind": "oracle",
            "sample": describe(n1, dt1, 1, False),
            "processes": {"value": nP / dtP, "unit": "grids/s", "cores": P, "affinity": avail,
                          "sample": describe(nP, dtP, P, True)},
            "paper_cpu_context": PAPER_CPU_CONTEXT}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="mol4096", choices=sorted(METRICS))
    ap.add_argument("--value", default="point", choices=("point", "box"),
                    help="voxel value: the Gaussian at the centre, or its mass in the voxel")
    ap.add_argument("--triclinic", action="store_true",
                    help="crystal8 in a sheared (triclinic) cell of the same edge length")
    ap.add_argument("--embed", type=int, default=0,
                    help="weighted channels: a dense seeded embedding of the element types "
                         "into this many channels (forward workloads)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-baseline", action="store_true", help="skip the plain fp32 baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--autotune", action="store_true",
                    help="re-measure the launch shapes before timing (default: the shipped "
                         "tuning table, so the timed launch is the one the committed kernel "
                         "traces show)")
    ap.add_argument("--no-autotune", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--parity-structures", type=int, default=64,
                    help="structures of the timed output compared with the FP64 oracle "
                         "(all of them for the crystal workload)")
    ap.add_argument("--graph", action="store_true",
                    help="replay captured HIP graphs (the library's graph option) instead of direct "
                         "launches; direct launches measured faster on MI355X")
    ap.add_argument("--save-tuning", default=None, help="write the tuning table to this path")
    ap.add_argument("--tuning", default=None, help="load this tuning table (instead of the shipped one)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference kernel for counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "batches shard across GPUs by structure without communication (see the design "
              "notes), and no multi-GPU figure is produced", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2211_08506_amd as pg
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    wl = synth.WORKLOADS[args.workload]
    log(f"[bench] generating {wl.name}: {wl.n_mol} structures")
    b = wl.batch()
    sig = wl.sigma()
    cell = wl.cell
    if args.triclinic:
        if wl.kind != "crystal":
            print("bench.py: --triclinic applies to the crystal workload", file=sys.stderr)
            sys.exit(2)
        # the same fractional positions in a sheared cell: column j of the
        # matrix is lattice vector j
        cell = wl.cell * np.array([[1.0, 0.15, 0.1], [0.0, 1.0, -0.15], [0.0, 0.0, 1.0]])
        b.xyz = ((b.xyz.astype(np.float64) / wl.cell) @ cell.T).astype(np.float32)
    xyz = torch.tensor(b.xyz, device=dev)
    types = torch.tensor(b.types, device=dev)
    offs = torch.tensor(b.offsets, device=dev)
    B = b.n_mol
    C = wl.n_types
    ntypes = 0
    E = None
    if args.embed:
        if wl.name in ("adjoint1024", "reversal1024") or args.triclinic:
            print("bench.py: --embed applies to the forward workloads (not triclinic cells)",
                  file=sys.stderr)
            sys.exit(2)
        table = synth.embedding(wl.seed + 100, wl.n_types, args.embed)
        E = table[b.types]
        C, ntypes = args.embed, wl.n_types
    bv = pg.BatchView(xyz, types, offs, offsets_host=b.offsets,
                      weights=None if E is None else torch.tensor(E, device=dev))
    D, H, W = wl.dims
    vox = C * D * H * W
    in_bytes = 16 * b.n_atoms + 4 * (B + 1) + (4 * C * b.n_atoms if E is not None else 0)
    # a dense embedding adds every atom to every channel
    evals = window_evals(b, wl) * (C if E is not None else 1)
    log(f"[bench] {b.n_atoms} atoms, {evals} atom-voxel evaluations per pass")

    ctx = pg.Context(0, tuning=args.tuning or "shipped")
    ctx.set_option(pg.PG_OPT_GRAPH, 1 if args.graph else 0)
    launch = "HIP graph" if args.graph else "direct launches"
    extra = {}
    value = args.value
    metric = METRICS[wl.name] + (" [box form]" if value == "box" else "") + \
        (f" [embedding {wl.n_types} types -> {C} channels]" if E is not None else "") + \
        (" [triclinic cells]" if args.triclinic else "")
    rec = {"metric": metric, "unit": "grids/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "data": "synthetic"}

    def forward_case(out_dt, form, autotune, steps, warmup):
        desc = pg.make_desc(C, wl.dims, wl.spacing, wl.origin, sig, wl.cutoff_k, cell,
                            out_dt, form, value, ntypes)
        out = pg.empty_grid(desc, B, dev)
        if autotune and args.autotune and not args.triclinic:
            log(f"[bench] autotuning {form} {out_dt}")
            ctx.autotune(desc, bv, out, reps=3)
        plan = ctx.plan(desc, bv, out)
        wall, ev = timed_steps(lambda: ctx.forward(desc, bv, out, stream), steps, warmup,
                               torch, stream)
        esz = 2 if out_dt == torch.bfloat16 else 4
        alg = B * vox * esz + in_bytes
        res = {"plan": plan, "ms_per_step": wall, "launch_ms": ev, "grids_per_s": B / (wall / 1e3),
               "alg_bytes": alg, "hbm_gbs": alg / (ev["mean"] / 1e3) / 1e9,
               "evals_per_s": evals / (ev["mean"] / 1e3)}
        log(f"[bench] {form} {out_dt} plan {plan}")
        log(f"[bench]   {wall:.3f} ms/step wall, {ev['mean']:.3f} ms/step (events, median "
            f"{ev['median']:.3f}), {res['grids_per_s'] / 1e6:.3f} M grids/s, "
            f"{res['hbm_gbs']:.0f} GB/s algorithmic")
        return desc, out, res

    if wl.name == "adjoint1024":
        desc = pg.make_desc(C, wl.dims, wl.spacing, wl.origin, sig, wl.cutoff_k, wl.cell,
                            torch.float32, "auto", value)
        U = torch.tensor(synth.upstream(wl.upstream_seed, wl.grid_shape()), device=dev)
        gxyz = torch.empty_like(xyz)
        wall, ev = timed_steps(lambda: ctx.backward(desc, bv, U, gxyz, stream), args.steps,
                               args.warmup, torch, stream)
        n_par = min(B, args.parity_structures)
        par_got = gxyz[:int(b.offsets[n_par])].double().cpu().numpy()
        # algorithmic bytes: the upstream values inside every window, the
        # inputs, and the gradient written
        alg = evals * 4 + in_bytes + 12 * b.n_atoms
        achieved = alg / (ev["mean"] / 1e3) / 1e9
        log(f"[bench] adjoint: {wall:.3f} ms/step wall, {ev['mean']:.3f} ms (events), "
            f"{B / (wall / 1e3) / 1e6:.3f} M grids/s, {achieved:.0f} GB/s algorithmic")
        rec.update({"value": B / (wall / 1e3), "ms_per_step": wall, "dtype": "f32",
                    "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                                 "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                                 "traffic": None, "kernel": "adjoint_kernel<float>",
                                 "algorithmic_bytes_per_launch": alg, "launch_ms": ev},
                    "evals_per_s": evals / (ev["mean"] / 1e3),
                    "upstream_bytes_read_dense": B * vox * 4})
        kind = "adjoint"
    elif wl.name == "reversal1024":
        desc = pg.make_desc(C, wl.dims, wl.spacing, wl.origin, sig, wl.cutoff_k, wl.cell,
                            torch.float32, "auto", value)
        # targets: the grids of the generating coordinates; the step starts
        # from displaced coordinates and updates them in place
        target = pg.empty_grid(desc, B, dev)
        ctx.forward(desc, bv, target, stream)
        x0 = b.xyz + synth.perturbation(wl.upstream_seed, b.n_atoms, 0.15)
        bvp = pg.BatchView(torch.tensor(x0, device=dev), types, offs, offsets_host=b.offsets)
        residual = torch.empty_like(target)
        loss = torch.empty(B, dtype=torch.float32, device=dev)
        lr = 0.01 if value == "point" else 2.0
        # no autotuning here: the tuner times the forward that writes the
        # grid, while the step's forward reads the target instead, and the
        # shape the tuner picks for the write (one run per lane) is slower
        # for the read (0.237 against 0.205 ms per box step); the step keeps
        # the shipped or default shape
        plan = ctx.plan(desc, bvp, residual)
        loss0 = None

        # the step keeps no residual grid where the library allows it (the
        # molecule window form): the adjoint forms the residual in the windows
        keep = not (plan["form"] == "window" and not plan["binned"] and E is None)
        res_arg = residual if keep else None

        def step():
            ctx.reversal_step(desc, bvp, target, res_arg, loss, None, bvp.xyz, lr, stream)

        step()
        torch.cuda.synchronize()
        loss0 = float(loss.sum().item())
        n_par = min(B, args.parity_structures)
        par_got = (loss[:n_par].double().cpu().numpy(),
                   bvp.xyz[:int(b.offsets[n_par])].double().cpu().numpy())
        wall, ev = timed_steps(step, args.steps, args.warmup, torch, stream)
        loss1 = float(loss.sum().item())
        # algorithmic bytes: the target read once (and the residual written
        # once when kept), the target (or residual) re-read inside every
        # window by the adjoint, the inputs, and the coordinates read and
        # written
        alg = (8 if keep else 4) * B * vox + evals * 4 + in_bytes + 24 * b.n_atoms
        achieved = alg / (ev["mean"] / 1e3) / 1e9
        if not keep:
            # the same step with the residual grid written, for comparison
            def step_res():
                ctx.reversal_step(desc, bvp, target, residual, loss, None, bvp.xyz, lr, stream)
            w2, e2 = timed_steps(step_res, max(5, args.steps // 2), 2, torch, stream)
            extra["with_residual_grid"] = {"ms_per_step": w2, "launch_ms": e2,
                                           "grids_per_s": B / (w2 / 1e3)}
            log(f"[bench]   with the residual grid written: {w2:.3f} ms/step wall, "
                f"{e2['mean']:.3f} ms (events)")
        log(f"[bench] reversal step: plan {plan}")
        log(f"[bench]   {wall:.3f} ms/step wall, {ev['mean']:.3f} ms (events), "
            f"{B / (wall / 1e3) / 1e6:.3f} M grids/s, {achieved:.0f} GB/s algorithmic; "
            f"loss {loss0:.4e} -> {loss1:.4e} over {args.steps + args.warmup + 1} steps")
        kname = (f"whole step: window_mol_kernel<float,{plan['vec']},{plan['unroll']},residual>"
                 + (" + adjoint_kernel<float> (update)" if keep else
                    " (no residual grid) + adjoint_kernel<float, recompute> (update)"))
        rec.update({"value": B / (wall / 1e3), "ms_per_step": wall, "dtype": "f32",
                    "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                                 "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                                 "traffic": None, "kernel": kname,
                                 "algorithmic_bytes_per_launch": alg, "launch_ms": ev},
                    "loss_first_step": loss0, "loss_last_step": loss1,
                    "residual_grid_kept": keep})
        kind = "reversal step"
        Th = None if args.no_cpu else target.cpu().numpy()   # the CPU leg's targets
    else:
        out_dt = torch.bfloat16 if wl.out_dtype == "bf16" or wl.kind == "crystal" else torch.float32
        desc, out, main_res = forward_case(out_dt, "auto", True, args.steps, args.warmup)
        esize = 2 if out_dt == torch.bfloat16 else 4
        achieved = main_res["hbm_gbs"]
        plan = main_res["plan"]
        # practical write ceiling: torch fill of the same byte count
        n_par = B if wl.kind == "crystal" else min(B, args.parity_structures)
        par_got = out[:n_par].float().cpu().numpy() if not args.no_cpu else None
        fill_buf = out.view(torch.uint8).view(-1)
        _, fill_ev = timed_steps(lambda: fill_buf.fill_(0), 10, 3, torch, stream)
        fill_gbs = B * vox * esize / (fill_ev["mean"] / 1e3) / 1e9
        log(f"[bench] torch fill of {B * vox * esize / 1e9:.2f} GB: {fill_ev['mean']:.3f} ms, "
            f"{fill_gbs:.0f} GB/s")
        del out
        if wl.kind == "crystal":
            kname = ("binned path, whole step: cr_clear, cr_prep, cr_scan, cr_place, "
                     + (f"cr_sort_slot, cr_tile_{'bf16' if esize == 2 else 'f32'}_kernel"
                        if plan["form"] == "mfma" else "cr_zsort, cr_window_kernel"))
            # the other form / dtype pairs, for the per-shape decision
            for form, dt in (("mfma", torch.bfloat16), ("window", torch.float32),
                             ("window", torch.bfloat16), ("mfma", torch.float32)):
                if form == plan["form"] and dt == out_dt:
                    continue
                _, o2, r2 = forward_case(dt, form, False, max(5, args.steps // 2), 2)
                extra[f"{form}_{'bf16' if dt == torch.bfloat16 else 'fp32'}"] = {
                    k: r2[k] for k in ("ms_per_step", "launch_ms", "grids_per_s", "hbm_gbs",
                                       "evals_per_s")}
                del o2
        else:
            kname = (f"window_mol_kernel<{'bf16' if esize == 2 else 'float'},"
                     f"{plan['vec']},{plan['unroll']}>")
        if wl.name == "mol4096":
            _, o32, r32 = forward_case(torch.float32, "auto", True, max(5, args.steps // 5), 2)
            extra["batched_fp32"] = {k: r32[k] for k in ("ms_per_step", "launch_ms",
                                                         "grids_per_s", "hbm_gbs")}
            del o32
            if not args.no_baseline:
                ctx_p = pg.Context(0)
                descp = pg.make_desc(C, wl.dims, wl.spacing, wl.origin, sig, wl.cutoff_k,
                                     cell, torch.float32, "plain", value, ntypes)
                outp = pg.empty_grid(descp, B, dev)
                wp, ep = timed_steps(lambda: ctx_p.forward(descp, bv, outp, stream), 3, 1, torch,
                                     stream)
                extra["baseline_plain_fp32"] = {
                    "grids_per_s": B / (wp / 1e3), "ms_per_step": wp, "launches_per_step": B + 1,
                    "hbm_gbs": (B * vox * 4 + in_bytes) / (ep["mean"] / 1e3) / 1e9}
                log(f"[bench] plain fp32 per-molecule launches: {wp:.2f} ms/step, "
                    f"{B / (wp / 1e3) / 1e6:.3f} M grids/s")
                del outp
        if args.save_tuning:
            ctx.tuning_save(args.save_tuning)
        traffic = None
        if wl.kind != "crystal" and value == "point" and E is None:
            traffic = measured_traffic(f"window_{wl.name}_{'bf16' if esize == 2 else 'f32'}",
                                       source_digest(WINDOW_SOURCES))
        rec.update({
            "value": main_res["grids_per_s"], "ms_per_step": main_res["ms_per_step"],
            "dtype": "bf16" if esize == 2 else "f32",
            "hbm_gbs": achieved,
            "evals_per_s": main_res["evals_per_s"],
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                         "kernel": kname, "algorithmic_bytes_per_launch": main_res["alg_bytes"],
                         "launch_ms": main_res["launch_ms"]},
            "fill_gbs_same_bytes": fill_gbs,
            "frac_of_fill": achieved / fill_gbs,
        })
        kind = "forward"
        if args.graph and plan["form"] == "window" and not plan["binned"]:
            # the library launches its one-kernel molecule form directly
            launch = "direct launch (one kernel; the graph option replays only multi-kernel steps)"

    if wl.kind == "crystal":
        shape = "triclinic (sheared) cells of edge" if args.triclinic else "cubic cells of"
        desc_w = (f"{wl.name}: {B} periodic {shape} {wl.cell:g} A, "
                  f"{min(b.counts())}-{max(b.counts())} atoms (uniform positions, {C} types uniform)")
    else:
        desc_w = (f"{wl.name}: {B} molecules of {wl.atoms[0]}-{wl.atoms[1]} atoms "
                  f"(H/C/N/O/F p=0.5/0.3/0.1/0.08/0.02, {wl.box:g} A box)")
    if E is not None:
        desc_w += f", weighted channels: dense U(0.1, 1) embedding of {wl.n_types} types"
    rec["config"] = {"workload": f"{desc_w}, {C}x{D}x{H}x{W} grid at {wl.spacing} A, cutoff "
                                 f"{wl.cutoff_k:g} sigma, {kind}, {value} form, {launch}",
                     "batch": B, "grid": [C, D, H, W], "n_atoms": int(b.n_atoms),
                     "evals_per_pass": evals}
    if kind in ("forward", "reversal step"):
        rec["config"]["plan"] = plan
    if kind == "reversal step":
        rec["config"]["start"] = "generating coordinates displaced by U(-0.15, 0.15) A per axis"

    cpu = None
    if not args.no_cpu:
        # the CPU baseline leg: the FP64 oracle (test infrastructure) on the
        # same structures, one structure per call
        import oracle as cpu_oracle
        chunk = 1 if wl.kind == "crystal" else 16
        units = [(m, b.subset(range(m, min(B, m + chunk)))) for m in range(0, B, chunk)]
        if kind == "reversal step":
            from oracle import reversal as cpu_reversal

            def make_spec(u):
                m, s = u
                a0, a1 = b.offsets[m], b.offsets[m + s.n_mol]
                return ("rev", (x0[a0:a1], s.types, s.offsets, sig, wl.dims, wl.spacing,
                                Th[m:m + s.n_mol], lr, wl.origin),
                        {"cutoff_k": wl.cutoff_k, "value": value}, s.n_mol)
        elif kind == "adjoint":
            Uh = synth.upstream(wl.upstream_seed, wl.grid_shape())

            def make_spec(u):
                m, s = u
                return ("grad", (s.xyz, s.types, s.offsets, sig, wl.dims, wl.spacing,
                                 Uh[m:m + s.n_mol], wl.origin),
                        {"cutoff_k": wl.cutoff_k, "value": value}, s.n_mol)
        else:
            def make_spec(u):
                s = u[1]
                if args.triclinic:
                    return ("grid_tri", (s.xyz, s.types, s.offsets, sig, wl.dims, wl.spacing,
                                         cell, wl.origin),
                            {"cutoff_k": wl.cutoff_k, "value": value}, s.n_mol)
                return ("grid", (s.xyz, s.types, s.offsets, sig, wl.dims, wl.spacing, wl.origin),
                        {"cutoff_k": wl.cutoff_k, "cell": wl.cell, "value": value,
                         "weights": None if E is None else table[s.types]}, s.n_mol)
        pool_units = units
        log(f"[bench] FP64 CPU oracle on a bounded sample (~{args.cpu_seconds:.0f} s)")
        per_unit = "cell" if wl.kind == "crystal" else "molecule"
        cpu = cpu_oracle_baseline(
            units, make_spec, args.cpu_seconds,
            lambda n, dt, P, pool: (
                f"{n} {kind} grids of the {B}-structure batch, {1 if pool else chunk} "
                f"{per_unit}(s) per oracle call cycling through the batch ({n / B:.2f} passes), "
                f"dense FP64 {C}x{D}x{H}x{W}, {P} process(es), {dt:.1f} s"),
            pool_units=pool_units)
    rec["cpu_baseline"] = cpu

    if not args.no_cpu:
        # parity of the timed result: the first structures of the batch
        # against the FP64 oracle (the same structures, one oracle call)
        sub = b.subset(range(n_par))
        if kind == "forward":
            if args.triclinic:
                from oracle import triclinic as cpu_triclinic
                ref = cpu_triclinic.grid_triclinic_fp64(sub.xyz, sub.types, sub.offsets, sig,
                                                        wl.dims, wl.spacing, cell, wl.origin,
                                                        cutoff_k=wl.cutoff_k, value=value)
            else:
                ref = cpu_oracle.grid_fp64(sub.xyz, sub.types, sub.offsets, sig, wl.dims,
                                           wl.spacing, wl.origin, cutoff_k=wl.cutoff_k,
                                           cell=wl.cell, value=value,
                                           weights=None if E is None else table[sub.types])
            rec["parity"] = parity_stats(par_got, ref, f"timed {rec['dtype']} grids")
        elif kind == "adjoint":
            ref = cpu_oracle.grad_fp64(sub.xyz, sub.types, sub.offsets, sig, wl.dims, wl.spacing,
                                       Uh[:n_par], wl.origin, cutoff_k=wl.cutoff_k, value=value)
            a_of = np.searchsorted(sub.offsets, np.arange(sub.n_atoms), side="right") - 1
            got_m = [par_got[a_of == m] for m in range(n_par)]
            ref_m = [ref[a_of == m] for m in range(n_par)]
            st = parity_stats(par_got[None], ref[None], "dL/dxyz of the timed pass")
            st["worst_structure_rel_l2"] = max(
                float(np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300))
                for g, r in zip(got_m, ref_m) if len(r))
            st["n_structures"] = n_par
            rec["parity"] = st
        else:
            a1 = int(b.offsets[n_par])
            loss_r, _, _, xyz_r = cpu_reversal.reversal_step(
                x0[:a1], sub.types, sub.offsets, sig, wl.dims, wl.spacing, Th[:n_par], lr,
                wl.origin, cutoff_k=wl.cutoff_k, value=value)
            st = parity_stats(par_got[0][:, None], loss_r[:, None], "loss of the first step")
            st["updated_xyz_max_abs"] = float(np.max(np.abs(par_got[1] - xyz_r)))
            log(f"[bench]   updated coordinates: max-abs {st['updated_xyz_max_abs']:.3e} A")
            rec["parity"] = st

    if args.calibrate_copy:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] calibration copy: 3 x 1 GiB")

    # the same roofline on the wall-clock time per step (ms_per_step), beside
    # the per-launch event time that `achieved` and `frac` use
    rf = rec["roofline"]
    work = rf.get("algorithmic_flops_per_launch") if rf["bound"] == "mfma" else \
        rf["algorithmic_bytes_per_launch"]
    scale = 1e12 if rf["bound"] == "mfma" else 1e9
    rf["achieved_wall"] = work / (rec["ms_per_step"] / 1e3) / scale
    rf["frac_wall"] = rf["achieved_wall"] / rf["peak"]
    rf["launch_ms_mean"] = rf["launch_ms"]["mean"]

    rec.update(extra)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
