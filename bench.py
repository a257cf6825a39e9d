"""Benchmark of the batched RGF hot path on one MI355X.

One step = the whole path over the workload: lead self-energies (Sancho-Rubio,
FP64) for every (k, E), forward + backward RGF sweeps for every (sample, k, E)
point in batches, and the density / current reductions.  Inputs are uploaded
before the timed region.  Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--workload C2] [--precision fp64|mixed]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6e12, "f32": 157.3e12}   # MI355X dense matrix-core peaks (FLOP/s)

WORKLOAD_DESC = {
    "C1": "single-orbital strip: block 8, 20 slabs, 256 E, 1 k",
    "C2": "sp3d5s*-sized cross-section: block 400 (40 atoms x 10 orbitals), 70 slabs, 512 E x 8 k, 10% Ge",
    "C3": "SCBA cross-section: block 240, 120 slabs, 1024 E x 4 k",
    "C4": "alloy ensemble: block 400, 128 samples x 256 E, 50-90 slabs",
    "C5": "paper-shaped slice: block 1200, 200 slabs, 16 E x 1 k",
}


def model_flops(wl, iters_L, iters_R):
    """Algorithmic flops of one step.  U = 8 b^3 (one complex b x b x b product
    or one complex inverse).  RGF for G^R + G^<: 8 U per slab per point (forward:
    inverse + g X g^dagger; backward: P = L G, G = g + P R, T = P Q, L G^< L^dagger).
    Sancho-Rubio: 7 U per decimation step per lead (1 inverse + 6 products)
    plus 3 U for the final surface inverse and tau g tau^dagger."""
    import numpy as np
    b = wl.nb
    U = 8.0 * b ** 3
    counts = np.diff(wl.slab_offset)
    rgf = 8.0 * U * float(np.sum(counts)) * wl.n_k * wl.n_e
    lead = U * (7.0 * (float(np.sum(iters_L)) + float(np.sum(iters_R))) + 3.0 * 2 * wl.n_k * wl.n_e)
    return rgf, lead


def cpu_baseline(wl, n_points, seed=0):
    """Time the oracle (as it stands) on a bounded sample of the same workload."""
    import numpy as np
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    rng = np.random.default_rng(seed)
    pts = wl.points()
    sel = pts[rng.choice(len(pts), size=min(n_points, len(pts)), replace=False)]
    t0 = time.perf_counter()
    O.solve_points(wl, [tuple(p) for p in sel])
    dt = time.perf_counter() - t0
    return {"value": len(sel) / dt, "unit": "(E,k) points/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sel)} random (sample,k,E) points of the same workload, leads included, "
                      f"{dt:.1f} s on the host"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="C2", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--capacity", type=int, default=None)
    ap.add_argument("--n-e", type=int, default=None, help="shrink the energy grid (not for reported runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-points", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the (E,k) points of a step "
              "shard over GPUs by energy blocks, which this build does not launch.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1510_04686_amd import negf as N
    from paper_1510_04686_amd.runtime import RGFSolver
    from synth import make_workload

    N.lib()   # fail loudly if the HIP library is missing
    kw = {}
    if args.n_e:
        kw["n_e"] = args.n_e
    wl = make_workload(args.workload, **kw)
    print(f"[bench] workload {args.workload}: nb={wl.nb} slabs={wl.total_slabs} n_k={wl.n_k} n_e={wl.n_e} "
          f"precision={args.precision}", file=sys.stderr, flush=True)
    solver = RGFSolver(wl, precision=args.precision, capacity=args.capacity)
    print(f"[bench] capacity={solver.capacity} points/batch, workspace "
          f"{N.negf_workspace_bytes(solver.ctx) / 2**30:.1f} GiB", file=sys.stderr, flush=True)
    out = solver.alloc_outputs(want=("GR", "GL", "GG", "bond"))
    stream = torch.cuda.current_stream()

    def step():
        solver.lead_selfenergies()
        solver.run_batches(out)
        return solver.observables(out["GL"], out["bond"])

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    N.negf_gemm_timing_enable(solver.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        n, J, jE = step()
        torch.cuda.synchronize()
        print(f"[bench] step {k + 1}/{args.steps} done at {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    dt = time.perf_counter() - t0
    launches, gemm_ms, gemm_flops = N.negf_gemm_timing(solver.ctx)
    st = solver.status()
    iters_L = solver.iters_L.cpu().numpy()
    iters_R = solver.iters_R.cpu().numpy()
    rgf_f, lead_f = model_flops(wl, iters_L, iters_R)
    points = solver.n_points * args.steps
    dtype = "f64" if args.precision == "fp64" else "f32+f64"
    peak = PEAK["f64"] if args.precision == "fp64" else PEAK["f32"]
    achieved = gemm_flops / (gemm_ms * 1e-3) if gemm_ms > 0 else None
    res = {
        "metric": "RGF (E,k) points/s",
        "value": points / dt,
        "unit": "(E,k) points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_DESC[args.workload]}",
                   "points_per_step": solver.n_points, "block": wl.nb, "slabs": int(wl.total_slabs),
                   "batch_capacity": solver.capacity, "precision": args.precision,
                   "parallelism": "single GPU, batched (sample,k,E) points"},
        "model_tflops": (rgf_f + lead_f) * args.steps / dt / 1e12,
        "model_flops_per_step": {"rgf": rgf_f, "leads": lead_f},
        "lead_iterations_mean": float((iters_L.mean() + iters_R.mean()) / 2),
        "roofline": {"bound": "mfma", "kernel": "batched complex GEMM (negf::gemm_kernel)",
                     "achieved": achieved / 1e12 if achieved else None, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": (achieved / peak) if achieved else None,
                     "traffic": None, "launches": launches,
                     "avg_launch_ms": gemm_ms / launches if launches else None},
        "status": N.STATUS.get(st, st),
    }
    if not args.no_cpu_baseline and args.cpu_points > 0:
        res["cpu_baseline"] = cpu_baseline(wl, args.cpu_points)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
