"""Benchmark of the batched RGF hot path on one MI355X.

Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--workload C2] [--precision fp64|mixed]

Workloads (default C2, the block-400 headline):
  C2  one step = one batch of bound points (512 points: the 512 energies of one
      k-point), or the two batches at k and -k, whose lead tables come from one
      decimation (the -k tables by transposition): their lead self-energies
      (Sancho-Rubio, FP64), forward + backward RGF sweeps, and the density /
      current reductions over the point set.  Steps cycle through the 5 groups
      of the 8 batches (k-points) of the 4096-point workload, so 5 steps make
      one full pass.
  C1  one step = the whole 256-point workload (one batch)
  C4  one step = leads + every batch of the alloy ensemble + reductions
  C3  one step = leads + the SCBA loop (iteration replayed from a HIP graph)
  C5  one step = leads + forward density; the adjoint dn/dV (VJP) is timed
      after the steps and reported as a cost ratio
Inputs are resident in HBM before the timed region starts.

    python bench.py --kernel-sweep 384,400,448 [--sweep-dtype f64|f32]

times the batched GEMM and block inverse alone at those block sizes (one JSON
line per size) instead of the step.
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
    "C3": "SCBA cross-section: block 240, 120 slabs, 1024 E x 4 k, acoustic + optical phonons",
    "C4": "alloy ensemble: block 400, 128 samples x 256 E, 50-90 slabs",
    "C5": "paper-shaped slice: block 1200, 200 slabs, 16 E x 1 k, smooth 0-0.3 eV potential",
}


def poisson_record(args, wl, solver):
    """Newton steps of the NEGF-Poisson loop (Eq. 9) on the workload's own
    device: silicon (eps_r 11.7) on a 0.2715 nm atom grid, insulating faces,
    contacts held at the mean starting potential of the first / last slab,
    donors N_D = n(V0) + 1e-3 per atom (a small excess, so the root lies near
    the starting potential).  Times every part of each step."""
    import numpy as np
    import torch
    from paper_1510_04686_amd.runtime import NewtonPoisson
    nz, ny = {"C5": (12, 10), "C2": (10, 4), "C3": (12, 2)}.get(args.workload, (1, wl.atoms_per_slab))
    opa = wl.orbs_per_atom
    v0 = (np.zeros((wl.total_slabs, wl.atoms_per_slab)) if wl.v_onsite is None
          else wl.v_onsite.reshape(wl.total_slabs, -1, opa)[:, :, 0])
    solver.set_potential(torch.from_numpy(np.repeat(v0, opa, axis=1)).cuda())
    n0 = solver.density().cpu().numpy()
    beta = 18.0951 / (11.7 * 0.2715)
    loop = NewtonPoisson(solver, nz, ny, beta, n0 + 1e-3, v_left=float(v0[0].mean()),
                         v_right=float(v0[-1].mean()), jacobian=args.poisson_jacobian, krylov_dim=20,
                         krylov_tol=1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    V, hist = loop.solve(v0, tol=1e-9, max_newton=args.poisson,
                         log=lambda m: print(f"[bench] poisson {m}", file=sys.stderr, flush=True))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = dict(loop.stats)
    return {"newton_steps": st["newton"], "krylov_iterations": st["krylov"], "cg_iterations": st["cg"],
            "jacobian": args.poisson_jacobian, "equilibrium": bool(wl.mu_L == wl.mu_R),
            "preconditioner": "local", "eta": wl.eta,
            "seconds": dt, "seconds_per_newton_step": dt / max(st["newton"], 1),
            "density_seconds": st["density_s"], "jacobian_seconds": st["jacobian_s"],
            "max_residual_history": hist, "atoms": int(wl.total_slabs * wl.atoms_per_slab),
            "max_potential_change_eV": float(np.max(np.abs(V.cpu().numpy() - v0)))}


GEMM_SOURCES = ["negf_gemm.hip", "negf_mfma.hpp", "negf_common.hpp", "negf_internal.hpp"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_traffic_C2.json")


def gemm_traffic_per_point_launch(precision):
    """Calibrated HBM bytes per point per GEMM launch from the committed
    rocprofv3 counter summary, or None when the GEMM sources changed since the
    counters were taken (or for another precision)."""
    import hashlib
    if precision != "fp64" or not os.path.exists(TRAFFIC_FILE):
        return None
    h = hashlib.sha1()
    for f in GEMM_SOURCES:
        with open(os.path.join(ROOT, "paper_1510_04686_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    if t.get("kernel_sources_sha1") != h.hexdigest():
        return None
    return float(t["hbm_bytes_per_point_launch"])


def cpu_baseline(wl, max_points=16, budget_s=15.0, seed=0):
    """Time the oracle (as it stands) on a bounded sample of the same workload:
    random points, each with its own lead decimations, until `budget_s` of host
    time or `max_points` points (at least two)."""
    import numpy as np
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    rng = np.random.default_rng(seed)
    pts = wl.points()
    sel = pts[rng.choice(len(pts), size=min(max_points, len(pts)), replace=False)]
    t0 = time.perf_counter()
    done = 0
    for p in sel:
        O.solve_points(wl, [tuple(p)])
        done += 1
        if done >= 2 and time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "(E,k) points/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} random (sample,k,E) points of the same workload, each with its own two lead "
                      f"decimations, {dt:.1f} s on the host"}


def inverse_record(N, solver, nb, reps=5):
    """The batched block inverse alone (the recursion's other dense kernel) on
    the step's context: its tuned shapes, its batch capacity, block nb; random
    complex blocks with nb on the diagonal; HIP events on the launch stream,
    median of `reps` launches.  Run after the timed region (it overwrites the
    workspace)."""
    import numpy as np
    import torch
    cap = solver.capacity
    g = torch.Generator(device="cuda").manual_seed(nb)
    A = torch.randn((cap, nb, nb), dtype=torch.complex128, device="cuda", generator=g)
    A += nb * torch.eye(nb, dtype=torch.complex128, device="cuda")
    W, C = torch.empty_like(A), torch.empty_like(A)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for r in range(reps + 1):
        W.copy_(A)
        e0.record(s)
        N.negf_zinv_batched(solver.ctx, W, C, stream=s)
        e1.record(s)
        torch.cuda.synchronize()
        if r:
            ms.append(e0.elapsed_time(e1))
    t = float(np.median(ms))
    tf = 8.0 * nb ** 3 * cap / (t * 1e-3) / 1e12
    del A, W, C
    torch.cuda.empty_cache()
    return {"kernel": "batched block inverse (negf::gj_panel + negf::gj_update)", "block": nb, "batch": cap,
            "ms": t, "achieved": tf, "peak": 78.6, "unit": "TFLOP/s", "frac": tf / 78.6,
            "flops": "8 b^3 per inverse (the Gauss-Jordan count, algorithmic)",
            "note": "standalone on the step's context and shapes, after the timed region"}


def kernel_sweep(sizes, dtype_name, reps=10):
    """Rates of the two dense kernels alone: the batched complex GEMM (C = A B,
    counted as 8 n^3 real flops per product) and the batched block inverse
    (counted as 8 n^3 per inverse, the Gauss-Jordan count), at each block size,
    with a batch that fills the chip; HIP events on the launch stream."""
    import torch
    from paper_1510_04686_amd import negf as N
    dt = torch.complex128 if dtype_name == "f64" else torch.complex64
    rows = []
    for n in sizes:
        batch = 512 if n <= 512 else (128 if n <= 800 else (64 if n <= 1200 else 32))
        ctx = N.negf_create(n, 1, batch, N.NEGF_FP64 if dtype_name == "f64" else N.NEGF_MIXED)
        g = torch.Generator(device="cuda").manual_seed(n)
        A = torch.randn((batch, n, n), dtype=dt, device="cuda", generator=g)
        B = torch.randn((batch, n, n), dtype=dt, device="cuda", generator=g)
        C = torch.empty_like(A)
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        rec = {"n": n, "batch": batch, "dtype": dtype_name}
        for name, call in (("gemm", lambda: N.negf_zgemm_batched(ctx, A, B, C, stream=s)),
                           ("inverse", lambda: N.negf_zinv_batched(ctx, A.clone(), C, stream=s))):
            call()
            torch.cuda.synchronize()
            ms = 0.0
            for _ in range(reps):
                if name == "inverse":
                    W = A.clone()
                    e0.record(s)
                    N.negf_zinv_batched(ctx, W, C, stream=s)
                    e1.record(s)
                else:
                    e0.record(s)
                    call()
                    e1.record(s)
                torch.cuda.synchronize()
                ms += e0.elapsed_time(e1)
            ms /= reps
            rec[name + "_ms"] = ms
            rec[name + "_tflops"] = 8.0 * n ** 3 * batch / ms / 1e9
        print(json.dumps(rec), flush=True)
        rows.append(rec)
        del A, B, C, ctx
        torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="C2", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--capacity", type=int, default=None)
    ap.add_argument("--n-e", type=int, default=None, help="shrink the energy grid (not for reported runs)")
    ap.add_argument("--samples", type=int, default=None, help="C4: number of alloy samples (default 128)")
    ap.add_argument("--scba-iters", type=int, default=None, help="C3: SCBA iterations (default 20)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--point-redo", type=float, default=float("inf"),
                    help="mixed precision: redo points whose block-refinement residual exceeds this in FP64 (inf: off)")
    ap.add_argument("--redo-frac", type=float, default=0.05,
                    help="mixed precision: also redo this share of the points with the highest redo score "
                         "(residual x largest weighted |Im G^<_jj|) in FP64")
    ap.add_argument("--atom-blocks", action="store_true",
                    help="C3: local scattering self-energies from the atom blocks of G (else orbital diagonals)")
    ap.add_argument("--cap-slabs", type=int, default=0,
                    help="C2/C4: absorbing-potential contacts of this many disordered slabs per side "
                         "instead of Sancho-Rubio leads")
    ap.add_argument("--poisson", type=int, default=0, metavar="K",
                    help="C5 (or any single-sample workload): after the timed steps, at most K Newton steps of "
                         "the NEGF-Poisson loop (Eq. 9) from the workload's potential, reported in a 'poisson' record")
    ap.add_argument("--poisson-jacobian", default="adjoint", choices=["adjoint", "fd"])
    ap.add_argument("--equilibrium", action="store_true",
                    help="set mu_R = mu_L and fill the device's eta sink at that level (one Fermi level)")
    ap.add_argument("--n-k", type=int, default=None, help="shrink the k grid (not for reported runs)")
    ap.add_argument("--eta", type=float, default=None, help="override the broadening eta (eV)")
    ap.add_argument("--lanes", type=int, default=1,
                    help="batches in flight at once, each on its own context and stream")
    ap.add_argument("--store", default="full", choices=["full", "checkpoint"],
                    help="g / g^< of every slab (full) or only at segment ends, recomputed per segment")
    ap.add_argument("--tune", default="auto", choices=["auto", "default"],
                    help="kernel shapes: measured on this GPU before timing (auto) or the library defaults")
    ap.add_argument("--cpu-points", type=int, default=16, help="oracle points at most (about 15 s of host time)")
    ap.add_argument("--kernel-sweep", default="", metavar="N1,N2,...",
                    help="instead of the step: time the batched GEMM and block inverse alone at these block sizes")
    ap.add_argument("--sweep-dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the multi-GPU form, which would "
              "shard the (E,k) points of a step over GPUs by energy blocks, is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1510_04686_amd import negf as N
    from paper_1510_04686_amd.runtime import RGFSolver
    from synth import make_workload

    N.lib()   # fail loudly if the HIP library is missing
    if args.kernel_sweep:
        kernel_sweep([int(x) for x in args.kernel_sweep.split(",")], args.sweep_dtype)
        return
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {nbytes} bytes read, {nbytes} bytes written", file=sys.stderr, flush=True)
        del src, dst
    kw = {}
    if args.n_e:
        kw["n_e"] = args.n_e
    if args.n_k:
        kw["n_k"] = args.n_k
    if args.workload == "C4" and args.samples:
        kw["n_samples"] = args.samples
    if args.cap_slabs:
        if args.workload not in ("C2", "C4"):
            sys.exit("--cap-slabs applies to C2 and C4")
        kw["cap_slabs"] = args.cap_slabs
    wl = make_workload(args.workload, **kw)
    if args.equilibrium or args.eta is not None:
        import dataclasses
        if args.equilibrium:
            wl = dataclasses.replace(wl, mu_R=wl.mu_L)
        if args.eta is not None:
            wl = dataclasses.replace(wl, eta=args.eta)
    print(f"[bench] workload {args.workload}: nb={wl.nb} samples={wl.n_samples} slabs={wl.total_slabs} "
          f"n_k={wl.n_k} n_e={wl.n_e} precision={args.precision}", file=sys.stderr, flush=True)
    adj_seg = -1 if (args.workload == "C5" or (args.poisson and args.poisson_jacobian == "adjoint")) else 0
    solver = RGFSolver(wl, precision=args.precision, capacity=args.capacity, adjoint_segment=adj_seg,
                       tune="auto" if args.tune == "auto" else None, lanes=args.lanes, point_redo=args.point_redo,
                       store=args.store, redo_frac=args.redo_frac or None)
    if args.equilibrium:
        solver.set_eta_fill(True)
    print(f"[bench] capacity={solver.capacity} points/batch, workspace "
          f"{sum(N.negf_workspace_bytes(c) for c in solver.ctxs) / 2**30:.1f} GiB", file=sys.stderr, flush=True)
    n_iter = (args.scba_iters or wl.n_scba) if args.workload == "C3" else 1
    out = solver.alloc_outputs(want=("GR", "GL", "GG", "bond"))
    batches = solver.batches()
    # C2: one step is one batch (the 512 energies of one k-point); the others run
    # the whole workload per step
    per_batch = args.workload == "C2" and args.precision == "fp64" and args.lanes == 1
    lead_steps = []        # (ik, e0, e1) lead ranges decimated in each timed step
    # C2 steps: a batch, or a batch together with its mirror batch (the one at -k),
    # whose lead tables are the transposes of the first's (RGFSolver.mirror)
    groups, used = [], set()
    for b in range(len(batches)):
        if b in used:
            continue
        g = [b]
        used.add(b)
        ks = {ik for ik, _, _ in solver.lead_ranges(*batches[b])}
        for b2 in range(b + 1, len(batches)):
            ks2 = {ik for ik, _, _ in solver.lead_ranges(*batches[b2])}
            if b2 not in used and any(solver.mirror.get(k2) in ks for k2 in ks2):
                g.append(b2)
                used.add(b2)
                break
        groups.append(g)

    def step(j):
        if per_batch:
            grp = groups[j % len(groups)]
            ranges = [r for b in grp for r in solver.lead_ranges(*batches[b])]
            dec = solver.lead_selfenergies_for_ranges(ranges)
            for b in grp:
                solver.run_batch(out, *batches[b])
            n, J, jE = solver.observables(out["GL"], out["bond"])
            return n, J, jE, sum(batches[b][1] for b in grp), dec
        solver.lead_selfenergies()
        ranges = list(solver.last_lead_ranges)
        if args.workload == "C3":
            o, hist = solver.scba(n_iter=n_iter, graph=True, atom_blocks=args.atom_blocks,
                                  progress=lambda i, n: print(f"[bench]   SCBA iteration {i}/{n} done",
                                                              file=sys.stderr, flush=True))
            return (*solver.observables(o["GL"], o["bond"]), solver.n_points, ranges)
        if args.workload == "C5":
            return solver.density(), None, None, solver.n_points, ranges
        solver.run_batches(out)
        return (*solver.observables(out["GL"], out["bond"]), solver.n_points, ranges)

    for w in range(args.warmup):
        step(w)
        torch.cuda.synchronize()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    # event records cannot sit inside the captured SCBA graph; a mixed run times the
    # FP32 matrix-core launches (its block algebra) against the FP32 peak, leaving
    # out its FP64 lead-decimation and residual products
    timed_gemm = args.workload != "C3"
    for c in solver.ctxs:
        N.negf_gemm_timing_enable(c, ("fp64" if args.precision == "fp64" else "fp32") if timed_gemm else False)
    torch.cuda.synchronize()
    points = 0
    rgf_f = lead_f = 0.0
    lead_iters = []
    counts = np.diff(wl.slab_offset)
    U = 8.0 * wl.nb ** 3
    t0 = time.perf_counter()
    for k in range(args.steps):
        n, J, jE, npts, ranges = step(args.warmup + k)
        torch.cuda.synchronize()
        points += npts
        lead_steps.append(ranges)
        print(f"[bench] step {k + 1}/{args.steps} done at {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    dt = time.perf_counter() - t0
    points *= n_iter
    launches, gemm_ms, gemm_flops, gemm_mfma = 0, 0.0, 0.0, 0.0
    for c in solver.ctxs:
        l_, m_, f_, x_ = N.negf_gemm_timing(c, executed=True)
        launches, gemm_ms, gemm_flops, gemm_mfma = launches + l_, gemm_ms + m_, gemm_flops + f_, gemm_mfma + x_
        N.negf_gemm_timing_enable(c, False)
    st = solver.status()
    iters_L = solver.iters_L.cpu().numpy()
    iters_R = solver.iters_R.cpu().numpy()
    # model flops of the timed steps (U = 8 b^3): 7 U per slab per point solved,
    # and per lead point 7 U per decimation step (max of the two leads with the
    # shared decimation) plus 3 U per lead for the surface inverse and tau g tau^dagger
    for k, ranges in enumerate(lead_steps):
        if per_batch:
            grp = groups[(args.warmup + k) % len(groups)]
            slabs = float(sum(np.sum(counts[solver.points[p0:p0 + np_, 0]])
                              for p0, np_ in (batches[b] for b in grp)))
        else:
            slabs = float(np.sum(counts)) * wl.n_k * wl.n_e
        rgf_f += 7.0 * U * slabs * n_iter
        for ik, e0, e1 in ranges:
            iL, iR = iters_L[ik, e0:e1], iters_R[ik, e0:e1]
            steps_ = float(np.sum(np.maximum(iL, iR))) if solver.lead_dual else float(np.sum(iL) + np.sum(iR))
            lead_f += U * (7.0 * steps_ + 3.0 * 2 * (e1 - e0))
            lead_iters.append((iL + iR) / 2.0)
    lead_iters = np.concatenate(lead_iters) if lead_iters else np.zeros(1)
    dtype = "f64" if args.precision == "fp64" else "f32+f64"
    peak = PEAK["f64"] if args.precision == "fp64" else PEAK["f32"]
    achieved = gemm_flops / (gemm_ms * 1e-3) if gemm_ms > 0 else None
    point_launches = gemm_flops / (8.0 * wl.nb ** 3)
    tpp = gemm_traffic_per_point_launch(args.precision) if wl.nb == 400 else None
    traffic = tpp * point_launches / launches if (tpp and launches) else None
    metric ="RGF (E,k) points/s" if args.workload != "C3" else "RGF (E,k) points x SCBA iterations/s"
    res = {
        "metric": metric,
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
                   "points_per_step": points // max(args.steps * n_iter, 1),
                   "step": ("one batch of bound points (one k-point's 512 energies), or two batches at k "
                            "and -k: their leads (decimated once for a mirror pair, the -k tables by "
                            "transposition), forward + backward sweeps, and the reductions over the point "
                            f"set; steps cycle over the {len(groups)} groups of the {len(batches)} batches"
                            if per_batch else "the whole workload"),
                   "lead_mirrors": {str(k): v for k, v in solver.mirror.items()},
                   "points_per_pass": solver.n_points, "block": wl.nb, "slabs": int(wl.total_slabs),
                   "samples": wl.n_samples, "n_e": wl.n_e, "n_k": wl.n_k,
                   "batch_capacity": solver.capacity, "lanes": solver.lanes, "precision": args.precision,
                   "store": args.store,
                   "contacts": (f"absorbing potential, {args.cap_slabs} disordered slabs per side"
                                if args.cap_slabs else "Sancho-Rubio leads"),
                   "parallelism": "single GPU, batched (sample,k,E) points"},
        "model_tflops": (rgf_f + lead_f) / dt / 1e12,
        "model_flops_per_step": {"rgf": rgf_f / args.steps, "leads": lead_f / args.steps},
        "lead_iterations_mean": float(np.mean(lead_iters)),
        "lead_shared_decimation": bool(solver.lead_dual),
        "kernel_shapes": solver.tuning,
        "roofline": {"bound": "mfma", "kernel": "batched complex GEMM (negf::gemm_kernel)" +
                     ("" if args.precision == "fp64" else ", FP32 matrix-core launches"),
                     "achieved": achieved / 1e12 if achieved else None, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": (achieved / peak) if achieved else None,
                     "traffic": traffic, "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, "
                                                         "copy-calibrated)",
                     "algorithmic_bytes_per_launch": 3 * 16 * wl.nb ** 2 * point_launches / launches if launches else None,
                     "launches": launches, "points_per_launch": point_launches / launches if launches else None,
                     "avg_launch_ms": gemm_ms / launches if launches else None,
                     # achieved counts 8 b^3 real flops per complex product (the algorithmic
                     # count); complex products run as three real MFMA products (3M), except
                     # the anti-Hermitian (lesser) products, which run as four
                     "mfma_flops_per_algorithmic_flop": gemm_mfma / gemm_flops if gemm_flops else None,
                     "executed_mfma_frac": (gemm_mfma / (gemm_ms * 1e-3)) / peak if gemm_ms > 0 else None},
        "status": N.STATUS.get(st, st),
    }
    if args.workload == "C3":
        res["config"]["scba_iterations"] = n_iter
        res["config"]["sigma_scat"] = "atom blocks" if args.atom_blocks else "orbital diagonal"
        res["roofline"]["note"] = "GEMM events are not recorded inside the captured SCBA graph"
    if args.precision == "mixed":
        stats = [N.negf_mixed_stats(c) for c in solver.ctxs]
        nfb, maxres = sum(x[0] for x in stats), max(x[1] for x in stats)
        res["mixed"] = {"fp64_fallback_inverses": nfb, "max_block_refinement_residual": maxres,
                        "point_redo_bound": solver.point_redo, "redo_frac": solver.redo_frac,
                        "points_redone_per_step": solver.points_redone}
    if args.workload == "C5":
        # adjoint dn/dV: one VJP with a seeded cotangent over all atoms, against
        # the forward RGF it differentiates (density from the stored lead
        # self-energies: forward and backward sweeps and the reduction, no
        # lead decimation), timed just before it
        wv = torch.from_numpy(np.random.default_rng(1510046865).normal(
            size=(wl.total_slabs, wl.atoms_per_slab))).cuda()
        torch.cuda.synchronize()
        tf = time.perf_counter()
        solver.density()
        torch.cuda.synchronize()
        t_rgf = time.perf_counter() - tf
        ta = time.perf_counter()
        g = solver.density_vjp(wv)
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - ta
        t_fwd = dt / args.steps
        ws = N.negf_workspace_bytes(solver.ctx)
        res["adjoint"] = {"ms": t_adj * 1e3, "forward_rgf_ms": t_rgf * 1e3, "cost_ratio": t_adj / t_rgf,
                          "forward_step_ms": t_fwd * 1e3, "cost_ratio_vs_step_with_leads": t_adj / t_fwd,
                          "store": args.store, "checkpoint_segment": int(np.ceil(np.sqrt(wl.total_slabs))),
                          "workspace_bytes_per_point": ws / solver.capacity,
                          "grad_norm": float(torch.linalg.norm(g))}
    if args.precision == "fp64" and wl.nb >= 64:
        res["inverse"] = inverse_record(N, solver, wl.nb)
    if args.workload in ("C2", "C4") and args.precision == "mixed":
        # per-sample density and current error of the mixed path against the FP64
        # GPU path (outside the timed region)
        n_mix, J_mix = n.cpu().numpy(), J.cpu().numpy()
        del solver
        torch.cuda.empty_cache()
        ref = RGFSolver(wl, precision="fp64", capacity=args.capacity,
                        tune="auto" if args.tune == "auto" else None)
        o64 = ref.alloc_outputs(want=("GR", "GL", "GG", "bond"))
        ref.lead_selfenergies()          # warm: leads and the autotuned shapes
        torch.cuda.synchronize()
        t64 = time.perf_counter()
        ref.lead_selfenergies()
        ref.run_batches(o64)
        n64, J64, _ = ref.observables(o64["GL"], o64["bond"])
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t64
        n64, J64 = n64.cpu().numpy(), J64.cpu().numpy()
        errs, jerrs = [], []
        for s_ in range(wl.n_samples):
            a0, a1 = int(wl.slab_offset[s_]), int(wl.slab_offset[s_ + 1])
            errs.append(float(np.max(np.abs(n_mix[a0:a1] - n64[a0:a1])) / np.max(np.abs(n64[a0:a1]))))
            jerrs.append(float(np.max(np.abs(J_mix[a0:a1] - J64[a0:a1])) / np.max(np.abs(J64[a0:a1]))))
        ref_note = "FP64 GPU path (oracle-checked)"
        res["mixed"]["per_sample_density_rel_err"] = {"max": max(errs), "median": float(np.median(errs)),
                                                     "reference": ref_note}
        res["mixed"]["per_sample_current_rel_err"] = {"max": max(jerrs), "median": float(np.median(jerrs)),
                                                     "reference": ref_note}
        # the same step in FP64 (leads, every batch, observables), timed once
        res["mixed"]["fp64_ms_same_step"] = t64 * 1e3
        res["mixed"]["speedup_vs_fp64"] = t64 / (dt / args.steps)
        res["mixed"]["target_rel_err"] = 1e-4
        res["mixed"]["target_met"] = bool(max(errs) <= 1e-4 and max(jerrs) <= 1e-4)
    if args.poisson > 0:
        res["poisson"] = poisson_record(args, wl, solver)
    if not args.no_cpu_baseline and args.cpu_points > 0:
        res["cpu_baseline"] = cpu_baseline(wl, args.cpu_points)
        res["gpu_over_cpu"] = res["value"] / res["cpu_baseline"]["value"]
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
