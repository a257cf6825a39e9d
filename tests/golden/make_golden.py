"""Write the oracle references of the GPU parity tests whose oracle runs take
minutes (block 1200, or a chain of SCBA solves at block 240).

    python tests/golden/make_golden.py [slice|full|scba|c4|all]

Calls only the oracle (and the seeded input generators): no value here comes
from the GPU path.  Each file is stamped with a SHA-1 of the generated
inputs so a test can tell when the generator has changed since:

* c5_slice.npz -- the paper-shaped cross-section (120 atoms x 10 orbitals,
  block 1200, smooth 0-0.3 eV potential) cut to 3 slabs, at two of its 16
  energies: orbital diagonals of G^R, G^<, G^>, bond currents and Caroli T,
  with the per-quantity FP64 drift that sets each tolerance (tests/parity.py).
* c5_full.npz -- the same device at its full 200 slabs (rank 240,000), one
  energy: the electron density per atom (Eq. 7) of that point, the orbital
  diagonals of G^R and G^< on a few slabs, and their drifts.

* c3_scba.npz -- the SCBA cross-section (block 240, 120 slabs, 2 k x 48 E on
  the 5 meV grid, acoustic and optical phonons): the second solve of the
  self-consistent Born loop (Eqs. 1-6) at one point, i.e. the ballistic pass at
  the points its scattering self-energy reads (all k at E and E -+ hw), the
  self-energy update, and the solve with it; orbital diagonals of G^R and G^<
  and their drifts.

* c4_density.npz -- two alloy samples of the random-alloy ensemble (block 400,
  their own slab counts, all 256 energies): the electron density per atom
  (Eq. 7) and the bond current per slab (Eq. 8) of each sample, with their
  drift over the variants of tests/parity.py, and per point the drift and
  largest magnitude of its G^< diagonals.  The reference of the
  mixed-precision accuracy figures.

The full case takes tens of minutes and ~20 GB of host memory; the C4 case
about an hour on 8 cores.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.dirname(HERE)):
    if p not in sys.path:
        sys.path.insert(0, p)

import oracle as O              # noqa: E402
import parity as P              # noqa: E402
from synth import make_workload  # noqa: E402

SLICE_PTS = [(0, 0, 4), (0, 0, 11)]
FULL_SLABS = (0, 1, 57, 100, 198, 199)


def inputs_sha1(wl):
    h = hashlib.sha1()
    for a in (wl.h_diag, wl.h_up, wl.lead_h00, wl.lead_h01_L, wl.lead_tau_L, wl.lead_h01_R, wl.lead_tau_R,
              wl.v_onsite, wl.energy):
        if a is not None:
            h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def slice_case():
    wl = make_workload("C5", n_slab=3)
    t0 = time.time()
    ref, tols = P.reference(wl, SLICE_PTS, transmission=True)
    d = lambda x: np.diagonal(x, axis1=1, axis2=2)
    out = {"inputs_sha1": inputs_sha1(wl), "points": np.array(SLICE_PTS)}
    for i, (r, t) in enumerate(zip(ref, tols)):
        for k in ("GR", "GL", "GG"):
            out[f"p{i}_{k}"] = d(r[k])
        out[f"p{i}_bond"] = r["bond"]
        out[f"p{i}_T"] = np.array(r["T"])
        out[f"p{i}_bond_scale"] = np.array(P._bond_scale(r))
        for k, v in t["drift"].items():
            out[f"p{i}_drift_{k}"] = np.array(v)
    np.savez_compressed(os.path.join(HERE, "c5_slice.npz"), **out)
    print(f"c5_slice.npz written ({time.time() - t0:.0f} s)", file=sys.stderr)


def full_case():
    """One energy of the full device; the density of that point and sampled
    slab diagonals, with the drift over the same variants as tests/parity.py
    (one at a time: the oracle holds every block of the 200-slab chain)."""
    wl = make_workload("C5", n_e=1)
    pts = [(0, 0, 0)]
    t0 = time.time()
    variants = [("ref", wl, None, None), ("alt", wl, "alt", None)] + [
        (f"perturb{s}", P._perturbed(wl, s), None, s) for s in range(P.N_PERTURB)]
    res = {}
    for name, w, var, seed in variants:
        leads = None if seed is None else P.perturbed_leads(wl, pts, seed, w)
        r = O.solve_points(w, pts, variant=var, leads=leads, diag_only=True)[0]
        GLd, GRd = r["GL"], r["GR"]
        n, _, _ = O.observables(wl, pts, [GLd], [r["bond"]])
        res[name] = {"n": n, "GR": GRd[list(FULL_SLABS)].copy(), "GL": GLd[list(FULL_SLABS)].copy()}
        del r, GLd, GRd
        print(f"  {name} done ({time.time() - t0:.0f} s)", file=sys.stderr, flush=True)
    ref = res.pop("ref")
    out = {"inputs_sha1": inputs_sha1(wl), "slabs": np.array(FULL_SLABS), "n": ref["n"],
           "GR": ref["GR"], "GL": ref["GL"]}
    for k in ("n", "GR", "GL"):
        out[f"drift_{k}"] = np.array(max(P.rel(v[k], ref[k]) for v in res.values()))
    np.savez_compressed(os.path.join(HERE, "c5_full.npz"), **out)
    print(f"c5_full.npz written ({time.time() - t0:.0f} s)", file=sys.stderr)


SCBA_PT = (0, 1, 20)


def scba_second_solve(wl, pt, variant=None, seed=None):
    """The point's solve in the second iteration of the Born loop: Sigma_scat
    starts at zero, the first (ballistic) pass gives the orbital diagonals at
    every k and at the energies Eqs. (4)-(6) read for this point's energy
    (E, E - hw, E + hw), the update builds Sigma_scat(E), and the point is
    solved with it."""
    _, ik, ie = pt
    es = [e for e in (ie - wl.shift, ie, ie + wl.shift) if 0 <= e < wl.n_e]
    first = [(0, k, e) for k in range(wl.n_k) for e in es]
    # perturbed variants: the lead self-energies perturbed norm-wise as in tests/parity.py
    leads = None if seed is None else P.perturbed_leads(wl, first, seed)
    res = O.solve_points(wl, first, variant=variant, leads=leads)
    N, b = wl.total_slabs, wl.nb
    GRd = np.zeros((wl.n_k, wl.n_e, N, b), dtype=np.complex128)
    GLd = np.zeros_like(GRd)
    for (_, k, e), r in zip(first, res):
        GRd[k, e] = np.diagonal(r["GR"], axis1=1, axis2=2)
        GLd[k, e] = np.diagonal(r["GL"], axis1=1, axis2=2)
    sigR, sigL = O.scba_selfenergy(GRd, GLd, wl.w_k, wl.D_ac, wl.M_op, wl.shift, wl.n_bose)
    scR = np.zeros_like(sigR)
    scL = np.zeros_like(sigL)
    scR[ie], scL[ie] = sigR[ie], sigL[ie]
    return O.solve_points(wl, [pt], scatR=scR, scatL=scL, variant=variant, leads=leads)[0]


def scba_case():
    wl = make_workload("C3", n_e=48, n_k=2)
    t0 = time.time()
    d = lambda x: np.diagonal(x, axis1=1, axis2=2)
    ref = scba_second_solve(wl, SCBA_PT)
    runs = [scba_second_solve(wl, SCBA_PT, "alt")] + [
        scba_second_solve(P._perturbed(wl, s), SCBA_PT, seed=s) for s in range(P.N_PERTURB)]
    out = {"inputs_sha1": inputs_sha1(wl), "point": np.array(SCBA_PT), "GR": d(ref["GR"]), "GL": d(ref["GL"])}
    for k in ("GR", "GL"):
        out[f"drift_{k}"] = np.array(max(P.rel(d(x[k]), d(ref[k])) for x in runs))
    np.savez_compressed(os.path.join(HERE, "c3_scba.npz"), **out)
    print(f"c3_scba.npz written ({time.time() - t0:.0f} s)", file=sys.stderr)


C4_SAMPLES = (0, 1)


def _c4_chunk(args):
    samples, pts, variant, seed = args
    os.environ.setdefault("OMP_NUM_THREADS", "2")
    wl = make_workload("C4", samples=list(samples))
    leads = None
    if seed is not None:          # inputs and lead self-energies perturbed as in tests/parity.py
        w = P._perturbed(wl, seed)
        leads = P.perturbed_leads(wl, pts, seed, w)
        wl = w
    res = O.solve_points(wl, pts, variant=variant, leads=leads, diag_only=True)
    return [r["GL"] for r in res], [r["bond"] for r in res]


def c4_case(workers=4):
    """Per-sample density and current of two alloy samples, and their drift over
    the same variants as tests/parity.py (the alternative association and
    N_PERTURB perturbed inputs), each variant's points spread over a process
    pool in 16 fixed chunks."""
    from concurrent.futures import ProcessPoolExecutor
    wl = make_workload("C4", samples=list(C4_SAMPLES))
    pts = [(s, 0, e) for s in range(wl.n_samples) for e in range(wl.n_e)]
    t0 = time.time()
    out = {"inputs_sha1": inputs_sha1(wl), "samples": np.array(C4_SAMPLES),
           "slab_offset": wl.slab_offset.copy()}
    chunks = [pts[i::16] for i in range(16)]
    variants = [("ref", None, None), ("alt", "alt", None)] + [(f"perturb{k}", None, k) for k in range(P.N_PERTURB)]
    res = {}
    ref_gl = None
    pdrift = np.zeros(len(pts))
    with ProcessPoolExecutor(workers) as ex:
        for name, variant, seed in variants:
            GL, bond = [None] * len(pts), [None] * len(pts)
            jobs = [(C4_SAMPLES, c, variant, None if seed is None else seed * 100 + ci) for ci, c in enumerate(chunks)]
            for ci, (gl, bd) in enumerate(ex.map(_c4_chunk, jobs)):
                for j, (g, b) in enumerate(zip(gl, bd)):
                    GL[ci + 16 * j], bond[ci + 16 * j] = g, b
            n, J, _ = O.observables(wl, pts, GL, bond)
            res[name] = (n, J)
            if ref_gl is None:
                ref_gl = GL
            else:                # per-point drift of the G^< diagonals
                pdrift = np.maximum(pdrift, [P.rel(a, b) for a, b in zip(GL, ref_gl)])
            print(f"  c4 {name} done ({time.time() - t0:.0f} s)", file=sys.stderr, flush=True)
    n, J = res.pop("ref")
    out["n"], out["J"] = n, J
    out["drift_n"] = np.array(max(P.rel(v[0], n) for v in res.values()))
    out["drift_J"] = np.array(max(P.rel(v[1], J) for v in res.values()))
    # per point: the drift of its G^< diagonals and their largest magnitude, so that
    # a test can bound the density by the per-point tolerances, weighted as Eq. 7 sums them
    out["points"] = np.array(pts)
    out["point_drift_GL"] = pdrift
    out["point_max_GL"] = np.array([float(np.max(np.abs(g))) for g in ref_gl])
    np.savez_compressed(os.path.join(HERE, "c4_density.npz"), **out)
    print(f"c4_density.npz written ({time.time() - t0:.0f} s)", file=sys.stderr)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("slice", "all"):
        slice_case()
    if what in ("full", "all"):
        full_case()
    if what in ("scba", "all"):
        scba_case()
    if what in ("c4", "all"):
        c4_case()
