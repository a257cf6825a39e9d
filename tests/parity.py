"""FP64 parity tolerances for the GPU tests, set from the oracle alone.

A point's tolerance is 1e-10 relative, or FACTOR times the point's measured
FP64 drift where that is larger.  The drift is how far correct FP64
evaluations of the same point land from each other: the oracle is re-run

  * once with every triple product and the lead decimation associated the
    other way (``variant="alt"``), and
  * N_PERTURB times on inputs whose every entry carries an independent relative
    perturbation of one unit roundoff (Hermitian blocks stay Hermitian), with
    the lead self-energies -- inputs of the recursion, computed by an
    inversion-based iteration whose FP64 errors are norm-wise, not entry-wise --
    then perturbed norm-wise, every entry by up to one unit roundoff of the
    largest entry (this reaches their small anti-Hermitian part, the source
    of G^< at energies where the leads carry almost no states),

and the drift of a quantity is the largest distance of those runs from the
plain oracle.  A backward-stable FP64 solve returns the exact result of inputs
perturbed at that level, so its distance from the oracle is of the size of this
drift, however ill-conditioned the point (eta = 1e-6 resonances); no GPU value
enters the estimate.

Every comparison can be logged: with NEGF_PARITY_LOG set to a file path, each
check appends one JSON line (test, point, quantity, error, drift, tolerance).
"""
from __future__ import annotations

import dataclasses
import json
import os

import numpy as np

import oracle as O

TOL = 1e-10          # relative FP64 parity bound
FACTOR = 10.0        # x the measured drift, for points that cannot meet TOL in FP64
N_PERTURB = 3
U64 = 2.0 ** -53     # unit roundoff of FP64


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def _perturbed(wl, seed):
    """The workload with every Hamiltonian, coupling and potential entry
    multiplied by (1 + d), |d| <= one unit roundoff, independently for real and
    imaginary parts; Hermitian blocks get a Hermitian perturbation."""
    rng = np.random.default_rng([seed, 9173])

    def gen(h):
        h = np.asarray(h)
        if np.iscomplexobj(h):
            return (h.real * (1 + rng.uniform(-U64, U64, h.shape))
                    + 1j * h.imag * (1 + rng.uniform(-U64, U64, h.shape)))
        return h * (1 + rng.uniform(-U64, U64, h.shape))

    def herm(h):
        p = gen(h) - h
        return h + (p + np.conj(np.swapaxes(p, -1, -2))) / 2

    return dataclasses.replace(
        wl, h_diag=herm(wl.h_diag), h_up=gen(wl.h_up), lead_h00=herm(wl.lead_h00),
        lead_h01_L=gen(wl.lead_h01_L), lead_h01_R=gen(wl.lead_h01_R),
        lead_tau_L=gen(wl.lead_tau_L), lead_tau_R=gen(wl.lead_tau_R),
        v_onsite=None if wl.v_onsite is None else gen(wl.v_onsite))


def perturbed_leads(wl, pts, seed, variant_wl=None):
    """Lead self-energy table for the points, computed from the (perturbed)
    workload ``variant_wl`` and then perturbed norm-wise at one unit roundoff."""
    w = wl if variant_wl is None else variant_wl
    rng = np.random.default_rng([seed, 5531])
    tab = O.lead_tables(w, ks=sorted({int(p[1]) for p in pts}), es=sorted({int(p[2]) for p in pts}))

    def noisy(S):
        m = float(np.max(np.abs(S)))
        return S + U64 * m * (rng.uniform(-1, 1, S.shape) + 1j * rng.uniform(-1, 1, S.shape))

    return {k: (noisy(v[0]), noisy(v[1]), v[2], v[3]) for k, v in tab.items()}


def _bond_scale(r):
    """Bond currents are traces that add terms of both signs (the net of in-
    and out-flow); they are compared norm-wise on the largest sum of term
    magnitudes of the point's bonds (the oracle's ``bond_mag``), the scale on
    which every FP64 evaluation of the trace rounds, in any order."""
    return max(float(np.max(r["bond_mag"])) if r["bond"].size else 0.0, 1e-300)


def _view(x, full):
    return x if full else np.diagonal(x, axis1=-2, axis2=-1)


def point_drift(ref, runs, full=False):
    """Per quantity, the largest distance of the variant runs from the plain
    oracle run of one point, in the norm the comparison uses (diagonal blocks
    when ``full``, else orbital diagonals)."""
    d = {}
    for k in ("GR", "GL", "GG"):
        d[k] = max(rel(_view(x[k], full), _view(ref[k], full)) for x in runs)
    if ref["bond"].size:
        sc = _bond_scale(ref)
        d["bond"] = max(float(np.max(np.abs(x["bond"] - ref["bond"]))) / sc for x in runs)
    if "T" in ref:
        d["T"] = max(abs(x["T"] - ref["T"]) / max(1.0, abs(ref["T"])) for x in runs)
    return d


def _gg_propagated(r, t, full=False):
    """G^> = G^< + G^R - G^R^dagger: the bound its parts' tolerances put on it,
    relative to max |G^>|."""
    m = lambda x: float(np.max(np.abs(_view(x, full))))
    return (t["GL"] * m(r["GL"]) + 2 * t["GR"] * m(r["GR"])) / max(m(r["GG"]), 1e-300)


def reference(wl, pts, full=False, **kw):
    """Oracle results of the points and, per point, a dict of tolerances (one
    per quantity) plus the drifts they come from, for comparisons of orbital
    diagonals (or of diagonal blocks when ``full``).  G^> also admits what the
    tolerances of G^< and G^R it is formed from allow."""
    ref = O.solve_points(wl, pts, bond_mag=True, **kw)
    runs = [O.solve_points(wl, pts, variant="alt", **kw)]
    for s in range(N_PERTURB):
        w = _perturbed(wl, s)
        runs.append(O.solve_points(w, pts, leads=perturbed_leads(wl, pts, s, w), **kw))
    tols = []
    for i, r in enumerate(ref):
        d = point_drift(r, [x[i] for x in runs], full)
        t = {"drift": d, **{k: max(TOL, FACTOR * v) for k, v in d.items()}}
        t["GG"] = max(t["GG"], _gg_propagated(r, t, full))
        tols.append(t)
    return ref, tols


def lead_reference(h00, h01, tau, z):
    """Oracle lead self-energy and its tolerance (same drift rule)."""
    r, it, _ = O.lead_selfenergy(h00, h01, tau, z)
    runs = [O.lead_selfenergy(h00, h01, tau, z, variant="alt")[0]]
    rng = np.random.default_rng(int(abs(z.real) * 1e6) % 2 ** 31)
    for _ in range(N_PERTURB):
        def gen(h):
            return (h.real * (1 + rng.uniform(-U64, U64, h.shape))
                    + 1j * h.imag * (1 + rng.uniform(-U64, U64, h.shape)))
        p = gen(h00) - h00
        runs.append(O.lead_selfenergy(h00 + (p + p.conj().T) / 2, gen(h01), gen(tau), z)[0])
    drift = max(rel(x, r) for x in runs)
    return r, it, max(TOL, FACTOR * drift), drift


def record(point, qty, err, tol, drift):
    """Append one comparison to the parity log (NEGF_PARITY_LOG), if set."""
    path = os.environ.get("NEGF_PARITY_LOG")
    if not path:
        return
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    with open(path, "a") as fh:
        fh.write(json.dumps({"test": test, "point": [int(x) for x in point], "qty": qty, "err": float(err),
                             "drift": float(drift), "tol": float(tol)}) + "\n")


def check(point, qty, err, tols):
    """Assert err < tols[qty] and log it."""
    record(point, qty, err, tols[qty], tols["drift"][qty])
    assert err < tols[qty], (point, qty, err, tols[qty], tols["drift"][qty])


def check_point(out, p, point, r, N, tols, full=False, T=False):
    """GPU outputs of bound point p against the oracle result r of that point
    (diagonal blocks when ``full``, else orbital diagonals)."""
    d = (lambda x: x) if full else (lambda x: np.diagonal(x, axis1=1, axis2=2))
    for key in ("GR", "GL", "GG"):
        if key in out:
            check(point, key, rel(out[key][p, :N].cpu().numpy(), d(r[key])), tols)
    if N > 1 and "bond" in out:
        b = out["bond"][p, :N - 1].cpu().numpy()
        check(point, "bond", float(np.max(np.abs(b - r["bond"]))) / _bond_scale(r), tols)
    if T:
        check(point, "T", abs(float(out["T"][p]) - r["T"]) / max(1.0, abs(r["T"])), tols)


def summarize(path):
    """Markdown summary of a parity log: per quantity, the number of
    comparisons, how many errors exceeded 1e-10, the largest error and
    error / tolerance, error / drift (median, and largest where the error
    exceeded 1e-10), and how many tolerances came from G^>'s parts rather than
    its own drift."""
    rows = [json.loads(ln) for ln in open(path)]
    out = ["| quantity | comparisons | error > 1e-10 | max error | max error / tolerance | "
           "median error / drift | max error / drift (error > 1e-10) | tolerance from the parts |",
           "|---|---|---|---|---|---|---|---|"]
    for q in sorted({r["qty"] for r in rows}):
        v = [r for r in rows if r["qty"] == q]
        e = np.array([r["err"] for r in v])
        d = np.array([max(r["drift"], 1e-300) for r in v])
        t = np.array([r["tol"] for r in v])
        big = e > TOL
        ed_big = f"{np.max(e[big] / d[big]):.1f}" if big.any() else "-"
        parts = int(np.sum(t > np.maximum(TOL, FACTOR * d) * (1 + 1e-9)))
        out.append(f"| {q} | {len(v)} | {int(big.sum())} | {e.max():.2e} | {np.max(e / t):.2f} | "
                   f"{np.median(e / d):.2f} | {ed_big} | {parts if q == 'GG' else '-'} |")
    return "\n".join(out)


if __name__ == "__main__":
    import sys
    if len(sys.argv) == 3 and sys.argv[1] == "summarize":
        print(summarize(sys.argv[2]))
