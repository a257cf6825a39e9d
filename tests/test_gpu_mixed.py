"""GPU: the mixed-precision form (complex FP32 matrix-core block algebra, one
FP64-residual Newton-Schulz step per block inverse, FP64 leads and FP64
accumulation of density and current) against the FP64 oracle at the 1e-4
relative bound on densities and currents."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from synth import make_workload, random_tiny

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-4


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _run(wl, precision, **kw):
    from paper_1510_04686_amd import negf as N
    from paper_1510_04686_amd.runtime import RGFSolver
    s = RGFSolver(wl, precision=precision, **kw)
    out = s.solve()
    n, J, _ = s.observables(out["GL"], out["bond"])
    torch.cuda.synchronize()
    stats = N.negf_mixed_stats(s.ctx) if precision == "mixed" else (0, 0.0)
    return s, out, n.cpu().numpy(), J.cpu().numpy(), stats


def _oracle_obs(wl, pts):
    ref = O.solve_points(wl, pts)
    GLd = [np.diagonal(r["GL"], axis1=1, axis2=2) for r in ref]
    n, J, _ = O.observables(wl, pts, GLd, [r["bond"] for r in ref])
    return ref, n, J


@pytest.mark.parametrize("case", ["tiny", "block400"])
def test_mixed_density_and_current_within_1e4(case):
    _say(f"mixed precision {case}")
    if case == "tiny":
        wl = random_tiny(20, 5, n_e=6, seed=31, up_block=10, eta=1e-3)
    else:
        wl = make_workload("C2", n_slab=6, n_e=4, n_k=2)
    s, out, n, J, (nfb, maxres) = _run(wl, "mixed")
    _say(f"  fallbacks={nfb} max NS residual={maxres:.2e}")
    pts = [tuple(p) for p in s.points]
    ref, rn, rJ = _oracle_obs(wl, pts)
    err_n = np.max(np.abs(n - rn)) / np.max(np.abs(rn))
    err_J = np.max(np.abs(J - rJ)) / max(np.max(np.abs(rJ)), 1e-300)
    _say(f"  density err {err_n:.2e}, current err {err_J:.2e}")
    assert err_n < TOL_MIXED
    # bond currents are a small net flow on top of O(density) terms: the 1e-4
    # bound applies relative to the current, with the density scale as floor
    assert np.max(np.abs(J - rJ)) < TOL_MIXED * max(np.max(np.abs(rJ)), 1e-3 * np.max(np.abs(rn)))


def test_mixed_matches_fp64_gpu_path_and_reports_stats():
    _say("mixed vs fp64 gpu")
    wl = make_workload("C2", n_slab=8, n_e=6, n_k=1)
    _, _, n64, J64, _ = _run(wl, "fp64")
    s, _, n32, J32, (nfb, maxres) = _run(wl, "mixed")
    assert maxres < 1e-2 or nfb > 0
    assert np.max(np.abs(n32 - n64)) / np.max(np.abs(n64)) < TOL_MIXED
