"""GPU: the one-launch solve of small blocks (at most 8 orbitals; one wavefront
per point, points pulled from a device work queue) against the oracle and
against the batched per-operation path, through the C ABI."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import parity as P
from synth import random_tiny, strip_workload

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _solver(wl, **kw):
    from paper_1510_04686_amd.runtime import RGFSolver
    return RGFSolver(wl, **kw)


def _samples(nb, lengths, n_e=3, seed=0, up=None):
    """Several independent random devices of different lengths concatenated
    along the slab axis (ragged samples sharing the leads of the first)."""
    parts = [random_tiny(nb, N, n_e=n_e, seed=seed + i, up_block=up, eta=1e-3) for i, N in enumerate(lengths)]
    base = parts[0]
    h_diag = np.concatenate([p.h_diag for p in parts], axis=1)
    h_up = np.concatenate([p.h_up for p in parts], axis=0)
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    return dataclasses.replace(base, name="ragged", slab_offset=off, h_diag=h_diag, h_up=h_up)


@pytest.mark.parametrize("nb,lengths,up", [(1, [1], None), (3, [2], None), (5, [4, 1, 6], 5), (8, [5, 3], 4),
                                           (8, [1, 7, 2], 2), (6, [3], 3)])
@pytest.mark.parametrize("full", [False, True])
def test_small_solve_matches_oracle(nb, lengths, up, full):
    _say(f"one-launch small solve nb={nb} lengths={lengths} full={full}")
    wl = _samples(nb, lengths, seed=40 + nb, up=up)
    rng = np.random.default_rng(nb)
    wl.v_onsite = rng.uniform(0, 0.3, size=(wl.total_slabs, nb))
    shp = (wl.n_e, wl.total_slabs, nb)
    scR = rng.normal(size=shp) * 0.02 - 0.03j * rng.uniform(size=shp)
    scL = 0.02j * rng.uniform(size=shp)
    s = _solver(wl, capacity=4)
    s.lead_selfenergies()
    out = s.solve(full_blocks=full, want_T=True, scat_R=torch.from_numpy(scR).cuda(),
                  scat_L=torch.from_numpy(scL).cuda())
    torch.cuda.synchronize()
    assert s.status() == 0
    pts = [tuple(int(x) for x in p) for p in s.points]
    ref, tols = P.reference(wl, pts, full=full, scatR=scR, scatL=scL, transmission=True)
    counts = np.diff(wl.slab_offset)
    for p, (pt, r, t) in enumerate(zip(pts, ref, tols)):
        P.check_point(out, p, pt, r, int(counts[pt[0]]), t, full=full, T=True)


def test_small_solve_work_queue_many_points_equals_batched_path():
    """4096 strip points (more than the persistent grid's wavefronts, so every
    wavefront takes several points from the queue): every output against the
    batched per-operation path (checkpointed stores force that path) and
    sampled points against the oracle."""
    _say("one-launch small solve, 4096 points vs the batched path")
    wl = strip_workload(n_e=4096, e_lo=-3.9, e_hi=3.9)
    res = {}
    for store in ("full", "checkpoint"):
        s = _solver(wl, capacity=4096, store=store)
        out = s.solve(want_T=True)
        torch.cuda.synchronize()
        assert s.status() == 0
        res[store] = {k: v.cpu().numpy() for k, v in out.items()}
    for k in res["full"]:
        a, b = res["full"][k], res["checkpoint"][k]
        if k in ("GR", "GL", "GG"):      # per point, relative to its largest element
            scale = np.max(np.abs(b), axis=(1, 2), keepdims=True)
        elif k == "T":
            scale = np.maximum(1.0, np.abs(b))
        else:                            # bond currents: on the scale of the largest current
            scale = np.max(np.abs(b))
        err = float(np.max(np.abs(a - b) / np.maximum(scale, 1e-300)))
        _say(f"  {k}: largest difference {err:.2e}")
        assert err < 1e-8, (k, err)
    rng = np.random.default_rng(3)
    pts = [(0, 0, int(e)) for e in rng.choice(wl.n_e, size=6, replace=False)]
    ref, tols = P.reference(wl, pts, transmission=True)
    outd = {k: torch.from_numpy(v) for k, v in res["full"].items()}
    for pt, r, t in zip(pts, ref, tols):
        P.check_point(outd, pt[2], pt, r, wl.total_slabs, t, T=True)
