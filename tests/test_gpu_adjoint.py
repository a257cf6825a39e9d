"""GPU: the adjoint RGF (dn/dV vector-Jacobian product) against the oracle's
dense-inverse gradient and the oracle's central finite differences."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from synth import make_workload, random_tiny

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _solver(wl, **kw):
    from paper_1510_04686_amd.runtime import RGFSolver
    return RGFSolver(wl, **kw)


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def _tiny(seed=3, nb=8, N=5, up=4, n_e=3):
    wl = random_tiny(nb, N, n_e=n_e, seed=seed, up_block=up, eta=1e-3)
    rng = np.random.default_rng(seed + 50)
    wl.v_onsite = np.repeat(rng.uniform(0, 0.3, size=(N, nb // up)), up, axis=1)
    return wl


@pytest.mark.parametrize("store", ["full", "checkpoint"])
@pytest.mark.parametrize("segment", [1, 2, -1, 5])
def test_adjoint_matches_dense_gradient(segment, store):
    _say(f"adjoint tiny segment={segment} store={store}")
    wl = _tiny()
    rng = np.random.default_rng(7)
    w = rng.normal(size=(wl.total_slabs, wl.atoms_per_slab))
    s = _solver(wl, adjoint_segment=segment, store=store)
    s.density()
    g = s.density_vjp(torch.from_numpy(w)).cpu().numpy()
    torch.cuda.synchronize()
    assert s.status() == 0
    pts = [tuple(p) for p in s.points]
    ref = O.dense_grad(wl, w, wl.v_onsite, pts, O.lead_tables(wl))
    assert _rel(g, ref) < 1e-10


@pytest.mark.parametrize("store", ["full", "checkpoint"])
def test_adjoint_ragged_samples_multi_batch(store):
    _say(f"adjoint ragged multi-sample, 3 batches, store={store}")
    wl = make_workload("C4", n_slab=5, n_e=2, n_z=1, n_y=2, n_samples=4)
    wl.eta = 1e-3
    wl.v_onsite = np.full((wl.total_slabs, wl.nb), 0.05)
    assert len(set(np.diff(wl.slab_offset).tolist())) > 1
    rng = np.random.default_rng(8)
    w = rng.normal(size=(wl.total_slabs, wl.atoms_per_slab))
    s = _solver(wl, capacity=3, adjoint_segment=2, store=store)
    s.density()
    g = s.density_vjp(torch.from_numpy(w)).cpu().numpy()
    pts = [tuple(p) for p in s.points]
    ref = O.dense_grad(wl, w, wl.v_onsite, pts, O.lead_tables(wl))
    assert _rel(g, ref) < 1e-10


def test_adjoint_matches_oracle_finite_differences():
    """Paper-shaped potential profile (smooth, 0..0.3 eV), central differences
    h = 1e-5 eV of the oracle's own density at a few atoms."""
    _say("adjoint vs oracle FD")
    wl = make_workload("C5", n_slab=6, n_e=2, n_z=1, n_y=2)
    wl.eta = 1e-3
    rng = np.random.default_rng(9)
    w = rng.normal(size=(wl.total_slabs, wl.atoms_per_slab))
    s = _solver(wl, adjoint_segment=-1)
    s.density()
    g = s.density_vjp(torch.from_numpy(w)).cpu().numpy()
    pts = [tuple(p) for p in s.points]
    leads = O.lead_tables(wl)
    h = 1e-5
    for sl, a in [(0, 0), (2, 1), (5, 0), (3, 1)]:
        vp, vm = wl.v_onsite.copy(), wl.v_onsite.copy()
        vp[sl, a * 10:(a + 1) * 10] += h
        vm[sl, a * 10:(a + 1) * 10] -= h
        fd = (O.density_objective(wl, w, vp, pts, leads) - O.density_objective(wl, w, vm, pts, leads)) / (2 * h)
        assert abs(fd - g[sl, a]) < 1e-6 * np.max(np.abs(g)) + 1e-12, (sl, a, fd, g[sl, a])


def test_autograd_function_backward():
    from paper_1510_04686_amd.runtime import RGFDensity
    _say("adjoint through torch.autograd")
    wl = _tiny(seed=11)
    s = _solver(wl, adjoint_segment=2)
    v = torch.from_numpy(wl.v_onsite[:, ::wl.orbs_per_atom].copy()).cuda().requires_grad_(True)
    n = RGFDensity.apply(v, s)
    w = torch.randn_like(n)
    (n * w).sum().backward()
    ref = O.dense_grad(wl, w.cpu().numpy(), wl.v_onsite, [tuple(p) for p in s.points], O.lead_tables(wl))
    assert _rel(v.grad.cpu().numpy(), ref) < 1e-10
    # density itself against the oracle
    res = O.solve_points(wl, [tuple(p) for p in s.points])
    GLd = [np.diagonal(r["GL"], axis1=1, axis2=2) for r in res]
    rn, _, _ = O.observables(wl, [tuple(p) for p in s.points], GLd, [r["bond"] for r in res])
    assert _rel(n.detach().cpu().numpy(), rn) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("segment", [1, 2, 3, -1, 9])
def test_checkpointed_stores_equal_full_stores(segment, precision):
    """Checkpointed g / g^< stores (every segment recomputed from its
    checkpoint in the backward sweep and the adjoint) give the full-store
    results bit for bit: the same kernels on the same values.  Ragged samples
    (5-11 slabs) in several batches, so segments end at different slabs of
    different points; every output of the backward sweep, and the adjoint."""
    _say(f"checkpointed vs full stores, segment={segment} {precision}")
    wl = make_workload("C4", n_slab=10, n_e=3, n_z=1, n_y=2, n_samples=4)
    wl.eta = 1e-3
    wl.v_onsite = np.full((wl.total_slabs, wl.nb), 0.05)
    assert len(set(np.diff(wl.slab_offset).tolist())) > 1
    w = torch.from_numpy(np.random.default_rng(12).normal(size=(wl.total_slabs, wl.atoms_per_slab)))
    res = {}
    for store in ("full", "checkpoint"):
        s = _solver(wl, capacity=5, adjoint_segment=segment, store=store,
                    precision=precision, point_redo=float("inf"))
        out = s.solve(want_T=True)
        torch.cuda.synchronize()
        assert s.status() in (0, 4)          # 4: mixed-precision block fallbacks (same in both)
        r = {k: v.cpu().numpy() for k, v in out.items()}
        if precision == "fp64":
            s.density()
            r["grad"] = s.density_vjp(w).cpu().numpy()
        res[store] = r
    for k in res["full"]:
        assert np.array_equal(res["full"][k], res["checkpoint"][k]), k


@pytest.mark.parametrize("store", ["full", "checkpoint"])
def test_adjoint_with_absorbing_contacts_matches_dense_gradient(store):
    """Disordered absorbing-potential contacts: the adjoint's recomputed forward
    slabs carry the contact self-energies too (two ragged samples, two batches)."""
    from synth.workloads import cross_section_workload
    _say(f"adjoint with absorbing contacts, store={store}")
    wl = cross_section_workload("cap", 1, 2, [3, 2], 1, np.linspace(-0.5, 0.5, 2), 17, cap_slabs=3, cap_w=0.5,
                                eta=1e-3)
    rng = np.random.default_rng(10)
    wl.v_onsite = rng.uniform(0, 0.1, size=(wl.total_slabs, wl.nb))
    w = rng.normal(size=(wl.total_slabs, wl.atoms_per_slab))
    s = _solver(wl, capacity=2, adjoint_segment=2, store=store)
    s.density()
    g = s.density_vjp(torch.from_numpy(w)).cpu().numpy()
    torch.cuda.synchronize()
    assert s.status() == 0
    pts = [tuple(p) for p in s.points]
    ref = O.dense_grad(wl, w, wl.v_onsite, pts, O.lead_tables(wl))
    assert _rel(g, ref) < 1e-10


@pytest.mark.parametrize("store", ["full", "checkpoint"])
def test_adjoint_with_fixed_scattering_matches_dense_gradient(store):
    """dn/dV at fixed scattering self-energies (a frozen Born-loop state): the
    forward pass and the adjoint's recomputed slabs both carry them."""
    _say(f"adjoint with fixed Sigma_scat, store={store}")
    wl = _tiny(seed=11, n_e=3)
    rng = np.random.default_rng(13)
    shp = (wl.n_e, wl.total_slabs, wl.nb)
    sR = 0.02 * rng.normal(size=shp) - 0.03j * rng.uniform(size=shp)
    sL = 0.02j * rng.uniform(size=shp)
    w = rng.normal(size=(wl.total_slabs, wl.atoms_per_slab))
    s = _solver(wl, capacity=2, adjoint_segment=2, store=store)
    tR, tL = torch.from_numpy(sR).cuda(), torch.from_numpy(sL).cuda()
    s.density(tR, tL)
    g = s.density_vjp(torch.from_numpy(w), tR, tL).cpu().numpy()
    torch.cuda.synchronize()
    assert s.status() == 0
    pts = [tuple(p) for p in s.points]
    ref = O.dense_grad(wl, w, wl.v_onsite, pts, O.lead_tables(wl), sR, sL)
    assert _rel(g, ref) < 1e-10
