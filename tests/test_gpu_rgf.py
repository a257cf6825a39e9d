"""GPU parity of the RGF path (leads, forward/backward sweeps, observables,
SCBA) against the CPU oracle on the same seeded inputs, through the C ABI."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from synth import make_workload, random_tiny

pytestmark = pytest.mark.gpu

import parity as P

TOL = P.TOL   # relative, FP64 path


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _solver(wl, **kw):
    from paper_1510_04686_amd.runtime import RGFSolver
    return RGFSolver(wl, **kw)


_rel = P.rel


def _ref_and_tol(wl, pts, full=False, **kw):
    """Oracle results plus per-point, per-quantity tolerances: 1e-10 relative, or
    10 x the point's FP64 drift measured by the oracle alone (tests/parity.py)."""
    ref, tols = P.reference(wl, pts, full=full, **kw)
    for t, p in zip(tols, pts):
        t["point"] = p
    return ref, tols


def _check_point(out, p, r, N, full=False, T=False, tol=None):
    P.check_point(out, p, tol["point"], r, N, tol, full=full, T=T)


# ---------------------------------------------------------------------------
# Leads
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nb,seed", [(1, 0), (6, 1), (20, 2)])
def test_lead_selfenergy_matches_oracle(nb, seed):
    _say(f"leads tiny nb={nb}")
    wl = random_tiny(nb, 2, n_e=5, seed=seed, eta=1e-4)
    s = _solver(wl)
    sL, sR = s.lead_selfenergies()
    torch.cuda.synchronize()
    assert s.lead_status == 0
    for ie in range(wl.n_e):
        z = wl.energy[ie] + 1j * wl.eta
        rL, itL, tL, dL = P.lead_reference(wl.lead_h00[0], wl.lead_h01_L, wl.lead_tau_L, z)
        rR, itR, tR, dR = P.lead_reference(wl.lead_h00[0], wl.lead_h01_R, wl.lead_tau_R, z)
        eL, eR = _rel(sL[0, ie].cpu().numpy(), rL), _rel(sR[0, ie].cpu().numpy(), rR)
        P.record((0, 0, ie), "sigma_L", eL, tL, dL)
        P.record((0, 0, ie), "sigma_R", eR, tR, dR)
        assert eL < tL
        assert eR < tR
        assert abs(int(s.iters_L[0, ie]) - itL) <= 1 and abs(int(s.iters_R[0, ie]) - itR) <= 1


@pytest.mark.parametrize("nb", [6, 10])
@pytest.mark.parametrize("complex_h", [False, True])
def test_lead_pair_shared_decimation(complex_h, nb):
    """h01_L = h01_R^dagger: one decimation serves both leads.  Each lead is
    checked against its own oracle decimation, and the shared run against two
    independent GPU decimations (nb = 6: the one-launch small-block
    decimation, nb = 10: the batched one)."""
    _say(f"leads shared decimation complex={complex_h} nb={nb}")
    wl = random_tiny(nb, 2, n_e=6, seed=11, eta=1e-3, complex_h=complex_h, n_k=2)
    s = _solver(wl)
    sL, sR = [x.clone() for x in s.lead_selfenergies(shared_decimation=True)]
    itL, itR = s.iters_L.clone(), s.iters_R.clone()
    assert s.lead_dual == 1 and s.lead_status == 0
    qL, qR = [x.clone() for x in s.lead_selfenergies(shared_decimation=False)]
    torch.cuda.synchronize()
    assert s.lead_dual == 0
    for ik in range(wl.n_k):
        for ie in range(wl.n_e):
            z = wl.energy[ie] + 1j * wl.eta
            for side, h01, tau, got, it, sep in (("L", wl.lead_h01_L, wl.lead_tau_L, sL, itL, qL),
                                                  ("R", wl.lead_h01_R, wl.lead_tau_R, sR, itR, qR)):
                r, itr, tol, dr = P.lead_reference(wl.lead_h00[ik], h01, tau, z)
                g = got[ik, ie].cpu().numpy()
                P.record((0, ik, ie), "sigma_" + side, _rel(g, r), tol, dr)
                assert _rel(g, r) < tol, (side, ik, ie, _rel(g, r))
                assert _rel(g, sep[ik, ie].cpu().numpy()) < tol, (side, "vs separate")
                assert abs(int(it[ik, ie]) - itr) <= 1, (side, int(it[ik, ie]), itr)


def test_lead_pair_falls_back_without_adjoint_couplings():
    _say("leads pair fallback")
    wl = random_tiny(6, 2, n_e=3, seed=12, eta=1e-3)
    wl.lead_h01_L = wl.lead_h01_L + 1e-6   # no longer h01_R^dagger
    s = _solver(wl)
    sL, sR = s.lead_selfenergies(shared_decimation=True)
    torch.cuda.synchronize()
    assert s.lead_dual == 0
    for ie in range(wl.n_e):
        z = wl.energy[ie] + 1j * wl.eta
        rL, _, _ = O.lead_selfenergy(wl.lead_h00[0], wl.lead_h01_L, wl.lead_tau_L, z)
        rR, _, _ = O.lead_selfenergy(wl.lead_h00[0], wl.lead_h01_R, wl.lead_tau_R, z)
        assert _rel(sL[0, ie].cpu().numpy(), rL) < 1e-9
        assert _rel(sR[0, ie].cpu().numpy(), rR) < 1e-9


def test_lead_selfenergy_reports_iteration_cap():
    _say("leads max_iter=1")
    wl = random_tiny(4, 2, n_e=2, seed=3, eta=1e-6)
    s = _solver(wl)
    s.lead_selfenergies(max_iter=1)
    assert s.lead_status == 1


# ---------------------------------------------------------------------------
# RGF sweeps
# ---------------------------------------------------------------------------

def _scat(wl, seed):
    rng = np.random.default_rng(seed)
    shp = (wl.n_e, wl.total_slabs, wl.nb)
    sR = rng.normal(size=shp) * 0.02 - 0.03j * rng.uniform(size=shp)
    sL = 0.02j * rng.uniform(size=shp)
    return sR, sL


@pytest.mark.parametrize("nb,N,up,seed", [(1, 1, None, 0), (3, 2, None, 1), (8, 5, 2, 2), (12, 4, 4, 3),
                                          (20, 3, 10, 4), (70, 3, 10, 5), (72, 2, 8, 6), (40, 6, 40, 7)])
@pytest.mark.parametrize("full", [False, True])
def test_rgf_matches_oracle_tiny(nb, N, up, seed, full):
    _say(f"rgf tiny nb={nb} N={N} up={up} full={full}")
    wl = random_tiny(nb, N, n_e=3, seed=seed, up_block=up, eta=1e-3)
    rng = np.random.default_rng(seed)
    wl.v_onsite = rng.uniform(0, 0.3, size=(N, nb))
    scR, scL = _scat(wl, seed)
    s = _solver(wl)
    s.lead_selfenergies()
    dR = torch.from_numpy(scR).cuda()
    dL = torch.from_numpy(scL).cuda()
    out = s.solve(full_blocks=full, want_T=True, scat_R=dR, scat_L=dL)
    torch.cuda.synchronize()
    assert s.status() == 0
    ref, tols = _ref_and_tol(wl, [tuple(p) for p in s.points], full=full, scatR=scR, scatL=scL,
                             transmission=True)
    for p, r in enumerate(ref):
        _check_point(out, p, r, N, full=full, T=True, tol=tols[p])


def test_rgf_strip_workload_all_energies():
    _say("rgf C1 strip, 256 energies")
    wl = make_workload("C1")
    s = _solver(wl)
    out = s.solve(want_T=True)
    torch.cuda.synchronize()
    assert s.status() == 0
    ref, tols = _ref_and_tol(wl, [tuple(p) for p in s.points], transmission=True)
    for p, r in enumerate(ref):
        _check_point(out, p, r, wl.total_slabs, T=True, tol=tols[p])


def test_rgf_ordered_strip_integer_transmission_on_gpu():
    from synth import strip_workload
    _say("rgf ordered strip integer T")
    wl = strip_workload(width=8, disorder=0.0, n_slab=20, eta=1e-9, n_e=64, e_lo=-3.9, e_hi=3.9)
    s = _solver(wl)
    s.lead_selfenergies(max_iter=200)
    out = s.solve(want_T=True, want=("GR", "GL", "GG", "bond"))
    T = out["T"].cpu().numpy()
    eps = -2 * np.cos(np.arange(1, 9) * np.pi / 9)
    for ie, E in enumerate(wl.energy):
        if np.min(np.abs(np.abs(E - eps) - 2)) < 0.05:
            continue
        assert abs(T[ie] - np.sum(np.abs(E - eps) < 2)) < 1e-5


def test_rgf_ragged_samples_and_observables():
    _say("rgf ragged multi-sample + observables")
    wl = make_workload("C4", n_slab=8, n_e=4, n_z=2, n_y=2, n_samples=5)
    counts = np.diff(wl.slab_offset)
    assert len(set(counts.tolist())) > 1
    s = _solver(wl, capacity=7)      # batches straddle samples of different length
    out = s.solve(want_T=True)
    n, J, jE = s.observables(out["GL"], out["bond"])
    torch.cuda.synchronize()
    assert s.status() == 0
    pts = [tuple(p) for p in s.points]
    ref, tols = _ref_and_tol(wl, pts, transmission=True)
    for p, r in enumerate(ref):
        _check_point(out, p, r, int(counts[pts[p][0]]), T=True, tol=tols[p])
    GLd = [np.diagonal(r["GL"], axis1=1, axis2=2) for r in ref]
    rn, rJ, rjE = O.observables(wl, pts, GLd, [r["bond"] for r in ref])
    # The reductions sum the per-point outputs with weights c_p = g_s w_E w_k: the
    # per-point bounds just checked bound their errors (plus the reductions' own
    # rounding, a few ulps of the sums).
    c = np.array([wl.g_s * wl.w_e[ie] * wl.w_k[ik] for (_, ik, ie) in pts])
    gl_err = np.array([t["GL"] * np.max(np.abs(np.diagonal(r["GL"], axis1=1, axis2=2))) for t, r in zip(tols, ref)])
    bd_err = np.array([t["bond"] * P._bond_scale(r) for t, r in zip(tols, ref)])
    n_bound = np.sum(c * gl_err) * wl.orbs_per_atom / (2 * np.pi) + 1e-14 * np.max(np.abs(rn))
    J_bound = np.sum(c * bd_err) + 1e-14 * np.max(np.abs(rJ))
    assert np.max(np.abs(n.cpu().numpy() - rn)) <= n_bound
    assert np.max(np.abs(J.cpu().numpy() - rJ)) <= J_bound
    jg = jE.cpu().numpy()[:, :, :rjE.shape[2]]
    for ie in range(wl.n_e):
        sel = [q for q, (_, _, e) in enumerate(pts) if e == ie]
        bound = np.sum((c / wl.w_e[ie])[sel] * bd_err[sel]) + 1e-14 * np.max(np.abs(rjE))
        assert np.max(np.abs(jg[:, ie] - rjE[:, ie])) <= bound, ie


def test_rgf_block400_reduced_length():
    _say("rgf block 400, 5 slabs, 2 k x 3 E")
    wl = make_workload("C2", n_slab=5, n_e=3, n_k=2)
    s = _solver(wl)
    out = s.solve(want_T=True)
    torch.cuda.synchronize()
    assert s.status() == 0
    pts = [tuple(p) for p in s.points]
    ref, tols = _ref_and_tol(wl, pts, transmission=True)
    for p, r in enumerate(ref):
        _check_point(out, p, r, 5, T=True, tol=tols[p])


def test_equilibrium_filled_eta_gives_kms_on_gpu():
    """mu_L = mu_R and a filled eta contact: G^< = -f (G - G^dagger) diagonal."""
    _say("rgf equilibrium")
    wl = random_tiny(10, 4, n_e=4, seed=9, up_block=5, eta=1e-3)
    wl.mu_L = wl.mu_R = 0.2
    s = _solver(wl)
    s.set_eta_fill(True)
    out = s.solve()
    GR = out["GR"].cpu().numpy()
    GL = out["GL"].cpu().numpy()
    for p, (_, _, ie) in enumerate(s.points):
        f = O.fermi(wl.energy[ie], 0.2, wl.kT)
        A = GR[p] - np.conj(GR[p])
        assert np.max(np.abs(GL[p] + f * A)) < 1e-10 * np.max(np.abs(A))


# ---------------------------------------------------------------------------
# SCBA (Eqs. 4-6) with the iteration captured in a HIP graph
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("graph", [True, False])
def test_scba_matches_oracle(graph):
    _say(f"scba graph={graph}")
    wl = make_workload("C3", n_slab=4, n_e=40, n_k=2, n_z=2, n_y=1)
    wl.D_ac, wl.M_op = 0.02, 0.03
    wl.eta = 1e-3
    n_iter = 3
    s = _solver(wl, capacity=23)
    out, hist = s.scba(n_iter=n_iter, graph=graph)
    torch.cuda.synchronize()
    assert s.status() == 0
    ref = O.scba(wl, n_iter)
    assert _rel(s.scat_R.cpu().numpy(), ref["sigR"]) < TOL
    assert _rel(s.scat_L.cpu().numpy(), ref["sigL"]) < TOL
    GR = out["GR"].cpu().numpy().reshape(wl.n_k, wl.n_e, -1, wl.nb)
    GL = out["GL"].cpu().numpy().reshape(wl.n_k, wl.n_e, -1, wl.nb)
    assert _rel(GR, ref["GRd"]) < TOL
    assert _rel(GL, ref["GLd"]) < TOL
    assert np.allclose(hist, ref["hist"], rtol=1e-8, atol=1e-14)


@pytest.mark.parametrize("graph", [True, False])
def test_scba_to_tolerance_matches_oracle(graph):
    """The Born loop run to a residual tolerance (at most 10 updates) stops at
    the oracle's update: with the tolerance between the third and fourth
    residuals of a fixed 4-update oracle run, it makes exactly 4 updates and
    returns that run's self-energies, diagonals and residuals (the update and
    the solve as two graphs with one residual read between them)."""
    _say(f"scba to tolerance, graph={graph}")
    wl = make_workload("C3", n_slab=4, n_e=40, n_k=2, n_z=2, n_y=1)
    wl.D_ac, wl.M_op = 0.02, 0.03
    wl.eta = 1e-3
    ref = O.scba(wl, 4)
    h = ref["hist"]
    assert h[0] > h[1] > h[2] > h[3] > 0
    tol = float(np.sqrt(h[2] * h[3]))
    s = _solver(wl, capacity=23)
    out, hist = s.scba(n_iter=10, graph=graph, tol=tol)
    torch.cuda.synchronize()
    assert s.status() == 0
    assert len(hist) == 4, hist
    assert np.allclose(hist, h, rtol=1e-8, atol=1e-14)
    assert _rel(s.scat_R.cpu().numpy(), ref["sigR"]) < TOL
    assert _rel(s.scat_L.cpu().numpy(), ref["sigL"]) < TOL
    GR = out["GR"].cpu().numpy().reshape(wl.n_k, wl.n_e, -1, wl.nb)
    GL = out["GL"].cpu().numpy().reshape(wl.n_k, wl.n_e, -1, wl.nb)
    assert _rel(GR, ref["GRd"]) < TOL
    assert _rel(GL, ref["GLd"]) < TOL
    # a tolerance no update reaches: all n_iter updates, as the fixed count
    out2, hist2 = s.scba(n_iter=3, graph=graph, tol=1e-30)
    ref3 = O.scba(wl, 3)
    torch.cuda.synchronize()
    assert len(hist2) == 3 and np.allclose(hist2, ref3["hist"], rtol=1e-8, atol=1e-14)
    assert _rel(s.scat_R.cpu().numpy(), ref3["sigR"]) < TOL


@pytest.mark.parametrize("graph", [False, True])
def test_two_lanes_match_one_lane(graph):
    """Batches spread over two contexts and streams give the results of one
    context (the same kernels, per point), in eager mode and inside the
    captured SCBA iteration."""
    _say(f"two lanes, graph={graph}")
    wl = make_workload("C3", n_slab=5, n_e=40, n_k=2, n_z=1, n_y=2)
    wl.n_scba = 3
    one = _solver(wl, capacity=16)
    two = _solver(wl, capacity=16, lanes=2)
    o1, h1 = one.scba(graph=graph)
    o2, h2 = two.scba(graph=graph)
    torch.cuda.synchronize()
    assert one.status() == 0 and two.status() == 0
    for k in ("GR", "GL", "bond"):
        a, b = o1[k].cpu().numpy(), o2[k].cpu().numpy()
        assert np.array_equal(a, b), (k, np.max(np.abs(a - b)))
    assert h1 == h2


@pytest.mark.parametrize("capacity", [64, 200])
def test_persistent_gemm_gives_the_same_solve(capacity):
    """The whole RGF path (ragged samples, several batches, anti-Hermitian and
    adding epilogues) with the persistent GEMM equals the per-tile GEMM bit for
    bit; block 80 gives four tiles per point, 800 tiles per full batch."""
    _say(f"persistent GEMM in the full solve, capacity={capacity}")
    wl = make_workload("C4", n_slab=8, n_e=40, n_z=2, n_y=4, n_samples=5)
    outs = []
    for pf in (2, 3):
        s = _solver(wl, capacity=capacity, tune={"gemm_prefetch": pf, "inv_outer": 64})
        o = s.solve(want_T=True)
        torch.cuda.synchronize()
        assert s.status() == 0
        outs.append({k: v.cpu().numpy() for k, v in o.items()})
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_three_level_inverse_in_the_full_solve():
    """Block 400 with the three-level inverse (outer 192, mid 64) against the
    oracle, every point."""
    _say("rgf block 400 with the three-level inverse")
    wl = make_workload("C2", n_slab=5, n_e=3, n_k=2)
    s = _solver(wl, tune={"gemm_prefetch": 2, "inv_outer": 192, "inv_mid": 64})
    assert s.tuning["inv_mid"] == 64
    out = s.solve(want_T=True)
    torch.cuda.synchronize()
    assert s.status() == 0
    pts = [tuple(p) for p in s.points]
    ref, tols = _ref_and_tol(wl, pts, transmission=True)
    for p, r in enumerate(ref):
        _check_point(out, p, r, wl.total_slabs, T=True, tol=tols[p])


def test_abi_rejects_empty_and_out_of_range_point_ranges():
    """Empty point sets, ranges past the bound points or the capacity, and calls
    out of order are refused on the host before anything is launched; the
    context then still solves correctly."""
    from paper_1510_04686_amd import negf as N
    _say("ABI: empty / out-of-range point ranges, call order")
    wl = random_tiny(4, 3, n_e=3, seed=11, eta=1e-3)
    s = _solver(wl, capacity=2)
    s.lead_selfenergies()
    c = s.ctx
    with pytest.raises(N.NegfError) as e:
        N.negf_rgf_forward(c, 0, 0, s.sigma_L, s.sigma_R)
    assert e.value.code == -1                       # NEGF_EINVAL: empty range
    with pytest.raises(N.NegfError) as e:
        N.negf_rgf_forward(c, s.n_points - 1, 2, s.sigma_L, s.sigma_R)
    assert e.value.code == -1                       # past the bound points
    with pytest.raises(N.NegfError) as e:
        N.negf_rgf_forward(c, 0, 3, s.sigma_L, s.sigma_R)
    assert e.value.code == -2                       # NEGF_ESHAPE: above the capacity
    GR = torch.zeros((2, s.slab_stride, wl.nb), dtype=torch.complex128, device="cuda")
    N.negf_rgf_forward(c, 0, 2, s.sigma_L, s.sigma_R)
    with pytest.raises(N.NegfError) as e:
        N.negf_rgf_backward(c, 1, 2, GR=GR, slab_stride=s.slab_stride)
    assert e.value.code == -5                       # NEGF_ESTATE: not the forward's range
    with pytest.raises(N.NegfError) as e:
        N.negf_bind(c, wl.nb, wl.slab_offset, wl.n_k, wl.n_e, s.h_diag, s.h_up, 0, wl.up_block, s.v, s.energy,
                    wl.eta, wl.mu_L, wl.mu_R, wl.kT, 0, np.zeros((0, 3), dtype=np.int32))
    assert e.value.code == -1                       # no points to bind
    s._bind()                                       # restore the solver's binding
    out = s.solve()
    torch.cuda.synchronize()
    assert s.status() == 0
    ref, tols = _ref_and_tol(wl, [tuple(p) for p in s.points])
    for p, r in enumerate(ref):
        _check_point(out, p, r, 3, tol=tols[p])


def test_transpose_batched_exact():
    from paper_1510_04686_amd import negf as N
    for n, cnt in [(1, 3), (31, 2), (33, 5), (400, 3)]:
        a = torch.randn(cnt, n, n, dtype=torch.complex128, device="cuda")
        b = torch.empty_like(a)
        N.negf_transpose_batched(a, b)
        assert torch.equal(b, a.transpose(1, 2))


def test_lead_mirror_tables_and_rgf_at_minus_k():
    """Four k-points: the k = 3 pi / 2 lead tables are the transposes of the
    k = pi / 2 ones (no decimation of their own).  They match a direct
    decimation at the lead tolerance, and the RGF outputs at every k match the
    oracle, which decimates every k-point."""
    from paper_1510_04686_amd.runtime import RGFSolver
    wl = make_workload("C2", n_slab=4, n_e=3, n_k=4, n_z=1, n_y=2)
    s = RGFSolver(wl)
    assert s.mirror == {3: 1}
    s.lead_selfenergies()
    assert s.last_lead_ranges == [(0, 0, wl.n_e), (1, 0, wl.n_e), (2, 0, wl.n_e)]
    mir_L, mir_R = s.sigma_L.clone(), s.sigma_R.clone()
    s.mirror = {}
    s.lead_selfenergies()
    torch.cuda.synchronize()
    for a, b in ((mir_L, s.sigma_L), (mir_R, s.sigma_R)):
        a3, b3 = a[3].cpu().numpy(), b[3].cpu().numpy()
        assert np.max(np.abs(a3 - b3)) <= 1e-10 * np.max(np.abs(b3))
    s.mirror = {3: 1}
    # the per-range form (one batch at -k alone): decimates k = pi / 2, transposes into k = 3 pi / 2
    s.sigma_L.zero_()
    s.sigma_R.zero_()
    assert s.lead_selfenergies_for_ranges([(3, 0, wl.n_e)]) == [(1, 0, wl.n_e)]
    for a_, b_ in ((s.sigma_L[3], mir_L[3]), (s.sigma_R[3], mir_R[3])):
        assert float((a_ - b_).abs().max()) <= 1e-12 * float(b_.abs().max())
    s.lead_selfenergies()
    out = s.solve()
    torch.cuda.synchronize()
    assert s.status() == 0
    pts = [tuple(int(x) for x in p) for p in s.points]
    sel = [i for i, p in enumerate(pts) if p[1] in (1, 3)]
    ref, tols = P.reference(wl, [pts[i] for i in sel])
    for i, r, t in zip(sel, ref, tols):
        P.check_point(out, i, pts[i], r, wl.total_slabs, t)
