"""GPU: the NEGF-Poisson loop (Eq. 9) -- the finite-difference operator, its
conjugate-gradient solve and the Krylov vector kernels against the oracle's
dense operator and NumPy, and the damped Newton loop (density through the RGF,
its Jacobian through the adjoint) against the oracle's Newton solution."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import oracle as O
from synth import make_workload

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("shape,gate", [((7, 3, 4), False), ((5, 2, 1), True), ((9, 1, 2), False),
                                        ((4, 3, 5), True)])
def test_poisson_operator_and_solve_match_oracle(shape, gate):
    from paper_1510_04686_amd import negf as N
    nx, nz, ny = shape
    _say(f"poisson operator {shape} gate={gate}")
    g = N.poisson_grid(nx, nz, ny, gate, 0.2, -0.1, 0.05)
    L0 = O.poisson_matrix(nx, nz, ny, gate)
    b = O.poisson_boundary(nx, nz, ny, gate, 0.2, -0.1, 0.05)
    rng = np.random.default_rng(nx * 100 + nz * 10 + ny)
    n = nx * nz * ny
    V = rng.normal(size=n)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    N.negf_poisson_apply(g, _cuda(V), out, with_boundary=True)
    ref = L0 @ V - b
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-14 * np.max(np.abs(ref)) * 8
    N.negf_poisson_apply(g, _cuda(V), out, with_boundary=False)
    assert np.max(np.abs(out.cpu().numpy() - L0 @ V)) <= 1e-14 * np.max(np.abs(L0 @ V)) * 8
    nd, dens = rng.uniform(size=n), rng.uniform(size=n)
    N.negf_poisson_residual(g, _cuda(V), _cuda(dens), _cuda(nd), 5.7, out)
    refF = L0 @ V - b - 5.7 * (dens - nd)
    assert np.max(np.abs(out.cpu().numpy() - refF)) <= 1e-13 * np.max(np.abs(refF))
    work = torch.empty(N.negf_poisson_work_bytes(g), dtype=torch.uint8, device="cuda")
    rhs = rng.normal(size=n)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    it, rr = N.negf_poisson_solve(g, _cuda(rhs), x, work, tol=1e-13)
    xs = np.linalg.solve(L0, rhs)
    _say(f"  CG {it} iterations, relative residual {rr:.1e}")
    assert rr <= 1e-13
    assert np.max(np.abs(x.cpu().numpy() - xs)) <= 1e-11 * np.max(np.abs(xs))
    # with a diagonal shift (negative entries count as zero)
    sh = rng.uniform(-0.5, 3.0, size=n)
    it, rr = N.negf_poisson_solve(g, _cuda(rhs), x, work, tol=1e-13, shift=_cuda(sh))
    xs = np.linalg.solve(L0 + np.diag(np.maximum(sh, 0.0)), rhs)
    assert rr <= 1e-13
    assert np.max(np.abs(x.cpu().numpy() - xs)) <= 1e-11 * np.max(np.abs(xs))


def test_krylov_vector_kernels():
    from paper_1510_04686_amd import negf as N
    rng = np.random.default_rng(5)
    for n, m in [(1, 1), (255, 3), (1000, 7), (300001, 21)]:
        X = rng.normal(size=(m + 1, n))
        y = rng.normal(size=n)
        Xd, yd = _cuda(X), _cuda(y)
        out = torch.empty(m + 1, dtype=torch.float64, device="cuda")
        work = torch.empty(N.negf_vec_work_bytes(n, m + 1), dtype=torch.uint8, device="cuda")
        N.negf_vec_dots(Xd, m, yd, out, work)
        ref = X[:m] @ y
        assert np.max(np.abs(out.cpu().numpy()[:m] - ref)) <= 1e-12 * max(1.0, np.max(np.abs(X[:m]) @ np.abs(y)))
        c = rng.normal(size=m)
        N.negf_vec_combine(Xd, m, _cuda(c), 0.5, yd)
        ref = 0.5 * y + c @ X[:m]
        assert np.max(np.abs(yd.cpu().numpy() - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
        N.negf_vec_norms(_cuda(y), out, work)
        o = out.cpu().numpy()
        assert abs(o[0] - y @ y) <= 1e-12 * (y @ y) and o[1] == np.max(np.abs(y))


@pytest.mark.parametrize("kind", ["strip", "section"])
def test_density_jacobian_local_matches_oracle(kind):
    from paper_1510_04686_amd import negf as N
    from paper_1510_04686_amd.runtime import RGFSolver
    from synth import strip_workload
    if kind == "strip":
        wl = dataclasses.replace(strip_workload(n_slab=4, n_e=6, e_lo=-3.0, e_hi=3.0), eta=1e-2)
    else:
        wl = _tiny(n_slab=3, n_e=8)
    rng = np.random.default_rng(6)
    v = rng.uniform(0.0, 0.1, size=(wl.total_slabs, wl.atoms_per_slab))
    pts = [(0, 0, e) for e in range(wl.n_e)]
    ref = O.density_jacobian_local(wl, v, pts, O.lead_tables(wl))
    s = RGFSolver(wl)
    s.set_potential(_cuda(np.repeat(v, wl.orbs_per_atom, axis=1)))
    out = s.solve(want=("GR", "GL"))
    d = torch.zeros((wl.total_slabs, wl.atoms_per_slab), dtype=torch.float64, device="cuda")
    N.negf_density_jacobian_local(s.ctx, out["GR"], out["GL"], s.slab_stride, s.w_e, s.w_k, wl.g_s,
                                  wl.orbs_per_atom, d)
    torch.cuda.synchronize()
    assert np.max(np.abs(d.cpu().numpy() - ref)) <= 1e-10 * np.max(np.abs(ref))


def _tiny(n_slab=4, n_z=1, n_y=2, n_e=48):
    wl = make_workload("C2", n_slab=n_slab, n_e=n_e, n_k=1, n_z=n_z, n_y=n_y)
    return dataclasses.replace(wl, eta=0.05, v_onsite=None)


@pytest.mark.parametrize("case,jac,pre", [("chain", "adjoint", "local"), ("chain", "adjoint", "poisson"),
                                          ("section_gated", "fd", "local"),
                                          ("section_equilibrium", "adjoint", "local")])
def test_newton_poisson_matches_oracle(case, jac, pre):
    """The damped Newton loop on the GPU (RGF density, its Jacobian through the
    adjoint or central differences, GMRES preconditioned by the Poisson CG) and
    the oracle's (dense Jacobian) reach the same potential; the GPU's final
    residual is re-evaluated by the oracle.  In equilibrium the adjoint gives
    the exact Newton step (dn/dV is symmetric there): quadratic convergence;
    under bias the adjoint step is inexact (linear convergence) and the
    central difference is exact again."""
    from paper_1510_04686_amd.runtime import NewtonPoisson, RGFSolver
    if case == "chain":
        wl, nz, ny, gate = _tiny(), 1, 2, False
    else:
        wl, nz, ny, gate = _tiny(n_slab=6, n_z=2, n_y=2, n_e=40), 2, 2, True
    fill = None
    if case == "section_equilibrium":      # one Fermi level: both leads and the device's eta sink
        wl = dataclasses.replace(wl, mu_R=wl.mu_L)
        fill = wl.mu_L
    _say(f"Newton-Poisson {case}: nb={wl.nb} slabs={wl.total_slabs} n_e={wl.n_e}")
    grid = O.PoissonGrid(nz=nz, ny=ny, z_gate=gate, v_left=0.0, v_right=-0.05, v_gate=0.03)
    pts = [(0, 0, e) for e in range(wl.n_e)]
    leads = O.lead_tables(wl)
    beta = O.poisson_beta(11.7, 0.2715)
    n0 = O.density_atoms(wl, np.zeros((wl.total_slabs, nz * ny)), pts, leads, fill)
    nd = n0 + 0.02
    V_ref, h_ref = O.newton_poisson(wl, grid, beta, nd, np.zeros(n0.shape), pts, leads, tol=1e-12,
                                    eta_fill=fill)
    _say(f"  oracle: {len(h_ref) - 1} Newton steps, max|F| {h_ref[-1]:.1e}")
    s = RGFSolver(wl, adjoint_segment=-1 if jac == "adjoint" else 0)
    if fill is not None:
        s.set_eta_fill(True)
    s.lead_selfenergies()
    loop = NewtonPoisson(s, nz, ny, beta, nd, z_gate=gate, v_left=0.0, v_right=-0.05, v_gate=0.03,
                         krylov_tol=1e-6, jacobian=jac, preconditioner=pre)
    V, hist = loop.solve(np.zeros(n0.shape), tol=1e-11, max_newton=60, log=_say)
    assert s.status() == 0
    _say(f"  GPU: {loop.stats}")
    assert hist[-1] <= 1e-11
    if case != "chain":                 # exact Newton steps: as few as the oracle's, give or take the damping
        assert len(hist) <= len(h_ref) + 3
    Vg = V.cpu().numpy()
    err = np.max(np.abs(Vg - V_ref))
    _say(f"  max |V_gpu - V_oracle| = {err:.2e} eV")
    assert err < 1e-9
    # the GPU's root, checked by the oracle's own residual
    L = O.poisson_matrix(wl.total_slabs, nz, ny, gate)
    b = O.poisson_boundary(wl.total_slabs, nz, ny, gate, 0.0, -0.05, 0.03)
    F = L @ Vg.reshape(-1) - b - beta * (O.density_atoms(wl, Vg, pts, leads, fill) - nd).reshape(-1)
    assert np.max(np.abs(F)) < 1e-10
