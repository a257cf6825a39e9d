"""Plain NumPy FP64 oracle of the NEGF-Poisson loop (Eq. 9) -- TEST
INFRASTRUCTURE ONLY (tests/, the smoke check and the benchmark's CPU baseline).

Eq. (9) ties the electrostatic potential Phi to the electron density of Eq. (7):
div(eps grad Phi) = e (n - N_D).  The onsite energy of Eq. (1) is the electron's
potential energy V = -e Phi, so per atom, on a finite-difference grid whose
nodes are the atoms (spacing h, cell volume h^3, n and N_D in electrons per
atom):

    (L V)_a = beta (n_a(V) - N_D,a),   beta = e^2 / (eps h),

with (L V)_a = sum over the six grid neighbours b of (V_a - V_b).  Readings of
the paper, which gives only Eq. (9) and says that it is iterated with the NEGF
equations until convergence (all stated again in the design notes):

* grid: atom (x, z, y) -- x the slab (transport), z across the body, y along
  the direction the transverse momentum k runs over, periodic;
* boundaries: x = -1 and x = N_x are the contacts, held at v_left / v_right;
  the z faces are either insulating (zero normal field) or gates held at
  v_gate; the y direction is periodic;
* the loop is Newton's method on F(V) = L V - beta (n(V) - N_D), with the
  Jacobian dF/dV = L - beta dn/dV, its steps capped at a largest change per
  atom (damping).

Pins (tests/test_oracle_pins.py): the operator reproduces the closed forms of
the discrete Laplace and uniform-charge problems; the density Jacobian matches
central differences of the density and the VJP of ``dense_grad``; the Newton
solution is pinned by its residual, evaluated through ``solve_points`` and
``observables`` independently of the Newton iteration.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .negf_oracle import dense, fermi, lead_tables, observables, solve_points

E2_OVER_EPS0 = 18.0951      # e^2 / eps_0 in eV nm


def poisson_beta(eps_r: float, h_nm: float) -> float:
    """beta = e^2 / (eps_r eps_0 h) in eV per electron."""
    return E2_OVER_EPS0 / (eps_r * h_nm)


def _idx(x, z, y, nz, ny):
    return (x * nz + z) * ny + y


def poisson_matrix(nx: int, nz: int, ny: int, z_gate: bool):
    """Dense L0 (boundary values zero) and the boundary map: L V = L0 V - b,
    b = poisson_boundary(...).  Plain loops over atoms and their six
    neighbours; a neighbour outside the grid in x (contact) or z (gate) adds
    its coupling to the diagonal only (its value goes to b); an insulating z
    face adds nothing."""
    n = nx * nz * ny
    L = np.zeros((n, n))
    for x in range(nx):
        for z in range(nz):
            for y in range(ny):
                a = _idx(x, z, y, nz, ny)
                for dx, dz, dy in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    xb, zb, yb = x + dx, z + dz, (y + dy) % ny
                    if dy != 0 and ny == 1:
                        continue                     # the periodic image is the atom itself
                    if zb < 0 or zb >= nz:
                        if z_gate:
                            L[a, a] += 1.0
                        continue
                    L[a, a] += 1.0
                    if 0 <= xb < nx:
                        L[a, _idx(xb, zb, yb, nz, ny)] -= 1.0
    return L


def poisson_boundary(nx: int, nz: int, ny: int, z_gate: bool, v_left: float, v_right: float,
                     v_gate: float = 0.0) -> np.ndarray:
    """b with L V = L0 V - b: the boundary values times their couplings."""
    b = np.zeros(nx * nz * ny)
    for x in range(nx):
        for z in range(nz):
            for y in range(ny):
                a = _idx(x, z, y, nz, ny)
                if x == 0:
                    b[a] += v_left
                if x == nx - 1:
                    b[a] += v_right
                if z_gate:
                    if z == 0:
                        b[a] += v_gate
                    if z == nz - 1:
                        b[a] += v_gate
    return b


def density_atoms(wl, v_atom, points, leads, eta_fill=None):
    """n per atom (Eq. 7) of a single-sample workload at the per-atom potential
    v_atom [N_x, atoms], through solve_points and observables (eta_fill: the
    Fermi level that fills the device's eta sink, None for an empty sink)."""
    v_orb = np.repeat(np.asarray(v_atom, dtype=np.float64), wl.orbs_per_atom, axis=1)
    w = dataclasses.replace(wl, v_onsite=v_orb)
    res = solve_points(w, points, leads=leads, diag_only=True, eta_fill=eta_fill)
    n, _, _ = observables(w, points, [r["GL"] for r in res], [r["bond"] for r in res])
    return n


def density_jacobian(wl, v_atom, points, leads, eta_fill=None):
    """dn_a/dV_b (atoms x atoms) of a single-sample workload.

    From dG^R = G^R dV G^R and dG^< = G^R dV G^< + G^< dV G^A (dV diagonal,
    the same on the orbitals of one atom):
      dn_a/dV_b = sum_points c_p sum_{o in a, o' in b} Im(G_oo' G^<_o'o + G^<_oo' conj(G_oo')),
    c_p = g_s w_E w_k / 2pi.  In equilibrium (one Fermi level f for both
    leads and the eta sink) G^< = -f (G - G^dagger) and each term becomes
    -2 f Im(G_oo' G_o'o), symmetric in (a, b).  Dense inversion; tiny systems
    only."""
    nat, opa = wl.atoms_per_slab, wl.orbs_per_atom
    N = wl.total_slabs
    na = N * nat
    v_orb = np.repeat(np.asarray(v_atom, dtype=np.float64), opa, axis=1)
    D = np.zeros((na, na))
    for s, ik, ie in points:
        hd, hu, _ = wl.sample_blocks(int(s), int(ik))
        E = float(wl.energy[ie])
        sL, sR = leads[(int(ik), int(ie))][:2]
        ef = None if eta_fill is None else float(fermi(E, eta_fill, wl.kT))
        r = dense(hd, hu, E, wl.eta, sL, sR, float(fermi(E, wl.mu_L, wl.kT)), float(fermi(E, wl.mu_R, wl.kT)),
                  v=[v_orb[i] for i in range(N)], full=True, eta_fill=ef)
        G, Gl = r["G"], r["Gl"]
        M = np.imag(G * Gl.T + Gl * np.conj(G))
        c = wl.g_s * wl.w_e[ie] * wl.w_k[ik] / (2 * np.pi)
        D += c * M.reshape(na, opa, na, opa).sum(axis=(1, 3))
    return D


def density_jacobian_local(wl, v_atom, points, leads, eta_fill=None):
    """The orbital-diagonal part of dn_a/dV_a per atom (the o' = o terms of
    ``density_jacobian``'s diagonal), from the orbital diagonals of G^R and G^<:
      d_a = sum_points c_p sum_{o in a} Im(G_oo G^<_oo + G^<_oo conj(G_oo)).
    Pinned by: equal to the diagonal of ``density_jacobian`` for one-orbital
    atoms."""
    nat, opa = wl.atoms_per_slab, wl.orbs_per_atom
    v_orb = np.repeat(np.asarray(v_atom, dtype=np.float64), opa, axis=1)
    w = dataclasses.replace(wl, v_onsite=v_orb)
    res = solve_points(w, points, leads=leads, diag_only=True, eta_fill=eta_fill)
    d = np.zeros((wl.total_slabs, nat))
    for (s, ik, ie), r in zip(points, res):
        g, gl = r["GR"], r["GL"]
        c = wl.g_s * wl.w_e[ie] * wl.w_k[ik] / (2 * np.pi)
        d += c * np.imag(g * gl + gl * np.conj(g)).reshape(wl.total_slabs, nat, opa).sum(axis=2)
    return d


@dataclasses.dataclass
class PoissonGrid:
    nz: int
    ny: int
    z_gate: bool = False
    v_left: float = 0.0
    v_right: float = 0.0
    v_gate: float = 0.0


def newton_poisson(wl, grid: PoissonGrid, beta: float, n_d, v0, points=None, leads=None, tol=1e-9,
                   max_iter=30, max_step=0.1, eta_fill=None):
    """Newton's method on F(V) = L V - beta (n(V) - N_D) for a single-sample
    workload; V per atom [N_x, atoms].  Each step solves (L - beta dn/dV) dV = -F
    with the dense Jacobian; a step larger than max_step (eV, on any atom) is
    scaled down to it, the usual damping of the NEGF-Poisson loop far from the
    solution.  Returns (V, history of max |F|)."""
    nx, nat = wl.total_slabs, wl.atoms_per_slab
    assert nat == grid.nz * grid.ny
    if points is None:
        points = [(0, k, e) for k in range(wl.n_k) for e in range(wl.n_e)]
    if leads is None:
        leads = lead_tables(wl)
    L = poisson_matrix(nx, grid.nz, grid.ny, grid.z_gate)
    b = poisson_boundary(nx, grid.nz, grid.ny, grid.z_gate, grid.v_left, grid.v_right, grid.v_gate)
    nd = np.asarray(n_d, dtype=np.float64).reshape(-1)
    V = np.asarray(v0, dtype=np.float64).reshape(-1).copy()
    hist = []
    for _ in range(max_iter + 1):
        n = density_atoms(wl, V.reshape(nx, nat), points, leads, eta_fill).reshape(-1)
        F = L @ V - b - beta * (n - nd)
        hist.append(float(np.max(np.abs(F))))
        if hist[-1] <= tol:
            break
        J = L - beta * density_jacobian(wl, V.reshape(nx, nat), points, leads, eta_fill)
        dV = np.linalg.solve(J, -F)
        V = V + dV * min(1.0, max_step / max(float(np.max(np.abs(dV))), 1e-300))
    return V.reshape(nx, nat), hist
