"""Plain NumPy complex-FP64 oracle of the NEGF/RGF hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline of the benchmark, never by the product path.

Notation follows the paper's Eqs. (1)-(8):
  G^R = (E - H - V - Sigma^R)^-1                             Eq. (1)
  G^< = G^R Sigma^< G^R^dagger                               Eq. (2)
  Sigma = Sigma_lead + Sigma_optical + Sigma_acoustic        Eq. (3)
  acoustic / optical phonon self-energies                   Eqs. (4)-(6)
  density and current                                       Eqs. (7)-(8)
plus standard RGF block recursions for a block-tridiagonal H (slabs i=0..N-1),
Sancho-Rubio decimation for the ordered semi-infinite leads, and the lesser
recursion for G^<.  Every product is a plain ``@`` and every inverse is
``numpy.linalg.inv``: no blocking, fusion or reordering.

Readings of the paper (where it is silent or garbled) are listed in the module
constants and docstrings; each is pinned by a test in tests/test_oracle_pins.py
unless it says "parity unpinned".
"""
from __future__ import annotations

import numpy as np

inv = np.linalg.inv


def dag(a):
    return a.conj().T


# ---------------------------------------------------------------------------
# Distribution functions
# ---------------------------------------------------------------------------

def fermi(E, mu, kT):
    """Fermi-Dirac occupation of the lead reservoirs (temperature kT in eV).
    Pinned by: equilibrium (KMS) identity test."""
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp((np.asarray(E, dtype=np.float64) - mu) / kT))


def norm1(a):
    """Matrix 1-norm (largest column sum of magnitudes)."""
    return float(np.abs(a).sum(axis=0).max())


# ---------------------------------------------------------------------------
# Lead self-energies (Eq. 3, Sigma_lead; ordered leads, Sancho-Rubio decimation)
# ---------------------------------------------------------------------------

def sancho_rubio(h00, h01, z, tol=1e-14, max_iter=100):
    """Surface Green's function of a semi-infinite ordered lead by iterative
    layer decimation (Lopez Sancho, Lopez Sancho & Rubio 1985).

    h00: principal-layer Hamiltonian; h01: coupling from a layer to the next
    layer deeper in the lead; z = E + i eta.  Each step eliminates every other
    layer, doubling the range the couplings alpha, beta span.  Stops when
    ||alpha||_1 + ||beta||_1 < tol * ||h01||_1 or after max_iter steps.
    Returns (g_s, iterations, converged).
    Pinned by: closed form of the 1-D chain and of the ordered strip
    (tests/test_oracle_pins.py) and the surface Dyson fixed point."""
    n = h00.shape[0]
    eye = np.eye(n)
    eps_s = h00.astype(np.complex128).copy()
    eps = eps_s.copy()
    alpha = h01.astype(np.complex128).copy()
    beta = dag(alpha)
    ref = norm1(h01)
    it = 0
    converged = False
    while it < max_iter:
        it += 1
        g = inv(z * eye - eps)
        agb = alpha @ g @ beta
        bga = beta @ g @ alpha
        eps_s = eps_s + agb
        eps = eps + agb + bga
        alpha = alpha @ g @ alpha
        beta = beta @ g @ beta
        if norm1(alpha) + norm1(beta) < tol * ref:
            converged = True
            break
    return inv(z * eye - eps_s), it, converged


def sancho_rubio_alt(h00, h01, z, tol=1e-14, max_iter=100):
    """The same decimation with every triple product associated the other way,
    a(g b) instead of (a g) b, and the inverse taken by an LU solve.  Used only
    to measure how far two correct FP64 evaluations of one point can drift
    apart (its conditioning; ~1/eta for propagating lead modes), which sets the
    per-point parity tolerance of the GPU tests."""
    n = h00.shape[0]
    eye = np.eye(n)
    eps_s = h00.astype(np.complex128).copy()
    eps = eps_s.copy()
    alpha = h01.astype(np.complex128).copy()
    beta = dag(alpha)
    ref = norm1(h01)
    it = 0
    converged = False
    while it < max_iter:
        it += 1
        g = np.linalg.solve(z * eye - eps, eye)
        agb = alpha @ (g @ beta)
        bga = beta @ (g @ alpha)
        eps_s = eps_s + agb
        eps = eps + agb + bga
        alpha = alpha @ (g @ alpha)
        beta = beta @ (g @ beta)
        if norm1(alpha) + norm1(beta) < tol * ref:
            converged = True
            break
    return np.linalg.solve(z * eye - eps_s, eye), it, converged


def lead_selfenergy(h00, h01, tau, z, tol=1e-14, max_iter=100, variant=None):
    """Retarded lead self-energy Sigma = tau g_s tau^dagger (tau: device edge
    slab -> lead surface layer).  Returns (Sigma, iterations, converged).
    variant="alt" uses ``sancho_rubio_alt`` (reproducibility estimate only)."""
    sr = sancho_rubio_alt if variant == "alt" else sancho_rubio
    gs, it, conv = sr(h00, h01, z, tol, max_iter)
    return tau @ gs @ dag(tau), it, conv


def lead_lesser(sigma, f):
    """Sigma^< = i f Gamma with Gamma = i (Sigma - Sigma^dagger)."""
    gamma = 1j * (sigma - dag(sigma))
    return 1j * f * gamma


# ---------------------------------------------------------------------------
# RGF (Eqs. 1-2 solved block-tridiagonally) -- the plain recursions
# ---------------------------------------------------------------------------

def scat_matrix(s):
    """The b x b self-energy block of one slab from its stored form: an
    orbital diagonal [b], or atom blocks [b, opa] (row o holds the entries of o
    with the orbitals of its own atom: a block-diagonal matrix with opa x opa
    blocks on the diagonal)."""
    s = np.asarray(s)
    if s.ndim == 1:
        return np.diag(s)
    b, opa = s.shape
    M = np.zeros((b, b), dtype=np.complex128)
    for a0 in range(0, b, opa):
        M[a0:a0 + opa, a0:a0 + opa] = s[a0:a0 + opa]
    return M


def atom_blocks(X, opa):
    """[..., b, b] diagonal blocks -> their atom blocks [..., b, opa]."""
    X = np.asarray(X)
    b = X.shape[-1]
    out = np.zeros(X.shape[:-1] + (opa,), dtype=X.dtype)
    for a0 in range(0, b, opa):
        out[..., a0:a0 + opa, :] = X[..., a0:a0 + opa, a0:a0 + opa]
    return out


def _assemble(hd, z, sigL, sigR, v, scatR):
    N = len(hd)
    b = hd[0].shape[0]
    A = []
    for i in range(N):
        a = z * np.eye(b) - hd[i]
        if v is not None:
            a = a - np.diag(v[i])
        if scatR is not None:
            a = a - scat_matrix(scatR[i])
        A.append(a)
    A[0] = A[0] - sigL
    A[N - 1] = A[N - 1] - sigR
    return A


def _lesser_sources(N, b, sigL, sigR, fL, fR, scatL, eta, eta_fill):
    S = []
    for i in range(N):
        s = np.zeros((b, b), dtype=np.complex128)
        if scatL is not None:
            s = s + scat_matrix(scatL[i])
        if eta_fill is not None:
            s = s + 2j * eta * eta_fill * np.eye(b)
        S.append(s)
    S[0] = S[0] + lead_lesser(sigL, fL)
    S[N - 1] = S[N - 1] + lead_lesser(sigR, fR)
    return S


def _m3(a, b, c, right):
    """a b c, associated (a b) c, or a (b c) when ``right``."""
    return a @ (b @ c) if right else (a @ b) @ c


def rgf(hd, hu, E, eta, sigL, sigR, fL, fR, v=None, scatR=None, scatL=None,
        eta_fill=None, transmission=False, assoc_right=False, bond_mag=False, diag_only=False):
    """Diagonal blocks of G^R, G^<, G^> plus bond currents (and optionally the
    Caroli transmission) of one (sample, k, E) point by recursive Green's
    functions.

    hd[i] = H_ii, hu[i] = H_{i,i+1} (so H_{i+1,i} = hu[i]^dagger); v[i] is the
    onsite potential per orbital; scatR/scatL[i] the orbital-diagonal scattering
    self-energies of slab i.  z = E + i eta enters every diagonal block (the
    device eta acts as an extra, empty contact unless ``eta_fill`` gives its
    occupation).

    Forward (left-connected) sweep, i = 0..N-1:
        g_i   = (A_ii - H_{i,i-1} g_{i-1} H_{i-1,i})^-1
        g^<_i = g_i (S_i + H_{i,i-1} g^<_{i-1} H_{i-1,i}) g_i^dagger
    Backward sweep, i = N-2..0, with L = g_i H_{i,i+1}, P = L G_{i+1}:
        G_ii   = g_i + P H_{i+1,i} g_i
        G^<_ii = g^<_i + L G^<_{i+1} L^dagger + T - T^dagger,  T = P H_{i+1,i} g^<_i
        G^<_{i+1,i} = G_{i+1} H_{i+1,i} g^<_i + G^<_{i+1} L^dagger
        j_i = 2 Re Tr[H_{i,i+1} G^<_{i+1,i}]   (bond current, units e/h per spin)
    G^> = G^< + G^R - G^R^dagger (no separate greater-than recursion).
    Transmission: T = Tr[Gamma_R G_{N1} Gamma_L G_{N1}^dagger] with the left
    column chain G_{i,1} = g_i H_{i,i-1} G_{i-1,1}.
    Pinned by: dense inversion (``dense``), Landauer, eta-sink current identity,
    spectral identity, reciprocity, integer transmission of ordered strips.
    ``assoc_right`` associates every triple product the other way; it only serves
    the reproducibility estimate (two correct FP64 evaluations of one point).
    ``bond_mag`` also returns, per bond, the sum of magnitudes of the terms the
    bond trace adds, 2 Tr[|H_{i,i+1}| (|G_{i+1}| |H_{i+1,i}| |g^<_i| + |G^<_{i+1}| |L|^T)]
    (|X| elementwise): the scale on which any FP64 evaluation of the trace, in
    any order, rounds (test tolerances only; no result depends on it).
    ``diag_only`` returns GR, GL, GG as orbital diagonals [N, b] and lets each
    block go once the backward sweep has used it (the same arithmetic, less
    memory for long devices with large blocks)."""
    N = len(hd)
    ar = assoc_right
    b = hd[0].shape[0]
    z = E + 1j * eta
    A = _assemble(hd, z, sigL, sigR, v, scatR)
    S = _lesser_sources(N, b, sigL, sigR, fL, fR, scatL, eta, eta_fill)

    g = [None] * N
    gl = [None] * N
    g[0] = inv(A[0])
    gl[0] = _m3(g[0], S[0], dag(g[0]), ar)
    for i in range(1, N):
        hl = dag(hu[i - 1])            # H_{i,i-1}
        g[i] = inv(A[i] - _m3(hl, g[i - 1], hu[i - 1], ar))
        gl[i] = _m3(g[i], S[i] + _m3(hl, gl[i - 1], hu[i - 1], ar), dag(g[i]), ar)

    GR = [None] * N
    GL = [None] * N
    GR[N - 1] = g[N - 1]
    GL[N - 1] = gl[N - 1]
    bond = np.zeros(max(N - 1, 0))
    mag = np.zeros(max(N - 1, 0))
    for i in range(N - 2, -1, -1):
        hr = dag(hu[i])                # H_{i+1,i}
        L = g[i] @ hu[i]
        P = L @ GR[i + 1]
        GR[i] = g[i] + _m3(P, hr, g[i], ar)
        T = _m3(P, hr, gl[i], ar)
        GL[i] = gl[i] + _m3(L, GL[i + 1], dag(L), ar) + T - dag(T)
        gl_10 = _m3(GR[i + 1], hr, gl[i], ar) + GL[i + 1] @ dag(L)
        bond[i] = 2.0 * np.real(np.trace(hu[i] @ gl_10))
        if bond_mag:
            a = np.abs
            mag[i] = 2.0 * np.trace(a(hu[i]) @ (a(GR[i + 1]) @ a(hr) @ a(gl[i]) + a(GL[i + 1]) @ a(L).T))
        if diag_only and not transmission:
            GR[i + 1] = np.diagonal(GR[i + 1]).copy()
            GL[i + 1] = np.diagonal(GL[i + 1]).copy()
            g[i + 1] = gl[i + 1] = None
    if diag_only and not transmission:
        GR[0] = np.diagonal(GR[0]).copy()
        GL[0] = np.diagonal(GL[0]).copy()
        GR = np.array(GR)
        GL = np.array(GL)
        out = dict(GR=GR, GL=GL, GG=GL + GR - np.conj(GR), bond=bond)
        if bond_mag:
            out["bond_mag"] = mag
        return out
    GR = np.array(GR)
    GL = np.array(GL)
    GG = GL + GR - np.conj(np.transpose(GR, (0, 2, 1)))
    out = dict(GR=GR, GL=GL, GG=GG, bond=bond)
    if bond_mag:
        out["bond_mag"] = mag
    if transmission:
        col = g[0]
        for i in range(1, N):
            col = g[i] @ dag(hu[i - 1]) @ col
        gamL = 1j * (sigL - dag(sigL))
        gamR = 1j * (sigR - dag(sigR))
        out["T"] = float(np.real(np.trace(gamR @ col @ gamL @ dag(col))))
    return out


def dense(hd, hu, E, eta, sigL, sigR, fL, fR, v=None, scatR=None, scatL=None,
          eta_fill=None, full=False):
    """The plain definition: build the whole (N b)^2 matrix, invert it, form
    G^< = G^R Sigma^< G^R^dagger (Eqs. 1-2) and read off the blocks.  Same
    outputs as ``rgf``; for tiny systems only."""
    N = len(hd)
    b = hd[0].shape[0]
    n = N * b
    z = E + 1j * eta
    A = _assemble(hd, z, sigL, sigR, v, scatR)
    S = _lesser_sources(N, b, sigL, sigR, fL, fR, scatL, eta, eta_fill)
    M = np.zeros((n, n), dtype=np.complex128)
    Sl = np.zeros((n, n), dtype=np.complex128)
    for i in range(N):
        r = slice(i * b, (i + 1) * b)
        M[r, r] = A[i]
        Sl[r, r] = S[i]
        if i + 1 < N:
            r2 = slice((i + 1) * b, (i + 2) * b)
            M[r, r2] = -hu[i]
            M[r2, r] = -dag(hu[i])
    G = inv(M)
    Gl = G @ Sl @ dag(G)
    blk = lambda X, i, j: X[i * b:(i + 1) * b, j * b:(j + 1) * b]
    GR = np.array([blk(G, i, i) for i in range(N)])
    GL = np.array([blk(Gl, i, i) for i in range(N)])
    GG = GL + GR - np.conj(np.transpose(GR, (0, 2, 1)))
    bond = np.array([2.0 * np.real(np.trace(hu[i] @ blk(Gl, i + 1, i))) for i in range(N - 1)])
    gamL = 1j * (sigL - dag(sigL))
    gamR = 1j * (sigR - dag(sigR))
    GN1 = blk(G, N - 1, 0)
    T = float(np.real(np.trace(gamR @ GN1 @ gamL @ dag(GN1))))
    out = dict(GR=GR, GL=GL, GG=GG, bond=bond, T=T)
    if full:
        out["G"] = G
        out["Gl"] = Gl
    return out


# ---------------------------------------------------------------------------
# Scattering self-energies (Eqs. 4-6)
# ---------------------------------------------------------------------------

def scba_selfenergy(GRd, GLd, w_k, D_ac, M_op, shift, n_bose):
    """Orbital-diagonal scattering self-energies from the orbital diagonals of
    G^R and G^< on the full (k, E) grid.

    GRd, GLd: [n_k, n_e, N, b].  Returns (Sigma^R, Sigma^<), each [n_e, N, b]
    and independent of k.  The k' integral is the weighted average sum_k w_k.
      acoustic (Eq. 4):  Sigma^{R,<} = D_ac <G^{R,<}(E)>
      optical  (Eq. 5):  Sigma^<  = M [(1+n0) <G^<(E+hw)> + n0 <G^<(E-hw)>]
      optical  (Eq. 6):  Sigma^R  = M [(1+n0) <G^R(E-hw)> + n0 <G^R(E+hw)>
                                      + 1/2 <G^<(E-hw)> - 1/2 <G^<(E+hw)>]
    (principal-value part dropped, as the paper states).  The phonon energy hw
    is ``shift`` grid steps.  Where E-hw (E+hw) is off the grid the whole
    (E-hw) ((E+hw)) group is dropped from both Sigma^R and Sigma^<.
    Pinned by: equilibrium KMS identity at every SCBA iterate and elastic
    current conservation (acoustic only)."""
    avgR = np.tensordot(w_k, GRd, axes=(0, 0))
    avgL = np.tensordot(w_k, GLd, axes=(0, 0))
    sigR = D_ac * avgR
    sigL = D_ac * avgL
    n_e = avgR.shape[0]
    if M_op != 0.0 and shift > 0:
        sigR = sigR.copy()
        sigL = sigL.copy()
        for e in range(n_e):
            lo = e - shift
            hi = e + shift
            if lo >= 0:     # (E - hw) group
                sigL[e] += M_op * n_bose * avgL[lo]
                sigR[e] += M_op * ((1.0 + n_bose) * avgR[lo] + 0.5 * avgL[lo])
            if hi < n_e:    # (E + hw) group
                sigL[e] += M_op * (1.0 + n_bose) * avgL[hi]
                sigR[e] += M_op * (n_bose * avgR[hi] - 0.5 * avgL[hi])
    return sigR, sigL


# ---------------------------------------------------------------------------
# Drivers over many points
# ---------------------------------------------------------------------------

def cap_selfenergy(wl):
    """Contact self-energies of a workload whose contacts are complex
    absorbing potentials (the paper's treatment of random-alloy leads, in the
    paragraph after Eq. 6, whose form it does not give; reading: an imaginary
    onsite potential -i W on every orbital of a contact slab, and the
    reservoir injection that the fluctuation-dissipation relation pairs with
    it, Sigma^< = -(Sigma^R - Sigma^A) f = 2 i W f(E; mu of that contact)).
    Returns (Sigma^R, Sigma^<), each [n_e, total_slabs, nb], orbital-diagonal.
    Pinned by: ordered devices reproduce the Sancho-Rubio transmission, and
    the equilibrium (KMS) identity."""
    W = np.asarray(wl.cap_w, dtype=np.float64)
    side = np.asarray(wl.cap_side)
    sR = np.zeros((wl.n_e, wl.total_slabs, wl.nb), dtype=np.complex128)
    sL = np.zeros_like(sR)
    for ie, E in enumerate(wl.energy):
        fL = float(fermi(E, wl.mu_L, wl.kT))
        fR = float(fermi(E, wl.mu_R, wl.kT))
        for i in range(wl.total_slabs):
            if W[i] == 0.0:
                continue
            f = fL if side[i] < 0 else fR
            sR[ie, i, :] = -1j * W[i]
            sL[ie, i, :] = 2j * W[i] * f
    return sR, sL


def lead_tables(wl, tol=1e-14, max_iter=100, ks=None, es=None, variant=None):
    """Sigma_L, Sigma_R for the (k, E) grid (or the listed subsets).  Zero
    for a workload with absorbing-potential contacts (no semi-infinite leads)."""
    ks = range(wl.n_k) if ks is None else ks
    es = range(wl.n_e) if es is None else es
    out = {}
    if getattr(wl, "cap_w", None) is not None:
        z0 = np.zeros((wl.nb, wl.nb), dtype=np.complex128)
        return {(ik, ie): (z0, z0, 0, 0) for ik in ks for ie in es}
    for ik in ks:
        for ie in es:
            z = wl.energy[ie] + 1j * wl.eta
            sL, itL, cL = lead_selfenergy(wl.lead_h00[ik], wl.lead_h01_L, wl.lead_tau_L, z, tol, max_iter, variant)
            sR, itR, cR = lead_selfenergy(wl.lead_h00[ik], wl.lead_h01_R, wl.lead_tau_R, z, tol, max_iter, variant)
            out[(ik, ie)] = (sL, sR, itL, itR)
    return out


def solve_points(wl, points, leads=None, scatR=None, scatL=None, transmission=False, eta_fill=None,
                 variant=None, bond_mag=False, diag_only=False):
    """RGF for a list of (sample, ik, ie) points.  scatR/scatL: [n_e, total_slabs, b].
    variant="alt": the reproducibility estimate, with the lead decimation and every
    triple product of the recursion associated the other way."""
    if leads is None:
        leads = lead_tables(wl, ks=sorted({int(p[1]) for p in points}),
                            es=sorted({int(p[2]) for p in points}), variant=variant)
    if getattr(wl, "cap_w", None) is not None:       # absorbing contacts enter as self-energies
        cR, cL = cap_selfenergy(wl)
        scatR = cR if scatR is None else scatR + cR
        scatL = cL if scatL is None else scatL + cL
    res = []
    for s, ik, ie in points:
        hd, hu, v = wl.sample_blocks(int(s), int(ik))
        a0, a1 = int(wl.slab_offset[s]), int(wl.slab_offset[s + 1])
        E = float(wl.energy[ie])
        sL, sR = leads[(int(ik), int(ie))][:2]
        fL = float(fermi(E, wl.mu_L, wl.kT))
        fR = float(fermi(E, wl.mu_R, wl.kT))
        sr = None if scatR is None else scatR[ie, a0:a1]
        sl = None if scatL is None else scatL[ie, a0:a1]
        ef = None if eta_fill is None else float(fermi(E, eta_fill, wl.kT))
        res.append(rgf(hd, hu, E, wl.eta, sL, sR, fL, fR, v=v, scatR=sr, scatL=sl,
                       transmission=transmission, eta_fill=ef, assoc_right=(variant == "alt"),
                       bond_mag=bond_mag, diag_only=diag_only))
    return res


def scba(wl, n_iter, leads=None, eta_fill=None, tol=None, atom_block_sigma=False):
    """Self-consistent Born loop (Eqs. 1-6) for a single-sample workload.

    Sigma_scat starts at zero (ballistic first pass); each iteration solves all
    (k, E) points with the current Sigma_scat, then rebuilds Sigma_scat from the
    orbital diagonals (no mixing) -- or, with ``atom_block_sigma``, from the atom
    blocks (orbs_per_atom x orbs_per_atom) of the diagonal blocks, the other
    reading of "diag G" in Eqs. (4)-(6): Sigma_scat is then block-diagonal
    with one block per atom, each entry given by the same formulas.  Runs
    ``n_iter`` iterations, or stops early once ||dSigma|| / ||Sigma|| < tol
    when ``tol`` is given.  Returns the last solution's diagonals (or atom
    blocks) and the residual history."""
    assert wl.n_samples == 1
    N, b = wl.total_slabs, wl.nb
    if leads is None:
        leads = lead_tables(wl)
    pts = [(0, ik, ie) for ik in range(wl.n_k) for ie in range(wl.n_e)]
    tail = (b, wl.orbs_per_atom) if atom_block_sigma else (b,)
    scatR = np.zeros((wl.n_e, N) + tail, dtype=np.complex128)
    scatL = np.zeros((wl.n_e, N) + tail, dtype=np.complex128)
    if atom_block_sigma:
        pick = lambda X: atom_blocks(X, wl.orbs_per_atom)
    else:
        pick = lambda X: np.diagonal(X, axis1=1, axis2=2)
    hist = []
    for _ in range(n_iter):
        res = solve_points(wl, pts, leads, scatR, scatL, eta_fill=eta_fill)
        GRd = np.array([pick(r["GR"]) for r in res]).reshape((wl.n_k, wl.n_e, N) + tail)
        GLd = np.array([pick(r["GL"]) for r in res]).reshape((wl.n_k, wl.n_e, N) + tail)
        newR, newL = scba_selfenergy(GRd, GLd, wl.w_k, wl.D_ac, wl.M_op, wl.shift, wl.n_bose)
        num = np.linalg.norm(newR - scatR) ** 2 + np.linalg.norm(newL - scatL) ** 2
        den = np.linalg.norm(newR) ** 2 + np.linalg.norm(newL) ** 2
        hist.append(float(np.sqrt(num / den)) if den > 0 else 0.0)
        scatR, scatL = newR, newL
        last = dict(res=res, GRd=GRd, GLd=GLd)
        if tol is not None and hist[-1] < tol:
            break
    return dict(sigR=scatR, sigL=scatL, hist=hist, **last)


# ---------------------------------------------------------------------------
# Observables (Eqs. 7-8)
# ---------------------------------------------------------------------------

def observables(wl, points, GLd, bond, g_s=None):
    """Density per atom and bond current per sample (deterministic sums).

    n_a = g_s sum_E w_E sum_k w_k (1/2pi) sum_{o in a} Im G^<_oo      (Eq. 7)
    J_i = g_s sum_E w_E sum_k w_k j_i(E, k)   (units e/h)           (Eq. 8)
    j_E[e, i] = g_s sum_k w_k j_i(E_e, k)     (spectral current)
    GLd: [n_points, N_p, b] orbital diagonal of G^<; bond: [n_points, N_p - 1].
    Returns (n [total_slabs, atoms], J [total_slabs], jE [n_samples, n_e, max_N])
    with J / jE zero beyond each sample's last bond.
    The prefactors are readings of Eqs. (7)-(8) (parity unpinned beyond them)."""
    g_s = wl.g_s if g_s is None else g_s
    nat = wl.atoms_per_slab
    opa = wl.orbs_per_atom
    n = np.zeros((wl.total_slabs, nat))
    J = np.zeros(wl.total_slabs)
    maxN = int(np.max(np.diff(wl.slab_offset)))
    jE = np.zeros((wl.n_samples, wl.n_e, maxN))
    for p, (s, ik, ie) in enumerate(points):
        a0, a1 = int(wl.slab_offset[s]), int(wl.slab_offset[s + 1])
        Np = a1 - a0
        w = g_s * wl.w_e[ie] * wl.w_k[ik]
        im = np.imag(np.asarray(GLd[p])[:Np]).reshape(Np, nat, opa).sum(axis=2)
        n[a0:a1] += w * im / (2 * np.pi)
        J[a0:a1 - 1] += w * np.asarray(bond[p])[:Np - 1]
        jE[s, ie, :Np - 1] += g_s * wl.w_k[ik] * np.asarray(bond[p])[:Np - 1]
    return n, J, jE


# ---------------------------------------------------------------------------
# Differentiation: VJP of the density with respect to the onsite potential
# ---------------------------------------------------------------------------

def _cap_terms(wl, ie, a0, a1, scatR=None, scatL=None):
    """The diagonal self-energies of the slabs [a0, a1) at energy ie: the given
    scattering ones [n_e, total_slabs, b] plus the absorbing contacts', or None."""
    R = None if scatR is None else scatR[ie, a0:a1]
    L = None if scatL is None else scatL[ie, a0:a1]
    if getattr(wl, "cap_w", None) is not None:
        cR, cL = cap_selfenergy(wl)
        R = cR[ie, a0:a1] if R is None else R + cR[ie, a0:a1]
        L = cL[ie, a0:a1] if L is None else L + cL[ie, a0:a1]
    return R, L


def density_objective(wl, w_atom, v_orb, points, leads, scatR=None, scatL=None):
    """f(V) = sum_a w_a n_a(V) for the given onsite potential (per orbital),
    with fixed scattering self-energies if given."""
    nat, opa = wl.atoms_per_slab, wl.orbs_per_atom
    f = 0.0
    for s, ik, ie in points:
        a0, a1 = int(wl.slab_offset[s]), int(wl.slab_offset[s + 1])
        hd, hu, _ = wl.sample_blocks(int(s), int(ik))
        E = float(wl.energy[ie])
        sL, sR = leads[(int(ik), int(ie))][:2]
        scR, scL = _cap_terms(wl, ie, a0, a1, scatR, scatL)
        r = rgf(hd, hu, E, wl.eta, sL, sR, float(fermi(E, wl.mu_L, wl.kT)),
                float(fermi(E, wl.mu_R, wl.kT)), v=[v_orb[i] for i in range(a0, a1)], scatR=scR, scatL=scL)
        im = np.imag(np.diagonal(r["GL"], axis1=1, axis2=2)).reshape(a1 - a0, nat, opa).sum(axis=2)
        f += wl.g_s * wl.w_e[ie] * wl.w_k[ik] / (2 * np.pi) * float(np.sum(w_atom[a0:a1] * im))
    return f


def dense_grad(wl, w_atom, v_orb, points, leads, scatR=None, scatL=None):
    """Gradient of f(V) = sum_a w_a n_a with respect to the per-atom potential.

    From dG^R = G^R dV G^R and dG^< = G^R dV G^< + G^< dV G^A:
      df/dV_o = sum_points c_p 2 Im[(G^< W G^R)_oo],  c_p = g_s w_E w_k / 2pi,
    W = diag(w) expanded to orbitals; summed over the orbitals of each atom.
    Dense inversion; tiny systems only.  Pinned by: central finite differences
    of ``density_objective``."""
    nat, opa, b = wl.atoms_per_slab, wl.orbs_per_atom, wl.nb
    grad = np.zeros((wl.total_slabs, nat))
    for s, ik, ie in points:
        a0, a1 = int(wl.slab_offset[s]), int(wl.slab_offset[s + 1])
        Np = a1 - a0
        hd, hu, _ = wl.sample_blocks(int(s), int(ik))
        E = float(wl.energy[ie])
        sL, sR = leads[(int(ik), int(ie))][:2]
        scR, scL = _cap_terms(wl, ie, a0, a1, scatR, scatL)
        r = dense(hd, hu, E, wl.eta, sL, sR, float(fermi(E, wl.mu_L, wl.kT)),
                  float(fermi(E, wl.mu_R, wl.kT)), v=[v_orb[i] for i in range(a0, a1)], scatR=scR, scatL=scL,
                  full=True)
        wdiag = np.repeat(np.asarray(w_atom[a0:a1]).reshape(-1), opa)
        X = r["Gl"] @ (wdiag[:, None] * r["G"])
        c = wl.g_s * wl.w_e[ie] * wl.w_k[ik] / (2 * np.pi)
        d = 2.0 * c * np.imag(np.diagonal(X))
        grad[a0:a1] += d.reshape(Np, nat, opa).sum(axis=2)
    return grad
