"""Pins of the CPU oracle against what mathematics and the paper fix.

Each test ties one oracle function to something other than itself: the plain
dense definition of Eqs. (1)-(2), closed forms of simple leads, Landauer
transmission of ordered strips, exact identities (spectral, eta-sink current,
equilibrium detailed balance, elastic current conservation), reciprocity,
finite differences, and the paper's printed sizes.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from synth import make_workload, random_tiny, strip_workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _leads(wl, ik, E, **kw):
    z = E + 1j * wl.eta
    sL, itL, cL = O.lead_selfenergy(wl.lead_h00[ik], wl.lead_h01_L, wl.lead_tau_L, z, **kw)
    sR, itR, cR = O.lead_selfenergy(wl.lead_h00[ik], wl.lead_h01_R, wl.lead_tau_R, z, **kw)
    assert cL and cR
    return sL, sR


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


# --------------------------------------------------------------------------
# RGF vs the plain dense definition (Eqs. 1-2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nb,N,up,seed", [(1, 1, None, 0), (3, 1, None, 1), (5, 2, None, 2),
                                          (6, 5, None, 3), (8, 4, 2, 4), (12, 6, 4, 5)])
def test_rgf_matches_dense_inversion(nb, N, up, seed):
    wl = random_tiny(nb, N, n_e=3, seed=seed, up_block=up, eta=1e-3)
    rng = np.random.default_rng(seed)
    hd, hu, _ = wl.sample_blocks(0, 0)
    v = [rng.uniform(0, 0.3, nb) for _ in range(N)]
    scatR = [rng.normal(size=nb) * 0.02 - 0.02j * rng.uniform(size=nb) for _ in range(N)]
    scatL = [0.03j * rng.uniform(size=nb) for _ in range(N)]
    for E in wl.energy:
        sL, sR = _leads(wl, 0, E)
        r = O.rgf(hd, hu, E, wl.eta, sL, sR, 0.8, 0.3, v=v, scatR=scatR, scatL=scatL, transmission=True)
        d = O.dense(hd, hu, E, wl.eta, sL, sR, 0.8, 0.3, v=v, scatR=scatR, scatL=scatL)
        for key in ("GR", "GL", "GG"):
            assert _rel(r[key], d[key]) < 1e-12, key
        if N > 1:
            assert _rel(r["bond"], d["bond"]) < 1e-11
        assert abs(r["T"] - d["T"]) <= 1e-12 * max(1.0, abs(d["T"]))


def test_rgf_matches_dense_on_strip_workload():
    wl = make_workload("C1", n_e=32)
    hd, hu, _ = wl.sample_blocks(0, 0)
    for E in wl.energy[::3]:
        sL, sR = _leads(wl, 0, E)
        fL, fR = O.fermi(E, wl.mu_L, wl.kT), O.fermi(E, wl.mu_R, wl.kT)
        r = O.rgf(hd, hu, E, wl.eta, sL, sR, fL, fR, transmission=True)
        d = O.dense(hd, hu, E, wl.eta, sL, sR, fL, fR)
        assert _rel(r["GR"], d["GR"]) < 1e-10
        assert abs(r["T"] - d["T"]) < 1e-9


# --------------------------------------------------------------------------
# Sancho-Rubio vs closed forms
# --------------------------------------------------------------------------

def _chain_sigma(x, t):
    """Self-energy t^2 g_s of a semi-infinite 1-D chain: (x - sqrt(x^2-4t^2))/2,
    the root with |sigma| < |t| (decaying / retarded branch)."""
    s = np.sqrt(x * x - 4 * t * t + 0j)
    r1, r2 = (x - s) / 2, (x + s) / 2
    return r1 if abs(r1) < abs(r2) else r2


@pytest.mark.parametrize("E", [-2.7, -1.3, -0.2, 0.0, 0.9, 1.99 - 0.5, 2.6])
def test_sancho_rubio_1d_chain_closed_form(E):
    t, eps, eta = -1.0, 0.1, 1e-6
    z = E + 1j * eta
    h = np.array([[eps]], dtype=complex)
    sig, it, conv = O.lead_selfenergy(h, np.array([[t]], dtype=complex), np.array([[t]], dtype=complex), z)
    assert conv
    ref = _chain_sigma(z - eps, t)
    assert abs(sig[0, 0] - ref) < 1e-10 * max(1, abs(ref))
    assert sig[0, 0].imag <= 0


def test_sancho_rubio_strip_closed_form():
    W, t, eta = 8, -1.0, 1e-6
    wl = strip_workload(width=W, disorder=0.0, eta=eta)
    m = np.arange(1, W + 1)
    eps_m = 2 * t * np.cos(m * np.pi / (W + 1))
    U = np.sqrt(2.0 / (W + 1)) * np.sin(np.outer(np.arange(1, W + 1), m) * np.pi / (W + 1))
    for E in np.linspace(-3.9, 3.9, 23):
        if np.min(np.abs(np.abs(E - eps_m) - 2)) < 1e-3:
            continue
        z = E + 1j * eta
        sL, sR = _leads(wl, 0, E)
        ref = U @ np.diag([_chain_sigma(z - e, t) for e in eps_m]) @ U.T
        assert np.max(np.abs(sL - ref)) < 1e-10
        assert np.max(np.abs(sR - ref)) < 1e-10


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sancho_rubio_surface_dyson_fixed_point(seed):
    wl = random_tiny(6, 2, n_e=3, seed=seed, eta=1e-4)
    for E in wl.energy:
        z = E + 1j * wl.eta
        for h01 in (wl.lead_h01_L, wl.lead_h01_R):
            gs, it, conv = O.sancho_rubio(wl.lead_h00[0], h01, z)
            assert conv
            rhs = np.linalg.inv(z * np.eye(6) - wl.lead_h00[0] - h01 @ gs @ h01.conj().T)
            assert np.max(np.abs(gs - rhs)) < 1e-8 * np.max(np.abs(gs))  # conditioning ~ 1/eta
            sig = wl.lead_tau_L @ gs @ wl.lead_tau_L.conj().T
            gam = 1j * (sig - sig.conj().T)
            assert np.min(np.linalg.eigvalsh(gam)) > -1e-10


def test_sancho_rubio_flags_iteration_cap():
    wl = random_tiny(4, 2, n_e=1, seed=3, eta=1e-6)
    _, it, conv = O.sancho_rubio(wl.lead_h00[0], wl.lead_h01_R, wl.energy[0] + 1e-6j, max_iter=1)
    assert it == 1 and not conv


# --------------------------------------------------------------------------
# Transmission: integer steps of ordered strips (Landauer)
# --------------------------------------------------------------------------

def test_ordered_strip_integer_transmission():
    W, t = 8, -1.0
    # eta -> 0 limit: the O(eta N / v) absorption of the device eta is < 1e-6 here
    wl = strip_workload(width=W, disorder=0.0, n_slab=20, eta=1e-9)
    hd, hu, _ = wl.sample_blocks(0, 0)
    eps_m = 2 * t * np.cos(np.arange(1, W + 1) * np.pi / (W + 1))
    checked = 0
    for E in wl.energy:
        dist = np.min(np.abs(np.abs(E - eps_m) - 2 * abs(t)))
        if dist < 0.05:
            continue
        sL, sR = _leads(wl, 0, E, max_iter=200)
        r = O.rgf(hd, hu, E, wl.eta, sL, sR, 1.0, 0.0, transmission=True)
        n_open = int(np.sum(np.abs(E - eps_m) < 2 * abs(t)))
        assert abs(r["T"] - n_open) < 1e-5, (E, r["T"], n_open)
        checked += 1
    assert checked > 150


def test_bond_current_equals_landauer():
    """Ballistic, eta -> 0: every bond current equals T (f_L - f_R)."""
    wl = random_tiny(4, 6, n_e=3, seed=2, eta=1e-9)
    hd, hu, _ = wl.sample_blocks(0, 0)
    for E in wl.energy:
        sL, sR = _leads(wl, 0, E, max_iter=200)
        r = O.rgf(hd, hu, E, wl.eta, sL, sR, 0.9, 0.2, transmission=True)
        assert np.max(np.abs(r["bond"] - r["T"] * 0.7)) < 1e-6 * max(r["T"], 1e-3)


def test_eta_sink_current_identity():
    """Exact at any eta: j_{i-1} - j_i = 2 eta Tr(-i G^<_ii) (current lost into the
    eta contact of slab i)."""
    wl = random_tiny(5, 7, n_e=3, seed=6, eta=2e-2)
    hd, hu, _ = wl.sample_blocks(0, 0)
    for E in wl.energy:
        sL, sR = _leads(wl, 0, E)
        r = O.rgf(hd, hu, E, wl.eta, sL, sR, 0.95, 0.1)
        j = r["bond"]
        for i in range(1, 6):
            sink = 2 * wl.eta * np.real(np.trace(-1j * r["GL"][i]))
            assert abs((j[i - 1] - j[i]) - sink) < 1e-12 * max(1, np.max(np.abs(j)))


def test_spectral_identity_via_lesser_recursion():
    """With every contact filled (f = 1, including eta and scattering),
    Sigma^< = i Gamma_total and the lesser recursion must return
    G^< = i A = -(G - G^dagger) blockwise, i.e. G^> = 0."""
    wl = random_tiny(6, 5, n_e=3, seed=7, eta=1e-3)
    rng = np.random.default_rng(7)
    hd, hu, _ = wl.sample_blocks(0, 0)
    scatR = [rng.normal(size=6) * 0.02 - 0.05j * rng.uniform(size=6) for _ in range(5)]
    scatL = [-2j * np.imag(s) for s in scatR]     # i * Gamma_scat, Gamma = -2 Im Sigma^R
    for E in wl.energy:
        sL, sR = _leads(wl, 0, E)
        r = O.rgf(hd, hu, E, wl.eta, sL, sR, 1.0, 1.0, scatR=scatR, scatL=scatL, eta_fill=1.0)
        A = -(r["GR"] - np.conj(np.transpose(r["GR"], (0, 2, 1))))
        assert _rel(r["GL"], A) < 1e-12
        assert np.max(np.abs(r["GG"])) < 1e-11 * np.max(np.abs(r["GR"]))


def test_reciprocity_k_minus_k():
    """Real-symmetric couplings, no magnetic field: G(-k) = G(k)^T blockwise;
    at k = 0 and k = pi, G = G^T."""
    wl = make_workload("C2", n_slab=3, n_e=2, n_k=4, n_z=2, n_y=2)
    pts = [(0, ik, ie) for ik in range(4) for ie in range(2)]
    res = O.solve_points(wl, pts)
    R = {(p[1], p[2]): r for p, r in zip(pts, res)}
    for ie in range(2):
        for k, mk in ((1, 3), (0, 0), (2, 2)):
            a = R[(k, ie)]["GR"]
            b = np.transpose(R[(mk, ie)]["GR"], (0, 2, 1))
            assert _rel(a, b) < 1e-10


# --------------------------------------------------------------------------
# Scattering self-energies (Eqs. 4-6) and SCBA
# --------------------------------------------------------------------------

def _tiny_scba_workload(seed, n_e, shift, D, M, n_k=2):
    wl = random_tiny(4, 4, n_e=n_e, seed=seed, eta=1e-3, complex_h=False, n_k=n_k)
    wl.energy = np.linspace(-1.0, 1.0, n_e)
    wl.w_e = np.full(n_e, wl.energy[1] - wl.energy[0])
    # k-dependent device and lead blocks, still Hermitian
    rng = np.random.default_rng(seed + 100)
    y = rng.normal(size=(4, 4)) * 0.1
    for ik, k in enumerate(2 * np.pi * np.arange(n_k) / n_k):
        wl.h_diag[ik] = wl.h_diag[0].real + np.exp(1j * k) * y + np.exp(-1j * k) * y.T
        wl.lead_h00[ik] = wl.lead_h00[0].real + np.exp(1j * k) * y + np.exp(-1j * k) * y.T
    wl.kpts = 2 * np.pi * np.arange(n_k) / n_k
    wl.D_ac, wl.M_op, wl.shift = D, M, shift
    wl.kT = 0.05
    wl.n_bose = 1.0 / np.expm1(shift * (wl.energy[1] - wl.energy[0]) / wl.kT) if shift else 0.0
    return wl


def test_kms_equilibrium_every_scba_iterate():
    """mu_L = mu_R, lead T = phonon T, eta contact filled: G^< = -f (G^R - G^A)
    holds at every SCBA iterate (detailed balance of each +-hw group, including
    the groups dropped at the grid ends)."""
    wl = _tiny_scba_workload(seed=11, n_e=9, shift=2, D=0.05, M=0.08)
    wl.mu_L = wl.mu_R = 0.1
    leads = O.lead_tables(wl)
    pts = [(0, ik, ie) for ik in range(wl.n_k) for ie in range(wl.n_e)]
    scatR = np.zeros((wl.n_e, 4, 4), dtype=complex)
    scatL = np.zeros_like(scatR)
    for it in range(4):
        res = O.solve_points(wl, pts, leads, scatR, scatL, eta_fill=wl.mu_L)
        for (s, ik, ie), r in zip(pts, res):
            f = O.fermi(wl.energy[ie], wl.mu_L, wl.kT)
            A = r["GR"] - np.conj(np.transpose(r["GR"], (0, 2, 1)))
            # roundoff scales with |A| (not with f |A|, which is tiny above mu)
            assert np.max(np.abs(r["GL"] + f * A)) < 1e-10 * np.max(np.abs(A)), (it, ik, ie)
        GRd = np.array([np.diagonal(r["GR"], axis1=1, axis2=2) for r in res]).reshape(wl.n_k, wl.n_e, 4, 4)
        GLd = np.array([np.diagonal(r["GL"], axis1=1, axis2=2) for r in res]).reshape(wl.n_k, wl.n_e, 4, 4)
        scatR, scatL = O.scba_selfenergy(GRd, GLd, wl.w_k, wl.D_ac, wl.M_op, wl.shift, wl.n_bose)
        assert np.max(np.abs(scatL)) > 0


def test_optical_selfenergy_detailed_balance_identity():
    """Per group, f(E) (1 + n0 - f(E - hw)) = n0 f(E - hw) (and its +hw mirror)."""
    kT, hw = 0.025852, 0.06
    n0 = 1.0 / np.expm1(hw / kT)
    for E in np.linspace(-0.3, 0.3, 13):
        f, fm, fp = (O.fermi(x, 0.0, kT) for x in (E, E - hw, E + hw))
        assert abs(f * (1 + n0 - fm) - n0 * fm) < 1e-15
        assert abs(f * (n0 + fp) - (1 + n0) * fp) < 1e-15


def test_elastic_scattering_conserves_current():
    """Acoustic (elastic, local) scattering at SCBA convergence: per energy the
    k-summed current divergence equals only the eta-sink loss."""
    # Undamped SCBA is a contraction only when D |G| is small; eta = 0.05 keeps it so.
    wl = _tiny_scba_workload(seed=12, n_e=3, shift=0, D=0.05, M=0.0)
    wl.eta = 0.05
    wl.mu_L, wl.mu_R = 0.3, -0.3
    out = O.scba(wl, 200, eta_fill=None, tol=1e-13)
    assert out["hist"][-1] < 1e-12
    res = out["res"]
    for ie in range(wl.n_e):
        div = np.zeros(2)
        for ik in range(wl.n_k):
            r = res[ik * wl.n_e + ie]
            j = r["bond"]
            for i in range(1, 3):       # interior slabs of the 4-slab device
                sink = 2 * wl.eta * np.real(np.trace(-1j * r["GL"][i]))
                div[i - 1] += wl.w_k[ik] * ((j[i - 1] - j[i]) - sink)
        jmax = max(abs(res[ik * wl.n_e + ie]["bond"]).max() for ik in range(wl.n_k))
        assert np.max(np.abs(div)) < 1e-10 * max(jmax, 1e-12)


def test_scattering_changes_current():
    """The paper's Fig. 2 claim in its weakest form: phonon scattering changes
    the current relative to the ballistic solution."""
    wl = _tiny_scba_workload(seed=13, n_e=7, shift=2, D=0.05, M=0.05)
    out = O.scba(wl, 3)
    b0 = O.solve_points(wl, [(0, 0, 3)])[0]["bond"]
    b1 = out["res"][3]["bond"]
    assert np.max(np.abs(b1 - b0)) > 1e-6 * np.max(np.abs(b0))


# --------------------------------------------------------------------------
# Observables (Eqs. 7-8)
# --------------------------------------------------------------------------

def test_density_sum_rule():
    """With every contact filled, Im G^< = A and sum_E w_E A_oo / 2pi -> 1 per
    orbital: the total density is g_s x (number of orbitals), up to the
    Lorentzian tails outside the energy window."""
    wl = random_tiny(3, 3, n_e=1, seed=21, eta=0.02)
    E = np.arange(-12.0, 12.0, 0.004)
    hd, hu, _ = wl.sample_blocks(0, 0)
    tot = np.zeros((3, 3))
    for e in E:
        sL, sR = _leads(wl, 0, e)
        r = O.rgf(hd, hu, e, wl.eta, sL, sR, 1.0, 1.0, eta_fill=1.0)
        tot += np.imag(np.diagonal(r["GL"], axis1=1, axis2=2))
    wl.energy = np.array([0.0])
    wl.w_e = np.array([0.004])
    n, _, _ = O.observables(wl, [(0, 0, 0)], [1j * tot],
                            [np.zeros(2)], g_s=2.0)
    assert abs(n.sum() - 2.0 * 9) < 2.0 * 9 * 2e-3


def test_current_observable_matches_landauer_integral():
    wl = random_tiny(4, 5, n_e=6, seed=22, eta=1e-9)
    wl.mu_L, wl.mu_R = 0.5, -0.5
    pts = [(0, 0, ie) for ie in range(wl.n_e)]
    leads = O.lead_tables(wl, max_iter=200)
    res = O.solve_points(wl, pts, leads, transmission=True)
    GLd = [np.diagonal(r["GL"], axis1=1, axis2=2) for r in res]
    n, J, jE = O.observables(wl, pts, GLd, [r["bond"] for r in res])
    ref = sum(wl.g_s * wl.w_e[ie] * r["T"] * (O.fermi(wl.energy[ie], 0.5, wl.kT) - O.fermi(wl.energy[ie], -0.5, wl.kT))
              for ie, r in enumerate(res))
    assert np.max(np.abs(J[:4] - ref)) < 1e-6 * abs(ref)


# --------------------------------------------------------------------------
# Differentiation: dense VJP vs finite differences
# --------------------------------------------------------------------------

def test_dense_grad_matches_finite_differences():
    wl = make_workload("C5", n_slab=4, n_e=2, n_z=1, n_y=2)
    wl.eta = 1e-3
    pts = [(0, 0, ie) for ie in range(wl.n_e)]
    leads = O.lead_tables(wl)
    rng = np.random.default_rng(5)
    w = rng.normal(size=(wl.total_slabs, wl.atoms_per_slab))
    v = wl.v_onsite.copy()
    g = O.dense_grad(wl, w, v, pts, leads)
    h = 1e-5
    for (s, a) in [(0, 0), (1, 1), (3, 0), (2, 1)]:
        vp, vm = v.copy(), v.copy()
        vp[s, a * 10:(a + 1) * 10] += h
        vm[s, a * 10:(a + 1) * 10] -= h
        fd = (O.density_objective(wl, w, vp, pts, leads) - O.density_objective(wl, w, vm, pts, leads)) / (2 * h)
        assert abs(fd - g[s, a]) < 1e-6 * np.max(np.abs(g)) + 1e-12


# --------------------------------------------------------------------------
# The paper's printed sizes
# --------------------------------------------------------------------------

def test_memory_model_matches_paper():
    """One stored set of 200 diagonal blocks of 1200^2 complex doubles is the
    paper's ~4.5 GB per (E,k) tuple; 24000 atoms x 10 orbitals = rank 240000."""
    with open(os.path.join(GOLDEN, "paper_sizes.json")) as fh:
        g = json.load(fh)
    n_slab = g["atoms"] // (g["block_rows_6x10"] // g["orbitals_per_atom"])
    assert n_slab == 200
    assert g["atoms"] * g["orbitals_per_atom"] == g["matrix_rank"]
    gb = n_slab * g["block_rows_6x10"] ** 2 * 16 / 1e9
    assert abs(gb - g["memory_per_ek_tuple_GB_6x10"]) / g["memory_per_ek_tuple_GB_6x10"] < 0.03
    wl_b = 12 * 10 * 10
    assert wl_b == g["block_rows_6x10"]


@pytest.mark.parametrize("E", [-2.7, -0.2, 0.9, 2.6])
def test_sancho_rubio_alternate_association_closed_form(E):
    """The reproducibility variant is the same method: it meets the closed form too."""
    t, eps, eta = -1.0, 0.1, 1e-6
    z = E + 1j * eta
    sig, it, conv = O.lead_selfenergy(np.array([[eps]], dtype=complex), np.array([[t]], dtype=complex),
                                      np.array([[t]], dtype=complex), z, variant="alt")
    assert conv
    ref = _chain_sigma(z - eps, t)
    assert abs(sig[0, 0] - ref) < 1e-10 * max(1, abs(ref))


# --------------------------------------------------------------------------
# Lead-coupling orientation with non-symmetric couplings (Eq. 3, Sigma_lead)
# --------------------------------------------------------------------------

def _bands(h00, h01, n_kx=8001):
    """Bulk bands E_n(kx) of an ordered lead, H(kx) = h00 + h01 e^{ikx} + h01^dagger e^{-ikx},
    on a closed kx grid over one period, each row sorted."""
    ks = np.linspace(0.0, 2 * np.pi, n_kx)
    return np.array([np.linalg.eigvalsh(h00 + h01 * np.exp(1j * k) + h01.conj().T * np.exp(-1j * k)) for k in ks])


def _open_channels(bands, E):
    """Number of right-moving Bloch states at E: upward crossings of E by the
    bands over one period (brute force on the kx grid)."""
    d = bands - E
    return int(np.sum((d[:-1] < 0) & (d[1:] >= 0)))


def _band_edges(bands):
    """Every extremum of every band (where the channel count changes)."""
    out = []
    for n in range(bands.shape[1]):
        b = bands[:, n]
        turn = np.where(np.diff(np.sign(np.diff(b))) != 0)[0] + 1
        out.extend(list(b[turn]) + [b.min(), b.max()])
    return np.array(out)


@pytest.mark.parametrize("ik", [0, 1])
def test_ordered_cross_section_integer_transmission_nonsymmetric_couplings(ik):
    """An ordered pure-Si cross-section (the device continues its leads) is a
    perfect conductor: T(E) equals the number of open bulk channels, counted
    here by brute force from the bulk bands.  The atom couplings are not
    symmetric (h01 != h01^T) and h00 is complex at k != 0, so this pins the
    orientation of Sigma = tau g_s tau^dagger, which lead layer h01 points to,
    and the left lead's h01 direction: a transposed or swapped coupling gives
    non-integer T (checked below by planting that mistake)."""
    from synth.workloads import cross_section_workload
    wl = cross_section_workload("ordered", 2, 1, [3], 4, np.zeros(1), 1510046862, ge_fraction=0.0, eta=1e-9)
    assert np.abs(wl.lead_h01_R - wl.lead_h01_R.T).max() > 0.1   # genuinely non-symmetric
    h00 = wl.lead_h00[ik]
    bands = _bands(h00, wl.lead_h01_R)
    edges = _band_edges(bands)
    grid = np.arange(-2.0, 2.0, 0.01)
    pick = [E for E in grid if _open_channels(bands, E) >= 1 and np.min(np.abs(edges - E)) >= 0.03]
    assert len(pick) >= 2
    pick = pick[:: max(1, len(pick) // 6)]
    hd, hu, _ = wl.sample_blocks(0, ik)
    swapped_misses = 0
    for E in pick:
        z = E + 1j * wl.eta
        sL, _, cL = O.lead_selfenergy(h00, wl.lead_h01_L, wl.lead_tau_L, z)
        sR, _, cR = O.lead_selfenergy(h00, wl.lead_h01_R, wl.lead_tau_R, z)
        assert cL and cR
        r = O.rgf(hd, hu, E, wl.eta, sL, sR, 1.0, 0.0, transmission=True)
        n_open = _open_channels(bands, E)
        assert abs(r["T"] - n_open) < 1e-5, (E, r["T"], n_open)
        # planted mistake: tau^dagger g_s tau instead of tau g_s tau^dagger
        gL, _, _ = O.sancho_rubio(h00, wl.lead_h01_L, z)
        gR, _, _ = O.sancho_rubio(h00, wl.lead_h01_R, z)
        tL, tR = wl.lead_tau_L, wl.lead_tau_R
        w = O.rgf(hd, hu, E, wl.eta, tL.conj().T @ gL @ tL, tR.conj().T @ gR @ tR, 1.0, 0.0, transmission=True)
        swapped_misses += abs(w["T"] - n_open) > 1e-2
    assert swapped_misses >= 1


# --------------------------------------------------------------------------
# SCBA closed forms (Eqs. 4 and 6): the Hermitian part of Sigma^R (full complex G^R)
# --------------------------------------------------------------------------

def _single_level(eps, energy, eta, D=0.0, M=0.0, shift=0, n0=0.0, mu=-50.0):
    """One orbital, one slab, leads decoupled (tau = 0): only the device eta
    and the scattering self-energies broaden the level.  mu far below the level
    leaves it empty (G^< = 0)."""
    from synth.workloads import Workload
    c = lambda x: np.array([[x]], dtype=np.complex128)
    n_e = len(energy)
    return Workload(name="level", seed=0, nb=1, orbs_per_atom=1, slab_offset=np.array([0, 1]),
                    kpts=np.zeros(1), w_k=np.ones(1), energy=np.asarray(energy, dtype=np.float64),
                    w_e=np.full(n_e, 0.01), h_diag=c(eps)[None, None], h_up=np.zeros((1, 1, 1), np.complex128),
                    up_block=1, lead_h00=c(0.0)[None], lead_h01_L=c(1.0), lead_tau_L=c(0.0), lead_h01_R=c(1.0),
                    lead_tau_R=c(0.0), lead_block=1, v_onsite=None, species=None, eta=eta, mu_L=mu, mu_R=mu,
                    D_ac=D, M_op=M, shift=shift, n_bose=n0)


def test_scba_acoustic_single_level_closed_form():
    """Sigma^R = D G^R on one level: the SCBA fixed point solves D G^2 - (z - eps) G + 1 = 0,
    G = (z - eps - sqrt((z - eps)^2 - 4 D)) / 2D on the branch with Im G < 0
    (a semicircle broadened by eta).  Pins reading Q8 (the full complex G^R,
    not i Im G^R): both the real and the imaginary part of G are compared."""
    E = np.linspace(-1.0, 1.0, 41)
    D, eps, eta = 0.04, 0.1, 0.05
    r = O.scba(_single_level(eps, E, eta, D=D), 400, tol=1e-15)
    assert r["hist"][-1] < 1e-14
    G = r["GRd"][0, :, 0, 0]
    z = E + 1j * eta - eps
    sq = np.sqrt(z * z - 4 * D)
    roots = np.stack([(z - sq) / (2 * D), (z + sq) / (2 * D)])
    assert np.all((roots.imag < 0).sum(axis=0) == 1)      # exactly one retarded root
    Gc = np.where(roots[0].imag < 0, roots[0], roots[1])
    assert np.max(np.abs(G.real - Gc.real)) < 1e-12 * np.max(np.abs(Gc))
    assert np.max(np.abs(G.imag - Gc.imag)) < 1e-12 * np.max(np.abs(Gc))
    assert np.max(np.abs(Gc.real)) > 0.5 * np.max(np.abs(Gc))   # the real part matters


def test_scba_optical_empty_level_continued_fraction():
    """Optical phonons on an empty level (G^< = 0) with n0 = 0: Eq. (6) leaves
    Sigma^R(E) = M G^R(E - hw), so the SCBA fixed point is the continued
    fraction G(E_j) = 1 / (z_j - eps - M G(E_{j-s})) built up from the bottom
    of the grid, with G(E_j) = 1 / (z_j - eps) for j < s (the off-grid group
    dropped, reading Q6).  Pins the direction of the emission shift and the
    (1 + n0) weight in Sigma^R, and the full complex G^R."""
    E = np.linspace(-1.0, 1.0, 41)
    eps, eta, M, s = 0.1, 0.05, 0.02, 3
    r = O.scba(_single_level(eps, E, eta, M=M, shift=s), 60, tol=1e-15)
    assert np.max(np.abs(r["GLd"])) == 0.0
    G = r["GRd"][0, :, 0, 0]
    Gc = np.zeros(len(E), dtype=np.complex128)
    for j in range(len(E)):
        Gc[j] = 1.0 / (E[j] + 1j * eta - eps - (M * Gc[j - s] if j >= s else 0.0))
    assert np.max(np.abs(G - Gc)) < 1e-13 * np.max(np.abs(Gc))


def test_rgf_diag_only_keeps_the_same_arithmetic():
    """The memory-lean mode returns exactly the orbital diagonals and bond
    currents of the full-block mode (it only drops blocks after use)."""
    wl = random_tiny(6, 5, n_e=2, seed=21, up_block=3, eta=1e-3)
    hd, hu, _ = wl.sample_blocks(0, 0)
    E = float(wl.energy[0])
    sL, sR = _leads(wl, 0, E)
    a = O.rgf(hd, hu, E, wl.eta, sL, sR, 0.7, 0.2, bond_mag=True)
    b = O.rgf(hd, hu, E, wl.eta, sL, sR, 0.7, 0.2, bond_mag=True, diag_only=True)
    for k in ("GR", "GL", "GG"):
        assert np.array_equal(np.diagonal(a[k], axis1=1, axis2=2), b[k]), k
    assert np.array_equal(a["bond"], b["bond"]) and np.array_equal(a["bond_mag"], b["bond_mag"])


# ---------------------------------------------------------------------------
# NEGF-Poisson loop (Eq. 9)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ny", [1, 2, 4])
def test_poisson_operator_laplace_closed_form(ny):
    """No charge, contacts at v_left / v_right, insulating z faces: the exact
    solution is linear in x and constant across the section; with gates at the
    contacts' common value the constant solves it."""
    nx, nz = 7, 3
    L = O.poisson_matrix(nx, nz, ny, False)
    b = O.poisson_boundary(nx, nz, ny, False, 0.3, -0.2)
    x = np.arange(nx)
    v = np.repeat(0.3 + (-0.2 - 0.3) * (x + 1) / (nx + 1), nz * ny)
    assert np.max(np.abs(L @ v - b)) < 1e-14
    Lg = O.poisson_matrix(nx, nz, ny, True)
    bg = O.poisson_boundary(nx, nz, ny, True, 0.1, 0.1, 0.1)
    assert np.max(np.abs(Lg @ np.full(nx * nz * ny, 0.1) - bg)) < 1e-14
    # symmetric, positive definite (every atom connects to a contact)
    assert np.array_equal(L, L.T)
    assert np.linalg.eigvalsh(L).min() > 0


def test_poisson_operator_uniform_charge_parabola():
    """Uniform charge q per atom between grounded contacts: the discrete
    solution is q (x + 1)(N_x - x) / 2 (its second difference is exactly -q)."""
    nx, nz, ny, q = 9, 2, 3, 0.37
    L = O.poisson_matrix(nx, nz, ny, False)
    x = np.arange(nx)
    v = np.repeat(q * (x + 1) * (nx - x) / 2.0, nz * ny)
    assert np.max(np.abs(L @ v - q)) < 1e-13


def _poisson_tiny(eta=0.05):
    import dataclasses
    wl = make_workload("C2", n_slab=4, n_e=48, n_k=1, n_z=1, n_y=2)
    return dataclasses.replace(wl, eta=eta, v_onsite=None)


def test_density_jacobian_matches_finite_differences_and_vjp():
    wl = _poisson_tiny()
    pts = [(0, 0, e) for e in range(wl.n_e)]
    leads = O.lead_tables(wl)
    rng = np.random.default_rng(9)
    v = rng.uniform(0.0, 0.2, size=(wl.total_slabs, wl.atoms_per_slab))
    D = O.density_jacobian(wl, v, pts, leads)
    h = 1e-5
    fd = np.zeros_like(D)
    for j in range(v.size):
        vp, vm = v.copy().reshape(-1), v.copy().reshape(-1)
        vp[j] += h
        vm[j] -= h
        fd[:, j] = (O.density_atoms(wl, vp.reshape(v.shape), pts, leads).reshape(-1)
                    - O.density_atoms(wl, vm.reshape(v.shape), pts, leads).reshape(-1)) / (2 * h)
    assert np.max(np.abs(D - fd)) < 1e-6 * np.max(np.abs(D))
    w = rng.normal(size=v.shape)
    g = O.dense_grad(wl, w, np.repeat(v, wl.orbs_per_atom, axis=1), pts, leads)
    assert np.max(np.abs(w.reshape(-1) @ D - g.reshape(-1))) < 1e-12 * np.max(np.abs(g))


def test_newton_poisson_pinned_by_its_residual():
    """The converged potential satisfies the discretised Eq. (9) with the
    density evaluated afresh (solve_points + observables), Newton converges
    quadratically, and a vanishing coupling beta returns the Laplace solution."""
    wl = _poisson_tiny()
    grid = O.PoissonGrid(nz=1, ny=2, v_left=0.0, v_right=-0.05)
    pts = [(0, 0, e) for e in range(wl.n_e)]
    leads = O.lead_tables(wl)
    beta = O.poisson_beta(11.7, 0.2715)
    n0 = O.density_atoms(wl, np.zeros((wl.total_slabs, 2)), pts, leads)
    nd = n0 + 0.02                # a small donor excess over the density at V = 0
    V, hist = O.newton_poisson(wl, grid, beta, nd, np.zeros(n0.shape), pts, leads, tol=1e-12)
    assert hist[-1] <= 1e-12 and len(hist) <= 8
    for a, b_ in zip(hist[1:], hist[2:]):          # quadratic once in the basin
        if a < 1e-3:
            assert b_ <= 10.0 * a * a + 1e-13
    L = O.poisson_matrix(wl.total_slabs, 1, 2, False)
    bb = O.poisson_boundary(wl.total_slabs, 1, 2, False, 0.0, -0.05)
    n = O.density_atoms(wl, V, pts, leads)
    F = L @ V.reshape(-1) - bb - beta * (n - nd).reshape(-1)
    assert np.max(np.abs(F)) < 1e-11
    V0, _ = O.newton_poisson(wl, grid, 1e-12, nd, np.zeros(n0.shape), pts, leads, tol=1e-14)
    x = np.arange(wl.total_slabs)
    lin = np.repeat(-0.05 * (x + 1) / (wl.total_slabs + 1), 2).reshape(V0.shape)
    assert np.max(np.abs(V0 - lin)) < 1e-12


def test_density_jacobian_symmetric_in_equilibrium_only():
    """One Fermi level for both leads and the eta sink: dn/dV is symmetric (its
    entries are sums of Im(G_ab G_ba)); under bias it is not."""
    import dataclasses
    wl = _poisson_tiny()
    pts = [(0, 0, e) for e in range(wl.n_e)]
    v = np.random.default_rng(2).uniform(0.0, 0.1, size=(wl.total_slabs, wl.atoms_per_slab))
    eq = dataclasses.replace(wl, mu_R=wl.mu_L)
    D = O.density_jacobian(eq, v, pts, O.lead_tables(eq), eta_fill=eq.mu_L)
    assert np.max(np.abs(D - D.T)) < 1e-12 * np.max(np.abs(D))
    Db = O.density_jacobian(wl, v, pts, O.lead_tables(wl))
    assert np.max(np.abs(Db - Db.T)) > 1e-3 * np.max(np.abs(Db))


# ---------------------------------------------------------------------------
# Complex-absorbing-potential contacts
# ---------------------------------------------------------------------------

def _cap_vs_leads(wl, energies, n_cap=80, w_max=1.0):
    """Bond current at the central device bond with absorbing contacts and
    with the exact (Sancho-Rubio) leads, for a wide bias window."""
    import dataclasses
    from synth.workloads import with_cap
    wl = dataclasses.replace(wl, energy=np.asarray(energies, dtype=np.float64), mu_L=6.0, mu_R=-6.0,
                             eta=1e-9)
    pts = [(0, 0, e) for e in range(len(energies))]
    exact = O.solve_points(wl, pts)
    capw = with_cap(wl, n_cap, w_max)
    cap = O.solve_points(capw, pts)
    mid = wl.total_slabs // 2
    return (np.array([r["bond"][mid] for r in exact]), np.array([r["bond"][n_cap + mid] for r in cap]))


def test_cap_contacts_reproduce_sancho_rubio_on_ordered_strip():
    """Long, smooth absorbing contacts on an ordered strip: the current is the
    exact open-boundary (Landauer) one to within the contacts' reflection."""
    wl = strip_workload(n_slab=6, disorder=0.0, n_e=4)
    ex, cap = _cap_vs_leads(wl, [-2.1, -0.7, 0.3, 1.9])
    assert np.all(np.abs(ex) > 1.0)
    assert np.max(np.abs(cap - ex) / np.abs(ex)) < 2e-3


def test_cap_contacts_reproduce_sancho_rubio_on_ordered_cross_section():
    """The same on a pure-Si cross-section, whose slab couplings are not
    symmetric: pins the orientation of the contact couplings too."""
    from synth.workloads import cross_section_workload
    wl = cross_section_workload("cap", 1, 2, [4], 1, np.zeros(1), 7, ge_fraction=0.0)
    ex, cap = _cap_vs_leads(wl, [-1.0, -0.1, 0.5, 1.2])     # 1, 2, 1, 1 open channels
    assert np.all(np.abs(ex) > 0.5)
    assert np.max(np.abs(cap - ex) / np.abs(ex)) < 1e-4


def test_cap_contacts_equilibrium_kms():
    """One Fermi level for both contacts and the eta sink: G^< = -f (G - G^dagger)
    on every slab of a disordered device with disordered absorbing contacts."""
    import dataclasses
    from synth.workloads import cross_section_workload
    wl = cross_section_workload("cap", 1, 2, [5], 1, np.linspace(-1, 1, 3), 11, cap_slabs=6, cap_w=0.5)
    wl = dataclasses.replace(wl, mu_R=wl.mu_L, eta=1e-3)
    pts = [(0, 0, e) for e in range(wl.n_e)]
    res = O.solve_points(wl, pts, eta_fill=wl.mu_L)
    for (s, k, e), r in zip(pts, res):
        f = float(O.fermi(wl.energy[e], wl.mu_L, wl.kT))
        A = r["GR"] - np.conj(np.swapaxes(r["GR"], 1, 2))
        assert np.max(np.abs(r["GL"] + f * A)) < 1e-12 * np.max(np.abs(A))


# ---------------------------------------------------------------------------
# Atom-block local scattering self-energies (the other reading of "diag G")
# ---------------------------------------------------------------------------

def _tiny_block_scba(seed=5, n_e=9, shift=2, D=0.02, M=0.03, eta=0.05, n_y=2):
    import dataclasses
    from synth.workloads import cross_section_workload
    energy = np.linspace(-0.2, 0.2, n_e)
    hw = shift * (energy[1] - energy[0])            # the phonon energy on the grid, Bose factor at kT
    wl = cross_section_workload("blk", 1, n_y, [3], 1, energy, seed, eta=eta, D_ac=D, M_op=M, hw_op=hw,
                                shift=shift, n_bose=1.0 / np.expm1(hw / 0.025852), n_scba=0)
    return dataclasses.replace(wl, species=None)


def test_scba_atom_blocks_reduce_to_orbital_diagonal_for_one_orbital_atoms():
    wl = _tiny_scba_workload(seed=13, n_e=7, shift=2, D=0.05, M=0.08)
    assert wl.orbs_per_atom == 1
    a = O.scba(wl, 3, atom_block_sigma=True)
    b = O.scba(wl, 3)
    assert np.array_equal(a["sigR"][..., 0], b["sigR"]) and np.array_equal(a["sigL"][..., 0], b["sigL"])


def test_scba_atom_blocks_kms_every_iterate():
    """Equilibrium with the eta contact filled: G^< = -f (G^R - G^A) on every
    diagonal block at every iterate of the atom-block loop."""
    wl = _tiny_block_scba()
    wl.mu_L = wl.mu_R = 0.1
    leads = O.lead_tables(wl)
    pts = [(0, 0, e) for e in range(wl.n_e)]
    opa, N, b = wl.orbs_per_atom, wl.total_slabs, wl.nb
    sR = np.zeros((wl.n_e, N, b, opa), dtype=complex)
    sL = np.zeros_like(sR)
    for it in range(3):
        res = O.solve_points(wl, pts, leads, sR, sL, eta_fill=wl.mu_L)
        for (s, ik, ie), r in zip(pts, res):
            f = O.fermi(wl.energy[ie], wl.mu_L, wl.kT)
            A = r["GR"] - np.conj(np.transpose(r["GR"], (0, 2, 1)))
            assert np.max(np.abs(r["GL"] + f * A)) < 1e-10 * np.max(np.abs(A)), (it, ie)
        GR = np.array([O.atom_blocks(r["GR"], opa) for r in res]).reshape(1, wl.n_e, N, b, opa)
        GL = np.array([O.atom_blocks(r["GL"], opa) for r in res]).reshape(1, wl.n_e, N, b, opa)
        sR, sL = O.scba_selfenergy(GR, GL, wl.w_k, wl.D_ac, wl.M_op, wl.shift, wl.n_bose)
        assert np.max(np.abs(sL[..., 1:])) > 0        # off-diagonal entries inside the atom blocks


def test_scba_atom_blocks_invariant_under_orbital_rotations_of_each_atom():
    """A unitary change of basis inside each atom (the same for that atom site
    in every slab and in the leads) maps G to U G U^dagger.  The atom-block
    self-energy transforms the same way, so the per-atom density and the bond
    currents of the Born loop do not change; with orbital-diagonal blocks they
    do -- which separates the two readings."""
    import dataclasses
    wl = _tiny_block_scba()
    opa, b = wl.orbs_per_atom, wl.nb
    rng = np.random.default_rng(77)
    U = np.zeros((b, b), dtype=complex)
    for a0 in range(0, b, opa):
        q, _ = np.linalg.qr(rng.normal(size=(opa, opa)) + 1j * rng.normal(size=(opa, opa)))
        U[a0:a0 + opa, a0:a0 + opa] = q
    rot = lambda X: U @ X @ U.conj().T
    wr = dataclasses.replace(
        wl, h_diag=np.array([[rot(h) for h in hk] for hk in wl.h_diag]), h_up=np.array([rot(h) for h in wl.h_up]),
        lead_h00=np.array([rot(h) for h in wl.lead_h00]), lead_h01_L=rot(wl.lead_h01_L),
        lead_h01_R=rot(wl.lead_h01_R), lead_tau_L=rot(wl.lead_tau_L), lead_tau_R=rot(wl.lead_tau_R))
    pts = [(0, 0, e) for e in range(wl.n_e)]

    def obs(w, blocks):
        out = O.scba(w, 4, atom_block_sigma=blocks)
        res = out["res"]
        return O.observables(w, pts, [np.diagonal(r["GL"], axis1=1, axis2=2) for r in res],
                             [r["bond"] for r in res])[:2]

    n0, J0 = obs(wl, True)
    n1, J1 = obs(wr, True)
    assert np.max(np.abs(n1 - n0)) < 1e-11 * np.max(np.abs(n0))
    assert np.max(np.abs(J1 - J0)) < 1e-11 * np.max(np.abs(n0))
    d0, _ = obs(wl, False)
    d1, _ = obs(wr, False)
    assert np.max(np.abs(d1 - d0)) > 1e-6 * np.max(np.abs(d0))


def test_lead_selfenergy_mirror_k_is_transpose():
    """The cross-section leads (real couplings, h00(-k) = h00(k)^T): the surface
    Green's function at -k solves the transposed equation, so Sigma(-k) =
    Sigma(k)^T for both leads; complex couplings break it."""
    import dataclasses
    wl = make_workload("C2", n_slab=3, n_e=3, n_k=4, n_z=1, n_y=2)
    tab = O.lead_tables(wl)
    for ie in range(wl.n_e):
        for a in range(2):
            S1, S3 = tab[(1, ie)][a], tab[(3, ie)][a]
            assert np.max(np.abs(S3 - S1.T)) < 1e-12 * np.max(np.abs(S1))
    # a complex (not gauge) change of the couplings: no longer real
    R = 0.05j * np.random.default_rng(3).normal(size=wl.lead_h01_R.shape)
    h01 = wl.lead_h01_R + R
    wc = dataclasses.replace(wl, lead_h01_R=h01, lead_tau_R=h01, lead_h01_L=h01.conj().T,
                             lead_tau_L=h01.conj().T)
    tc = O.lead_tables(wc, es=[1])
    S1, S3 = tc[(1, 1)][1], tc[(3, 1)][1]
    assert np.max(np.abs(S3 - S1.T)) > 1e-6 * np.max(np.abs(S1))


def test_density_jacobian_local_is_the_diagonal_for_one_orbital_atoms():
    """For one-orbital atoms the o' = o part is the whole diagonal of dn/dV."""
    wl = strip_workload(n_slab=4, n_e=6, e_lo=-3.0, e_hi=3.0, eta=1e-2)
    pts = [(0, 0, e) for e in range(wl.n_e)]
    leads = O.lead_tables(wl)
    v = np.random.default_rng(4).uniform(0.0, 0.1, size=(wl.total_slabs, wl.atoms_per_slab))
    D = O.density_jacobian(wl, v, pts, leads)
    d = O.density_jacobian_local(wl, v, pts, leads)
    assert np.max(np.abs(d.reshape(-1) - np.diag(D))) < 1e-12 * np.max(np.abs(D))


def test_dense_grad_with_absorbing_contacts_matches_finite_differences():
    from synth.workloads import cross_section_workload
    wl = cross_section_workload("cap", 1, 2, [3], 1, np.linspace(-0.5, 0.5, 2), 17, cap_slabs=3, cap_w=0.5,
                                eta=1e-3)
    pts = [(0, 0, ie) for ie in range(wl.n_e)]
    leads = O.lead_tables(wl)
    rng = np.random.default_rng(6)
    w = rng.normal(size=(wl.total_slabs, wl.atoms_per_slab))
    v = rng.uniform(0, 0.1, size=(wl.total_slabs, wl.nb))
    g = O.dense_grad(wl, w, v, pts, leads)
    h = 1e-5
    for (s, a) in [(0, 0), (3, 1), (5, 0), (8, 1)]:
        vp, vm = v.copy(), v.copy()
        vp[s, a * 10:(a + 1) * 10] += h
        vm[s, a * 10:(a + 1) * 10] -= h
        fd = (O.density_objective(wl, w, vp, pts, leads) - O.density_objective(wl, w, vm, pts, leads)) / (2 * h)
        assert abs(fd - g[s, a]) < 1e-6 * np.max(np.abs(g)) + 1e-12


def test_dense_grad_with_fixed_scattering_matches_finite_differences():
    wl = make_workload("C5", n_slab=3, n_e=2, n_z=1, n_y=2)
    wl.eta = 1e-3
    pts = [(0, 0, ie) for ie in range(wl.n_e)]
    leads = O.lead_tables(wl)
    rng = np.random.default_rng(12)
    shp = (wl.n_e, wl.total_slabs, wl.nb)
    sR = 0.02 * rng.normal(size=shp) - 0.03j * rng.uniform(size=shp)
    sL = 0.02j * rng.uniform(size=shp)
    w = rng.normal(size=(wl.total_slabs, wl.atoms_per_slab))
    v = wl.v_onsite.copy()
    g = O.dense_grad(wl, w, v, pts, leads, sR, sL)
    assert np.max(np.abs(g - O.dense_grad(wl, w, v, pts, leads))) > 1e-6 * np.max(np.abs(g))
    h = 1e-5
    for (s, a) in [(0, 0), (1, 1), (2, 0)]:
        vp, vm = v.copy(), v.copy()
        vp[s, a * 10:(a + 1) * 10] += h
        vm[s, a * 10:(a + 1) * 10] -= h
        fd = (O.density_objective(wl, w, vp, pts, leads, sR, sL)
              - O.density_objective(wl, w, vm, pts, leads, sR, sL)) / (2 * h)
        assert abs(fd - g[s, a]) < 1e-6 * np.max(np.abs(g)) + 1e-12
