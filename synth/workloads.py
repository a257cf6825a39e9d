"""Seeded synthetic workloads (inputs only; no Green's-function arithmetic).

Five workloads mirror the shapes of the paper's device runs (Sec. "System and
environment": 1200^2 / 720^2 / 240^2 dense blocks; Sec. "Overview": 10 orbitals
per atom, ~24,000 atoms, rank 240,000; Si with 10 % Ge).  The sp3d5s* parameters,
the device geometry and the phonon constants are not printed in the paper, so
every number here is a seeded stand-in with the same sizes and structure:

* ``C1``  single-orbital square-lattice strip, width 8, 20 slabs, t = -1 eV,
          onsite U(-0.25, 0.25) eV, ordered leads with onsite 0, 256 energies
          in [-4, 4] eV, one k-point.
* ``C2``  40-atom cross-section (10 confined x 4 periodic), 10 orbitals/atom
          (block 400), 70 slabs, 10 % Ge, 512 energies in [-2, 2] eV x 8 k.
* ``C3``  24-atom cross-section (12 x 2, block 240), 120 slabs, 1024 energies
          on a 5 meV grid x 4 k, acoustic + optical phonon parameters.
* ``C4``  128 alloy samples, block 400, slab counts U{50..90}, 256 energies.
* ``C5``  120-atom cross-section (12 x 10, block 1200), 200 slabs, 16 energies,
          smooth seeded onsite potential 0..0.3 eV.

Layout conventions (all arrays NumPy, row-major):

* ``h_diag[k, s, :, :]``   H_ss(k) for global slab ``s`` (samples concatenated
                           along the slab axis, ``slab_offset`` gives ranges).
* ``h_up[s, :, :]``        H_{s,s+1}; block-diagonal in atoms (``up_block``
                           orbitals per block); unused (zero) on the last slab
                           of each sample.  Independent of k.
* ``lead_h00[k]``          principal-layer Hamiltonian of both ordered leads.
* ``lead_h01_L/R``         coupling from the lead's surface layer to the next
                           layer deeper inside that lead.
* ``lead_tau_L/R``         coupling from the device edge slab to the lead
                           surface layer (H_{1,0} on the left, H_{N,N+1} on
                           the right).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

KT_300K = 0.025852  # eV, k_B * 300 K
WORKLOAD_NAMES = ("C1", "C2", "C3", "C4", "C5")

# Per-workload base seeds.
SEEDS = {"C1": 1510046861, "C2": 1510046862, "C3": 1510046863, "C4": 1510046864, "C5": 1510046865}


@dataclasses.dataclass
class Workload:
    name: str
    seed: int
    nb: int
    orbs_per_atom: int
    slab_offset: np.ndarray          # int64 [n_samples+1]
    kpts: np.ndarray                 # float64 [n_k]
    w_k: np.ndarray                  # float64 [n_k]
    energy: np.ndarray               # float64 [n_e]
    w_e: np.ndarray                  # float64 [n_e]
    h_diag: np.ndarray               # complex128 [n_k, total_slabs, nb, nb]
    h_up: np.ndarray                 # complex128 [total_slabs, nb, nb]
    up_block: int
    lead_h00: np.ndarray             # complex128 [n_k, nb, nb]
    lead_h01_L: np.ndarray           # complex128 [nb, nb]
    lead_tau_L: np.ndarray           # complex128 [nb, nb]
    lead_h01_R: np.ndarray
    lead_tau_R: np.ndarray
    lead_block: int                  # block size of the block-diagonal h01 / tau
    v_onsite: Optional[np.ndarray]   # float64 [total_slabs, nb] or None
    species: Optional[np.ndarray]    # int8 [total_slabs, atoms_per_slab] (1 = Ge)
    eta: float = 1e-6
    mu_L: float = 0.05
    mu_R: float = -0.05
    kT: float = KT_300K
    g_s: float = 2.0
    # phonon scattering (Eqs. 4-6); zero for ballistic workloads
    D_ac: float = 0.0
    M_op: float = 0.0
    hw_op: float = 0.0
    shift: int = 0
    n_bose: float = 0.0
    n_scba: int = 0
    # complex absorbing potential contacts (None: Sancho-Rubio leads)
    cap_w: Optional[np.ndarray] = None      # float64 [total_slabs] absorbing strength W per slab (eV)
    cap_side: Optional[np.ndarray] = None   # int8 [total_slabs]: -1 left contact region, +1 right, 0 device

    @property
    def n_samples(self) -> int:
        return len(self.slab_offset) - 1

    @property
    def n_k(self) -> int:
        return len(self.kpts)

    @property
    def n_e(self) -> int:
        return len(self.energy)

    @property
    def total_slabs(self) -> int:
        return int(self.slab_offset[-1])

    @property
    def atoms_per_slab(self) -> int:
        return self.nb // self.orbs_per_atom

    def n_slab(self, sample: int) -> int:
        return int(self.slab_offset[sample + 1] - self.slab_offset[sample])

    def points(self) -> np.ndarray:
        """All (sample, ik, ie) points, sample-major, then k, then energy."""
        s, k, e = np.meshgrid(np.arange(self.n_samples), np.arange(self.n_k),
                              np.arange(self.n_e), indexing="ij")
        return np.stack([s.ravel(), k.ravel(), e.ravel()], axis=1).astype(np.int32)

    def sample_blocks(self, sample: int, ik: int):
        """(H_ii list, H_{i,i+1} list, onsite-potential list) of one sample at one k."""
        a, b = int(self.slab_offset[sample]), int(self.slab_offset[sample + 1])
        hd = [self.h_diag[ik, s] for s in range(a, b)]
        hu = [self.h_up[s] for s in range(a, b - 1)]
        v = None if self.v_onsite is None else [self.v_onsite[s] for s in range(a, b)]
        return hd, hu, v


# --------------------------------------------------------------------------
# C1: single-orbital strip
# --------------------------------------------------------------------------

def strip_workload(width: int = 8, n_slab: int = 20, t: float = -1.0, disorder: float = 0.25,
                   n_e: int = 256, e_lo: float = -4.0, e_hi: float = 4.0, eta: float = 1e-6,
                   seed: int = SEEDS["C1"], name: str = "C1") -> Workload:
    """Square-lattice strip of ``width`` sites with hard walls; ``disorder`` = 0
    gives the ordered strip whose transmission counts open subbands."""
    rng = np.random.default_rng([seed, 2])
    nb = width
    hop = np.zeros((nb, nb))
    for i in range(nb - 1):
        hop[i, i + 1] = hop[i + 1, i] = t
    onsite = rng.uniform(-disorder, disorder, size=(n_slab, nb)) if disorder > 0 else np.zeros((n_slab, nb))
    h_diag = np.zeros((1, n_slab, nb, nb), dtype=np.complex128)
    for s in range(n_slab):
        h_diag[0, s] = hop + np.diag(onsite[s])
    h_up = np.zeros((n_slab, nb, nb), dtype=np.complex128)
    for s in range(n_slab - 1):
        h_up[s] = t * np.eye(nb)
    tI = (t * np.eye(nb)).astype(np.complex128)
    energy = np.linspace(e_lo, e_hi, n_e)
    de = (e_hi - e_lo) / max(n_e - 1, 1)
    return Workload(
        name=name, seed=seed, nb=nb, orbs_per_atom=1,
        slab_offset=np.array([0, n_slab], dtype=np.int64),
        kpts=np.zeros(1), w_k=np.ones(1), energy=energy, w_e=np.full(n_e, de),
        h_diag=h_diag, h_up=h_up, up_block=1,
        lead_h00=hop.astype(np.complex128)[None].copy(),
        lead_h01_L=tI.copy(), lead_tau_L=tI.copy(), lead_h01_R=tI.copy(), lead_tau_R=tI.copy(),
        lead_block=1, v_onsite=None, species=None, eta=eta)


# --------------------------------------------------------------------------
# C2-C5: multi-orbital cross-section with Si/Ge species
# --------------------------------------------------------------------------

ORB = 10  # orbitals per atom (sp3d5s*-sized)


def _material(seed: int, bandwidth_half: float = 5.0):
    """Onsite blocks E[species] and couplings C[d][sp_a][sp_b] (10x10, real)."""
    rng = np.random.default_rng([seed, 0])
    E = []
    for sp in range(2):
        m = rng.normal(0.0, 0.1, size=(ORB, ORB))
        m = np.triu(m, 1)
        m = m + m.T
        m[np.diag_indices(ORB)] = rng.uniform(-1.5, 1.5, size=ORB) + (0.1 if sp == 1 else 0.0)
        E.append(m)
    C = []
    for d in range(3):  # x, y, z
        c_ss = rng.normal(0.0, 1.0, size=(ORB, ORB))
        c_sg = rng.normal(0.0, 1.0, size=(ORB, ORB))
        c_gg = rng.normal(0.0, 1.0, size=(ORB, ORB))
        C.append([[c_ss, c_sg], [c_sg.T.copy(), c_gg]])
    # Scale all couplings by one factor so that the pure-Si bulk Gershgorin
    # bound (onsite block plus six bonds) equals bandwidth_half.
    a = np.abs(E[0]).sum(axis=1)
    bsum = np.zeros(ORB)
    for d in range(3):
        bsum += np.abs(C[d][0][0]).sum(axis=1) + np.abs(C[d][0][0]).sum(axis=0)
    scale = float(np.min((bandwidth_half - a) / bsum))
    C = [[[scale * C[d][p][q] for q in range(2)] for p in range(2)] for d in range(3)]
    return E, C


def _slab_blocks(species_slab, n_z, n_y, E, C):
    """Real parts of H_ii: (H0, Y) with H_ii(k) = H0 + e^{ik} Y + e^{-ik} Y^T.

    Atom index a = z * n_y + y.  +z bonds stop at the hard walls; +y bonds wrap
    around with a Bloch phase on the wrapping bond."""
    nat = n_z * n_y
    nb = nat * ORB
    H0 = np.zeros((nb, nb))
    Y = np.zeros((nb, nb))
    for z in range(n_z):
        for y in range(n_y):
            a = z * n_y + y
            sa = species_slab[a]
            ra = slice(a * ORB, (a + 1) * ORB)
            H0[ra, ra] += E[sa]
            if z + 1 < n_z:  # +z bond
                bidx = (z + 1) * n_y + y
                rb = slice(bidx * ORB, (bidx + 1) * ORB)
                blk = C[2][sa][species_slab[bidx]]
                H0[ra, rb] += blk
                H0[rb, ra] += blk.T
            yb = y + 1
            wrap = yb == n_y
            bidx = z * n_y + (yb % n_y)
            rb = slice(bidx * ORB, (bidx + 1) * ORB)
            blk = C[1][sa][species_slab[bidx]]
            if wrap:
                Y[ra, rb] += blk       # phase e^{+ik} on a -> b(cell+1)
            else:
                H0[ra, rb] += blk
                H0[rb, ra] += blk.T
    return H0, Y


def _up_block(species_i, species_j, C):
    nat = len(species_i)
    U = np.zeros((nat * ORB, nat * ORB))
    for a in range(nat):
        r = slice(a * ORB, (a + 1) * ORB)
        U[r, r] = C[0][species_i[a]][species_j[a]]
    return U


def _smooth_potential(rng, n_slab, n_z, n_y, vmax=0.3):
    x = (np.arange(n_slab) + 0.5) / n_slab
    amp = rng.normal(0.0, 1.0, size=3)
    ph = rng.uniform(0.0, 2 * np.pi, size=3)
    prof = sum(amp[m] * np.sin((m + 1) * np.pi * x + ph[m]) for m in range(3))
    cz = rng.normal(0.0, 0.5)
    zz = np.cos(np.pi * (np.arange(n_z) + 0.5) / n_z)
    v = prof[:, None, None] + cz * zz[None, :, None] + np.zeros((1, 1, n_y))
    v = (v - v.min()) / max(v.max() - v.min(), 1e-300) * vmax
    return v.reshape(n_slab, n_z * n_y)


def cap_profile(n_dev: int, n_cap: int, w_max: float, power: float = 2.0):
    """Absorbing strength and side of every slab of one sample extended by
    n_cap contact slabs on each side: W = w_max (d / n_cap)^power at depth d =
    1..n_cap into a contact region, 0 in the n_dev device slabs."""
    n = n_dev + 2 * n_cap
    w = np.zeros(n)
    side = np.zeros(n, dtype=np.int8)
    for d in range(1, n_cap + 1):
        v = w_max * (d / n_cap) ** power
        w[n_cap - d], side[n_cap - d] = v, -1
        w[n_cap + n_dev - 1 + d], side[n_cap + n_dev - 1 + d] = v, 1
    return w, side


def with_cap(wl: Workload, n_cap: int, w_max: float, power: float = 2.0) -> Workload:
    """The workload with its ordered leads made explicit: every sample gets
    n_cap slabs of lead material on each side (onsite blocks lead_h00, the
    leads' couplings), carrying the absorbing profile of ``cap_profile`` --
    the complex-absorbing-potential stand-in for the semi-infinite leads."""
    counts = np.diff(wl.slab_offset)
    hd, hu, vv, ww, ss = [], [], [], [], []
    for smp in range(wl.n_samples):
        a0, a1 = int(wl.slab_offset[smp]), int(wl.slab_offset[smp + 1])
        n = a1 - a0
        lead = np.repeat(wl.lead_h00[:, None], n_cap, axis=1)
        hd.append(np.concatenate([lead, wl.h_diag[:, a0:a1], lead], axis=1))
        up = np.zeros((n + 2 * n_cap, wl.nb, wl.nb), dtype=np.complex128)
        # left contact slabs: H_{j,j+1} = (h01_L)^dagger inside, tau_L^dagger onto the device
        up[:n_cap - 1] = wl.lead_h01_L.conj().T
        up[n_cap - 1] = wl.lead_tau_L.conj().T
        up[n_cap:n_cap + n - 1] = wl.h_up[a0:a1 - 1]
        up[n_cap + n - 1] = wl.lead_tau_R
        up[n_cap + n:n + 2 * n_cap - 1] = wl.lead_h01_R
        hu.append(up)
        if wl.v_onsite is not None:
            z = np.zeros((n_cap, wl.nb))
            vv.append(np.concatenate([z, wl.v_onsite[a0:a1], z]))
        w, side = cap_profile(n, n_cap, w_max, power)
        ww.append(w)
        ss.append(side)
    off = np.concatenate([[0], np.cumsum(counts + 2 * n_cap)]).astype(np.int64)
    return dataclasses.replace(
        wl, slab_offset=off, h_diag=np.concatenate(hd, axis=1), h_up=np.concatenate(hu),
        v_onsite=np.concatenate(vv) if vv else None, species=None,
        cap_w=np.concatenate(ww), cap_side=np.concatenate(ss))


def cross_section_workload(name: str, n_z: int, n_y: int, n_slabs, n_k: int, energy: np.ndarray,
                           seed: int, ge_fraction: float = 0.1, potential: bool = False,
                           eta: float = 1e-6, samples=None, cap_slabs: int = 0, cap_w: float = 1.0,
                           cap_power: float = 2.0, **params) -> Workload:
    """Si/Ge cross-section device.  ``n_slabs`` is one slab count per sample.

    Ge sites are drawn per sample (own seeded stream), exactly
    round(ge_fraction * eligible) of them, without replacement, among the
    interior slabs 2..N-1; the two edge slabs stay pure Si so that the
    ordered pure-Si leads (and their self-energies) are shared by all samples.
    ``samples`` restricts generation to a subset of sample indices (the draws of
    each sample do not depend on the others).
    ``cap_slabs`` > 0: disordered contacts -- every sample is extended by that
    many slabs on each side, the random alloy runs through them (Ge drawn among
    all slabs, own stream), and they carry the absorbing profile of
    ``cap_profile`` instead of ordered leads."""
    E, C = _material(seed)
    nat = n_z * n_y
    nb = nat * ORB
    n_slabs = list(n_slabs)
    sample_ids = list(range(len(n_slabs))) if samples is None else list(samples)
    if cap_slabs > 0:
        n_slabs = [n + 2 * cap_slabs for n in n_slabs]
    counts = [n_slabs[s] for s in sample_ids]
    slab_offset = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    total = int(slab_offset[-1])
    kpts = 2 * np.pi * np.arange(n_k) / n_k
    species = np.zeros((total, nat), dtype=np.int8)
    for j, s in enumerate(sample_ids):
        n = n_slabs[s]
        if cap_slabs > 0:          # the alloy runs through the contact regions
            rng = np.random.default_rng([seed, 1000 + s, 7])
            n_ge = int(round(ge_fraction * n * nat))
            sp = np.zeros(n * nat, dtype=np.int8)
            sp[rng.choice(n * nat, size=n_ge, replace=False)] = 1
            blk = sp.reshape(n, nat)
            species[slab_offset[j]:slab_offset[j + 1]] = blk
            continue
        rng = np.random.default_rng([seed, 1000 + s])
        interior = max(n - 2, 0) * nat
        n_ge = int(round(ge_fraction * interior))
        sp = np.zeros(interior, dtype=np.int8)
        if n_ge > 0:
            sp[rng.choice(interior, size=n_ge, replace=False)] = 1
        blk = np.zeros((n, nat), dtype=np.int8)
        if n > 2:
            blk[1:n - 1] = sp.reshape(n - 2, nat)
        species[slab_offset[j]:slab_offset[j + 1]] = blk
    h_diag = np.empty((n_k, total, nb, nb), dtype=np.complex128)
    h_up = np.zeros((total, nb, nb), dtype=np.complex128)
    cache = {}
    for j in range(len(sample_ids)):
        a0, a1 = int(slab_offset[j]), int(slab_offset[j + 1])
        for s in range(a0, a1):
            key = species[s].tobytes()
            if key not in cache:
                cache.clear()
                cache[key] = _slab_blocks(species[s], n_z, n_y, E, C)
            H0, Y = cache[key]
            for ik, k in enumerate(kpts):
                h_diag[ik, s] = H0 + np.exp(1j * k) * Y + np.exp(-1j * k) * Y.T
            if s + 1 < a1:
                h_up[s] = _up_block(species[s], species[s + 1], C)
    si = np.zeros(nat, dtype=np.int8)
    H0s, Ys = _slab_blocks(si, n_z, n_y, E, C)
    lead_h00 = np.stack([H0s + np.exp(1j * k) * Ys + np.exp(-1j * k) * Ys.T for k in kpts])
    Uss = _up_block(si, si, C).astype(np.complex128)
    v_onsite = None
    if potential:
        rng = np.random.default_rng([seed, 3])
        vfull = [_smooth_potential(rng, n, n_z, n_y) for n in n_slabs]
        v_atom = np.concatenate([vfull[s] for s in sample_ids], axis=0)
        v_onsite = np.repeat(v_atom, ORB, axis=1)
    de = float(energy[1] - energy[0]) if len(energy) > 1 else 1.0
    cw = cs = None
    if cap_slabs > 0:
        prof = [cap_profile(n_slabs[s] - 2 * cap_slabs, cap_slabs, cap_w, cap_power) for s in sample_ids]
        cw = np.concatenate([p[0] for p in prof])
        cs = np.concatenate([p[1] for p in prof])
    return Workload(
        cap_w=cw, cap_side=cs,
        name=name, seed=seed, nb=nb, orbs_per_atom=ORB, slab_offset=slab_offset,
        kpts=kpts, w_k=np.full(n_k, 1.0 / n_k), energy=np.asarray(energy, dtype=np.float64),
        w_e=np.full(len(energy), de), h_diag=h_diag, h_up=h_up, up_block=ORB,
        lead_h00=lead_h00, lead_h01_L=Uss.T.copy(), lead_tau_L=Uss.T.copy(),
        lead_h01_R=Uss.copy(), lead_tau_R=Uss.copy(), lead_block=ORB,
        v_onsite=v_onsite, species=species, eta=eta, **params)


def scba_params(kT: float = KT_300K, hw: float = 0.060, de: float = 0.005):
    """Phonon parameters of the SCBA workload (Eqs. 4-6 with lumped prefactors)."""
    return dict(D_ac=1e-3, M_op=1e-3, hw_op=hw, shift=int(round(hw / de)),
                n_bose=1.0 / math.expm1(hw / kT), n_scba=20)


def make_workload(name: str, n_slab: Optional[int] = None, n_e: Optional[int] = None,
                  n_k: Optional[int] = None, n_z: Optional[int] = None, n_y: Optional[int] = None,
                  n_samples: Optional[int] = None, samples=None, cap_slabs: int = 0) -> Workload:
    """The named workload; keyword overrides shrink it for tests (same recipe).
    cap_slabs (C2, C4): disordered absorbing-potential contacts of that many
    slabs per side instead of the ordered leads."""
    seed = SEEDS[name]
    if name == "C1":
        return strip_workload(n_slab=n_slab or 20, n_e=n_e or 256, seed=seed)
    if name == "C2":
        ne = n_e or 512
        return cross_section_workload("C2", n_z or 10, n_y or 4, [n_slab or 70], n_k or 8,
                                      np.linspace(-2.0, 2.0, ne), seed, cap_slabs=cap_slabs)
    if name == "C3":
        ne = n_e or 1024
        energy = -2.56 + 0.005 * np.arange(ne)
        return cross_section_workload("C3", n_z or 12, n_y or 2, [n_slab or 120], n_k or 4,
                                      energy, seed, **scba_params())
    if name == "C4":
        ns = n_samples or 128
        counts = np.random.default_rng([seed, 1]).integers(50, 91, size=ns)
        if n_slab is not None:
            counts = np.maximum(2, np.round(counts * n_slab / 70.0)).astype(int)
        ne = n_e or 256
        return cross_section_workload("C4", n_z or 10, n_y or 4, [int(c) for c in counts], n_k or 1,
                                      np.linspace(-2.0, 2.0, ne), seed, samples=samples, cap_slabs=cap_slabs)
    if name == "C5":
        ne = n_e or 16
        return cross_section_workload("C5", n_z or 12, n_y or 10, [n_slab or 200], n_k or 1,
                                      np.linspace(-0.1, 0.1, ne), seed, potential=True)
    raise KeyError(name)


# --------------------------------------------------------------------------
# Tiny random systems (tests)
# --------------------------------------------------------------------------

def _herm(rng, n, scale=1.0):
    a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return scale * (a + a.conj().T) / 2


def random_tiny(nb: int, n_slab: int, n_e: int = 4, seed: int = 0, up_block: Optional[int] = None,
                eta: float = 1e-3, complex_h: bool = True, n_k: int = 1) -> Workload:
    """A small random block-tridiagonal system with random ordered leads.

    ``up_block`` (a divisor of ``nb``) makes H_{i,i+1} and the lead couplings
    block-diagonal with blocks of that size; None means dense couplings."""
    rng = np.random.default_rng([seed, 77])
    m = nb if up_block is None else up_block
    assert nb % m == 0

    def coupling(scale):
        U = np.zeros((nb, nb), dtype=np.complex128)
        for a in range(nb // m):
            r = slice(a * m, (a + 1) * m)
            blk = rng.normal(size=(m, m)) + (1j * rng.normal(size=(m, m)) if complex_h else 0)
            U[r, r] = scale * blk
        return U

    def herm(scale):
        h = _herm(rng, nb, scale)
        return h if complex_h else h.real.astype(np.complex128)

    h_diag = np.stack([herm(0.6) for _ in range(n_slab)])[None].repeat(n_k, axis=0)
    h_up = np.zeros((n_slab, nb, nb), dtype=np.complex128)
    for s in range(n_slab - 1):
        h_up[s] = coupling(0.4)
    lead00 = herm(0.5)
    lead01 = coupling(0.4)
    tauL = coupling(0.4)
    tauR = coupling(0.4)
    energy = rng.uniform(-1.5, 1.5, size=n_e)
    return Workload(
        name=f"tiny{nb}x{n_slab}", seed=seed, nb=nb, orbs_per_atom=m if up_block else 1,
        slab_offset=np.array([0, n_slab], dtype=np.int64), kpts=np.zeros(n_k),
        w_k=np.full(n_k, 1.0 / n_k), energy=energy, w_e=np.full(n_e, 0.01),
        h_diag=h_diag, h_up=h_up, up_block=m,
        lead_h00=lead00[None].repeat(n_k, axis=0), lead_h01_L=lead01.conj().T.copy(), lead_tau_L=tauL,
        lead_h01_R=lead01, lead_tau_R=tauR, lead_block=m,
        v_onsite=None, species=None, eta=eta)
