"""GPU: absorbing-potential contacts (disordered leads) -- the contact
self-energy kernel against the oracle, the RGF with such contacts against the
oracle at the FP64 tolerance (one-launch small-block path and batched path,
ragged disordered samples), and the contacts against the exact leads on an
ordered strip, all through the C ABI."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import oracle as O
import parity as P
from synth import make_workload, strip_workload
from synth.workloads import cross_section_workload, with_cap

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _disordered(n_slabs, n_e=6, cap=6, n_z=1, n_y=2):
    return cross_section_workload("cap", n_z, n_y, n_slabs, 1, np.linspace(-0.8, 0.8, n_e), 31,
                                  cap_slabs=cap, cap_w=0.5, eta=1e-6)


def test_cap_selfenergy_kernel_matches_oracle():
    from paper_1510_04686_amd.runtime import RGFSolver
    wl = _disordered([3, 5])
    s = RGFSolver(wl, capacity=8)
    s.lead_selfenergies()
    torch.cuda.synchronize()
    R, L = O.cap_selfenergy(wl)
    for got, ref in ((s.cap_R, R), (s.cap_L, L)):
        g = got.cpu().numpy()
        assert np.max(np.abs(g - ref)) <= 4e-16 * np.max(np.abs(ref))
    assert float(s.sigma_L.abs().max()) == 0.0 and float(s.sigma_R.abs().max()) == 0.0


@pytest.mark.parametrize("kind", ["strip_small_block", "section_batched"])
def test_cap_contacts_rgf_matches_oracle(kind):
    """Ragged disordered samples whose contacts are absorbing regions of the
    same random alloy: every orbital diagonal, bond current and density
    against the oracle at the FP64 tolerance."""
    from paper_1510_04686_amd.runtime import RGFSolver
    if kind == "strip_small_block":            # blocks of 8 orbitals: the one-launch kernel
        base = strip_workload(n_slab=5, n_e=5, e_lo=-3.0, e_hi=3.0)
        wl = with_cap(base, 12, 0.8)
    else:
        wl = _disordered([4, 2], n_e=4)
    _say(f"absorbing contacts {kind}: nb={wl.nb} slabs={np.diff(wl.slab_offset).tolist()}")
    s = RGFSolver(wl, capacity=16)
    out = s.solve()
    n, J, _ = s.observables(out["GL"], out["bond"])
    torch.cuda.synchronize()
    assert s.status() == 0
    pts = [tuple(int(x) for x in p) for p in s.points]
    ref, tols = P.reference(wl, pts)
    counts = np.diff(wl.slab_offset)
    for p, (pt, r, t) in enumerate(zip(pts, ref, tols)):
        P.check_point(out, p, pt, r, int(counts[pt[0]]), t)
    rn, rJ, _ = O.observables(wl, pts, [np.diagonal(r["GL"], axis1=1, axis2=2) for r in ref],
                              [r["bond"] for r in ref])
    # the sums of Eqs. (7)-(8) over those outputs (each point already held to
    # its FP64 tolerance above): a consistency check of the reductions
    assert P.rel(n.cpu().numpy(), rn) < 1e-6
    assert np.max(np.abs(J.cpu().numpy() - rJ)) < 1e-6 * max(np.max(np.abs(rJ)), np.max(np.abs(rn)))


def test_cap_contacts_match_exact_leads_on_gpu():
    """Ordered strip, wide bias window: the GPU's current with long absorbing
    contacts equals its current with the exact Sancho-Rubio leads."""
    from paper_1510_04686_amd.runtime import RGFSolver
    base = strip_workload(n_slab=6, disorder=0.0, n_e=4)
    base = dataclasses.replace(base, energy=np.array([-2.1, -0.7, 0.3, 1.9]), mu_L=6.0, mu_R=-6.0, eta=1e-9)
    s0 = RGFSolver(base)
    o0 = s0.solve()
    s1 = RGFSolver(with_cap(base, 80, 1.0))
    o1 = s1.solve()
    torch.cuda.synchronize()
    j0 = o0["bond"].cpu().numpy()[:, 3]
    j1 = o1["bond"].cpu().numpy()[:, 80 + 3]
    _say(f"  exact leads {j0}, absorbing contacts {j1}")
    assert np.all(np.abs(j0) > 1.0)
    assert np.max(np.abs(j1 - j0) / np.abs(j0)) < 2e-3


@pytest.mark.parametrize("graph", [False, True])
def test_scba_with_absorbing_contacts_matches_oracle(graph):
    """Phonon scattering (acoustic + optical) in a device whose disordered
    contacts are absorbing regions: the Born loop adds its self-energies to the
    contacts' on the device (also inside the captured graph)."""
    from paper_1510_04686_amd.runtime import RGFSolver
    energy = np.linspace(-0.2, 0.2, 9)
    hw = 2 * (energy[1] - energy[0])
    wl = cross_section_workload("cap", 1, 2, [3], 1, energy, 23, cap_slabs=4, cap_w=0.5, eta=0.05,
                                D_ac=0.02, M_op=0.03, hw_op=hw, shift=2, n_bose=1.0 / np.expm1(hw / 0.025852),
                                n_scba=4)
    ref = O.scba(wl, 4)
    s = RGFSolver(wl)
    out, hist = s.scba(n_iter=4, graph=graph)
    torch.cuda.synchronize()
    assert s.status() == 0
    for got, want in ((s.scat_R, ref["sigR"]), (s.scat_L, ref["sigL"])):
        err = float(np.max(np.abs(got.cpu().numpy() - want)) / np.max(np.abs(want)))
        _say(f"  Sigma_scat rel err {err:.2e}")
        assert err < 1e-10
    d = lambda x: np.diagonal(x, axis1=1, axis2=2)
    for key in ("GR", "GL"):
        got = out[key].cpu().numpy()[:, :wl.total_slabs]
        want = np.array([d(r[key]) for r in ref["res"]])
        assert float(np.max(np.abs(got - want)) / np.max(np.abs(want))) < 1e-10
