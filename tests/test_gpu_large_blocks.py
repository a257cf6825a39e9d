"""GPU: blocks wider than 512 orbitals, where the inverse switches panel shapes
(FP64: 16 columns x 2-3 rows per thread, 8 x 4 up to 2048; FP32: 32 x 2-3,
16 x 4), against NumPy through the C ABI; and the paper-shaped block-1200
cross-section against oracle references written by
tests/golden/make_golden.py (the oracle at block 1200 takes minutes per
point, so its values are stored, never taken from the GPU)."""
import os
import sys

import numpy as np
import pytest
import torch

import parity as P
from synth import make_workload

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
if GOLDEN not in sys.path:
    sys.path.insert(0, GOLDEN)


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_1510_04686_amd import negf
    return negf.negf_create(nb=2048, n_slab_max=1, capacity=3)


def _rand(rng, shape, dtype=np.complex128):
    return (rng.normal(size=shape) + 1j * rng.normal(size=shape)).astype(dtype)


def _norm2(M, iters=40):
    """Spectral norm by power iteration on M^H M (from below; cheap at n = 2048)."""
    v = np.random.default_rng(0).normal(size=M.shape[1]) + 0j
    for _ in range(iters):
        v = M.conj().T @ (M @ v)
        v /= np.linalg.norm(v)
    return float(np.linalg.norm(M @ v))


def _cond(A, Ainv):
    return _norm2(A.astype(np.complex128)) * _norm2(Ainv)


def _inverse_cases(rng, n, dtype):
    """A random matrix, one with a zero diagonal (every pivot needs a row
    exchange) and a permuted identity with a small random part."""
    A = _rand(rng, (3, n, n), dtype)
    A[1][np.diag_indices(n)] = 0
    A[2] = (np.eye(n)[rng.permutation(n)] + 1e-3 * A[2]).astype(dtype)
    return A


@pytest.mark.parametrize("n", [513, 600, 1024, 1025, 1200, 1536, 1537, 2048])
@pytest.mark.parametrize("W", [0, 128])
def test_zinv_fp64_large(ctx, n, W):
    from paper_1510_04686_amd import negf
    _say(f"zinv fp64 n={n} outer={W}")
    rng = np.random.default_rng(9000 + n + W)
    A = _inverse_cases(rng, n, np.complex128)
    ref = np.linalg.inv(A)
    old = negf.negf_get_tuning(ctx)
    try:
        negf.negf_set_tuning(ctx, old["gemm_prefetch"], W, 0)
        dX = torch.zeros((3, n, n), dtype=torch.complex128, device="cuda")
        negf.negf_zinv_batched(ctx, torch.from_numpy(A.copy()).cuda(), dX)
        assert negf.negf_sync_status(ctx) == 0
    finally:
        negf.negf_set_tuning(ctx, old["gemm_prefetch"], old["inv_outer"], old["inv_mid"])
    X = dX.cpu().numpy()
    for b in range(3):
        # normwise forward error of a backward-stable inverse: ~ n u cond(A)
        cond = _cond(A[b], ref[b])
        err = np.max(np.abs(X[b] - ref[b])) / np.max(np.abs(ref[b]))
        _say(f"  case {b}: err {err:.2e} cond {cond:.1e}")
        assert err < 1e-14 * cond * n + 1e-13, (b, err, cond)


@pytest.mark.parametrize("n", [513, 1024, 1200, 1537, 2048])
def test_zinv_fp32_large(ctx, n):
    from paper_1510_04686_amd import negf
    _say(f"zinv fp32 n={n}")
    rng = np.random.default_rng(9500 + n)
    A = _rand(rng, (2, n, n), np.complex64) + np.float32(np.sqrt(n)) * np.eye(n, dtype=np.complex64)
    ref = np.linalg.inv(A.astype(np.complex128))
    dX = torch.zeros((2, n, n), dtype=torch.complex64, device="cuda")
    negf.negf_zinv_batched(ctx, torch.from_numpy(A.copy()).cuda(), dX)
    assert negf.negf_sync_status(ctx) == 0
    X = dX.cpu().numpy()
    for b in range(2):
        cond = _cond(A[b], ref[b])
        err = np.max(np.abs(X[b] - ref[b])) / np.max(np.abs(ref[b]))
        _say(f"  case {b}: err {err:.2e} cond {cond:.1e}")
        assert err < 1e-6 * cond * np.sqrt(n), (b, err, cond)


@pytest.mark.parametrize("n", [513, 1200, 2048])
@pytest.mark.parametrize("opa,opb", [(0, 0), (0, 1), (1, 0)])
def test_zgemm_large(ctx, n, opa, opb):
    from paper_1510_04686_amd import negf
    _say(f"zgemm n={n} op=({opa},{opb})")
    rng = np.random.default_rng(9900 + n + 3 * opa + opb)
    A, B = _rand(rng, (2, n, n)), _rand(rng, (2, n, n))
    opf = lambda a, op: a.conj().transpose(0, 2, 1) if op else a
    ref = opf(A, opa) @ opf(B, opb)
    for dt, tol in ((torch.complex128, 1e-13), (torch.complex64, 2e-6)):
        dA = torch.from_numpy(A).to(dt).cuda()
        dB = torch.from_numpy(B).to(dt).cuda()
        dC = torch.zeros_like(dA)
        negf.negf_zgemm_batched(ctx, dA, dB, dC, opa, opb)
        err = np.max(np.abs(dC.cpu().numpy() - ref)) / np.max(np.abs(ref))
        assert err < tol * np.sqrt(n), (dt, err)


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.fail(f"{path} missing: run tests/golden/make_golden.py")
    return np.load(path)


def test_block1200_slice_matches_oracle():
    """The block-1200 cross-section with its smooth potential, cut to 3 slabs:
    two energies against the stored oracle values, at 1e-10 or 10 x the
    point's FP64 drift (stored with the values)."""
    from make_golden import SLICE_PTS, inputs_sha1
    from paper_1510_04686_amd.runtime import RGFSolver
    _say("C5 cross-section (block 1200) x 3 slabs x 16 E vs oracle at 2 energies")
    g = _golden("c5_slice.npz")
    wl = make_workload("C5", n_slab=3)
    assert inputs_sha1(wl) == str(g["inputs_sha1"]), "input generator changed: rerun make_golden.py"
    s = RGFSolver(wl, tune="auto")
    out = s.solve(want_T=True)
    torch.cuda.synchronize()
    assert s.status() == 0 and s.lead_status == 0
    for i, pt in enumerate(SLICE_PTS):
        p = s.index[tuple(pt)]
        drift = {k: float(g[f"p{i}_drift_{k}"]) for k in ("GR", "GL", "GG", "bond", "T")}
        tols = {"drift": drift, **{k: max(P.TOL, P.FACTOR * v) for k, v in drift.items()}}
        _say(f"  point {list(pt)} tol GR {tols['GR']:.1e} GL {tols['GL']:.1e}")
        for k in ("GR", "GL", "GG"):
            P.check(pt, k, P.rel(out[k][p, :3].cpu().numpy(), g[f"p{i}_{k}"]), tols)
        bond = out["bond"][p, :2].cpu().numpy()
        P.check(pt, "bond", float(np.max(np.abs(bond - g[f"p{i}_bond"]))) / float(g[f"p{i}_bond_scale"]), tols)
        T = float(out["T"][p])
        P.check(pt, "T", abs(T - float(g[f"p{i}_T"])) / max(1.0, abs(float(g[f"p{i}_T"]))), tols)


def test_block1200_200_slabs_density_matches_oracle():
    """The full paper-shaped device (block 1200, 200 slabs, rank 240,000) at one
    energy: the electron density per atom (Eq. 7) and the orbital diagonals of
    G^R and G^< on sampled slabs against the stored oracle values."""
    from make_golden import inputs_sha1
    from paper_1510_04686_amd.runtime import RGFSolver
    _say("C5 (block 1200, 200 slabs) x 1 E: density and sampled diagonals vs oracle")
    g = _golden("c5_full.npz")
    wl = make_workload("C5", n_e=1)
    assert inputs_sha1(wl) == str(g["inputs_sha1"]), "input generator changed: rerun make_golden.py"
    s = RGFSolver(wl, tune="auto")
    out = s.solve(want=("GR", "GL"))
    n, _, _ = s.observables(out["GL"], None)
    torch.cuda.synchronize()
    assert s.status() == 0 and s.lead_status == 0
    sl = [int(x) for x in g["slabs"]]
    pt = (0, 0, 0)
    for k, got in (("n", n.cpu().numpy()), ("GR", out["GR"][0, sl].cpu().numpy()),
                   ("GL", out["GL"][0, sl].cpu().numpy())):
        drift = float(g[f"drift_{k}"])
        tol = max(P.TOL, P.FACTOR * drift)
        err = P.rel(got, g[k])
        _say(f"  {k}: err {err:.2e} tol {tol:.1e}")
        P.record(pt, k, err, tol, drift)
        assert err < tol, (k, err, tol)
