"""GPU: the two dense block kernels (batched complex GEMM on MFMA, batched
Gauss-Jordan inverse) against NumPy, through the C ABI."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    from paper_1510_04686_amd import negf
    return negf.negf_create(nb=416, n_slab_max=1, capacity=6)


def _rand(rng, shape, dtype=np.complex128):
    return (rng.normal(size=shape) + 1j * rng.normal(size=shape)).astype(dtype)


def _op(a, op):
    return a.conj().transpose(0, 2, 1) if op else a


@pytest.mark.parametrize("n", [1, 3, 16, 17, 64, 65, 100, 130, 400])
@pytest.mark.parametrize("opa,opb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_zgemm_fp64(ctx, n, opa, opb):
    from paper_1510_04686_amd import negf
    _say(f"zgemm fp64 n={n} op=({opa},{opb})")
    rng = np.random.default_rng(n * 10 + opa * 2 + opb)
    A, B = _rand(rng, (3, n, n)), _rand(rng, (3, n, n))
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.zeros_like(dA)
    negf.negf_zgemm_batched(ctx, dA, dB, dC, opa, opb)
    ref = _op(A, opa) @ _op(B, opb)
    err = np.max(np.abs(dC.cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert err < 1e-13 * max(1, np.sqrt(n)), err


@pytest.mark.parametrize("n", [5, 64, 100, 400])
@pytest.mark.parametrize("opa,opb", [(0, 0), (0, 1)])
def test_zgemm_fp32(ctx, n, opa, opb):
    from paper_1510_04686_amd import negf
    _say(f"zgemm fp32 n={n} op=({opa},{opb})")
    rng = np.random.default_rng(n + 7)
    A, B = _rand(rng, (2, n, n), np.complex64), _rand(rng, (2, n, n), np.complex64)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    dC = torch.zeros_like(dA)
    negf.negf_zgemm_batched(ctx, dA, dB, dC, opa, opb)
    ref = _op(A.astype(np.complex128), opa) @ _op(B.astype(np.complex128), opb)
    err = np.max(np.abs(dC.cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert err < 2e-6 * max(1, np.sqrt(n)), err


# 128/129/256/257/400/416 cover the two-level scheme (outer panels of 128 columns,
# a ragged last outer panel, a last inner panel narrower than 32)
@pytest.mark.parametrize("n", [1, 2, 5, 16, 17, 33, 64, 65, 100, 128, 129, 130, 256, 257, 400, 416])
def test_zinv_fp64(ctx, n):
    from paper_1510_04686_amd import negf
    _say(f"zinv fp64 n={n}")
    rng = np.random.default_rng(1000 + n)
    A = _rand(rng, (4, n, n))
    # matrices 2 and 3 need row exchanges: zero diagonal / permuted identity
    if n > 1:
        A[2][np.diag_indices(n)] = 0
    perm = rng.permutation(n)
    A[3] = np.eye(n)[perm] + 1e-3 * A[3]
    ref = np.linalg.inv(A)
    dA = torch.from_numpy(A.copy()).cuda()
    dX = torch.zeros_like(dA)
    negf.negf_zinv_batched(ctx, dA, dX)
    assert negf.negf_sync_status(ctx) == 0
    X = dX.cpu().numpy()
    for b in range(4):
        cond = np.linalg.cond(A[b])
        err = np.max(np.abs(X[b] - ref[b])) / np.max(np.abs(ref[b]))
        assert err < 1e-14 * cond * n + 1e-13, (b, err, cond)


@pytest.mark.parametrize("n", [7, 64, 100, 130, 300])
def test_zinv_fp32(ctx, n):
    from paper_1510_04686_amd import negf
    _say(f"zinv fp32 n={n}")
    rng = np.random.default_rng(2000 + n)
    A = _rand(rng, (2, n, n), np.complex64) + 4 * np.eye(n, dtype=np.complex64)
    ref = np.linalg.inv(A.astype(np.complex128))
    dA = torch.from_numpy(A.copy()).cuda()
    dX = torch.zeros_like(dA)
    negf.negf_zinv_batched(ctx, dA, dX)
    X = dX.cpu().numpy()
    for b in range(2):
        cond = np.linalg.cond(A[b])
        err = np.max(np.abs(X[b] - ref[b])) / np.max(np.abs(ref[b]))
        assert err < 1e-6 * cond * np.sqrt(n), (b, err, cond)


@pytest.mark.parametrize("W,Wm,n", [(128, 0, 300), (128, 64, 300), (192, 64, 400), (96, 32, 130)])
def test_zinv_fp32_outer_and_mid_widths(ctx, W, Wm, n):
    """FP32 (the mixed-precision path) through the two- and three-level schemes."""
    from paper_1510_04686_amd import negf
    _say(f"zinv fp32 outer {W} mid {Wm} n={n}")
    old = negf.negf_get_tuning(ctx)
    rng = np.random.default_rng(2500 + n + W + Wm)
    A = _rand(rng, (2, n, n), np.complex64) + 4 * np.eye(n, dtype=np.complex64)
    ref = np.linalg.inv(A.astype(np.complex128))
    try:
        negf.negf_set_tuning(ctx, old["gemm_prefetch"], W, Wm)
        dX = torch.zeros((2, n, n), dtype=torch.complex64, device="cuda")
        negf.negf_zinv_batched(ctx, torch.from_numpy(A.copy()).cuda(), dX)
        assert negf.negf_sync_status(ctx) == 0
    finally:
        negf.negf_set_tuning(ctx, old["gemm_prefetch"], old["inv_outer"], old["inv_mid"])
    X = dX.cpu().numpy()
    for b in range(2):
        cond = np.linalg.cond(A[b])
        err = np.max(np.abs(X[b] - ref[b])) / np.max(np.abs(ref[b]))
        assert err < 1e-6 * cond * np.sqrt(n), (b, err, cond)


def test_zinv_flags_singular_block(ctx):
    from paper_1510_04686_amd import negf
    _say("zinv singular")
    A = torch.zeros((1, 8, 8), dtype=torch.complex128, device="cuda")
    X = torch.zeros_like(A)
    negf.negf_zinv_batched(ctx, A, X)
    assert negf.negf_sync_status(ctx) in (2, 3)
    assert negf.negf_sync_status(ctx) == 0     # cleared by the previous read


def test_zinv_rejects_oversized(ctx):
    from paper_1510_04686_amd import negf
    A = torch.zeros((1, 420, 420), dtype=torch.complex128, device="cuda")
    with pytest.raises(negf.NegfError):
        negf.negf_zinv_batched(ctx, A, torch.zeros_like(A))


def test_tuning_validation_and_roundtrip(ctx):
    from paper_1510_04686_amd import negf
    _say("tuning set/get")
    old = negf.negf_get_tuning(ctx)
    for bad in ((0, 128), (4, 128), (2, 32), (2, 100), (2, 288), (2, 128, 16), (2, 128, 48), (2, 128, 288)):
        with pytest.raises(negf.NegfError):
            negf.negf_set_tuning(ctx, *bad)
    negf.negf_set_tuning(ctx, 1, 64)
    assert negf.negf_get_tuning(ctx) == {"gemm_prefetch": 1, "inv_outer": 64, "inv_mid": 0}
    negf.negf_set_tuning(ctx, 3, 192, 64)
    assert negf.negf_get_tuning(ctx) == {"gemm_prefetch": 3, "inv_outer": 192, "inv_mid": 64}
    negf.negf_set_tuning(ctx, old["gemm_prefetch"], old["inv_outer"], old["inv_mid"])


@pytest.mark.parametrize("W,Wm,n", [(0, 0, 400), (64, 0, 400), (96, 0, 400), (192, 0, 400), (256, 0, 400),
                                    (128, 64, 400), (192, 64, 400), (256, 64, 400), (256, 128, 400),
                                    (96, 32, 400), (128, 64, 416), (128, 64, 300), (192, 64, 130)])
def test_zinv_every_outer_width(ctx, W, Wm, n):
    """Each outer panel width, with and without mid blocks (three levels), and
    the one-level scheme give the same inverse; 416 and 300 merge a remainder
    into the last outer panel (300: its last mid block ends in a 12-column
    panel that is not fused)."""
    from paper_1510_04686_amd import negf
    _say(f"zinv outer width {W}, mid {Wm}, n={n}")
    old = negf.negf_get_tuning(ctx)
    rng = np.random.default_rng(3000 + W + 7 * Wm + n)
    A = _rand(rng, (3, n, n))
    A[1][np.diag_indices(n)] = 0
    ref = np.linalg.inv(A)
    try:
        negf.negf_set_tuning(ctx, old["gemm_prefetch"], W, Wm)
        dX = torch.zeros((3, n, n), dtype=torch.complex128, device="cuda")
        negf.negf_zinv_batched(ctx, torch.from_numpy(A.copy()).cuda(), dX)
        assert negf.negf_sync_status(ctx) == 0
    finally:
        negf.negf_set_tuning(ctx, old["gemm_prefetch"], old["inv_outer"], old["inv_mid"])
    X = dX.cpu().numpy()
    for b in range(3):
        err = np.max(np.abs(X[b] - ref[b])) / np.max(np.abs(ref[b]))
        assert err < 1e-14 * np.linalg.cond(A[b]) * n + 1e-13, (b, err)


@pytest.mark.parametrize("pf", [1, 2, 3])
@pytest.mark.parametrize("n", [16, 17, 100, 400])
def test_zgemm_prefetch_depths_agree(ctx, pf, n):
    from paper_1510_04686_amd import negf
    _say(f"zgemm prefetch {pf} n={n}")
    old = negf.negf_get_tuning(ctx)
    rng = np.random.default_rng(4000 + n)
    A, B = _rand(rng, (2, n, n)), _rand(rng, (2, n, n))
    dC = torch.zeros((2, n, n), dtype=torch.complex128, device="cuda")
    try:
        negf.negf_set_tuning(ctx, pf, old["inv_outer"])
        negf.negf_zgemm_batched(ctx, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), dC, 0, 1)
    finally:
        negf.negf_set_tuning(ctx, old["gemm_prefetch"], old["inv_outer"], old["inv_mid"])
    ref = A @ B.conj().transpose(0, 2, 1)
    assert np.max(np.abs(dC.cpu().numpy() - ref)) / np.max(np.abs(ref)) < 1e-13 * np.sqrt(n)


def test_autotune_returns_a_valid_choice():
    from paper_1510_04686_amd import negf
    _say("autotune")
    c = negf.negf_create(nb=200, n_slab_max=1, capacity=4)
    t = negf.negf_autotune(c, reps=1)
    assert t["gemm_prefetch"] in (1, 2, 3)
    assert t["inv_outer"] == 0 or (64 <= t["inv_outer"] < 200 and t["inv_outer"] % 32 == 0)
    assert t["inv_mid"] in (0, 64, 128)
    assert negf.negf_get_tuning(c) == t


@pytest.mark.parametrize("n,batch", [(65, 300), (100, 160), (400, 12)])
def test_zgemm_persistent_walks_many_tiles(n, batch):
    """The persistent form (prefetch 3) with far more output tiles than
    resident workgroups, so each workgroup carries its K pipeline across
    several tiles (edge tiles included at n = 65): every operand form must
    equal the per-tile kernel bit for bit, and NumPy on sampled entries."""
    from paper_1510_04686_amd import negf
    _say(f"persistent zgemm n={n} batch={batch}")
    c = negf.negf_create(nb=n, n_slab_max=1, capacity=batch)
    rng = np.random.default_rng(7000 + n)
    A = torch.from_numpy(_rand(rng, (batch, n, n))).cuda()
    B = torch.from_numpy(_rand(rng, (batch, n, n))).cuda()
    for opa, opb in [(0, 0), (0, 1), (1, 0)]:
        out = {}
        for pf in (2, 3):
            negf.negf_set_tuning(c, pf, negf.negf_get_tuning(c)["inv_outer"])
            C = torch.zeros_like(A)
            negf.negf_zgemm_batched(c, A, B, C, opa, opb)
            torch.cuda.synchronize()
            out[pf] = C.cpu().numpy()
        assert np.array_equal(out[2], out[3]), (opa, opb)
        idx = rng.choice(batch, size=3, replace=False)
        a, b = A.cpu().numpy()[idx], B.cpu().numpy()[idx]
        ref = _op(a, opa) @ _op(b, opb)
        assert np.max(np.abs(out[3][idx] - ref)) / np.max(np.abs(ref)) < 1e-13 * np.sqrt(n)
    del c


def test_gemm_timing_filters_by_matrix_core_precision(ctx):
    """Timing mode "fp64" records only FP64 products and "fp32" only FP32 ones,
    each with the algorithmic 8 n^3 flops per point; mode 1 records both."""
    from paper_1510_04686_amd import negf
    _say("gemm timing filter")
    n, batch = 100, 3
    rng = np.random.default_rng(11)
    A64 = torch.from_numpy(_rand(rng, (batch, n, n))).cuda()
    A32 = A64.to(torch.complex64)
    C64, C32 = torch.empty_like(A64), torch.empty_like(A32)
    for mode, want in (("fp64", (1, 0)), ("fp32", (0, 1)), ("all", (1, 1))):
        negf.negf_gemm_timing_enable(ctx, mode)
        negf.negf_zgemm_batched(ctx, A64, A64, C64, 0, 0)
        negf.negf_zgemm_batched(ctx, A32, A32, C32, 0, 0)
        launches, ms, flops = negf.negf_gemm_timing(ctx)
        assert launches == sum(want), (mode, launches)
        assert flops == pytest.approx(8.0 * n ** 3 * batch * sum(want)), mode
        assert ms > 0
    negf.negf_gemm_timing_enable(ctx, False)
    assert negf.lib().negf_gemm_timing_enable(ctx.handle, 4) == -1   # NEGF_EINVAL
