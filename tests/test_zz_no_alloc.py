"""GPU: the block inverse that allocates nothing (negf_zinv_batched_noalloc,
scratch in the library's static device array) against the context's
negf_zinv_batched with the same one-level scheme, through the C ABI."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _cases(rng, batch, n, dtype):
    A = rng.normal(size=(batch, n, n)) + 1j * rng.normal(size=(batch, n, n))
    A[0][np.diag_indices(n)] = 0                          # every pivot needs a row exchange
    if batch > 1:
        A[1] = np.eye(n)[rng.permutation(n)] + 1e-3 * A[1]
    return A.astype(dtype)


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_noalloc_inverse_matches_context_inverse(dtype):
    from paper_1510_04686_amd import negf
    tdt = torch.complex128 if dtype == np.complex128 else torch.complex64
    ctx = negf.negf_create(nb=400, n_slab_max=1, capacity=22)
    negf.negf_set_tuning(ctx, negf.negf_get_tuning(ctx)["gemm_prefetch"], 0, 0)   # one level, as the no-alloc path
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    free = []
    # two calls in a row, the second on a smaller input, then the first size again
    for call, (n, batch) in enumerate([(400, 22), (130, 7), (400, 22)]):
        _say(f"no-alloc inverse call {call}: n={n} batch={batch} {dtype.__name__}")
        assert negf.negf_zinv_noalloc_bytes(n, batch, tdt) <= negf.NOALLOC_SCRATCH_BYTES
        rng = np.random.default_rng(100 * call + n)
        A = _cases(rng, batch, n, dtype)
        X_ctx = torch.zeros((batch, n, n), dtype=tdt, device="cuda")
        negf.negf_zinv_batched(ctx, torch.from_numpy(A.copy()).cuda(), X_ctx)
        assert negf.negf_sync_status(ctx) == 0
        X_na = torch.full((batch, n, n), float("nan"), dtype=tdt, device="cuda")
        dA = torch.from_numpy(A.copy()).cuda()
        torch.cuda.synchronize()
        f0 = torch.cuda.mem_get_info()[0]
        negf.negf_zinv_batched_noalloc(dA, X_na, status)
        torch.cuda.synchronize()
        free.append((f0, torch.cuda.mem_get_info()[0]))
        assert int(status.item()) == 0
        a, b = X_na.cpu().numpy(), X_ctx.cpu().numpy()
        assert np.array_equal(a, b), float(np.max(np.abs(a - b)))
        ref = np.linalg.inv(A.astype(np.complex128))
        for q in range(batch):
            cond = np.linalg.cond(A[q].astype(np.complex128))
            err = np.max(np.abs(a[q] - ref[q])) / np.max(np.abs(ref[q]))
            bound = 1e-14 * cond * n + 1e-13 if dtype == np.complex128 else 1e-6 * cond * np.sqrt(n)
            assert err < bound, (q, err, cond)
    # after the first call has looked the array up, calls leave device memory as it was
    assert free[1][0] == free[1][1] and free[2][0] == free[2][1], free


def test_noalloc_inverse_flags_singular_and_rejects_oversize():
    from paper_1510_04686_amd import negf
    _say("no-alloc inverse: singular flag, size limit")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    Z = torch.zeros((2, 16, 16), dtype=torch.complex128, device="cuda")
    negf.negf_zinv_batched_noalloc(Z, torch.zeros_like(Z), status)
    torch.cuda.synchronize()
    assert int(status.item()) in (1, 2, 3)
    big = 1
    while negf.negf_zinv_noalloc_bytes(400, big + 1) <= negf.NOALLOC_SCRATCH_BYTES:
        big += 1
    A = torch.zeros((big + 1, 400, 400), dtype=torch.complex128, device="cuda")
    with pytest.raises(negf.NegfError) as e:
        negf.negf_zinv_batched_noalloc(A, torch.zeros_like(A))
    assert e.value.code == -2                       # NEGF_ESHAPE, nothing launched
