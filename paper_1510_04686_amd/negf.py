"""ctypes binding of the C ABI declared in include/negf.h.

Argument marshalling only: every function has the name of the C entry point it
calls, takes torch tensors already on the GPU, checks dtype / contiguity /
device, and passes raw pointers.  No arithmetic of the method happens here.
The library must have been built (paper_1510_04686_amd.build); loading fails
loudly otherwise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_longlong, c_void_p

import torch

from .build import LIB_PATH, sources_sha1

_lib = None

NEGF_FP64 = 0
NEGF_MIXED = 1
NEGF_WANT_TRANSMISSION = 1
NEGF_WNOCONV, NEGF_WSINGULAR, NEGF_WNONFINITE, NEGF_WFALLBACK = 1, 2, 3, 4

STATUS = {0: "OK", -1: "EINVAL", -2: "ESHAPE", -3: "ENOMEM", -4: "EHIP", -5: "ESTATE",
          1: "WNOCONV", 2: "WSINGULAR", 3: "WNONFINITE", 4: "WFALLBACK"}


class NegfError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {STATUS.get(code, code)} ({lib().negf_error_string(code).decode()})")
        self.code = code


class negf_config(ctypes.Structure):
    _fields_ = [("nb", c_int), ("n_slab_max", c_int), ("capacity", c_int), ("precision", c_int),
                ("adjoint_segment", c_int), ("store_checkpoint", c_int)]


class negf_tuning(ctypes.Structure):
    _fields_ = [("gemm_prefetch", c_int), ("inv_outer", c_int), ("inv_mid", c_int)]


class negf_system(ctypes.Structure):
    _fields_ = [
        ("nb", c_int), ("n_samples", c_int), ("slab_offset", POINTER(c_longlong)),
        ("n_k", c_int), ("n_e", c_int),
        ("h_diag", c_void_p), ("h_up", c_void_p), ("h_up_k_stride", c_longlong), ("up_block", c_int),
        ("v_onsite", c_void_p), ("energy", c_void_p),
        ("eta", c_double), ("mu_L", c_double), ("mu_R", c_double), ("kT", c_double),
        ("eta_fill", c_int),
    ]


class negf_poisson_grid(ctypes.Structure):
    _fields_ = [
        ("n_x", c_int), ("n_z", c_int), ("n_y", c_int), ("z_gate", c_int),
        ("v_left", c_double), ("v_right", c_double), ("v_gate", c_double),
    ]


EXPORTS = [
    "negf_create", "negf_destroy", "negf_workspace_bytes", "negf_sync_status", "negf_error_string",
    "negf_bind", "negf_lead_selfenergy", "negf_lead_selfenergy_pair", "negf_rgf_forward", "negf_rgf_backward",
    "negf_scba_selfenergy", "negf_observables", "negf_rgf_adjoint", "negf_zgemm_batched", "negf_zinv_batched", "negf_mixed_stats",
    "negf_set_mixed_threshold", "negf_mixed_point_residuals", "negf_mixed_point_scores", "negf_cap_selfenergy", "negf_set_scattering_blocks", "negf_transpose_batched", "negf_density_jacobian_local", "negf_gemm_timing_enable", "negf_gemm_timing", "negf_get_tuning", "negf_set_tuning", "negf_autotune",
    "negf_build_id", "negf_scba_history", "negf_rgf_solve", "negf_zinv_noalloc_bytes", "negf_zinv_batched_noalloc",
    "negf_poisson_apply", "negf_poisson_residual", "negf_poisson_work_bytes", "negf_poisson_solve",
    "negf_vec_work_bytes", "negf_vec_dots", "negf_vec_combine", "negf_vec_norms",
]


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} missing (run paper_1510_04686_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    L.negf_build_id.restype = ctypes.c_char_p
    L.negf_build_id.argtypes = []
    built, now = L.negf_build_id().decode(), sources_sha1()
    if built != now:
        raise RuntimeError(f"HIP library {LIB_PATH} is stale: built from sources {built[:12]}, the sources are now "
                           f"{now[:12]} (run paper_1510_04686_amd.build)")
    vp, i, d, ll = c_void_p, c_int, c_double, c_longlong
    sig = {
        "negf_create": (i, [POINTER(negf_config), POINTER(vp)]),
        "negf_destroy": (None, [vp]),
        "negf_workspace_bytes": (ll, [vp]),
        "negf_sync_status": (i, [vp, vp]),
        "negf_error_string": (ctypes.c_char_p, [i]),
        "negf_bind": (i, [vp, POINTER(negf_system), i, POINTER(c_int)]),
        "negf_lead_selfenergy": (i, [vp, vp, i, vp, vp, vp, i, vp, d, d, i, vp, vp]),
        "negf_lead_selfenergy_pair": (i, [vp, vp, i, vp, vp, vp, vp, vp, i, vp, d, d, i, vp, vp, vp, vp, vp]),
        "negf_rgf_forward": (i, [vp, vp, i, i, vp, vp, vp, vp, i]),
        "negf_rgf_backward": (i, [vp, vp, i, i, vp, vp, vp, i, i, vp, vp]),
        "negf_rgf_solve": (i, [vp, vp, i, i, vp, vp, vp, vp, i, vp, vp, vp, i, i, vp, vp]),
        "negf_scba_selfenergy": (i, [vp, vp, vp, vp, i, vp, d, d, i, d, vp, vp, vp]),
        "negf_observables": (i, [vp, vp, vp, vp, i, vp, vp, d, i, vp, vp, vp, i]),
        "negf_set_scattering_blocks": (i, [vp, i]),
        "negf_transpose_batched": (i, [vp, i, i, vp, ll, vp, ll]),
        "negf_scba_history": (i, [vp, vp, POINTER(d), i, POINTER(i)]),
        "negf_rgf_adjoint": (i, [vp, vp, i, i, vp, vp, i]),
        "negf_zgemm_batched": (i, [vp, vp, i, i, i, i, vp, vp, vp, i]),
        "negf_zinv_batched": (i, [vp, vp, i, i, vp, vp, i]),
        "negf_zinv_noalloc_bytes": (ll, [i, i, i]),
        "negf_zinv_batched_noalloc": (i, [vp, i, i, vp, vp, i, vp]),
        "negf_mixed_stats": (i, [vp, vp, POINTER(ll), POINTER(d)]),
        "negf_set_mixed_threshold": (i, [vp, d]),
        "negf_mixed_point_residuals": (i, [vp, vp, i, vp]),
        "negf_mixed_point_scores": (i, [vp, vp, vp, i, vp, vp, vp, vp]),
        "negf_cap_selfenergy": (i, [vp, vp, vp, vp, vp, vp]),
        "negf_gemm_timing_enable": (i, [vp, i]),
        "negf_gemm_timing": (i, [vp, vp, POINTER(ll), POINTER(d), POINTER(d), POINTER(d)]),
        "negf_get_tuning": (i, [vp, POINTER(negf_tuning)]),
        "negf_set_tuning": (i, [vp, POINTER(negf_tuning)]),
        "negf_autotune": (i, [vp, vp, i, POINTER(negf_tuning)]),
        "negf_poisson_apply": (i, [vp, POINTER(negf_poisson_grid), vp, i, vp]),
        "negf_poisson_residual": (i, [vp, POINTER(negf_poisson_grid), vp, vp, vp, d, vp]),
        "negf_poisson_work_bytes": (ll, [POINTER(negf_poisson_grid)]),
        "negf_poisson_solve": (i, [vp, POINTER(negf_poisson_grid), vp, vp, vp, d, i, vp, POINTER(i), POINTER(d)]),
        "negf_density_jacobian_local": (i, [vp, vp, vp, vp, i, vp, vp, d, i, vp]),
        "negf_vec_work_bytes": (ll, [ll, i]),
        "negf_vec_dots": (i, [vp, ll, i, vp, ll, vp, vp, vp]),
        "negf_vec_combine": (i, [vp, ll, i, vp, ll, vp, d, vp]),
        "negf_vec_norms": (i, [vp, ll, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(fn, code, warn_ok=False):
    if code < 0 or (code > 0 and not warn_ok):
        raise NegfError(fn, code)
    return code


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t.data_ptr()


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return c_void_p(s.cuda_stream)


class Context:
    """Owns a negf_ctx handle (negf_create / negf_destroy)."""

    def __init__(self, handle, cfg):
        self.handle = handle
        self.cfg = cfg
        self._keep = []

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                lib().negf_destroy(h)
            except Exception:
                pass
            self.handle = None


def negf_create(nb, n_slab_max, capacity, precision=NEGF_FP64, adjoint_segment=0, store_checkpoint=0):
    cfg = negf_config(nb, n_slab_max, capacity, precision, adjoint_segment, int(store_checkpoint))
    h = c_void_p()
    _check("negf_create", lib().negf_create(ctypes.byref(cfg), ctypes.byref(h)))
    return Context(h, cfg)


def negf_workspace_bytes(ctx):
    return int(lib().negf_workspace_bytes(ctx.handle))


def negf_sync_status(ctx, stream=None):
    return int(lib().negf_sync_status(ctx.handle, _stream(stream)))


def negf_bind(ctx, nb, slab_offset, n_k, n_e, h_diag, h_up, h_up_k_stride, up_block, v_onsite, energy,
              eta, mu_L, mu_R, kT, eta_fill, points):
    """slab_offset and points are host sequences; the tensors are device tensors
    kept alive by the context while bound."""
    import numpy as np
    off = np.ascontiguousarray(np.asarray(slab_offset, dtype=np.int64))
    pts = np.ascontiguousarray(np.asarray(points, dtype=np.int32).reshape(-1, 3))
    sys_ = negf_system(
        nb, len(off) - 1, off.ctypes.data_as(POINTER(c_longlong)), n_k, n_e,
        _ptr(h_diag, torch.complex128, "h_diag"), _ptr(h_up, torch.complex128, "h_up"), int(h_up_k_stride),
        int(up_block), _ptr(v_onsite, torch.float64, "v_onsite"), _ptr(energy, torch.float64, "energy"),
        float(eta), float(mu_L), float(mu_R), float(kT), int(eta_fill))
    code = lib().negf_bind(ctx.handle, ctypes.byref(sys_), len(pts), pts.ctypes.data_as(POINTER(c_int)))
    _check("negf_bind", code)
    ctx._keep = [h_diag, h_up, v_onsite, energy]


def negf_lead_selfenergy(ctx, h00, h01, tau, energy, eta, tol, max_iter, sigma, iters=None, stream=None):
    n_k = h00.shape[0]
    n_e = energy.shape[0]
    code = lib().negf_lead_selfenergy(
        ctx.handle, _stream(stream), n_k, _ptr(h00, torch.complex128, "h00"), _ptr(h01, torch.complex128, "h01"),
        _ptr(tau, torch.complex128, "tau"), n_e, _ptr(energy, torch.float64, "energy"), float(eta), float(tol),
        int(max_iter), _ptr(sigma, torch.complex128, "sigma"), _ptr(iters, torch.int32, "iters"))
    return _check("negf_lead_selfenergy", code, warn_ok=True)


def negf_lead_selfenergy_pair(ctx, h00, h01_L, tau_L, h01_R, tau_R, energy, eta, tol, max_iter, sigma_L, sigma_R,
                              iters_L=None, iters_R=None, stream=None):
    """Returns (status, dual_used)."""
    n_k = h00.shape[0]
    n_e = energy.shape[0]
    used = ctypes.c_int(0)
    code = lib().negf_lead_selfenergy_pair(
        ctx.handle, _stream(stream), n_k, _ptr(h00, torch.complex128, "h00"),
        _ptr(h01_L, torch.complex128, "h01_L"), _ptr(tau_L, torch.complex128, "tau_L"),
        _ptr(h01_R, torch.complex128, "h01_R"), _ptr(tau_R, torch.complex128, "tau_R"), n_e,
        _ptr(energy, torch.float64, "energy"), float(eta), float(tol), int(max_iter),
        _ptr(sigma_L, torch.complex128, "sigma_L"), _ptr(sigma_R, torch.complex128, "sigma_R"),
        _ptr(iters_L, torch.int32, "iters_L"), _ptr(iters_R, torch.int32, "iters_R"), ctypes.byref(used))
    return _check("negf_lead_selfenergy_pair", code, warn_ok=True), used.value


def negf_rgf_forward(ctx, p0, np_, sigma_L, sigma_R, scat_R=None, scat_L=None, flags=0, stream=None):
    code = lib().negf_rgf_forward(
        ctx.handle, _stream(stream), int(p0), int(np_), _ptr(sigma_L, torch.complex128, "sigma_L"),
        _ptr(sigma_R, torch.complex128, "sigma_R"), _ptr(scat_R, torch.complex128, "scat_R"),
        _ptr(scat_L, torch.complex128, "scat_L"), int(flags))
    _check("negf_rgf_forward", code)


def negf_rgf_backward(ctx, p0, np_, GR=None, GL=None, GG=None, full_blocks=0, slab_stride=1, bond_j=None,
                      transmission=None, stream=None):
    code = lib().negf_rgf_backward(
        ctx.handle, _stream(stream), int(p0), int(np_), _ptr(GR, torch.complex128, "GR"),
        _ptr(GL, torch.complex128, "GL"), _ptr(GG, torch.complex128, "GG"), int(full_blocks), int(slab_stride),
        _ptr(bond_j, torch.float64, "bond_j"), _ptr(transmission, torch.float64, "transmission"))
    _check("negf_rgf_backward", code)


def negf_scba_selfenergy(ctx, GR, GL, slab_stride, w_k, D_ac, M_op, shift, n_bose, sig_R, sig_L, rel_change=None,
                         stream=None):
    code = lib().negf_scba_selfenergy(
        ctx.handle, _stream(stream), _ptr(GR, torch.complex128, "GR"), _ptr(GL, torch.complex128, "GL"),
        int(slab_stride), _ptr(w_k, torch.float64, "w_k"), float(D_ac), float(M_op), int(shift), float(n_bose),
        _ptr(sig_R, torch.complex128, "sig_R"), _ptr(sig_L, torch.complex128, "sig_L"),
        _ptr(rel_change, torch.float64, "rel_change"))
    _check("negf_scba_selfenergy", code)


def negf_rgf_solve(ctx, p0, np_, sigma_L, sigma_R, scat_R=None, scat_L=None, flags=0, GR=None, GL=None, GG=None,
                   full_blocks=0, slab_stride=1, bond_j=None, transmission=None, stream=None):
    """negf_rgf_forward + negf_rgf_backward in one call (one persistent launch
    for blocks of at most 8 orbitals)."""
    code = lib().negf_rgf_solve(
        ctx.handle, _stream(stream), int(p0), int(np_), _ptr(sigma_L, torch.complex128, "sigma_L"),
        _ptr(sigma_R, torch.complex128, "sigma_R"), _ptr(scat_R, torch.complex128, "scat_R"),
        _ptr(scat_L, torch.complex128, "scat_L"), int(flags), _ptr(GR, torch.complex128, "GR"),
        _ptr(GL, torch.complex128, "GL"), _ptr(GG, torch.complex128, "GG"), int(full_blocks), int(slab_stride),
        _ptr(bond_j, torch.float64, "bond_j"), _ptr(transmission, torch.float64, "transmission"))
    _check("negf_rgf_solve", code)


def negf_scba_history(ctx, max_n=4096, stream=None):
    """Residuals ||dSigma|| / ||Sigma|| of the negf_scba_selfenergy calls since the
    last read, oldest first (synchronises the stream and clears the list)."""
    buf = (c_double * max_n)()
    n = c_int(0)
    _check("negf_scba_history", lib().negf_scba_history(ctx.handle, _stream(stream), buf, int(max_n),
                                                         ctypes.byref(n)))
    return [float(buf[j]) for j in range(min(n.value, max_n))]


def negf_observables(ctx, GL, bond_j, slab_stride, w_e, w_k, g_s, orbs_per_atom, n=None, J=None, j_E=None,
                     stream=None, gl_opa=1):
    """Density / current sums; GL holds orbital diagonals (gl_opa = 1) or atom
    blocks [p][slab_stride][nb][gl_opa]."""
    code = lib().negf_observables(
        ctx.handle, _stream(stream), _ptr(GL, torch.complex128, "GL"), _ptr(bond_j, torch.float64, "bond_j"),
        int(slab_stride), _ptr(w_e, torch.float64, "w_e"), _ptr(w_k, torch.float64, "w_k"), float(g_s),
        int(orbs_per_atom), _ptr(n, torch.float64, "n"), _ptr(J, torch.float64, "J"),
        _ptr(j_E, torch.float64, "j_E"), int(gl_opa))
    _check("negf_observables", code)


def negf_transpose_batched(src, dst, stream=None):
    """dst[m] = src[m]^T for [count][n][n] complex128 device tensors (distinct buffers)."""
    n = src.shape[-1]
    count = src.numel() // (n * n)
    if src.shape != dst.shape or src.shape[-2] != n:
        raise ValueError("src and dst must be [..., n, n] of one shape")
    _check("negf_transpose_batched",
           lib().negf_transpose_batched(_stream(stream), int(n), int(count), _ptr(src, torch.complex128, "src"),
                                        n * n, _ptr(dst, torch.complex128, "dst"), n * n))


def negf_set_scattering_blocks(ctx, opa):
    """Orbital-diagonal (opa = 1) or atom-block (opa > 1) scattering self-energies."""
    _check("negf_set_scattering_blocks", lib().negf_set_scattering_blocks(ctx.handle, int(opa)))


def negf_rgf_adjoint(ctx, p0, np_, w_orb, dX, slab_stride, stream=None):
    """dX[p][i][o] = 2 (G^< W G^R)_oo for the points of the preceding forward sweep."""
    code = lib().negf_rgf_adjoint(ctx.handle, _stream(stream), int(p0), int(np_), _ptr(w_orb, torch.float64, "w_orb"),
                                  _ptr(dX, torch.complex128, "dX"), int(slab_stride))
    _check("negf_rgf_adjoint", code)


def _cdt(t):
    if t.dtype == torch.complex128:
        return 0
    if t.dtype == torch.complex64:
        return 1
    raise TypeError("complex128 or complex64 expected")


def negf_zgemm_batched(ctx, A, B, C, opa=0, opb=0, stream=None):
    """C[b] = op(A[b]) op(B[b]) for [batch, n, n] tensors of one complex dtype."""
    batch, n = A.shape[0], A.shape[-1]
    dt = A.dtype
    code = lib().negf_zgemm_batched(ctx.handle, _stream(stream), int(n), int(batch), int(opa), int(opb),
                                    _ptr(A, dt, "A"), _ptr(B, dt, "B"), _ptr(C, dt, "C"), _cdt(A))
    _check("negf_zgemm_batched", code)


def negf_zinv_batched(ctx, A, Ainv, stream=None):
    """Ainv[b] = A[b]^-1 ([batch, n, n]); A is overwritten."""
    batch, n = A.shape[0], A.shape[-1]
    dt = A.dtype
    code = lib().negf_zinv_batched(ctx.handle, _stream(stream), int(n), int(batch), _ptr(A, dt, "A"),
                                   _ptr(Ainv, dt, "Ainv"), _cdt(A))
    _check("negf_zinv_batched", code)


NOALLOC_SCRATCH_BYTES = 64 << 20   # NEGF_NOALLOC_SCRATCH_BYTES


def negf_zinv_noalloc_bytes(n, batch, dtype=torch.complex128):
    return int(lib().negf_zinv_noalloc_bytes(int(n), int(batch), _cdt(torch.empty(0, dtype=dtype))))


def negf_zinv_batched_noalloc(A, Ainv, status=None, stream=None):
    """Ainv[b] = A[b]^-1 without a context: scratch in the library's static
    device array (no allocation).  `status` (device int32 tensor of one element
    or None) receives the OR of the pivot status bits."""
    batch, n = A.shape[0], A.shape[-1]
    dt = A.dtype
    code = lib().negf_zinv_batched_noalloc(_stream(stream), int(n), int(batch), _ptr(A, dt, "A"),
                                           _ptr(Ainv, dt, "Ainv"), _cdt(A), _ptr(status, torch.int32, "status"))
    _check("negf_zinv_batched_noalloc", code)


def negf_mixed_stats(ctx, stream=None):
    nf = c_longlong()
    mr = c_double()
    _check("negf_mixed_stats", lib().negf_mixed_stats(ctx.handle, _stream(stream), ctypes.byref(nf), ctypes.byref(mr)))
    return int(nf.value), float(mr.value)


def negf_set_mixed_threshold(ctx, thr):
    """Refinement residual ||I - A X0||_F above which a mixed-precision block
    inverse is redone in FP64 (0: always, inf: only non-finite residuals)."""
    _check("negf_set_mixed_threshold", lib().negf_set_mixed_threshold(ctx.handle, float(thr)))


def negf_mixed_point_residuals(ctx, out, n=None, stream=None):
    """Per-point largest refinement residual of the last mixed forward sweep
    into the float64 device tensor `out` (first n points of the batch)."""
    n = out.numel() if n is None else int(n)
    _check("negf_mixed_point_residuals",
           lib().negf_mixed_point_residuals(ctx.handle, _stream(stream), n, _ptr(out, torch.float64, "out")))


def negf_cap_selfenergy(ctx, w_slab, side, scat_R, scat_L, stream=None):
    """Absorbing-contact self-energies into scat_R / scat_L [n_e][total_slabs][nb]."""
    _check("negf_cap_selfenergy",
           lib().negf_cap_selfenergy(ctx.handle, _stream(stream), _ptr(w_slab, torch.float64, "w_slab"),
                                     _ptr(side, torch.int32, "side"), _ptr(scat_R, torch.complex128, "scat_R"),
                                     _ptr(scat_L, torch.complex128, "scat_L")))


def negf_mixed_point_scores(ctx, GL, slab_stride, w_e, w_k, resid, score, stream=None):
    """Redo score of every bound point into the float64 device tensor `score`:
    residual x quadrature weight x largest |Im G^<_jj| of the point."""
    _check("negf_mixed_point_scores",
           lib().negf_mixed_point_scores(ctx.handle, _stream(stream), _ptr(GL, torch.complex128, "GL"),
                                         int(slab_stride), _ptr(w_e, torch.float64, "w_e"),
                                         _ptr(w_k, torch.float64, "w_k"), _ptr(resid, torch.float64, "resid"),
                                         _ptr(score, torch.float64, "score")))


# ------------------------------------------------------------------ Poisson (Eq. 9)
def poisson_grid(n_x, n_z, n_y, z_gate=False, v_left=0.0, v_right=0.0, v_gate=0.0):
    return negf_poisson_grid(int(n_x), int(n_z), int(n_y), int(bool(z_gate)), float(v_left), float(v_right),
                             float(v_gate))


def _vec(t, n, name):
    p = _ptr(t, torch.float64, name)
    if t.numel() != n:
        raise ValueError(f"{name} must hold {n} doubles, got {t.numel()}")
    return p


def _atoms(g):
    return g.n_x * g.n_z * g.n_y


def negf_poisson_apply(grid, V, out, with_boundary=True, stream=None):
    n = _atoms(grid)
    _check("negf_poisson_apply", lib().negf_poisson_apply(_stream(stream), ctypes.byref(grid), _vec(V, n, "V"),
                                                          int(bool(with_boundary)), _vec(out, n, "out")))


def negf_poisson_residual(grid, V, n_atom, n_d, beta, F, stream=None):
    n = _atoms(grid)
    _check("negf_poisson_residual",
           lib().negf_poisson_residual(_stream(stream), ctypes.byref(grid), _vec(V, n, "V"),
                                       _vec(n_atom, n, "n_atom"), _vec(n_d, n, "n_d"), float(beta),
                                       _vec(F, n, "F")))


def negf_poisson_work_bytes(grid):
    return int(lib().negf_poisson_work_bytes(ctypes.byref(grid)))


def negf_poisson_solve(grid, rhs, x, work, tol=1e-12, max_iter=10000, stream=None, shift=None):
    """x = (L0 + diag(shift))^-1 rhs (conjugate gradients); returns (iterations,
    relative residual)."""
    n = _atoms(grid)
    if work.numel() * work.element_size() < negf_poisson_work_bytes(grid):
        raise ValueError("work too small")
    it, rr = c_int(0), c_double(0.0)
    _check("negf_poisson_solve",
           lib().negf_poisson_solve(_stream(stream), ctypes.byref(grid),
                                    None if shift is None else _vec(shift, n, "shift"), _vec(rhs, n, "rhs"),
                                    _vec(x, n, "x"), float(tol), int(max_iter), _ptr(work, None, "work"),
                                    ctypes.byref(it), ctypes.byref(rr)))
    return it.value, rr.value


def negf_density_jacobian_local(ctx, GR, GL, slab_stride, w_e, w_k, g_s, orbs_per_atom, d_out, stream=None):
    """Per atom, the orbital-diagonal part of dn_a/dV_a into d_out [total_slabs][atoms]."""
    _check("negf_density_jacobian_local",
           lib().negf_density_jacobian_local(ctx.handle, _stream(stream), _ptr(GR, torch.complex128, "GR"),
                                             _ptr(GL, torch.complex128, "GL"), int(slab_stride),
                                             _ptr(w_e, torch.float64, "w_e"), _ptr(w_k, torch.float64, "w_k"),
                                             float(g_s), int(orbs_per_atom), _ptr(d_out, torch.float64, "d_out")))


def negf_vec_work_bytes(n, m):
    return int(lib().negf_vec_work_bytes(int(n), int(m)))


def _rows(X, m, n):
    p = _ptr(X, torch.float64, "X")
    if X.dim() != 2 or X.shape[0] < m or X.shape[1] != n:
        raise ValueError(f"X must be [>= {m}, {n}]")
    return p


def negf_vec_dots(X, m, y, out, work, stream=None):
    """out[:m] = X[:m] @ y on the device."""
    n = y.numel()
    if out.numel() < m or work.numel() * work.element_size() < negf_vec_work_bytes(n, m):
        raise ValueError("out / work too small")
    _check("negf_vec_dots", lib().negf_vec_dots(_stream(stream), n, int(m), _rows(X, m, n), n, _vec(y, n, "y"),
                                                _ptr(out, torch.float64, "out"), _ptr(work, None, "work")))


def negf_vec_norms(x, out, work, stream=None):
    """out[0] = x . x, out[1] = max |x_i| on the device."""
    n = x.numel()
    if out.numel() < 2 or work.numel() * work.element_size() < negf_vec_work_bytes(n, 1):
        raise ValueError("out / work too small")
    _check("negf_vec_norms", lib().negf_vec_norms(_stream(stream), n, _vec(x, n, "x"),
                                                  _ptr(out, torch.float64, "out"), _ptr(work, None, "work")))


def negf_vec_combine(X, m, c, b, y, stream=None):
    """y = b y + sum_j c[j] X[j] on the device."""
    n = y.numel()
    if m > 0 and c.numel() < m:
        raise ValueError("c too small")
    _check("negf_vec_combine", lib().negf_vec_combine(_stream(stream), n, int(m), _rows(X, m, n) if m else None, n,
                                                      _ptr(c, torch.float64, "c") if m else None, float(b),
                                                      _vec(y, n, "y")))


GEMM_TIMING = {False: 0, True: 1, "all": 1, "fp64": 2, "fp32": 3}


def negf_gemm_timing_enable(ctx, enable=True):
    """enable: False/True, or "all", "fp64", "fp32" (only launches on matrix cores of that precision)."""
    _check("negf_gemm_timing_enable", lib().negf_gemm_timing_enable(ctx.handle, GEMM_TIMING[enable]))


def negf_gemm_timing(ctx, stream=None, executed=False):
    """(launches, ms, algorithmic flops), plus the executed matrix-core flops
    when ``executed``."""
    n = c_longlong()
    ms = c_double()
    fl = c_double()
    ex = c_double()
    _check("negf_gemm_timing", lib().negf_gemm_timing(ctx.handle, _stream(stream), ctypes.byref(n),
                                                       ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(ex)))
    if executed:
        return int(n.value), float(ms.value), float(fl.value), float(ex.value)
    return int(n.value), float(ms.value), float(fl.value)


def negf_get_tuning(ctx):
    t = negf_tuning()
    _check("negf_get_tuning", lib().negf_get_tuning(ctx.handle, ctypes.byref(t)))
    return {"gemm_prefetch": int(t.gemm_prefetch), "inv_outer": int(t.inv_outer), "inv_mid": int(t.inv_mid)}


def negf_set_tuning(ctx, gemm_prefetch, inv_outer, inv_mid=0):
    t = negf_tuning(int(gemm_prefetch), int(inv_outer), int(inv_mid))
    _check("negf_set_tuning", lib().negf_set_tuning(ctx.handle, ctypes.byref(t)))


def negf_autotune(ctx, reps=3, stream=None):
    """Times the kernel-shape candidates on the context's workspace, applies the
    fastest and returns it as a dict."""
    t = negf_tuning()
    _check("negf_autotune", lib().negf_autotune(ctx.handle, _stream(stream), int(reps), ctypes.byref(t)))
    return {"gemm_prefetch": int(t.gemm_prefetch), "inv_outer": int(t.inv_outer), "inv_mid": int(t.inv_mid)}

