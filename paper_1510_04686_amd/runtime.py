"""Host driver: uploads a workload, then issues the C ABI calls in order.

Leads once per (k, E) grid -> batched forward / backward sweeps over the bound
points (`capacity` points per call) -> observables; the SCBA loop captures one
whole iteration (self-energy update + every batch) into a HIP graph and
replays it.  All arithmetic runs in the HIP library; this module only
allocates device buffers and sequences calls.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

from . import negf as N


def _dev(a, dtype, device):
    a = np.ascontiguousarray(a)
    if not a.flags.writeable:
        a = a.copy()
    return torch.from_numpy(a).to(device=device, dtype=dtype)


class RGFSolver:
    """Batched RGF over every (sample, k, E) point of a workload on one GPU."""

    def __init__(self, wl, precision="fp64", capacity=None, device="cuda", mem_fraction=0.75, adjoint_segment=0,
                 tune=None, lanes=1, point_redo=math.inf, store="full", redo_frac=0.05):
        """tune: None keeps the library's default kernel shapes; "auto" measures
        them on this context once (negf_autotune) and caches the choice per
        (device, block, capacity, precision); a dict sets them explicitly.
        lanes: batches in flight at once, each on its own context and HIP
        stream (default priority), so the latency-bound phases of one batch
        (the inverse's panels) overlap the matrix-core phases of another;
        `capacity` is then the points per batch of each lane.
        point_redo (mixed precision only): after each pass, every point whose
        largest block-refinement residual ||I - M X0||_F exceeds this bound is
        solved again on an FP64 context and its outputs replaced.  The FP32
        recursion loses roughly that residual in relative accuracy on a point
        (its conditioning), so the bound trades accuracy against the share of
        points redone; math.inf (the default) turns this rule off.
        redo_frac (mixed precision only, default 0.05): also redo, in FP64, this
        fraction of the points with the highest redo score
        (negf_mixed_point_scores: the residual times the point's largest
        weighted |Im G^<_jj|), and every point with a non-finite score, when the
        pass writes the G^< diagonals.  The score ranks the points by their
        likely FP32 error in the density, which the residual alone does not;
        0 turns this rule off.
        store: "full" keeps g and g^< of every slab; "checkpoint" keeps them
        only at the end of every segment of K = ceil(sqrt(N)) slabs (or
        `adjoint_segment` slabs) plus one segment, and the backward sweep and
        the adjoint recompute each segment (memory ~2 sqrt(N) blocks per point
        and store instead of N)."""
        self.wl = wl
        self.device = torch.device(device)
        self.prec = N.NEGF_MIXED if precision == "mixed" else N.NEGF_FP64
        nb = wl.nb
        counts = np.diff(wl.slab_offset).astype(np.int64)
        self.n_slab_max = int(counts.max())
        self.slab_stride = self.n_slab_max
        # Longest sample first, so every launch covers only an active prefix.
        order = np.argsort(-counts, kind="stable")
        pts = [(int(s), ik, ie) for s in order for ik in range(wl.n_k) for ie in range(wl.n_e)]
        self.points = np.array(pts, dtype=np.int32).reshape(-1, 3)
        self.n_points = len(self.points)
        # index of the bound point of each (sample, ik, ie)
        self.index = {tuple(p): i for i, p in enumerate(self.points.tolist())}
        c128, f64 = torch.complex128, torch.float64
        self.h_diag = _dev(wl.h_diag, c128, self.device)
        self.h_up = _dev(wl.h_up, c128, self.device)
        self.energy = _dev(wl.energy, f64, self.device)
        # absorbing-potential contacts instead of semi-infinite leads
        self.cap = getattr(wl, "cap_w", None) is not None
        self.cap_R = self.cap_L = None
        if self.cap:
            self.cap_w = _dev(np.asarray(wl.cap_w, dtype=np.float64), f64, self.device)
            self.cap_side = torch.from_numpy(np.asarray(wl.cap_side, dtype=np.int32)).to(self.device)
        self.w_e = _dev(wl.w_e, f64, self.device)
        self.w_k = _dev(wl.w_k, f64, self.device)
        self.v = None if wl.v_onsite is None else _dev(wl.v_onsite, f64, self.device)
        nk = wl.n_k
        self.lead_h00 = _dev(wl.lead_h00, c128, self.device)
        rep = lambda m: _dev(np.broadcast_to(m, (nk, nb, nb)), c128, self.device)
        self.lead_h01_L, self.lead_tau_L = rep(wl.lead_h01_L), rep(wl.lead_tau_L)
        self.lead_h01_R, self.lead_tau_R = rep(wl.lead_h01_R), rep(wl.lead_tau_R)
        if store not in ("full", "checkpoint"):
            raise ValueError(f"store must be 'full' or 'checkpoint', not {store!r}")
        self.store = store
        nsm = self.n_slab_max
        K = adjoint_segment if adjoint_segment > 0 else int(math.ceil(math.sqrt(nsm)))
        K = max(1, min(K, nsm))
        blocks = nsm if store == "full" else K + -(-nsm // K)        # per store
        adj_blocks = 0 if adjoint_segment == 0 else 2 * (K + -(-nsm // K))
        if capacity is None:
            ce = 8 if self.prec == N.NEGF_MIXED else 16
            per_point = (2 * blocks * nb * nb * ce + (24 + adj_blocks) * nb * nb * 16
                         + (64 + 2 * 256 + 64) * nb * 16)
            free, _ = torch.cuda.mem_get_info(self.device)
            lanes = max(1, int(lanes))
            # up to 512 points per batch: two inverse panels per CU hide each other's latency
            capacity = int(max(1, min(-(-self.n_points // lanes), 512 // lanes,
                                      (free * mem_fraction) // (per_point * lanes))))
        self.capacity = int(capacity)
        self.lanes = max(1, int(lanes))
        # the adjoint runs on the first lane only
        self.ctxs = [N.negf_create(nb, self.n_slab_max, self.capacity, self.prec, adjoint_segment if i == 0 else 0,
                                   store_checkpoint=(store == "checkpoint"))
                     for i in range(self.lanes)]
        self.ctx = self.ctxs[0]
        self.streams = [torch.cuda.Stream(self.device) for _ in range(self.lanes)] if self.lanes > 1 else None
        self.tuning = self._tune(tune, precision)
        for c in self.ctxs[1:]:
            N.negf_set_tuning(c, self.tuning["gemm_prefetch"], self.tuning["inv_outer"], self.tuning["inv_mid"])
        self._last_fwd = None
        self.eta_fill = 0
        mixed = self.prec == N.NEGF_MIXED
        self.point_redo = float(point_redo) if mixed else math.inf
        self.redo_frac = float(redo_frac) if (mixed and redo_frac) else 0.0
        if not 0.0 <= self.redo_frac <= 1.0:
            raise ValueError("redo_frac must lie in [0, 1]")
        self.resid = torch.zeros(self.n_points, dtype=torch.float64, device=self.device) if mixed else None
        self.redo_ctx = None
        self.points_redone = 0
        self.scat_opa = 1             # scattering self-energies: orbital diagonal (1) or atom blocks
        self._bind()
        self.sigma_L = self.sigma_R = None
        self.lead_dual = 0
        self.mirror = self._lead_mirrors()
        self.last_lead_ranges = []

    def _tune(self, tune, precision):
        if tune is None:
            return N.negf_get_tuning(self.ctx)
        if isinstance(tune, dict):
            N.negf_set_tuning(self.ctx, tune["gemm_prefetch"], tune["inv_outer"], tune.get("inv_mid", 0))
            return N.negf_get_tuning(self.ctx)
        if tune != "auto":
            raise ValueError(f"tune must be None, 'auto' or a dict, not {tune!r}")
        path = os.environ.get("NEGF_TUNING_CACHE",
                              os.path.join(os.path.expanduser("~"), ".cache", "paper_1510_04686_amd", "tuning.json"))
        # the key names the candidate set too, so choices made among fewer shapes are redone
        key = f"{torch.cuda.get_device_name(self.device)}|nb={self.wl.nb}|cap={self.capacity}|{precision}|shapes=3"
        cache = {}
        try:
            with open(path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            t = cache[key]
            N.negf_set_tuning(self.ctx, t["gemm_prefetch"], t["inv_outer"], t.get("inv_mid", 0))
            return N.negf_get_tuning(self.ctx)
        t = N.negf_autotune(self.ctx, reps=3)
        cache[key] = t
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
        except OSError:
            pass
        return t

    def _bind(self):
        wl = self.wl
        for c in self.ctxs:
            N.negf_bind(c, wl.nb, wl.slab_offset, wl.n_k, wl.n_e, self.h_diag, self.h_up, 0, wl.up_block,
                        self.v, self.energy, wl.eta, wl.mu_L, wl.mu_R, wl.kT, self.eta_fill, self.points)

    def set_eta_fill(self, on: bool):
        self.eta_fill = int(bool(on))
        self._bind()

    def set_potential(self, v_orb: torch.Tensor):
        self.v = v_orb.contiguous()
        self._bind()

    # ------------------------------------------------------------------ leads
    def _alloc_lead_tables(self):
        wl = self.wl
        shape = (wl.n_k, wl.n_e, wl.nb, wl.nb)
        if self.sigma_L is None:
            self.sigma_L = torch.zeros(shape, dtype=torch.complex128, device=self.device)
            self.sigma_R = torch.zeros(shape, dtype=torch.complex128, device=self.device)
            self.iters_L = torch.zeros((wl.n_k, wl.n_e), dtype=torch.int32, device=self.device)
            self.iters_R = torch.zeros((wl.n_k, wl.n_e), dtype=torch.int32, device=self.device)

    def lead_ranges(self, p0, np_):
        """(ik, e0, e1) energy ranges of the lead self-energies that bound points
        [p0, p0 + np_) read: one range per k-point, spanning the batch's energies
        of that k."""
        sel = self.points[p0:p0 + np_]
        out = []
        for ik in np.unique(sel[:, 1]):
            es = sel[sel[:, 1] == ik, 2]
            out.append((int(ik), int(es.min()), int(es.max()) + 1))
        return out

    def _lead_mirrors(self):
        """{ik: ik_src} for the k-points whose lead tables are the transposes of
        an earlier k-point's.  Each lead is a reservoir in equilibrium; with real
        couplings (h01, tau) and h00(-k) = h00(k)^T its surface Green's function
        solves the transposed equation at -k, so Sigma(-k) = Sigma(k)^T for both
        leads and the mirror needs no decimation.  Checked on the inputs: the k
        values must be mirrors modulo 2 pi and h00 equal to the transpose to
        within a few rounding units; otherwise every k-point is decimated."""
        wl = self.wl
        if self.cap or wl.n_k < 2:
            return {}
        for x in (wl.lead_h01_L, wl.lead_tau_L, wl.lead_h01_R, wl.lead_tau_R):
            if np.iscomplexobj(x) and np.any(np.imag(x) != 0):
                return {}
        scale = max(float(np.max(np.abs(wl.lead_h00))), 1e-300)
        two_pi = 2.0 * math.pi
        out = {}
        for j in range(wl.n_k):
            for i in range(j):
                d = (float(wl.kpts[i]) + float(wl.kpts[j])) % two_pi
                if (min(d, two_pi - d) < 1e-12 and i not in out and
                        float(np.max(np.abs(wl.lead_h00[j] - wl.lead_h00[i].T))) <= 8 * 2.0 ** -53 * scale):
                    out[j] = i
                    break
        return out

    def _cap_contacts(self):
        """Zero lead tables and the absorbing contacts' self-energies
        (negf_cap_selfenergy), once: they depend on neither k nor the batch."""
        self._alloc_lead_tables()
        if self.cap_R is None:
            wl = self.wl
            shp = (wl.n_e, wl.total_slabs, wl.nb)
            self.cap_R = torch.empty(shp, dtype=torch.complex128, device=self.device)
            self.cap_L = torch.empty(shp, dtype=torch.complex128, device=self.device)
            N.negf_cap_selfenergy(self.ctx, self.cap_w, self.cap_side, self.cap_R, self.cap_L)
        self.lead_status, self.lead_dual = 0, 0
        return self.sigma_L, self.sigma_R

    def _scat(self, scat_R, scat_L):
        """The self-energies the forward sweep adds to the diagonal blocks: the
        caller's scattering terms, plus the absorbing contacts' on a workload
        that has them (summed into buffers of the solver by negf_vec_combine,
        so that this also runs inside a captured graph)."""
        if not self.cap:
            return scat_R, scat_L
        if self.cap_R is None:
            self._cap_contacts()
        if scat_R is None and scat_L is None:
            return self.cap_R, self.cap_L
        if scat_R is None or scat_L is None or scat_R.shape != self.cap_R.shape:
            raise ValueError("with absorbing contacts, scattering self-energies must be orbital-diagonal "
                             "[n_e][total_slabs][nb] and given for both R and <")
        if getattr(self, "_tot_R", None) is None:
            self._tot_R = torch.empty_like(self.cap_R)
            self._tot_L = torch.empty_like(self.cap_L)
            self._one = torch.ones(1, dtype=torch.float64, device=self.device)
        for src, cap, tot in ((scat_R, self.cap_R, self._tot_R), (scat_L, self.cap_L, self._tot_L)):
            t = torch.view_as_real(tot).view(1, -1)
            N.negf_vec_combine(torch.view_as_real(src).reshape(1, -1), 1, self._one, 0.0, t.view(-1))
            N.negf_vec_combine(torch.view_as_real(cap).reshape(1, -1), 1, self._one, 1.0, t.view(-1))
        return self._tot_R, self._tot_L

    def lead_selfenergies_for(self, p0, np_, tol=1e-14, max_iter=100):
        """Lead self-energies of only the (k, E) points that the batch [p0, p0 + np_)
        reads, written into their slots of the full tables.  Returns the
        (ik, e0, e1) ranges decimated."""
        return self.lead_selfenergies_for_ranges(self.lead_ranges(p0, np_), tol, max_iter)

    def lead_selfenergies_for_ranges(self, ranges, tol=1e-14, max_iter=100):
        """Lead self-energies of the (ik, e0, e1) ranges: one shared decimation
        call per range whose k-point has no mirror among the decimated ones, the
        mirrored ranges by transposing their source's tables (negf_transpose_batched).
        Returns the ranges decimated."""
        if self.cap:
            self._cap_contacts()
            return []
        self._alloc_lead_tables()
        dec = []
        for ik, e0, e1 in ranges:
            r = (self.mirror.get(ik, ik), e0, e1)
            if r not in dec:
                dec.append(r)
        status, dual = 0, 1
        for ik, e0, e1 in dec:
            k = slice(ik, ik + 1)
            st, du = N.negf_lead_selfenergy_pair(
                self.ctx, self.lead_h00[k], self.lead_h01_L[k], self.lead_tau_L[k], self.lead_h01_R[k],
                self.lead_tau_R[k], self.energy[e0:e1], self.wl.eta, tol, max_iter,
                self.sigma_L[ik, e0:e1], self.sigma_R[ik, e0:e1], self.iters_L[ik, e0:e1],
                self.iters_R[ik, e0:e1])
            status, dual = max(status, st), min(dual, du)
        for ik, e0, e1 in ranges:
            if ik in self.mirror:
                self._mirror_tables(ik, self.mirror[ik], e0, e1)
        self.lead_status, self.lead_dual = status, dual
        self.last_lead_ranges = dec
        return dec

    def _mirror_tables(self, ik, src, e0, e1):
        N.negf_transpose_batched(self.sigma_L[src, e0:e1], self.sigma_L[ik, e0:e1])
        N.negf_transpose_batched(self.sigma_R[src, e0:e1], self.sigma_R[ik, e0:e1])
        self.iters_L[ik, e0:e1].copy_(self.iters_L[src, e0:e1])
        self.iters_R[ik, e0:e1].copy_(self.iters_R[src, e0:e1])

    def lead_selfenergies(self, tol=1e-14, max_iter=100, shared_decimation=True):
        if self.cap:
            return self._cap_contacts()
        self.sigma_L = None
        self._alloc_lead_tables()
        wl = self.wl
        if shared_decimation:
            # decimate the k-points without a mirror, in contiguous runs, then transpose
            todo = [ik for ik in range(wl.n_k) if ik not in self.mirror]
            runs, status, dual = [], 0, 1
            for ik in todo:
                if runs and runs[-1][1] == ik:
                    runs[-1][1] = ik + 1
                else:
                    runs.append([ik, ik + 1])
            for a, b in runs:
                st, du = N.negf_lead_selfenergy_pair(
                    self.ctx, self.lead_h00[a:b], self.lead_h01_L[a:b], self.lead_tau_L[a:b],
                    self.lead_h01_R[a:b], self.lead_tau_R[a:b], self.energy, wl.eta, tol, max_iter,
                    self.sigma_L[a:b], self.sigma_R[a:b], self.iters_L[a:b], self.iters_R[a:b])
                status, dual = max(status, st), min(dual, du)
            for ik, src in self.mirror.items():
                self._mirror_tables(ik, src, 0, wl.n_e)
            self.lead_status, self.lead_dual = status, dual
            self.last_lead_ranges = [(ik, 0, wl.n_e) for ik in todo]
            return self.sigma_L, self.sigma_R
        cL = N.negf_lead_selfenergy(self.ctx, self.lead_h00, self.lead_h01_L, self.lead_tau_L, self.energy, wl.eta,
                                    tol, max_iter, self.sigma_L, self.iters_L)
        cR = N.negf_lead_selfenergy(self.ctx, self.lead_h00, self.lead_h01_R, self.lead_tau_R, self.energy, wl.eta,
                                    tol, max_iter, self.sigma_R, self.iters_R)
        self.lead_status, self.lead_dual = max(cL, cR), 0
        return self.sigma_L, self.sigma_R

    # ------------------------------------------------------------------ RGF
    def alloc_outputs(self, full_blocks=False, want=("GR", "GL", "GG", "bond"), want_T=False):
        nb, P, S = self.wl.nb, self.n_points, self.slab_stride
        shp = {0: (P, S, nb), 1: (P, S, nb, nb), 2: (P, S, nb, self.scat_opa)}[int(full_blocks)]
        out = {}
        for k in ("GR", "GL", "GG"):
            if k in want:
                out[k] = torch.zeros(shp, dtype=torch.complex128, device=self.device)
        if "bond" in want:
            out["bond"] = torch.zeros((P, S), dtype=torch.float64, device=self.device)
        if want_T:
            out["T"] = torch.zeros(P, dtype=torch.float64, device=self.device)
        return out

    def batches(self):
        """(p0, np) of each batch of bound points, in order."""
        return [(p0, min(self.capacity, self.n_points - p0)) for p0 in range(0, self.n_points, self.capacity)]

    def run_batch(self, out, p0, np_, full_blocks=False, want_T=False, scat_R=None, scat_L=None, stream=None):
        """Forward + backward sweep of one batch of bound points on the first
        lane's context (the mixed-precision point redo is not applied)."""
        scat_R, scat_L = self._scat(scat_R, scat_L)
        flags = N.NEGF_WANT_TRANSMISSION if want_T else 0
        N.negf_rgf_solve(self.ctx, p0, np_, self.sigma_L, self.sigma_R, scat_R, scat_L, flags, out.get("GR"),
                         out.get("GL"), out.get("GG"), int(full_blocks), self.slab_stride, out.get("bond"),
                         out.get("T"), stream=stream)
        self._last_fwd = (p0, np_)
        if self.resid is not None:
            N.negf_mixed_point_residuals(self.ctx, self.resid[p0:p0 + np_], stream=stream)

    def run_batches(self, out, full_blocks=False, want_T=False, scat_R=None, scat_L=None, stream=None):
        scat_R, scat_L = self._scat(scat_R, scat_L)
        flags = N.NEGF_WANT_TRANSMISSION if want_T else 0
        base = torch.cuda.current_stream(self.device) if stream is None else stream
        if self.lanes > 1:
            for ls in self.streams:          # fork (also inside a graph capture)
                ls.wait_stream(base)
        for b, p0 in enumerate(range(0, self.n_points, self.capacity)):
            np_ = min(self.capacity, self.n_points - p0)
            lane = b % self.lanes
            ctx = self.ctxs[lane]
            st = base if self.lanes == 1 else self.streams[lane]
            N.negf_rgf_solve(ctx, p0, np_, self.sigma_L, self.sigma_R, scat_R, scat_L, flags, out.get("GR"),
                             out.get("GL"), out.get("GG"), int(full_blocks), self.slab_stride, out.get("bond"),
                             out.get("T"), stream=st)
            if lane == 0:
                self._last_fwd = (p0, np_)
            if self.resid is not None:
                N.negf_mixed_point_residuals(ctx, self.resid[p0:p0 + np_], stream=st)
        if self.lanes > 1:
            for ls in self.streams:          # join
                base.wait_stream(ls)
        if self._redo_on() and not torch.cuda.is_current_stream_capturing():
            self._redo(out, full_blocks, want_T, scat_R, scat_L, base)

    def _redo_on(self):
        return math.isfinite(self.point_redo) or self.redo_frac > 0

    def _redo(self, out, full_blocks, want_T, scat_R, scat_L, stream):
        """FP64 pass over the points whose mixed-precision residual exceeded
        `point_redo`, and over the `redo_frac` share of points with the highest
        redo score; their outputs replace the mixed ones in place."""
        with torch.cuda.stream(stream):
            sel = self.resid > self.point_redo
            k = int(math.ceil(self.redo_frac * self.n_points))
            if k > 0 and "GL" in out and not full_blocks:
                score = torch.empty_like(self.resid)
                N.negf_mixed_point_scores(self.ctx, out["GL"], self.slab_stride, self.w_e, self.w_k, self.resid,
                                          score, stream=stream)
                sel[torch.topk(score, k).indices] = True
                sel |= ~torch.isfinite(score)
            idx = torch.nonzero(sel).flatten()
        self.points_redone = int(idx.numel())          # synchronises the stream
        if self.points_redone == 0:
            return
        wl, nb = self.wl, self.wl.nb
        if self.redo_ctx is None:
            per_point = 2 * self.n_slab_max * nb * nb * 16 + 24 * nb * nb * 16 + (64 + 2 * 256 + 64) * nb * 16
            free, _ = torch.cuda.mem_get_info(self.device)
            cap = int(max(1, min(64, self.capacity, (free // 2) // per_point)))
            self.redo_ctx = N.negf_create(nb, self.n_slab_max, cap, N.NEGF_FP64, 0)
            self.redo_cap = cap
        N.negf_set_scattering_blocks(self.redo_ctx, self.scat_opa)
        pts = self.points[idx.cpu().numpy()]
        N.negf_bind(self.redo_ctx, wl.nb, wl.slab_offset, wl.n_k, wl.n_e, self.h_diag, self.h_up, 0, wl.up_block,
                    self.v, self.energy, wl.eta, wl.mu_L, wl.mu_R, wl.kT, self.eta_fill, pts)
        R = len(pts)
        sub = {k: torch.zeros((R,) + tuple(v.shape[1:]), dtype=v.dtype, device=self.device) for k, v in out.items()}
        flags = N.NEGF_WANT_TRANSMISSION if want_T else 0
        for q0 in range(0, R, self.redo_cap):
            nq = min(self.redo_cap, R - q0)
            N.negf_rgf_forward(self.redo_ctx, q0, nq, self.sigma_L, self.sigma_R, scat_R, scat_L, flags,
                               stream=stream)
            N.negf_rgf_backward(self.redo_ctx, q0, nq, sub.get("GR"), sub.get("GL"), sub.get("GG"),
                                int(full_blocks), self.slab_stride, sub.get("bond"), sub.get("T"), stream=stream)
        with torch.cuda.stream(stream):
            for k, v in out.items():
                v.index_copy_(0, idx, sub[k])

    def solve(self, full_blocks=False, want=("GR", "GL", "GG", "bond"), want_T=False, scat_R=None, scat_L=None):
        if self.sigma_L is None:
            self.lead_selfenergies()
        out = self.alloc_outputs(full_blocks, want, want_T)
        self.run_batches(out, full_blocks, want_T, scat_R, scat_L)
        return out

    def observables(self, GL, bond, g_s=None, spectral=True):
        wl = self.wl
        g_s = wl.g_s if g_s is None else g_s
        n = torch.zeros((wl.total_slabs, wl.atoms_per_slab), dtype=torch.float64, device=self.device)
        J = None if bond is None else torch.zeros(wl.total_slabs, dtype=torch.float64, device=self.device)
        jE = (torch.zeros((wl.n_samples, wl.n_e, self.slab_stride), dtype=torch.float64, device=self.device)
              if (spectral and bond is not None) else None)
        gl_opa = 1 if GL is None or GL.dim() == 3 else int(GL.shape[-1])   # diagonals or (atom) blocks
        N.negf_observables(self.ctx, GL, bond, self.slab_stride, self.w_e, self.w_k, g_s, wl.orbs_per_atom,
                           n, J, jE, gl_opa=gl_opa)
        return n, J, jE

    # ------------------------------------------------------------------ adjoint
    def density(self, scat_R=None, scat_L=None):
        """Electron density per atom (Eq. 7) for the current potential (with the
        given orbital-diagonal scattering self-energies, if any)."""
        if self.sigma_L is None:
            self.lead_selfenergies()
        out = self.alloc_outputs(want=("GL",))
        self.run_batches(out, scat_R=scat_R, scat_L=scat_L)
        n, _, _ = self.observables(out["GL"], None)
        return n

    def density_vjp(self, w_atom, scat_R=None, scat_L=None):
        """grad_V (per atom) of sum_a w_a n_a through the adjoint RGF, at the
        potential of the last forward pass and with the scattering
        self-energies it used (held fixed: their own dependence on V, through
        the Born loop, is not differentiated)."""
        wl = self.wl
        w_orb = w_atom.to(device=self.device, dtype=torch.float64).reshape(wl.total_slabs, -1)
        w_orb = w_orb.repeat_interleave(wl.orbs_per_atom, dim=1).contiguous()
        dX = torch.zeros((self.n_points, self.slab_stride, wl.nb), dtype=torch.complex128, device=self.device)
        batches = [(p0, min(self.capacity, self.n_points - p0)) for p0 in range(0, self.n_points, self.capacity)]
        # the batch whose stores are still in the context goes first
        if self._last_fwd in batches:
            batches.remove(self._last_fwd)
            batches.insert(0, self._last_fwd)
        for p0, np_ in batches:
            if self._last_fwd != (p0, np_):
                N.negf_rgf_forward(self.ctx, p0, np_, self.sigma_L, self.sigma_R, *self._scat(scat_R, scat_L))
                self._last_fwd = (p0, np_)
            N.negf_rgf_adjoint(self.ctx, p0, np_, w_orb, dX, self.slab_stride)
        g, _, _ = self.observables(dX, None)
        return g

    def status(self):
        """Most severe device status over the contexts (non-finite pivot, zero
        pivot, then mixed-precision fallback), cleared by the call."""
        ctxs = self.ctxs + ([self.redo_ctx] if self.redo_ctx is not None else [])
        codes = [N.negf_sync_status(c) for c in ctxs]
        for code in (N.NEGF_WNONFINITE, N.NEGF_WSINGULAR, N.NEGF_WFALLBACK):
            if code in codes:
                return code
        return max(codes)

    # ------------------------------------------------------------------ SCBA
    def scba(self, n_iter=None, graph=True, atom_blocks=False, progress=None, tol=None):
        """Self-consistent Born loop (Eqs. 1-6) for a single-sample grid
        workload.  One iteration = scattering self-energy update from the last
        diagonals + a full forward/backward pass; captured once into a HIP
        graph and replayed when ``graph`` is true.  atom_blocks: build the
        local self-energies from the atom blocks (orbs_per_atom square) of the
        diagonal blocks instead of the orbital diagonals; the outputs are then
        atom blocks [P][slab][nb][orbs_per_atom] (negf_set_scattering_blocks,
        which stays set on the solver's contexts).  progress(i, n): called after
        iteration i, after waiting for it (one host synchronisation per
        iteration; without it the replays run with no host read).
        tol: stop at the first update whose residual ||dSigma|| / ||Sigma|| is
        below tol (at most n_iter updates): the update and the solve are then
        two graphs (or eager calls) with one residual read between them, and
        the outputs are the last solve's with the self-energy of that update,
        as after a fixed count."""
        wl = self.wl
        assert wl.n_samples == 1
        n_iter = wl.n_scba if n_iter is None else n_iter
        if self._redo_on():
            graph = False      # the mixed-precision point redo decides on the host after every pass
        if self.sigma_L is None:
            self.lead_selfenergies()
        self.scat_opa = wl.orbs_per_atom if atom_blocks else 1
        for c in self.ctxs + ([self.redo_ctx] if self.redo_ctx is not None else []):
            N.negf_set_scattering_blocks(c, self.scat_opa)
        fb = 2 if atom_blocks else 0
        Ns = wl.total_slabs
        shp = (wl.n_e, Ns, wl.nb) + ((self.scat_opa,) if atom_blocks else ())
        self.scat_R = torch.zeros(shp, dtype=torch.complex128, device=self.device)
        self.scat_L = torch.zeros(shp, dtype=torch.complex128, device=self.device)
        out = self.alloc_outputs(full_blocks=fb, want=("GR", "GL", "bond"))
        N.negf_scba_history(self.ctx, 0)          # clear the device residual list
        # iteration 0: ballistic pass (Sigma_scat = 0)
        self.run_batches(out, full_blocks=fb, scat_R=self.scat_R, scat_L=self.scat_L)

        def update(stream=None):
            N.negf_scba_selfenergy(self.ctx, out["GR"], out["GL"], self.slab_stride, self.w_k, wl.D_ac, wl.M_op,
                                   wl.shift, wl.n_bose, self.scat_R, self.scat_L, None, stream=stream)

        def solve(stream=None):
            self.run_batches(out, full_blocks=fb, scat_R=self.scat_R, scat_L=self.scat_L, stream=stream)

        def one_iteration(stream=None):
            update(stream)
            solve(stream)

        def capture(fn):
            g = torch.cuda.CUDAGraph()
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                torch.cuda.synchronize()
            with torch.cuda.graph(g, stream=s):
                fn(stream=s)
            torch.cuda.current_stream().wait_stream(s)
            return g

        if tol is not None:
            run_u, run_s = update, solve
            if graph:
                gu, gs = capture(update), capture(solve)
                run_u, run_s = (lambda: gu.replay()), (lambda: gs.replay())
            hist = []
            for i in range(max(n_iter, 1)):
                run_u()
                hist += N.negf_scba_history(self.ctx, 1)      # waits for the update
                if hist[-1] < tol or i == max(n_iter, 1) - 1:
                    break
                run_s()
                if progress:
                    torch.cuda.synchronize(self.device)
                    progress(i + 2, n_iter)
            self.scba_out = out
            return out, hist

        if n_iter <= 1 or not graph:
            for i in range(n_iter - 1):
                one_iteration()
                if progress:
                    torch.cuda.synchronize(self.device)
                    progress(i + 2, n_iter)
        else:
            g = capture(one_iteration)
            # the residuals stay on the device: no host read between replays
            for i in range(n_iter - 1):
                g.replay()
                if progress:
                    torch.cuda.synchronize(self.device)
                    progress(i + 2, n_iter)
        # last update: Sigma_n from the n-th solve (the solve itself is not redone)
        N.negf_scba_selfenergy(self.ctx, out["GR"], out["GL"], self.slab_stride, self.w_k, wl.D_ac, wl.M_op,
                               wl.shift, wl.n_bose, self.scat_R, self.scat_L, None)
        hist = N.negf_scba_history(self.ctx, max(n_iter, 1))
        self.scba_out = out
        return out, hist


class RGFDensity(torch.autograd.Function):
    """n = RGFDensity.apply(v_atom, solver): density per atom (Eq. 7) as a
    differentiable function of the onsite potential per atom; backward runs the
    adjoint RGF (one VJP per call)."""

    @staticmethod
    def forward(ctx, v_atom, solver):
        wl = solver.wl
        v = v_atom.detach().to(device=solver.device, dtype=torch.float64).reshape(wl.total_slabs, -1)
        solver.set_potential(v.repeat_interleave(wl.orbs_per_atom, dim=1).contiguous())
        n = solver.density()
        ctx.solver = solver
        return n

    @staticmethod
    def backward(ctx, grad_n):
        g = ctx.solver.density_vjp(grad_n.contiguous())
        return g, None


class NewtonPoisson:
    """The NEGF-Poisson loop (Eq. 9 iterated with Eqs. 1-8) on one device.

    Unknown: the electron's potential energy V per atom (eV), the onsite
    potential of Eq. (1).  Residual, on the atom grid (negf_poisson_residual):
        F(V) = L V - beta (n(V) - N_D),
    n from the RGF density (Eq. 7) of `solver`, a single-sample RGFSolver.
    Each Newton step solves (L0 - beta dn/dV) dV = -F by GMRES, right-
    preconditioned with L0 (conjugate gradients, negf_poisson_solve).  The
    density's Jacobian enters each Krylov iteration in one of two ways:
      jacobian="adjoint": one VJP of the adjoint RGF (the solver needs
        adjoint_segment != 0), i.e. the operator L0 - beta (dn/dV)^T.  In
        equilibrium (one Fermi level) dn/dV is symmetric -- its (a, b) entry
        is a sum of Im(G_ab G_ba) terms -- so this is the exact Newton step;
        under bias the lesser part makes dn/dV non-symmetric, the step is an
        inexact Newton step and the loop converges linearly to the same root
        (F is always evaluated exactly);
      jacobian="fd": the central difference (n(V + h z) - n(V - h z)) / 2h,
        two forward densities per iteration, exact to O(h^2) with or without
        bias (h z at most fd_step eV on any atom).
    Preconditioner: preconditioner="local" (default) solves with
    L0 + diag(s), s = -beta d, d the orbital-diagonal part of dn_a/dV_a
    (negf_density_jacobian_local, from the G^R and G^< diagonals of the same
    pass; entries of s below zero count as zero): where beta dn/dV outweighs L
    (quantum capacitance) L0 alone leaves GMRES almost stalled; "poisson" uses
    L0 alone.  A step whose largest change exceeds max_step (eV) is scaled down
    to it, and halved (up to three times) while max |F| does not decrease.
    Every vector operation runs in the library's kernels; the host keeps the
    small Hessenberg least-squares problem of GMRES."""

    def __init__(self, solver, n_z, n_y, beta, n_d, z_gate=False, v_left=0.0, v_right=0.0, v_gate=0.0,
                 max_step=0.1, krylov_dim=20, krylov_tol=1e-3, cg_tol=1e-13, jacobian="adjoint",
                 fd_step=1e-5, preconditioner="local"):
        wl = solver.wl
        if wl.n_samples != 1:
            raise ValueError("the NEGF-Poisson loop runs one device (one sample)")
        if wl.atoms_per_slab != n_z * n_y:
            raise ValueError("atoms per slab must equal n_z * n_y")
        if jacobian not in ("adjoint", "fd"):
            raise ValueError("jacobian must be 'adjoint' or 'fd'")
        if preconditioner not in ("local", "poisson"):
            raise ValueError("preconditioner must be 'local' or 'poisson'")
        self.local = preconditioner == "local"
        self.s, self.wl = solver, wl
        self.mode, self.fd_step = jacobian, float(fd_step)
        self._V = None
        self._log = None
        self.grid = N.poisson_grid(wl.total_slabs, n_z, n_y, z_gate, v_left, v_right, v_gate)
        self.n = wl.total_slabs * wl.atoms_per_slab
        dev = solver.device
        f64 = dict(dtype=torch.float64, device=dev)
        self.beta = float(beta)
        self.nd = torch.as_tensor(np.asarray(n_d, dtype=np.float64).reshape(-1), **f64).contiguous()
        if self.nd.numel() != self.n:
            raise ValueError("n_d must hold one value per atom")
        self.max_step, self.m, self.ktol, self.cg_tol = float(max_step), int(krylov_dim), float(krylov_tol), cg_tol
        self.pwork = torch.empty(N.negf_poisson_work_bytes(self.grid), dtype=torch.uint8, device=dev)
        self.vwork = torch.empty(N.negf_vec_work_bytes(self.n, self.m + 1), dtype=torch.uint8, device=dev)
        self.Q = torch.empty((self.m + 1, self.n), **f64)      # Krylov basis
        self.Z = torch.empty((self.m, self.n), **f64)          # preconditioned directions L0^-1 q_j
        self.F = torch.empty(self.n, **f64)
        self.w = torch.empty(self.n, **f64)
        self.h = torch.empty(self.m + 1, **f64)
        self.c = torch.empty(self.m + 1, **f64)
        self.nrm = torch.empty(2, **f64)
        self.stats = {"newton": 0, "krylov": 0, "cg": 0, "density_s": 0.0, "jacobian_s": 0.0}
        self.vp = torch.empty(self.n, **f64)
        self.dloc = torch.zeros(self.n, **f64)      # local part of dn/dV
        self.shift = torch.zeros(self.n, **f64)     # -beta dloc (the preconditioner's diagonal)

    # -- small helpers (device kernels; one host read each where noted)
    def _norms(self, x):
        N.negf_vec_norms(x, self.nrm, self.vwork)
        a = self.nrm.cpu().numpy()
        return math.sqrt(max(float(a[0]), 0.0)), float(a[1])

    def _combine(self, X, coef, b, y):
        m = len(coef)
        if m:
            self.c[:m].copy_(torch.from_numpy(np.asarray(coef, dtype=np.float64)))
        N.negf_vec_combine(X, m, self.c, b, y)

    def _set_v(self, V):
        wl = self.wl
        self.s.set_potential(V.view(wl.total_slabs, wl.atoms_per_slab).repeat_interleave(wl.orbs_per_atom, dim=1))

    def residual(self, V):
        """F(V) into self.F; returns (F, n)."""
        import time
        t = time.perf_counter()
        self._set_v(V)
        self._V = V.clone()
        s, wl = self.s, self.wl
        if self.local:
            out = s.alloc_outputs(want=("GR", "GL"))
            s.run_batches(out)
            n = s.observables(out["GL"], None)[0].reshape(-1).contiguous()
            N.negf_density_jacobian_local(s.ctx, out["GR"], out["GL"], s.slab_stride, s.w_e, s.w_k, wl.g_s,
                                          wl.orbs_per_atom, self.dloc.view(wl.total_slabs, -1))
            self._combine(self.dloc.view(1, -1), [-self.beta], 0.0, self.shift)
            del out
        else:
            n = s.density().reshape(-1).contiguous()
        torch.cuda.synchronize(s.device)
        self.stats["density_s"] += time.perf_counter() - t
        N.negf_poisson_residual(self.grid, V, n, self.nd, self.beta, self.F)
        return self.F, n

    def _jac(self, z, out):
        """out = L0 z - beta J_n z at the potential of the last residual, J_n
        = (dn/dV)^T (adjoint) or the central difference of n along z (fd)."""
        import time
        N.negf_poisson_apply(self.grid, z, out, with_boundary=False)
        t = time.perf_counter()
        if self.mode == "adjoint":
            g = self.s.density_vjp(z.view(self.wl.total_slabs, -1)).reshape(1, -1).contiguous()
            self._combine(g, [-self.beta], 1.0, out)
        else:
            _, zmax = self._norms(z)
            h = self.fd_step / max(zmax, 1e-300)
            dn = []
            for sgn in (1.0, -1.0):
                self.vp.copy_(self._V)
                self._combine(z.view(1, -1), [sgn * h], 1.0, self.vp)
                self._set_v(self.vp)
                dn.append(self.s.density().reshape(1, -1).contiguous())
            self._combine(torch.cat(dn), [-self.beta / (2 * h), self.beta / (2 * h)], 1.0, out)
            self._set_v(self._V)
        torch.cuda.synchronize(self.s.device)
        self.stats["jacobian_s"] += time.perf_counter() - t

    def _precond(self, q, z):
        it, _ = N.negf_poisson_solve(self.grid, q, z, self.pwork, tol=self.cg_tol, max_iter=20 * self.n + 100,
                                     shift=self.shift if self.local else None)
        self.stats["cg"] += it

    def _gmres(self, rhs, out):
        """out ~= J^-1 rhs: one GMRES cycle of at most krylov_dim iterations,
        classical Gram-Schmidt applied twice, Givens rotations on the host."""
        m = self.m
        b0, _ = self._norms(rhs)
        out.zero_()
        if b0 == 0.0:
            return 0
        self.Q[0].copy_(rhs)
        self._combine(self.Q, [], 1.0 / b0, self.Q[0])
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = b0
        k = 0
        for j in range(m):
            self._precond(self.Q[j], self.Z[j])
            self._jac(self.Z[j], self.w)
            hj = np.zeros(j + 1)
            for _ in range(2):
                N.negf_vec_dots(self.Q, j + 1, self.w, self.h, self.vwork)
                hh = self.h[:j + 1].cpu().numpy().copy()
                self._combine(self.Q, list(-hh), 1.0, self.w)
                hj += hh
            wn, _ = self._norms(self.w)
            H[:j + 1, j] = hj
            H[j + 1, j] = wn
            for i in range(j):                     # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            r = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = (H[j, j] / r, H[j + 1, j] / r) if r > 0 else (1.0, 0.0)
            H[j, j] = r
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            self.stats["krylov"] += 1
            if self._log:
                self._log(f"  krylov {k}: residual ratio {abs(g[j + 1]) / b0:.2e}")
            if abs(g[j + 1]) <= self.ktol * b0 or wn == 0.0:
                break
            self.Q[j + 1].copy_(self.w)
            self._combine(self.Q, [], 1.0 / wn, self.Q[j + 1])
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        self._combine(self.Z, list(y), 0.0, out)
        return k

    def solve(self, V0, tol=1e-9, max_newton=30, log=None):
        """Newton iterations from V0 (per atom, [N_x, atoms] or flat) until
        max |F| <= tol.  Returns (V [N_x, atoms], history of max |F|)."""
        V = torch.as_tensor(np.asarray(V0, dtype=np.float64) if not torch.is_tensor(V0) else V0,
                            dtype=torch.float64, device=self.s.device).reshape(-1).clone()
        dV = torch.empty_like(V)
        rhs = torch.empty_like(V)
        self._log = log
        hist = []
        F, _ = self.residual(V)
        _, fmax = self._norms(F)
        for it in range(max_newton + 1):
            hist.append(fmax)
            if log:
                log(f"newton {it}: max|F| = {fmax:.3e}")
            if not math.isfinite(fmax) or fmax <= tol or it == max_newton:
                break
            rhs.copy_(F)
            self._combine(self.Q, [], -1.0, rhs)           # rhs = -F
            self._gmres(rhs, dV)
            _, dmax = self._norms(dV)
            scale = min(1.0, self.max_step / max(dmax, 1e-300))
            base = V.clone()
            for bt in range(4):                            # backtracking on max |F|
                V.copy_(base)
                self._combine(dV.view(1, -1), [scale], 1.0, V)
                F, _ = self.residual(V)
                _, ft = self._norms(F)
                if ft < fmax or bt == 3:
                    break
                scale *= 0.5
                if log:
                    log(f"  step halved to {scale:.3e}")
            fmax = ft
            self.stats["newton"] += 1
        return V.view(self.wl.total_slabs, -1), hist
