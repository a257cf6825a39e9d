/*
 * negf.h -- C ABI of the MI355X (gfx950) recursive Green's function library.
 *
 * The library solves, for many independent (sample, k, E) points, the
 * block-tridiagonal NEGF system of the paper's Eqs. (1)-(3):
 *
 *     G^R(k,E) = (E + i eta - H(k) - V - Sigma^R_lead - Sigma^R_scat)^-1      (Eq. 1)
 *     G^<(k,E) = G^R Sigma^< G^R^dagger                                       (Eq. 2)
 *
 * by recursive Green's functions (RGF) over the slabs of the device, with
 * ordered semi-infinite leads (Sancho-Rubio decimation), the acoustic and
 * optical phonon self-energies of Eqs. (4)-(6) and the density and current
 * of Eqs. (7)-(8).
 *
 * Conventions
 * -----------
 * - Complex numbers are interleaved {re, im} (torch.complex128 layout).
 *   Matrices are dense, row-major, contiguous, nb x nb.
 * - Unless stated otherwise every array pointer is a DEVICE pointer owned by
 *   the caller; the library never frees caller memory and keeps no pointer to
 *   it beyond the bound system (negf_bind).  Energies are in eV.
 * - Every call is asynchronous on the caller's HIP stream (passed as void*,
 *   NULL = default stream).  A context must not be used from two streams at
 *   once.
 * - Return codes: 0 = OK; < 0 = error detected on the host, nothing was
 *   launched; > 0 = warning (results written).  Faults met inside kernels
 *   (singular or non-finite pivots) set bits in a device status word that
 *   negf_sync_status() returns and clears.
 * - The hot calls (negf_rgf_forward / negf_rgf_backward /
 *   negf_scba_selfenergy / negf_observables) allocate nothing and issue no
 *   host<->device copies, so a caller may capture them into a HIP graph.
 */
#ifndef NEGF_H
#define NEGF_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct negf_ctx negf_ctx;
typedef struct { double re, im; } negf_c128;

enum {
    NEGF_OK = 0,
    NEGF_EINVAL = -1,     /* bad argument */
    NEGF_ESHAPE = -2,     /* sizes exceed the context configuration */
    NEGF_ENOMEM = -3,     /* device allocation failed (negf_create / negf_bind only) */
    NEGF_EHIP = -4,       /* a HIP runtime call failed */
    NEGF_ESTATE = -5,     /* call order violated (e.g. no bound system) */
    NEGF_WNOCONV = 1,     /* Sancho-Rubio hit max_iter for some point */
    NEGF_WSINGULAR = 2,   /* a block inverse met an exactly zero pivot */
    NEGF_WNONFINITE = 3,  /* a block inverse met a non-finite pivot */
    NEGF_WFALLBACK = 4    /* mixed precision redid some block inverses in FP64 */
};

enum { NEGF_FP64 = 0, NEGF_MIXED = 1 };   /* negf_config.precision */

/* negf_rgf_forward flags */
enum { NEGF_WANT_TRANSMISSION = 1 };

typedef struct {
    int nb;           /* orbitals per slab (block size), 1 <= nb <= 2048 */
    int n_slab_max;   /* largest slab count of any sample that will be bound */
    int capacity;     /* points per negf_rgf_forward/backward call and per lead batch */
    int precision;    /* NEGF_FP64, or NEGF_MIXED: FP32 MFMA block algebra with one
                         FP64-residual Newton-Schulz step per block inverse */
    int adjoint_segment; /* 0: no adjoint workspace; > 0: slabs per checkpoint segment of
                            negf_rgf_adjoint; -1: ceil(sqrt(n_slab_max)) */
    int store_checkpoint;/* 0: the forward sweep keeps g and g^< of every slab (n_slab_max
                            blocks each per point); 1: only of the last slab of every
                            segment of K slabs (K = adjoint_segment if > 0, else
                            ceil(sqrt(n_slab_max))) plus one segment buffer, about
                            2 sqrt(n_slab_max) blocks each per point; the backward sweep
                            and the adjoint then recompute each segment's g and g^< from
                            its checkpoint (the same kernels, so the same values) */
} negf_config;

/* Create a context and allocate its device workspace (the only allocation of
 * the hot path): two stores of capacity * n_slab_max blocks for the
 * left-connected g^R and g^< (or their checkpoints and one segment, with
 * store_checkpoint = 1) plus per-point temporaries.
 * Errors: NEGF_EINVAL (bad sizes), NEGF_ENOMEM. */
int negf_create(const negf_config* cfg, negf_ctx** out);
void negf_destroy(negf_ctx* ctx);

/* SHA-1 of the library's sources (HIP files, headers and this header) it was
 * built from, as a NUL-terminated hex string owned by the library.  A binding
 * compares it with the sources at hand and refuses a stale build. */
const char* negf_build_id(void);

/* Bytes of device workspace the context holds. */
long long negf_workspace_bytes(const negf_ctx* ctx);

/* Return and clear the device status word (synchronises `stream`).
 * Returns NEGF_OK, or the warning code of the most severe bit set. */
int negf_sync_status(negf_ctx* ctx, void* stream);
const char* negf_error_string(int status);

/*
 * The block-tridiagonal device (Eq. 1).  Samples (alloy realisations) are
 * concatenated along the slab axis; sample s owns global slabs
 * [slab_offset[s], slab_offset[s+1]).
 */
typedef struct {
    int nb;                          /* must equal negf_config.nb */
    int n_samples;
    const long long* slab_offset;    /* HOST [n_samples+1] */
    int n_k, n_e;
    const negf_c128* h_diag;         /* [n_k][total_slabs][nb][nb]  H_ii(k) (Hermitian) */
    const negf_c128* h_up;           /* [n_kup][total_slabs][nb][nb] H_{i,i+1}; entry of a
                                        sample's last slab unused.  H_{i+1,i} = H_{i,i+1}^dagger */
    long long h_up_k_stride;         /* elements between k-points in h_up; 0 = shared by all k */
    int up_block;                    /* H_{i,i+1} is block-diagonal with up_block x up_block
                                        blocks (up_block divides nb, up_block <= 48); only
                                        those blocks are read */
    const double* v_onsite;          /* [total_slabs][nb] potential energy added to diag(H),
                                        or NULL */
    const double* energy;            /* [n_e] */
    double eta;                      /* z = E + i eta in every diagonal block and in the leads */
    double mu_L, mu_R, kT;           /* lead Fermi functions for Sigma^<_lead = i f Gamma */
    int eta_fill;                    /* 0: the device eta is an empty sink; 1: filled with
                                        f(E; mu_L, kT), Sigma^<_eta = 2 i eta f  (equilibrium) */
} negf_system;

/* Bind a system and a point set.  `points` is a HOST array [n_points][3] of
 * (sample, ik, ie).  Uploads the descriptors (synchronously, so never inside a
 * graph capture); the device pointers inside `sys` must stay valid while bound.
 * Points should be ordered longest sample first: batched launches then cover
 * only the active prefix of a range.
 * Errors: NEGF_EINVAL, NEGF_ESHAPE (nb mismatch, n_slab > n_slab_max), NEGF_ENOMEM. */
int negf_bind(negf_ctx* ctx, const negf_system* sys, int n_points, const int* points);

/*
 * Retarded self-energies of the two ordered semi-infinite leads (Eq. 3,
 * Sigma_lead), by Sancho-Rubio decimation in complex FP64 (always FP64).
 *   h00  [n_k][nb][nb]  principal-layer Hamiltonian of the lead
 *   h01  [n_k][nb][nb]  coupling from a lead layer to the next layer deeper in the lead
 *   tau  [n_k][nb][nb]  coupling from the device edge slab to the lead surface layer
 *   energy [n_e] (device); z = E + i eta.
 * Out: sigma [n_k][n_e][nb][nb] = tau g_s tau^dagger; iters [n_k][n_e] (device int,
 * may be NULL) decimation steps used.  Stops per point when
 * ||alpha||_1 + ||beta||_1 < tol ||h01||_1 or at max_iter.  Processes the grid in
 * batches of `capacity` points and synchronises `stream` once per decimation step.
 * Returns NEGF_WNOCONV if any point hit max_iter.  Errors: NEGF_EINVAL. */
int negf_lead_selfenergy(negf_ctx* ctx, void* stream, int n_k,
                         const negf_c128* h00, const negf_c128* h01, const negf_c128* tau,
                         int n_e, const double* energy, double eta, double tol, int max_iter,
                         negf_c128* sigma, int* iters);

/*
 * Both lead self-energies at once, exploiting a dependency between them (the
 * section "Quantitative discussion of current state of the art" credits
 * NEMO5's savings to analytical dependencies among the Green's functions and
 * self-energies).  When the left lead's coupling into the lead is the adjoint
 * of the right lead's (h01_L = h01_R^dagger at every k) and both share h00,
 * the left lead is the right lead's bulk seen from the other end: one
 * Sancho-Rubio decimation of (h00, h01_R) yields both surface functions (the
 * dual surface accumulates beta g alpha instead of alpha g beta), at one extra
 * surface inverse and two extra GEMMs per point instead of a second
 * decimation.  The condition is checked on the device (max deviation
 * <= 1e-15 max|h01_R|); if it fails, two independent decimations run.
 *   h00 [n_k][nb][nb]; h01_L, tau_L, h01_R, tau_R [n_k][nb][nb] as in
 *   negf_lead_selfenergy.  Outputs as there, for each lead; iters_L/R may be NULL.
 *   dual_used (host int*, may be NULL): 1 when the shared decimation ran.
 * Each lead stops counting at its own criterion (its own ||h01||_1); the
 * shared decimation runs until both have converged.  Synchronises `stream`.
 * Returns NEGF_WNOCONV if any point hit max_iter.  Errors: NEGF_EINVAL. */
int negf_lead_selfenergy_pair(negf_ctx* ctx, void* stream, int n_k, const negf_c128* h00,
                              const negf_c128* h01_L, const negf_c128* tau_L,
                              const negf_c128* h01_R, const negf_c128* tau_R,
                              int n_e, const double* energy, double eta, double tol, int max_iter,
                              negf_c128* sigma_L, negf_c128* sigma_R, int* iters_L, int* iters_R,
                              int* dual_used);

/*
 * Forward (left-connected) RGF sweep over bound points [p0, p0+np), np <= capacity:
 *   g_i   = (A_ii - H_{i,i-1} g_{i-1} H_{i-1,i})^-1                         (Eq. 1)
 *   g^<_i = g_i (Sigma^<_i + H_{i,i-1} g^<_{i-1} H_{i-1,i}) g_i^dagger     (Eq. 2)
 * with A_ii = (E + i eta) I - H_ii - diag(V_i) - diag(Sigma^R_scat,i) - Sigma_L (i=0)
 * - Sigma_R (i=N-1) and Sigma^<_i = diag(Sigma^<_scat,i) + lead terms i f Gamma.
 *   sigma_L, sigma_R  [n_k][n_e][nb][nb] lead self-energies (negf_lead_selfenergy)
 *   scat_R, scat_L    [n_e][total_slabs][nb] orbital-diagonal scattering
 *                     self-energies (Eqs. 4-6), or NULL (ballistic); atom
 *                     blocks [n_e][total_slabs][nb][opa] after
 *                     negf_set_scattering_blocks(opa > 1)
 *   flags             NEGF_WANT_TRANSMISSION keeps the left-column chain G_{N,1}.
 * g and g^< stay in the context for negf_rgf_backward.  Errors: NEGF_ESTATE,
 * NEGF_EINVAL, NEGF_ESHAPE. */
int negf_rgf_forward(negf_ctx* ctx, void* stream, int p0, int np,
                     const negf_c128* sigma_L, const negf_c128* sigma_R,
                     const negf_c128* scat_R, const negf_c128* scat_L, int flags);

/*
 * Backward sweep for the same points (after negf_rgf_forward):
 *   G_ii   = g_i + g_i H_{i,i+1} G_{i+1,i+1} H_{i+1,i} g_i
 *   G^<_ii = g^<_i + L G^<_{i+1} L^dagger + T - T^dagger,  L = g_i H_{i,i+1},
 *            T = L G_{i+1} H_{i+1,i} g^<_i
 *   G^>_ii = G^<_ii + G_ii - G_ii^dagger   (no greater-than recursion, Eq. 6 remark)
 *   j_i    = 2 Re Tr[H_{i,i+1} G^<_{i+1,i}]  bond current (units e/h per spin, Eq. 8)
 * Outputs (each may be NULL), indexed by bound point p:
 *   GR, GL, GG   full_blocks = 0: [p][slab_stride][nb] orbital diagonals,
 *                full_blocks = 1: [p][slab_stride][nb][nb] diagonal blocks,
 *                full_blocks = 2: [p][slab_stride][nb][opa] atom blocks (opa of
 *                negf_set_scattering_blocks; row o holds o's entries with the
 *                orbitals of its own atom)
 *   bond_j       [p][slab_stride] (entry i = bond i -> i+1, i < N_p - 1)
 *   transmission [p] Caroli T = Tr[Gamma_R G_{N1} Gamma_L G_{N1}^dagger]
 *                (requires NEGF_WANT_TRANSMISSION in the forward call)
 * slab_stride >= the longest bound sample.  Errors: NEGF_ESTATE, NEGF_EINVAL. */
int negf_rgf_backward(negf_ctx* ctx, void* stream, int p0, int np,
                      negf_c128* GR, negf_c128* GL, negf_c128* GG, int full_blocks,
                      int slab_stride, double* bond_j, double* transmission);

/*
 * negf_rgf_forward followed by negf_rgf_backward for points [p0, p0+np), in
 * one call (same arguments, outputs and errors as the two).  For blocks of at
 * most 8 orbitals in FP64 with full stores the whole solve of every point --
 * forward sweep, backward sweep, bond currents and Caroli T -- runs in ONE
 * persistent launch: each wavefront takes the next point from a device work
 * queue (bound order, longest sample first) and keeps that point's blocks in
 * its registers and LDS.  The g and g^< stores are written as by
 * negf_rgf_forward, so negf_rgf_adjoint may follow.  Larger blocks, mixed
 * precision and checkpointed stores run the two calls' batched launches. */
int negf_rgf_solve(negf_ctx* ctx, void* stream, int p0, int np,
                   const negf_c128* sigma_L, const negf_c128* sigma_R,
                   const negf_c128* scat_R, const negf_c128* scat_L, int flags,
                   negf_c128* GR, negf_c128* GL, negf_c128* GG, int full_blocks,
                   int slab_stride, double* bond_j, double* transmission);

/*
 * Scattering self-energies of Eqs. (4)-(6) for a bound single-sample system
 * whose points are the full grid in (ik, ie) order (p = ik * n_e + ie):
 *   acoustic: Sigma^{R,<} = D_ac <G^{R,<}(E)>_k
 *   optical:  Sigma^<  = M_op <(1+n0) G^<(E+hw) + n0 G^<(E-hw)>_k
 *             Sigma^R  = M_op <(1+n0) G^R(E-hw) + n0 G^R(E+hw)
 *                              + G^<(E-hw)/2 - G^<(E+hw)/2>_k
 * with hw = `shift` energy-grid steps and <.>_k = sum_k w_k (.).  A (E-hw) or
 * (E+hw) group that falls off the grid is dropped from both Sigma^R and Sigma^<.
 *   GR, GL   [n_k][n_e][slab_stride][nb] orbital diagonals (negf_rgf_backward),
 *            or with atom blocks set (negf_set_scattering_blocks, opa > 1) the
 *            atom blocks [n_k][n_e][slab_stride][nb][opa] (full_blocks = 2):
 *            every entry of a block follows the same formulas
 *   w_k      [n_k] (device)
 *   sig_R, sig_L  [n_e][N][nb] (or [n_e][N][nb][opa]), updated in place
 *   rel_change    device double[1]: ||Sigma_new - Sigma_old||_F / ||Sigma_new||_F, or NULL
 * Errors: NEGF_ESTATE (not a single-sample full grid), NEGF_EINVAL. */
int negf_scba_selfenergy(negf_ctx* ctx, void* stream,
                         const negf_c128* GR, const negf_c128* GL, int slab_stride,
                         const double* w_k, double D_ac, double M_op, int shift, double n_bose,
                         negf_c128* sig_R, negf_c128* sig_L, double* rel_change);

/*
 * The residual history of the self-consistent Born loop kept on the device:
 * every negf_scba_selfenergy call appends its ||Sigma_new - Sigma_old||_F /
 * ||Sigma_new||_F to a device list (the first 4096 are kept), so a loop
 * replayed from a captured HIP graph needs no host read per iteration.  This
 * call synchronises `stream`, copies min(count, 4096, max_n) entries to the
 * HOST array out[max_n], returns in *n_out the number of calls since the
 * previous read, and clears the list.
 * Errors: NEGF_EINVAL (NULL context or n_out, max_n < 0, out NULL with max_n > 0). */
int negf_scba_history(negf_ctx* ctx, void* stream, double* out, int max_n, int* n_out);

/*
 * Observables of Eqs. (7)-(8) over the whole bound point set, summed in a
 * fixed order (deterministic, no floating-point atomics):
 *   n[s_glob][a] = g_s sum_p w_e[ie] w_k[ik] (1/2pi) sum_{o in atom a} Im G^<_oo
 *   J[s_glob]    = g_s sum_p w_e[ie] w_k[ik] j_i                         (units e/h)
 *   j_E[sample][ie][i] = g_s sum_{p at ie} w_k[ik] j_i        (spectral current, or NULL)
 * Atoms are consecutive groups of orbs_per_atom orbitals of a slab.
 *   GL [p][slab_stride][nb] orbital diagonals (gl_opa = 1) or atom blocks
 *      [p][slab_stride][nb][gl_opa] (full_blocks = 2), bond_j [p][slab_stride]
 *      (negf_rgf_backward layout)
 *   n  [total_slabs][nb / orbs_per_atom], J [total_slabs], j_E [n_samples][n_e][slab_stride]
 * Errors: NEGF_ESTATE, NEGF_EINVAL. */
int negf_observables(negf_ctx* ctx, void* stream, const negf_c128* GL, const double* bond_j,
                     int slab_stride, const double* w_e, const double* w_k, double g_s,
                     int orbs_per_atom, double* n, double* J, double* j_E, int gl_opa);

/*
 * Form of the local scattering self-energies (Eqs. 4-6 read "diag G"):
 * opa = 1 (default) keeps the orbital diagonal; opa > 1 keeps the opa x opa
 * atom blocks on the diagonal of every diagonal block (atoms are consecutive
 * groups of opa orbitals), so Sigma_scat is block-diagonal with one block per
 * atom.  Then scat_R / scat_L of negf_rgf_forward are [n_e][total_slabs][nb][opa]
 * (row o: o's entries with the orbitals of its atom), negf_rgf_backward writes
 * atom blocks with full_blocks = 2 and negf_scba_selfenergy builds the blocks
 * from them.  The one-launch small-block solve is not used with opa > 1.
 * Errors: NEGF_EINVAL (opa < 1, opa > 64, nb not a multiple), NEGF_ENOMEM. */
int negf_set_scattering_blocks(negf_ctx* ctx, int opa);

/*
 * Vector-Jacobian product of the density with respect to the onsite potential
 * (the differentiation form; the consumer is the Newton step of the
 * Poisson loop, Eq. 9).  For f = sum_o w_o n_o with n from Eq. (7):
 *   df/dV_o = sum_points c_p 2 Im[(G^< W G^R)_oo],  W = diag(w),
 * since dG^R = G^R dV G^R and dG^< = G^R dV G^< + G^< dV G^A.  (G^< W G^R) is
 * the (1,3) level of the inverse of the level-upper-triangular system
 * [[A, -Sigma^<, 0], [0, A^dagger, -W], [0, 0, A]]; its RGF reuses the g and
 * g^< the preceding negf_rgf_forward stored (same p0, np), adds a forward
 * recursion for y = g^dagger (W + H y H) g and x = g^< (W + H y H) g +
 * g (H x H) g, checkpointed every `adjoint_segment` slabs and recomputed per
 * segment, and a backward recursion for the (2,3) and (1,3) levels.
 *   w_orb  [total_slabs][nb] cotangent weight per orbital (device double)
 *   dX     out [p][slab_stride][nb]: 2 (G^< W G^R)_oo per point (complex); the
 *          per-atom gradient is then negf_observables(GL = dX): same weights
 *          g_s w_E w_k / 2pi and the same deterministic reduction.
 * Requires a context created with adjoint_segment != 0.  FP64 only.
 * Errors: NEGF_ESTATE (no matching forward sweep / no adjoint workspace), NEGF_EINVAL. */
int negf_rgf_adjoint(negf_ctx* ctx, void* stream, int p0, int np, const double* w_orb,
                     negf_c128* dX, int slab_stride);

/*
 * The two dense block kernels of every slab step, exposed on their own (the
 * zgemm / zgesv of the paper's Sec. "System and environment"), batched over
 * `batch` independent n x n matrices (row-major, contiguous, [batch][n][n]).
 *   dtype 0: complex128 operands, FP64 matrix-core arithmetic;
 *   dtype 1: complex64 operands (interleaved float pairs), FP32 matrix cores.
 * negf_zgemm_batched: C = op(A) op(B), op = 0 none, 1 conjugate transpose.
 * negf_zinv_batched:  Ainv = A^-1 by Gauss-Jordan with partial pivoting; A is
 *   overwritten (used as workspace).  Requires n <= nb and batch <= capacity of
 *   the context; a zero or non-finite pivot sets the device status word.
 * Errors: NEGF_EINVAL, NEGF_ESHAPE.
 */
int negf_zgemm_batched(negf_ctx* ctx, void* stream, int n, int batch, int opa, int opb,
                       const void* A, const void* B, void* C, int dtype);
int negf_zinv_batched(negf_ctx* ctx, void* stream, int n, int batch, void* A, void* Ainv, int dtype);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * negf_zinv_batched without a context.  Its scratch (the matrices' ping-pong
 * partner, the panel transform, the pivot rows and the row and column maps)
 * lives in one device array of NEGF_NOALLOC_SCRATCH_BYTES inside the library,
 * one copy per GPU, held until the process ends.  The call allocates nothing
 * and frees nothing; it looks the array's address up once per device (on the
 * first call with that device current).
 *   n, batch, A, Ainv, dtype   as negf_zinv_batched (A is overwritten); the
 *                              one-level Gauss-Jordan scheme is used (bitwise
 *                              the result of negf_zinv_batched with
 *                              inv_outer = 0)
 *   status  DEVICE int or NULL: zero/non-finite pivots OR the NEGF status bits
 *           (1 singular, 2 non-finite) into it; the caller clears it.
 * Requires negf_zinv_noalloc_bytes(n, batch, dtype) <= NEGF_NOALLOC_SCRATCH_BYTES
 * (n = 400: up to 22 points in FP64, 45 in FP32; n = 1200: 2 and 5), else
 * NEGF_ESHAPE; n <= 2048.
 * All calls on one GPU share its array: calls that overlap in time on one GPU
 * (different streams or host threads) race and give wrong results.  The
 * array holds the last call's contents; every byte a call reads was written
 * by that call.
 * Errors: NEGF_EINVAL, NEGF_ESHAPE, NEGF_EHIP.
 */
#define NEGF_NOALLOC_SCRATCH_BYTES (64ll << 20)
long long negf_zinv_noalloc_bytes(int n, int batch, int dtype);   /* -1 for bad arguments */
int negf_zinv_batched_noalloc(void* stream, int n, int batch, void* A, void* Ainv, int dtype, int* status);

/* Mixed-precision diagnostics of the last forward sweeps since the previous call:
 * number of block inverses redone in FP64 and the largest refinement residual
 * ||I - A X0||_F seen (host outputs; synchronises `stream`). */
int negf_mixed_stats(negf_ctx* ctx, void* stream, long long* n_fallback, double* max_residual);

/* Mixed precision: the residual ||I - A X0||_F of the FP32 block inverse X0
 * above which that block inverse is redone in FP64 (default 1e-2).  Below it the
 * one Newton-Schulz step leaves a relative inverse error of at most thr^2 plus
 * FP32 rounding, since the Frobenius norm bounds the spectral norm.  0 redoes
 * every block inverse in FP64; +infinity never does (non-finite residuals
 * still do).  Applies to later forward sweeps of the context.
 * Errors: NEGF_EINVAL for a NULL context, a negative or NaN threshold. */
int negf_set_mixed_threshold(negf_ctx* ctx, double thr);

/* Mixed precision: for each of the first n points of the last forward sweep
 * (batch order, n <= its np), the largest ||I - A X0||_F over that point's slabs,
 * written to the DEVICE array out[n] on `stream`.  The FP32 recursion loses
 * about this factor times its rounding unit on ill-conditioned points, so a
 * caller can redo points above a bound in FP64.
 * Errors: NEGF_EINVAL (NULL, n < 1), NEGF_ESTATE (not a mixed context, or no
 * forward sweep yet), NEGF_ESHAPE (n larger than the sweep). */
int negf_mixed_point_residuals(negf_ctx* ctx, void* stream, int n, double* out);

/* Batched transpose, dst[m] = src[m]^T for m < count (n x n complex128, matrix
 * m at src + m * src_stride, dst + m * dst_stride elements; DEVICE buffers that
 * must not overlap).  Its use here: each lead is in equilibrium and, where its
 * couplings are real and h00(-k) = h00(k)^T, its surface Green's function and
 * self-energy obey Sigma(-k) = Sigma(k)^T, so the lead tables of a k-point's
 * mirror need no decimation of their own.  No context; allocates nothing.
 * Errors: NEGF_EINVAL (sizes, NULL, overlap). */
int negf_transpose_batched(void* stream, int n, int count, const negf_c128* src, long long src_stride,
                           negf_c128* dst, long long dst_stride);

/* Absorbing-potential contacts (the paper treats random-alloy leads with a
 * complex absorbing potential, paragraph after Eq. 6): the contact regions are
 * slabs of the bound device itself, each carrying an imaginary onsite potential
 * -i W on every orbital, and each contact region is a reservoir at its lead's
 * Fermi level.  Writes, for every energy e, global slab s and orbital o,
 *   scat_R[e][s][o] = -i W_s,   scat_L[e][s][o] = 2 i W_s f(E_e; mu_side(s), kT)
 * (the fluctuation-dissipation pair of an absorbing self-energy), to be passed
 * as the scat_R / scat_L of negf_rgf_forward / negf_rgf_solve together with
 * ZERO lead self-energy tables (no semi-infinite leads).  w_slab: DEVICE
 * [total_slabs] W >= 0 (0 in the device region); side: DEVICE int [total_slabs],
 * < 0 for the left contact (mu_L), otherwise mu_R.  Outputs: DEVICE
 * [n_e][total_slabs][nb] complex128, every entry written.  The Caroli
 * transmission is not defined for such contacts; currents come from the bond
 * currents (Eq. 8).  Errors: NEGF_EINVAL (NULL), NEGF_ESTATE (no bound system). */
int negf_cap_selfenergy(negf_ctx* ctx, void* stream, const double* w_slab, const int* side,
                        negf_c128* scat_R, negf_c128* scat_L);

/* Mixed precision: a redo score for every bound point p (the bind's order),
 * written to the DEVICE array score[n_points] on `stream`:
 *   score[p] = resid[p] * w_e[e_p] * w_k[k_p] * max_j |Im G^<_jj(p)|,
 * the point's largest refinement residual (resid, device, one per bound point,
 * as collected from negf_mixed_point_residuals) times its largest weighted
 * contribution to the density sum of Eq. 7.  GL holds the orbital diagonals of
 * G^< of all bound points, [n_points][slab_stride][nb] complex128 (device),
 * as negf_rgf_backward writes them; w_e, w_k are the quadrature weights
 * (device).  A non-finite input gives +inf.  The FP32 error of a point's
 * density contribution grows with both factors, so a caller redoes the
 * highest-scoring points in FP64 (the residual alone misses weakly occupied
 * but ill-conditioned points and over-ranks empty ones).
 * Errors: NEGF_EINVAL (NULL pointer, slab_stride below the longest sample),
 * NEGF_ESTATE (no bound system). */
int negf_mixed_point_scores(negf_ctx* ctx, void* stream, const negf_c128* GL, int slab_stride,
                            const double* w_e, const double* w_k, const double* resid, double* score);

/* Kernel timing of the dominant kernel family (the batched complex GEMM):
 * enable = 1 records a HIP event pair around every GEMM launch on the launch
 * stream, 2 only around launches whose products run on FP64 matrix cores, 3
 * only around those on FP32 matrix cores (the block algebra of a mixed
 * context, whose lead decimation and residual products stay FP64); 0 stops.
 * negf_gemm_timing returns the launch count, summed kernel milliseconds,
 * summed algorithmic flops (8 n^3 per point per launch, of the output tiles a
 * launch computes) and the flops its matrix-core products execute (3/4 of
 * that in the three-product form, all of it for the anti-Hermitian products,
 * which use four real products) since enabling; each output may be NULL.
 * Synchronises `stream`.  Errors: NEGF_EINVAL (NULL, enable outside 0..3). */
int negf_gemm_timing_enable(negf_ctx* ctx, int enable);
int negf_gemm_timing(negf_ctx* ctx, void* stream, long long* launches, double* ms, double* flops,
                     double* mfma_flops);

/*
 * Kernel shape choices of a context (the batching form picks tile shapes by
 * measurement, not by a fixed table).
 *   gemm_prefetch  K slices of the batched GEMM in flight: 1 or 2 (default 2);
 *                  3 = two, with persistent workgroups that carry the K pipeline
 *                  from one output tile to the next (FP64 products of blocks
 *                  wider than 16; the form 2 kernel otherwise)
 *   inv_outer      outer panel width of the two-level block inverse: 0 (one
 *                  level) or a multiple of 32 in [64, 256] (default 128)
 *   inv_mid        mid block width of a three-level inverse: 0 (two levels,
 *                  default) or a multiple of 32 in [32, 256]; used when narrower
 *                  than inv_outer and the inner panels hold one row per thread
 *                  (b <= 512 in FP64): inside an outer panel the inner panels
 *                  then update only their mid block, which passes its
 *                  composite transform to the rest of the outer panel in one
 *                  rank-inv_mid product
 * negf_autotune times every candidate on the context's own workspace (block nb,
 * batch = capacity, the context's precision) with synthetic well-conditioned
 * blocks, `reps` launches each, applies the fastest and returns it.  It
 * synchronises `stream` and overwrites the workspace: call it between solves,
 * never inside a graph capture.  Results depend only on (device, nb, capacity,
 * precision), so callers may cache them and apply them with negf_set_tuning.
 * Errors: NEGF_EINVAL (bad values), NEGF_EHIP. */
typedef struct {
    int gemm_prefetch;
    int inv_outer;
    int inv_mid;
} negf_tuning;
int negf_get_tuning(const negf_ctx* ctx, negf_tuning* out);
int negf_set_tuning(negf_ctx* ctx, const negf_tuning* tuning);
int negf_autotune(negf_ctx* ctx, void* stream, int reps, negf_tuning* out);

/* ---------------------------------------------------------------------------
 * The NEGF-Poisson loop (Eq. 9: div(eps grad Phi) = e (n - N_D), iterated with
 * Eqs. (1)-(8) until the two agree).  With V = -e Phi the electron's potential
 * energy per atom (eV, the onsite potential of Eq. 1), n and N_D in electrons
 * per atom and a finite-difference grid whose nodes are the atoms (spacing h):
 *     (L V)_a = beta (n_a - N_D,a),   beta = e^2 / (eps h),
 *     (L V)_a = sum over the six neighbours b of (V_a - V_b).
 * Atom (x, z, y) has index (x * n_z + z) * n_y + y: x the slab (transport), z
 * across the body, y along the transverse direction of the k grid (periodic),
 * the same order as the density's [slab][atom] with atom = z * n_y + y.  A
 * neighbour beyond x = 0 / x = n_x - 1 is a contact held at v_left / v_right;
 * beyond a z face it is a gate at v_gate (z_gate = 1) or absent (insulating
 * face, z_gate = 0).  L0 denotes L with every boundary value zero (symmetric
 * positive definite).  All vectors are DEVICE arrays of n_x n_z n_y doubles;
 * the calls issue their kernels on `stream` and allocate nothing.
 * ------------------------------------------------------------------------- */
typedef struct {
    int n_x, n_z, n_y;
    int z_gate;
    double v_left, v_right, v_gate;
} negf_poisson_grid;

/* out = L V (with_boundary = 1) or L0 V (0).  Errors: NEGF_EINVAL. */
int negf_poisson_apply(void* stream, const negf_poisson_grid* grid, const double* V, int with_boundary,
                       double* out);

/* The loop's residual F = L V - beta (n - N_D).  Errors: NEGF_EINVAL. */
int negf_poisson_residual(void* stream, const negf_poisson_grid* grid, const double* V, const double* n_atom,
                          const double* n_d, double beta, double* F);

/* Device bytes of the `work` argument of negf_poisson_solve (-1: bad grid). */
long long negf_poisson_work_bytes(const negf_poisson_grid* grid);

/* x = (L0 + diag(shift))^-1 rhs by conjugate gradients from x = 0, until
 * ||r|| <= tol ||rhs|| or max_iter iterations (checked every 16).  shift:
 * DEVICE [atoms] diagonal (e.g. beta times minus the local part
 * of dn/dV, the preconditioner of the Newton step; negative entries count as
 * zero, so the operator stays positive definite), or NULL for L0 alone.
 * Writes the iteration count and the final relative residual (host outputs;
 * synchronises `stream`).  `work`: negf_poisson_work_bytes bytes of device
 * memory, owned by the caller.  Errors: NEGF_EINVAL, NEGF_EHIP. */
int negf_poisson_solve(void* stream, const negf_poisson_grid* grid, const double* shift, const double* rhs,
                       double* x, double tol, int max_iter, void* work, int* iters, double* rel_res);

/* The local part of the density Jacobian: for every atom a,
 *   d_a = g_s sum_p w_e w_k (1/2pi) sum_{o in a} Im(G^R_oo G^<_oo + G^<_oo conj(G^R_oo)),
 * the o' = o terms of dn_a/dV_a (the full Jacobian also has the products of
 * G_oo' and G^<_o'o within the atom and between atoms).  GR, GL: orbital
 * diagonals [p][slab_stride][nb] of the bound points (negf_rgf_backward);
 * d_out [total_slabs][nb / orbs_per_atom] (DEVICE).  Summed in the fixed
 * order of negf_observables.  Errors: NEGF_ESTATE, NEGF_EINVAL. */
int negf_density_jacobian_local(negf_ctx* ctx, void* stream, const negf_c128* GR, const negf_c128* GL,
                                int slab_stride, const double* w_e, const double* w_k, double g_s,
                                int orbs_per_atom, double* d_out);

/* Vector kernels of the Newton step's Krylov solver (device arrays; X holds m
 * vectors of length n, row j at X + j * ld).
 *   negf_vec_dots:    out[j] = sum_i X[j, i] y[i], j < m (out on the device);
 *                     `work`: negf_vec_work_bytes(n, m) bytes of device memory.
 *   negf_vec_combine: y = b y + sum_j c[j] X[j, :] (c: m device doubles; y is
 *                     not read when b = 0).
 *   negf_vec_norms:   out[0] = x . x, out[1] = max_i |x_i| (out on the device;
 *                     `work` as for negf_vec_dots with m = 1).
 * Deterministic: fixed reduction order.  Errors: NEGF_EINVAL. */
long long negf_vec_work_bytes(long long n, int m);
int negf_vec_dots(void* stream, long long n, int m, const double* X, long long ld, const double* y, double* out,
                  void* work);
int negf_vec_combine(void* stream, long long n, int m, const double* X, long long ld, const double* c, double b,
                     double* y);
int negf_vec_norms(void* stream, long long n, const double* x, double* out, void* work);

#ifdef __cplusplus
}
#endif
#endif /* NEGF_H */
