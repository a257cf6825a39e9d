// Argument blocks and launchers of the non-GEMM kernels.
#pragma once
#include "negf_internal.hpp"

namespace negf {

struct SandArgs {
    const void* X; long long sX;        // X operand per point (NULL: no sandwich term)
    const double2* hup; long long hup_k;  // H_{i,i+1} blocks and their k stride (elements)
    int ub, tile;                       // coupling block size and output tile edge
    int uslab;                          // local slab index u of U = H_{u,u+1}
    int opL, opR;                       // 0: none, 1: U, 2: U^dagger
    double sign;
    void* O; long long sO;
    int mode;                           // 0 plain, 1 retarded assembly, 2 lesser assembly
    int slab;                           // local slab index of the assembled block
    const double2* hdiag; long long hdiag_k;
    const double* v;                    // [total][n] or NULL
    const double2* scat;                // [n_e][total][n][sopa] or NULL (R for mode 1, < for mode 2)
    int sopa;                           // 1: orbital-diagonal scat; > 1: atom blocks of sopa orbitals
    long long total;
    const double2* sigL; const double2* sigR; int n_e;
    const double* energy; double eta, muL, muR, kT; int eta_fill;
    int lesser_ref;                     // mode 2: drop the f_R-equilibrium source (mixed precision)
    const double* wdiag;                // mode 3: [total][n] diagonal weights
    const double2* scat2;               // Sigma^R_scat (for lesser_ref), or NULL
    int n, np;
    Active act;
    PointSet ps;
};

struct ExtArgs {
    const void* G; const void* GL; long long sG;
    double2* outR; double2* outL; double2* outG;
    int full, slab_stride, slab, n, np, p0;   // full: 0 orbital diagonal, 1 whole block, 2 atom blocks
    int opa;                            // full = 2: orbitals per atom
    Active act;
    int lesser_ref;                     // GL holds the non-equilibrium part: add -f_R (G - G^dagger)
    const double* energy; double muR, kT;
};

struct BondArgs {
    const double2* hup; long long hup_k;
    int ub, slab;
    const void* G; const void* GL; const void* Q; const void* L; long long sM;
    const void* gls; long long s_gls;   // g^<_i (anti-Hermitian) per point
    double* partial;                    // [np][BOND_NWB]
    int n, np;
    Active act;
    PointSet ps;
};

struct SrArgs {
    const double2* h00; const double2* h01; const double2* tauin;   // [n_k][n][n]
    double2 *eps_s, *eps, *alpha, *beta, *tau;                      // [np][n][n]
    int* flags; int* iters; double* ref; int* count;
    // dual surface (the lead on the other side, coupling h01^dagger), or NULL
    double2* eps_d; double2* tau2; const double2* tauin2; int* iters2; double* ref2;
    const double* energy; double eta, tol;
    long long f0;
    int n, n_e, np;
};

// Whole-point RGF for blocks of at most 8 orbitals (one wavefront per point,
// points pulled from a device work queue).
constexpr int SMALL_NMAX = 8;
struct SmallArgs {
    const double2* hdiag; long long hdiag_k;   // [n_k][total][n][n]
    const double2* hup; long long hup_k; int ub;
    const double* v;                           // [total][n] or NULL
    const double2* scatR; const double2* scatL;   // [n_e][total][n] or NULL
    long long total;
    const double2* sigL; const double2* sigR; int n_e;
    const double* energy; double eta, muL, muR, kT; int eta_fill;
    PointSet ps; int np, n;
    double2* outR; double2* outL; double2* outG; int full, slab_stride;
    double* bond;                              // [p][slab_stride] or NULL
    double* trans;                             // [p] or NULL (no transmission)
    double2* gst; double2* glst; long long sst;   // per-point stores of g, g^< (for the adjoint)
    int* queue;                                // work-queue counter, zero at launch
    int* status;
};
hipError_t small_launch(hipStream_t s, const SmallArgs& a, int grid);

// Sancho-Rubio of one (k, E) point per wavefront for leads of at most 8
// orbitals, over the whole grid f = ik * n_e + ie < total in one launch.
struct SrSmallArgs {
    const double2* h00; const double2* h01; const double2* tau;   // [n_k][n][n]
    const double2* tau2;                        // dual surface's coupling, or NULL
    const double* energy; double eta, tol; int max_iter;
    int n, n_e, total;
    double2* sigma; double2* sigma2;            // [total][n][n] (sigma2 NULL: one surface)
    int* iters; int* iters2;                    // [total] or NULL
    int* queue; int* noconv; int* status;
};
hipError_t sr_small_launch(hipStream_t s, const SrSmallArgs& a, int grid);

struct ScbaArgs {
    const double2* GR; const double2* GL;     // [n_k][n_e][slab_stride][n]
    const double* w_k;
    double D, M, n0;
    int shift, n_k, n_e, N, n, slab_stride;
    double2* sigR; double2* sigL;             // [n_e][N][n]
    double* partial;
};

struct ObsArgs {
    const double2* GL; const double* bond;
    int slab_stride;
    const double* w_e; const double* w_k;
    double g_s;
    int opa, n, n_e, n_samples;
    int gopa;                           // GL layout: 1 orbital diagonals, > 1 atom blocks [n][gopa]
    const double2* GR;                  // non-NULL: sum Im(G^R_oo G^<_oo + G^<_oo conj(G^R_oo)) instead of
                                        // Im G^<_oo (the local part of dn/dV; orbital diagonals only)
    long long total;
    const int4* desc; const long long* slab_off; const int* slab_sample;
    const int* csr_off; const int* csr_pts;
    double* orb_tmp; double* n_out; double* J; double* jE;
};

constexpr int BOND_NWB = 64;            // partials per point of the bond-current reduction
int sandwich_tile(int ub);
size_t sandwich_lds(int ub);
hipError_t sandwich_init();
hipError_t sandwich_launch(hipStream_t s, int xdt, int odt, const SandArgs& a);
hipError_t copy_launch(hipStream_t s, int tdi, int tdo, const void* src, long long ss, void* dst, long long sd,
                       long long nel, int np, const Active& act);
hipError_t extract_launch(hipStream_t s, int dt, const ExtArgs& a);
hipError_t diag_out_launch(hipStream_t s, const double2* X, long long sX, int n, int np, const Active& act,
                           double scale, double2* out, int slab_stride, int slab, int p0);
hipError_t bond_launch(hipStream_t s, int dt, const BondArgs& a, double* out, int slab_stride);
hipError_t gamma_launch(hipStream_t s, int dt, const double2* sig, int n_e, const PointSet& ps, void* out,
                        long long so, int n, int np);
hipError_t trace_prod_launch(hipStream_t s, int dt, const void* W1, const void* W2, long long sw, int n, int np,
                             double* out, int p0);
hipError_t sr_launch_init(hipStream_t s, const SrArgs& a);
hipError_t sr_launch_zminus(hipStream_t s, const SrArgs& a, const double2* X, double2* M, const Active& act);
hipError_t sr_launch_check(hipStream_t s, const SrArgs& a, const double2* alpha, const double2* beta, int it);
hipError_t sr_launch_iters(hipStream_t s, const SrArgs& a, const int* it, int* out);
// rel_change (may be NULL) gets ||dSigma||_F / ||Sigma||_F; it is also appended to
// hist[*hcount] (while *hcount < hmax) and *hcount incremented, on the device.
hipError_t scba_launch(hipStream_t s, const ScbaArgs& a, double* rel_change, double* hist, int* hcount, int hmax);
hipError_t observables_launch(hipStream_t s, const ObsArgs& a);
// partial[2 b] = block-b maximum of |h01L - h01R^dagger|, partial[2 b + 1] = of |h01R|
hipError_t lead_dual_check_launch(hipStream_t s, const double2* h01L, const double2* h01R, int n_k, int n,
                                  double* partial, int nblk);

}  // namespace negf
