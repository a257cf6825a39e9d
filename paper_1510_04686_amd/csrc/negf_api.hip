// C ABI of the RGF library: context, binding, and the host-side schedule of
// the batched kernels (one launch per operation per slab step, covering every
// point of the batch).
#include "negf_kernels.hpp"
#include "negf.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

using namespace negf;

namespace {

constexpr int NTMP = 24;
constexpr int DUAL_NBLK = 64;   // blocks of the h01_L = h01_R^dagger check
constexpr int NBMAX_INV = 32;   // widest Gauss-Jordan panel
constexpr int EV_POOL = 2048;
constexpr int SCBA_HMAX = 4096; // SCBA residual history entries kept on the device
constexpr int SR_CHECK = 4;         // decimation iterations between host reads of the active count

struct TimedLaunch {
    hipEvent_t a, b;
    double flops;       // algorithmic: 8 n^3 per point (of the tiles computed)
    double mfma;        // executed on matrix cores: 6 n^3 (3M form) or 8 n^3 (four products)
};

}  // namespace

struct negf_ctx {
    negf_config cfg{};
    int nb = 0, nsm = 0, cap = 0, prec = 0;
    int sdt = DT_C128;            // store element type
    size_t ce = 16;               // bytes per store element
    std::vector<void*> allocs;
    void* gst = nullptr;          // [cap][nsm][nb][nb]  left-connected g^R (checkpoint mode: [cap][segK][nb][nb],
                                  // the slabs of the segment being worked on, slab i in slot i % segK)
    void* glst = nullptr;         // the same for the left-connected g^<
    bool ckpt = false;            // checkpointed stores: only the last slab of every segment is kept
    int segK = 0, segN = 0;       // slabs per segment and segments (checkpoint mode)
    void* ckg = nullptr;          // [cap][segN][nb][nb]  g at the last slab of each segment
    void* ckgl = nullptr;         // [cap][segN][nb][nb]  g^< at the last slab of each segment
    int seg_loaded = -1;          // segment whose stores the segment buffers hold (checkpoint mode)
    double2* tmp[NTMP] = {};
    void* invE = nullptr;
    void* invP = nullptr;
    void* invN0 = nullptr;        // narrow outer-panel copies of the two-level inverse
    void* invN1 = nullptr;
    int* invComp = nullptr;
    int* invComp2 = nullptr;      // mid-block composite row sources of the three-level inverse
    int* rowsrc = nullptr;
    int* piv = nullptr;
    int* coldst = nullptr;
    double* bond_partial = nullptr;
    int* sr_flags = nullptr;
    int* sr_iters = nullptr;
    double* sr_ref = nullptr;
    int* sr_iters2 = nullptr;     // dual surface (other lead) iteration counts
    double* sr_ref2 = nullptr;    // dual surface reference norms
    double* dual_partial = nullptr;
    int* d_count = nullptr;
    int* queue = nullptr;         // work-queue counter of the one-launch small-block solve
    int* status = nullptr;
    double* ns_res = nullptr;     // [cap] largest refinement residual of each point in the last forward sweep
    int* ns_flag = nullptr;       // [cap] fallback flag per point
    int* ns_count = nullptr;      // device fallback counter
    double* ns_max = nullptr;     // device: per-point max residual history (max)
    double* scba_hist = nullptr;  // [SCBA_HMAX] ||dSigma|| / ||Sigma|| of each negf_scba_selfenergy call
    int* scba_count = nullptr;    // entries appended since the last negf_scba_history
    double ns_thr = 1e-2;         // ||I - M X0||_F above which a block inverse is redone in FP64
    int scat_opa = 1;             // scattering self-energies: 1 orbital-diagonal, > 1 atom blocks of that size
    int adj_K = 0, adj_nseg = 0;  // adjoint checkpoint segment length and count
    double2* adj_yseg = nullptr;  // [cap][K][nb][nb]  y of the segment being swept
    double2* adj_xseg = nullptr;  // [cap][K][nb][nb]  x of the segment being swept
    double2* adj_yck = nullptr;   // [cap][nseg][nb][nb] y at segment ends
    double2* adj_xck = nullptr;   // [cap][nseg][nb][nb] x at segment ends
    int* h_pinned = nullptr;      // host pinned scratch
    long long ws_bytes = 0;

    // bound system
    bool bound = false;
    negf_system sys{};
    std::vector<long long> soff_h;
    std::vector<int4> desc_h;
    int n_points = 0;
    bool is_grid = false;
    std::vector<void*> bound_allocs;
    int4* desc_d = nullptr;
    long long* soff_d = nullptr;
    int* slab_sample_d = nullptr;
    int* csr_off_d = nullptr;
    int* csr_pts_d = nullptr;
    double* orb_tmp_d = nullptr;
    double* scba_partial_d = nullptr;
    double* trans_d = nullptr;

    // tuning choices (negf_set_tuning / negf_autotune)
    negf_tuning tune{2, 128, 0};

    // forward state
    bool fwd_done = false;
    int fwd_p0 = -1, fwd_np = 0, fwd_flags = 0, fwd_maxN = 0;
    const double2* fwd_sL = nullptr;   // the forward's inputs (checkpoint mode recomputes segments from them)
    const double2* fwd_sR = nullptr;
    const double2* fwd_scR = nullptr;
    const double2* fwd_scL = nullptr;

    // timing of the GEMM family
    bool timing = false;
    int timing_acc = -1;          // accumulation type to time (DT_C128 / DT_C64), -1 = every launch
    std::vector<TimedLaunch> pending;
    std::vector<hipEvent_t> ev_free;
    long long t_launches = 0;
    double t_ms = 0.0, t_flops = 0.0, t_mfma = 0.0;

    ~negf_ctx() {
        for (auto& t : pending) { hipEventDestroy(t.a); hipEventDestroy(t.b); }
        for (auto e : ev_free) hipEventDestroy(e);
        for (void* p : bound_allocs) hipFree(p);
        for (void* p : allocs) hipFree(p);
        if (h_pinned) hipHostFree(h_pinned);
    }
};

namespace {

template <typename T>
bool dev_alloc(negf_ctx* c, T** p, size_t bytes, std::vector<void*>& list) {
    if (bytes == 0) bytes = 16;
    void* q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) { hipGetLastError(); return false; }
    list.push_back(q);
    c->ws_bytes += (long long)bytes;
    *p = reinterpret_cast<T*>(q);
    return true;
}

hipError_t drain_timing(negf_ctx* c) {
    for (auto& t : c->pending) {
        hipError_t e = hipEventSynchronize(t.b);
        if (e != hipSuccess) return e;
        float ms = 0.f;
        hipEventElapsedTime(&ms, t.a, t.b);
        c->t_ms += ms;
        c->t_flops += t.flops;
        c->t_mfma += t.mfma;
        c->t_launches += 1;
        c->ev_free.push_back(t.a);
        c->ev_free.push_back(t.b);
    }
    c->pending.clear();
    return hipSuccess;
}

hipEvent_t get_event(negf_ctx* c) {
    if (c->ev_free.empty()) {
        hipEvent_t e;
        hipEventCreate(&e);
        return e;
    }
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
}

// Batched GEMM with optional timing.  `active` = number of points that do work.
hipError_t run_gemm(negf_ctx* c, hipStream_t s, GemmTypes ty, int opa, int opb, int epi, const GemmArgs& g,
                    long long active) {
    if (g.np <= 0 || active <= 0) return hipSuccess;
    GemmArgs gt = g;
    gt.pf = c->tune.gemm_prefetch;
    if (!c->timing || (c->timing_acc >= 0 && ty.acc != c->timing_acc)) return gemm_launch(s, ty, opa, opb, epi, gt);
    if ((int)c->pending.size() >= EV_POOL) {
        hipError_t e = drain_timing(c);
        if (e != hipSuccess) return e;
    }
    const double tl = (double)((g.n + 63) / 64);
    const double frac = (double)gemm_tiles(g.n, epi) / (tl * tl);   // executed share of the full product
    const double fl = 8.0 * (double)g.n * g.n * g.n * (double)active * frac;
    const bool four = epi == EPI_STORE_AH || epi == EPI_ADD_TTD_AH;   // the kernels' four-product launches
    TimedLaunch t{get_event(c), get_event(c), fl, four ? fl : 0.75 * fl};
    hipEventRecord(t.a, s);
    hipError_t e = gemm_launch(s, ty, opa, opb, epi, gt);
    hipEventRecord(t.b, s);
    c->pending.push_back(t);
    return e;
}

GemmArgs gargs(int n, int np, const Active& act) {
    GemmArgs g{};
    g.n = n;
    g.np = np;
    g.act = act;
    return g;
}

// Slab `slab` of a working store (g or g^<): every slab in the full store, or
// the slot of the segment buffer (checkpoint mode; valid while its segment is loaded).
void* slot(const negf_ctx* c, void* store, int slab) {
    const int k = c->ckpt ? slab % c->segK : slab;
    return static_cast<char*>(store) + (size_t)k * c->nb * c->nb * c->ce;
}

long long store_stride(const negf_ctx* c) { return (long long)(c->ckpt ? c->segK : c->nsm) * c->nb * c->nb; }

// Checkpoint of segment `sg` (its last slab) in ckg / ckgl.
void* ckslot(const negf_ctx* c, void* ck, int sg) {
    return static_cast<char*>(ck) + (size_t)sg * c->nb * c->nb * c->ce;
}

long long ck_stride(const negf_ctx* c) { return (long long)c->segN * c->nb * c->nb; }

// Active point counts and grid extents over [p0, p0+np) for predicate mode at step.
void extent(const negf_ctx* c, int p0, int np, int mode, int step, int* hi, long long* cnt) {
    int h = 0;
    long long k = 0;
    for (int q = 0; q < np; ++q) {
        int ns = c->desc_h[p0 + q].w;
        bool a = (mode == PRED_FWD) ? (step < ns) : (mode == PRED_BWD) ? (step < ns - 1)
               : (mode == PRED_INIT) ? (step == ns - 1) : true;
        if (a) { h = q + 1; ++k; }
    }
    *hi = h;
    *cnt = k;
}

SandArgs sand_base(const negf_ctx* c, int p0, const Active& act, int np) {
    SandArgs a{};
    const negf_system& S = c->sys;
    a.hup = reinterpret_cast<const double2*>(S.h_up);
    a.hup_k = S.h_up_k_stride;
    a.ub = S.up_block;
    a.tile = sandwich_tile(S.up_block);
    a.hdiag = reinterpret_cast<const double2*>(S.h_diag);
    a.hdiag_k = c->soff_h.back() * (long long)c->nb * c->nb;
    a.v = S.v_onsite;
    a.total = c->soff_h.back();
    a.n_e = S.n_e;
    a.energy = S.energy;
    a.eta = S.eta;
    a.muL = S.mu_L;
    a.muR = S.mu_R;
    a.kT = S.kT;
    a.eta_fill = S.eta_fill;
    a.sopa = c->scat_opa;
    a.n = c->nb;
    a.np = np;
    a.act = act;
    a.ps = PointSet{c->desc_d, c->soff_d, p0};
    a.sign = 1.0;
    return a;
}

InvWork invwork(negf_ctx* c, void* partner) {
    return InvWork{partner, c->invE, c->invP, c->rowsrc, c->piv, c->coldst, c->status,
                   c->invN0, c->invN1, c->invComp, c->invN0 ? c->tune.inv_outer : 0,
                   c->invComp2, c->invN0 ? c->tune.inv_mid : 0};
}

// Synthetic well-conditioned blocks for timing: entries in [-1, 1) from an
// integer hash, plus `diag` on the diagonal.
template <typename C>
__global__ void tune_fill_kernel(C* M, long long nn, int n, long long total, double diag) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    unsigned long long h = (unsigned long long)i * 0x9E3779B97F4A7C15ull;
    h ^= h >> 29; h *= 0xBF58476D1CE4E5B9ull; h ^= h >> 32;
    const double re = (double)(h & 0xFFFFF) / 524288.0 - 1.0, im = (double)((h >> 20) & 0xFFFFF) / 524288.0 - 1.0;
    const long long e = i % nn;
    const int r = (int)(e / n), c = (int)(e - (long long)r * n);
    C v; v.x = re + (r == c ? diag : 0.0); v.y = im;
    M[i] = v;
}

__global__ void fill_int_kernel(int* p, int v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void copy_d_kernel(const double* a, double* b, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// Mixed precision: per-point Frobenius norm of the refinement residual
// R = I - M X0; flags a fallback when it exceeds `thr`.  ||R||_F bounds the
// spectral norm, so below the threshold one Newton-Schulz step X1 = X0 + X0 R
// leaves a relative inverse error of at most ||R||_F^2 (plus FP32 rounding).
__global__ __launch_bounds__(256) void ns_check_kernel(const double2* R, long long sR, int n, int np, Active act,
                                                       double thr, double* res, int* flag, int* count, double* histmax,
                                                       int* status) {
    const int q = blockIdx.x;
    if (q >= np) return;
    __shared__ double red[256];
    double m = 0.0;
    bool on = act(q);
    if (on) {
        const double2* X = R + q * sR;
        for (long long i = threadIdx.x; i < (long long)n * n; i += 256) {
            double2 v = X[i];
            m = fma(v.x, v.x, fma(v.y, v.y, m));
        }
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double r = on ? sqrt(red[0]) : 0.0;
        if (!(r == r)) r = INFINITY;
        if (on && r > res[q]) res[q] = r;
        int f = (on && !(r <= thr)) ? 1 : 0;
        flag[q] = f;
        if (f && count) atomicAdd(count, 1);
        if (f) raise_status(status, ST_FALLBACK);
        if (on && histmax && r > histmax[q]) histmax[q] = r;
    }
}

__global__ void zero_d_kernel(double* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Absorbing-potential contact self-energies, one thread per (energy, slab,
// orbital): Sigma^R = -i W_s, Sigma^< = 2 i W_s f(E; mu of the slab's contact).
__global__ __launch_bounds__(256) void cap_kernel(const double* energy, int n_e, long long total, int n,
                                                  const double* w, const int* side, double muL, double muR,
                                                  double kT, double2* sR, double2* sL) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long per_e = total * n;
    if (i >= per_e * n_e) return;
    const int ie = (int)(i / per_e);
    const long long s = (i - ie * per_e) / n;
    const double W = w[s];
    double f = 0.0;
    if (W != 0.0) {
        const double mu = side[s] < 0 ? muL : muR;
        f = 1.0 / (1.0 + exp((energy[ie] - mu) / kT));
    }
    sR[i] = make_double2(0.0, -W);
    sL[i] = make_double2(0.0, 2.0 * W * f);
}

// dst[m] = src[m]^T for a batch of n x n complex matrices: 32 x 32 tiles staged
// through LDS so that both the reads and the writes run along rows.
__global__ __launch_bounds__(256) void transpose_kernel(const double2* src, long long ss, double2* dst, long long sd,
                                                        int n) {
    __shared__ double2 t[32][33];
    const int tiles = (n + 31) / 32;
    const int m = blockIdx.y;
    const int r0 = (blockIdx.x / tiles) * 32, c0 = (blockIdx.x % tiles) * 32;
    const double2* S = src + (long long)m * ss;
    double2* D = dst + (long long)m * sd;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;     // 32 x 8 threads
    for (int y = ty; y < 32; y += 8) {
        const int r = r0 + y, c = c0 + tx;
        if (r < n && c < n) t[y][tx] = S[(long long)r * n + c];
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int r = c0 + y, c = r0 + tx;                       // element (c, r) of S
        if (r < n && c < n) D[(long long)r * n + c] = t[tx][y];
    }
}

// Mixed precision: per-point redo score = (largest block refinement residual of
// the point) x (its energy and k weights) x (largest |Im G^<_jj| over its
// orbitals), i.e. the residual times the point's largest contribution to the
// density sum of Eq. 7.  One workgroup per point; a non-finite entry gives +inf.
__global__ __launch_bounds__(256) void mixed_score_kernel(const double2* GL, int slab_stride, int n,
                                                          const int4* desc, const double* w_e, const double* w_k,
                                                          const double* resid, double* score) {
    const int p = blockIdx.x;
    const int4 d = desc[p];
    const long long m = (long long)d.w * n;
    const double2* X = GL + (long long)p * slab_stride * n;
    __shared__ double red[256];
    double mx = 0.0;
    for (long long i = threadIdx.x; i < m; i += 256) {
        const double v = fabs(X[i].y);
        mx = (v <= mx) ? mx : v;          // NaN propagates
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double u = red[threadIdx.x + o];
            if (!(u <= red[threadIdx.x])) red[threadIdx.x] = u;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double r = resid[p] * w_e[d.z] * w_k[d.y] * red[0];
        if (!(r == r) || !(red[0] < INFINITY) || !(resid[p] < INFINITY)) r = INFINITY;
        score[p] = r;
    }
}

}  // namespace

// ===========================================================================
extern "C" {

const char* negf_error_string(int st) {
    switch (st) {
        case NEGF_OK: return "ok";
        case NEGF_EINVAL: return "invalid argument";
        case NEGF_ESHAPE: return "sizes exceed the context configuration";
        case NEGF_ENOMEM: return "device allocation failed";
        case NEGF_EHIP: return "HIP runtime error";
        case NEGF_ESTATE: return "call order violated (no bound system or no forward sweep)";
        case NEGF_WNOCONV: return "Sancho-Rubio decimation hit max_iter for some point";
        case NEGF_WSINGULAR: return "a block inverse met an exactly zero pivot";
        case NEGF_WNONFINITE: return "a block inverse met a non-finite pivot";
        case NEGF_WFALLBACK: return "mixed precision redid some block inverses in FP64";
        default: return "unknown status";
    }
}

int negf_create(const negf_config* cfg, negf_ctx** out) {
    if (!cfg || !out) return NEGF_EINVAL;
    *out = nullptr;
    if (cfg->nb < 1 || cfg->nb > INV_NMAX || cfg->n_slab_max < 1 || cfg->capacity < 1) return NEGF_EINVAL;
    if (cfg->store_checkpoint != 0 && cfg->store_checkpoint != 1) return NEGF_EINVAL;
    if (cfg->precision != NEGF_FP64 && cfg->precision != NEGF_MIXED) return NEGF_EINVAL;
    negf_ctx* c = new (std::nothrow) negf_ctx();
    if (!c) return NEGF_ENOMEM;
    c->cfg = *cfg;
    c->nb = cfg->nb;
    c->nsm = cfg->n_slab_max;
    c->cap = cfg->capacity;
    c->prec = cfg->precision;
    c->sdt = (c->prec == NEGF_MIXED) ? DT_C64 : DT_C128;
    c->ce = (c->prec == NEGF_MIXED) ? 8 : 16;
    const size_t nn = (size_t)c->nb * c->nb;
    const size_t cap = (size_t)c->cap;
    // checkpointed stores: segments of K slabs (K = adjoint_segment when given,
    // else ceil(sqrt(n_slab_max))); the adjoint then uses the same segments
    int K0 = cfg->adjoint_segment > 0 ? cfg->adjoint_segment : (int)std::ceil(std::sqrt((double)c->nsm));
    K0 = std::max(1, std::min(K0, c->nsm));
    c->ckpt = cfg->store_checkpoint != 0;
    if (c->ckpt) { c->segK = K0; c->segN = (c->nsm + K0 - 1) / K0; }
    const size_t slots = c->ckpt ? (size_t)c->segK : (size_t)c->nsm;
    bool ok = dev_alloc(c, &c->gst, cap * slots * nn * c->ce, c->allocs) &&
              dev_alloc(c, &c->glst, cap * slots * nn * c->ce, c->allocs) &&
              (!c->ckpt || (dev_alloc(c, &c->ckg, cap * c->segN * nn * c->ce, c->allocs) &&
                            dev_alloc(c, &c->ckgl, cap * c->segN * nn * c->ce, c->allocs)));
    for (int i = 0; ok && i < NTMP; ++i) ok = dev_alloc(c, &c->tmp[i], cap * nn * sizeof(double2), c->allocs);
    ok = ok && dev_alloc(c, &c->invE, cap * c->nb * NBMAX_INV * sizeof(double2), c->allocs) &&
         dev_alloc(c, &c->invP, cap * c->nb * NBMAX_INV * sizeof(double2), c->allocs) &&
         (c->nb <= 64 || (dev_alloc(c, &c->invN0, cap * c->nb * INV_WMAX * sizeof(double2), c->allocs) &&
                          dev_alloc(c, &c->invN1, cap * c->nb * INV_WMAX * sizeof(double2), c->allocs) &&
                          dev_alloc(c, &c->invComp, cap * c->nb * sizeof(int), c->allocs) &&
                          dev_alloc(c, &c->invComp2, cap * c->nb * sizeof(int), c->allocs))) &&
         dev_alloc(c, &c->rowsrc, cap * c->nb * sizeof(int), c->allocs) &&
         dev_alloc(c, &c->piv, cap * c->nb * sizeof(int), c->allocs) &&
         dev_alloc(c, &c->coldst, cap * c->nb * sizeof(int), c->allocs) &&
         dev_alloc(c, &c->bond_partial, cap * BOND_NWB * sizeof(double), c->allocs) &&
         dev_alloc(c, &c->sr_flags, cap * sizeof(int), c->allocs) &&
         dev_alloc(c, &c->sr_iters, cap * sizeof(int), c->allocs) &&
         dev_alloc(c, &c->sr_ref, cap * sizeof(double), c->allocs) &&
         dev_alloc(c, &c->sr_iters2, cap * sizeof(int), c->allocs) &&
         dev_alloc(c, &c->sr_ref2, cap * sizeof(double), c->allocs) &&
         dev_alloc(c, &c->dual_partial, 2 * DUAL_NBLK * sizeof(double), c->allocs) &&
         dev_alloc(c, &c->d_count, 4 * sizeof(int), c->allocs) &&
         dev_alloc(c, &c->queue, 4 * sizeof(int), c->allocs) &&
         dev_alloc(c, &c->status, 4 * sizeof(int), c->allocs) &&
         dev_alloc(c, &c->ns_res, cap * sizeof(double), c->allocs) &&
         dev_alloc(c, &c->ns_flag, cap * sizeof(int), c->allocs) &&
         dev_alloc(c, &c->ns_count, 4 * sizeof(int), c->allocs) &&
         dev_alloc(c, &c->ns_max, cap * sizeof(double), c->allocs) &&
         dev_alloc(c, &c->scba_hist, SCBA_HMAX * sizeof(double), c->allocs) &&
         dev_alloc(c, &c->scba_count, 4 * sizeof(int), c->allocs);
    if (ok && cfg->adjoint_segment != 0) {
        const int K = K0;
        c->adj_K = K;
        c->adj_nseg = (c->nsm + K - 1) / K;
        ok = dev_alloc(c, &c->adj_yseg, cap * K * nn * sizeof(double2), c->allocs) &&
             dev_alloc(c, &c->adj_xseg, cap * K * nn * sizeof(double2), c->allocs) &&
             dev_alloc(c, &c->adj_yck, cap * c->adj_nseg * nn * sizeof(double2), c->allocs) &&
             dev_alloc(c, &c->adj_xck, cap * c->adj_nseg * nn * sizeof(double2), c->allocs);
    }
    if (ok && hipHostMalloc((void**)&c->h_pinned, 64) != hipSuccess) { c->h_pinned = nullptr; ok = false; }
    if (!ok) { delete c; return NEGF_ENOMEM; }
    if (inverse_init() != hipSuccess || sandwich_init() != hipSuccess) { delete c; return NEGF_EHIP; }
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, 0, c->status, 0, 4);
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, 0, c->ns_count, 0, 4);
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, 0, c->scba_count, 0, 4);
    hipLaunchKernelGGL(zero_d_kernel, dim3((c->cap + 255) / 256), dim3(256), 0, 0, c->ns_max, c->cap);
    if (hipDeviceSynchronize() != hipSuccess) { delete c; return NEGF_EHIP; }
    *out = c;
    return NEGF_OK;
}

void negf_destroy(negf_ctx* c) { delete c; }

#ifndef NEGF_BUILD_ID
#error "NEGF_BUILD_ID (the SHA-1 of the sources) must be defined by the build"
#endif
const char* negf_build_id(void) { return NEGF_BUILD_ID; }

long long negf_workspace_bytes(const negf_ctx* c) { return c ? c->ws_bytes : 0; }

int negf_sync_status(negf_ctx* c, void* stream) {
    if (!c) return NEGF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    NEGF_HIP_CHECK(hipMemcpyAsync(c->h_pinned, c->status, sizeof(int), hipMemcpyDeviceToHost, s));
    NEGF_HIP_CHECK(hipStreamSynchronize(s));
    int st = c->h_pinned[0];
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, s, c->status, 0, 1);
    NEGF_HIP_CHECK(hipGetLastError());
    if (st & ST_NONFINITE) return NEGF_WNONFINITE;
    if (st & ST_SINGULAR) return NEGF_WSINGULAR;
    if (st & ST_FALLBACK) return NEGF_WFALLBACK;
    return NEGF_OK;
}

int negf_bind(negf_ctx* c, const negf_system* S, int n_points, const int* points) {
    if (!c || !S || !points || n_points < 1) return NEGF_EINVAL;
    if (S->nb != c->nb) return NEGF_ESHAPE;
    if (S->n_samples < 1 || !S->slab_offset || S->n_k < 1 || S->n_e < 1) return NEGF_EINVAL;
    if (!S->h_diag || !S->h_up || !S->energy) return NEGF_EINVAL;
    if (S->up_block < 1 || S->up_block > 48 || S->nb % S->up_block != 0) return NEGF_EINVAL;
    if (!(S->kT > 0) || !(S->eta >= 0)) return NEGF_EINVAL;
    if (S->h_up_k_stride < 0) return NEGF_EINVAL;
    std::vector<long long> soff(S->slab_offset, S->slab_offset + S->n_samples + 1);
    if (soff[0] != 0) return NEGF_EINVAL;
    for (int s = 0; s < S->n_samples; ++s) {
        long long ns = soff[s + 1] - soff[s];
        if (ns < 1) return NEGF_EINVAL;
        if (ns > c->nsm) return NEGF_ESHAPE;
    }
    std::vector<int4> desc(n_points);
    for (int p = 0; p < n_points; ++p) {
        int s = points[3 * p], k = points[3 * p + 1], e = points[3 * p + 2];
        if (s < 0 || s >= S->n_samples || k < 0 || k >= S->n_k || e < 0 || e >= S->n_e) return NEGF_EINVAL;
        desc[p] = make_int4(s, k, e, (int)(soff[s + 1] - soff[s]));
    }
    for (void* p : c->bound_allocs) hipFree(p);
    c->bound_allocs.clear();
    c->bound = false;
    c->fwd_done = false;
    const long long total = soff.back();
    // slab -> sample map, (sample, ie) -> points CSR
    std::vector<int> slab_sample(total);
    for (int s = 0; s < S->n_samples; ++s)
        for (long long i = soff[s]; i < soff[s + 1]; ++i) slab_sample[i] = s;
    const long long nkey = (long long)S->n_samples * S->n_e;
    std::vector<int> csr_off(nkey + 1, 0), csr_pts(n_points);
    for (int p = 0; p < n_points; ++p) csr_off[(long long)desc[p].x * S->n_e + desc[p].z + 1]++;
    for (long long k = 0; k < nkey; ++k) csr_off[k + 1] += csr_off[k];
    {
        std::vector<int> fill(csr_off.begin(), csr_off.end() - 1);
        for (int p = 0; p < n_points; ++p) csr_pts[fill[(long long)desc[p].x * S->n_e + desc[p].z]++] = p;
    }
    bool grid = (S->n_samples == 1 && (long long)n_points == (long long)S->n_k * S->n_e);
    for (int p = 0; grid && p < n_points; ++p)
        grid = desc[p].y == p / S->n_e && desc[p].z == p % S->n_e;
    bool ok = dev_alloc(c, &c->desc_d, n_points * sizeof(int4), c->bound_allocs) &&
              dev_alloc(c, &c->soff_d, soff.size() * sizeof(long long), c->bound_allocs) &&
              dev_alloc(c, &c->slab_sample_d, total * sizeof(int), c->bound_allocs) &&
              dev_alloc(c, &c->csr_off_d, csr_off.size() * sizeof(int), c->bound_allocs) &&
              dev_alloc(c, &c->csr_pts_d, n_points * sizeof(int), c->bound_allocs) &&
              dev_alloc(c, &c->orb_tmp_d, total * c->nb * sizeof(double), c->bound_allocs) &&
              dev_alloc(c, &c->trans_d, n_points * sizeof(double), c->bound_allocs);
    if (ok && grid) {
        long long nblk = ((long long)S->n_e * total * c->nb * c->scat_opa + 255) / 256;
        ok = dev_alloc(c, &c->scba_partial_d, nblk * 2 * sizeof(double), c->bound_allocs);
    }
    if (!ok) return NEGF_ENOMEM;
    NEGF_HIP_CHECK(hipMemcpy(c->desc_d, desc.data(), n_points * sizeof(int4), hipMemcpyHostToDevice));
    NEGF_HIP_CHECK(hipMemcpy(c->soff_d, soff.data(), soff.size() * sizeof(long long), hipMemcpyHostToDevice));
    NEGF_HIP_CHECK(hipMemcpy(c->slab_sample_d, slab_sample.data(), total * sizeof(int), hipMemcpyHostToDevice));
    NEGF_HIP_CHECK(hipMemcpy(c->csr_off_d, csr_off.data(), csr_off.size() * sizeof(int), hipMemcpyHostToDevice));
    NEGF_HIP_CHECK(hipMemcpy(c->csr_pts_d, csr_pts.data(), n_points * sizeof(int), hipMemcpyHostToDevice));
    c->sys = *S;
    c->sys.slab_offset = nullptr;   // host copy kept in soff_h
    c->soff_h = soff;
    c->desc_h = desc;
    c->n_points = n_points;
    c->is_grid = grid;
    c->bound = true;
    return NEGF_OK;
}

}  // extern "C"

// Sancho-Rubio over the (k, E) grid in batches of `capacity` points; writes
// Sigma = tau g_s tau^dagger to `sigma`.  With `sigma2` set, the same
// decimation also carries the dual surface: the lead on the other side of the
// device, whose coupling into the lead is h01^dagger (alpha and beta swap
// roles, so only the surface accumulator is extra); its self-energy
// tau2 g_s' tau2^dagger goes to `sigma2`.
static int lead_sr(negf_ctx* c, hipStream_t s, int n_k, const negf_c128* h00, const negf_c128* h01,
                   const negf_c128* tau, int n_e, const double* energy, double eta, double tol, int max_iter,
                   negf_c128* sigma, int* iters, const negf_c128* tau2, negf_c128* sigma2, int* iters2) {
    const int n = c->nb;
    const long long nn = (long long)n * n;
    const long long total = (long long)n_k * n_e;
    const GemmTypes T64{DT_C128, DT_C128, DT_C128, DT_C128};
    const bool dual = sigma2 != nullptr;
    if (n <= SMALL_NMAX && total <= (1ll << 30)) {
        // small leads: every (k, E) point decimated to convergence in one launch
        SrSmallArgs a{};
        a.h00 = reinterpret_cast<const double2*>(h00);
        a.h01 = reinterpret_cast<const double2*>(h01);
        a.tau = reinterpret_cast<const double2*>(tau);
        a.tau2 = reinterpret_cast<const double2*>(tau2);
        a.energy = energy; a.eta = eta; a.tol = tol; a.max_iter = max_iter;
        a.n = n; a.n_e = n_e; a.total = (int)total;
        a.sigma = reinterpret_cast<double2*>(sigma);
        a.sigma2 = reinterpret_cast<double2*>(sigma2);
        a.iters = iters; a.iters2 = iters2;
        a.queue = c->queue; a.noconv = c->queue + 1; a.status = c->status;
        hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, s, c->queue, 0, 2);
        NEGF_HIP_CHECK(hipGetLastError());
        NEGF_HIP_CHECK(sr_small_launch(s, a, (int)std::min<long long>(total, 256 * 8)));
        NEGF_HIP_CHECK(hipMemcpyAsync(c->h_pinned, c->queue + 1, sizeof(int), hipMemcpyDeviceToHost, s));
        NEGF_HIP_CHECK(hipStreamSynchronize(s));
        return c->h_pinned[0] > 0 ? NEGF_WNOCONV : NEGF_OK;
    }
    bool noconv = false;
    for (long long f0 = 0; f0 < total; f0 += c->cap) {
        const int cnt = (int)std::min<long long>(c->cap, total - f0);
        SrArgs a{};
        a.h00 = reinterpret_cast<const double2*>(h00);
        a.h01 = reinterpret_cast<const double2*>(h01);
        a.tauin = reinterpret_cast<const double2*>(tau);
        a.eps_s = c->tmp[0]; a.eps = c->tmp[1]; a.alpha = c->tmp[2]; a.beta = c->tmp[3]; a.tau = c->tmp[13];
        a.flags = c->sr_flags; a.iters = c->sr_iters; a.ref = c->sr_ref; a.count = c->d_count;
        if (dual) {
            a.eps_d = c->tmp[4]; a.tau2 = c->tmp[5]; a.tauin2 = reinterpret_cast<const double2*>(tau2);
            a.iters2 = c->sr_iters2; a.ref2 = c->sr_ref2;
        }
        a.energy = energy; a.eta = eta; a.tol = tol; a.f0 = f0; a.n = n; a.n_e = n_e; a.np = cnt;
        NEGF_HIP_CHECK(sr_launch_init(s, a));
        double2 *al = c->tmp[2], *be = c->tmp[3], *al2 = c->tmp[6], *be2 = c->tmp[7];
        double2 *g = c->tmp[8], *X1 = c->tmp[9], *X2 = c->tmp[10], *M = c->tmp[11];
        long long active = cnt;
        for (int it = 1; it <= max_iter && active > 0; ++it) {
            Active act{c->desc_d, 0, 0, PRED_FLAG, c->sr_flags};
            NEGF_HIP_CHECK(sr_launch_zminus(s, a, a.eps, M, act));
            NEGF_HIP_CHECK(inverse_launch(s, DT_C128, M, nn, g, nn, n, cnt, act, invwork(c, c->tmp[12])));
            GemmArgs G = gargs(n, cnt, act);
            G.A = al; G.sA = nn; G.B = g; G.sB = nn; G.C = X1; G.sC = nn;
            NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_N, OP_N, EPI_STORE, G, active));
            G.A = be; G.C = X2;
            NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_N, OP_N, EPI_STORE, G, active));
            // eps_s += X1 beta ; eps += X1 beta
            G.A = X1; G.B = be; G.C = a.eps_s; G.C2 = a.eps; G.sC2 = nn;
            NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_N, OP_N, EPI_DUAL, G, active));
            // eps += X2 alpha  (and eps_dual += X2 alpha)
            G.A = X2; G.B = al;
            if (dual) {
                G.C = a.eps_d; G.C2 = a.eps; G.sC2 = nn;
                NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_N, OP_N, EPI_DUAL, G, active));
            } else {
                G.C = a.eps; G.D = a.eps; G.sD = nn;
                NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_N, OP_N, EPI_ADD, G, active));
            }
            // alpha' = X1 alpha ; beta' = X2 beta
            G = gargs(n, cnt, act);
            G.A = X1; G.sA = nn; G.B = al; G.sB = nn; G.C = al2; G.sC = nn;
            NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_N, OP_N, EPI_STORE, G, active));
            G.A = X2; G.B = be; G.C = be2;
            NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_N, OP_N, EPI_STORE, G, active));
            std::swap(al, al2);
            std::swap(be, be2);
            hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, s, c->d_count, 0, 1);
            NEGF_HIP_CHECK(sr_launch_check(s, a, al, be, it));
            // The host reads the active count every SR_CHECK iterations only: a point
            // that has converged is frozen (its workgroups exit at once and its flag
            // stays set), so the iterations run past the last convergence change
            // nothing, and the loop needs a quarter of the host synchronisations.
            // With GEMM timing on, every iteration's count is read: the timed launches
            // are credited with the products of the points still active.
            if (c->timing || it % SR_CHECK == 0 || it == max_iter) {
                NEGF_HIP_CHECK(hipMemcpyAsync(c->h_pinned, c->d_count, sizeof(int), hipMemcpyDeviceToHost, s));
                NEGF_HIP_CHECK(hipStreamSynchronize(s));
                active = c->h_pinned[0];
            }
        }
        if (active > 0) noconv = true;
        // g_s = (z - eps_s)^-1 ; Sigma = tau g_s tau^dagger  (then the same for the dual surface)
        Active all{c->desc_d, 0, 0, PRED_ALL, nullptr};
        for (int side = 0; side < (dual ? 2 : 1); ++side) {
            const double2* es = side ? a.eps_d : a.eps_s;
            const double2* tq = side ? a.tau2 : a.tau;
            negf_c128* out = side ? sigma2 : sigma;
            NEGF_HIP_CHECK(sr_launch_zminus(s, a, es, M, all));
            NEGF_HIP_CHECK(inverse_launch(s, DT_C128, M, nn, g, nn, n, cnt, all, invwork(c, c->tmp[12])));
            GemmArgs G = gargs(n, cnt, all);
            G.A = tq; G.sA = nn; G.B = g; G.sB = nn; G.C = X1; G.sC = nn;
            NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_N, OP_N, EPI_STORE, G, cnt));
            G.A = X1; G.B = tq; G.C = reinterpret_cast<double2*>(out) + f0 * nn;
            NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_N, OP_C, EPI_STORE, G, cnt));
        }
        if (iters) NEGF_HIP_CHECK(sr_launch_iters(s, a, c->sr_iters, iters));
        if (dual && iters2) NEGF_HIP_CHECK(sr_launch_iters(s, a, c->sr_iters2, iters2));
    }
    return noconv ? NEGF_WNOCONV : NEGF_OK;
}

extern "C" {

int negf_lead_selfenergy(negf_ctx* c, void* stream, int n_k, const negf_c128* h00, const negf_c128* h01,
                         const negf_c128* tau, int n_e, const double* energy, double eta, double tol,
                         int max_iter, negf_c128* sigma, int* iters) {
    if (!c || !h00 || !h01 || !tau || !energy || !sigma) return NEGF_EINVAL;
    if (n_k < 1 || n_e < 1 || max_iter < 1 || !(tol > 0) || !(eta >= 0)) return NEGF_EINVAL;
    return lead_sr(c, (hipStream_t)stream, n_k, h00, h01, tau, n_e, energy, eta, tol, max_iter, sigma, iters,
                   nullptr, nullptr, nullptr);
}

int negf_lead_selfenergy_pair(negf_ctx* c, void* stream, int n_k, const negf_c128* h00, const negf_c128* h01_L,
                              const negf_c128* tau_L, const negf_c128* h01_R, const negf_c128* tau_R, int n_e,
                              const double* energy, double eta, double tol, int max_iter, negf_c128* sigma_L,
                              negf_c128* sigma_R, int* iters_L, int* iters_R, int* dual_used) {
    if (!c || !h00 || !h01_L || !tau_L || !h01_R || !tau_R || !energy || !sigma_L || !sigma_R) return NEGF_EINVAL;
    if (n_k < 1 || n_e < 1 || max_iter < 1 || !(tol > 0) || !(eta >= 0)) return NEGF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    NEGF_HIP_CHECK(lead_dual_check_launch(s, reinterpret_cast<const double2*>(h01_L),
                                          reinterpret_cast<const double2*>(h01_R), n_k, c->nb, c->dual_partial,
                                          DUAL_NBLK));
    double part[2 * DUAL_NBLK];
    NEGF_HIP_CHECK(hipMemcpyAsync(part, c->dual_partial, sizeof(part), hipMemcpyDeviceToHost, s));
    NEGF_HIP_CHECK(hipStreamSynchronize(s));
    double dev = 0.0, scale = 0.0;
    for (int b = 0; b < DUAL_NBLK; ++b) { dev = std::max(dev, part[2 * b]); scale = std::max(scale, part[2 * b + 1]); }
    const bool dual = dev <= 1e-15 * scale;
    if (dual_used) *dual_used = dual ? 1 : 0;
    if (dual)
        return lead_sr(c, s, n_k, h00, h01_R, tau_R, n_e, energy, eta, tol, max_iter, sigma_R, iters_R, tau_L,
                       sigma_L, iters_L);
    int a = lead_sr(c, s, n_k, h00, h01_L, tau_L, n_e, energy, eta, tol, max_iter, sigma_L, iters_L, nullptr,
                    nullptr, nullptr);
    if (a < 0) return a;
    int b = lead_sr(c, s, n_k, h00, h01_R, tau_R, n_e, energy, eta, tol, max_iter, sigma_R, iters_R, nullptr,
                    nullptr, nullptr);
    if (b < 0) return b;
    return std::max(a, b);
}

}  // extern "C"

// One slab of the forward sweep for points [p0, p0 + np): reads g_{i-1} and
// g^<_{i-1} at (gp, glp) with point stride sp (unused at i = 0) and writes g_i,
// g^<_i to the working stores (slot(i)).  With `stats` false (a checkpoint
// segment being recomputed) the mixed-precision fallback counter and residual
// history are not touched again.
static int fwd_slab(negf_ctx* c, hipStream_t s, int p0, int np, int i, const void* gp, const void* glp,
                    long long sp, bool stats) {
    const int n = c->nb;
    const long long nn = (long long)n * n;
    const long long sst = store_stride(c);
    const bool mixed = c->prec == NEGF_MIXED;
    const int sdt = c->sdt;
    const GemmTypes TS{sdt, sdt, sdt, sdt};
    int hi;
    long long cnt;
    extent(c, p0, np, PRED_FWD, i, &hi, &cnt);
    if (cnt == 0) return NEGF_OK;
    Active act{c->desc_d, p0, i, PRED_FWD, nullptr};
    // M = A_ii - H_{i,i-1} g_{i-1} H_{i-1,i}   (FP64 assembly)
    SandArgs sa = sand_base(c, p0, act, hi);
    sa.sigL = c->fwd_sL; sa.sigR = c->fwd_sR;
    sa.X = (i > 0) ? gp : nullptr; sa.sX = sp;
    sa.uslab = i - 1; sa.opL = 2; sa.opR = 1; sa.sign = -1.0;
    sa.O = c->tmp[0]; sa.sO = nn; sa.mode = 1; sa.slab = i;
    sa.scat = c->fwd_scR;
    NEGF_HIP_CHECK(sandwich_launch(s, sdt, DT_C128, sa));
    if (!mixed) {
        NEGF_HIP_CHECK(inverse_launch(s, DT_C128, c->tmp[0], nn, slot(c, c->gst, i), sst, n, hi, act,
                                      invwork(c, c->tmp[3])));
    } else {
        // X0 = M^-1 in FP32, R = I - M X0 in FP64, X1 = X0 + X0 R in FP32.
        Active all{c->desc_d, p0, i, PRED_FWD, nullptr};
        NEGF_HIP_CHECK(copy_launch(s, DT_C128, DT_C64, c->tmp[0], nn, c->tmp[4], nn, nn, hi, act));
        NEGF_HIP_CHECK(inverse_launch(s, DT_C64, c->tmp[4], nn, c->tmp[2], nn, n, hi, act,
                                      invwork(c, c->tmp[3])));
        GemmArgs G = gargs(n, hi, act);
        G.A = c->tmp[0]; G.sA = nn; G.B = c->tmp[2]; G.sB = nn; G.C = c->tmp[1]; G.sC = nn;
        NEGF_HIP_CHECK(run_gemm(c, s, GemmTypes{DT_C128, DT_C64, DT_C128, DT_C128}, OP_N, OP_N, EPI_IMINUS, G, cnt));
        hipLaunchKernelGGL(ns_check_kernel, dim3(hi), dim3(256), 0, s, c->tmp[1], nn, n, hi, all, c->ns_thr,
                           c->ns_res, c->ns_flag, stats ? c->ns_count : nullptr, stats ? c->ns_max : nullptr,
                           c->status);
        NEGF_HIP_CHECK(hipGetLastError());
        G.A = c->tmp[2]; G.B = c->tmp[1]; G.D = c->tmp[2]; G.sD = nn; G.C = slot(c, c->gst, i); G.sC = sst;
        NEGF_HIP_CHECK(run_gemm(c, s, GemmTypes{DT_C64, DT_C128, DT_C64, DT_C64}, OP_N, OP_N, EPI_ADD, G, cnt));
        // FP64 fallback for flagged points (M is still in tmp[0]).
        Active fb{c->desc_d, p0, i, PRED_SET, c->ns_flag};
        NEGF_HIP_CHECK(inverse_launch(s, DT_C128, c->tmp[0], nn, c->tmp[1], nn, n, hi, fb, invwork(c, c->tmp[3])));
        NEGF_HIP_CHECK(copy_launch(s, DT_C128, DT_C64, c->tmp[1], nn, slot(c, c->gst, i), sst, nn, hi, fb));
    }
    // X = Sigma^<_i + H_{i,i-1} g^<_{i-1} H_{i-1,i}
    sa.X = (i > 0) ? glp : nullptr; sa.sX = sp;
    sa.sign = 1.0; sa.mode = 2; sa.O = c->tmp[1];
    sa.scat = c->fwd_scL;
    sa.lesser_ref = mixed ? 1 : 0;
    sa.scat2 = c->fwd_scR;
    NEGF_HIP_CHECK(sandwich_launch(s, sdt, sdt, sa));
    // g^<_i = g_i X g_i^dagger
    GemmArgs G = gargs(n, hi, act);
    G.A = slot(c, c->gst, i); G.sA = sst; G.B = c->tmp[1]; G.sB = nn; G.C = c->tmp[2]; G.sC = nn;
    NEGF_HIP_CHECK(run_gemm(c, s, TS, OP_N, OP_N, EPI_STORE, G, cnt));
    G.A = c->tmp[2]; G.sA = nn; G.B = slot(c, c->gst, i); G.sB = sst; G.C = slot(c, c->glst, i); G.sC = sst;
    NEGF_HIP_CHECK(run_gemm(c, s, TS, OP_N, OP_C, EPI_STORE_AH, G, cnt));   // anti-Hermitian
    return NEGF_OK;
}

// Checkpoint mode: make the segment buffers hold segment `sg` of the last
// forward sweep, recomputing its slabs from the checkpoint of segment sg - 1.
static int load_segment(negf_ctx* c, hipStream_t s, int sg) {
    if (!c->ckpt || c->seg_loaded == sg) return NEGF_OK;
    const int i0 = sg * c->segK, i1 = std::min((sg + 1) * c->segK, c->fwd_maxN);
    const long long sst = store_stride(c), sck = ck_stride(c);
    for (int i = i0; i < i1; ++i) {
        const void *gp = nullptr, *glp = nullptr;
        long long sp = sst;
        if (i == i0 && sg > 0) {
            gp = ckslot(c, c->ckg, sg - 1); glp = ckslot(c, c->ckgl, sg - 1); sp = sck;
        } else if (i > i0) {
            gp = slot(c, c->gst, i - 1); glp = slot(c, c->glst, i - 1);
        }
        const int st = fwd_slab(c, s, c->fwd_p0, c->fwd_np, i, gp, glp, sp, false);
        if (st != NEGF_OK) return st;
    }
    c->seg_loaded = sg;
    return NEGF_OK;
}

extern "C" {

int negf_rgf_forward(negf_ctx* c, void* stream, int p0, int np, const negf_c128* sigma_L,
                     const negf_c128* sigma_R, const negf_c128* scat_R, const negf_c128* scat_L, int flags) {
    if (!c) return NEGF_EINVAL;
    if (!c->bound) return NEGF_ESTATE;
    if (!sigma_L || !sigma_R || p0 < 0 || np < 1 || p0 + np > c->n_points) return NEGF_EINVAL;
    if (np > c->cap) return NEGF_ESHAPE;
    if ((scat_R == nullptr) != (scat_L == nullptr)) return NEGF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int n = c->nb;
    const long long nn = (long long)n * n;
    const long long sst = store_stride(c);
    const bool mixed = c->prec == NEGF_MIXED;
    const int sdt = c->sdt;
    const GemmTypes TS{sdt, sdt, sdt, sdt};
    int maxN = 0;
    for (int q = 0; q < np; ++q) maxN = std::max(maxN, c->desc_h[p0 + q].w);
    const bool wantT = (flags & NEGF_WANT_TRANSMISSION) != 0;
    const double2* sL = reinterpret_cast<const double2*>(sigma_L);
    const double2* sR = reinterpret_cast<const double2*>(sigma_R);
    c->fwd_done = false;
    c->fwd_p0 = p0;
    c->fwd_np = np;
    c->fwd_maxN = maxN;
    c->fwd_sL = sL;
    c->fwd_sR = sR;
    c->fwd_scR = reinterpret_cast<const double2*>(scat_R);
    c->fwd_scL = reinterpret_cast<const double2*>(scat_L);
    c->seg_loaded = -1;
    if (mixed) {
        hipLaunchKernelGGL(zero_d_kernel, dim3((np + 255) / 256), dim3(256), 0, s, c->ns_res, np);
        NEGF_HIP_CHECK(hipGetLastError());
    }
    for (int i = 0; i < maxN; ++i) {
        int hi;
        long long cnt;
        extent(c, p0, np, PRED_FWD, i, &hi, &cnt);
        Active act{c->desc_d, p0, i, PRED_FWD, nullptr};
        const int st = fwd_slab(c, s, p0, np, i, i > 0 ? slot(c, c->gst, i - 1) : nullptr,
                                i > 0 ? slot(c, c->glst, i - 1) : nullptr, sst, true);
        if (st != NEGF_OK) return st;
        if (c->ckpt && i % c->segK == c->segK - 1 && i + 1 < maxN) {
            // checkpoint: the segment's last slab (the next one only overwrites its slot later)
            const int sg = i / c->segK;
            NEGF_HIP_CHECK(copy_launch(s, sdt, sdt, slot(c, c->gst, i), sst, ckslot(c, c->ckg, sg), ck_stride(c), nn,
                                       hi, act));
            NEGF_HIP_CHECK(copy_launch(s, sdt, sdt, slot(c, c->glst, i), sst, ckslot(c, c->ckgl, sg), ck_stride(c),
                                       nn, hi, act));
        }
        if (wantT) {
            // left-column chain G_{i,1} = g_i H_{i,i-1} G_{i-1,1}
            if (i == 0) {
                NEGF_HIP_CHECK(copy_launch(s, sdt, sdt, slot(c, c->gst, 0), sst, c->tmp[5], nn, nn, hi, act));
            } else {
                SandArgs sc = sand_base(c, p0, act, hi);
                sc.X = c->tmp[5]; sc.sX = nn; sc.uslab = i - 1; sc.opL = 2; sc.opR = 0;
                sc.O = c->tmp[6]; sc.sO = nn; sc.mode = 0;
                NEGF_HIP_CHECK(sandwich_launch(s, sdt, sdt, sc));
                GemmArgs Gc = gargs(n, hi, act);
                Gc.A = slot(c, c->gst, i); Gc.sA = sst; Gc.B = c->tmp[6]; Gc.sB = nn; Gc.C = c->tmp[5]; Gc.sC = nn;
                NEGF_HIP_CHECK(run_gemm(c, s, TS, OP_N, OP_N, EPI_STORE, Gc, cnt));
            }
        }
    }
    if (c->ckpt) c->seg_loaded = (maxN - 1) / c->segK;
    if (wantT) {
        // T = Tr[Gamma_R C Gamma_L C^dagger], C = G_{N,1}
        PointSet ps{c->desc_d, c->soff_d, p0};
        Active all{c->desc_d, p0, 0, PRED_ALL, nullptr};
        NEGF_HIP_CHECK(gamma_launch(s, sdt, sL, c->sys.n_e, ps, c->tmp[7], nn, n, np));
        NEGF_HIP_CHECK(gamma_launch(s, sdt, sR, c->sys.n_e, ps, c->tmp[8], nn, n, np));
        GemmArgs G = gargs(n, np, all);
        G.A = c->tmp[8]; G.sA = nn; G.B = c->tmp[5]; G.sB = nn; G.C = c->tmp[9]; G.sC = nn;
        NEGF_HIP_CHECK(run_gemm(c, s, TS, OP_N, OP_N, EPI_STORE, G, np));
        G.A = c->tmp[7]; G.B = c->tmp[5]; G.C = c->tmp[10];
        NEGF_HIP_CHECK(run_gemm(c, s, TS, OP_N, OP_C, EPI_STORE, G, np));
        NEGF_HIP_CHECK(trace_prod_launch(s, sdt, c->tmp[9], c->tmp[10], nn, n, np, c->trans_d, p0));
    }
    c->fwd_done = true;
    c->fwd_flags = flags;
    return NEGF_OK;
}

int negf_rgf_backward(negf_ctx* c, void* stream, int p0, int np, negf_c128* GR, negf_c128* GL, negf_c128* GG,
                      int full_blocks, int slab_stride, double* bond_j, double* transmission) {
    if (!c) return NEGF_EINVAL;
    if (!c->bound || !c->fwd_done || p0 != c->fwd_p0 || np != c->fwd_np) return NEGF_ESTATE;
    if (transmission && !(c->fwd_flags & NEGF_WANT_TRANSMISSION)) return NEGF_ESTATE;
    if (full_blocks < 0 || full_blocks > 2) return NEGF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int n = c->nb;
    const long long nn = (long long)n * n;
    const long long sst = store_stride(c);
    const int sdt = c->sdt;
    const GemmTypes TS{sdt, sdt, sdt, sdt};
    int maxN = 0;
    for (int q = 0; q < np; ++q) maxN = std::max(maxN, c->desc_h[p0 + q].w);
    if (slab_stride < maxN) return NEGF_EINVAL;
    double2* Gb[2] = {c->tmp[8], c->tmp[9]};
    double2* GLb[2] = {c->tmp[10], c->tmp[11]};
    PointSet ps{c->desc_d, c->soff_d, p0};
    for (int st = maxN - 1; st >= 0; --st) {
        if (c->ckpt && (st == maxN - 1 || st % c->segK == c->segK - 1)) {
            const int e = load_segment(c, s, st / c->segK);
            if (e != NEGF_OK) return e;
        }
        const int cur = st & 1, nxt = cur ^ 1;
        int hiF, hiB, hiI;
        long long cF, cB, cI;
        extent(c, p0, np, PRED_FWD, st, &hiF, &cF);
        extent(c, p0, np, PRED_BWD, st, &hiB, &cB);
        extent(c, p0, np, PRED_INIT, st, &hiI, &cI);
        Active aI{c->desc_d, p0, st, PRED_INIT, nullptr};
        Active aB{c->desc_d, p0, st, PRED_BWD, nullptr};
        Active aF{c->desc_d, p0, st, PRED_FWD, nullptr};
        if (cI > 0) {
            NEGF_HIP_CHECK(copy_launch(s, sdt, sdt, slot(c, c->gst, st), sst, Gb[cur], nn, nn, hiI, aI));
            NEGF_HIP_CHECK(copy_launch(s, sdt, sdt, slot(c, c->glst, st), sst, GLb[cur], nn, nn, hiI, aI));
        }
        if (cB > 0) {
            SandArgs sa = sand_base(c, p0, aB, hiB);
            sa.uslab = st; sa.mode = 0;
            // L = g_s H_{s,s+1}
            sa.X = slot(c, c->gst, st); sa.sX = sst; sa.opL = 0; sa.opR = 1; sa.O = c->tmp[0]; sa.sO = nn;
            NEGF_HIP_CHECK(sandwich_launch(s, sdt, sdt, sa));
            // R = H_{s+1,s} g_s
            sa.opL = 2; sa.opR = 0; sa.O = c->tmp[1];
            NEGF_HIP_CHECK(sandwich_launch(s, sdt, sdt, sa));
            // Q = H_{s+1,s} g^<_s
            sa.X = slot(c, c->glst, st); sa.O = c->tmp[3];
            NEGF_HIP_CHECK(sandwich_launch(s, sdt, sdt, sa));
            GemmArgs G = gargs(n, hiB, aB);
            // P = L G_{s+1}
            G.A = c->tmp[0]; G.sA = nn; G.B = Gb[nxt]; G.sB = nn; G.C = c->tmp[2]; G.sC = nn;
            NEGF_HIP_CHECK(run_gemm(c, s, TS, OP_N, OP_N, EPI_STORE, G, cB));
            // G_s = g_s + P R
            G.A = c->tmp[2]; G.B = c->tmp[1]; G.C = Gb[cur]; G.D = slot(c, c->gst, st); G.sD = sst;
            NEGF_HIP_CHECK(run_gemm(c, s, TS, OP_N, OP_N, EPI_ADD, G, cB));
            // T = P Q
            G.A = c->tmp[2]; G.B = c->tmp[3]; G.C = c->tmp[6];
            NEGF_HIP_CHECK(run_gemm(c, s, TS, OP_N, OP_N, EPI_STORE, G, cB));
            // W = L G^<_{s+1}
            G.A = c->tmp[0]; G.B = GLb[nxt]; G.C = c->tmp[7];
            NEGF_HIP_CHECK(run_gemm(c, s, TS, OP_N, OP_N, EPI_STORE, G, cB));
            // G^<_s = g^<_s + W L^dagger + T - T^dagger
            G.A = c->tmp[7]; G.B = c->tmp[0]; G.C = GLb[cur]; G.D = slot(c, c->glst, st); G.sD = sst;
            G.T = c->tmp[6]; G.sT = nn;
            NEGF_HIP_CHECK(run_gemm(c, s, TS, OP_N, OP_C, EPI_ADD_TTD_AH, G, cB));   // anti-Hermitian
            if (bond_j) {
                BondArgs b{};
                b.hup = reinterpret_cast<const double2*>(c->sys.h_up);
                b.hup_k = c->sys.h_up_k_stride;
                b.ub = c->sys.up_block; b.slab = st;
                b.G = Gb[nxt]; b.GL = GLb[nxt]; b.Q = c->tmp[3]; b.L = c->tmp[0]; b.sM = nn;
                b.gls = slot(c, c->glst, st); b.s_gls = sst;
                b.partial = c->bond_partial; b.n = n; b.np = hiB; b.act = aB; b.ps = ps;
                NEGF_HIP_CHECK(bond_launch(s, sdt, b, bond_j, slab_stride));
            }
        }
        if (GR || GL || GG) {
            ExtArgs e{};
            e.G = Gb[cur]; e.GL = GLb[cur]; e.sG = nn;
            e.outR = reinterpret_cast<double2*>(GR); e.outL = reinterpret_cast<double2*>(GL);
            e.outG = reinterpret_cast<double2*>(GG);
            e.full = full_blocks; e.opa = c->scat_opa; e.slab_stride = slab_stride; e.slab = st; e.n = n;
            e.np = hiF; e.p0 = p0;
            e.act = aF;
            e.lesser_ref = (c->prec == NEGF_MIXED) ? 1 : 0;
            e.energy = c->sys.energy; e.muR = c->sys.mu_R; e.kT = c->sys.kT;
            NEGF_HIP_CHECK(extract_launch(s, sdt, e));
        }
    }
    if (transmission) {
        hipLaunchKernelGGL(copy_d_kernel, dim3((np + 255) / 256), dim3(256), 0, s, c->trans_d + p0, transmission + p0, np);
        NEGF_HIP_CHECK(hipGetLastError());
    }
    return NEGF_OK;
}

int negf_rgf_solve(negf_ctx* c, void* stream, int p0, int np, const negf_c128* sigma_L, const negf_c128* sigma_R,
                   const negf_c128* scat_R, const negf_c128* scat_L, int flags, negf_c128* GR, negf_c128* GL,
                   negf_c128* GG, int full_blocks, int slab_stride, double* bond_j, double* transmission) {
    if (!c) return NEGF_EINVAL;
    if (!c->bound) return NEGF_ESTATE;
    if (!sigma_L || !sigma_R || p0 < 0 || np < 1 || p0 + np > c->n_points) return NEGF_EINVAL;
    if (np > c->cap) return NEGF_ESHAPE;
    if ((scat_R == nullptr) != (scat_L == nullptr)) return NEGF_EINVAL;
    if (transmission && !(flags & NEGF_WANT_TRANSMISSION)) return NEGF_ESTATE;
    int maxN = 0;
    for (int q = 0; q < np; ++q) maxN = std::max(maxN, c->desc_h[p0 + q].w);
    if (slab_stride < maxN) return NEGF_EINVAL;
    const bool fused = c->nb <= SMALL_NMAX && c->prec == NEGF_FP64 && !c->ckpt && c->scat_opa == 1 &&
                       full_blocks != 2;
    if (!fused) {
        const int st = negf_rgf_forward(c, stream, p0, np, sigma_L, sigma_R, scat_R, scat_L, flags);
        if (st != NEGF_OK) return st;
        return negf_rgf_backward(c, stream, p0, np, GR, GL, GG, full_blocks, slab_stride, bond_j, transmission);
    }
    hipStream_t s = (hipStream_t)stream;
    const negf_system& S = c->sys;
    SmallArgs a{};
    a.hdiag = reinterpret_cast<const double2*>(S.h_diag);
    a.hdiag_k = c->soff_h.back() * (long long)c->nb * c->nb;
    a.hup = reinterpret_cast<const double2*>(S.h_up);
    a.hup_k = S.h_up_k_stride;
    a.ub = S.up_block;
    a.v = S.v_onsite;
    a.scatR = reinterpret_cast<const double2*>(scat_R);
    a.scatL = reinterpret_cast<const double2*>(scat_L);
    a.total = c->soff_h.back();
    a.sigL = reinterpret_cast<const double2*>(sigma_L);
    a.sigR = reinterpret_cast<const double2*>(sigma_R);
    a.n_e = S.n_e;
    a.energy = S.energy; a.eta = S.eta; a.muL = S.mu_L; a.muR = S.mu_R; a.kT = S.kT; a.eta_fill = S.eta_fill;
    a.ps = PointSet{c->desc_d, c->soff_d, p0};
    a.np = np; a.n = c->nb;
    a.outR = reinterpret_cast<double2*>(GR); a.outL = reinterpret_cast<double2*>(GL);
    a.outG = reinterpret_cast<double2*>(GG);
    a.full = full_blocks ? 1 : 0; a.slab_stride = slab_stride;
    a.bond = bond_j;
    a.trans = (flags & NEGF_WANT_TRANSMISSION) ? c->trans_d : nullptr;
    a.gst = static_cast<double2*>(c->gst); a.glst = static_cast<double2*>(c->glst); a.sst = store_stride(c);
    a.queue = c->queue;
    a.status = c->status;
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, s, c->queue, 0, 1);
    NEGF_HIP_CHECK(hipGetLastError());
    // persistent: enough wavefronts to fill every CU a few times over, each
    // pulling points until the queue is drained
    NEGF_HIP_CHECK(small_launch(s, a, std::min(np, 256 * 8)));
    if (transmission) {
        hipLaunchKernelGGL(copy_d_kernel, dim3((np + 255) / 256), dim3(256), 0, s, c->trans_d + p0, transmission + p0,
                           np);
        NEGF_HIP_CHECK(hipGetLastError());
    }
    c->fwd_done = true;
    c->fwd_p0 = p0;
    c->fwd_np = np;
    c->fwd_maxN = maxN;
    c->fwd_flags = flags;
    c->fwd_sL = a.sigL; c->fwd_sR = a.sigR; c->fwd_scR = a.scatR; c->fwd_scL = a.scatL;
    c->seg_loaded = -1;
    return NEGF_OK;
}

int negf_scba_selfenergy(negf_ctx* c, void* stream, const negf_c128* GR, const negf_c128* GL, int slab_stride,
                         const double* w_k, double D_ac, double M_op, int shift, double n_bose, negf_c128* sig_R,
                         negf_c128* sig_L, double* rel_change) {
    if (!c) return NEGF_EINVAL;
    if (!c->bound || !c->is_grid) return NEGF_ESTATE;
    if (!GR || !GL || !w_k || !sig_R || !sig_L || shift < 0) return NEGF_EINVAL;
    const int N = (int)c->soff_h.back();
    if (slab_stride < N) return NEGF_EINVAL;
    ScbaArgs a{};
    a.GR = reinterpret_cast<const double2*>(GR);
    a.GL = reinterpret_cast<const double2*>(GL);
    a.w_k = w_k; a.D = D_ac; a.M = M_op; a.n0 = n_bose; a.shift = shift;
    a.n_k = c->sys.n_k; a.n_e = c->sys.n_e; a.N = N; a.n = c->nb * c->scat_opa; a.slab_stride = slab_stride;
    a.sigR = reinterpret_cast<double2*>(sig_R);
    a.sigL = reinterpret_cast<double2*>(sig_L);
    a.partial = c->scba_partial_d;
    NEGF_HIP_CHECK(scba_launch((hipStream_t)stream, a, rel_change, c->scba_hist, c->scba_count, SCBA_HMAX));
    return NEGF_OK;
}

int negf_scba_history(negf_ctx* c, void* stream, double* out, int max_n, int* n_out) {
    if (!c || !n_out || max_n < 0 || (max_n > 0 && !out)) return NEGF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    NEGF_HIP_CHECK(hipMemcpyAsync(c->h_pinned, c->scba_count, sizeof(int), hipMemcpyDeviceToHost, s));
    NEGF_HIP_CHECK(hipStreamSynchronize(s));
    const int cnt = c->h_pinned[0];
    *n_out = cnt;
    const int m = std::min(std::min(cnt, SCBA_HMAX), max_n);
    if (m > 0) NEGF_HIP_CHECK(hipMemcpy(out, c->scba_hist, m * sizeof(double), hipMemcpyDeviceToHost));
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, s, c->scba_count, 0, 1);
    NEGF_HIP_CHECK(hipGetLastError());
    return NEGF_OK;
}

int negf_observables(negf_ctx* c, void* stream, const negf_c128* GL, const double* bond_j, int slab_stride,
                     const double* w_e, const double* w_k, double g_s, int orbs_per_atom, double* n_out, double* J,
                     double* j_E, int gl_opa) {
    if (!c) return NEGF_EINVAL;
    if (!c->bound) return NEGF_ESTATE;
    if (!w_e || !w_k || orbs_per_atom < 1 || c->nb % orbs_per_atom != 0) return NEGF_EINVAL;
    if (gl_opa < 1 || c->nb % gl_opa != 0) return NEGF_EINVAL;
    if ((n_out && !GL) || ((J || j_E) && !bond_j)) return NEGF_EINVAL;
    int maxN = 0;
    for (size_t s = 0; s + 1 < c->soff_h.size(); ++s) maxN = std::max<long long>(maxN, c->soff_h[s + 1] - c->soff_h[s]);
    if (slab_stride < maxN) return NEGF_EINVAL;
    ObsArgs a{};
    a.GL = reinterpret_cast<const double2*>(GL);
    a.bond = bond_j; a.slab_stride = slab_stride; a.w_e = w_e; a.w_k = w_k; a.g_s = g_s;
    a.opa = orbs_per_atom; a.n = c->nb; a.n_e = c->sys.n_e; a.n_samples = c->sys.n_samples; a.gopa = gl_opa;
    a.total = c->soff_h.back();
    a.desc = c->desc_d; a.slab_off = c->soff_d; a.slab_sample = c->slab_sample_d;
    a.csr_off = c->csr_off_d; a.csr_pts = c->csr_pts_d; a.orb_tmp = c->orb_tmp_d;
    a.n_out = n_out; a.J = J; a.jE = j_E;
    NEGF_HIP_CHECK(observables_launch((hipStream_t)stream, a));
    return NEGF_OK;
}


int negf_rgf_adjoint(negf_ctx* c, void* stream, int p0, int np, const double* w_orb, negf_c128* dX,
                     int slab_stride) {
    if (!c) return NEGF_EINVAL;
    if (!c->bound || !c->fwd_done || p0 != c->fwd_p0 || np != c->fwd_np) return NEGF_ESTATE;
    if (c->adj_K <= 0 || c->prec != NEGF_FP64) return NEGF_ESTATE;
    if (!w_orb || !dX) return NEGF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int n = c->nb;
    const long long nn = (long long)n * n;
    const long long sst = store_stride(c);
    const GemmTypes T64{DT_C128, DT_C128, DT_C128, DT_C128};
    int maxN = 0;
    for (int q = 0; q < np; ++q) maxN = std::max(maxN, c->desc_h[p0 + q].w);
    if (slab_stride < maxN) return NEGF_EINVAL;
    const int K = c->adj_K;
    const int nseg = (maxN + K - 1) / K;
    const long long sseg = (long long)K * nn, sck = (long long)c->adj_nseg * nn;
    double2** t = c->tmp;
    double2 *tw = t[0], *tWG = t[1], *tc = t[2], *tcg = t[3];

    // One slab of the forward recursion for y_i, x_i (g_i, g^<_i from the stores).
    auto fwd_step = [&](int i, const double2* yp, const double2* xp, long long sp, double2* yo, double2* xo,
                        long long so) -> int {
        int hi;
        long long cnt;
        extent(c, p0, np, PRED_FWD, i, &hi, &cnt);
        if (cnt == 0) return NEGF_OK;
        Active act{c->desc_d, p0, i, PRED_FWD, nullptr};
        SandArgs sa = sand_base(c, p0, act, hi);
        sa.mode = 3; sa.wdiag = w_orb; sa.slab = i;
        sa.X = (i > 0) ? yp : nullptr; sa.sX = sp; sa.uslab = i - 1; sa.opL = 2; sa.opR = 1;
        sa.O = tw; sa.sO = nn;
        NEGF_HIP_CHECK(sandwich_launch(s, DT_C128, DT_C128, sa));          // w_i = W_i + H y H
        GemmArgs G = gargs(n, hi, act);
        G.A = tw; G.sA = nn; G.B = slot(c, c->gst, i); G.sB = sst; G.C = tWG; G.sC = nn;
        NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_N, OP_N, EPI_STORE, G, cnt));   // w_i g_i
        G.A = slot(c, c->gst, i); G.sA = sst; G.B = tWG; G.sB = nn; G.C = yo; G.sC = so;
        NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_C, OP_N, EPI_STORE, G, cnt));   // y_i = g^dag w g
        G.A = slot(c, c->glst, i); G.C = xo;
        NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_N, OP_N, EPI_STORE, G, cnt));   // x_i = g^< w g
        if (i > 0) {
            SandArgs sc = sand_base(c, p0, act, hi);
            sc.mode = 0; sc.X = xp; sc.sX = sp; sc.uslab = i - 1; sc.opL = 2; sc.opR = 1;
            sc.O = tc; sc.sO = nn;
            NEGF_HIP_CHECK(sandwich_launch(s, DT_C128, DT_C128, sc));      // c_i = H x H
            GemmArgs H = gargs(n, hi, act);
            H.A = tc; H.sA = nn; H.B = slot(c, c->gst, i); H.sB = sst; H.C = tcg; H.sC = nn;
            NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_N, OP_N, EPI_STORE, H, cnt));
            H.A = slot(c, c->gst, i); H.sA = sst; H.B = tcg; H.sB = nn; H.C = xo; H.sC = so; H.D = xo; H.sD = so;
            NEGF_HIP_CHECK(run_gemm(c, s, T64, OP_N, OP_N, EPI_ADD, H, cnt));  // x_i += g c g
        }
        return NEGF_OK;
    };

    // Pass 1: forward over all slabs, keeping (y, x) at the end of every segment.
    double2* yp[2] = {t[4], t[5]};
    double2* xp[2] = {t[6], t[7]};
    for (int i = 0; i < maxN; ++i) {
        if (c->ckpt && i % c->segK == 0) {
            const int e = load_segment(c, s, i / c->segK);
            if (e != NEGF_OK) return e;
        }
        int st = fwd_step(i, yp[(i + 1) & 1], xp[(i + 1) & 1], nn, yp[i & 1], xp[i & 1], nn);
        if (st != NEGF_OK) return st;
        if ((i + 1) % K == 0 && i + 1 < maxN) {
            int hi;
            long long cnt;
            extent(c, p0, np, PRED_FWD, i, &hi, &cnt);
            Active act{c->desc_d, p0, i, PRED_FWD, nullptr};
            const int sg = (i + 1) / K - 1;
            NEGF_HIP_CHECK(copy_launch(s, DT_C128, DT_C128, yp[i & 1], nn, c->adj_yck + sg * nn, sck, nn, hi, act));
            NEGF_HIP_CHECK(copy_launch(s, DT_C128, DT_C128, xp[i & 1], nn, c->adj_xck + sg * nn, sck, nn, hi, act));
        }
    }

    // Pass 2: per segment (last first), recompute (y, x) and sweep backward.
    double2* Gb[2] = {t[8], t[9]};
    double2* GLb[2] = {t[10], t[11]};
    double2* Yb[2] = {t[12], t[13]};
    double2* Xb[2] = {t[14], t[15]};
    double2 *tL = t[16], *tR = t[17], *tQ = t[18], *tP = t[19], *tT = t[20], *tW = t[21], *tGR = t[22],
            *tK1 = t[23], *tK2 = t[0], *tLg = t[1], *tRy = t[2], *tLy = t[3], *tRx = t[4], *tLx = t[5];
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int lst = load_segment(c, s, sg);
        if (lst != NEGF_OK) return lst;
        const int i0 = sg * K, i1 = std::min((sg + 1) * K, maxN);
        for (int i = i0; i < i1; ++i) {
            const double2 *ypv, *xpv;
            long long spv;
            if (i == i0) {
                ypv = sg > 0 ? c->adj_yck + (sg - 1) * nn : nullptr;
                xpv = sg > 0 ? c->adj_xck + (sg - 1) * nn : nullptr;
                spv = sck;
            } else {
                ypv = c->adj_yseg + (i - 1 - i0) * nn;
                xpv = c->adj_xseg + (i - 1 - i0) * nn;
                spv = sseg;
            }
            int st = fwd_step(i, ypv, xpv, spv, c->adj_yseg + (i - i0) * nn, c->adj_xseg + (i - i0) * nn, sseg);
            if (st != NEGF_OK) return st;
        }
        for (int st = i1 - 1; st >= i0; --st) {
            const int cur = st & 1, nxt = cur ^ 1;
            double2* ys = c->adj_yseg + (st - i0) * nn;
            double2* xs = c->adj_xseg + (st - i0) * nn;
            int hiF, hiB, hiI;
            long long cF, cB, cI;
            extent(c, p0, np, PRED_FWD, st, &hiF, &cF);
            extent(c, p0, np, PRED_BWD, st, &hiB, &cB);
            extent(c, p0, np, PRED_INIT, st, &hiI, &cI);
            Active aI{c->desc_d, p0, st, PRED_INIT, nullptr};
            Active aB{c->desc_d, p0, st, PRED_BWD, nullptr};
            Active aF{c->desc_d, p0, st, PRED_FWD, nullptr};
            if (cI > 0) {
                NEGF_HIP_CHECK(copy_launch(s, DT_C128, DT_C128, slot(c, c->gst, st), sst, Gb[cur], nn, nn, hiI, aI));
                NEGF_HIP_CHECK(copy_launch(s, DT_C128, DT_C128, slot(c, c->glst, st), sst, GLb[cur], nn, nn, hiI, aI));
                NEGF_HIP_CHECK(copy_launch(s, DT_C128, DT_C128, ys, sseg, Yb[cur], nn, nn, hiI, aI));
                NEGF_HIP_CHECK(copy_launch(s, DT_C128, DT_C128, xs, sseg, Xb[cur], nn, nn, hiI, aI));
            }
            if (cB > 0) {
                SandArgs sa = sand_base(c, p0, aB, hiB);
                sa.uslab = st; sa.mode = 0; sa.sO = nn;
                struct { const void* X; long long sX; int opL, opR; double2* O; } sw[8] = {
                    {slot(c, c->gst, st), sst, 0, 1, tL},  {slot(c, c->gst, st), sst, 2, 0, tR},
                    {slot(c, c->glst, st), sst, 2, 0, tQ}, {slot(c, c->glst, st), sst, 0, 1, tLg},
                    {ys, sseg, 2, 0, tRy},                  {ys, sseg, 0, 1, tLy},
                    {xs, sseg, 2, 0, tRx},                  {xs, sseg, 0, 1, tLx}};
                for (auto& w : sw) {
                    sa.X = w.X; sa.sX = w.sX; sa.opL = w.opL; sa.opR = w.opR; sa.O = w.O;
                    NEGF_HIP_CHECK(sandwich_launch(s, DT_C128, DT_C128, sa));
                }
                auto mm = [&](int opa, int opb, int epi, const void* A, long long sA, const void* B, long long sB,
                              void* C, long long sC, const void* D = nullptr, long long sD = 0,
                              const void* T = nullptr) -> hipError_t {
                    GemmArgs G = gargs(n, hiB, aB);
                    G.A = A; G.sA = sA; G.B = B; G.sB = sB; G.C = C; G.sC = sC; G.D = D; G.sD = sD;
                    G.T = T; G.sT = nn;
                    return run_gemm(c, s, T64, opa, opb, epi, G, cB);
                };
                // retarded and lesser levels (as in negf_rgf_backward)
                NEGF_HIP_CHECK(mm(OP_N, OP_N, EPI_STORE, tL, nn, Gb[nxt], nn, tP, nn));
                NEGF_HIP_CHECK(mm(OP_N, OP_N, EPI_ADD, tP, nn, tR, nn, Gb[cur], nn, slot(c, c->gst, st), sst));
                NEGF_HIP_CHECK(mm(OP_N, OP_N, EPI_STORE, tP, nn, tQ, nn, tT, nn));
                NEGF_HIP_CHECK(mm(OP_N, OP_N, EPI_STORE, tL, nn, GLb[nxt], nn, tW, nn));
                NEGF_HIP_CHECK(mm(OP_N, OP_C, EPI_ADD_TTD_AH, tW, nn, tL, nn, GLb[cur], nn, slot(c, c->glst, st), sst, tT));
                // (2,3) level: Y_i = y + R^dag (G^dag R_y + Y R) + L_y G R
                NEGF_HIP_CHECK(mm(OP_N, OP_N, EPI_STORE, Gb[nxt], nn, tR, nn, tGR, nn));
                NEGF_HIP_CHECK(mm(OP_C, OP_N, EPI_STORE, Gb[nxt], nn, tRy, nn, tK1, nn));
                NEGF_HIP_CHECK(mm(OP_N, OP_N, EPI_ADD, Yb[nxt], nn, tR, nn, tK1, nn, tK1, nn));
                NEGF_HIP_CHECK(mm(OP_C, OP_N, EPI_ADD, tR, nn, tK1, nn, Yb[cur], nn, ys, sseg));
                NEGF_HIP_CHECK(mm(OP_N, OP_N, EPI_ADD, tLy, nn, tGR, nn, Yb[cur], nn, Yb[cur], nn));
                // (1,3) level: X_i = x + L (G R_x + G^< R_y + X R) + L_g K1 + L_x G R
                NEGF_HIP_CHECK(mm(OP_N, OP_N, EPI_STORE, Gb[nxt], nn, tRx, nn, tK2, nn));
                NEGF_HIP_CHECK(mm(OP_N, OP_N, EPI_ADD, GLb[nxt], nn, tRy, nn, tK2, nn, tK2, nn));
                NEGF_HIP_CHECK(mm(OP_N, OP_N, EPI_ADD, Xb[nxt], nn, tR, nn, tK2, nn, tK2, nn));
                NEGF_HIP_CHECK(mm(OP_N, OP_N, EPI_ADD, tL, nn, tK2, nn, Xb[cur], nn, xs, sseg));
                NEGF_HIP_CHECK(mm(OP_N, OP_N, EPI_ADD, tLg, nn, tK1, nn, Xb[cur], nn, Xb[cur], nn));
                NEGF_HIP_CHECK(mm(OP_N, OP_N, EPI_ADD, tLx, nn, tGR, nn, Xb[cur], nn, Xb[cur], nn));
            }
            NEGF_HIP_CHECK(diag_out_launch(s, Xb[cur], nn, n, hiF, aF, 2.0, reinterpret_cast<double2*>(dX),
                                           slab_stride, st, p0));
        }
    }
    return NEGF_OK;
}

int negf_zgemm_batched(negf_ctx* c, void* stream, int n, int batch, int opa, int opb, const void* A, const void* B,
                       void* C, int dtype) {
    if (!c || !A || !B || !C || n < 1 || batch < 1) return NEGF_EINVAL;
    if ((opa != 0 && opa != 1) || (opb != 0 && opb != 1) || (dtype != 0 && dtype != 1)) return NEGF_EINVAL;
    const int dt = dtype == 0 ? DT_C128 : DT_C64;
    const long long nn = (long long)n * n;
    Active all{nullptr, 0, 0, PRED_ALL, nullptr};
    GemmArgs G = gargs(n, batch, all);
    G.A = A; G.sA = nn; G.B = B; G.sB = nn; G.C = C; G.sC = nn;
    NEGF_HIP_CHECK(run_gemm(c, (hipStream_t)stream, GemmTypes{dt, dt, dt, dt}, opa, opb, EPI_STORE, G, batch));
    return NEGF_OK;
}

int negf_zinv_batched(negf_ctx* c, void* stream, int n, int batch, void* A, void* Ainv, int dtype) {
    if (!c || !A || !Ainv || n < 1 || batch < 1 || (dtype != 0 && dtype != 1)) return NEGF_EINVAL;
    if (n > c->nb || batch > c->cap) return NEGF_ESHAPE;
    const long long nn = (long long)n * n;
    Active all{nullptr, 0, 0, PRED_ALL, nullptr};
    NEGF_HIP_CHECK(inverse_launch((hipStream_t)stream, dtype == 0 ? DT_C128 : DT_C64, A, nn, Ainv, nn, n, batch, all,
                                  invwork(c, c->tmp[14])));
    return NEGF_OK;
}

int negf_mixed_stats(negf_ctx* c, void* stream, long long* n_fallback, double* max_residual) {
    if (!c) return NEGF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> mx(c->cap);
    NEGF_HIP_CHECK(hipMemcpyAsync(c->h_pinned, c->ns_count, sizeof(int), hipMemcpyDeviceToHost, s));
    NEGF_HIP_CHECK(hipStreamSynchronize(s));
    NEGF_HIP_CHECK(hipMemcpy(mx.data(), c->ns_max, c->cap * sizeof(double), hipMemcpyDeviceToHost));
    if (n_fallback) *n_fallback = c->h_pinned[0];
    if (max_residual) *max_residual = mx.empty() ? 0.0 : *std::max_element(mx.begin(), mx.end());
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(64), 0, s, c->ns_count, 0, 1);
    hipLaunchKernelGGL(zero_d_kernel, dim3((c->cap + 255) / 256), dim3(256), 0, s, c->ns_max, c->cap);
    NEGF_HIP_CHECK(hipGetLastError());
    return NEGF_OK;
}

int negf_mixed_point_residuals(negf_ctx* c, void* stream, int n, double* out) {
    if (!c || !out || n < 1) return NEGF_EINVAL;
    if (c->prec != NEGF_MIXED || !c->fwd_done) return NEGF_ESTATE;
    if (n > c->fwd_np) return NEGF_ESHAPE;
    hipLaunchKernelGGL(copy_d_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, c->ns_res, out, n);
    NEGF_HIP_CHECK(hipGetLastError());
    return NEGF_OK;
}

int negf_mixed_point_scores(negf_ctx* c, void* stream, const negf_c128* GL, int slab_stride, const double* w_e,
                            const double* w_k, const double* resid, double* score) {
    if (!c || !GL || !w_e || !w_k || !resid || !score) return NEGF_EINVAL;
    if (!c->bound) return NEGF_ESTATE;
    int maxN = 0;
    for (size_t s = 0; s + 1 < c->soff_h.size(); ++s) maxN = std::max<long long>(maxN, c->soff_h[s + 1] - c->soff_h[s]);
    if (slab_stride < maxN) return NEGF_EINVAL;
    hipLaunchKernelGGL(mixed_score_kernel, dim3(c->n_points), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const double2*>(GL), slab_stride, c->nb, c->desc_d, w_e, w_k, resid, score);
    NEGF_HIP_CHECK(hipGetLastError());
    return NEGF_OK;
}

int negf_transpose_batched(void* stream, int n, int count, const negf_c128* src, long long src_stride,
                           negf_c128* dst, long long dst_stride) {
    if (n < 1 || count < 1 || count > 65535 || !src || !dst) return NEGF_EINVAL;
    const long long nn = (long long)n * n;
    if (src_stride < nn || dst_stride < nn) return NEGF_EINVAL;
    const char *s0 = reinterpret_cast<const char*>(src), *d0 = reinterpret_cast<const char*>(dst);
    const long long sb = ((count - 1) * src_stride + nn) * 16, db = ((count - 1) * dst_stride + nn) * 16;
    if (s0 < d0 + db && d0 < s0 + sb) return NEGF_EINVAL;       // overlapping buffers
    const int tiles = (n + 31) / 32;
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)(tiles * tiles), (unsigned)count), dim3(256), 0,
                       (hipStream_t)stream, reinterpret_cast<const double2*>(src), src_stride,
                       reinterpret_cast<double2*>(dst), dst_stride, n);
    NEGF_HIP_CHECK(hipGetLastError());
    return NEGF_OK;
}

int negf_cap_selfenergy(negf_ctx* c, void* stream, const double* w_slab, const int* side, negf_c128* scat_R,
                        negf_c128* scat_L) {
    if (!c || !w_slab || !side || !scat_R || !scat_L) return NEGF_EINVAL;
    if (!c->bound) return NEGF_ESTATE;
    const long long total = c->soff_h.back();
    const long long m = (long long)c->sys.n_e * total * c->nb;
    hipLaunchKernelGGL(cap_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       c->sys.energy, c->sys.n_e, total, c->nb, w_slab, side, c->sys.mu_L, c->sys.mu_R, c->sys.kT,
                       reinterpret_cast<double2*>(scat_R), reinterpret_cast<double2*>(scat_L));
    NEGF_HIP_CHECK(hipGetLastError());
    return NEGF_OK;
}

int negf_density_jacobian_local(negf_ctx* c, void* stream, const negf_c128* GR, const negf_c128* GL,
                                int slab_stride, const double* w_e, const double* w_k, double g_s,
                                int orbs_per_atom, double* d_out) {
    if (!c) return NEGF_EINVAL;
    if (!c->bound) return NEGF_ESTATE;
    if (!GR || !GL || !w_e || !w_k || !d_out || orbs_per_atom < 1 || c->nb % orbs_per_atom != 0)
        return NEGF_EINVAL;
    int maxN = 0;
    for (size_t s = 0; s + 1 < c->soff_h.size(); ++s) maxN = std::max<long long>(maxN, c->soff_h[s + 1] - c->soff_h[s]);
    if (slab_stride < maxN) return NEGF_EINVAL;
    ObsArgs a{};
    a.GL = reinterpret_cast<const double2*>(GL);
    a.GR = reinterpret_cast<const double2*>(GR);
    a.slab_stride = slab_stride; a.w_e = w_e; a.w_k = w_k; a.g_s = g_s;
    a.opa = orbs_per_atom; a.n = c->nb; a.n_e = c->sys.n_e; a.n_samples = c->sys.n_samples; a.gopa = 1;
    a.total = c->soff_h.back();
    a.desc = c->desc_d; a.slab_off = c->soff_d; a.slab_sample = c->slab_sample_d;
    a.csr_off = c->csr_off_d; a.csr_pts = c->csr_pts_d; a.orb_tmp = c->orb_tmp_d;
    a.n_out = d_out;
    NEGF_HIP_CHECK(observables_launch((hipStream_t)stream, a));
    return NEGF_OK;
}

int negf_set_scattering_blocks(negf_ctx* c, int opa) {
    if (!c || opa < 1 || opa > 64 || c->nb % opa != 0) return NEGF_EINVAL;
    if (opa == c->scat_opa) return NEGF_OK;
    if (c->bound && c->is_grid) {      // the SCBA reduction's partials grow with the entries per slab
        const long long nblk = ((long long)c->sys.n_e * c->soff_h.back() * c->nb * opa + 255) / 256;
        double* p = nullptr;
        if (!dev_alloc(c, &p, nblk * 2 * sizeof(double), c->bound_allocs)) return NEGF_ENOMEM;
        c->scba_partial_d = p;
    }
    c->scat_opa = opa;
    return NEGF_OK;
}

int negf_set_mixed_threshold(negf_ctx* c, double thr) {
    if (!c || !(thr >= 0.0)) return NEGF_EINVAL;
    c->ns_thr = thr;
    return NEGF_OK;
}

int negf_gemm_timing_enable(negf_ctx* c, int enable) {
    if (!c || enable < 0 || enable > 3) return NEGF_EINVAL;
    c->timing = enable != 0;
    c->timing_acc = enable == 2 ? DT_C128 : (enable == 3 ? DT_C64 : -1);
    if (c->timing) { c->t_launches = 0; c->t_ms = 0; c->t_flops = 0; c->t_mfma = 0; }
    return NEGF_OK;
}

int negf_get_tuning(const negf_ctx* c, negf_tuning* out) {
    if (!c || !out) return NEGF_EINVAL;
    *out = c->tune;
    return NEGF_OK;
}

int negf_set_tuning(negf_ctx* c, const negf_tuning* t) {
    if (!c || !t) return NEGF_EINVAL;
    if (t->gemm_prefetch < 1 || t->gemm_prefetch > 3) return NEGF_EINVAL;
    if (t->inv_outer != 0 && (t->inv_outer < 64 || t->inv_outer > INV_WMAX || t->inv_outer % 32 != 0)) return NEGF_EINVAL;
    if (t->inv_mid != 0 && (t->inv_mid < 32 || t->inv_mid > INV_WMAX || t->inv_mid % 32 != 0)) return NEGF_EINVAL;
    c->tune = *t;
    return NEGF_OK;
}

int negf_autotune(negf_ctx* c, void* stream, int reps, negf_tuning* out) {
    if (!c) return NEGF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    reps = std::max(1, std::min(reps, 100));
    const int n = c->nb, np = c->cap, dt = c->sdt;
    const long long nn = (long long)n * n, total = nn * np;
    const bool was_timing = c->timing;
    c->timing = false;
    hipEvent_t e0, e1;
    NEGF_HIP_CHECK(hipEventCreate(&e0));
    NEGF_HIP_CHECK(hipEventCreate(&e1));
    auto fill = [&](void* M, double diag) {
        const unsigned blocks = (unsigned)((total + 255) / 256);
        if (dt == DT_C128)
            hipLaunchKernelGGL(tune_fill_kernel<double2>, dim3(blocks), dim3(256), 0, s, (double2*)M, nn, n, total, diag);
        else
            hipLaunchKernelGGL(tune_fill_kernel<float2>, dim3(blocks), dim3(256), 0, s, (float2*)M, nn, n, total, diag);
        return hipGetLastError();
    };
    auto elapsed = [&](float* ms) {
        hipError_t e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
        return e;
    };
    negf_tuning best = c->tune;
    hipError_t err = hipSuccess;
    Active all{nullptr, 0, 0, PRED_ALL, nullptr};
    // batched GEMM: K slices in flight
    if ((err = fill(c->tmp[0], 0.0)) == hipSuccess) err = fill(c->tmp[1], 0.0);
    float best_ms = 0.0f;
    for (int pf = 1; pf <= 3 && err == hipSuccess; ++pf) {
        GemmArgs G = gargs(n, np, all);
        G.A = c->tmp[0]; G.sA = nn; G.B = c->tmp[1]; G.sB = nn; G.C = c->tmp[2]; G.sC = nn; G.pf = pf;
        const GemmTypes ty{dt, dt, dt, dt};
        err = gemm_launch(s, ty, OP_N, OP_N, EPI_STORE, G);
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        for (int r = 0; r < reps && err == hipSuccess; ++r) err = gemm_launch(s, ty, OP_N, OP_N, EPI_STORE, G);
        float ms = 0.0f;
        if (err == hipSuccess) err = elapsed(&ms);
        if (err == hipSuccess && (pf == 1 || ms < best_ms)) { best_ms = ms; best.gemm_prefetch = pf; }
    }
    // block inverse: outer panel width (0: one level) and mid block width (0: two levels)
    const int cands[][2] = {{0, 0}, {64, 0}, {96, 0}, {128, 0}, {160, 0}, {192, 0}, {256, 0},
                            {128, 64}, {192, 64}, {256, 64}, {256, 128}};
    best_ms = 0.0f;
    bool first = true;
    for (const auto& cw : cands) {
        const int W = cw[0], Wm = cw[1];
        if (err != hipSuccess) break;
        if (W != 0 && (!c->invN0 || W >= n)) continue;
        InvWork w = invwork(c, c->tmp[5]);
        w.W = W;
        w.Wm = Wm;
        float ms = 0.0f;
        for (int r = 0; r <= reps && err == hipSuccess; ++r) {   // r == 0 warms up
            err = fill(c->tmp[3], (double)n);
            if (err == hipSuccess) err = hipEventRecord(e0, s);
            if (err == hipSuccess) err = inverse_launch(s, dt, c->tmp[3], nn, c->tmp[4], nn, n, np, all, w);
            float one = 0.0f;
            if (err == hipSuccess) err = elapsed(&one);
            if (r > 0) ms += one;
        }
        if (err == hipSuccess && (first || ms < best_ms)) {
            best_ms = ms; best.inv_outer = W; best.inv_mid = Wm; first = false;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->timing = was_timing;
    if (err != hipSuccess) return NEGF_EHIP;
    c->tune = best;
    if (out) *out = best;
    return NEGF_OK;
}

int negf_gemm_timing(negf_ctx* c, void* stream, long long* launches, double* ms, double* flops,
                     double* mfma_flops) {
    if (!c) return NEGF_EINVAL;
    NEGF_HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
    NEGF_HIP_CHECK(drain_timing(c));
    if (launches) *launches = c->t_launches;
    if (ms) *ms = c->t_ms;
    if (flops) *flops = c->t_flops;
    if (mfma_flops) *mfma_flops = c->t_mfma;
    return NEGF_OK;
}

}  // extern "C"
