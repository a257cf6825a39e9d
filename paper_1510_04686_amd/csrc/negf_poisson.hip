// The NEGF-Poisson loop (Eq. 9) on the atom grid: the finite-difference
// operator, the loop's residual, a conjugate-gradient solve of the operator and
// the vector kernels of the Krylov solver that runs each Newton step.
//
// Grid: atom (x, z, y) at index (x * n_z + z) * n_y + y -- x the slab, z across
// the body, y periodic (the direction the transverse momentum runs over).  With
// V the electron's potential energy per atom (eV):
//   (L V)_a = sum over the six neighbours b of (V_a - V_b),
// where a neighbour beyond x = 0 or x = n_x - 1 is the contact (v_left,
// v_right), one beyond a z face is the gate (v_gate) or, for insulating faces,
// absent, and y wraps round.  L0 is L with every boundary value zero; it is
// symmetric positive definite because every atom reaches a contact.
//
// Every kernel here streams a few vectors of n_atoms doubles once (HBM-bound,
// a few MB at the paper's 24,000 atoms); the Newton step's cost is the density
// and its adjoint, not these.
#include "negf_internal.hpp"
#include "negf.h"

#include <cmath>
#include <vector>

using namespace negf;

namespace {

constexpr int PB = 256;                 // threads per workgroup of every kernel here
constexpr int RED_MAX = 4096;           // partial sums per reduction (grid-stride beyond)

struct Grid {
    int nx, nz, ny, gate;
    double vl, vr, vg;
};

__device__ inline double stencil(const Grid& g, const double* __restrict__ V, long long a, bool bc) {
    const int y = (int)(a % g.ny);
    const long long t = a / g.ny;
    const int z = (int)(t % g.nz);
    const int x = (int)(t / g.nz);
    const double v = V[a];
    double s = 0.0;
    // x neighbours (contacts beyond the ends)
    s += v - (x + 1 < g.nx ? V[a + (long long)g.nz * g.ny] : (bc ? g.vr : 0.0));
    s += v - (x > 0 ? V[a - (long long)g.nz * g.ny] : (bc ? g.vl : 0.0));
    // z neighbours (gates or nothing beyond the faces)
    if (z + 1 < g.nz) s += v - V[a + g.ny];
    else if (g.gate) s += v - (bc ? g.vg : 0.0);
    if (z > 0) s += v - V[a - g.ny];
    else if (g.gate) s += v - (bc ? g.vg : 0.0);
    // y neighbours (periodic; one atom per row has no distinct neighbour)
    if (g.ny > 1) {
        const long long row = a - y;
        s += v - V[row + (y + 1 == g.ny ? 0 : y + 1)];
        s += v - V[row + (y == 0 ? g.ny - 1 : y - 1)];
    }
    return s;
}

__global__ __launch_bounds__(PB) void apply_kernel(Grid g, const double* V, int bc, double* out, long long n) {
    const long long a = (long long)blockIdx.x * PB + threadIdx.x;
    if (a < n) out[a] = stencil(g, V, a, bc != 0);
}

// F = L V - beta (n - n_d)
__global__ __launch_bounds__(PB) void residual_kernel(Grid g, const double* V, const double* dens,
                                                      const double* nd, double beta, double* F, long long n) {
    const long long a = (long long)blockIdx.x * PB + threadIdx.x;
    if (a < n) F[a] = stencil(g, V, a, true) - beta * (dens[a] - nd[a]);
}

__device__ inline double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = PB / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    return red[0];
}

// Ap = (L0 + diag(shift)) p and the workgroup's partial of p . Ap
__global__ __launch_bounds__(PB) void cg_apply_kernel(Grid g, const double* p, const double* shift, double* Ap,
                                                      double* part, long long n) {
    __shared__ double red[PB];
    double acc = 0.0;
    for (long long a = (long long)blockIdx.x * PB + threadIdx.x; a < n; a += (long long)gridDim.x * PB) {
        double q = stencil(g, p, a, false);
        if (shift) q = fma(fmax(shift[a], 0.0), p[a], q);     // negative entries count as zero
        Ap[a] = q;
        acc = fma(p[a], q, acc);
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// sc[0] = r.r (current), sc[1] = p.Ap, sc[2] = alpha.  One workgroup.
__global__ __launch_bounds__(PB) void cg_alpha_kernel(const double* part, int np_, double* sc) {
    __shared__ double red[PB];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np_; i += PB) acc += part[i];
    const double pap = block_sum(acc, red);
    if (threadIdx.x == 0) {
        sc[1] = pap;
        sc[2] = (pap > 0.0) ? sc[0] / pap : 0.0;
    }
}

// x += alpha p, r -= alpha Ap, partial of r.r
__global__ __launch_bounds__(PB) void cg_update_kernel(double* x, double* r, const double* p, const double* Ap,
                                                       const double* sc, double* part, long long n) {
    __shared__ double red[PB];
    const double al = sc[2];
    double acc = 0.0;
    for (long long a = (long long)blockIdx.x * PB + threadIdx.x; a < n; a += (long long)gridDim.x * PB) {
        x[a] = fma(al, p[a], x[a]);
        const double ra = fma(-al, Ap[a], r[a]);
        r[a] = ra;
        acc = fma(ra, ra, acc);
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// sc[3] = new r.r, sc[4] = beta = new / old, sc[0] = new.  One workgroup.
__global__ __launch_bounds__(PB) void cg_beta_kernel(const double* part, int np_, double* sc) {
    __shared__ double red[PB];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np_; i += PB) acc += part[i];
    const double rr = block_sum(acc, red);
    if (threadIdx.x == 0) {
        sc[3] = rr;
        sc[4] = (sc[0] > 0.0) ? rr / sc[0] : 0.0;
        sc[0] = rr;
    }
}

__global__ __launch_bounds__(PB) void cg_dir_kernel(double* p, const double* r, const double* sc, long long n) {
    const double be = sc[4];
    for (long long a = (long long)blockIdx.x * PB + threadIdx.x; a < n; a += (long long)gridDim.x * PB)
        p[a] = fma(be, p[a], r[a]);
}

// CG start: r = rhs (x = 0), p = r, partial of r.r
__global__ __launch_bounds__(PB) void cg_init_kernel(const double* rhs, double* x, double* r, double* p,
                                                     double* part, long long n) {
    __shared__ double red[PB];
    double acc = 0.0;
    for (long long a = (long long)blockIdx.x * PB + threadIdx.x; a < n; a += (long long)gridDim.x * PB) {
        const double v = rhs[a];
        x[a] = 0.0;
        r[a] = v;
        p[a] = v;
        acc = fma(v, v, acc);
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(PB) void cg_first_kernel(const double* part, int np_, double* sc) {
    __shared__ double red[PB];
    double acc = 0.0;
    for (int i = threadIdx.x; i < np_; i += PB) acc += part[i];
    const double rr = block_sum(acc, red);
    if (threadIdx.x == 0) { sc[0] = rr; sc[3] = rr; sc[5] = rr; }
}

// out[j] partials: part[j * nblk + blk] = sum over the workgroup's chunk of X[j, i] y[i]
__global__ __launch_bounds__(PB) void dots_kernel(const double* X, long long ld, const double* y, long long n,
                                                  double* part) {
    __shared__ double red[PB];
    const int j = blockIdx.y;
    const double* xr = X + (long long)j * ld;
    double acc = 0.0;
    for (long long a = (long long)blockIdx.x * PB + threadIdx.x; a < n; a += (long long)gridDim.x * PB)
        acc = fma(xr[a], y[a], acc);
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[(long long)j * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(PB) void dots_final_kernel(const double* part, int nblk, double* out) {
    __shared__ double red[PB];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nblk; i += PB) acc += part[(long long)j * nblk + i];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[j] = s;
}

// partials of (x . x, max |x|); NaN propagates into the maximum
__global__ __launch_bounds__(PB) void norms_kernel(const double* x, long long n, double* part) {
    __shared__ double red[PB];
    __shared__ double mx[PB];
    double acc = 0.0, m = 0.0;
    for (long long a = (long long)blockIdx.x * PB + threadIdx.x; a < n; a += (long long)gridDim.x * PB) {
        const double v = x[a];
        acc = fma(v, v, acc);
        const double u = fabs(v);
        m = (u <= m) ? m : u;
    }
    mx[threadIdx.x] = m;
    const double s = block_sum(acc, red);      // its barriers also order mx
    for (int o = PB / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double u = mx[threadIdx.x + o];
            if (!(u <= mx[threadIdx.x])) mx[threadIdx.x] = u;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s;
        part[2 * blockIdx.x + 1] = mx[0];
    }
}

__global__ __launch_bounds__(PB) void norms_final_kernel(const double* part, int nblk, double* out) {
    __shared__ double red[PB];
    __shared__ double mx[PB];
    double acc = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < nblk; i += PB) {
        acc += part[2 * i];
        const double u = part[2 * i + 1];
        m = (u <= m) ? m : u;
    }
    mx[threadIdx.x] = m;
    const double s = block_sum(acc, red);
    for (int o = PB / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double u = mx[threadIdx.x + o];
            if (!(u <= mx[threadIdx.x])) mx[threadIdx.x] = u;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s;
        out[1] = mx[0];
    }
}

// y = b y + sum_j c[j] X[j, :]
__global__ __launch_bounds__(PB) void combine_kernel(const double* X, long long ld, int m, const double* c,
                                                     double b, double* y, long long n) {
    const long long a = (long long)blockIdx.x * PB + threadIdx.x;
    if (a >= n) return;
    double v = (b == 0.0) ? 0.0 : b * y[a];
    for (int j = 0; j < m; ++j) v = fma(c[j], X[(long long)j * ld + a], v);
    y[a] = v;
}

bool grid_ok(const negf_poisson_grid* g) {
    return g && g->n_x >= 1 && g->n_z >= 1 && g->n_y >= 1 && (long long)g->n_x * g->n_z * g->n_y <= (1ll << 31) &&
           std::isfinite(g->v_left) && std::isfinite(g->v_right) && std::isfinite(g->v_gate);
}

Grid to_grid(const negf_poisson_grid* g) {
    return Grid{g->n_x, g->n_z, g->n_y, g->z_gate ? 1 : 0, g->v_left, g->v_right, g->v_gate};
}

long long atoms(const negf_poisson_grid* g) { return (long long)g->n_x * g->n_z * g->n_y; }

int red_blocks(long long n) { return (int)std::min<long long>(RED_MAX, (n + PB - 1) / PB); }

}  // namespace

extern "C" {

int negf_poisson_apply(void* stream, const negf_poisson_grid* g, const double* V, int with_boundary, double* out) {
    if (!grid_ok(g) || !V || !out) return NEGF_EINVAL;
    const long long n = atoms(g);
    hipLaunchKernelGGL(apply_kernel, dim3((unsigned)((n + PB - 1) / PB)), dim3(PB), 0, (hipStream_t)stream,
                       to_grid(g), V, with_boundary, out, n);
    NEGF_HIP_CHECK(hipGetLastError());
    return NEGF_OK;
}

int negf_poisson_residual(void* stream, const negf_poisson_grid* g, const double* V, const double* n_atom,
                          const double* n_d, double beta, double* F) {
    if (!grid_ok(g) || !V || !n_atom || !n_d || !F || !std::isfinite(beta)) return NEGF_EINVAL;
    const long long n = atoms(g);
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)((n + PB - 1) / PB)), dim3(PB), 0, (hipStream_t)stream,
                       to_grid(g), V, n_atom, n_d, beta, F, n);
    NEGF_HIP_CHECK(hipGetLastError());
    return NEGF_OK;
}

long long negf_poisson_work_bytes(const negf_poisson_grid* g) {
    if (!grid_ok(g)) return -1;
    const long long n = atoms(g);
    return (3 * n + RED_MAX + 8) * (long long)sizeof(double);
}

int negf_poisson_solve(void* stream, const negf_poisson_grid* g, const double* shift, const double* rhs,
                       double* x, double tol, int max_iter, void* work, int* iters, double* rel_res) {
    if (!grid_ok(g) || !rhs || !x || !work || !(tol >= 0.0) || max_iter < 1) return NEGF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const long long n = atoms(g);
    const Grid gr = to_grid(g);
    double* r = static_cast<double*>(work);
    double* p = r + n;
    double* Ap = p + n;
    double* part = Ap + n;
    double* sc = part + RED_MAX;
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(cg_init_kernel, dim3(nb), dim3(PB), 0, s, rhs, x, r, p, part, n);
    hipLaunchKernelGGL(cg_first_kernel, dim3(1), dim3(PB), 0, s, part, nb, sc);
    NEGF_HIP_CHECK(hipGetLastError());
    double h[6];
    NEGF_HIP_CHECK(hipMemcpyAsync(h, sc, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
    NEGF_HIP_CHECK(hipStreamSynchronize(s));
    const double r0 = std::sqrt(h[5]);
    int it = 0;
    double rr = h[5];
    constexpr int CHECK = 16;             // iterations between host reads of the residual
    while (r0 > 0.0 && std::sqrt(rr) > tol * r0 && it < max_iter) {
        const int k = std::min(CHECK, max_iter - it);
        for (int q = 0; q < k; ++q) {
            hipLaunchKernelGGL(cg_apply_kernel, dim3(nb), dim3(PB), 0, s, gr, p, shift, Ap, part, n);
            hipLaunchKernelGGL(cg_alpha_kernel, dim3(1), dim3(PB), 0, s, part, nb, sc);
            hipLaunchKernelGGL(cg_update_kernel, dim3(nb), dim3(PB), 0, s, x, r, p, Ap, sc, part, n);
            hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(PB), 0, s, part, nb, sc);
            hipLaunchKernelGGL(cg_dir_kernel, dim3(nb), dim3(PB), 0, s, p, r, sc, n);
        }
        NEGF_HIP_CHECK(hipGetLastError());
        it += k;
        NEGF_HIP_CHECK(hipMemcpyAsync(h, sc, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
        NEGF_HIP_CHECK(hipStreamSynchronize(s));
        rr = h[3];
    }
    if (iters) *iters = it;
    if (rel_res) *rel_res = r0 > 0.0 ? std::sqrt(rr) / r0 : 0.0;
    return NEGF_OK;
}

long long negf_vec_work_bytes(long long n, int m) {
    if (n < 1 || m < 1) return -1;
    return (long long)std::max(m, 2) * red_blocks(n) * (long long)sizeof(double);
}

int negf_vec_dots(void* stream, long long n, int m, const double* X, long long ld, const double* y, double* out,
                  void* work) {
    if (n < 1 || m < 1 || m > 65535 || ld < n || !X || !y || !out || !work) return NEGF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int nb = red_blocks(n);
    double* part = static_cast<double*>(work);
    hipLaunchKernelGGL(dots_kernel, dim3(nb, m), dim3(PB), 0, s, X, ld, y, n, part);
    hipLaunchKernelGGL(dots_final_kernel, dim3(m), dim3(PB), 0, s, part, nb, out);
    NEGF_HIP_CHECK(hipGetLastError());
    return NEGF_OK;
}

int negf_vec_norms(void* stream, long long n, const double* x, double* out, void* work) {
    if (n < 1 || !x || !out || !work) return NEGF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int nb = red_blocks(n);
    double* part = static_cast<double*>(work);
    hipLaunchKernelGGL(norms_kernel, dim3(nb), dim3(PB), 0, s, x, n, part);
    hipLaunchKernelGGL(norms_final_kernel, dim3(1), dim3(PB), 0, s, part, nb, out);
    NEGF_HIP_CHECK(hipGetLastError());
    return NEGF_OK;
}

int negf_vec_combine(void* stream, long long n, int m, const double* X, long long ld, const double* c, double b,
                     double* y) {
    if (n < 1 || m < 0 || ld < n || (m > 0 && (!X || !c)) || !y || !std::isfinite(b)) return NEGF_EINVAL;
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)((n + PB - 1) / PB)), dim3(PB), 0, (hipStream_t)stream, X, ld,
                       m, c, b, y, n);
    NEGF_HIP_CHECK(hipGetLastError());
    return NEGF_OK;
}

}  // extern "C"
