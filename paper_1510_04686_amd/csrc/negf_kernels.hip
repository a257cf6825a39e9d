// Non-GEMM kernels of the RGF path: slab-block assembly with the
// block-diagonal inter-slab couplings, output extraction, bond-current and
// transmission traces, Sancho-Rubio helpers, the scattering self-energies of
// Eqs. (4)-(6) and the observables of Eqs. (7)-(8).
#include "negf_kernels.hpp"

namespace negf {

__device__ inline double fermi_d(double E, double mu, double kT) {
    return 1.0 / (1.0 + exp((E - mu) / kT));
}

// ---------------------------------------------------------------------------
// Assembly / block-sparse sandwich:
//   O = base + sign * opL(U) X opR(U)
// U = H_{u,u+1}(k) of local slab `uslab` is block-diagonal with ub x ub blocks,
// so each output tile (aligned to whole blocks) needs only the matching
// diagonal blocks of U and the same tile of X: 2 ub complex FMAs per element.
// base (mode 1, retarded):  (E + i eta - V - Sigma^R_scat) I - H_ii - Sigma_L(i=0) - Sigma_R(i=N-1)
// base (mode 2, lesser):    diag(Sigma^<_scat) + 2 i eta f_L I (if filled)
//                           - f_L (Sigma_L - Sigma_L^dagger)(i=0) - f_R (Sigma_R - Sigma_R^dagger)(i=N-1)
// ---------------------------------------------------------------------------
// Adds the mode's base term to element (gr, gc) of the assembled block.
// With `hpre`, element (gr, gc) of H_ii has already been read into *hpre.
__device__ inline void sandwich_base(const SandArgs& a, double2& z, int gr, int gc, int ik, int ie, int ns,
                                     long long gslab, double E, const double2* hpre = nullptr) {
    const int n = a.n;
    if (a.mode == 1) {
        const double2* H = a.hdiag + ik * a.hdiag_k + gslab * (long long)n * n;
        double2 h = hpre ? *hpre : H[(long long)gr * n + gc];
        z.x -= h.x; z.y -= h.y;
        if (gr == gc) {
            z.x += E; z.y += a.eta;
            if (a.v) z.x -= a.v[gslab * n + gr];
        }
        if (a.scat && gr / a.sopa == gc / a.sopa) {
            const double2 s = a.scat[(((long long)ie * a.total + gslab) * n + gr) * a.sopa + gc % a.sopa];
            z.x -= s.x; z.y -= s.y;
        }
        const long long lo = ((long long)ik * a.n_e + ie) * n * n;
        if (a.slab == 0) { double2 s = a.sigL[lo + (long long)gr * n + gc]; z.x -= s.x; z.y -= s.y; }
        if (a.slab == ns - 1) { double2 s = a.sigR[lo + (long long)gr * n + gc]; z.x -= s.x; z.y -= s.y; }
    } else if (a.mode == 3) {
        // adjoint source: the cotangent weights W_i on the diagonal
        if (gr == gc) z.x += a.wdiag[gslab * n + gr];
    } else if (a.mode == 2) {
        // lesser_ref: subtract the equilibrium source at the right-lead
        // occupation, i f_R (Gamma_L + Gamma_R + Gamma_scat + 2 eta); the
        // remaining source drives only the non-equilibrium part of G^<.
        const double fR = a.lesser_ref ? fermi_d(E, a.muR, a.kT) : 0.0;
        if (gr / a.sopa == gc / a.sopa) {
            const long long base = ((long long)ie * a.total + gslab) * n;
            if (a.scat) {
                const double2 s = a.scat[(base + gr) * a.sopa + gc % a.sopa];
                z.x += s.x; z.y += s.y;
            }
            if (a.lesser_ref && a.scat2) {
                // + f_R (Sigma^R - Sigma^R^dagger)_rc
                const double2 s1 = a.scat2[(base + gr) * a.sopa + gc % a.sopa];
                const double2 s2 = a.scat2[(base + gc) * a.sopa + gr % a.sopa];
                z.x += fR * (s1.x - s2.x); z.y += fR * (s1.y + s2.y);
            }
        }
        if (gr == gc) {
            if (a.eta_fill) z.y += 2.0 * a.eta * fermi_d(E, a.muL, a.kT);
            z.y -= 2.0 * a.eta * fR;
        }
        const long long lo = ((long long)ik * a.n_e + ie) * n * n;
        if (a.slab == 0) {
            double f = fermi_d(E, a.muL, a.kT) - fR;
            double2 s1 = a.sigL[lo + (long long)gr * n + gc], s2 = a.sigL[lo + (long long)gc * n + gr];
            z.x -= f * (s1.x - s2.x); z.y -= f * (s1.y + s2.y);
        }
        if (a.slab == ns - 1) {
            double f = fermi_d(E, a.muR, a.kT) - fR;
            double2 s1 = a.sigR[lo + (long long)gr * n + gc], s2 = a.sigR[lo + (long long)gc * n + gr];
            z.x -= f * (s1.x - s2.x); z.y -= f * (s1.y + s2.y);
        }
    }
}

template <typename TX, typename TO>
__global__ __launch_bounds__(256) void sandwich_kernel(SandArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double2* sm = reinterpret_cast<double2*>(smem_raw);
    const int n = a.n, ub = a.ub, T = a.tile;
    const int tiles = (n + T - 1) / T, tpp = tiles * tiles;
    const int q = blockIdx.x / tpp;
    if (q >= a.np || !a.act(q)) return;
    const int t = blockIdx.x - q * tpp;
    const int r0 = (t / tiles) * T, c0 = (t % tiles) * T;
    const int tr = min(T, n - r0), tc = min(T, n - c0);
    const int tid = threadIdx.x;
    const int4 d = a.ps.desc[a.ps.p0 + q];
    const int ik = d.y, ie = d.z, ns = d.w;
    const long long sfirst = a.ps.slab_off[d.x];
    const int TP = T + 1;
    double2* Xs = sm;
    double2* Ys = Xs + T * TP;
    double2* UL = Ys + T * TP;
    double2* UR = UL + T * ub;
    const bool has_x = a.X != nullptr;
    if (has_x) {
        const TX* X = reinterpret_cast<const TX*>(a.X) + q * a.sX;
        for (int idx = tid; idx < tr * tc; idx += 256) {
            int r = idx / tc, c = idx - r * tc;
            Xs[r * TP + c] = cconv<double2>(X[(long long)(r0 + r) * n + c0 + c]);
        }
        const double2* U = a.hup + ik * a.hup_k + (sfirst + a.uslab) * (long long)n * n;
        if (a.opR) {
            for (int idx = tid; idx < tc * ub; idx += 256) {
                int c = idx / ub, j = idx - c * ub;
                int gc = c0 + c, l = (gc / ub) * ub + j;
                // opR(U)[l][gc]
                if (a.opR == 1) UR[c * ub + j] = U[(long long)l * n + gc];
                else UR[c * ub + j] = cconj(U[(long long)gc * n + l]);
            }
        }
        if (a.opL) {
            for (int idx = tid; idx < tr * ub; idx += 256) {
                int r = idx / ub, j = idx - r * ub;
                int gr = r0 + r, l = (gr / ub) * ub + j;
                // opL(U)[gr][l]
                if (a.opL == 1) UL[r * ub + j] = U[(long long)gr * n + l];
                else UL[r * ub + j] = cconj(U[(long long)l * n + gr]);
            }
        }
        __syncthreads();
        if (a.opR) {
            for (int idx = tid; idx < tr * tc; idx += 256) {
                int r = idx / tc, c = idx - r * tc;
                int cb = ((c0 + c) / ub) * ub - c0;
                double2 s = make_double2(0, 0);
                for (int j = 0; j < ub; ++j) cfma(s, Xs[r * TP + cb + j], UR[c * ub + j]);
                Ys[r * TP + c] = s;
            }
            __syncthreads();
        } else {
            double2* tmp = Xs; Xs = Ys; Ys = tmp;   // Y = X
        }
    }
    TO* O = reinterpret_cast<TO*>(a.O) + q * a.sO;
    const long long gslab = sfirst + a.slab;
    const double E = a.energy ? a.energy[ie] : 0.0;
    for (int idx = tid; idx < tr * tc; idx += 256) {
        int r = idx / tc, c = idx - r * tc;
        int gr = r0 + r, gc = c0 + c;
        double2 z = make_double2(0, 0);
        if (has_x) {
            if (a.opL) {
                int rb = (gr / ub) * ub - r0;
                for (int j = 0; j < ub; ++j) cfma(z, UL[r * ub + j], Ys[(rb + j) * TP + c]);
            } else {
                z = Ys[r * TP + c];
            }
            z.x *= a.sign; z.y *= a.sign;
        }
        sandwich_base(a, z, gr, gc, ik, ie, ns, gslab, E);
        O[(long long)gr * n + gc] = cconv<TO>(z);
    }
}

// The same operation for the common block sizes (1, 2, 4, 8, 10, 16): one
// workgroup per (point, block row of UB rows, chunk of whole column blocks),
// one thread per column.  Each thread reads its UB entries of X once
// (coalesced); for X U they go through LDS, where every thread finds the UB
// columns of its block; U^dagger Y mixes the thread's own rows in registers
// with the diagonal block of U from LDS.  UB and the operand forms are
// compile-time, so the loops carry no guards.
// Threads per workgroup of the column-chunk form: 128 keeps the X U chunk in
// LDS at about 20 KB, so twice as many workgroups (and their reads) fit on a CU.
constexpr int SAND_NT = 128;

template <typename TX, typename TO, int UB, int OPL, int OPR>
__global__ __launch_bounds__(SAND_NT) void sandwich_cols_kernel(SandArgs a) {
    constexpr int CW = (SAND_NT / UB) * UB;   // columns per chunk
    __shared__ double2 xs[OPR == 1 ? UB : 1][OPR == 1 ? CW : 1];
    __shared__ double2 ul[OPL == 2 ? UB : 1][OPL == 2 ? UB : 1];
    const int n = a.n;
    const int nblk = n / UB, nch = (n + CW - 1) / CW;
    const int per = nblk * nch;
    const int q = blockIdx.x / per;
    if (q >= a.np || !a.act(q)) return;
    const int t = blockIdx.x - q * per;
    const int blk = t / nch, c0 = (t - blk * nch) * CW;
    const int tid = threadIdx.x;
    const int c = c0 + tid;
    const bool on = tid < CW && c < n;
    const int rb = blk * UB, cb = on ? (c / UB) * UB : 0;
    const int4 d = a.ps.desc[a.ps.p0 + q];
    const int ik = d.y, ie = d.z, ns = d.w;
    const long long sfirst = a.ps.slab_off[d.x];
    double2 y[UB];
#pragma unroll
    for (int i = 0; i < UB; ++i) y[i] = make_double2(0, 0);
    if (a.X) {   // uniform over the workgroup
        const TX* X = reinterpret_cast<const TX*>(a.X) + q * a.sX;
        const double2* U = a.hup + ik * a.hup_k + (sfirst + a.uslab) * (long long)n * n;
        if constexpr (OPL == 2) {
            for (int e = tid; e < UB * UB; e += SAND_NT) ul[e / UB][e % UB] = U[(long long)(rb + e / UB) * n + rb + e % UB];
        }
        if (on) {
#pragma unroll
            for (int i = 0; i < UB; ++i) {
                const double2 x = cconv<double2>(X[(long long)(rb + i) * n + c]);
                if constexpr (OPR == 1) xs[i][tid] = x;
                else y[i] = x;
            }
        }
        if constexpr (OPR == 1 || OPL == 2) __syncthreads();
        if constexpr (OPR == 1) {
            if (on) {
                double2 uc[UB];   // U[cb + j][c]
#pragma unroll
                for (int j = 0; j < UB; ++j) uc[j] = U[(long long)(cb + j) * n + c];
                const int lb = cb - c0;
#pragma unroll
                for (int i = 0; i < UB; ++i)
#pragma unroll
                    for (int j = 0; j < UB; ++j) cfma(y[i], xs[i][lb + j], uc[j]);
            }
        }
        if constexpr (OPL == 2) {
            double2 z[UB];
#pragma unroll
            for (int i = 0; i < UB; ++i) {
                z[i] = make_double2(0, 0);
#pragma unroll
                for (int k = 0; k < UB; ++k) cfma(z[i], cconj(ul[k][i]), y[k]);
            }
#pragma unroll
            for (int i = 0; i < UB; ++i) y[i] = z[i];
        }
    }
    if (!on) return;
    TO* O = reinterpret_cast<TO*>(a.O) + q * a.sO;
    const long long gslab = sfirst + a.slab;
    const double E = a.energy ? a.energy[ie] : 0.0;
    // the assembly's H_ii entries of all UB rows are read at once (the stores
    // of the row loop would otherwise keep each read behind the previous row);
    // the assembly is the U^dagger X U form, the only one whose registers it costs
    constexpr bool PRE = (OPL == 2 && OPR == 1);
    double2 hv[PRE ? UB : 1];
    if (PRE && a.mode == 1) {
        const double2* H = a.hdiag + ik * a.hdiag_k + gslab * (long long)n * n;
#pragma unroll
        for (int i = 0; i < UB; ++i) hv[i] = H[(long long)(rb + i) * n + c];
    }
#pragma unroll
    for (int i = 0; i < UB; ++i) {
        double2 z = y[i];
        z.x *= a.sign; z.y *= a.sign;
        sandwich_base(a, z, rb + i, c, ik, ie, ns, gslab, E, (PRE && a.mode == 1) ? &hv[PRE ? i : 0] : nullptr);
        O[(long long)(rb + i) * n + c] = cconv<TO>(z);
    }
}

int sandwich_tile(int ub) { int m = 48 / ub; if (m < 1) m = 1; return ub * m; }
size_t sandwich_lds(int ub) {
    int T = sandwich_tile(ub);
    return (size_t)(2 * T * (T + 1) + 2 * T * ub) * sizeof(double2);
}

hipError_t sandwich_init() {
    const void* k[4] = {(const void*)sandwich_kernel<double2, double2>, (const void*)sandwich_kernel<float2, double2>,
                        (const void*)sandwich_kernel<double2, float2>, (const void*)sandwich_kernel<float2, float2>};
    for (const void* f : k) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sandwich_lds(48));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename TX, typename TO, int UB>
static bool sandwich_cols_ops(hipStream_t s, const SandArgs& a, dim3 grid) {
    if (a.opL == 0 && a.opR == 1) hipLaunchKernelGGL((sandwich_cols_kernel<TX, TO, UB, 0, 1>), grid, dim3(SAND_NT), 0, s, a);
    else if (a.opL == 2 && a.opR == 0) hipLaunchKernelGGL((sandwich_cols_kernel<TX, TO, UB, 2, 0>), grid, dim3(SAND_NT), 0, s, a);
    else if (a.opL == 2 && a.opR == 1) hipLaunchKernelGGL((sandwich_cols_kernel<TX, TO, UB, 2, 1>), grid, dim3(SAND_NT), 0, s, a);
    else if (a.opL == 0 && a.opR == 0) hipLaunchKernelGGL((sandwich_cols_kernel<TX, TO, UB, 0, 0>), grid, dim3(SAND_NT), 0, s, a);
    else return false;
    return true;
}

template <typename TX, typename TO>
static bool sandwich_cols_launch(hipStream_t s, const SandArgs& a) {
    const int cw = (SAND_NT / a.ub) * a.ub;
    const long long per = (long long)(a.n / a.ub) * ((a.n + cw - 1) / cw);
    dim3 grid((unsigned)((long long)a.np * per));
    switch (a.ub) {
        case 1: return sandwich_cols_ops<TX, TO, 1>(s, a, grid);
        case 2: return sandwich_cols_ops<TX, TO, 2>(s, a, grid);
        case 4: return sandwich_cols_ops<TX, TO, 4>(s, a, grid);
        case 8: return sandwich_cols_ops<TX, TO, 8>(s, a, grid);
        case 10: return sandwich_cols_ops<TX, TO, 10>(s, a, grid);
        case 16: return sandwich_cols_ops<TX, TO, 16>(s, a, grid);
        default: return false;
    }
}

hipError_t sandwich_launch(hipStream_t s, int xdt, int odt, const SandArgs& a) {
    if (a.np <= 0) return hipSuccess;
    bool done;
    if (xdt == DT_C128 && odt == DT_C128) done = sandwich_cols_launch<double2, double2>(s, a);
    else if (xdt == DT_C64 && odt == DT_C128) done = sandwich_cols_launch<float2, double2>(s, a);
    else if (xdt == DT_C128 && odt == DT_C64) done = sandwich_cols_launch<double2, float2>(s, a);
    else done = sandwich_cols_launch<float2, float2>(s, a);
    if (done) return hipGetLastError();
    const int tiles = (a.n + a.tile - 1) / a.tile;
    dim3 grid((unsigned)((long long)a.np * tiles * tiles));
    size_t lds = sandwich_lds(a.ub);
    if (xdt == DT_C128 && odt == DT_C128) hipLaunchKernelGGL((sandwich_kernel<double2, double2>), grid, dim3(256), lds, s, a);
    else if (xdt == DT_C64 && odt == DT_C128) hipLaunchKernelGGL((sandwich_kernel<float2, double2>), grid, dim3(256), lds, s, a);
    else if (xdt == DT_C128 && odt == DT_C64) hipLaunchKernelGGL((sandwich_kernel<double2, float2>), grid, dim3(256), lds, s, a);
    else hipLaunchKernelGGL((sandwich_kernel<float2, float2>), grid, dim3(256), lds, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Plain batched copy with type conversion (active points only).
// ---------------------------------------------------------------------------
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void copy_kernel(const void* src, long long ss, void* dst, long long sd,
                                                   long long nel, int np, Active act) {
    const long long per = (nel + 255) / 256;
    const int q = (int)(blockIdx.x / per);
    if (q >= np || !act(q)) return;
    const long long i = (blockIdx.x - (long long)q * per) * 256 + threadIdx.x;
    if (i >= nel) return;
    reinterpret_cast<TO*>(dst)[q * sd + i] = cconv<TO>(reinterpret_cast<const TI*>(src)[q * ss + i]);
}

hipError_t copy_launch(hipStream_t s, int tdi, int tdo, const void* src, long long ss, void* dst, long long sd,
                       long long nel, int np, const Active& act) {
    if (np <= 0 || nel <= 0) return hipSuccess;
    dim3 grid((unsigned)((long long)np * ((nel + 255) / 256)));
    if (tdi == DT_C128 && tdo == DT_C128) hipLaunchKernelGGL((copy_kernel<double2, double2>), grid, dim3(256), 0, s, src, ss, dst, sd, nel, np, act);
    else if (tdi == DT_C128) hipLaunchKernelGGL((copy_kernel<double2, float2>), grid, dim3(256), 0, s, src, ss, dst, sd, nel, np, act);
    else if (tdo == DT_C128) hipLaunchKernelGGL((copy_kernel<float2, double2>), grid, dim3(256), 0, s, src, ss, dst, sd, nel, np, act);
    else hipLaunchKernelGGL((copy_kernel<float2, float2>), grid, dim3(256), 0, s, src, ss, dst, sd, nel, np, act);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Output extraction: diagonal (or full) blocks of G^R, G^<, and
// G^> = G^< + G^R - G^R^dagger, written at bound point p = p0 + q, slab `slab`.
// ---------------------------------------------------------------------------
template <typename TI>
__global__ __launch_bounds__(256) void extract_kernel(ExtArgs a) {
    const int n = a.n;
    const long long nel = a.full == 1 ? (long long)n * n : (a.full == 2 ? (long long)n * a.opa : n);
    const long long per = (nel + 255) / 256;
    const int q = (int)(blockIdx.x / per);
    if (q >= a.np || !a.act(q)) return;
    const long long i = (blockIdx.x - (long long)q * per) * 256 + threadIdx.x;
    if (i >= nel) return;
    const TI* G = reinterpret_cast<const TI*>(a.G) + q * a.sG;
    const TI* GL = reinterpret_cast<const TI*>(a.GL) + q * a.sG;
    const long long p = a.p0 + q;
    int r, c;
    if (a.full == 1) {
        r = (int)(i / n); c = (int)(i - (long long)r * n);
    } else if (a.full == 2) {            // entry (r, c) of r's atom block, stored at [r][c mod opa]
        r = (int)(i / a.opa); c = (r / a.opa) * a.opa + (int)(i - (long long)r * a.opa);
    } else {
        r = c = (int)i;
    }
    double2 g = cconv<double2>(G[(long long)r * n + c]);
    double2 gl = cconv<double2>(GL[(long long)r * n + c]);
    double2 gt = g;
    if (r != c) gt = cconv<double2>(G[(long long)c * n + r]);
    // spectral part (G - G^dagger)_rc = g - conj(gt)
    const double2 sp = make_double2(g.x - gt.x, g.y + gt.y);
    if (a.lesser_ref) {
        // G^< = G^<_noneq - f_R (G - G^dagger)
        const int ie = a.act.desc[p].z;
        const double fR = 1.0 / (1.0 + exp((a.energy[ie] - a.muR) / a.kT));
        gl.x -= fR * sp.x; gl.y -= fR * sp.y;
    }
    const long long o = (p * a.slab_stride + a.slab) * nel + i;
    if (a.outR) a.outR[o] = g;
    if (a.outL) a.outL[o] = gl;
    if (a.outG) a.outG[o] = make_double2(gl.x + sp.x, gl.y + sp.y);
}

// out[p][slab][o] = scale * X_q[o][o]  (FP64 blocks, active points only)
__global__ __launch_bounds__(256) void diag_out_kernel(const double2* X, long long sX, int n, int np, Active act,
                                                       double scale, double2* out, int slab_stride, int slab, int p0) {
    const int per = (n + 255) / 256;
    const int q = blockIdx.x / per;
    if (q >= np || !act(q)) return;
    const int o = (blockIdx.x - q * per) * 256 + threadIdx.x;
    if (o >= n) return;
    double2 v = X[q * sX + (long long)o * n + o];
    out[((long long)(p0 + q) * slab_stride + slab) * n + o] = make_double2(scale * v.x, scale * v.y);
}

hipError_t diag_out_launch(hipStream_t s, const double2* X, long long sX, int n, int np, const Active& act,
                           double scale, double2* out, int slab_stride, int slab, int p0) {
    if (np <= 0) return hipSuccess;
    const int per = (n + 255) / 256;
    hipLaunchKernelGGL(diag_out_kernel, dim3(np * per), dim3(256), 0, s, X, sX, n, np, act, scale, out,
                       slab_stride, slab, p0);
    return hipGetLastError();
}

hipError_t extract_launch(hipStream_t s, int dt, const ExtArgs& a) {
    if (a.np <= 0) return hipSuccess;
    const long long nel = a.full == 1 ? (long long)a.n * a.n : (a.full == 2 ? (long long)a.n * a.opa : a.n);
    dim3 grid((unsigned)((long long)a.np * ((nel + 255) / 256)));
    if (dt == DT_C128) hipLaunchKernelGGL(extract_kernel<double2>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(extract_kernel<float2>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Bond current  j_i = 2 Re Tr[H_{i,i+1} G^<_{i+1,i}]  with
//   G^<_{i+1,i} = G_{i+1} H_{i+1,i} g^<_i + G^<_{i+1} L^dagger,  L = g_i H_{i,i+1},
// U = H_{i,i+1} (block-diagonal with ub x ub blocks):
//   j_i = 2 Re[ Tr(U G U^dagger g^<_i) + sum_ab (U G^<)_ab conj(L_ab) ].
// g^<_i is anti-Hermitian, so Tr(U G U^dagger g^<) = -sum_ab (U G)_ab conj((g^< U)_ab):
// every factor is then read row-major, in the order the threads walk b.
// One workgroup per (point, group of atom blocks) walks the columns in chunks
// of whole coupling blocks: the ub rows of G, G^<, L and g^<_i at a thread's
// column are read once from HBM (those of L as they are used), the g^<_i rows of the chunk are staged in LDS
// for the column-block product g^< U, and the diagonal block of U for the
// row-block products sits in LDS.  The partials are added in a fixed order.
// ---------------------------------------------------------------------------
template <typename TI, int UB>
__global__ __launch_bounds__(256) void bond_rows_kernel(BondArgs a) {
    constexpr int CW = (256 / UB) * UB;   // columns per chunk, whole coupling blocks
    __shared__ double2 gsl[UB][CW];       // g^<_i rows r0.. of the chunk
    __shared__ double2 ub[UB][UB];        // U[r0 + i][r0 + j]
    __shared__ double red[256];
    const int q = blockIdx.x / BOND_NWB, w = blockIdx.x - q * BOND_NWB;
    if (q >= a.np || !a.act(q)) return;
    const int n = a.n, tid = threadIdx.x;
    const int nblk = n / UB;
    const int4 d = a.ps.desc[a.ps.p0 + q];
    const long long sfirst = a.ps.slab_off[d.x];
    const double2* U = a.hup + d.y * a.hup_k + (sfirst + a.slab) * (long long)n * n;
    const TI* G = reinterpret_cast<const TI*>(a.G) + q * a.sM;
    const TI* GL = reinterpret_cast<const TI*>(a.GL) + q * a.sM;
    const TI* L = reinterpret_cast<const TI*>(a.L) + q * a.sM;
    const TI* GS = reinterpret_cast<const TI*>(a.gls) + q * a.s_gls;
    double acc = 0.0;
    for (int A = w; A < nblk; A += BOND_NWB) {
        const int r0 = A * UB;
        if (tid < UB * UB) ub[tid / UB][tid % UB] = U[(long long)(r0 + tid / UB) * n + r0 + tid % UB];
        for (int c0 = 0; c0 < n; c0 += CW) {
            const int b = c0 + tid;
            const bool on = tid < CW && b < n;
            double2 gc[UB], glc[UB], uc[UB];
            const int bb = on ? (b / UB) * UB : 0;
            if (on) {
                // the g^< rows first, all in flight at once, then their LDS
                // stores; then the G, G^< and U rows, all in flight at once
                // (two memory round trips instead of one per row, in the same
                // registers)
                {
                    double2 gs[UB];
#pragma unroll
                    for (int j = 0; j < UB; ++j) gs[j] = cconv<double2>(GS[(long long)(r0 + j) * n + b]);
#pragma unroll
                    for (int j = 0; j < UB; ++j) gsl[j][tid] = gs[j];
                }
#pragma unroll
                for (int j = 0; j < UB; ++j) {
                    const long long o = (long long)(r0 + j) * n + b;
                    gc[j] = cconv<double2>(G[o]);
                    glc[j] = cconv<double2>(GL[o]);
                    uc[j] = U[(long long)(bb + j) * n + b];
                }
            }
            __syncthreads();
            if (on) {
                const int lb = bb - c0;   // the thread's column block, chunk-local
#pragma unroll
                for (int i = 0; i < UB; ++i) {
                    double2 ug = make_double2(0, 0), ugl = make_double2(0, 0), gu = make_double2(0, 0);
#pragma unroll
                    for (int j = 0; j < UB; ++j) {
                        const double2 u = ub[i][j];
                        cfma(ug, u, gc[j]);
                        cfma(ugl, u, glc[j]);
                        cfma(gu, gsl[i][lb + j], uc[j]);
                    }
                    const double2 l = cconv<double2>(L[(long long)(r0 + i) * n + b]);
                    acc += (ugl.x * l.x + ugl.y * l.y) - (ug.x * gu.x + ug.y * gu.y);
                }
            }
            __syncthreads();   // gsl (and ub, at the next row block) are rewritten next
        }
    }
    red[tid] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) a.partial[(long long)q * BOND_NWB + w] = red[0];
}

// Blocks wider than the register path: j_i = 2 Re[ sum_ab (U G)_ab Q_ba + (U G^<)_ab conj(L_ab) ]
// with Q = U^dagger g^<_i, rows split over BOND_NWB workgroups.
template <typename TI>
__global__ __launch_bounds__(256) void bond_partial_kernel(BondArgs a) {
    const int q = blockIdx.x / BOND_NWB, w = blockIdx.x - q * BOND_NWB;
    if (q >= a.np || !a.act(q)) return;
    const int n = a.n, ub = a.ub, tid = threadIdx.x;
    const int4 d = a.ps.desc[a.ps.p0 + q];
    const long long sfirst = a.ps.slab_off[d.x];
    const double2* U = a.hup + d.y * a.hup_k + (sfirst + a.slab) * (long long)n * n;
    const TI* G = reinterpret_cast<const TI*>(a.G) + q * a.sM;
    const TI* GL = reinterpret_cast<const TI*>(a.GL) + q * a.sM;
    const TI* Q = reinterpret_cast<const TI*>(a.Q) + q * a.sM;
    const TI* L = reinterpret_cast<const TI*>(a.L) + q * a.sM;
    const int rows = (n + BOND_NWB - 1) / BOND_NWB;
    const int a0 = min(n, w * rows), a1 = min(n, a0 + rows);
    double acc = 0.0;
    for (long long idx = (long long)a0 * n + tid; idx < (long long)a1 * n; idx += 256) {
        const int r = (int)(idx / n), b = (int)(idx - (long long)r * n);
        const int rb = (r / ub) * ub;
        double2 ug = make_double2(0, 0), ugl = make_double2(0, 0);
        for (int j = 0; j < ub; ++j) {
            double2 u = U[(long long)r * n + rb + j];
            cfma(ug, u, cconv<double2>(G[(long long)(rb + j) * n + b]));
            cfma(ugl, u, cconv<double2>(GL[(long long)(rb + j) * n + b]));
        }
        double2 qv = cconv<double2>(Q[(long long)b * n + r]);
        double2 lv = cconv<double2>(L[(long long)r * n + b]);
        acc += ug.x * qv.x - ug.y * qv.y;          // Re(ug * qv)
        acc += ugl.x * lv.x + ugl.y * lv.y;        // Re(ugl * conj(lv))
    }
    __shared__ double red[256];
    red[tid] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    if (tid == 0) a.partial[(long long)q * BOND_NWB + w] = red[0];
}

__global__ void bond_final_kernel(const double* partial, double* out, int slab_stride, int slab, int p0, int np,
                                  Active act) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= np || !act(q)) return;
    double s = 0.0;
    for (int w = 0; w < BOND_NWB; ++w) s += partial[(long long)q * BOND_NWB + w];
    out[(long long)(p0 + q) * slab_stride + slab] = 2.0 * s;
}

template <typename TI>
static void bond_dispatch(hipStream_t s, const BondArgs& a, dim3 grid) {
    const bool rows = a.gls != nullptr;
    if (rows && a.ub == 1) hipLaunchKernelGGL((bond_rows_kernel<TI, 1>), grid, dim3(256), 0, s, a);
    else if (rows && a.ub == 2) hipLaunchKernelGGL((bond_rows_kernel<TI, 2>), grid, dim3(256), 0, s, a);
    else if (rows && a.ub == 4) hipLaunchKernelGGL((bond_rows_kernel<TI, 4>), grid, dim3(256), 0, s, a);
    else if (rows && a.ub == 8) hipLaunchKernelGGL((bond_rows_kernel<TI, 8>), grid, dim3(256), 0, s, a);
    else if (rows && a.ub == 10) hipLaunchKernelGGL((bond_rows_kernel<TI, 10>), grid, dim3(256), 0, s, a);
    else if (rows && a.ub == 16) hipLaunchKernelGGL((bond_rows_kernel<TI, 16>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(bond_partial_kernel<TI>, grid, dim3(256), 0, s, a);
}

hipError_t bond_launch(hipStream_t s, int dt, const BondArgs& a, double* out, int slab_stride) {
    if (a.np <= 0) return hipSuccess;
    dim3 grid((unsigned)(a.np * BOND_NWB));
    if (dt == DT_C128) bond_dispatch<double2>(s, a, grid);
    else bond_dispatch<float2>(s, a, grid);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bond_final_kernel, dim3((a.np + 255) / 256), dim3(256), 0, s, a.partial, out, slab_stride,
                       a.slab, a.ps.p0, a.np, a.act);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Broadening Gamma = i (Sigma - Sigma^dagger) of a lead, per point.
// ---------------------------------------------------------------------------
template <typename TO>
__global__ __launch_bounds__(256) void gamma_kernel(const double2* sig, int n_e, PointSet ps, void* out, long long so,
                                                    int n, int np) {
    const long long nel = (long long)n * n, per = (nel + 255) / 256;
    const int q = (int)(blockIdx.x / per);
    if (q >= np) return;
    const long long i = (blockIdx.x - (long long)q * per) * 256 + threadIdx.x;
    if (i >= nel) return;
    const int4 d = ps.desc[ps.p0 + q];
    const double2* S = sig + ((long long)d.y * n_e + d.z) * nel;
    const int r = (int)(i / n), c = (int)(i - (long long)r * n);
    double2 a = S[i], b = S[(long long)c * n + r];
    // i (a - conj(b)) = i((a.x - b.x) + i (a.y + b.y)) = -(a.y + b.y) + i (a.x - b.x)
    reinterpret_cast<TO*>(out)[q * so + i] = cconv<TO>(make_double2(-(a.y + b.y), a.x - b.x));
}

hipError_t gamma_launch(hipStream_t s, int dt, const double2* sig, int n_e, const PointSet& ps, void* out,
                        long long so, int n, int np) {
    if (np <= 0) return hipSuccess;
    const long long nel = (long long)n * n;
    dim3 grid((unsigned)((long long)np * ((nel + 255) / 256)));
    if (dt == DT_C128) hipLaunchKernelGGL(gamma_kernel<double2>, grid, dim3(256), 0, s, sig, n_e, ps, out, so, n, np);
    else hipLaunchKernelGGL(gamma_kernel<float2>, grid, dim3(256), 0, s, sig, n_e, ps, out, so, n, np);
    return hipGetLastError();
}

// T_p = Re sum_ab W1_ab W2_ba  (one workgroup per point, fixed-order reduction)
template <typename TI>
__global__ __launch_bounds__(256) void trace_prod_kernel(const void* W1, const void* W2, long long sw, int n, int np,
                                                         double* out, int p0) {
    const int q = blockIdx.x;
    if (q >= np) return;
    const TI* A = reinterpret_cast<const TI*>(W1) + q * sw;
    const TI* B = reinterpret_cast<const TI*>(W2) + q * sw;
    double acc = 0.0;
    for (long long idx = threadIdx.x; idx < (long long)n * n; idx += 256) {
        int r = (int)(idx / n), c = (int)(idx - (long long)r * n);
        double2 x = cconv<double2>(A[idx]), y = cconv<double2>(B[(long long)c * n + r]);
        acc += x.x * y.x - x.y * y.y;
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[p0 + q] = red[0];
}

hipError_t trace_prod_launch(hipStream_t s, int dt, const void* W1, const void* W2, long long sw, int n, int np,
                             double* out, int p0) {
    if (np <= 0) return hipSuccess;
    if (dt == DT_C128) hipLaunchKernelGGL(trace_prod_kernel<double2>, dim3(np), dim3(256), 0, s, W1, W2, sw, n, np, out, p0);
    else hipLaunchKernelGGL(trace_prod_kernel<float2>, dim3(np), dim3(256), 0, s, W1, W2, sw, n, np, out, p0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sancho-Rubio helpers.  Chunk point q is flat grid index f = f0 + q,
// ik = f / n_e, ie = f % n_e.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sr_init_kernel(SrArgs a) {
    const long long nel = (long long)a.n * a.n, per = (nel + 255) / 256;
    const int q = (int)(blockIdx.x / per);
    if (q >= a.np) return;
    const long long i = (blockIdx.x - (long long)q * per) * 256 + threadIdx.x;
    const long long f = a.f0 + q;
    const int ik = (int)(f / a.n_e);
    if (i < nel) {
        const int n = a.n, r = (int)(i / n), c = (int)(i - (long long)r * n);
        const long long kb = (long long)ik * nel;
        double2 h = a.h00[kb + i];
        a.eps_s[q * nel + i] = h;
        a.eps[q * nel + i] = h;
        a.alpha[q * nel + i] = a.h01[kb + i];
        a.beta[q * nel + i] = cconj(a.h01[kb + (long long)c * n + r]);
        a.tau[q * nel + i] = a.tauin[kb + i];
        if (a.eps_d) {
            a.eps_d[q * nel + i] = h;
            a.tau2[q * nel + i] = a.tauin2[kb + i];
        }
    }
    if (i == 0) {
        a.flags[q] = 0;
        a.iters[q] = 0;
        if (a.eps_d) a.iters2[q] = 0;
    }
}

// M = z I - X  (X = eps or eps_s), z = E + i eta
__global__ __launch_bounds__(256) void sr_zminus_kernel(SrArgs a, const double2* X, double2* M, Active act) {
    const long long nel = (long long)a.n * a.n, per = (nel + 255) / 256;
    const int q = (int)(blockIdx.x / per);
    if (q >= a.np || !act(q)) return;
    const long long i = (blockIdx.x - (long long)q * per) * 256 + threadIdx.x;
    if (i >= nel) return;
    const long long f = a.f0 + q;
    const int ie = (int)(f % a.n_e);
    const int n = a.n, r = (int)(i / n), c = (int)(i - (long long)r * n);
    double2 x = X[q * nel + i];
    double2 m = make_double2(-x.x, -x.y);
    if (r == c) { m.x += a.energy[ie]; m.y += a.eta; }
    M[q * nel + i] = m;
}

// Matrix 1-norm (largest column sum of |x|) of one n x n matrix by one workgroup.
__device__ double norm1_block(const double2* X, int n, double* red) {
    double best = 0.0;
    for (int c = threadIdx.x; c < n; c += 256) {
        double s = 0.0;
        for (int r = 0; r < n; ++r) { double2 v = X[(long long)r * n + c]; s += hypot(v.x, v.y); }
        best = fmax(best, s);
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    double v = red[0];
    __syncthreads();
    return v;
}

// Reference norms per chunk point: ||h01||_1, and for the dual surface
// ||h01^dagger||_1 (the largest row sum of |h01|).
__global__ __launch_bounds__(256) void sr_refnorm_kernel(SrArgs a) {
    const int q = blockIdx.x;
    if (q >= a.np) return;
    __shared__ double red[256];
    const long long f = a.f0 + q;
    const int ik = (int)(f / a.n_e);
    const double2* h = a.h01 + (long long)ik * a.n * a.n;
    double v = norm1_block(h, a.n, red);
    if (threadIdx.x == 0) a.ref[q] = v;
    if (!a.eps_d) return;
    double best = 0.0;
    for (int r = threadIdx.x; r < a.n; r += 256) {
        double t = 0.0;
        for (int c = 0; c < a.n; ++c) { double2 x = h[(long long)r * a.n + c]; t += hypot(x.x, x.y); }
        best = fmax(best, t);
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) a.ref2[q] = red[0];
}

// Convergence test after a decimation step: ||alpha||_1 + ||beta||_1 < tol ||h01||_1.
// The dual surface shares alpha and beta (with their roles swapped), so it
// differs only in its reference norm.  An iteration count is stored negated
// once its surface has converged; a point is done when every surface it
// carries has.
__global__ __launch_bounds__(256) void sr_check_kernel(SrArgs a, const double2* alpha, const double2* beta, int it) {
    const int q = blockIdx.x;
    if (q >= a.np || a.flags[q] != 0) return;
    __shared__ double red[256];
    const long long nel = (long long)a.n * a.n;
    double na = norm1_block(alpha + q * nel, a.n, red);
    double nb = norm1_block(beta + q * nel, a.n, red);
    if (threadIdx.x == 0) {
        const double sum = na + nb;
        if (a.iters[q] >= 0) a.iters[q] = sum < a.tol * a.ref[q] ? -it : it;
        bool done = a.iters[q] < 0;
        if (a.eps_d) {
            if (a.iters2[q] >= 0) a.iters2[q] = sum < a.tol * a.ref2[q] ? -it : it;
            done = done && a.iters2[q] < 0;
        }
        if (done) a.flags[q] = 1;
        else atomicAdd(a.count, 1);
    }
}

__global__ void sr_iters_out_kernel(const int* it, long long f0, int np, int* out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= np) return;
    out[f0 + q] = abs(it[q]);
}

// ---------------------------------------------------------------------------
// Scattering self-energies (Eqs. 4-6), in place, with partial norms.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void scba_kernel(ScbaArgs a) {
    const long long tot = (long long)a.n_e * a.N * a.n;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    double dif = 0.0, nrm = 0.0;
    if (i < tot) {
        const int o = (int)(i % a.n);
        const int s = (int)((i / a.n) % a.N);
        const int ie = (int)(i / ((long long)a.n * a.N));
        auto avg = [&](const double2* G, int e) {
            double2 acc = make_double2(0, 0);
            for (int k = 0; k < a.n_k; ++k) {
                double2 g = G[(((long long)k * a.n_e + e) * a.slab_stride + s) * a.n + o];
                acc.x += a.w_k[k] * g.x; acc.y += a.w_k[k] * g.y;
            }
            return acc;
        };
        double2 aR = avg(a.GR, ie), aL = avg(a.GL, ie);
        double2 nR = make_double2(a.D * aR.x, a.D * aR.y), nL = make_double2(a.D * aL.x, a.D * aL.y);
        if (a.M != 0.0 && a.shift > 0) {
            const int lo = ie - a.shift, hi = ie + a.shift;
            if (lo >= 0) {
                double2 r = avg(a.GR, lo), l = avg(a.GL, lo);
                nL.x += a.M * a.n0 * l.x; nL.y += a.M * a.n0 * l.y;
                nR.x += a.M * ((1.0 + a.n0) * r.x + 0.5 * l.x);
                nR.y += a.M * ((1.0 + a.n0) * r.y + 0.5 * l.y);
            }
            if (hi < a.n_e) {
                double2 r = avg(a.GR, hi), l = avg(a.GL, hi);
                nL.x += a.M * (1.0 + a.n0) * l.x; nL.y += a.M * (1.0 + a.n0) * l.y;
                nR.x += a.M * (a.n0 * r.x - 0.5 * l.x);
                nR.y += a.M * (a.n0 * r.y - 0.5 * l.y);
            }
        }
        double2 oR = a.sigR[i], oL = a.sigL[i];
        dif = (nR.x - oR.x) * (nR.x - oR.x) + (nR.y - oR.y) * (nR.y - oR.y) +
              (nL.x - oL.x) * (nL.x - oL.x) + (nL.y - oL.y) * (nL.y - oL.y);
        nrm = nR.x * nR.x + nR.y * nR.y + nL.x * nL.x + nL.y * nL.y;
        a.sigR[i] = nR;
        a.sigL[i] = nL;
    }
    __shared__ double rd[256], rn[256];
    rd[threadIdx.x] = dif;
    rn[threadIdx.x] = nrm;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) { rd[threadIdx.x] += rd[threadIdx.x + o]; rn[threadIdx.x] += rn[threadIdx.x + o]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { a.partial[2 * blockIdx.x] = rd[0]; a.partial[2 * blockIdx.x + 1] = rn[0]; }
}

__global__ __launch_bounds__(256) void scba_final_kernel(const double* partial, int nblk, double* out, double* hist,
                                                         int* hcount, int hmax) {
    double d = 0.0, m = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) { d += partial[2 * b]; m += partial[2 * b + 1]; }
    __shared__ double rd[256], rn[256];
    rd[threadIdx.x] = d;
    rn[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) { rd[threadIdx.x] += rd[threadIdx.x + o]; rn[threadIdx.x] += rn[threadIdx.x + o]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double r = rn[0] > 0 ? sqrt(rd[0] / rn[0]) : 0.0;
        if (out) out[0] = r;
        // append to the device history (read back once after a captured loop)
        const int c = *hcount;
        if (c < hmax) hist[c] = r;
        *hcount = c + 1;
    }
}

hipError_t scba_launch(hipStream_t s, const ScbaArgs& a, double* rel_change, double* hist, int* hcount,
                       int hmax) {
    const long long tot = (long long)a.n_e * a.N * a.n;
    const int nblk = (int)((tot + 255) / 256);
    hipLaunchKernelGGL(scba_kernel, dim3(nblk), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scba_final_kernel, dim3(1), dim3(256), 0, s, a.partial, nblk, rel_change, hist, hcount,
                       hmax);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Observables (Eqs. 7-8).  Points of each (sample, ie) pair are listed in
// csr_pts[csr_off[s*n_e + ie] .. csr_off[s*n_e + ie + 1]) in bound order; all
// sums run over ie, then that list: a fixed order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void obs_orbital_kernel(ObsArgs a) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;   // (global slab, orbital)
    if (i >= (long long)a.total * a.n) return;
    const long long sg = i / a.n;
    const int o = (int)(i - sg * a.n);
    const int smp = a.slab_sample[sg];
    const int li = (int)(sg - a.slab_off[smp]);
    double acc = 0.0;
    for (int ie = 0; ie < a.n_e; ++ie) {
        const int b = a.csr_off[smp * a.n_e + ie], e = a.csr_off[smp * a.n_e + ie + 1];
        double se = 0.0;
        for (int t = b; t < e; ++t) {
            const int p = a.csr_pts[t];
            const int ik = a.desc[p].y;
            const long long ix = (((long long)p * a.slab_stride + li) * a.n + o) * a.gopa + o % a.gopa;
            const double2 gl = a.GL[ix];
            double v = gl.y;
            if (a.GR) {                  // Im(g gl + gl conj(g)) = 2 Re(g) Im(gl)
                const double2 g = a.GR[ix];
                v = 2.0 * g.x * gl.y;
            }
            se += a.w_k[ik] * v;
        }
        acc += a.w_e[ie] * se;
    }
    a.orb_tmp[i] = acc;
}

__global__ __launch_bounds__(256) void obs_atom_kernel(ObsArgs a) {
    const int nat = a.n / a.opa;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)a.total * nat) return;
    const long long sg = i / nat;
    const int at = (int)(i - sg * nat);
    double s = 0.0;
    for (int o = 0; o < a.opa; ++o) s += a.orb_tmp[sg * a.n + at * a.opa + o];
    a.n_out[i] = a.g_s * s / (2.0 * 3.14159265358979323846);
}

__global__ __launch_bounds__(256) void obs_current_kernel(ObsArgs a) {
    const long long sg = (long long)blockIdx.x * 256 + threadIdx.x;
    if (sg >= a.total) return;
    const int smp = a.slab_sample[sg];
    const int li = (int)(sg - a.slab_off[smp]);
    const int ns = (int)(a.slab_off[smp + 1] - a.slab_off[smp]);
    double acc = 0.0;
    if (li < ns - 1) {
        for (int ie = 0; ie < a.n_e; ++ie) {
            const int b = a.csr_off[smp * a.n_e + ie], e = a.csr_off[smp * a.n_e + ie + 1];
            double se = 0.0;
            for (int t = b; t < e; ++t) {
                const int p = a.csr_pts[t];
                se += a.w_k[a.desc[p].y] * a.bond[(long long)p * a.slab_stride + li];
            }
            acc += a.w_e[ie] * se;
        }
    }
    a.J[sg] = a.g_s * acc;
}

__global__ __launch_bounds__(256) void obs_spectral_kernel(ObsArgs a) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;   // (sample, ie, bond)
    if (i >= (long long)a.n_samples * a.n_e * a.slab_stride) return;
    const int li = (int)(i % a.slab_stride);
    const long long se_i = i / a.slab_stride;
    const int ie = (int)(se_i % a.n_e);
    const int smp = (int)(se_i / a.n_e);
    const int ns = (int)(a.slab_off[smp + 1] - a.slab_off[smp]);
    double acc = 0.0;
    if (li < ns - 1) {
        const int b = a.csr_off[smp * a.n_e + ie], e = a.csr_off[smp * a.n_e + ie + 1];
        for (int t = b; t < e; ++t) {
            const int p = a.csr_pts[t];
            acc += a.w_k[a.desc[p].y] * a.bond[(long long)p * a.slab_stride + li];
        }
    }
    a.jE[i] = a.g_s * acc;
}

hipError_t observables_launch(hipStream_t s, const ObsArgs& a) {
    const long long norb = a.total * a.n;
    if (a.n_out) {
        hipLaunchKernelGGL(obs_orbital_kernel, dim3((unsigned)((norb + 255) / 256)), dim3(256), 0, s, a);
        const long long nat = a.total * (a.n / a.opa);
        hipLaunchKernelGGL(obs_atom_kernel, dim3((unsigned)((nat + 255) / 256)), dim3(256), 0, s, a);
    }
    if (a.J) hipLaunchKernelGGL(obs_current_kernel, dim3((unsigned)((a.total + 255) / 256)), dim3(256), 0, s, a);
    if (a.jE) {
        const long long m = (long long)a.n_samples * a.n_e * a.slab_stride;
        hipLaunchKernelGGL(obs_spectral_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t sr_launch_init(hipStream_t s, const SrArgs& a) {
    const long long nel = (long long)a.n * a.n;
    hipLaunchKernelGGL(sr_init_kernel, dim3((unsigned)((long long)a.np * ((nel + 255) / 256))), dim3(256), 0, s, a);
    hipLaunchKernelGGL(sr_refnorm_kernel, dim3(a.np), dim3(256), 0, s, a);
    return hipGetLastError();
}
hipError_t sr_launch_zminus(hipStream_t s, const SrArgs& a, const double2* X, double2* M, const Active& act) {
    const long long nel = (long long)a.n * a.n;
    hipLaunchKernelGGL(sr_zminus_kernel, dim3((unsigned)((long long)a.np * ((nel + 255) / 256))), dim3(256), 0, s, a, X, M, act);
    return hipGetLastError();
}
hipError_t sr_launch_check(hipStream_t s, const SrArgs& a, const double2* alpha, const double2* beta, int it) {
    hipLaunchKernelGGL(sr_check_kernel, dim3(a.np), dim3(256), 0, s, a, alpha, beta, it);
    return hipGetLastError();
}
hipError_t sr_launch_iters(hipStream_t s, const SrArgs& a, const int* it, int* out) {
    hipLaunchKernelGGL(sr_iters_out_kernel, dim3((a.np + 255) / 256), dim3(256), 0, s, it, a.f0, a.np, out);
    return hipGetLastError();
}

}  // namespace negf

namespace negf {

// Checks h01_L = h01_R^dagger over all k, which lets one decimation serve both
// leads (the dual surface).  Per-block maxima of the deviation and of |h01_R|.
__global__ __launch_bounds__(256) void lead_dual_check_kernel(const double2* h01L, const double2* h01R, int n,
                                                              long long tot, double* partial) {
    const long long nn = (long long)n * n;
    double d = 0.0, m = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < tot; i += (long long)gridDim.x * 256) {
        const long long k = i / nn, e = i - k * nn;
        const int r = (int)(e / n), c = (int)(e - (long long)r * n);
        const double2 x = h01L[i], y = h01R[k * nn + (long long)c * n + r];
        d = fmax(d, fmax(fabs(x.x - y.x), fabs(x.y + y.y)));
        m = fmax(m, fmax(fabs(y.x), fabs(y.y)));
    }
    __shared__ double rd[256], rm[256];
    rd[threadIdx.x] = d;
    rm[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            rd[threadIdx.x] = fmax(rd[threadIdx.x], rd[threadIdx.x + o]);
            rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { partial[2 * blockIdx.x] = rd[0]; partial[2 * blockIdx.x + 1] = rm[0]; }
}

hipError_t lead_dual_check_launch(hipStream_t s, const double2* h01L, const double2* h01R, int n_k, int n,
                                  double* partial, int nblk) {
    hipLaunchKernelGGL(lead_dual_check_kernel, dim3(nblk), dim3(256), 0, s, h01L, h01R, n,
                       (long long)n_k * n * n, partial);
    return hipGetLastError();
}

}  // namespace negf
