// Whole recursive Green's function solve of one (sample, k, E) point per
// wavefront, for blocks of at most 8 orbitals (the single-orbital strip).
//
// At such sizes a slab step is a handful of 8 x 8 complex products: the
// batched per-operation launches of the large-block path are pure launch
// latency.  Here one persistent launch covers every point: each wavefront
// pulls the next point from a device work queue (an atomic counter, points in
// bound order, longest sample first) and runs the forward sweep (Eqs. 1-2 by
// the left-connected recursion), the backward sweep, the bond currents and
// the Caroli transmission for it.  Lane l holds element (l / 8, l % 8) of
// every 8 x 8 block; products and the pivoted Gauss-Jordan inverse exchange
// rows and columns through the wavefront's LDS.  Blocks narrower than 8 are
// padded: zero couplings and self-energies, identity on the padded diagonal
// of the inverted block, so the padding never mixes with the physical part.
#include "negf_kernels.hpp"

namespace negf {

namespace {

constexpr int SB = 8;        // padded block edge
constexpr int SL = SB * SB;  // lanes per point

__device__ inline double fermi_s(double E, double mu, double kT) { return 1.0 / (1.0 + exp((E - mu) / kT)); }

struct Lds {
    double2 a[SL];
    double2 b[SL];
    int perm[SB];
    int bad;
};

// C = op(A) op(B), op = conjugate transpose when CA / CB; each lane passes
// its element of A and B and gets its element of C.
template <bool CA, bool CB>
__device__ inline double2 mmt(Lds& s, int lane, double2 a, double2 b) {
    const int r = lane >> 3, c = lane & 7;
    s.a[lane] = a;
    s.b[lane] = b;
    __syncthreads();
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll 4
    for (int k = 0; k < SB; ++k) {
        const double2 x = CA ? cconj(s.a[k * SB + r]) : s.a[r * SB + k];
        const double2 y = CB ? cconj(s.b[c * SB + k]) : s.b[k * SB + c];
        cfma(acc, x, y);
    }
    __syncthreads();
    return acc;
}

__device__ __noinline__ double2 mm_nn(Lds& s, int lane, double2 a, double2 b) { return mmt<false, false>(s, lane, a, b); }
__device__ __noinline__ double2 mm_cn(Lds& s, int lane, double2 a, double2 b) { return mmt<true, false>(s, lane, a, b); }
__device__ __noinline__ double2 mm_nc(Lds& s, int lane, double2 a, double2 b) { return mmt<false, true>(s, lane, a, b); }

__device__ inline double2 mm(Lds& s, int lane, double2 a, double2 b, bool ca, bool cb) {
    if (ca) return mm_cn(s, lane, a, b);
    if (cb) return mm_nc(s, lane, a, b);
    return mm_nn(s, lane, a, b);
}

// Element (c, r) of the block whose element (r, c) this lane holds.
__device__ inline double2 transposed(Lds& s, int lane, double2 x) {
    const int r = lane >> 3, c = lane & 7;
    s.a[lane] = x;
    __syncthreads();
    const double2 y = s.a[c * SB + r];
    __syncthreads();
    return y;
}

// Exact anti-Hermitian part (X - X^dagger) / 2 of a block meant to be
// anti-Hermitian (g^<, G^<): keeps rounding from accumulating a Hermitian part.
__device__ inline double2 anti_herm(Lds& s, int lane, double2 x) {
    const double2 t = transposed(s, lane, x);
    return make_double2(0.5 * (x.x - t.x), 0.5 * (x.y + t.y));
}

// Next work item of the queue, wave-uniform: every lane takes part in the
// atomic (lane 0 adds 1, the others 0) and the value lane 0 got is read back
// as a scalar.  No lane-dependent branch may sit in a persistent loop whose
// lanes must stay together: with a branch that only lane 0 takes (the
// atomic, a store of a per-point result) the compiler, which drops the
// barriers of a one-wave workgroup, was free to split the loop so that lanes
// 1-63 went round again without lane 0 -- and without its next atomic: a loop
// that never ended.  Per-point results are therefore stored by every lane
// (the same value to the same address).
__device__ inline int next_item(int* queue, int lane) {
    const int v = atomicAdd(queue, lane == 0 ? 1 : 0);
    return __builtin_amdgcn_readfirstlane(v);
}

// Wavefront sum (every lane gets it).
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// In-place Gauss-Jordan inverse with partial pivoting (largest |re| + |im|
// in the column); the row exchanges are undone as column exchanges at the end.
__device__ __noinline__ double2 inv8(Lds& s, int lane, double2 m) {
    const int r = lane >> 3, c = lane & 7;
    s.a[lane] = m;
    __syncthreads();
    for (int k = 0; k < SB; ++k) {
        int p = k;
        double best = -1.0;
        for (int i = k; i < SB; ++i) {
            const double2 v = s.a[i * SB + k];
            const double mg = fabs(v.x) + fabs(v.y);
            if (mg > best) { best = mg; p = i; }
        }
        s.perm[k] = p;                        // every lane writes the same value
        if (!(best > 0.0)) s.bad |= (best == 0.0) ? ST_SINGULAR : ST_NONFINITE;
        double2 x = s.a[lane];
        if (p != k) {
            if (r == k) x = s.a[p * SB + c];
            else if (r == p) x = s.a[k * SB + c];
        }
        __syncthreads();
        s.a[lane] = x;
        __syncthreads();
        const double2 piv = s.a[k * SB + k];
        const double den = piv.x * piv.x + piv.y * piv.y;
        const double2 ip = make_double2(piv.x / den, -piv.y / den);
        const double2 ak = s.a[r * SB + k], kc = s.a[k * SB + c];
        double2 y;
        if (r == k && c == k) y = ip;
        else if (r == k) y = cmul(kc, ip);
        else if (c == k) y = cmul(make_double2(-ak.x, -ak.y), ip);
        else y = x - cmul(ak, cmul(kc, ip));
        __syncthreads();
        s.a[lane] = y;
        __syncthreads();
    }
    // A^-1 = X S_{n-1} ... S_0 : column exchanges in reverse order
    for (int k = SB - 1; k >= 0; --k) {
        const int p = s.perm[k];
        double2 x = s.a[lane];
        if (p != k) {
            if (c == k) x = s.a[r * SB + p];
            else if (c == p) x = s.a[r * SB + k];
        }
        __syncthreads();
        s.a[lane] = x;
        __syncthreads();
    }
    const double2 out = s.a[lane];
    __syncthreads();
    return out;
}

}  // namespace

__global__ __launch_bounds__(SL) void rgf_small_kernel(SmallArgs a) {
    __shared__ Lds s;
    const int lane = threadIdx.x;
    const int r = lane >> 3, c = lane & 7;
    const int n = a.n;
    const bool in = r < n && c < n;
    const long long nn = (long long)n * n;
    s.bad = 0;
    for (;;) {
        const int q = next_item(a.queue, lane);
        if (q >= a.np) break;
        const int p = a.ps.p0 + q;
        const int4 d = a.ps.desc[p];
        const int ik = d.y, ie = d.z, N = d.w;
        const long long off = a.ps.slab_off[d.x];
        const double E = a.energy[ie];
        const double fL = fermi_s(E, a.muL, a.kT), fR = fermi_s(E, a.muR, a.kT);
        const long long lo = ((long long)ik * a.n_e + ie) * nn;
        const double2 zero = make_double2(0.0, 0.0);
        const double2 sLrc = in ? a.sigL[lo + r * n + c] : zero, sLcr = in ? a.sigL[lo + c * n + r] : zero;
        const double2 sRrc = in ? a.sigR[lo + r * n + c] : zero, sRcr = in ? a.sigR[lo + c * n + r] : zero;
        // Gamma = i (Sigma - Sigma^dagger); Sigma^< = i f Gamma = -f (Sigma - Sigma^dagger)
        const double2 dL = make_double2(sLrc.x - sLcr.x, sLrc.y + sLcr.y);
        const double2 dR = make_double2(sRrc.x - sRcr.x, sRrc.y + sRcr.y);
        const double2 gamL = make_double2(-dL.y, dL.x), gamR = make_double2(-dR.y, dR.x);
        auto hup = [&](long long gs) -> double2 {   // element of H_{gs, gs+1} (block-diagonal part only)
            if (!in || r / a.ub != c / a.ub) return zero;
            return a.hup[ik * a.hup_k + gs * nn + r * n + c];
        };
        double2* gq = a.gst + q * a.sst;
        double2* glq = a.glst + q * a.sst;
        const bool wantT = a.trans != nullptr;

        // ---- forward sweep
        double2 g = zero, gl = zero, C = zero;
        for (int i = 0; i < N; ++i) {
            const long long gs = off + i;
            double2 m;
            if (in) {
                const double2 h = a.hdiag[ik * a.hdiag_k + gs * nn + r * n + c];
                m = make_double2(-h.x, -h.y);
                if (r == c) {
                    m.x += E - (a.v ? a.v[gs * n + r] : 0.0);
                    m.y += a.eta;
                    if (a.scatR) { const double2 sc = a.scatR[((long long)ie * a.total + gs) * n + r]; m = m - sc; }
                }
                if (i == 0) m = m - sLrc;
                if (i == N - 1) m = m - sRrc;
            } else {
                m = make_double2(r == c ? 1.0 : 0.0, 0.0);
            }
            double2 sg = zero;   // Sigma^<_i
            if (in) {
                if (r == c) {
                    if (a.scatL) sg = sg + a.scatL[((long long)ie * a.total + gs) * n + r];
                    if (a.eta_fill) sg.y += 2.0 * a.eta * fL;
                }
                if (i == 0) sg = sg + make_double2(-fL * dL.x, -fL * dL.y);
                if (i == N - 1) sg = sg + make_double2(-fR * dR.x, -fR * dR.y);
            }
            double2 u = zero;
            if (i > 0) {
                u = hup(gs - 1);                                   // H_{i-1,i}
                m = m - mm(s, lane, u, mm(s, lane, g, u, false, false), true, false);
                sg = sg + mm(s, lane, u, mm(s, lane, gl, u, false, false), true, false);
            }
            g = inv8(s, lane, m);
            gl = anti_herm(s, lane, mm(s, lane, mm(s, lane, g, sg, false, false), g, false, true));
            if (in) { gq[i * nn + r * n + c] = g; glq[i * nn + r * n + c] = gl; }
            if (wantT) C = (i == 0) ? g : mm(s, lane, g, mm(s, lane, u, C, true, false), false, false);
        }

        // ---- backward sweep; slab N-1 is its own fully connected block
        double2 G = g, GL = gl;
        for (int i = N - 1; i >= 0; --i) {
            if (i < N - 1) {
                const long long gs = off + i;
                const double2 gi = in ? gq[i * nn + r * n + c] : make_double2(r == c ? 1.0 : 0.0, 0.0);
                const double2 gli = in ? glq[i * nn + r * n + c] : zero;
                const double2 u = hup(gs);                          // H_{i,i+1}
                const double2 L = mm(s, lane, gi, u, false, false);
                const double2 P = mm(s, lane, L, G, false, false);
                const double2 R = mm(s, lane, u, gi, true, false);
                const double2 Q = mm(s, lane, u, gli, true, false);
                const double2 T = mm(s, lane, P, Q, false, false);
                const double2 W = mm(s, lane, L, GL, false, false);
                // G^<_{i+1,i} = G_{i+1} H_{i+1,i} g^<_i + G^<_{i+1} L^dagger; j_i = 2 Re Tr[H_{i,i+1} G^<_{i+1,i}]
                const double2 Y = mm(s, lane, G, Q, false, false) + mm(s, lane, GL, L, false, true);
                const double2 Yt = transposed(s, lane, Y);
                const double j = 2.0 * wave_sum(u.x * Yt.x - u.y * Yt.y);
                if (a.bond) a.bond[(long long)p * a.slab_stride + i] = j;     // same value from every lane
                const double2 Tt = transposed(s, lane, T);
                G = gi + mm(s, lane, P, R, false, false);
                GL = anti_herm(s, lane, gli + mm(s, lane, W, L, false, true) + T -
                                            make_double2(Tt.x, -Tt.y));
            }
            const double2 Gt = transposed(s, lane, G);
            const double2 GG = GL + G - make_double2(Gt.x, -Gt.y);   // G^> = G^< + G - G^dagger
            if (in) {
                const long long o = (long long)p * a.slab_stride + i;
                if (a.full) {
                    if (a.outR) a.outR[o * nn + r * n + c] = G;
                    if (a.outL) a.outL[o * nn + r * n + c] = GL;
                    if (a.outG) a.outG[o * nn + r * n + c] = GG;
                } else if (r == c) {
                    if (a.outR) a.outR[o * n + r] = G;
                    if (a.outL) a.outL[o * n + r] = GL;
                    if (a.outG) a.outG[o * n + r] = GG;
                }
            }
        }
        if (wantT) {
            // T = Tr[Gamma_R C Gamma_L C^dagger], C = G_{N,1}
            const double2 X1 = mm(s, lane, gamR, C, false, false);
            const double2 X2 = mm(s, lane, gamL, C, false, true);
            const double2 X2t = transposed(s, lane, X2);
            const double t = wave_sum(X1.x * X2t.x - X1.y * X2t.y);
            a.trans[p] = t;                                               // same value from every lane
        }
    }
    __syncthreads();
    if (lane == 0 && s.bad) raise_status(a.status, s.bad);
}

// Matrix 1-norm (largest column sum of |x|) and infinity norm (largest row
// sum) of the block whose element (l / 8, l % 8) lane l holds.
__device__ inline double norm1_8(double2 x) {
    double v = hypot(x.x, x.y);
#pragma unroll
    for (int o = 8; o < SL; o <<= 1) v += __shfl_xor(v, o);     // column sums
#pragma unroll
    for (int o = 1; o < SB; o <<= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ inline double norminf_8(double2 x) {
    double v = hypot(x.x, x.y);
#pragma unroll
    for (int o = 1; o < SB; o <<= 1) v += __shfl_xor(v, o);     // row sums
#pragma unroll
    for (int o = 8; o < SL; o <<= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Sancho-Rubio decimation of one (k, E) point per wavefront, iterated to
// convergence inside the kernel (no host round trip per decimation step):
// the same steps and stopping rule as the batched lead path.
__global__ __launch_bounds__(SL) void sr_small_kernel(SrSmallArgs a) {
    __shared__ Lds s;
    const int lane = threadIdx.x;
    const int r = lane >> 3, c = lane & 7;
    const int n = a.n;
    const bool in = r < n && c < n;
    const long long nn = (long long)n * n;
    const double2 zero = make_double2(0.0, 0.0);
    const bool dual = a.sigma2 != nullptr;
    s.bad = 0;
    for (;;) {
        const int f = next_item(a.queue, lane);
        if (f >= a.total) break;
        const int ik = f / a.n_e, ie = f - ik * a.n_e;
        const double E = a.energy[ie];
        const long long kb = (long long)ik * nn;
        const double2 h = in ? a.h00[kb + r * n + c] : zero;
        const double2 h01 = in ? a.h01[kb + r * n + c] : zero;
        const double2 h01t = in ? a.h01[kb + c * n + r] : zero;
        double2 eps_s = h, eps = h, eps_d = h;
        double2 al = h01, be = cconj(h01t);
        const double ref = norm1_8(h01), ref2 = norm1_8(cconj(h01t));   // ||h01||_1, ||h01^dagger||_1
        auto zminus = [&](double2 x) -> double2 {   // z I - x (identity on the padding)
            if (!in) return make_double2(r == c ? 1.0 : 0.0, 0.0);
            double2 m = make_double2(-x.x, -x.y);
            if (r == c) { m.x += E; m.y += a.eta; }
            return m;
        };
        int it1 = 0, it2 = 0;
        bool done = false;
        for (int it = 1; it <= a.max_iter && !done; ++it) {
            const double2 g = inv8(s, lane, zminus(eps));
            const double2 X1 = mm(s, lane, al, g, false, false);
            const double2 X2 = mm(s, lane, be, g, false, false);
            const double2 t1 = mm(s, lane, X1, be, false, false);
            eps_s = eps_s + t1;
            eps = eps + t1;
            const double2 t2 = mm(s, lane, X2, al, false, false);
            if (dual) eps_d = eps_d + t2;
            eps = eps + t2;
            const double2 al2 = mm(s, lane, X1, al, false, false);
            be = mm(s, lane, X2, be, false, false);
            al = al2;
            const double sum = norm1_8(al) + norm1_8(be);
            if (it1 >= 0) it1 = sum < a.tol * ref ? -it : it;
            if (dual && it2 >= 0) it2 = sum < a.tol * ref2 ? -it : it;
            done = __builtin_amdgcn_readfirstlane((int)(it1 < 0 && (!dual || it2 < 0))) != 0;
        }
        atomicAdd(a.noconv, (!done && lane == 0) ? 1 : 0);
        // Sigma = tau (z - eps_s)^-1 tau^dagger (and the dual surface's)
        for (int side = 0; side < (dual ? 2 : 1); ++side) {
            const double2* tin = side ? a.tau2 : a.tau;
            const double2 t = in ? tin[kb + r * n + c] : zero;
            const double2 gs = inv8(s, lane, zminus(side ? eps_d : eps_s));
            const double2 sig = mm(s, lane, mm(s, lane, t, gs, false, false), t, false, true);
            double2* out = side ? a.sigma2 : a.sigma;
            if (in) out[(long long)f * nn + r * n + c] = sig;
        }
        if (a.iters) a.iters[f] = it1 < 0 ? -it1 : it1;                    // same value from every lane
        if (dual && a.iters2) a.iters2[f] = it2 < 0 ? -it2 : it2;
    }
    __syncthreads();
    if (lane == 0 && s.bad) raise_status(a.status, s.bad);
}

hipError_t sr_small_launch(hipStream_t st, const SrSmallArgs& a, int grid) {
    hipLaunchKernelGGL(sr_small_kernel, dim3(grid), dim3(SL), 0, st, a);
    return hipGetLastError();
}

hipError_t small_launch(hipStream_t st, const SmallArgs& a, int grid) {
    hipLaunchKernelGGL(rgf_small_kernel, dim3(grid), dim3(SL), 0, st, a);
    return hipGetLastError();
}

}  // namespace negf
