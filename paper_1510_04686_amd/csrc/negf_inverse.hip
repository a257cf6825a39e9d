// Batched dense complex block inverse: blocked Gauss-Jordan with partial
// (row) pivoting, one independent matrix per batch point.
//
// The paper inverts each slab block with LAPACK's zgesv (Sec. "System and
// environment").  Here the inverse is organised for matrix cores: for every
// panel of nbk columns,
//   1. gj_panel  (one workgroup per point): loads the n x nbk column panel into
//      LDS, picks the largest-magnitude pivot of each column among the rows not
//      yet used, swaps rows, and runs the in-place Gauss-Jordan eliminations on
//      the panel only.  The panel then holds the columns E_K of the elimination
//      transform; the pivot rows of the old matrix are copied out.
//   2. gj_update (64 x 64 tiles on MFMA): every other column is transformed
//      at once, X'[r][c] = X[src(r)][c] + sum_j (E[r][j] - delta) Xpiv[j][c],
//      a rank-nbk product, written out of place (ping-pong buffers).
// After the last panel the column permutation of the recorded row swaps is
// applied while writing the result, giving A^-1 = X P.
#include "negf_internal.hpp"
#include "negf_mfma.hpp"

namespace negf {

constexpr int NBMAX = 16;          // widest panel
constexpr int PANEL_LDS = 150 * 1024;

struct PanelArgs {
    const void* X; long long sX;   // current matrix
    void* E;                       // [np][n][NBMAX]
    void* Prow;                    // [np][NBMAX][n]
    int* rowsrc;                   // [np][n]
    int* piv;                      // [np][n]
    int* coldst;                   // [np][n]
    int n, k0, nbk, np, last;
    Active act;
    int* status;
};

template <typename R>
__global__ __launch_bounds__(256) void gj_panel(PanelArgs a) {
    typedef cplx<R> C;
    extern __shared__ __align__(16) unsigned char smem[];
    const int q = blockIdx.x;
    if (q >= a.np || !a.act(q)) return;
    const int n = a.n, k0 = a.k0, nbk = a.nbk, tid = threadIdx.x;
    C* P = reinterpret_cast<C*>(smem);                 // column-major panel P[j * n + r]
    int* rsrc = reinterpret_cast<int*>(P + (size_t)nbk * n);
    __shared__ C rowc[NBMAX];
    __shared__ R red_v[4];
    __shared__ int red_i[4];
    __shared__ int sh_piv[NBMAX];
    __shared__ int sh_bad;

    const C* X = reinterpret_cast<const C*>(a.X) + q * a.sX;
    for (int idx = tid; idx < n * nbk; idx += 256) {
        int r = idx / nbk, j = idx - r * nbk;
        P[j * n + r] = X[(long long)r * n + k0 + j];
    }
    for (int r = tid; r < n; r += 256) rsrc[r] = r;
    if (tid == 0) sh_bad = 0;
    __syncthreads();

    for (int j = 0; j < nbk; ++j) {
        const int c = k0 + j;
        // (a) pivot: largest |re| + |im| in column j among rows c..n-1 (ties: lowest row)
        R best = (R)-1;
        int bi = n;
        for (int r = c + tid; r < n; r += 256) {
            C v = P[j * n + r];
            R m = fabs(v.x) + fabs(v.y);
            if (m > best) { best = m; bi = r; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            R ob = __shfl_xor(best, off);
            int oi = __shfl_xor(bi, off);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if ((tid & 63) == 0) { red_v[tid >> 6] = best; red_i[tid >> 6] = bi; }
        __syncthreads();
        if (tid == 0) {
            R b = red_v[0];
            int i = red_i[0];
            for (int w = 1; w < 4; ++w)
                if (red_v[w] > b || (red_v[w] == b && red_i[w] < i)) { b = red_v[w]; i = red_i[w]; }
            if (!(b > (R)0)) { sh_bad |= (b == (R)0) ? ST_SINGULAR : ST_NONFINITE; i = c; }
            else if (!isfinite(b)) sh_bad |= ST_NONFINITE;
            sh_piv[j] = i;
            int t = rsrc[c]; rsrc[c] = rsrc[i]; rsrc[i] = t;
        }
        __syncthreads();
        const int pv = sh_piv[j];
        // (b) swap rows c and pv of the panel
        if (pv != c && tid < nbk) {
            C t = P[tid * n + c]; P[tid * n + c] = P[tid * n + pv]; P[tid * n + pv] = t;
        }
        __syncthreads();
        // (c) scaled pivot row
        if (tid < nbk) {
            C p = P[j * n + c];
            R d = p.x * p.x + p.y * p.y;
            C inv; inv.x = p.x / d; inv.y = -p.y / d;
            rowc[tid] = (tid == j) ? inv : cmul(P[tid * n + c], inv);
        }
        __syncthreads();
        // (d) eliminate column j from every other row
        for (int r = tid; r < n; r += 256) {
            if (r == c) {
                for (int jj = 0; jj < nbk; ++jj) P[jj * n + r] = rowc[jj];
            } else {
                C f = P[j * n + r];
                for (int jj = 0; jj < nbk; ++jj) {
                    C v = (jj == j) ? C{0, 0} : P[jj * n + r];
                    C w = rowc[jj];
                    v.x -= f.x * w.x - f.y * w.y;
                    v.y -= f.x * w.y + f.y * w.x;
                    P[jj * n + r] = v;
                }
            }
        }
        __syncthreads();
    }

    C* E = reinterpret_cast<C*>(a.E) + (long long)q * n * NBMAX;
    for (int idx = tid; idx < n * nbk; idx += 256) {
        int r = idx / nbk, j = idx - r * nbk;
        E[r * NBMAX + j] = P[j * n + r];
    }
    C* Pr = reinterpret_cast<C*>(a.Prow) + (long long)q * NBMAX * n;
    for (int idx = tid; idx < n * nbk; idx += 256) {
        int j = idx / n, col = idx - j * n;
        Pr[j * n + col] = X[(long long)rsrc[k0 + j] * n + col];
    }
    int* rs = a.rowsrc + (long long)q * n;
    for (int r = tid; r < n; r += 256) rs[r] = rsrc[r];
    int* pg = a.piv + (long long)q * n;
    if (tid < nbk) pg[k0 + tid] = sh_piv[tid];
    if (tid == 0 && sh_bad) raise_status(a.status, sh_bad);

    if (a.last) {
        // Column permutation of the final result: A^-1 = X S_{n-1} ... S_0.
        __syncthreads();
        int* src = rsrc;   // reuse
        for (int r = tid; r < n; r += 256) src[r] = r;
        __syncthreads();
        if (tid == 0) {
            for (int c = n - 1; c >= 0; --c) {
                int p = (c >= k0) ? sh_piv[c - k0] : pg[c];
                int t = src[c]; src[c] = src[p]; src[p] = t;
            }
        }
        __syncthreads();
        int* cd = a.coldst + (long long)q * n;
        for (int j = tid; j < n; j += 256) cd[src[j]] = j;
    }
}

struct UpdArgs {
    const void* X; long long sX;   // current matrix
    void* Y; long long sY;         // next matrix (or the destination on the last panel)
    const void* E; const void* Prow;
    const int* rowsrc; const int* coldst;
    int n, k0, nbk, np, last;
    Active act;
};

template <typename R>
__global__ __launch_bounds__(256) void gj_update(UpdArgs a) {
    typedef cplx<R> C;
    __shared__ R Es[2][BK][LP];
    __shared__ R Ps[2][BK][LP];
    const int n = a.n;
    const int tiles = (n + BM - 1) / BM;
    const int tpp = tiles * tiles;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int q = lid / tpp;
    if (q >= a.np || !a.act(q)) return;
    const int t = lid - q * tpp;
    const int m0 = (t / tiles) * BM, n0 = (t % tiles) * BM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k0 = a.k0, nbk = a.nbk;
    const C* E = reinterpret_cast<const C*>(a.E) + (long long)q * n * NBMAX;
    const C* Pr = reinterpret_cast<const C*>(a.Prow) + (long long)q * NBMAX * n;
    // Ecoef tile: rows m0.., k = 0..15 (pattern X); Prow tile: k rows, cols n0.. (pattern Y)
    {
        int o = tid >> 2, k = (tid & 3) * 4, row = m0 + o;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            C v{0, 0};
            if (row < n && k + j < nbk) {
                v = E[(long long)row * NBMAX + k + j];
                if (row == k0 + k + j) v.x -= (R)1;
            }
            Es[0][k + j][o] = v.x;
            Es[1][k + j][o] = v.y;
        }
        int kk = tid >> 4, oc = (tid & 15) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            C v{0, 0};
            int col = n0 + oc + j;
            if (kk < nbk && col < n) v = Pr[(long long)kk * n + col];
            Ps[0][kk][oc + j] = v.x;
            Ps[1][kk][oc + j] = v.y;
        }
    }
    __syncthreads();
    const int wm = wave >> 1, wn = wave & 1;
    const int rowbase = m0 + wm * 32, colbase = n0 + wn * 32;
    const int nmi = rowbase >= n ? 0 : (rowbase + 16 >= n ? 1 : 2);
    const int nnj = colbase >= n ? 0 : (colbase + 16 >= n ? 1 : 2);
    typename MF<R>::V cr[2][2], ci[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) { cr[x][y][r] = 0; ci[x][y][r] = 0; }
    if (nmi == 2 && nnj == 2) mma_slice<R, 2, 2>(Es, Ps, lane, wm, wn, cr, ci);
    else if (nmi == 2 && nnj == 1) mma_slice<R, 2, 1>(Es, Ps, lane, wm, wn, cr, ci);
    else if (nmi == 1 && nnj == 2) mma_slice<R, 1, 2>(Es, Ps, lane, wm, wn, cr, ci);
    else if (nmi == 1 && nnj == 1) mma_slice<R, 1, 1>(Es, Ps, lane, wm, wn, cr, ci);

    const C* X = reinterpret_cast<const C*>(a.X) + q * a.sX;
    C* Y = reinterpret_cast<C*>(a.Y) + q * a.sY;
    const int* rs = a.rowsrc + (long long)q * n;
    const int* cd = a.coldst + (long long)q * n;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
        if (mi >= nmi) break;
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
            if (nj >= nnj) break;
            const int col = colbase + nj * 16 + (lane & 15);
            const int ocol = (a.last && col < n) ? cd[col] : col;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rowbase + mi * 16 + out_row<R>(lane, r);
                if (row < n && col < n) {
                    C v;
                    if (col >= k0 && col < k0 + nbk) {
                        v = E[(long long)row * NBMAX + (col - k0)];
                    } else {
                        v = X[(long long)rs[row] * n + col];
                        v.x += cr[mi][nj][r];
                        v.y += ci[mi][nj][r];
                    }
                    Y[(long long)row * n + ocol] = v;
                }
            }
        }
    }
}

template <typename R>
static hipError_t inverse_typed(hipStream_t s, void* src, long long s_src, void* dst, long long s_dst,
                                int n, int np, const Active& act, const InvWork& w) {
    typedef cplx<R> C;
    int nbk_max = (int)((PANEL_LDS - n * sizeof(int)) / ((size_t)n * sizeof(C)));
    if (nbk_max > NBMAX) nbk_max = NBMAX;
    if (nbk_max < 1) return hipErrorInvalidValue;
    const int tiles = (n + BM - 1) / BM;
    void* cur = src;
    void* other = w.pa;
    long long s_cur = s_src, s_other = (long long)n * n;
    for (int k0 = 0; k0 < n; k0 += nbk_max) {
        const int nbk = (n - k0 < nbk_max) ? (n - k0) : nbk_max;
        const int last = (k0 + nbk == n);
        PanelArgs pa{cur, s_cur, w.E, w.Prow, w.rowsrc, w.piv, w.coldst, n, k0, nbk, np, last, act, w.status};
        size_t lds = (size_t)nbk * n * sizeof(C) + (size_t)n * sizeof(int);
        hipLaunchKernelGGL(gj_panel<R>, dim3(np), dim3(256), lds, s, pa);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        UpdArgs ua{cur, s_cur, last ? dst : other, last ? s_dst : s_other, w.E, w.Prow, w.rowsrc, w.coldst,
                   n, k0, nbk, np, last, act};
        hipLaunchKernelGGL(gj_update<R>, dim3((unsigned)((long long)np * tiles * tiles)), dim3(256), 0, s, ua);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        void* t = cur; cur = other; other = t;
        long long ts = s_cur; s_cur = s_other; s_other = ts;
    }
    return hipSuccess;
}

hipError_t inverse_launch(hipStream_t s, int dt, void* src, long long s_src, void* dst, long long s_dst,
                          int n, int np, const Active& act, const InvWork& w) {
    if (np <= 0) return hipSuccess;
    if (dt == DT_C128) return inverse_typed<double>(s, src, s_src, dst, s_dst, n, np, act, w);
    return inverse_typed<float>(s, src, s_src, dst, s_dst, n, np, act, w);
}

hipError_t inverse_init() {
    hipError_t e = hipFuncSetAttribute((const void*)gj_panel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       PANEL_LDS + 4096);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)gj_panel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               PANEL_LDS + 4096);
}

}  // namespace negf
