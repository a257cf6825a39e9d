// Batched dense complex block inverse: blocked Gauss-Jordan with partial
// (row) pivoting, one independent matrix per batch point.
//
// The paper inverts each slab block with LAPACK's zgesv (Sec. "System and
// environment").  Here the inverse is organised for matrix cores: for every
// panel of nbk (<= 32) columns,
//   1. gj_panel  (one workgroup per point): the n x nbk column panel lives in
//      registers, rows spread over the threads.  Per column: the largest
//      |re| + |im| among the rows not yet used is the pivot, the pivot row and
//      the row it replaces are exchanged through LDS, and the Gauss-Jordan
//      elimination is applied to every row.  The panel is kept rotated (the
//      column being eliminated always sits in register 0 and the transform
//      column it produces is appended at the end), so all register indices are
//      compile-time constants.  Two barriers per column.  Output: the columns
//      E_K of the elimination transform and the pivot rows of the old matrix.
//   2. gj_update (64 x 64 tiles on MFMA): every other column is transformed at
//      once, X'[r][c] = X[src(r)][c] + sum_j (E[r][j] - delta) Xpiv[j][c], a
//      rank-nbk product, written out of place (ping-pong buffers).
// After the last panel the column permutation of the recorded row swaps is
// applied while writing the result, giving A^-1 = X P.
//
// Blocks wider than the outer panel width W (a tuning choice, a multiple of
// 32) use two levels: inside an outer panel of W columns the inner steps
// update only that panel (a narrow n x W copy), and the rest of the matrix
// receives the composite transform of the outer panel in one rank-W update.  Because Gauss-Jordan
// transforms a column using only that column and the panel's transform, the
// outer panel's columns evolve exactly as in the one-level scheme; the other
// columns receive the same composite transform in one pass instead of
// W / nbk passes, which cuts the full-matrix HBM sweeps by that factor.
#include "negf_internal.hpp"
#include "negf_mfma.hpp"

namespace negf {

constexpr int NBMAX = 32;          // widest panel (E / pivot-row buffers are sized for it)

struct PanelArgs {
    const void* X; long long sX;   // current matrix: global columns [xcol0, ..) with row stride ldX
    int ldX, xcol0;
    void* E;                       // [np][n][NBMAX]
    void* Prow;                    // [np][NBMAX][pnc]: pivot rows over global columns [pc0, pc0 + pnc)
    int pc0, pnc;
    int* rowsrc;                   // [np][n]
    int* piv;                      // [np][n]
    int* coldst;                   // [np][n]
    int* comp;                     // [np][n] composite row source over an outer panel, or NULL
    int comp_first;                // first inner step of the outer panel
    int* comp2;                    // [np][n] composite row source over a mid block, or NULL
    int comp2_first;               // first inner step of the mid block
    int n, k0, nbk, np, last;
    Active act;
    int* status;
    // fused mode: also apply the panel's transform to global columns [uc0, uc0 + unc)
    // and write them, with the panel's own columns, to Y (which may alias X)
    void* Y; long long sY; int ldY, ycol0, uc0, unc;
};

// Pivot search key: the bit pattern of a non-negative double is monotone in
// its value (NaN sorts above +inf), so one unsigned 64-bit maximum finds the
// largest candidate.  The 12 low mantissa bits carry 4095 - position, which
// breaks ties (to 2^-40 relative) toward the lowest position and keeps every
// candidate's key non-zero.
__device__ inline unsigned long long pivot_key(double m, int pos) {
    return ((unsigned long long)__double_as_longlong(m) & ~0xFFFull) | (unsigned long long)(4095 - pos);
}

template <int CTRL, int ROWM>
__device__ inline unsigned long long dpp64(unsigned long long x) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)x, CTRL, ROWM, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(x >> 32), CTRL, ROWM, 0xf, false);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// Maximum over a wavefront, returned uniformly: row shifts reduce each row of
// 16 lanes into its lane 15, two row broadcasts carry rows 0-1 and 2-3 into
// lane 63, which is read back.
__device__ inline unsigned long long wave_max_u64(unsigned long long x) {
    unsigned long long y;
    y = dpp64<0x111, 0xf>(x); x = x > y ? x : y;   // row_shr:1
    y = dpp64<0x112, 0xf>(x); x = x > y ? x : y;   // row_shr:2
    y = dpp64<0x114, 0xf>(x); x = x > y ? x : y;   // row_shr:4
    y = dpp64<0x118, 0xf>(x); x = x > y ? x : y;   // row_shr:8
    y = dpp64<0x142, 0xa>(x); x = x > y ? x : y;   // row_bcast:15 -> rows 1, 3
    y = dpp64<0x143, 0xc>(x); x = x > y ? x : y;   // row_bcast:31 -> rows 2, 3
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

// Compiler-only fence: the accumulators must hold their values here and no
// memory access moves across (emits no instruction).
template <typename C, int CW>
__device__ inline void pin_acc(C (&acc)[CW]) {
#pragma unroll
    for (int i = 0; i < CW; ++i) asm volatile("" : "+v"(acc[i].x), "+v"(acc[i].y) : : "memory");
}

// Rows stay in the thread that loaded them; a row exchange only swaps the
// positions two threads stand for (pos[]).  Per column: every thread offers
// its candidate key, a DPP maximum per wavefront and one LDS round across
// wavefronts pick the pivot, the pivot thread publishes its row and 1/p, and
// every row is eliminated with the same formula (the pivot row with f - 1 in
// place of f, which turns the update into the scaling by 1/p).
template <typename R, int NB, int RPT, int NT, bool FUSE>
__global__ __launch_bounds__(NT) void gj_panel(PanelArgs a) {
    typedef cplx<R> C;
    constexpr int NW = NT / 64;
    constexpr int CW = 8;                                // fused update: columns per chunk
    __shared__ C rowP[NB];
    __shared__ C sh_inv;
    __shared__ unsigned long long cand[NW];
    __shared__ int sh_piv[NB];
    __shared__ int sh_bad;
    __shared__ C Pch[FUSE ? NB : 1][FUSE ? CW : 1];      // fused: pivot rows of one chunk
    extern __shared__ int rsrc[];   // [n] position -> row of X (dynamic)
    const int q = blockIdx.x;
    if (q >= a.np || !a.act(q)) return;
    const int n = a.n, k0 = a.k0, nbk = a.nbk, tid = threadIdx.x, lane = tid & 63;
    const C* X = reinterpret_cast<const C*>(a.X) + q * a.sX;

    C v[RPT][NB];
    int pos[RPT];
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
        const int r = tid + NT * t;
        pos[t] = r;
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) {
            v[t][jj].x = 0; v[t][jj].y = 0;
            if (r < n && jj < nbk) v[t][jj] = X[(long long)r * a.ldX + (k0 - a.xcol0) + jj];
        }
    }
    for (int r = tid; r < n; r += NT) rsrc[r] = r;
    if (tid == 0) sh_bad = 0;
    __syncthreads();

    for (int j = 0; j < nbk; ++j) {
        const int c = k0 + j;
        unsigned long long key = 0;
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
            const int r = tid + NT * t;
            if (r < n && pos[t] >= c) {
                const unsigned long long k = pivot_key((double)(fabs(v[t][0].x) + fabs(v[t][0].y)), pos[t]);
                key = k > key ? k : key;
            }
        }
        key = wave_max_u64(key);
        if (lane == 0) cand[tid >> 6] = key;
        __syncthreads();                                           // B1
        unsigned long long best = cand[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) best = cand[w] > best ? cand[w] : best;
        const double b = __longlong_as_double((long long)(best & ~0xFFFull));
        int pv = 4095 - (int)(best & 0xFFFull);
        if (!(b > 0) || pv >= n) pv = c;    // zero / non-finite column: flagged below
        if (tid == 0) {
            if (!(b > 0)) sh_bad |= (b == 0) ? ST_SINGULAR : ST_NONFINITE;
            else if (!isfinite(b)) sh_bad |= ST_NONFINITE;
            sh_piv[j] = pv;
            int tmp = rsrc[c]; rsrc[c] = rsrc[pv]; rsrc[pv] = tmp;
        }
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
            if (tid + NT * t < n && pos[t] == pv) {
#pragma unroll
                for (int jj = 1; jj < NB; ++jj) rowP[jj] = v[t][jj];
                const C p = v[t][0];
                const R rd = (R)1 / (p.x * p.x + p.y * p.y);
                C inv; inv.x = p.x * rd; inv.y = -p.y * rd;
                sh_inv = inv;
            }
        }
        __syncthreads();                                           // B2
        const C inv = sh_inv;
        C g[RPT];
        bool isp[RPT];
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
            isp[t] = pos[t] == pv;
            C f = v[t][0];
            f.x -= isp[t] ? (R)1 : (R)0;
            g[t] = cmul(f, inv);
        }
        // v[jj - 1] = v[jj] - g w[jj] for jj = 1 .. NB-1, the pivot row read from LDS
        // in groups of 8 with the next group's reads in flight (LDS latency, not
        // the arithmetic, bounds this loop otherwise)
        constexpr int GW = 8;
        constexpr int NG = (NB - 1 + GW - 1) / GW;
        C wb[2][GW];
#pragma unroll
        for (int u = 0; u < GW; ++u) if (1 + u < NB) wb[0][u] = rowP[1 + u];
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            if (gi + 1 < NG) {
#pragma unroll
                for (int u = 0; u < GW; ++u) {
                    const int jj = 1 + (gi + 1) * GW + u;
                    if (jj < NB) wb[(gi + 1) & 1][u] = rowP[jj];
                }
            }
#pragma unroll
            for (int u = 0; u < GW; ++u) {
                const int jj = 1 + gi * GW + u;
                if (jj < NB) {
                    const C w = wb[gi & 1][u];
#pragma unroll
                    for (int t = 0; t < RPT; ++t) {
                        C o;
                        o.x = fma(-g[t].x, w.x, v[t][jj].x);
                        o.x = fma(g[t].y, w.y, o.x);
                        o.y = fma(-g[t].x, w.y, v[t][jj].y);
                        o.y = fma(-g[t].y, w.x, o.y);
                        v[t][jj - 1] = o;
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
            C e; e.x = -g[t].x + (isp[t] ? (R)1 : (R)0); e.y = -g[t].y;
            v[t][NB - 1] = e;
            pos[t] = isp[t] ? c : (pos[t] == c ? pv : pos[t]);
        }
    }

    int* pg = a.piv + (long long)q * n;
    if (tid < nbk) pg[k0 + tid] = sh_piv[tid];
    if (tid == 0 && sh_bad) raise_status(a.status, sh_bad);
    if (a.comp) {
        // composite row sources of the outer panel (and of the mid block):
        // comp'[p] = comp[rsrc[p]], starting from rsrc at the first inner step
        int* cm = a.comp + (long long)q * n;
        int* cm2 = a.comp2 ? a.comp2 + (long long)q * n : nullptr;
        int nv[RPT], nv2[RPT];
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
            const int r = tid + NT * t;
            nv[t] = (r < n) ? (a.comp_first ? rsrc[r] : cm[rsrc[r]]) : 0;
            nv2[t] = (r < n && cm2) ? (a.comp2_first ? rsrc[r] : cm2[rsrc[r]]) : 0;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
            const int r = tid + NT * t;
            if (r < n) cm[r] = nv[t];
            if (r < n && cm2) cm2[r] = nv2[t];
        }
    }

    if constexpr (FUSE) {
        // The transform columns are v[0][0 .. NB) (nbk == NB).  Write them in place of
        // the panel's columns, then update the other columns chunk by chunk:
        //   Y[p][col] = X[rsrc[p]][col] + sum_j (E[p][j] - delta(p, k0 + j)) X[rsrc[k0 + j]][col].
        C* Y = reinterpret_cast<C*>(a.Y) + q * a.sY;
        const int r = tid;
        const int p = pos[0];
        if (r < n) {
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) Y[(long long)p * a.ldY + (k0 - a.ycol0) + jj] = v[0][jj];
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) v[0][jj].x -= (p == k0 + jj) ? (R)1 : (R)0;
        }
        // Chunks of CW columns, skipping the panel itself; the next chunk's global reads
        // are issued before the current chunk's arithmetic.
        const int cend = a.uc0 + a.unc;
        auto next_chunk = [&](int cc) {
            cc += CW;
            if (cc >= k0 && cc < k0 + NB) cc = k0 + NB;
            return cc;
        };
        int cc = a.uc0;
        if (cc >= k0 && cc < k0 + NB) cc = k0 + NB;
        const int prow = tid / CW, pc2 = tid - (tid / CW) * CW;   // this thread's element of the pivot tile
        const bool pown = tid < NB * CW;
        C pv_n, xa_n[CW];
        auto fetch = [&](int c0) {
            pv_n.x = 0; pv_n.y = 0;
            if (pown && c0 + pc2 < cend) pv_n = X[(long long)rsrc[k0 + prow] * a.ldX + (c0 + pc2 - a.xcol0)];
#pragma unroll
            for (int c2 = 0; c2 < CW; ++c2) {
                xa_n[c2].x = 0; xa_n[c2].y = 0;
                if (r < n && c0 + c2 < cend) xa_n[c2] = X[(long long)rsrc[p] * a.ldX + (c0 + c2 - a.xcol0)];
            }
        };
        static_assert(NB * CW <= NT, "one pivot-tile element per thread");
        if (cc < cend) fetch(cc);
        while (cc < cend) {
            __syncthreads();                                        // Pch reuse
            if (pown) Pch[prow][pc2] = pv_n;
            C acc[CW];
#pragma unroll
            for (int c2 = 0; c2 < CW; ++c2) acc[c2] = xa_n[c2];
            const int cn = next_chunk(cc);
            if (cn < cend) fetch(cn);
            __syncthreads();                                        // every read of the chunk is done
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) {
                const C e = v[0][jj];
#pragma unroll
                for (int c2 = 0; c2 < CW; ++c2) {
                    const C w = Pch[jj][c2];
                    acc[c2].x = fma(e.x, w.x, acc[c2].x);
                    acc[c2].x = fma(-e.y, w.y, acc[c2].x);
                    acc[c2].y = fma(e.x, w.y, acc[c2].y);
                    acc[c2].y = fma(e.y, w.x, acc[c2].y);
                }
                // keep each row of pivot values next to its use: hoisting every LDS read of the
                // unrolled loop ahead of the arithmetic would exceed the register budget.  The
                // empty statement orders the LDS reads and pins the accumulators here.
                pin_acc<C, CW>(acc);
            }
            if (r < n) {
#pragma unroll
                for (int c2 = 0; c2 < CW; ++c2)
                    if (cc + c2 < cend) Y[(long long)p * a.ldY + (cc + c2 - a.ycol0)] = acc[c2];
            }
            cc = cn;
        }
    } else {
        // The transform columns sit in registers NB-nbk .. NB-1.
        C* E = reinterpret_cast<C*>(a.E) + (long long)q * n * NBMAX;
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
            const int r = tid + NT * t;
            if (r < n) {
#pragma unroll
                for (int pp = 0; pp < NB; ++pp)
                    if (pp >= NB - nbk) E[(long long)pos[t] * NBMAX + (pp - (NB - nbk))] = v[t][pp];
            }
        }
        __syncthreads();
        C* Pr = reinterpret_cast<C*>(a.Prow) + (long long)q * NBMAX * a.pnc;
        for (int idx = tid; idx < a.pnc * nbk; idx += NT) {
            int jr = idx / a.pnc, cc = idx - jr * a.pnc;
            Pr[(long long)jr * a.pnc + cc] = X[(long long)rsrc[k0 + jr] * a.ldX + (a.pc0 + cc - a.xcol0)];
        }
        int* rs = a.rowsrc + (long long)q * n;
        for (int r = tid; r < n; r += NT) rs[r] = rsrc[r];
    }

    if (a.last) {
        // Column permutation of the final result: A^-1 = X S_{n-1} ... S_0.
        __syncthreads();
        int* src = rsrc;   // reuse
        for (int r = tid; r < n; r += NT) src[r] = r;
        __syncthreads();
        if (tid == 0) {
            for (int cc = n - 1; cc >= 0; --cc) {
                int pp = (cc >= k0) ? sh_piv[cc - k0] : pg[cc];
                int tmp = src[cc]; src[cc] = src[pp]; src[pp] = tmp;
            }
        }
        __syncthreads();
        int* cd = a.coldst + (long long)q * n;
        for (int jr = tid; jr < n; jr += NT) cd[src[jr]] = jr;
    }
}

struct UpdArgs {
    const void* X; long long sX; int ldX, xcol0;   // current matrix (global columns from xcol0, row stride ldX)
    void* Y; long long sY; int ldY, ycol0;         // next matrix, same convention (full n x n when last)
    int c0, nc;                                    // global columns to produce
    const void* E; int ldE;                        // transform columns E[r][j], j < nbk (global column k0 + j)
    const void* Prow; int ldP, pc0;                // pivot rows [nbk][..] from global column pc0, or NULL:
                                                   // gathered as X[rowsrc[k0 + j]]
    const int* rowsrc; const int* coldst;
    int n, k0, nbk, np, last;
    Active act;
};

// Y[r][c] = X[rs(r)][c] + sum_j (E[r][j] - delta(r, k0 + j)) Prow[j][c] for c outside
// [k0, k0 + nbk), Y[r][c] = E[r][c - k0] inside; 64 x 64 output tiles, K in
// slices of BK, two slices staged in LDS at a time.
template <typename R>
__global__ __launch_bounds__(256) void gj_update(UpdArgs a) {
    typedef cplx<R> C;
    __shared__ R Es[2][2][BK][LP];   // [buffer][re/im][k][m]
    __shared__ R Ps[2][2][BK][LP];
    const int n = a.n;
    const int tm = (n + BM - 1) / BM, tn = (a.nc + BM - 1) / BM;
    const int tpp = tm * tn;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int q = lid / tpp;
    if (q >= a.np || !a.act(q)) return;
    const int t = lid - q * tpp;
    const int cend = a.c0 + a.nc;
    const int m0 = (t / tn) * BM, n0 = a.c0 + (t % tn) * BM;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k0 = a.k0, nbk = a.nbk;
    const int nsl = (nbk + BK - 1) / BK;
    const WaveTile wt = wave_tile(wave, n - m0, cend - n0);
    const int am0 = wt.am0, bn0 = wt.bn0, nmi = wt.nmi, nnj = wt.nnj;
    const int rowbase = m0 + am0, colbase = n0 + bn0;
    const C* X = reinterpret_cast<const C*>(a.X) + q * a.sX;
    const C* E = reinterpret_cast<const C*>(a.E) + (long long)q * n * a.ldE;
    const C* Pr = a.Prow ? reinterpret_cast<const C*>(a.Prow) + (long long)q * NBMAX * a.ldP : nullptr;
    const int* rs = a.rowsrc + (long long)q * n;
    const int ldX = a.ldX, xc = a.xcol0;
    // Row sources read ahead: the pivot row this thread loads in the next K slice (when
    // gathered from X) and the tile rows it gathers at the end, so no global read of
    // the matrix waits on an index read.
    const int pk = tid >> 4, poc = tid & 15;   // pivot-row columns poc + 16 j
    auto row_of = [&](int s) { const int kk = s * BK + pk; return (!Pr && kk < nbk) ? rs[k0 + kk] : 0; };
    int src_next = row_of(0);   // pivot-row source of the slice loaded next (read one slice ahead)
    int rsr[2][4];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = rowbase + mi * 16 + out_row<R>(lane, r);
            rsr[mi][r] = (row < n) ? rs[row] : 0;
        }
    // output columns (the final column permutation on the last update), read
    // here so that the epilogue's stores do not wait for them
    int ocols[2];
#pragma unroll
    for (int nj = 0; nj < 2; ++nj) {
        const int col = colbase + nj * 16 + (lane & 15);
        ocols[nj] = (a.last && col < cend) ? a.coldst[(long long)q * n + col] : col;
    }

    typename MF<R>::V cr[2][2], ci[2][2], cs[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) { cr[x][y][r] = 0; ci[x][y][r] = 0; cs[x][y][r] = 0; }
    // K slices double-buffered through LDS, the next slice's reads in flight during
    // the current slice's products.  E tile: rows m0.., k (pattern X); pivot-row
    // tile: k rows, cols n0.. (pattern Y).
    const int eo = tid >> 2, ek = (tid & 3) * 4, erow = m0 + eo;
    C re[4], rp[4];
    // The E reads use indices clamped into the block and are masked (and the
    // -delta applied) only when stored to LDS, after the slice's products: a
    // select on a loaded value would make each read wait before the next.
    const long long erow_off = (long long)min(erow, n - 1) * a.ldE;
    auto load = [&](int s) {
#pragma unroll
        for (int j = 0; j < 4; ++j) re[j] = E[erow_off + min(s * BK + ek + j, nbk - 1)];
        const int kk = s * BK + pk;
        const C* prow = nullptr;
        const int src = src_next;
        src_next = row_of(s + 1);
        if (kk < nbk) prow = Pr ? Pr + (long long)kk * a.ldP - a.pc0 : X + (long long)src * ldX - xc;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = n0 + poc + 16 * j;
            rp[j].x = 0; rp[j].y = 0;
            if (prow && col < cend) rp[j] = prow[col];
        }
    };
    auto store = [&](int b, int s) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int pc = poc + 16 * j;
            const int kk = s * BK + ek + j;
            const bool ok = erow < n && kk < nbk;
            const R ex = ok ? re[j].x - (erow == k0 + kk ? (R)1 : (R)0) : (R)0;
            Es[b][0][ek + j][swz(ek + j, eo)] = ex;
            Es[b][1][ek + j][swz(ek + j, eo)] = ok ? re[j].y : (R)0;
            Ps[b][0][pk][swz(pk, pc)] = rp[j].x;
            Ps[b][1][pk][swz(pk, pc)] = rp[j].y;
        }
    };
    auto mma = [&](int b) {
        if (nmi == 2 && nnj == 2) mma_slice<R, 2, 2>(Es[b], Ps[b], lane, am0, bn0, cr, ci, cs);
        else if (nmi == 2 && nnj == 1) mma_slice<R, 2, 1>(Es[b], Ps[b], lane, am0, bn0, cr, ci, cs);
        else if (nmi == 1 && nnj == 2) mma_slice<R, 1, 2>(Es[b], Ps[b], lane, am0, bn0, cr, ci, cs);
        else if (nmi == 1 && nnj == 1) mma_slice<R, 1, 1>(Es[b], Ps[b], lane, am0, bn0, cr, ci, cs);
    };
    // A tile whose columns all lie inside the panel's K range only copies the
    // transform columns: its products would be discarded (uniform per workgroup).
    const bool copy_only = n0 >= k0 && min(n0 + BM, cend) <= k0 + nbk;
    if (!copy_only) {
        load(0);
        store(0, 0);
        __syncthreads();
        for (int s = 0; s + 1 < nsl; ++s) {
            const int b = s & 1;
            load(s + 1);
            mma(b);
            store(b ^ 1, s + 1);
            __syncthreads();
        }
        mma((nsl - 1) & 1);
        finish_products<R>(cr, ci, cs);
    }

    // Epilogue, one 16-row block at a time: gather the old rows (or the transform
    // columns inside the K range) and write the new tile.  The gather selects
    // addresses, not loaded values (a lane outside the tile reads element 0 and
    // discards it), so the reads of a block are in flight together.
    C* Y = reinterpret_cast<C*>(a.Y) + q * a.sY;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
        if (mi >= nmi) break;
        C xo[2][4];
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
            const int col = colbase + nj * 16 + (lane & 15);
            const bool inK = col >= k0 && col < k0 + nbk;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rowbase + mi * 16 + out_row<R>(lane, r);
                const bool v = nj < nnj && row < n && col < cend;
                const C* src = !v ? X : (inK ? E + ((long long)row * a.ldE + (col - k0))
                                             : X + ((long long)rsr[mi][r] * ldX + (col - xc)));
                xo[nj][r] = *src;
            }
        }
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
            if (nj >= nnj) break;
            const int col = colbase + nj * 16 + (lane & 15);
            const bool inK = col >= k0 && col < k0 + nbk;
            const int ocol = ocols[nj];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rowbase + mi * 16 + out_row<R>(lane, r);
                if (row < n && col < cend) {
                    C v = xo[nj][r];
                    if (!inK) { v.x += cr[mi][nj][r]; v.y += ci[mi][nj][r]; }
                    Y[(long long)row * a.ldY + (ocol - a.ycol0)] = v;
                }
            }
        }
    }
}

struct PanelShape { int nb, rpt, nt; };

// Panel width, rows per thread and threads per workgroup for a block size n:
// the register panel (RPT x NB complex per thread) must stay inside the
// per-lane register budget of the occupancy the shape implies.
template <typename R> struct Shapes;
template <> struct Shapes<double> {
    static PanelShape get(int n) {
        if (n <= 512) return {32, 1, 512};
        if (n <= 1024) return {16, 2, 512};
        if (n <= 1536) return {16, 3, 512};
        return {8, 4, 512};   // up to 2048
    }
};
template <> struct Shapes<float> {
    static PanelShape get(int n) {
        if (n <= 256) return {32, 1, 256};
        if (n <= 512) return {32, 1, 512};
        if (n <= 1024) return {32, 2, 512};
        if (n <= 1536) return {32, 3, 512};
        return {16, 4, 512};  // up to 2048
    }
};

template <typename R>
static void launch_panel(hipStream_t s, const PanelShape& ps, int np, size_t lds, const PanelArgs& pa, bool fuse) {
#define NEGF_PANEL(NB_, RPT_, NT_)                                                                        \
    if (ps.nb == NB_ && ps.rpt == RPT_ && ps.nt == NT_) {                                                 \
        if constexpr (RPT_ == 1) {                                                                        \
            if (fuse) {                                                                                   \
                hipLaunchKernelGGL((gj_panel<R, NB_, RPT_, NT_, true>), dim3(np), dim3(NT_), lds, s, pa); \
                return;                                                                                   \
            }                                                                                             \
        }                                                                                                 \
        hipLaunchKernelGGL((gj_panel<R, NB_, RPT_, NT_, false>), dim3(np), dim3(NT_), lds, s, pa);        \
        return;                                                                                           \
    }
    if constexpr (sizeof(R) == 8) {
        NEGF_PANEL(32, 1, 512) NEGF_PANEL(16, 2, 512) NEGF_PANEL(16, 3, 512) NEGF_PANEL(8, 4, 512)
    } else {
        NEGF_PANEL(32, 1, 256) NEGF_PANEL(32, 1, 512) NEGF_PANEL(32, 2, 512) NEGF_PANEL(32, 3, 512)
        NEGF_PANEL(16, 4, 512)
    }
#undef NEGF_PANEL
}

template <typename R>
static hipError_t launch_update(hipStream_t s, const UpdArgs& ua) {
    const int tm = (ua.n + BM - 1) / BM, tn = (ua.nc + BM - 1) / BM;
    hipLaunchKernelGGL(gj_update<R>, dim3((unsigned)((long long)ua.np * tm * tn)), dim3(256), 0, s, ua);
    return hipGetLastError();
}

template <typename R>
static hipError_t inverse_typed(hipStream_t s, void* src, long long s_src, void* dst, long long s_dst,
                                int n, int np, const Active& act, const InvWork& w) {
    if (n > INV_NMAX) return hipErrorInvalidValue;
    const PanelShape ps = Shapes<R>::get(n);
    const size_t lds = (size_t)n * sizeof(int);
    const long long nn = (long long)n * n;
    void* cur = src;
    void* other = w.pa;
    long long s_cur = s_src, s_other = nn;
    const bool two = w.W > 0 && w.W % 32 == 0 && w.W <= INV_WMAX && n > w.W && w.N0 && w.N1 && w.comp;
    if (!two) {
        for (int k0 = 0; k0 < n; k0 += ps.nb) {
            const int nbk = (n - k0 < ps.nb) ? (n - k0) : ps.nb;
            const int last = (k0 + nbk == n);
            PanelArgs pa{cur, s_cur, n, 0, w.E, w.Prow, 0, n, w.rowsrc, w.piv, w.coldst, nullptr, 0, nullptr, 0,
                         n, k0, nbk, np, last, act, w.status, nullptr, 0, 0, 0, 0, 0};
            launch_panel<R>(s, ps, np, lds, pa, false);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            UpdArgs ua{cur, s_cur, n, 0, last ? dst : other, last ? s_dst : s_other, n, 0, 0, n,
                       w.E, NBMAX, w.Prow, n, 0, w.rowsrc, w.coldst, n, k0, nbk, np, last, act};
            e = launch_update<R>(s, ua);
            if (e != hipSuccess) return e;
            void* tp = cur; cur = other; other = tp;
            long long ts = s_cur; s_cur = s_other; s_other = ts;
        }
        return hipSuccess;
    }
    // three levels: mid blocks of Wm columns inside an outer panel (fused inner panels
    // with one row per thread only); the last mid block of each outer panel is fused
    // over the whole outer panel, the others get a rank-Wm update of the outer panel
    const bool three = w.Wm > 0 && w.Wm % 32 == 0 && w.comp2 && ps.rpt == 1 && ps.nb == 32;
    int Wk = w.W;
    for (int K0 = 0; K0 < n; K0 += Wk) {
        // a remainder narrower than half an outer panel joins the current one (one
        // full-matrix sweep less), as long as the widened panel fits its buffers
        Wk = (n - K0 < w.W) ? (n - K0) : w.W;
        const int rest = n - K0 - Wk;
        if (rest > 0 && 2 * rest < w.W && n - K0 <= INV_WMAX) Wk = n - K0;
        const int W = Wk;
        const int lastK = (K0 + W == n);
        const long long sN = (long long)n * W;
        // inner steps: the outer panel's columns, full matrix -> narrow copy.  A full-width
        // panel with one row per thread updates the other columns itself (in place once
        // the narrow copy exists); otherwise a separate update writes the other narrow buffer.
        const void* ncur = cur;
        long long s_ncur = s_cur;
        int ld_ncur = n, xc_ncur = 0;
        bool in_narrow = false;
        void* nbuf[2] = {w.N0, w.N1};
        int nb_i = 0;
        const int Wm = (three && w.Wm < W) ? w.Wm : W;
        for (int M0 = K0; M0 < K0 + W; M0 += Wm) {
            const bool last_mid = M0 + Wm >= K0 + W;
            const int Wmid = last_mid ? K0 + W - M0 : Wm;
            // the values the mid update transforms: the outer panel before this mid block
            const void* mold = ncur;
            const long long s_mold = s_ncur;
            const int ld_mold = ld_ncur, xc_mold = xc_ncur;
            // fused range of the inner panels: this mid block, or the whole outer panel
            const int uc0 = last_mid ? K0 : M0, unc = last_mid ? W : Wmid;
            for (int k0 = M0; k0 < M0 + Wmid; k0 += ps.nb) {
                const int nbk = (M0 + Wmid - k0 < ps.nb) ? (M0 + Wmid - k0) : ps.nb;
                const int last = (k0 + nbk == n);
                const bool fuse = ps.rpt == 1 && nbk == ps.nb;
                void* ydst = fuse && in_narrow ? const_cast<void*>(ncur) : nbuf[nb_i];
                PanelArgs pa{ncur, s_ncur, ld_ncur, xc_ncur, w.E, w.Prow, K0, W, w.rowsrc, w.piv, w.coldst,
                             w.comp, k0 == K0, last_mid ? nullptr : w.comp2, k0 == M0, n, k0, nbk, np, last, act,
                             w.status, ydst, sN, W, K0, uc0, unc};
                launch_panel<R>(s, ps, np, lds, pa, fuse);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) return e;
                if (!fuse) {
                    UpdArgs ua{ncur, s_ncur, ld_ncur, xc_ncur, ydst, sN, W, K0, K0, W,
                               w.E, NBMAX, w.Prow, W, K0, w.rowsrc, w.coldst, n, k0, nbk, np, 0, act};
                    e = launch_update<R>(s, ua);
                    if (e != hipSuccess) return e;
                }
                if (ydst == nbuf[nb_i]) nb_i ^= 1;
                ncur = ydst; s_ncur = sN; ld_ncur = W; xc_ncur = K0;
                in_narrow = true;
            }
            if (!last_mid) {
                // mid update: the mid block's composite transform on the rest of the outer
                // panel, from its values before the block; the block's own columns are
                // copied from the transform columns.  Out of place into the other buffer.
                const void* Emid = static_cast<const char*>(ncur) + (size_t)(M0 - K0) * sizeof(cplx<R>);
                void* ynext = nbuf[nb_i];
                UpdArgs ua{mold, s_mold, ld_mold, xc_mold, ynext, sN, W, K0, K0, W,
                           Emid, W, nullptr, 0, 0, w.comp2, w.coldst, n, M0, Wmid, np, 0, act};
                hipError_t e = launch_update<R>(s, ua);
                if (e != hipSuccess) return e;
                nb_i ^= 1;
                ncur = ynext; s_ncur = sN; ld_ncur = W; xc_ncur = K0;
            }
        }
        // outer update: every column from the matrix before the outer panel, the panel's
        // columns from the narrow copy; the composite row map gathers rows and pivot rows
        UpdArgs ua{cur, s_cur, n, 0, lastK ? dst : other, lastK ? s_dst : s_other, n, 0, 0, n,
                   ncur, W, nullptr, 0, 0, w.comp, w.coldst, n, K0, W, np, lastK, act};
        hipError_t e = launch_update<R>(s, ua);
        if (e != hipSuccess) return e;
        void* tp = cur; cur = other; other = tp;
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

hipError_t inverse_init() { return hipSuccess; }

}  // namespace negf
