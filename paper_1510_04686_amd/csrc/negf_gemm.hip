// Batched complex GEMM on CDNA4 matrix cores.
//
// Every slab step of the RGF recursions (g_i X, Y g_i^dagger, L G_{i+1},
// P R, ...) is a dense complex b x b x b product for each (sample, k, E)
// point of a batch.  One launch covers the whole batch: a 64 x 64 output tile
// of one point per 256-thread workgroup (4 wavefronts of 32 x 32), K staged
// through LDS in 16-wide double-buffered slices, split real/imaginary planes.
// A complex product is three real MFMA products (the 3M form) on
// v_mfma_f64_16x16x4f64 (FP64) or v_mfma_f32_16x16x4f32 (FP32).
#include <algorithm>

#include "negf_internal.hpp"
#include "negf_mfma.hpp"

namespace negf {

static_assert(BM == 64, "gemm_tiles() assumes 64-wide tiles");

// Products whose results are anti-Hermitian (the lesser functions) keep their
// diagonal -- the occupation the density reads -- in the imaginary part, where
// the 3M form's rounding bound u (|Ar| + |Ai|)(|Br| + |Bi|) is loose: they use
// four real products, whose imaginary part is bounded by u (|Ar||Bi| + |Ai||Br|).
template <int EPI> struct FourM { static constexpr bool value = EPI == EPI_STORE_AH || EPI == EPI_ADD_TTD_AH; };

template <typename Acc, bool FM>
__device__ inline void mma_tile(Acc (*As)[BK][LP], Acc (*Bs)[BK][LP], int lane, int am0, int bn0, int nmi, int nnj,
                                typename MF<Acc>::V (&cr)[2][2], typename MF<Acc>::V (&ci)[2][2],
                                typename MF<Acc>::V (&cs)[2][2]) {
    if (nmi == 2 && nnj == 2) mma_slice<Acc, 2, 2, FM>(As, Bs, lane, am0, bn0, cr, ci, cs);
    else if (nmi == 2 && nnj == 1) mma_slice<Acc, 2, 1, FM>(As, Bs, lane, am0, bn0, cr, ci, cs);
    else if (nmi == 1 && nnj == 2) mma_slice<Acc, 1, 2, FM>(As, Bs, lane, am0, bn0, cr, ci, cs);
    else if (nmi == 1 && nnj == 1) mma_slice<Acc, 1, 1, FM>(As, Bs, lane, am0, bn0, cr, ci, cs);
}

// Output tile t of one point: row-major over all tiles, or over the lower
// triangle (tj <= ti) for the anti-Hermitian epilogues.
template <bool AH>
__device__ inline void tile_of(int t, int tiles, int& ti, int& tj) {
    if (AH) {
        ti = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        tj = t - ti * (ti + 1) / 2;
    } else {
        ti = t / tiles;
        tj = t - ti * tiles;
    }
}

// Writes this wave's part of the finished tile (m0, n0) of point q.
template <typename TC, typename Acc, int EPI>
__device__ inline void gemm_epilogue(const GemmArgs& g, int q, int m0, int n0, const WaveTile& wt, int lane,
                                     const typename MF<Acc>::V (&cr)[2][2], const typename MF<Acc>::V (&ci)[2][2]) {
    constexpr bool AH = (EPI == EPI_STORE_AH || EPI == EPI_ADD_TTD_AH);
    const int n = g.n;
    const int rowbase = m0 + wt.am0, colbase = n0 + wt.bn0;
    TC* __restrict__ C = (TC*)g.C + q * g.sC;
    const TC* D = (const TC*)g.D + q * g.sD;
    const TC* T = (const TC*)g.T + q * g.sT;
    TC* C2 = (TC*)g.C2 + q * g.sC2;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
        if (mi >= wt.nmi) break;
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
            if (nj >= wt.nnj) break;
            const int col = colbase + nj * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rowbase + mi * 16 + out_row<Acc>(lane, r);
                if (row < n && col < n && !(AH && m0 == n0 && row < col)) {
                    const long long idx = (long long)row * n + col;
                    double vr = (double)cr[mi][nj][r], vi = (double)ci[mi][nj][r];
                    TC out;
                    if (EPI == EPI_STORE_AH) {
                        out.x = (row == col) ? 0.0 : vr; out.y = vi; C[idx] = out;
                    } else if (EPI == EPI_STORE) {
                        out.x = vr; out.y = vi; C[idx] = out;
                    } else if (EPI == EPI_ADD || EPI == EPI_SUB) {
                        TC d = D[idx];
                        double s = (EPI == EPI_ADD) ? 1.0 : -1.0;
                        out.x = (double)d.x + s * vr; out.y = (double)d.y + s * vi; C[idx] = out;
                    } else if (EPI == EPI_ADD_TTD || EPI == EPI_ADD_TTD_AH) {
                        TC d = D[idx], t1 = T[idx], t2 = T[(long long)col * n + row];
                        out.x = (double)d.x + vr + (double)t1.x - (double)t2.x;
                        out.y = (double)d.y + vi + (double)t1.y + (double)t2.y;
                        if (EPI == EPI_ADD_TTD_AH && row == col) out.x = 0.0;
                        C[idx] = out;
                    } else if (EPI == EPI_DUAL) {
                        TC c1 = C[idx], c2 = C2[idx];
                        out.x = (double)c1.x + vr; out.y = (double)c1.y + vi; C[idx] = out;
                        out.x = (double)c2.x + vr; out.y = (double)c2.y + vi; C2[idx] = out;
                    } else if (EPI == EPI_IMINUS) {
                        out.x = (row == col ? 1.0 : 0.0) - vr; out.y = -vi; C[idx] = out;
                    }
                    if (AH && row != col) {
                        TC m; m.x = -out.x; m.y = out.y;
                        C[(long long)col * n + row] = m;
                    }
                }
            }
        }
    }
}

template <typename TA, typename TB, typename TC, typename Acc, int OPA, int OPB, int EPI, int PF>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
    __shared__ Acc As[2][2][BK][LP];
    __shared__ Acc Bs[2][2][BK][LP];
    constexpr bool AH = (EPI == EPI_STORE_AH || EPI == EPI_ADD_TTD_AH);
    const int n = g.n;
    const int tiles = (n + BM - 1) / BM;
    const int tpp = AH ? tiles * (tiles + 1) / 2 : tiles * tiles;
    const int lid = xcd_remap(blockIdx.x, gridDim.x);
    const int q = lid / tpp;
    if (q >= g.np || !g.act(q)) return;
    const int t = lid - q * tpp;
    int ti, tj;
    tile_of<AH>(t, tiles, ti, tj);
    const int m0 = ti * BM, n0 = tj * BM;
    const TA* __restrict__ A = (const TA*)g.A + q * g.sA;
    const TB* __restrict__ B = (const TB*)g.B + q * g.sB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const WaveTile wt = wave_tile(wave, n - m0, n - n0);
    const int am0 = wt.am0, bn0 = wt.bn0, nmi = wt.nmi, nnj = wt.nnj;

    typename MF<Acc>::V cr[2][2], ci[2][2], cs[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) { cr[a][b][r] = 0; ci[a][b][r] = 0; cs[a][b][r] = 0; }

    // op(A) slice: OPA = N -> rows m, contiguous k (pattern X); C -> rows k (pattern Y)
    // op(B) slice: OPB = N -> rows k (pattern Y); C -> rows n, contiguous k (pattern X)
    constexpr bool AK = (OPA == OP_C);
    constexpr bool BKR = (OPB == OP_N);
    const int nkt = (n + BK - 1) / BK;
    if constexpr (PF == 1) {
        TA ra[4];
        TB rb[4];
        load_slice<TA, AK>(A, n, m0, 0, tid, ra);
        load_slice<TB, BKR>(B, n, n0, 0, tid, rb);
        store_slice<Acc, TA, AK, OPA == OP_C>(As[0], tid, ra);
        store_slice<Acc, TB, BKR, OPB == OP_C>(Bs[0], tid, rb);
        __syncthreads();
        for (int kt = 0; kt < nkt; ++kt) {
            const int buf = kt & 1;
            const bool more = kt + 1 < nkt;
            if (more) {
                load_slice<TA, AK>(A, n, m0, (kt + 1) * BK, tid, ra);
                load_slice<TB, BKR>(B, n, n0, (kt + 1) * BK, tid, rb);
            }
            mma_tile<Acc, FourM<EPI>::value>(As[buf], Bs[buf], lane, am0, bn0, nmi, nnj, cr, ci, cs);
            if (more) {
                store_slice<Acc, TA, AK, OPA == OP_C>(As[buf ^ 1], tid, ra);
                store_slice<Acc, TB, BKR, OPB == OP_C>(Bs[buf ^ 1], tid, rb);
            }
            __syncthreads();
        }
    } else {
        // two slices in flight: slice kt + 2 is read into registers while slice kt is
        // multiplied and slice kt + 1 (read one step earlier) moves into LDS
        TA ra[2][4];
        TB rb[2][4];
        load_slice<TA, AK>(A, n, m0, 0, tid, ra[0]);
        load_slice<TB, BKR>(B, n, n0, 0, tid, rb[0]);
        if (nkt > 1) {
            load_slice<TA, AK>(A, n, m0, BK, tid, ra[1]);
            load_slice<TB, BKR>(B, n, n0, BK, tid, rb[1]);
        }
        store_slice<Acc, TA, AK, OPA == OP_C>(As[0], tid, ra[0]);
        store_slice<Acc, TB, BKR, OPB == OP_C>(Bs[0], tid, rb[0]);
        __syncthreads();
#define NEGF_GEMM_STEP(KT, CUR, NXT)                                                                      \
    {                                                                                                     \
        if ((KT) + 2 < nkt) {                                                                             \
            load_slice<TA, AK>(A, n, m0, ((KT) + 2) * BK, tid, ra[CUR]);                                  \
            load_slice<TB, BKR>(B, n, n0, ((KT) + 2) * BK, tid, rb[CUR]);                                 \
        }                                                                                                 \
        mma_tile<Acc, FourM<EPI>::value>(As[CUR], Bs[CUR], lane, am0, bn0, nmi, nnj, cr, ci, cs);                                  \
        if ((KT) + 1 < nkt) {                                                                             \
            store_slice<Acc, TA, AK, OPA == OP_C>(As[NXT], tid, ra[NXT]);                                 \
            store_slice<Acc, TB, BKR, OPB == OP_C>(Bs[NXT], tid, rb[NXT]);                                \
        }                                                                                                 \
        __syncthreads();                                                                                  \
    }
        for (int kt = 0; kt < nkt; kt += 2) {
            NEGF_GEMM_STEP(kt, 0, 1)
            if (kt + 1 < nkt) NEGF_GEMM_STEP(kt + 1, 1, 0)
        }
#undef NEGF_GEMM_STEP
    }
    finish_products<Acc, FourM<EPI>::value>(cr, ci, cs);
    gemm_epilogue<TC, Acc, EPI>(g, q, m0, n0, wt, lane, cr, ci);
}

// Persistent form of the two-slices-in-flight kernel: each workgroup walks the
// tiles lid, lid + G, ... (G = workgroups in the grid, sized to the resident
// slots) and keeps the K pipeline running across tile boundaries: the next
// tile's first slice is read during the current tile's last two products and
// staged in LDS with its last one; its second slice is read right after the
// epilogue (so no prefetch registers are live across it) and lands during the
// next tile's first products; a tile's epilogue stores overlap those products.
// Requires n > BK (at least two K slices per tile).
template <typename TA, typename TB, typename TC, typename Acc, int OPA, int OPB, int EPI>
__global__ __launch_bounds__(256, 2) void gemm_persist_kernel(GemmArgs g) {
    __shared__ Acc As[2][2][BK][LP];
    __shared__ Acc Bs[2][2][BK][LP];
    constexpr bool AH = (EPI == EPI_STORE_AH || EPI == EPI_ADD_TTD_AH);
    constexpr bool AK = (OPA == OP_C);
    constexpr bool BKR = (OPB == OP_N);
    const int n = g.n;
    const int tiles = (n + BM - 1) / BM;
    const int tpp = AH ? tiles * (tiles + 1) / 2 : tiles * tiles;
    const long long total = (long long)g.np * tpp;
    const int G = gridDim.x;
    const int nkt = (n + BK - 1) / BK;
    int tid = threadIdx.x;   // per tile an opaque copy (see the tile loop)
    // next tile of an active point at or after lt in this workgroup's sequence
    auto advance = [&](long long lt) {
        while (lt < total && !g.act((int)(lt / tpp))) lt += G;
        return lt;
    };
    long long lc = advance(xcd_remap(blockIdx.x, G));
    if (lc >= total) return;
    long long ln = advance(lc + G);
    int cq, cm0, cn0, nq = 0, nm0 = 0, nn0 = 0;
    {
        int ti, tj;
        cq = (int)(lc / tpp);
        tile_of<AH>((int)(lc - (long long)cq * tpp), tiles, ti, tj);
        cm0 = ti * BM; cn0 = tj * BM;
    }
    auto set_next = [&]() {
        if (ln < total) {
            int ti, tj;
            nq = (int)(ln / tpp);
            tile_of<AH>((int)(ln - (long long)nq * tpp), tiles, ti, tj);
            nm0 = ti * BM; nn0 = tj * BM;
        }
    };
    set_next();
    auto ldA = [&](int q, int m0, int kt, TA (&r)[4]) {
        load_slice<TA, AK>((const TA*)g.A + q * g.sA, n, m0, kt * BK, tid, r);
    };
    auto ldB = [&](int q, int n0, int kt, TB (&r)[4]) {
        load_slice<TB, BKR>((const TB*)g.B + q * g.sB, n, n0, kt * BK, tid, r);
    };
    TA ra[2][4];
    TB rb[2][4];
    ldA(cq, cm0, 0, ra[0]); ldB(cq, cn0, 0, rb[0]);
    ldA(cq, cm0, 1, ra[1]); ldB(cq, cn0, 1, rb[1]);
    store_slice<Acc, TA, AK, OPA == OP_C>(As[0], tid, ra[0]);
    store_slice<Acc, TB, BKR, OPB == OP_C>(Bs[0], tid, rb[0]);
    __syncthreads();

    typename MF<Acc>::V cr[2][2], ci[2][2], cs[2][2];
    int lb = 0;   // LDS buffer holding the slice about to be multiplied
    // One step: RC receives the slice two ahead, RN holds the next slice, which
    // is staged into the other LDS buffer while buffer lb is multiplied.  Within
    // a tile the register sets alternate with kt; the LDS buffers alternate with
    // every slice of the workgroup's sequence.
#define NEGF_PERSIST_STEP(KT, RC, RN, MI, NJ)                                                             \
    {                                                                                                     \
        const int k2 = (KT) + 2;                                                                          \
        if (k2 < nkt) {                                                                                   \
            ldA(cq, cm0, k2, ra[RC]); ldB(cq, cn0, k2, rb[RC]);                                           \
        } else if (k2 == nkt && ln < total) {                                                             \
            ldA(nq, nm0, 0, ra[RC]); ldB(nq, nn0, 0, rb[RC]);                                             \
        }                                                                                                 \
        if constexpr (MI > 0 && NJ > 0)                                                                   \
            mma_slice<Acc, (MI > 0 ? MI : 1), (NJ > 0 ? NJ : 1), FourM<EPI>::value>(As[lb], Bs[lb], lane,   \
                                                                                    wt.am0, wt.bn0,     \
                                                                 cr, ci, cs);                             \
        if ((KT) + 1 < nkt || ln < total) {                                                               \
            store_slice<Acc, TA, AK, OPA == OP_C>(As[lb ^ 1], tid, ra[RN]);                               \
            store_slice<Acc, TB, BKR, OPB == OP_C>(Bs[lb ^ 1], tid, rb[RN]);                              \
        }                                                                                                 \
        __syncthreads();                                                                                  \
        lb ^= 1;                                                                                          \
    }
    // the K loop of one tile for a wave owning MI x NJ blocks (0: loads and barriers only)
#define NEGF_PERSIST_TILE(MI, NJ)                                                                         \
    for (int kt = 0; kt < nkt; kt += 2) {                                                                 \
        NEGF_PERSIST_STEP(kt, 0, 1, MI, NJ)                                                               \
        if (kt + 1 < nkt) NEGF_PERSIST_STEP(kt + 1, 1, 0, MI, NJ)                                         \
    }
    for (;;) {
        // LDS buffer lb holds slice 0 of the current tile, registers 1 its slice 1.
        // The thread id is passed through an empty asm once per tile, so the
        // per-thread address offsets derived from it are recomputed here instead
        // of being hoisted out of the tile loop and kept alive across the epilogue.
        asm volatile("" : "+v"(tid));
        const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) { cr[a][b][r] = 0; ci[a][b][r] = 0; cs[a][b][r] = 0; }
        const WaveTile wt = wave_tile(wave, n - cm0, n - cn0);
        if (wt.nmi == 2 && wt.nnj == 2) NEGF_PERSIST_TILE(2, 2)
        else if (wt.nmi == 2 && wt.nnj == 1) NEGF_PERSIST_TILE(2, 1)
        else if (wt.nmi == 1 && wt.nnj == 2) NEGF_PERSIST_TILE(1, 2)
        else if (wt.nmi == 1 && wt.nnj == 1) NEGF_PERSIST_TILE(1, 1)
        else NEGF_PERSIST_TILE(0, 0)
        finish_products<Acc, FourM<EPI>::value>(cr, ci, cs);
        gemm_epilogue<TC, Acc, EPI>(g, cq, cm0, cn0, wt, lane, cr, ci);
        if (ln >= total) return;
        cq = nq; cm0 = nm0; cn0 = nn0;
        // the new tile's second slice: both register sets are free here
        ldA(cq, cm0, 1, ra[1]); ldB(cq, cn0, 1, rb[1]);
        ln = advance(ln + G);
        set_next();
    }
#undef NEGF_PERSIST_TILE
#undef NEGF_PERSIST_STEP
}

// Resident workgroup slots of the current device for the persistent kernel:
// two 80 KB-LDS workgroups per compute unit.
static int persist_slots() {
    static int slots[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (slots[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 0;
        slots[dev] = 2 * cus;
    }
    return slots[dev];
}

template <typename TA, typename TB, typename TC, typename Acc, int OPA, int OPB>
static hipError_t launch_epi(hipStream_t s, int epi, const GemmArgs& g, dim3 grid) {
    // pf 3: the persistent two-slice kernel (FP64 products, at least two K slices)
    const int slots = (g.pf == 3 && sizeof(Acc) == 8 && g.n > BK) ? persist_slots() : 0;
    const bool persist = slots > 0;
    dim3 pgrid(persist ? (unsigned)std::min<long long>((long long)grid.x, slots) : 1u);
    switch (epi) {
#define NEGF_EPI(E)                                                                                       \
    case E:                                                                                               \
        if (persist)                                                                                      \
            hipLaunchKernelGGL((gemm_persist_kernel<TA, TB, TC, Acc, OPA, OPB, E>), pgrid, dim3(256), 0, s, g); \
        else if (g.pf != 1)                                                                               \
            hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, Acc, OPA, OPB, E, 2>), grid, dim3(256), 0, s, g); \
        else                                                                                              \
            hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, Acc, OPA, OPB, E, 1>), grid, dim3(256), 0, s, g); \
        break;
        NEGF_EPI(EPI_STORE) NEGF_EPI(EPI_ADD) NEGF_EPI(EPI_ADD_TTD) NEGF_EPI(EPI_DUAL) NEGF_EPI(EPI_IMINUS) NEGF_EPI(EPI_SUB)
        NEGF_EPI(EPI_STORE_AH) NEGF_EPI(EPI_ADD_TTD_AH)
#undef NEGF_EPI
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TA, typename TB, typename TC, typename Acc>
static hipError_t launch_ops(hipStream_t s, int opa, int opb, int epi, const GemmArgs& g, dim3 grid) {
    if (opa == OP_N && opb == OP_N) return launch_epi<TA, TB, TC, Acc, OP_N, OP_N>(s, epi, g, grid);
    if (opa == OP_N && opb == OP_C) return launch_epi<TA, TB, TC, Acc, OP_N, OP_C>(s, epi, g, grid);
    if (opa == OP_C && opb == OP_N) return launch_epi<TA, TB, TC, Acc, OP_C, OP_N>(s, epi, g, grid);
    return launch_epi<TA, TB, TC, Acc, OP_C, OP_C>(s, epi, g, grid);
}

hipError_t gemm_launch(hipStream_t s, GemmTypes ty, int opa, int opb, int epi, const GemmArgs& g) {
    if (g.np <= 0 || g.n <= 0) return hipSuccess;
    dim3 grid((unsigned)((long long)g.np * gemm_tiles(g.n, epi)));
    if (ty.ta == DT_C128 && ty.tb == DT_C128 && ty.tc == DT_C128 && ty.acc == DT_C128)
        return launch_ops<double2, double2, double2, double>(s, opa, opb, epi, g, grid);
    if (ty.ta == DT_C64 && ty.tb == DT_C64 && ty.tc == DT_C64 && ty.acc == DT_C64)
        return launch_ops<float2, float2, float2, float>(s, opa, opb, epi, g, grid);
    // Mixed-precision refinement: FP64 residual R = I - A X0 with X0 in FP32.
    if (ty.ta == DT_C128 && ty.tb == DT_C64 && ty.tc == DT_C128 && ty.acc == DT_C128 &&
        opa == OP_N && opb == OP_N && epi == EPI_IMINUS) {
        hipLaunchKernelGGL((gemm_kernel<double2, float2, double2, double, OP_N, OP_N, EPI_IMINUS, 2>),
                           grid, dim3(256), 0, s, g);
        return hipGetLastError();
    }
    // Mixed-precision correction X1 = X0 + X0 R in FP32 with R read in FP64.
    if (ty.ta == DT_C64 && ty.tb == DT_C128 && ty.tc == DT_C64 && ty.acc == DT_C64 &&
        opa == OP_N && opb == OP_N && epi == EPI_ADD) {
        hipLaunchKernelGGL((gemm_kernel<float2, double2, float2, float, OP_N, OP_N, EPI_ADD, 2>),
                           grid, dim3(256), 0, s, g);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

}  // namespace negf
