// Batched complex GEMM on CDNA4 matrix cores.
//
// Every slab step of the RGF recursions (g_i X, Y g_i^dagger, L G_{i+1},
// P R, ...) is a dense complex b x b x b product for each (sample, k, E)
// point of a batch.  One launch covers the whole batch: a 64 x 64 output tile
// of one point per 256-thread workgroup (4 wavefronts of 32 x 32), K staged
// through LDS in 16-wide double-buffered slices, split real/imaginary planes.
// A complex product is three real MFMA products on v_mfma_f64_16x16x4f64
// (FP64, the 3M form) or four on v_mfma_f32_16x16x4f32 (FP32).
#include "negf_internal.hpp"
#include "negf_mfma.hpp"

namespace negf {

static_assert(BM == 64, "gemm_tiles() assumes 64-wide tiles");

template <typename Acc>
__device__ inline void mma_tile(Acc (*As)[BK][LP], Acc (*Bs)[BK][LP], int lane, int am0, int bn0, int nmi, int nnj,
                                typename MF<Acc>::V (&cr)[2][2], typename MF<Acc>::V (&ci)[2][2],
                                typename MF<Acc>::V (&cs)[2][2]) {
    if (nmi == 2 && nnj == 2) mma_slice<Acc, 2, 2>(As, Bs, lane, am0, bn0, cr, ci, cs);
    else if (nmi == 2 && nnj == 1) mma_slice<Acc, 2, 1>(As, Bs, lane, am0, bn0, cr, ci, cs);
    else if (nmi == 1 && nnj == 2) mma_slice<Acc, 1, 2>(As, Bs, lane, am0, bn0, cr, ci, cs);
    else if (nmi == 1 && nnj == 1) mma_slice<Acc, 1, 1>(As, Bs, lane, am0, bn0, cr, ci, cs);
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
    if (AH) {
        // t -> (ti, tj), tj <= ti, row-major over the lower triangle of tiles
        ti = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
        while (ti * (ti + 1) / 2 > t) --ti;
        tj = t - ti * (ti + 1) / 2;
    } else {
        ti = t / tiles;
        tj = t - ti * tiles;
    }
    const int m0 = ti * BM, n0 = tj * BM;
    const TA* __restrict__ A = (const TA*)g.A + q * g.sA;
    const TB* __restrict__ B = (const TB*)g.B + q * g.sB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const WaveTile wt = wave_tile(wave, n - m0, n - n0);
    const int am0 = wt.am0, bn0 = wt.bn0, nmi = wt.nmi, nnj = wt.nnj;
    const int rowbase = m0 + am0, colbase = n0 + bn0;

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
            mma_tile<Acc>(As[buf], Bs[buf], lane, am0, bn0, nmi, nnj, cr, ci, cs);
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
        mma_tile<Acc>(As[CUR], Bs[CUR], lane, am0, bn0, nmi, nnj, cr, ci, cs);                                  \
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
    finish_products<Acc>(cr, ci, cs);

    TC* __restrict__ C = (TC*)g.C + q * g.sC;
    const TC* D = (const TC*)g.D + q * g.sD;
    const TC* T = (const TC*)g.T + q * g.sT;
    TC* C2 = (TC*)g.C2 + q * g.sC2;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
        if (mi >= nmi) break;
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) {
            if (nj >= nnj) break;
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

template <typename TA, typename TB, typename TC, typename Acc, int OPA, int OPB>
static hipError_t launch_epi(hipStream_t s, int epi, const GemmArgs& g, dim3 grid) {
    switch (epi) {
#define NEGF_EPI(E)                                                                                       \
    case E:                                                                                               \
        if (g.pf != 1)                                                                                    \
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
