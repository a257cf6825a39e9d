// MFMA tile helpers shared by the batched GEMM and the block-inverse update.
#pragma once
#include "negf_common.hpp"

namespace negf {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename Acc> struct MF;
template <> struct MF<double> {
    typedef v4d V;
    __device__ static inline V mma(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct MF<float> {
    typedef v4f V;
    __device__ static inline V mma(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// Row (within a 16 x 16 output block) held in accumulator register r of `lane`;
// the column is lane % 16.  The two 16x16x4 forms differ:
//   f64: D[i][j] in lane j + 16 (i % 4), register i / 4
//   f32: D[i][j] in lane j + 16 (i / 4), register i % 4
template <typename Acc> __device__ inline int out_row(int lane, int r);
template <> __device__ inline int out_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }
template <> __device__ inline int out_row<float>(int lane, int r) { return (lane >> 4) * 4 + r; }

constexpr int BM = 64;   // tile rows = tile cols
constexpr int BK = 16;   // K slice
constexpr int LP = 80;   // LDS row stride (elements): rows k, k+1 of a fragment read land on disjoint banks

// LDS column of element (k, c) of a staged slice: each group of four k rows
// XORs the column by a different multiple of 4, so the four k rows one store
// instruction of the row-outer pattern touches start 8 dwords apart and fill
// all 32 LDS banks, while every fragment read (one k group) stays a plain
// permutation of 16-column blocks.
__device__ __host__ constexpr int swz(int k, int c) { return c ^ (((k >> 2) & 3) << 2); }

// Element j (0..3) of a thread's share of one K slice, as (k row, outer index)
// within the slice.
//   KROWS = false ("pattern X"): 64 outer rows, 16 contiguous k: 4 consecutive k.
//   KROWS = true  ("pattern Y"): 16 k rows, 64 contiguous outer indices:
//   columns l, l + 16, l + 32, l + 48 (l = tid mod 16), so that the 16 lanes of
//   a k row store 16 consecutive values (all 32 banks) per instruction.
template <bool KROWS>
__device__ inline void slice_slot(int tid, int j, int& k, int& o) {
    if (!KROWS) { o = tid >> 2; k = (tid & 3) * 4 + j; }
    else { k = tid >> 4; o = (tid & 15) + 16 * j; }
}

// Loads one K slice of op(X) into registers.
template <typename TX, bool KROWS>
__device__ inline void load_slice(const TX* __restrict__ X, int n, int o0, int k0, int tid, TX (&r)[4]) {
    if (!KROWS) {
        const int row = o0 + (tid >> 2), col = k0 + (tid & 3) * 4;
        const TX* p = X + (long long)row * n + col;
        if (row < n && col + 3 < n) {
#pragma unroll
            for (int j = 0; j < 4; ++j) r[j] = p[j];
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (row < n && col + j < n) r[j] = p[j];
                else { r[j].x = 0; r[j].y = 0; }
            }
        }
    } else {
        const int row = k0 + (tid >> 4), col = o0 + (tid & 15);
        const TX* p = X + (long long)row * n + col;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (row < n && col + 16 * j < n) r[j] = p[16 * j];
            else { r[j].x = 0; r[j].y = 0; }
        }
    }
}

// Writes the register slice into LDS planes S[re/im][k][outer] (conjugated if CONJ).
template <typename Acc, typename TX, bool KROWS, bool CONJ>
__device__ inline void store_slice(Acc (*S)[BK][LP], int tid, const TX (&r)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        int k, o;
        slice_slot<KROWS>(tid, j, k, o);
        S[0][k][swz(k, o)] = (Acc)r[j].x;
        S[1][k][swz(k, o)] = CONJ ? -(Acc)r[j].y : (Acc)r[j].y;
    }
}

// Complex products use three real MFMA products (the 3M form): with
// P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi), the product is
// (P1 - P2) + i (P3 - P1 - P2), 12 MFMAs per complex 16x16x4 step instead of
// 16.  The imaginary part's rounding is bounded by the unit roundoff times
// (|Ar| + |Ai|)(|Br| + |Bi|) instead of |Ar||Bi| + |Ai||Br|.

// The part of a 64 x 64 output tile a wave computes: tile-local origin
// (am0, bn0) and its count of 16-row and 16-column blocks inside the valid
// vr x vc corner of the tile.  Normally a 32 x 32 quarter; in a tile with at
// most 16 valid rows (or columns), such as the last tile row at b = 400, the
// four waves take one 16-wide block each along the other direction instead,
// so none of them idles while the workgroup holds its slot.
struct WaveTile { int am0, bn0, nmi, nnj; };
__device__ inline WaveTile wave_tile(int wave, int vr, int vc) {
    WaveTile w;
    if (vr <= 16 && vc > 16) {
        w.am0 = 0; w.bn0 = 16 * wave; w.nmi = 1; w.nnj = w.bn0 < vc ? 1 : 0;
    } else if (vc <= 16 && vr > 16) {
        w.am0 = 16 * wave; w.bn0 = 0; w.nmi = w.am0 < vr ? 1 : 0; w.nnj = 1;
    } else {
        w.am0 = (wave >> 1) * 32; w.bn0 = (wave & 1) * 32;
        w.nmi = w.am0 >= vr ? 0 : (w.am0 + 16 >= vr ? 1 : 2);
        w.nnj = w.bn0 >= vc ? 0 : (w.bn0 + 16 >= vc ? 1 : 2);
    }
    return w;
}

// Accumulates one staged K slice into the (up to) 2 x 2 blocks of 16 x 16 at
// tile-local (am0, bn0) that this wave owns; cr, ci, cs accumulate P1, P2, P3
// of the 3M form until finish_products().
template <typename Acc, int MI, int NJ, bool FOURM = false>
__device__ inline void mma_slice(Acc (*As)[BK][LP], Acc (*Bs)[BK][LP], int lane, int am0, int bn0,
                                 typename MF<Acc>::V (&cr)[2][2], typename MF<Acc>::V (&ci)[2][2],
                                 typename MF<Acc>::V (&cs)[2][2]) {
    const int o = lane & 15;
    // Fragments of step kk + 1 are read from LDS into the other register set
    // while the products of step kk run.
    Acc ar[2][MI], ai[2][MI], br[2][NJ], bi[2][NJ];
    auto frag = [&](int kk, int set) {
        const int k = kk * 4 + (lane >> 4);
#pragma unroll
        for (int mi = 0; mi < MI; ++mi) {
            ar[set][mi] = As[0][k][swz(k, am0 + mi * 16 + o)];
            ai[set][mi] = As[1][k][swz(k, am0 + mi * 16 + o)];
        }
#pragma unroll
        for (int nj = 0; nj < NJ; ++nj) {
            br[set][nj] = Bs[0][k][swz(k, bn0 + nj * 16 + o)];
            bi[set][nj] = Bs[1][k][swz(k, bn0 + nj * 16 + o)];
        }
    };
    frag(0, 0);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
        const int c = kk & 1;
        if (kk + 1 < BK / 4) frag(kk + 1, c ^ 1);
        __builtin_amdgcn_sched_barrier(0);   // the reads stay ahead of this step's products
        Acc sa[MI], sb[NJ];
#pragma unroll
        for (int mi = 0; mi < MI; ++mi) sa[mi] = ar[c][mi] + ai[c][mi];
#pragma unroll
        for (int nj = 0; nj < NJ; ++nj) sb[nj] = br[c][nj] + bi[c][nj];
        if constexpr (FOURM) {
            // four real products: cr += Ar Br - Ai Bi, ci += Ar Bi + Ai Br (cs unused)
            (void)sa; (void)sb;
#pragma unroll
            for (int mi = 0; mi < MI; ++mi)
#pragma unroll
                for (int nj = 0; nj < NJ; ++nj) {
                    const Acc nai = -ai[c][mi];
                    cr[mi][nj] = MF<Acc>::mma(ar[c][mi], br[c][nj], cr[mi][nj]);
                    cr[mi][nj] = MF<Acc>::mma(nai, bi[c][nj], cr[mi][nj]);
                    ci[mi][nj] = MF<Acc>::mma(ar[c][mi], bi[c][nj], ci[mi][nj]);
                    ci[mi][nj] = MF<Acc>::mma(ai[c][mi], br[c][nj], ci[mi][nj]);
                }
        } else {
#pragma unroll
            for (int mi = 0; mi < MI; ++mi)
#pragma unroll
                for (int nj = 0; nj < NJ; ++nj) {
                    cr[mi][nj] = MF<Acc>::mma(ar[c][mi], br[c][nj], cr[mi][nj]);
                    ci[mi][nj] = MF<Acc>::mma(ai[c][mi], bi[c][nj], ci[mi][nj]);
                    cs[mi][nj] = MF<Acc>::mma(sa[mi], sb[nj], cs[mi][nj]);
                }
        }
    }
}

// Turns the partial products P1, P2, P3 into real and imaginary parts.
template <typename Acc, bool FOURM = false>
__device__ inline void finish_products(typename MF<Acc>::V (&cr)[2][2], typename MF<Acc>::V (&ci)[2][2],
                                       const typename MF<Acc>::V (&cs)[2][2]) {
    if constexpr (FOURM) return;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const Acc p1 = cr[mi][nj][r], p2 = ci[mi][nj][r];
                cr[mi][nj][r] = p1 - p2;
                ci[mi][nj][r] = (cs[mi][nj][r] - p1) - p2;
            }
}

}  // namespace negf
