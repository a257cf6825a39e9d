// Host-side launchers shared by the library's translation units.
#pragma once
#include "negf_common.hpp"

namespace negf {

// ------------------------------------------------------------- batched GEMM
enum Op : int { OP_N = 0, OP_C = 1 };   // op(X) = X or X^dagger
enum Epi : int {
    EPI_STORE = 0,     // C = op(A) op(B)
    EPI_ADD = 1,       // C = D + op(A) op(B)
    EPI_ADD_TTD = 2,   // C = D + op(A) op(B) + T - T^dagger
    EPI_DUAL = 3,      // C += op(A) op(B);  C2 += op(A) op(B)
    EPI_IMINUS = 4,    // C = I - op(A) op(B)
    EPI_SUB = 5,       // C = D - op(A) op(B)
    // Anti-Hermitian results: only the tiles on and below the diagonal are
    // computed; each element below the diagonal is also written, as -conj, to
    // its mirror above it, and the diagonal keeps only its imaginary part.  A
    // rounding-level real part left on the diagonal would be carried forward
    // by the next sandwich g (.) g^dagger with positive weights |g_am|^2 and
    // grow slab after slab; with the exact symmetry there is nothing to grow.
    EPI_STORE_AH = 6,    // C = op(A) op(B)
    EPI_ADD_TTD_AH = 7,  // C = D + op(A) op(B) + T - T^dagger
};
enum Dt : int { DT_C128 = 0, DT_C64 = 1 };

// One batched product over points q in [0, np): every operand X of point q
// sits at X + q * sX (elements of its own type).
struct GemmArgs {
    const void* A; long long sA;
    const void* B; long long sB;
    void* C; long long sC;
    const void* D; long long sD;
    const void* T; long long sT;
    void* C2; long long sC2;
    int n;
    int np;
    Active act;
    int pf;              // K slices in flight: 1 or 2 (0: 2); 3: two, persistent workgroups
};

struct GemmTypes {
    int ta, tb, tc;   // Dt of A, B and of C/D/T/C2
    int acc;          // DT_C128: FP64 MFMA, DT_C64: FP32 MFMA
};

// Output tiles a launch computes per point (BM-wide tiles; the anti-Hermitian
// epilogues cover the lower triangle of tiles only).
inline long long gemm_tiles(int n, int epi) {
    const long long t = (n + 63) / 64;
    return (epi == EPI_STORE_AH || epi == EPI_ADD_TTD_AH) ? t * (t + 1) / 2 : t * t;
}

// Launches C = op(A) op(B) (+ epilogue).  Returns hipError_t.
hipError_t gemm_launch(hipStream_t s, GemmTypes ty, int opa, int opb, int epi, const GemmArgs& g);

// ------------------------------------------------- batched block inverse
struct InvWork {
    void* pa;            // ping-pong partner of the source matrix, [np][n][n]
    void* E;             // panel buffer [np][n][NB] (complex, matrix type)
    void* Prow;          // pivot rows [np][NB][n]
    int* rowsrc;         // [np][n]
    int* piv;            // [np][n]
    int* coldst;         // [np][n]
    int* status;
    void* N0; void* N1;  // narrow ping-pong copies of an outer panel, [np][n][INV_WMAX] each (NULL: one level)
    int* comp;           // [np][n] composite row source of an outer panel
    int W;               // outer panel width (a multiple of 32, <= INV_WMAX), 0: one level
    int* comp2;          // [np][n] composite row source of a mid block, or NULL
    int Wm;              // mid block width (three levels; a multiple of 32 below W), 0: two levels
};
// dst = src^-1 for every active point (Gauss-Jordan, partial pivoting).  src
// is destroyed.  dt = DT_C128 or DT_C64 (matrix and arithmetic type).
constexpr int INV_NMAX = 2048;   // largest block the inverse handles
constexpr int INV_WMAX = 256;    // widest outer panel of the two-level inverse
hipError_t inverse_init();
hipError_t inverse_launch(hipStream_t s, int dt, void* src, long long s_src, void* dst, long long s_dst,
                          int n, int np, const Active& act, const InvWork& w);

}  // namespace negf
