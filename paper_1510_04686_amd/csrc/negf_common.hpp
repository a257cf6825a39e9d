// Internal shared definitions of the MI355X (gfx950) RGF library.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace negf {

// ---------------------------------------------------------------------------
// Complex scalars: interleaved (re, im), the layout of torch.complex128 / 64.
// ---------------------------------------------------------------------------
template <typename R> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };
template <typename R> using cplx = typename cplx_of<R>::type;

template <typename C> __host__ __device__ inline C mk(double re, double im) {
    C c; c.x = re; c.y = im; return c;
}
__host__ __device__ inline double2 operator+(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 operator-(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 operator+(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 operator-(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

template <typename C> __host__ __device__ inline C cmul(C a, C b) {
    C c; c.x = a.x * b.x - a.y * b.y; c.y = a.x * b.y + a.y * b.x; return c;
}
// a * conj(b)
template <typename C> __host__ __device__ inline C cmulc(C a, C b) {
    C c; c.x = a.x * b.x + a.y * b.y; c.y = a.y * b.x - a.x * b.y; return c;
}
template <typename C> __host__ __device__ inline C cconj(C a) { a.y = -a.y; return a; }
// acc += a * b
template <typename C> __host__ __device__ inline void cfma(C& acc, C a, C b) {
    acc.x += a.x * b.x - a.y * b.y; acc.y += a.x * b.y + a.y * b.x;
}
template <typename C> __host__ __device__ inline C cscale(C a, double s) { a.x *= s; a.y *= s; return a; }

// Component-wise select.  A ?: on the two-element struct itself is lowered to a
// select between stack addresses (scratch memory); selecting each component
// keeps both operands in registers.
template <typename C> __host__ __device__ inline C csel(bool c, C a, C b) {
    C r; r.x = c ? a.x : b.x; r.y = c ? a.y : b.y; return r;
}

template <typename Cto, typename Cfrom> __device__ inline Cto cconv(Cfrom a) {
    Cto c; c.x = a.x; c.y = a.y; return c;
}

// ---------------------------------------------------------------------------
// Point descriptors.  One (sample, ik, ie) point of the bound set, with the
// slab count of its sample.  Workspace slots are indexed by q = p - p0.
// ---------------------------------------------------------------------------
struct PointSet {
    const int4* desc;            // [n_bound] = (sample, ik, ie, n_slab)
    const long long* slab_off;   // [n_samples + 1]
    int p0;                      // first bound point of the current call
};

// Activity predicates used by batched kernels.
enum Pred : int {
    PRED_ALL = 0,       // every point of the launch
    PRED_FWD = 1,       // slab `step` exists: step < n_slab
    PRED_BWD = 2,       // backward recursion step: step < n_slab - 1
    PRED_FLAG = 3,      // flags[q] == 0 (lead decimation not yet converged)
    PRED_INIT = 4,      // last slab of the point: step == n_slab - 1
    PRED_SET = 5,       // flags[q] != 0 (mixed precision: block inverse to redo in FP64)
};

struct Active {
    const int4* desc;
    int p0;
    int step;
    int mode;
    const int* flags;
    __device__ inline bool operator()(int q) const {
        if (mode == PRED_ALL) return true;
        if (mode == PRED_FLAG) return flags[q] == 0;
        if (mode == PRED_SET) return flags[q] != 0;
        int ns = desc[p0 + q].w;
        if (mode == PRED_FWD) return step < ns;
        if (mode == PRED_BWD) return step < ns - 1;
        return step == ns - 1;
    }
};

// Device status bits (accumulated with atomicOr, read by negf_sync_status).
enum StatusBits : int {
    ST_SINGULAR = 1,     // a zero pivot was met in a block inverse
    ST_NONFINITE = 2,    // a non-finite pivot was met
    ST_FALLBACK = 4,     // mixed precision redid a block inverse in FP64
};

__device__ inline void raise_status(int* status, int bits) {
    if (status) atomicOr(status, bits);
}

// Map a hardware workgroup id to a logical tile id so that consecutive
// logical tiles (the tiles of one batch point) run on the same XCD and share
// its L2.  Workgroups are dispatched round-robin over the 8 XCDs of MI355X.
__device__ inline int xcd_remap(int wg, int nwg) {
    constexpr int NXCD = 8;
    int per = nwg / NXCD;          // full rounds
    int rem = nwg - per * NXCD;
    int xcd = wg % NXCD;
    int slot = wg / NXCD;
    // XCD x owns the contiguous logical range [x*per, (x+1)*per); the
    // workgroups of the last, partial round take the ids after per*NXCD.
    if (slot < per) return xcd * per + slot;
    (void)rem;
    return per * NXCD + xcd;
}

}  // namespace negf

#define NEGF_HIP_CHECK(expr)                                   \
    do {                                                       \
        hipError_t _e = (expr);                                \
        if (_e != hipSuccess) return NEGF_EHIP;                \
    } while (0)
