// Batched block inverse for callers that cannot allocate device memory: the
// inverse's scratch (the ping-pong partner of the matrix, the panel transform,
// the pivot rows and the row/column maps) lives in one file-scope device array
// instead of a context's workspace.
#include "negf_internal.hpp"
#include "negf.h"

#include <mutex>

using namespace negf;

// One copy per GPU the library runs on, held until the process ends.  Host
// code never uses this name as an address: it passes the pointer
// hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) unsigned char scratch[NEGF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t NOALLOC_BYTES = (size_t)NEGF_NOALLOC_SCRATCH_BYTES;
constexpr int NB_PANEL = 32;      // widest Gauss-Jordan panel (E / pivot-row buffers are sized for it)
constexpr int MAX_DEVICES = 64;

std::mutex g_lock;
void* g_ptr[MAX_DEVICES] = {};

// Address of this device's scratch array, looked up once per device with that
// device current.
hipError_t scratch_for_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

long long negf_zinv_noalloc_bytes(int n, int batch, int dtype) {
    if (n < 1 || batch < 1 || (dtype != 0 && dtype != 1)) return -1;
    const size_t ce = dtype == 0 ? 16 : 8;
    const size_t b = (size_t)batch;
    return (long long)(align256(b * n * n * ce) + 2 * align256(b * n * NB_PANEL * ce) +
                       3 * align256(b * n * sizeof(int)));
}

int negf_zinv_batched_noalloc(void* stream, int n, int batch, void* A, void* Ainv, int dtype, int* status) {
    if (!A || !Ainv || n < 1 || batch < 1 || (dtype != 0 && dtype != 1)) return NEGF_EINVAL;
    if (n > INV_NMAX) return NEGF_ESHAPE;
    const long long need = negf_zinv_noalloc_bytes(n, batch, dtype);
    if (need < 0 || (size_t)need > NOALLOC_BYTES) return NEGF_ESHAPE;
    void* base = nullptr;
    NEGF_HIP_CHECK(scratch_for_current_device(&base));
    const size_t ce = dtype == 0 ? 16 : 8;
    const size_t b = (size_t)batch;
    char* p = static_cast<char*>(base);
    void* partner = p;
    p += align256(b * n * n * ce);
    void* E = p;
    p += align256(b * n * NB_PANEL * ce);
    void* Prow = p;
    p += align256(b * n * NB_PANEL * ce);
    int* rowsrc = reinterpret_cast<int*>(p);
    p += align256(b * n * sizeof(int));
    int* piv = reinterpret_cast<int*>(p);
    p += align256(b * n * sizeof(int));
    int* coldst = reinterpret_cast<int*>(p);
    // one-level Gauss-Jordan (no outer-panel copies): every buffer above is
    // written by the kernels before it is read, so nothing needs clearing
    InvWork w{partner, E, Prow, rowsrc, piv, coldst, status, nullptr, nullptr, nullptr, 0, nullptr, 0};
    const long long nn = (long long)n * n;
    Active all{nullptr, 0, 0, PRED_ALL, nullptr};
    NEGF_HIP_CHECK(inverse_launch((hipStream_t)stream, dtype == 0 ? DT_C128 : DT_C64, A, nn, Ainv, nn, n, batch,
                                  all, w));
    return NEGF_OK;
}

}  // extern "C"
