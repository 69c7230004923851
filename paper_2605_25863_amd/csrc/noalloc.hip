// linac_solve_noalloc: the solve for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  Its scratch space is a fixed array in this file, one copy
// per GPU, instead of a caller workspace.
#include <mutex>
#include <vector>

#include "internal.h"

namespace linac {

namespace {

// One copy per GPU, held until the process ends.  In host code `scratch` names
// a host-side stand-in, not device memory: kernels only ever get the device
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[LINAC_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device; NULL until looked up

// The device address of this GPU's copy, looked up once per device with that
// device current (the first call on it).
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

}  // namespace linac

using namespace linac;

extern "C" linac_status linac_solve_noalloc(const uint32_t* A, int64_t m, int64_t n, int64_t lda,
                                            const uint32_t* B, int64_t k, int64_t ldb, uint32_t p,
                                            uint32_t* X, int64_t ldx, int32_t* rank,
                                            int32_t* pivots, uint8_t* consistent,
                                            const linac_opts* opts, hipStream_t s) {
    int path = 0;
    size_t need = 0;
    linac_status st = solve_check(A, m, n, lda, B, k, ldb, p, X, ldx, rank, pivots, consistent,
                                  opts, &path, &need);
    if (st != LINAC_OK) return st;
    if (need > LINAC_NOALLOC_SCRATCH_BYTES) return LINAC_E_WORKSPACE;
    if (opts && opts->validate) return LINAC_E_UNSUPPORTED;  // it would read a flag back
    void* ws = nullptr;
    const hipError_t e = scratch_address(&ws);
    if (e != hipSuccess) return hip_status(e);
    // every buffer the path reads is initialised by the path itself, so what an
    // earlier call left in the array does not matter
    return solve_launch(A, m, n, lda, B, k, ldb, p, X, ldx, rank, pivots, consistent, ws, path, opts,
                        s, false, "solve_noalloc");
}
