// noalloc.hip -- mpgemm_ex_noalloc: the _ex entry points with their scratch
// taken from a static device buffer instead of a caller workspace, for callers
// that cannot allocate.
//
// The buffer is a file-scope device array.  In host code its name is only a
// host-side handle of the symbol, not a device address, so host code never
// passes it to a kernel or a copy: the first call on each device looks up the
// array's address on that device (each GPU holds its own copy) and keeps it;
// every later use goes through that address.
#include "mpgemm.h"

#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

static __device__ __align__(256) unsigned char scratch[MPGEMM_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's buffer (looked up once per device).
int scratch_for_current_device(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return MPGEMM_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return MPGEMM_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MPGEMM_ERR_HIP;
        if ((uintptr_t)p % 256 != 0) return MPGEMM_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

}  // namespace

extern "C" int mpgemm_ex_noalloc(int prec, char ta, char tb, int64_t m, int64_t n, int64_t k,
                                 const double* alpha, const double* A, int64_t lda, int64_t sa,
                                 const double* B, int64_t ldb, int64_t sb, const double* beta,
                                 double* C, int64_t ldc, int64_t sc, hipStream_t st,
                                 const mpgemm_opts* opts) {
    if (prec < 2 || prec > 4) return -1;
    int rc = mpg::gemm_ex_check(prec, ta, tb, m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc,
                                opts);
    if (rc) return rc < 0 ? rc - 1 : rc;             // prec is argument 1
    if (opts->workspace || opts->workspace_bytes) return -19;
    void* ptr = nullptr;
    rc = scratch_for_current_device(&ptr);
    if (rc) return rc;
    mpgemm_opts o = *opts;
    o.workspace = ptr;
    o.workspace_bytes = MPGEMM_STATIC_SCRATCH_BYTES;
    rc = mpg::gemm_ex_entry(prec, ta, tb, m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, st,
                            &o);
    if (rc < 0) return rc - 1;                       // prec is argument 1
    // the buffer is non-null and aligned, so a workspace error means too small
    if (rc == MPGEMM_ERR_WORKSPACE) return MPGEMM_ERR_SCRATCH;
    return rc;
}
