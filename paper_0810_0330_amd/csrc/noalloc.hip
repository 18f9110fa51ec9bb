// sc_project_noalloc: the projection X += V T^{-1} V^H R0 of sc_project with
// its scratch space (the coefficient block, the contraction's per-chunk
// partials and the tridiagonal solve's work) in a fixed array of device memory
// that the library owns, so the call itself allocates nothing: for callers
// that cannot allocate (code under stream capture, serving loops).
//
// The array is a file-scope __device__ variable: every GPU the library runs on
// holds its own copy until the process ends.  Its device address is looked up
// once per device, at the first call on that device, with hipGetSymbolAddress;
// host code uses only that address (the variable's name in host code is a
// host-side stand-in, not a device pointer).  The kernels of the projection
// write every scratch element they read, so nothing has to start at zero.
// Calls that overlap on one device share the array and race.
#include <mutex>

#include "sc_internal.h"
#include "sc_timer.h"

namespace sc {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;  // SC_NOALLOC_SCRATCH_BYTES in seedcg.h
static_assert(kNoAllocScratchBytes == SC_NOALLOC_SCRATCH_BYTES, "header and library disagree on the scratch size");

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the current device's copy of `scratch`, looked up on the first call per device
sc_status scratch_for_current_device(void** out) {
    int dev = -1;
    SC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("sc_project_noalloc: device index out of range");
        return SC_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        SC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("sc_project_noalloc: hipGetSymbolAddress returned a null address");
            return SC_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SC_OK;
}
}  // namespace

}  // namespace sc

using namespace sc;

extern "C" sc_status sc_project_noalloc(int64_t n, const void* V_dev, int64_t ldv, sc_dtype v_dtype, int m,
                                        const double* alpha_dev, const double* beta_dev, sc_dtype vec_dtype,
                                        const void* R0_dev, int64_t ldr, int k, void* X_dev, int64_t ldx,
                                        void* stream) {
    clear_error();
    try {
        SC_ARG(n >= 1, "n must be >= 1");
        SC_ARG(m >= 1, "m must be >= 1");
        SC_ARG(k >= 0, "k must be >= 0");
        SC_ARG(vec_dtype == SC_C128 || vec_dtype == SC_R64, "vec_dtype must be SC_C128 or SC_R64");
        SC_ARG(double_of(v_dtype) == vec_dtype, "v_dtype and vec_dtype must both be complex or both real");
        if (k == 0) return SC_OK;
        SC_ARG(V_dev && alpha_dev && beta_dev && R0_dev && X_dev, "NULL device pointer");
        SC_ARG(((uintptr_t)V_dev % dtype_bytes(v_dtype)) == 0 && ((uintptr_t)R0_dev % dtype_bytes(vec_dtype)) == 0 &&
                   ((uintptr_t)X_dev % dtype_bytes(vec_dtype)) == 0,
               "misaligned device pointer");
        SC_ARG(ldv >= n && ldr >= n && ldx >= n, "leading dimension smaller than n");
        const size_t need = project_workspace(n, m, k, is_complex(vec_dtype));
        if (need > kNoAllocScratchBytes) {
            set_error("sc_project_noalloc: n = " + std::to_string(n) + ", m = " + std::to_string(m) + " needs " +
                      std::to_string(need) + " bytes of scratch, more than the library's fixed " +
                      std::to_string(kNoAllocScratchBytes) + "; use sc_project with a work buffer");
            return SC_ERR_WORKSPACE;
        }
        void* p = nullptr;
        SC_TRY(scratch_for_current_device(&p));
        TimerMute mute;  // the optional benchmark timer would create events
        return project_impl(n, V_dev, ldv, v_dtype, m, alpha_dev, beta_dev, vec_dtype, R0_dev, ldr, k, X_dev, ldx, p,
                            kNoAllocScratchBytes, (hipStream_t)stream);
    } catch (...) {
        set_error("unexpected host exception");
        return SC_ERR_ARG;
    }
}
