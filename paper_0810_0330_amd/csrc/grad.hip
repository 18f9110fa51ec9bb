// Derivative of L = sum_j Re<eta_j, x_j> with respect to kappa, for
// x_j = A^{-1} b_j and A = D^H D, D = 1 - kappa H (so dA/dkappa =
// -(H^H D + D^H H)).  With the adjoint solutions lambda_j = A^{-1} eta_j:
//   dL/dkappa = sum_j Re[(H lambda_j)^H (D x_j) + (D lambda_j)^H (H x_j)].
// Four stencil passes and two column dot products, all in FP64.
#include <vector>

#include "sc_internal.h"

namespace sc {

size_t kappa_grad_workspace(const sc_op* op, int k) {
    Carver c(nullptr, 0);
    for (int i = 0; i < 4; ++i) c.take<double>((size_t)op->n * 2 * k);
    c.take<double>((size_t)kMaxRedBlocks * k);
    c.take<double>((size_t)2 * k);
    return c.off + 256;
}

sc_status kappa_grad(const sc_op* op, const void* X, int64_t ldx, const void* L, int64_t ldl, int k, double* out,
                     void* work, size_t work_bytes, hipStream_t s) {
    Carver c(work, work_bytes);
    double* dx = c.take<double>((size_t)op->n * 2 * k);
    double* hx = c.take<double>((size_t)op->n * 2 * k);
    double* dl = c.take<double>((size_t)op->n * 2 * k);
    double* hl = c.take<double>((size_t)op->n * 2 * k);
    double* part = c.take<double>((size_t)kMaxRedBlocks * k);
    double* res = c.take<double>((size_t)2 * k);
    if (!c.ok()) {
        set_error("kappa_grad: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    const int64_t n = op->n, N2 = 2 * n;
    SC_TRY(wilson_pass(op, false, 0, X, ldx, dx, n, k, s));
    SC_TRY(wilson_pass(op, false, 2, X, ldx, hx, n, k, s));
    SC_TRY(wilson_pass(op, false, 0, L, ldl, dl, n, k, s));
    SC_TRY(wilson_pass(op, false, 2, L, ldl, hl, n, k, s));
    // Re(a^H b) is the dot product of the real views
    SC_TRY(dot(0, hl, N2, 0, dx, N2, N2, k, res, part, nullptr, s));
    SC_TRY(dot(0, dl, N2, 0, hx, N2, N2, k, res + k, part, nullptr, s));
    std::vector<double> h(2 * k);
    SC_HIP(hipMemcpyAsync(h.data(), res, sizeof(double) * 2 * k, hipMemcpyDeviceToHost, s));
    SC_HIP(hipStreamSynchronize(s));
    double g = 0.0;
    for (int j = 0; j < k; ++j) g += h[j] + h[k + j];
    *out = g;
    return SC_OK;
}

}  // namespace sc
