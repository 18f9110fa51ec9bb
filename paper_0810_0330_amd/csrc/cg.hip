// Batched CG (Hestenes-Stiefel) for the seeded systems (Section 2.2): every
// right-hand side runs its own recurrence with its own FP64 scalars, held on
// the device; converged columns are frozen by a per-column flag.  The host
// synchronises once per chunk of iterations to see whether any column is
// still active, then verifies the true residual b - A x of every column and
// restarts the ones still above tol.
//
// mixed = 1: the vectors and the operator run in FP32; x and the true
// residual are FP64.  A reliable update (x64 += x32, r = b - A64 x64, r32 =
// r, x32 = 0, p kept) is made when a column's FP32 residual has fallen by 10x
// since its last update, and whenever it reaches tol.
#include "sc_internal.h"

#include <vector>

namespace sc {

struct CGCol {
    double rho;      // ||r||^2 of the current recurrence
    double alpha;    // rho / <p, A p>
    double beta;     // rho_new / rho
    double bnorm2;   // ||b||^2
    double tol2;     // tol^2 ||b||^2
    double rmax2;    // largest ||r||^2 since the last reliable update
    double rho_prev; // rho of the previous iteration
    int active;      // iterating
    int iters;       // A-applies inside the loop so far
    int maxit;
    int flag;        // 1: FP32 residual fell below tol (mixed: wants a reliable update)
};

__global__ void k_cg_setup(CGCol* st, const double* rho, const double* bn, int k, double tol, int maxit, int first) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    CGCol c = st[j];
    if (first) {
        c.iters = 0;
        c.bnorm2 = bn[j];
        c.tol2 = tol * tol * bn[j];
        c.maxit = maxit;
    }
    c.rho = rho[j];
    c.rho_prev = rho[j];
    c.rmax2 = rho[j];
    c.alpha = c.beta = 0.0;
    c.flag = 0;
    c.active = (c.bnorm2 > 0.0) && (c.rho > c.tol2) && (c.iters < c.maxit) && isfinite(c.rho);
    st[j] = c;
}

// alpha = rho / Re<p, q>
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cg_alpha(const R* __restrict__ p, const R* __restrict__ q, int64_t ld,
                                                     int64_t N, CGCol* st, double* part, unsigned* ctr) {
    __shared__ double sh[kWaves];
    const int col = blockIdx.y;
    if (!st[col].active) return;
    const R* pc = p + col * ld;
    const R* qc = q + col * ld;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock)
        acc += (double)pc[i] * (double)qc[i];
    double tot;
    if (split_reduce(acc, part + (int64_t)col * gridDim.x, ctr + col, &tot, sh) && threadIdx.x == 0)
        st[col].alpha = st[col].rho / tot;
}

// x += alpha p; r -= alpha q; rho_new = ||r||^2; convergence and beta
template <typename XT, typename R>
__global__ __launch_bounds__(kBlock) void k_cg_xr(XT* __restrict__ x, int64_t ldx, R* __restrict__ r,
                                                  const R* __restrict__ p, const R* __restrict__ q, int64_t ld,
                                                  int64_t N, CGCol* st, int mixed, double* part, unsigned* ctr) {
    __shared__ double sh[kWaves];
    const int col = blockIdx.y;
    if (!st[col].active) return;
    const double a = st[col].alpha;
    const R aR = (R)a;
    XT* xc = x + col * ldx;
    R* rc = r + col * ld;
    const R* pc = p + col * ld;
    const R* qc = q + col * ld;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock) {
        xc[i] = (XT)(xc[i] + (XT)aR * (XT)pc[i]);
        const R rv = rc[i] - aR * qc[i];
        rc[i] = rv;
        acc += (double)rv * (double)rv;
    }
    double tot;
    if (split_reduce(acc, part + (int64_t)col * gridDim.x, ctr + col, &tot, sh) && threadIdx.x == 0) {
        CGCol c = st[col];
        c.iters += 1;
        c.rho_prev = c.rho;
        c.rho = tot;
        c.beta = tot / c.rho_prev;
        c.rmax2 = fmax(c.rmax2, tot);
        if (!(tot > c.tol2) || !isfinite(tot)) {
            c.flag = 1;          // recursive residual at tol (mixed: verify with an update)
            c.active = 0;
        } else if (mixed && tot < 0.01 * c.rmax2) {
            c.flag = 2;          // FP32 residual fell 10x: pause for a reliable update
            c.active = 0;
        }
        if (c.iters >= c.maxit) c.active = 0;
        st[col] = c;
    }
}

// p = r + beta p
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cg_p(R* __restrict__ p, const R* __restrict__ r, int64_t ld, int64_t N,
                                                 const CGCol* st) {
    const int col = blockIdx.y;
    if (!st[col].active) return;
    const R b = (R)st[col].beta;
    R* pc = p + col * ld;
    const R* rc = r + col * ld;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock)
        pc[i] = rc[i] + b * pc[i];
}

// ----------------------------------------------------------------------------
struct CGWork {
    void* r;       // k x N2 (vector precision)
    void* p;
    void* q;
    void* tmp;     // op scratch, k columns (vector precision)
    void* xs;      // mixed: FP32 increment of x (k x N2)
    double* r64;   // mixed: FP64 true residual (k x N2)
    double* ax64;  // A x in FP64 (k x N2)
    void* tmp64;   // FP64 op scratch (k columns)
    double* part;
    unsigned* ctr;
    CGCol* st;
    double* rho;
    double* bn;
};

static CGWork carve_cg(Carver& c, const sc_op* op, int k, bool mixed) {
    const bool cpl = is_complex(op->dtype);
    const int64_t N2 = op->n * (cpl ? 2 : 1);
    const size_t vb = mixed ? 4 : 8;
    const int64_t tmpn = std::max<int64_t>(op_apply_tmp_elems(op) * (cpl ? 2 : 1), 1);
    CGWork w{};
    w.r = c.take<char>(N2 * k * vb);
    w.p = c.take<char>(N2 * k * vb);
    w.q = c.take<char>(N2 * k * vb);
    w.tmp = c.take<char>(tmpn * k * vb);
    if (mixed) {
        w.xs = c.take<float>(N2 * k);
        w.r64 = c.take<double>(N2 * k);
    }
    w.ax64 = c.take<double>(N2 * k);
    w.tmp64 = c.take<double>(tmpn * k);
    w.part = c.take<double>((size_t)kMaxRedBlocks * k);
    w.ctr = c.take<unsigned>(k);
    w.st = c.take<CGCol>(k);
    w.rho = c.take<double>(k);
    w.bn = c.take<double>(k);
    return w;
}

size_t cg_workspace(const sc_op* op, int k, bool mixed) {
    Carver c(nullptr, 0);
    carve_cg(c, op, k, mixed);
    return c.off + 256;
}

// r64 = b - A x (FP64), rr[j] = ||r64_j||^2
static sc_status true_residual(const sc_op* op, const double* B, int64_t ldb2, const double* X, int64_t ldx2,
                               int k, const CGWork& w, double* r64, double* rr, hipStream_t s) {
    const bool cpl = is_complex(op->dtype);
    const int64_t N2 = op->n * (cpl ? 2 : 1);
    const int64_t div = cpl ? 2 : 1;
    SC_TRY(op_apply(op, false, X, ldx2 / div, w.ax64, op->n, k, w.tmp64, s));
    SC_TRY(lincomb(0, r64, N2, 0, B, ldb2, 0, w.ax64, N2, N2, k, 1.0, -1.0, s));
    SC_TRY(dot(0, r64, N2, 0, r64, N2, N2, k, rr, w.part, w.ctr, s));
    return SC_OK;
}

template <typename R>
static sc_status cg_run(const sc_op* op, bool mixed, const double* B, int64_t ldb, double* X, int64_t ldx, int k,
                        double tol, int maxit, int* iters, double* relres, const CGWork& w, hipStream_t s,
                        sc_status* result) {
    const bool cpl = is_complex(op->dtype);
    const int64_t N2 = op->n * (cpl ? 2 : 1);
    const int64_t mul = cpl ? 2 : 1;
    const int64_t ldb2 = ldb * mul, ldx2 = ldx * mul;
    const int vt = mixed ? 1 : 0;
    R* r = (R*)w.r;
    R* p = (R*)w.p;
    R* q = (R*)w.q;
    const dim3 blk(kBlock);
    const int g = red_grid(N2);
    const dim3 grid(g, k);
    std::vector<CGCol> hst(k);
    std::vector<double> hrr(k);
    const int chunk = 8;

    SC_TRY(fill<unsigned>(w.ctr, k, 0u, s));
    SC_TRY(dot(0, B, ldb2, 0, B, ldb2, N2, k, w.bn, w.part, w.ctr, s));
    // r = b - A x; rho = ||r||^2
    double* r64 = mixed ? w.r64 : (double*)r;
    SC_TRY(true_residual(op, B, ldb2, X, ldx2, k, w, r64, w.rho, s));
    if (mixed) {
        SC_TRY(lincomb(1, r, N2, 0, r64, N2, 0, nullptr, 0, N2, k, 1.0, 0.0, s));
        SC_TRY(fill<float>((float*)w.xs, N2 * k, 0.0f, s));
    }
    SC_TRY(lincomb(vt, p, N2, vt, r, N2, 0, nullptr, 0, N2, k, 1.0, 0.0, s));
    hipLaunchKernelGGL(k_cg_setup, dim3((k + 63) / 64), dim3(64), 0, s, w.st, w.rho, w.bn, k, tol, maxit, 1);
    SC_LAUNCH_CHECK();

    // columns with b = 0 are solved by x = 0
    SC_HIP(hipMemcpyAsync(hst.data(), w.st, sizeof(CGCol) * k, hipMemcpyDeviceToHost, s));
    SC_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < k; ++j)
        if (!(hst[j].bnorm2 > 0.0)) SC_TRY(lincomb(0, X + j * ldx2, N2, 0, X + j * ldx2, N2, 0, nullptr, 0, N2, 1, 0.0, 0.0, s));

    int restarts = 0;
    for (;;) {
        bool any = false;
        for (int j = 0; j < k; ++j) any |= hst[j].active != 0;
        while (any) {
            for (int it = 0; it < chunk; ++it) {
                SC_TRY(op_apply(op, mixed, p, op->n, q, op->n, k, w.tmp, s));
                hipLaunchKernelGGL(k_cg_alpha<R>, grid, blk, 0, s, p, q, N2, N2, w.st, w.part, w.ctr);
                SC_LAUNCH_CHECK();
                if (mixed)
                    hipLaunchKernelGGL((k_cg_xr<float, R>), grid, blk, 0, s, (float*)w.xs, N2, r, p, q, N2, N2, w.st, 1,
                                       w.part, w.ctr);
                else
                    hipLaunchKernelGGL((k_cg_xr<double, R>), grid, blk, 0, s, X, ldx2, r, p, q, N2, N2, w.st, 0,
                                       w.part, w.ctr);
                SC_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_cg_p<R>, grid, blk, 0, s, p, r, N2, N2, w.st);
                SC_LAUNCH_CHECK();
            }
            SC_HIP(hipMemcpyAsync(hst.data(), w.st, sizeof(CGCol) * k, hipMemcpyDeviceToHost, s));
            SC_HIP(hipStreamSynchronize(s));
            any = false;
            bool upd = false;
            for (int j = 0; j < k; ++j) {
                any |= hst[j].active != 0;
                upd |= mixed && hst[j].flag != 0 && hst[j].iters < hst[j].maxit;
            }
            if (mixed && upd) {
                // reliable update of the paused columns: x64 += xs; r64 = b - A x64; r = r64; xs = 0
                for (int j = 0; j < k; ++j) {
                    if (!hst[j].flag || hst[j].iters >= hst[j].maxit) continue;
                    float* xs = (float*)w.xs + j * N2;
                    SC_TRY(lincomb(0, X + j * ldx2, N2, 0, X + j * ldx2, N2, 1, xs, N2, N2, 1, 1.0, 1.0, s));
                    SC_TRY(fill<float>(xs, N2, 0.0f, s));
                }
                SC_TRY(true_residual(op, B, ldb2, X, ldx2, k, w, w.r64, w.rho, s));
                SC_HIP(hipMemcpyAsync(hrr.data(), w.rho, sizeof(double) * k, hipMemcpyDeviceToHost, s));
                SC_HIP(hipStreamSynchronize(s));
                for (int j = 0; j < k; ++j) {
                    CGCol& c = hst[j];
                    if (!c.flag || c.iters >= c.maxit) continue;
                    R* rj = r + j * N2;
                    R* pj = p + j * N2;
                    SC_TRY(lincomb(1, rj, N2, 0, w.r64 + j * N2, N2, 0, nullptr, 0, N2, 1, 1.0, 0.0, s));
                    const bool done = !(hrr[j] > c.tol2);
                    if (!done) {
                        // flag 1: the FP32 recurrence drifted below tol; restart the direction.
                        // flag 2: continue CG with the true residual: p = r + (rho_true / rho_prev) p.
                        const double b = c.flag == 1 ? 0.0 : hrr[j] / c.rho_prev;
                        SC_TRY(lincomb(1, pj, N2, 1, rj, N2, 1, pj, N2, N2, 1, 1.0, b, s));
                    }
                    c.rho = hrr[j];
                    c.rho_prev = hrr[j];
                    c.rmax2 = hrr[j];
                    c.active = done ? 0 : 1;
                    c.flag = 0;
                    any |= c.active != 0;
                }
                SC_HIP(hipMemcpyAsync(w.st, hst.data(), sizeof(CGCol) * k, hipMemcpyHostToDevice, s));
                SC_HIP(hipStreamSynchronize(s));
            }
        }
        if (mixed) {
            // fold any remaining FP32 increment into x
            SC_TRY(lincomb(0, X, ldx2, 0, X, ldx2, 1, w.xs, N2, N2, k, 1.0, 1.0, s));
            SC_TRY(fill<float>((float*)w.xs, N2 * k, 0.0f, s));
        }
        // verify on the true residual
        SC_TRY(true_residual(op, B, ldb2, X, ldx2, k, w, mixed ? w.r64 : (double*)r, w.rho, s));
        SC_HIP(hipMemcpyAsync(hrr.data(), w.rho, sizeof(double) * k, hipMemcpyDeviceToHost, s));
        SC_HIP(hipStreamSynchronize(s));
        bool again = false;
        for (int j = 0; j < k; ++j) {
            const double bn = hst[j].bnorm2;
            relres[j] = bn > 0.0 ? std::sqrt(hrr[j] / bn) : 0.0;
            iters[j] = hst[j].iters;
            if (bn > 0.0 && !(relres[j] <= tol) && hst[j].iters < maxit) again = true;
        }
        if (!again || restarts >= 5) break;
        ++restarts;
        // restart every column from its true residual (converged ones stay inactive)
        if (mixed) {
            SC_TRY(lincomb(1, r, N2, 0, w.r64, N2, 0, nullptr, 0, N2, k, 1.0, 0.0, s));
        }
        SC_TRY(lincomb(vt, p, N2, vt, r, N2, 0, nullptr, 0, N2, k, 1.0, 0.0, s));
        hipLaunchKernelGGL(k_cg_setup, dim3((k + 63) / 64), dim3(64), 0, s, w.st, w.rho, w.bn, k, tol, maxit, 0);
        SC_LAUNCH_CHECK();
        SC_HIP(hipMemcpyAsync(hst.data(), w.st, sizeof(CGCol) * k, hipMemcpyDeviceToHost, s));
        SC_HIP(hipStreamSynchronize(s));
    }
    *result = SC_OK;
    for (int j = 0; j < k; ++j)
        if (!(relres[j] <= tol)) *result = SC_NOT_CONVERGED;
    return SC_OK;
}

sc_status solve_cg(const sc_op* op, int mixed, const void* B, int64_t ldb, void* X, int64_t ldx, int k, double tol,
                   int maxit, int* iters, double* relres, void* work, size_t work_bytes, hipStream_t s) {
    Carver c(work, work_bytes);
    CGWork w = carve_cg(c, op, k, mixed != 0);
    if (!c.ok()) {
        set_error("solve_cg: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    sc_status result = SC_OK;
    if (mixed)
        SC_TRY(cg_run<float>(op, true, (const double*)B, ldb, (double*)X, ldx, k, tol, maxit, iters, relres, w, s, &result));
    else
        SC_TRY(cg_run<double>(op, false, (const double*)B, ldb, (double*)X, ldx, k, tol, maxit, iters, relres, w, s, &result));
    if (result == SC_NOT_CONVERGED) set_error("solve_cg: some right-hand side is above tol at maxit");
    return result;
}

}  // namespace sc
