// Standard (multiple) seed CG, the comparator the paper argues against
// (Section 2.1, after Chan and Wan; Example 1, Table 2.1).  The systems are
// solved in order by CG; during the solve of system j every later system i is
// projected over each new A-conjugate direction p (q = A p):
//   c = (p^H r^i) / (p^H q),  x^i += c p,  r^i -= c q,
// so that system i starts its own CG from a guess that is Galerkin over the
// Krylov spaces of all earlier systems.  FP64 throughout; the host reads two
// scalars per iteration.
#include <cmath>
#include <vector>

#include "sc_internal.h"

namespace sc {

namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr int kMsCols = 32;  // later systems per contraction

struct MsPlan {
    size_t r_off, x_off, rr_off, p_off, q_off, tmp_off, g_off, part_off, gpart_off, s_off, total;
};

MsPlan plan(const sc_op* op, int k) {
    MsPlan p{};
    const size_t eb = dtype_bytes(op->dtype);
    const size_t vec = op->n * eb;
    size_t off = 0;
    p.r_off = off;  // carried residuals of all systems, n x k
    off = al256(off + (size_t)k * vec);
    p.x_off = off;
    off = al256(off + vec);
    p.rr_off = off;
    off = al256(off + vec);
    p.p_off = off;
    off = al256(off + vec);
    p.q_off = off;
    off = al256(off + vec);
    p.tmp_off = off;  // the operator's scratch (and A x at the start)
    off = al256(off + 2 * vec);
    p.g_off = off;
    off = al256(off + 2 * 8 * kMsCols);
    p.part_off = off;
    off = al256(off + 8 * (size_t)kMaxRedBlocks);
    p.gpart_off = off;
    off = al256(off + 8 * gemm_cn_part_doubles(op->n, 1, kMsCols, is_complex(op->dtype)));
    p.s_off = off;  // device scalars
    off = al256(off + 4 * 8);
    p.total = off + 256;
    return p;
}

// X_c += (G_c / pq) p; R_c -= (G_c / pq) q for the listed later systems
__global__ __launch_bounds__(kBlock) void k_ms_update(const double* __restrict__ G, bool cpl,
                                                      const double* __restrict__ pq, const double* __restrict__ p,
                                                      const double* __restrict__ q, ColPtrs<void> X, ColPtrs<void> R,
                                                      int64_t n) {
    const int c = blockIdx.y;
    const double inv = 1.0 / pq[0];
    const double cr = (cpl ? G[2 * c] : G[c]) * inv, ci = cpl ? G[2 * c + 1] * inv : 0.0;
    double* x = (double*)X.p[c];
    double* r = (double*)R.p[c];
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        if (cpl) {
            const double pr = p[2 * i], pi = p[2 * i + 1], qr = q[2 * i], qi = q[2 * i + 1];
            x[2 * i] += cr * pr - ci * pi;
            x[2 * i + 1] += cr * pi + ci * pr;
            r[2 * i] -= cr * qr - ci * qi;
            r[2 * i + 1] -= cr * qi + ci * qr;
        } else {
            x[i] += cr * p[i];
            r[i] -= cr * q[i];
        }
    }
}

}  // namespace

size_t multiseed_workspace(const sc_op* op, int k) { return plan(op, std::max(k, 1)).total; }

sc_status multiseed_solve(const sc_op* op, const void* B, int64_t ldb, void* X, int64_t ldx, int k, double tol,
                          int maxit, int* iters, double* relres, void* work, size_t work_bytes, hipStream_t s) {
    const MsPlan pl = plan(op, k);
    char* base = (char*)(((uintptr_t)work + 255) & ~uintptr_t(255));
    if ((size_t)(base - (char*)work) + pl.total - 256 > work_bytes) {
        set_error("multiple_seed_solve: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    const bool cpl = is_complex(op->dtype);
    const int64_t mul = cpl ? 2 : 1;
    const int64_t N2 = op->n * mul, ldb2 = ldb * mul, ldx2 = ldx * mul;
    const double* Bd = (const double*)B;
    double* Xd = (double*)X;
    double* R = (double*)(base + pl.r_off);
    double* x = (double*)(base + pl.x_off);
    double* r = (double*)(base + pl.rr_off);
    double* p = (double*)(base + pl.p_off);
    double* q = (double*)(base + pl.q_off);
    double* tmp = (double*)(base + pl.tmp_off);
    double* G = (double*)(base + pl.g_off);
    double* part = (double*)(base + pl.part_off);
    double* gpart = (double*)(base + pl.gpart_off);
    double* dv = (double*)(base + pl.s_off);  // [0] pq, [1] rho, [2] ||b||^2
    SC_TRY(fill<double>(Xd, (k - 1) * ldx2 + N2, 0.0, s));
    SC_TRY(lincomb(0, R, N2, 0, Bd, ldb2, 0, nullptr, 0, N2, k, 1.0, 0.0, s));  // X = 0: r^i = b^i
    sc_status out = SC_OK;
    for (int j = 0; j < k; ++j) {
        double* xj = Xd + j * ldx2;
        // r = b - A x from the guess the earlier systems built (FP64, true residual)
        SC_TRY(op_apply(op, false, xj, ldx, tmp, op->n, 1, tmp + N2, s));
        SC_TRY(lincomb(0, r, N2, 0, Bd + j * ldb2, ldb2, 0, tmp, N2, N2, 1, 1.0, -1.0, s));
        SC_TRY(lincomb(0, x, N2, 0, xj, ldx2, 0, nullptr, 0, N2, 1, 1.0, 0.0, s));
        SC_TRY(lincomb(0, p, N2, 0, r, N2, 0, nullptr, 0, N2, 1, 1.0, 0.0, s));
        SC_TRY(dot(0, Bd + j * ldb2, ldb2, 0, Bd + j * ldb2, ldb2, N2, 1, dv + 2, part, nullptr, s));
        SC_TRY(dot(0, r, N2, 0, r, N2, N2, 1, dv + 1, part, nullptr, s));
        double h[3];
        SC_HIP(hipMemcpyAsync(h, dv, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        SC_HIP(hipStreamSynchronize(s));
        double rho = h[1];
        const double bn2 = h[2];
        const double tol2 = tol * tol * bn2;
        int it = 0;
        while (bn2 > 0.0 && rho > tol2 && it < maxit) {
            SC_TRY(op_apply(op, false, p, op->n, q, op->n, 1, tmp, s));
            SC_TRY(dot(0, p, N2, 0, q, N2, N2, 1, dv, part, nullptr, s));
            SC_HIP(hipMemcpyAsync(h, dv, sizeof(double), hipMemcpyDeviceToHost, s));
            SC_HIP(hipStreamSynchronize(s));
            const double pq = h[0];
            if (!(pq > 0.0) || !std::isfinite(pq)) {
                set_error("multiple_seed_solve: p^H A p is not positive");
                return SC_ERR_NOT_PD;
            }
            const double a = rho / pq;
            SC_TRY(lincomb(0, x, N2, 0, x, N2, 0, p, N2, N2, 1, 1.0, a, s));
            SC_TRY(lincomb(0, r, N2, 0, r, N2, 0, q, N2, N2, 1, 1.0, -a, s));
            // project the later systems over this direction
            for (int i0 = j + 1; i0 < k; i0 += kMsCols) {
                const int nc = std::min(kMsCols, k - i0);
                ColPtrs<const void> wc{};
                ColPtrs<void> xp{}, rp{};
                for (int c = 0; c < nc; ++c) {
                    wc.p[c] = R + (i0 + c) * N2;
                    xp.p[c] = Xd + (i0 + c) * ldx2;
                    rp.p[c] = R + (i0 + c) * N2;
                }
                SC_TRY(gemm_cn(cpl, false, p, op->n, op->n, 1, false, wc, nc, G, gpart, nullptr, s));
                hipLaunchKernelGGL(k_ms_update, dim3((unsigned)red_grid(op->n, 4), (unsigned)nc), dim3(kBlock), 0, s,
                                   G, cpl, dv, p, q, xp, rp, op->n);
                SC_LAUNCH_CHECK();
            }
            SC_TRY(dot(0, r, N2, 0, r, N2, N2, 1, dv + 1, part, nullptr, s));
            SC_HIP(hipMemcpyAsync(h + 1, dv + 1, sizeof(double), hipMemcpyDeviceToHost, s));
            SC_HIP(hipStreamSynchronize(s));
            const double rho_new = h[1];
            ++it;
            if (!(rho_new > tol2)) {
                rho = rho_new;
                break;
            }
            SC_TRY(lincomb(0, p, N2, 0, r, N2, 0, p, N2, N2, 1, 1.0, rho_new / rho, s));
            rho = rho_new;
        }
        SC_TRY(lincomb(0, xj, ldx2, 0, x, N2, 0, nullptr, 0, N2, 1, 1.0, 0.0, s));
        // true residual of the result
        SC_TRY(op_apply(op, false, xj, ldx, tmp, op->n, 1, tmp + N2, s));
        SC_TRY(lincomb(0, r, N2, 0, Bd + j * ldb2, ldb2, 0, tmp, N2, N2, 1, 1.0, -1.0, s));
        SC_TRY(dot(0, r, N2, 0, r, N2, N2, 1, dv + 1, part, nullptr, s));
        SC_HIP(hipMemcpyAsync(h + 1, dv + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        SC_HIP(hipStreamSynchronize(s));
        iters[j] = it;
        relres[j] = bn2 > 0.0 ? std::sqrt(h[1] / bn2) : 0.0;
        if (!(relres[j] <= tol)) out = SC_NOT_CONVERGED;
    }
    if (out == SC_NOT_CONVERGED) set_error("multiple_seed_solve: some right-hand side is above tol");
    return out;
}

}  // namespace sc
