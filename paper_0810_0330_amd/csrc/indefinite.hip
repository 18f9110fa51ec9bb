// The indefinite variant of the single-seed method, for Q = gamma_5 D
// (Hermitian indefinite; Section 4 names this alternative to A^H A, Section 3
// the QR factorization of the Lanczos tridiagonal matrix it needs):
//   1. the Lanczos part of the seed algorithm (steps 1, 2, 5, 8, 9) on column 0
//      of B from x = 0 (no LU pivots: the seed loop is told to skip the
//      positive-pivot check, so any Hermitian op can be used);
//   2. minimum-residual guesses over the basis for every column:
//      x^j = V_m y_j, y_j = argmin || c_j - T~_m y || with T~_m the (m+1) x m
//      tridiagonal matrix, c_j = V_{m+1}^H b^j and c_1 = beta_0 e_1, solved by
//      the QR factorization of T~_m (tridiag_lsq);
//   3. MINRES from those guesses for every column.
#include "sc_internal.h"

namespace sc {

namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

struct IndefPlan {
    size_t v_off, a_off, b_off, seed_off, seed_bytes, c_off, lsq_off, part_off, mr_off, mr_bytes, total;
    int ngroups;
};

IndefPlan plan(const sc_op* op, int k, int m) {
    IndefPlan p{};
    const bool cpl = is_complex(op->dtype);
    p.ngroups = (k + kMaxCols - 1) / kMaxCols;
    size_t off = 0;
    p.v_off = off;
    off = al256(off + (size_t)(m + 1) * op->n * dtype_bytes(op->dtype));
    p.a_off = off;
    off = al256(off + (size_t)m * 8);
    p.b_off = off;
    off = al256(off + (size_t)(m + 1) * 8);
    p.seed_off = off;
    p.seed_bytes = seed_workspace(op, m, false);
    off = al256(off + p.seed_bytes);
    p.c_off = off;  // c_j = V_{m+1}^H b^j per group: (m+1) x kMaxCols complex
    off = al256(off + (size_t)p.ngroups * (m + 1) * kMaxCols * 2 * 8);
    p.lsq_off = off;
    off = al256(off + (size_t)m * 5 * 8);
    p.part_off = off;
    off = al256(off + gemm_cn_part_doubles(op->n, m + 1, kMaxCols, cpl) * 8);
    p.mr_off = off;
    p.mr_bytes = minres_workspace(op, k);
    off = al256(off + p.mr_bytes);
    p.total = off + 256;
    return p;
}

// column 0 of C (rows x nc elements of es doubles, row-major) = beta_0 e_1
__global__ void k_col0_e1(double* C, int rows, int nc, int es, const double* beta0) {
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < rows; a += gridDim.x * blockDim.x)
        for (int e = 0; e < es; ++e) C[((int64_t)a * nc) * es + e] = (a == 0 && e == 0) ? *beta0 : 0.0;
}

}  // namespace

size_t indefinite_workspace(const sc_op* op, int k, int m) { return plan(op, std::max(k, 1), std::max(m, 1)).total; }

sc_status indefinite_solve(const sc_op* op, const void* B, int64_t ldb, void* X, int64_t ldx, int k, int m, int freq,
                           double tol, int maxit, int* iters, double* relres, int* m_done, void* work,
                           size_t work_bytes, hipStream_t s) {
    const IndefPlan p = plan(op, k, m);
    char* base = (char*)(((uintptr_t)work + 255) & ~uintptr_t(255));
    if ((size_t)(base - (char*)work) + p.total - 256 > work_bytes) {
        set_error("indefinite_solve: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    const bool cpl = is_complex(op->dtype);
    const int64_t mul = cpl ? 2 : 1;
    const int64_t N2 = op->n * mul, ldx2 = ldx * mul;
    const size_t eb = dtype_bytes(op->dtype);
    double* alpha = (double*)(base + p.a_off);
    double* beta = (double*)(base + p.b_off);
    double* lsq = (double*)(base + p.lsq_off);
    double* part = (double*)(base + p.part_off);
    void* V = base + p.v_off;
    auto Cg = [&](int g) { return (double*)(base + p.c_off) + (size_t)g * (m + 1) * kMaxCols * 2; };

    SC_TRY(fill<double>((double*)X, (k - 1) * ldx2 + N2, 0.0, s));
    bool ok = false;
    SeedWork sw = seed_carve(base + p.seed_off, p.seed_bytes, op, m, false, &ok);
    if (!ok) {
        set_error("indefinite_solve: seed workspace carving failed");
        return SC_ERR_WORKSPACE;
    }
    SC_TRY(seed_pretune(op, false, sw, s));
    SC_TRY(seed_enqueue_any(op, B, X, m, freq, V, op->n, op->dtype, alpha, beta, sw, s, true));
    sc_status seed_status = SC_OK;
    SC_TRY(seed_finalize_any(op, X, V, op->n, op->dtype, alpha, beta, m_done, sw, s, &seed_status, false));
    if (seed_status == SC_ERR_NONFINITE || seed_status == SC_ERR_NOT_PD) {
        set_error("indefinite_solve: the seed phase stopped (non-finite values)");
        return seed_status;
    }
    const int md = *m_done;
    if (md >= 1) {
        for (int g = 0; g < p.ngroups; ++g) {
            const int nc = std::min(kMaxCols, k - g * kMaxCols);
            ColPtrs<const void> wc{};
            ColPtrs<void> xc{};
            for (int j = 0; j < nc; ++j) {
                wc.p[j] = (const char*)B + (size_t)(g * kMaxCols + j) * ldb * eb;
                xc.p[j] = (char*)X + (size_t)(g * kMaxCols + j) * ldx * eb;
            }
            double* C = Cg(g);
            SC_TRY(gemm_cn(cpl, false, V, op->n, op->n, md + 1, false, wc, nc, C, part, nullptr, s));
            if (g == 0) {
                hipLaunchKernelGGL(k_col0_e1, dim3((md + 1 + 255) / 256), dim3(256), 0, s, C, md + 1, nc, (int)mul,
                                   beta);
                SC_LAUNCH_CHECK();
            }
            SC_TRY(tridiag_lsq(alpha, beta, md, C, nc, cpl, lsq, s));
            SC_TRY(gemm_nn(cpl, false, V, op->n, op->n, md, C, nc, false, xc, 1.0, nullptr, s));
        }
    }
    sc_status out = minres_solve(op, B, ldb, X, ldx, k, tol, maxit, iters, relres, base + p.mr_off, p.mr_bytes, s);
    if (out < 0) return out;
    iters[0] += md;
    if (out == SC_OK && seed_status == SC_BREAKDOWN) out = SC_BREAKDOWN;
    return out;
}

}  // namespace sc
