// Single seeding of related right-hand sides (Section 2.3, the algorithm for
// related systems, steps 1-4).  System 1 is seeded by the Lanczos phase and
// finished with CG; the others are first projected over its basis.  Then the
// systems are solved in order, and after system j converges its CG correction
// x_cg = x^j - x^j_bcg (x^j_bcg: its guess before CG; for system 1 the seed
// started from zero, so the correction is its whole solution) seeds every
// later system i by a Galerkin projection over that one vector:
//   delta = (x_cg^H r^i) / (x_cg^H r^j_bcg),  x^i += delta x_cg,  r^i -= delta r^j_bcg,
// where r^j_bcg stands for A x_cg (the residual system j started CG from).
// The r^i are carried residuals, updated by these corrections only.
#include "sc_internal.h"

namespace sc {

namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

struct RelPlan {
    size_t v_off, a_off, b_off, seed_off, seed_bytes, proj_off, proj_bytes, cg_off, cg_bytes;
    size_t r_off, tmp_off, xb_off, rb_off, xc_off, g_off, part_off, total;
    sc_dtype vdt;
};

constexpr int kRelCols = 31;  // later systems per contraction (plus r_bcg: 32 columns)

RelPlan plan(const sc_op* op, int k, int m, bool mixed) {
    RelPlan p{};
    const bool cpl = is_complex(op->dtype);
    const size_t eb = dtype_bytes(op->dtype);
    p.vdt = mixed ? single_of(op->dtype) : op->dtype;
    size_t off = 0;
    p.v_off = off;
    off = al256(off + (size_t)(m + 1) * op->n * dtype_bytes(p.vdt));
    p.a_off = off;
    off = al256(off + (size_t)m * 8);
    p.b_off = off;
    off = al256(off + (size_t)(m + 1) * 8);
    p.seed_off = off;
    p.seed_bytes = seed_workspace(op, m, mixed);
    off = al256(off + p.seed_bytes);
    p.proj_off = off;
    p.proj_bytes = project_workspace(op->n, m, k - 1, cpl);
    off = al256(off + p.proj_bytes);
    p.cg_off = off;
    p.cg_bytes = cg_workspace(op, k, mixed);
    off = al256(off + p.cg_bytes);
    p.r_off = off;  // carried residuals, n x k
    off = al256(off + (size_t)k * op->n * eb);
    p.tmp_off = off;  // A X and the operator's scratch, 2 n x k
    off = al256(off + 2 * (size_t)k * op->n * eb);
    p.xb_off = off;
    off = al256(off + op->n * eb);
    p.rb_off = off;
    off = al256(off + op->n * eb);
    p.xc_off = off;
    off = al256(off + op->n * eb);
    p.g_off = off;
    off = al256(off + 2 * 8 * (kRelCols + 1));
    p.part_off = off;
    off = al256(off + 8 * gemm_cn_part_doubles(op->n, 1, kRelCols + 1, cpl));
    p.total = off + 256;
    return p;
}

// X_c += d_c xcg; R_c -= d_c rbcg with d_c = G[1 + c] / G[0] (0 when G[0] = 0)
__global__ __launch_bounds__(kBlock) void k_rank1(const double* __restrict__ G, bool cpl,
                                                  const double* __restrict__ xcg, const double* __restrict__ rbcg,
                                                  ColPtrs<void> X, ColPtrs<void> R, int64_t n) {
    const int c = blockIdx.y;
    double dr, di = 0.0;
    if (cpl) {
        const double ar = G[0], ai = G[1], br = G[2 * (c + 1)], bi = G[2 * (c + 1) + 1];
        const double den = ar * ar + ai * ai;
        dr = den > 0.0 ? (br * ar + bi * ai) / den : 0.0;  // b / a
        di = den > 0.0 ? (bi * ar - br * ai) / den : 0.0;
    } else {
        dr = G[0] != 0.0 ? G[c + 1] / G[0] : 0.0;
    }
    double* x = (double*)X.p[c];
    double* r = (double*)R.p[c];
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        if (cpl) {
            const double xr = xcg[2 * i], xi = xcg[2 * i + 1], rr = rbcg[2 * i], ri = rbcg[2 * i + 1];
            x[2 * i] += dr * xr - di * xi;
            x[2 * i + 1] += dr * xi + di * xr;
            r[2 * i] -= dr * rr - di * ri;
            r[2 * i + 1] -= dr * ri + di * rr;
        } else {
            x[i] += dr * xcg[i];
            r[i] -= dr * rbcg[i];
        }
    }
}

}  // namespace

size_t related_workspace(const sc_op* op, int k, int m, bool mixed) {
    return plan(op, std::max(k, 1), std::max(m, 1), mixed).total;
}

sc_status related_solve(const sc_op* op, int mixed, const void* B, int64_t ldb, void* X, int64_t ldx, int k, int m,
                        int freq, double tol, int maxit, int* iters, double* relres, int* m_done, void* work,
                        size_t work_bytes, hipStream_t s) {
    const RelPlan p = plan(op, k, m, mixed != 0);
    char* base = (char*)(((uintptr_t)work + 255) & ~uintptr_t(255));
    if ((size_t)(base - (char*)work) + p.total - 256 > work_bytes) {
        set_error("related_solve: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    const bool cpl = is_complex(op->dtype);
    const int64_t mul = cpl ? 2 : 1;
    const int64_t N2 = op->n * mul, ldb2 = ldb * mul, ldx2 = ldx * mul;
    const double* Bd = (const double*)B;
    double* Xd = (double*)X;
    double* R = (double*)(base + p.r_off);
    double* AX = (double*)(base + p.tmp_off);
    double* OT = AX + (size_t)k * N2;
    double* xb = (double*)(base + p.xb_off);
    double* rb = (double*)(base + p.rb_off);
    double* xc = (double*)(base + p.xc_off);
    double* G = (double*)(base + p.g_off);
    double* part = (double*)(base + p.part_off);
    double* alpha = (double*)(base + p.a_off);
    double* beta = (double*)(base + p.b_off);
    void* V = base + p.v_off;

    // steps 1-2: seed on system 1 from x = 0, project the others over its basis
    SC_TRY(fill<double>(Xd, (k - 1) * ldx2 + N2, 0.0, s));
    bool ok = false;
    SeedWork sw = seed_carve(base + p.seed_off, p.seed_bytes, op, m, mixed != 0, &ok);
    if (!ok) {
        set_error("related_solve: seed workspace carving failed");
        return SC_ERR_WORKSPACE;
    }
    SC_TRY(seed_pretune(op, mixed != 0, sw, s));
    SC_TRY(seed_enqueue_any(op, B, X, m, freq, V, op->n, p.vdt, alpha, beta, sw, s));
    sc_status seed_status = SC_OK;
    SC_TRY(seed_finalize_any(op, X, V, op->n, p.vdt, alpha, beta, m_done, sw, s, &seed_status));
    if (seed_status == SC_ERR_NOT_PD || seed_status == SC_ERR_NONFINITE) {
        set_error("related_solve: the seed phase stopped (operator not positive definite or non-finite values)");
        return seed_status;
    }
    const size_t eb = dtype_bytes(op->dtype);
    if (k > 1 && *m_done >= 1)
        SC_TRY(project_impl(op->n, V, op->n, p.vdt, *m_done, alpha, beta, op->dtype, (const char*)B + ldb * eb, ldb,
                            k - 1, (char*)X + ldx * eb, ldx, base + p.proj_off, p.proj_bytes, s));
    void* cgw = base + p.cg_off;
    sc_status out = SC_OK;
    auto cg1 = [&](int j) -> sc_status {
        sc_status r = solve_cg(op, mixed, (const char*)B + j * ldb * eb, ldb, (char*)X + j * ldx * eb, ldx, 1, tol,
                               maxit, iters + j, relres + j, cgw, p.cg_bytes, s);
        if (r == SC_NOT_CONVERGED) out = SC_NOT_CONVERGED;
        return r < 0 ? r : SC_OK;
    };
    SC_TRY(cg1(0));
    iters[0] += *m_done;
    if (k > 1) {
        // carried residuals of the projected guesses: R = B - A X (FP64)
        SC_TRY(op_apply(op, false, X, ldx, AX, op->n, k, OT, s));
        SC_TRY(lincomb(0, R, N2, 0, B, ldb2, 0, AX, N2, N2, k, 1.0, -1.0, s));
    }
    for (int j = 0; j < k; ++j) {
        if (j > 0) {
            // step 4: system j starts CG from its carried guess and residual
            SC_TRY(lincomb(0, xb, N2, 0, Xd + j * ldx2, ldx2, 0, nullptr, 0, N2, 1, 1.0, 0.0, s));
            SC_TRY(lincomb(0, rb, N2, 0, R + j * N2, N2, 0, nullptr, 0, N2, 1, 1.0, 0.0, s));
            SC_TRY(cg1(j));
        } else {
            SC_TRY(fill<double>(xb, N2, 0.0, s));
            SC_TRY(lincomb(0, rb, N2, 0, Bd, ldb2, 0, nullptr, 0, N2, 1, 1.0, 0.0, s));
        }
        if (j == k - 1) break;
        // step 3: project the later systems over x_cg = x^j - x^j_bcg
        SC_TRY(lincomb(0, xc, N2, 0, Xd + j * ldx2, ldx2, 0, xb, N2, N2, 1, 1.0, -1.0, s));
        for (int i0 = j + 1; i0 < k; i0 += kRelCols) {
            const int nc = std::min(kRelCols, k - i0);
            ColPtrs<const void> wc{};
            wc.p[0] = rb;
            ColPtrs<void> xp{}, rp{};
            for (int c = 0; c < nc; ++c) {
                wc.p[1 + c] = R + (i0 + c) * N2;
                xp.p[c] = Xd + (i0 + c) * ldx2;
                rp.p[c] = R + (i0 + c) * N2;
            }
            SC_TRY(gemm_cn(cpl, false, xc, op->n, op->n, 1, false, wc, nc + 1, G, part, nullptr, s));
            hipLaunchKernelGGL(k_rank1, dim3((unsigned)red_grid(op->n, 4), (unsigned)nc), dim3(kBlock), 0, s, G, cpl,
                               xc, rb, xp, rp, op->n);
            SC_LAUNCH_CHECK();
        }
    }
    SC_HIP(hipStreamSynchronize(s));
    if (out == SC_OK && seed_status == SC_BREAKDOWN) out = SC_BREAKDOWN;
    if (out == SC_NOT_CONVERGED) set_error("related_solve: some right-hand side is above tol at maxit");
    return out;
}

}  // namespace sc
