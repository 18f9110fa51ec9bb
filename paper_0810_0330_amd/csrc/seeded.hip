// The single-seed method as one call (Section 3 algorithm, steps 1-9, then
// Section 2.2): column 0 of B is the seed system, solved by m Lanczos steps
// from x = 0; columns 1..k-1 are seeded by the projection over its basis
// (steps 4 and 7, batched); then CG finishes every column from its guess.
//
// It differs from calling sc_seed_lanczos, sc_project and sc_solve_cg in turn
// only in how the work is laid out: x^1 = V T^{-1} (beta_0 e_1) of the seed
// system and the guesses V T^{-1} V^H b^j of the others are formed by one pass
// over the basis, with beta_0 e_1 as the first column of the coefficient
// block.  (Contracting V^H b^j on a second stream while the seed phase runs,
// every 128 steps over the vectors made final so far, was measured slower on
// the 16^3 x 32 workload: the one-column Lanczos passes lose more time to the
// shared chip than the contraction hides.)
#include "sc_internal.h"

namespace sc {

namespace {

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Systems whose vectors hold at most this many reals run their seed phase from
// a cached graph: each Lanczos step is then a chain of launches of a few
// microseconds of work, and the launches, not the kernels, set its time.
constexpr int64_t kSeedGraphMax = int64_t(1) << 20;

struct SeededPlan {
    size_t v_off, a_off, b_off, seed_off, seed_bytes, g_off, y_off, part_off, trid_off, cg_off, cg_bytes, total;
    int ngroups;
    sc_dtype vdt;
};

// Column groups of at most kMaxCols solution columns; group 0 holds the seed
// system (its coefficient column is beta_0 e_1) and the first kMaxCols - 1
// other systems.
int group_cols(int k, int g) { return std::min(kMaxCols, k - g * kMaxCols); }

SeededPlan plan(const sc_op* op, int k, int m, bool mixed) {
    SeededPlan p{};
    const bool cpl = is_complex(op->dtype);
    p.vdt = mixed ? single_of(op->dtype) : op->dtype;
    p.ngroups = (k + kMaxCols - 1) / kMaxCols;
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
    p.g_off = off;  // V^H b^j per group: m x kMaxCols (complex pairs)
    off = al256(off + (size_t)p.ngroups * m * kMaxCols * 2 * 8);
    p.y_off = off;  // group 0's coefficient block [beta_0 e_1 | V^H b^1..]
    off = al256(off + (size_t)m * kMaxCols * 2 * 8);
    p.part_off = off;
    off = al256(off + gemm_cn_part_doubles(op->n, m, kMaxCols, cpl) * 8);
    p.trid_off = off;
    off = al256(off + (size_t)m * 2 * 8);
    p.cg_off = off;
    p.cg_bytes = cg_workspace(op, k, mixed);
    off = al256(off + p.cg_bytes);
    p.total = off + 256;
    (void)cpl;
    return p;
}

// Y (M x N elements of es doubles, row-major): column 0 = beta_0 e_1, columns
// 1..N-1 = the contraction G (M x (N - 1)).
__global__ __launch_bounds__(kBlock) void k_seed_coeffs(double* __restrict__ Y, const double* __restrict__ G, int M,
                                                        int N, int es, const double* __restrict__ beta0) {
    const int64_t tot = (int64_t)M * N * es;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < tot; e += (int64_t)gridDim.x * kBlock) {
        const int64_t el = e / es;
        const int part = (int)(e % es);
        const int a = (int)(el / N), j = (int)(el % N);
        Y[e] = j == 0 ? ((a == 0 && part == 0) ? *beta0 : 0.0) : G[((int64_t)a * (N - 1) + (j - 1)) * es + part];
    }
}

}  // namespace

size_t seeded_workspace(const sc_op* op, int k, int m, bool mixed) {
    return plan(op, std::max(k, 1), std::max(m, 1), mixed).total;
}

sc_status seeded_solve(const sc_op* op, int mixed, const void* B, int64_t ldb, void* X, int64_t ldx, int k, int m,
                       int freq, double tol, int maxit, int* iters, double* relres, int* m_done, void* work,
                       size_t work_bytes, hipStream_t s) {
    const SeededPlan p = plan(op, k, m, mixed != 0);
    char* base = (char*)(((uintptr_t)work + 255) & ~uintptr_t(255));
    if ((size_t)(base - (char*)work) + p.total - 256 > work_bytes) {
        set_error("seeded_solve: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    const bool cpl = is_complex(op->dtype);
    const bool vs = is_single(p.vdt);
    const int64_t mul = cpl ? 2 : 1;
    const int64_t N2 = op->n * mul, ldx2 = ldx * mul;
    const size_t eb = dtype_bytes(op->dtype);
    double* alpha = (double*)(base + p.a_off);
    double* beta = (double*)(base + p.b_off);
    double* Gb = (double*)(base + p.g_off);
    double* Y0 = (double*)(base + p.y_off);
    double* part = (double*)(base + p.part_off);
    double* trid = (double*)(base + p.trid_off);
    void* V = base + p.v_off;
    auto Gg = [&](int g) { return Gb + (size_t)g * m * kMaxCols * 2; };
    // the right-hand columns contracted for group g, and where they start in B
    auto wcols = [&](int g) { return g == 0 ? group_cols(k, 0) - 1 : group_cols(k, g); };
    auto wfirst = [&](int g) { return g == 0 ? 1 : g * kMaxCols; };

    SC_TRY(fill<double>((double*)X, (k - 1) * ldx2 + N2, 0.0, s));
    bool ok = false;
    SeedWork sw = seed_carve(base + p.seed_off, p.seed_bytes, op, m, mixed != 0, &ok);
    if (!ok) {
        set_error("seeded_solve: seed workspace carving failed");
        return SC_ERR_WORKSPACE;
    }
    SC_TRY(seed_pretune(op, mixed != 0, sw, s));

    auto contract = [&](int rows) -> sc_status {
        for (int g = 0; g < p.ngroups; ++g) {
            const int nw = wcols(g);
            if (nw <= 0) continue;
            ColPtrs<const void> wc{};
            for (int j = 0; j < nw; ++j) wc.p[j] = (const char*)B + (size_t)(wfirst(g) + j) * ldb * eb;
            SC_TRY(gemm_cn(cpl, vs, V, op->n, op->n, rows, false, wc, nw, Gg(g), part, nullptr, s));
        }
        return SC_OK;
    };
    // a small system's seed phase is a chain of short launches: replay it from a
    // cached graph (its kernels are then not seen by the in-library timer).  X
    // is zero here, so the phase gets x0 = 0 without a pointer to X, which
    // would tie the graph to the caller's output buffer.
    if (N2 <= kSeedGraphMax)
        SC_TRY(seed_enqueue_cached(op, B, nullptr, m, freq, V, op->n, p.vdt, alpha, beta, sw, s, mixed != 0));
    else
        SC_TRY(seed_enqueue_any(op, B, X, m, freq, V, op->n, p.vdt, alpha, beta, sw, s));
    sc_status seed_status = SC_OK;
    SC_TRY(seed_finalize_any(op, X, V, op->n, p.vdt, alpha, beta, m_done, sw, s, &seed_status, false));
    if (seed_status == SC_ERR_NOT_PD || seed_status == SC_ERR_NONFINITE) {
        set_error("seeded_solve: the seed phase stopped (operator not positive definite or non-finite values)");
        return seed_status;
    }
    const int md = *m_done;
    if (md >= 1) {
        if (k > 1) SC_TRY(contract(md));
        for (int g = 0; g < p.ngroups; ++g) {
            const int nc = group_cols(k, g);
            double* Y = Gg(g);
            if (g == 0) {
                const int64_t tot = (int64_t)md * nc * mul;
                hipLaunchKernelGGL(k_seed_coeffs, dim3((unsigned)std::min<int64_t>((tot + kBlock - 1) / kBlock, 1024)),
                                   dim3(kBlock), 0, s, Y0, Gg(0), md, nc, (int)mul, beta);
                SC_LAUNCH_CHECK();
                Y = Y0;
            }
            SC_TRY(tridiag_solve(alpha, beta, md, Y, nc, cpl, nullptr, trid, nullptr, s));
            ColPtrs<void> xc{};
            for (int j = 0; j < nc; ++j) xc.p[j] = (char*)X + (size_t)(g * kMaxCols + j) * ldx * eb;
            SC_TRY(gemm_nn(cpl, vs, V, op->n, op->n, md, Y, nc, false, xc, 1.0, nullptr, s));
        }
    }
    void* cgw = base + p.cg_off;
    sc_status out = solve_cg(op, mixed, B, ldb, X, ldx, k, tol, maxit, iters, relres, cgw, p.cg_bytes, s);
    if (out < 0) return out;
    iters[0] += md;
    if (out == SC_OK && seed_status == SC_BREAKDOWN) out = SC_BREAKDOWN;
    return out;
}

}  // namespace sc
