// C ABI entry points (declared in include/seedcg.h): argument validation,
// workspace queries and dispatch to the drivers.  Nothing throws across the
// boundary; every failure is a status code plus a message in sc_last_error().
#include <atomic>
#include <cmath>
#include <new>

#include "sc_internal.h"
#include "sc_timer.h"

namespace sc {

thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

sc_status seed_lanczos(const sc_op* op, const void* b1, void* x1, int m, int freq, void* V, int64_t ldv, sc_dtype vdt,
                       double* alpha, double* beta, int* m_done, void* work, size_t work_bytes, hipStream_t s);

size_t kappa_grad_workspace(const sc_op* op, int k);
sc_status kappa_grad(const sc_op* op, const void* X, int64_t ldx, const void* L, int64_t ldl, int k, double* out,
                     void* work, size_t work_bytes, hipStream_t s);
size_t batch_workspace(int nsys, const sc_batch_system* sys);
sc_status batch_solve(int nsys, sc_batch_system* sys, void* work, size_t work_bytes, hipStream_t s);

static bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

static std::atomic<uint64_t> g_op_gen{0};
static sc_op* new_op() {
    sc_op* op = new sc_op();
    op->gen = ++g_op_gen;
    return op;
}

// the op's precision or its single counterpart
static bool dtype_ok_for(const sc_op* op, sc_dtype d) { return d == op->dtype || d == single_of(op->dtype); }

static size_t apply_workspace(const sc_op* op, int k, sc_dtype d) {
    return (size_t)std::max<int64_t>(op_apply_tmp_elems(op), 0) * dtype_bytes(d) * (size_t)std::max(k, 1) + 256;
}

// columns of one pass of the projection (k right-hand sides go in groups of at most kMaxCols)
static int project_group(int k) { return std::max(1, std::min(k, kMaxCols)); }

size_t project_workspace(int64_t n, int m, int k, bool cpl) {
    const int N = project_group(k);
    Carver c(nullptr, 0);
    c.take<double>((size_t)m * N * 2);
    c.take<double>(gemm_cn_part_doubles(n, m, N, cpl));
    c.take<double>((size_t)m * 2);
    return c.off + 256;
}

sc_status project_impl(int64_t n, const void* V, int64_t ldv, sc_dtype vdt, int m, const double* alpha,
                              const double* beta, sc_dtype xdt, const void* R0, int64_t ldr, int k, void* X,
                              int64_t ldx, void* work, size_t work_bytes, hipStream_t s) {
    const bool cpl = is_complex(vdt);
    const bool vs = is_single(vdt);
    const int N = project_group(k);
    Carver c(work, work_bytes);
    double* G = c.take<double>((size_t)m * N * 2);
    double* part = c.take<double>(gemm_cn_part_doubles(n, m, N, cpl));
    double* trid = c.take<double>((size_t)m * 2);
    if (!c.ok()) {
        set_error("project: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    const size_t eb = dtype_bytes(xdt);
    for (int j0 = 0; j0 < k; j0 += N) {
        const int nb = std::min(N, k - j0);
        ColPtrs<const void> rc{};
        ColPtrs<void> xc{};
        for (int j = 0; j < nb; ++j) {
            rc.p[j] = (const char*)R0 + (size_t)(j0 + j) * ldr * eb;
            xc.p[j] = (char*)X + (size_t)(j0 + j) * ldx * eb;
        }
        SC_TRY(gemm_cn(cpl, vs, V, ldv, n, m, false, rc, nb, G, part, nullptr, s));
        SC_TRY(tridiag_solve(alpha, beta, m, G, nb, cpl, nullptr, trid, nullptr, s));
        SC_TRY(gemm_nn(cpl, vs, V, ldv, n, m, G, nb, false, xc, 1.0, nullptr, s));
    }
    return SC_OK;
}

}  // namespace sc

using namespace sc;

#define SC_GUARD_BEGIN \
    clear_error();     \
    try {
#define SC_GUARD_END                                  \
    }                                                 \
    catch (const std::bad_alloc&) {                   \
        set_error("host allocation failed");          \
        return SC_ERR_ARG;                            \
    }                                                 \
    catch (...) {                                     \
        set_error("unexpected host exception");       \
        return SC_ERR_ARG;                            \
    }

extern "C" {

const char* sc_last_error(void) { return g_last_error.c_str(); }

sc_status sc_op_laplace2d(int nx, int ny, sc_op** out) {
    SC_GUARD_BEGIN
    SC_ARG(out, "out is NULL");
    SC_ARG(nx >= 1 && ny >= 1, "nx and ny must be >= 1");
    sc_op* op = new_op();
    op->kind = SC_OPK_LAPLACE2D;
    op->nx = nx;
    op->ny = ny;
    op->n = (int64_t)nx * ny;
    op->dtype = SC_R64;
    *out = op;
    return SC_OK;
    SC_GUARD_END
}

sc_status sc_op_diag(const double* d_dev, int64_t n, sc_op** out) {
    SC_GUARD_BEGIN
    SC_ARG(out, "out is NULL");
    SC_ARG(d_dev && aligned(d_dev, 8), "d_dev is NULL or misaligned");
    SC_ARG(n >= 1, "n must be >= 1");
    sc_op* op = new_op();
    op->kind = SC_OPK_DIAG;
    op->d = d_dev;
    op->n = n;
    op->dtype = SC_R64;
    *out = op;
    return SC_OK;
    SC_GUARD_END
}

sc_status sc_op_wilson_normal(const int dims[4], const void* U64_dev, const void* U32_dev, double kappa,
                              int t_antiperiodic, sc_op** out) {
    SC_GUARD_BEGIN
    SC_ARG(out, "out is NULL");
    SC_ARG(dims, "dims is NULL");
    SC_ARG(dims[0] >= 1 && dims[1] >= 1 && dims[2] >= 1 && dims[3] >= 1, "lattice dimensions must be >= 1");
    SC_ARG(U64_dev && aligned(U64_dev, 16), "U64_dev is NULL or not 16-byte aligned");
    SC_ARG(!U32_dev || aligned(U32_dev, 8), "U32_dev is not 8-byte aligned");
    SC_ARG(std::isfinite(kappa), "kappa must be finite");
    const int64_t vol = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    SC_ARG(vol * 36 < (int64_t(1) << 31), "lattice too large: 32-bit site indexing needs 36 * volume < 2^31");
    sc_op* op = new_op();
    op->kind = SC_OPK_WILSON;
    for (int i = 0; i < 4; ++i) op->dims[i] = dims[i];
    op->vol = vol;
    op->n = vol * 12;
    op->dtype = SC_C128;
    op->U64 = U64_dev;
    op->U32 = U32_dev;
    op->kappa = kappa;
    op->antiperiodic = t_antiperiodic ? 1 : 0;
    *out = op;
    return SC_OK;
    SC_GUARD_END
}

sc_status sc_op_wilson_g5(const int dims[4], const void* U64_dev, const void* U32_dev, double kappa,
                          int t_antiperiodic, sc_op** out) {
    SC_GUARD_BEGIN
    const sc_status st = sc_op_wilson_normal(dims, U64_dev, U32_dev, kappa, t_antiperiodic, out);
    if (st == SC_OK) (*out)->kind = SC_OPK_WILSON_G5;
    return st;
    SC_GUARD_END
}

sc_status sc_op_wilson_check_su3(sc_op* op, void* stream, double* deviation, int* rebuild) {
    SC_GUARD_BEGIN
    SC_ARG(op && has_links(op), "op is NULL or not a Wilson operator");
    return wilson_check_su3(op, (hipStream_t)stream, deviation, rebuild);
    SC_GUARD_END
}

sc_status sc_op_destroy(sc_op* op) {
    SC_GUARD_BEGIN
    if (op) batch_forget_op(op);
    delete op;
    return SC_OK;
    SC_GUARD_END
}

sc_status sc_op_info(const sc_op* op, int64_t* n, sc_dtype* dtype) {
    SC_GUARD_BEGIN
    SC_ARG(op && n && dtype, "NULL argument");
    *n = op->n;
    *dtype = op->dtype;
    return SC_OK;
    SC_GUARD_END
}

sc_status sc_workspace_size(const sc_op* op, int call, int k, int m, sc_dtype dtype, size_t* bytes) {
    SC_GUARD_BEGIN
    SC_ARG(bytes, "bytes is NULL");
    SC_ARG(k >= 0 && m >= 0, "k and m must be >= 0");
    switch (call) {
        case SC_CALL_APPLY:
            SC_ARG(op && dtype_ok_for(op, dtype), "op NULL or dtype not valid for the op");
            *bytes = apply_workspace(op, k, dtype);
            return SC_OK;
        case SC_CALL_SEED:
            SC_ARG(op && dtype_ok_for(op, dtype), "op NULL or dtype not valid for the op");
            *bytes = seed_workspace(op, std::max(m, 1), is_single(dtype));
            return SC_OK;
        case SC_CALL_PROJECT: {
            int64_t n = op ? op->n : (int64_t)*bytes;
            SC_ARG(n >= 1, "project size query needs an op or n in *bytes");
            *bytes = project_workspace(n, std::max(m, 1), k, is_complex(dtype));
            return SC_OK;
        }
        case SC_CALL_CG:
            SC_ARG(op && dtype_ok_for(op, dtype), "op NULL or dtype not valid for the op");
            *bytes = cg_workspace(op, std::max(k, 1), is_single(dtype));
            return SC_OK;
        case SC_CALL_KAPPA_GRAD:
            SC_ARG(op && op->kind == SC_OPK_WILSON, "kappa gradient needs a Wilson op");
            *bytes = kappa_grad_workspace(op, std::max(k, 1));
            return SC_OK;
        case SC_CALL_MULTISEED:
            SC_ARG(op && dtype_ok_for(op, dtype), "op NULL or dtype not valid for the op");
            *bytes = multiseed_workspace(op, std::max(k, 1));
            return SC_OK;
        case SC_CALL_RELATED:
            SC_ARG(op && dtype_ok_for(op, dtype), "op NULL or dtype not valid for the op");
            *bytes = related_workspace(op, std::max(k, 1), std::max(m, 1), is_single(dtype));
            return SC_OK;
        case SC_CALL_MINRES:
            SC_ARG(op && dtype == op->dtype, "op NULL or dtype not the op's (MINRES runs in FP64)");
            *bytes = minres_workspace(op, std::max(k, 1));
            return SC_OK;
        case SC_CALL_INDEFINITE:
            SC_ARG(op && dtype == op->dtype, "op NULL or dtype not the op's (the indefinite variant runs in FP64)");
            *bytes = indefinite_workspace(op, std::max(k, 1), std::max(m, 1));
            return SC_OK;
        case SC_CALL_SEEDED:
            SC_ARG(op && dtype_ok_for(op, dtype), "op NULL or dtype not valid for the op");
            *bytes = seeded_workspace(op, std::max(k, 1), std::max(m, 1), is_single(dtype));
            return SC_OK;
        default:
            SC_ARG(false, "unknown call id");
    }
    SC_GUARD_END
}

sc_status sc_op_apply(const sc_op* op, sc_dtype dtype, const void* X_dev, int64_t ldx, void* Y_dev, int64_t ldy,
                      int k, void* work_dev, size_t work_bytes, void* stream) {
    SC_GUARD_BEGIN
    SC_ARG(op, "op is NULL");
    SC_ARG(dtype_ok_for(op, dtype), "dtype not valid for the op");
    SC_ARG(k >= 0, "k must be >= 0");
    if (k == 0) return SC_OK;
    SC_ARG(X_dev && Y_dev, "X or Y is NULL");
    SC_ARG(aligned(X_dev, dtype_bytes(dtype)) && aligned(Y_dev, dtype_bytes(dtype)), "X or Y misaligned");
    SC_ARG(ldx >= op->n && ldy >= op->n, "leading dimension smaller than n");
    SC_ARG(!(has_links(op) && is_single(dtype) && !op->U32), "single precision needs U32 links");
    if (work_bytes < apply_workspace(op, k, dtype) - 256 || (op_apply_tmp_elems(op) > 0 && !work_dev)) {
        set_error("op_apply: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    return op_apply(op, is_single(dtype), X_dev, ldx, Y_dev, ldy, k, work_dev, (hipStream_t)stream);
    SC_GUARD_END
}

sc_status sc_wilson_dslash(const sc_op* op, sc_dtype dtype, int which, const void* X_dev, int64_t ldx, void* Y_dev,
                           int64_t ldy, int k, void* stream) {
    SC_GUARD_BEGIN
    SC_ARG(op && has_links(op), "not a Wilson op");
    SC_ARG(dtype == SC_C128 || dtype == SC_C64, "dtype must be SC_C128 or SC_C64");
    SC_ARG(which >= 0 && which <= 3, "which must be 0..3");
    SC_ARG(k >= 0, "k must be >= 0");
    if (k == 0) return SC_OK;
    SC_ARG(X_dev && Y_dev && X_dev != Y_dev, "X or Y NULL, or X == Y (the stencil cannot run in place)");
    SC_ARG(aligned(X_dev, dtype_bytes(dtype)) && aligned(Y_dev, dtype_bytes(dtype)), "X or Y misaligned");
    SC_ARG(ldx >= op->n && ldy >= op->n, "leading dimension smaller than n");
    SC_ARG(!(dtype == SC_C64 && !op->U32), "single precision needs U32 links");
    return wilson_pass(op, dtype == SC_C64, which, X_dev, ldx, Y_dev, ldy, k, (hipStream_t)stream);
    SC_GUARD_END
}

sc_status sc_seed_lanczos(const sc_op* op, const void* b1_dev, void* x1_dev, int m, int reorth_freq, void* V_dev,
                          int64_t ldv, sc_dtype v_dtype, double* alpha_dev, double* beta_dev, int* m_done,
                          void* work_dev, size_t work_bytes, void* stream) {
    SC_GUARD_BEGIN
    SC_ARG(op, "op is NULL");
    SC_ARG(m_done, "m_done is NULL");
    SC_ARG(m >= 1, "m must be >= 1");
    SC_ARG(reorth_freq >= 0, "reorth_freq must be >= 0");
    SC_ARG(dtype_ok_for(op, v_dtype), "v_dtype not valid for the op");
    SC_ARG(!(has_links(op) && is_single(v_dtype) && !op->U32), "single precision needs U32 links");
    SC_ARG(b1_dev && x1_dev && V_dev && alpha_dev && beta_dev && work_dev, "NULL device pointer");
    SC_ARG(aligned(b1_dev, dtype_bytes(op->dtype)) && aligned(x1_dev, dtype_bytes(op->dtype)) &&
               aligned(V_dev, dtype_bytes(v_dtype)) && aligned(alpha_dev, 8) && aligned(beta_dev, 8),
           "misaligned device pointer");
    SC_ARG(ldv >= op->n, "ldv smaller than n");
    if (work_bytes < seed_workspace(op, m, is_single(v_dtype)) - 256) {
        set_error("seed_lanczos: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    *m_done = 0;
    return seed_lanczos(op, b1_dev, x1_dev, m, reorth_freq, V_dev, ldv, v_dtype, alpha_dev, beta_dev, m_done, work_dev,
                        work_bytes, (hipStream_t)stream);
    SC_GUARD_END
}

sc_status sc_project(int64_t n, const void* V_dev, int64_t ldv, sc_dtype v_dtype, int m, const double* alpha_dev,
                     const double* beta_dev, sc_dtype vec_dtype, const void* R0_dev, int64_t ldr, int k, void* X_dev,
                     int64_t ldx, void* work_dev, size_t work_bytes, void* stream) {
    SC_GUARD_BEGIN
    SC_ARG(n >= 1, "n must be >= 1");
    SC_ARG(m >= 1, "m must be >= 1");
    SC_ARG(k >= 0, "k must be >= 0");
    SC_ARG(vec_dtype == SC_C128 || vec_dtype == SC_R64, "vec_dtype must be SC_C128 or SC_R64");
    SC_ARG(double_of(v_dtype) == vec_dtype, "v_dtype and vec_dtype must both be complex or both real");
    if (k == 0) return SC_OK;
    SC_ARG(V_dev && alpha_dev && beta_dev && R0_dev && X_dev && work_dev, "NULL device pointer");
    SC_ARG(aligned(V_dev, dtype_bytes(v_dtype)) && aligned(R0_dev, dtype_bytes(vec_dtype)) &&
               aligned(X_dev, dtype_bytes(vec_dtype)),
           "misaligned device pointer");
    SC_ARG(ldv >= n && ldr >= n && ldx >= n, "leading dimension smaller than n");
    if (work_bytes < project_workspace(n, m, k, is_complex(vec_dtype)) - 256) {
        set_error("project: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    return project_impl(n, V_dev, ldv, v_dtype, m, alpha_dev, beta_dev, vec_dtype, R0_dev, ldr, k, X_dev, ldx, work_dev,
                        work_bytes, (hipStream_t)stream);
    SC_GUARD_END
}

sc_status sc_solve_cg(const sc_op* op, int mixed, const void* B_dev, int64_t ldb, void* X_dev, int64_t ldx, int k,
                      double tol, int maxit, int* iters, double* relres, void* work_dev, size_t work_bytes,
                      void* stream) {
    SC_GUARD_BEGIN
    SC_ARG(op, "op is NULL");
    SC_ARG(k >= 1, "k must be >= 1");
    SC_ARG(iters && relres, "iters or relres is NULL");
    SC_ARG(std::isfinite(tol) && tol > 0.0, "tol must be finite and > 0");
    SC_ARG(maxit >= 0, "maxit must be >= 0");
    SC_ARG(B_dev && X_dev && work_dev, "NULL device pointer");
    SC_ARG(aligned(B_dev, dtype_bytes(op->dtype)) && aligned(X_dev, dtype_bytes(op->dtype)),
           "misaligned device pointer");
    SC_ARG(ldb >= op->n && ldx >= op->n, "leading dimension smaller than n");
    SC_ARG(!(mixed && has_links(op) && !op->U32), "mixed precision needs U32 links");
    if (work_bytes < cg_workspace(op, k, mixed != 0) - 256) {
        set_error("solve_cg: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    return solve_cg(op, mixed, B_dev, ldb, X_dev, ldx, k, tol, maxit, iters, relres, work_dev, work_bytes,
                    (hipStream_t)stream);
    SC_GUARD_END
}

sc_status sc_wilson_kappa_grad(const sc_op* op, const void* X_dev, int64_t ldx, const void* L_dev, int64_t ldl,
                                int k, double* grad, void* work_dev, size_t work_bytes, void* stream) {
    SC_GUARD_BEGIN
    SC_ARG(op && has_links(op), "not a Wilson op");
    SC_ARG(grad, "grad is NULL");
    SC_ARG(k >= 1, "k must be >= 1");
    SC_ARG(X_dev && L_dev && work_dev, "NULL device pointer");
    SC_ARG(aligned(X_dev, 16) && aligned(L_dev, 16), "misaligned device pointer");
    SC_ARG(ldx >= op->n && ldl >= op->n, "leading dimension smaller than n");
    if (work_bytes < kappa_grad_workspace(op, k) - 256) {
        set_error("kappa_grad: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    return kappa_grad(op, X_dev, ldx, L_dev, ldl, k, grad, work_dev, work_bytes, (hipStream_t)stream);
    SC_GUARD_END
}

static sc_status check_batch(int nsys, const sc_batch_system* sys) {
    SC_ARG(nsys >= 1 && nsys <= 64 && sys, "nsys must be 1..64 and systems non-NULL");
    for (int i = 0; i < nsys; ++i) {
        const sc_batch_system& b = sys[i];
        SC_ARG(b.op, "system op is NULL");
        SC_ARG(b.k >= 1 && b.m >= 1 && b.reorth_freq >= 0 && b.maxit >= 0, "system k, m >= 1, freq, maxit >= 0");
        SC_ARG(std::isfinite(b.tol) && b.tol > 0.0, "system tol must be finite and > 0");
        SC_ARG(b.B_dev && b.X_dev && b.iters && b.relres, "system pointer is NULL");
        SC_ARG(aligned(b.B_dev, dtype_bytes(b.op->dtype)) && aligned(b.X_dev, dtype_bytes(b.op->dtype)),
               "system B or X misaligned");
        SC_ARG(b.ldb >= b.op->n && b.ldx >= b.op->n, "system leading dimension smaller than n");
        SC_ARG(!(b.mixed && has_links(b.op) && !b.op->U32), "mixed precision needs U32 links");
    }
    return SC_OK;
}

sc_status sc_batch_workspace_size(int nsys, const sc_batch_system* systems, size_t* bytes) {
    SC_GUARD_BEGIN
    SC_ARG(bytes, "bytes is NULL");
    SC_TRY(check_batch(nsys, systems));
    *bytes = batch_workspace(nsys, systems);
    return SC_OK;
    SC_GUARD_END
}

sc_status sc_batch_solve(int nsys, sc_batch_system* systems, void* work_dev, size_t work_bytes, void* stream) {
    SC_GUARD_BEGIN
    SC_TRY(check_batch(nsys, systems));
    SC_ARG(work_dev, "work is NULL");
    if (work_bytes < batch_workspace(nsys, systems) - 256) {
        set_error("batch_solve: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    return batch_solve(nsys, systems, work_dev, work_bytes, (hipStream_t)stream);
    SC_GUARD_END
}

sc_status sc_wilson_tune_info(const sc_op* op, sc_dtype dtype, int k, int* variant, float* us) {
    SC_GUARD_BEGIN
    SC_ARG(op && has_links(op), "not a Wilson op");
    SC_ARG(dtype == SC_C128 || dtype == SC_C64, "dtype must be SC_C128 or SC_C64");
    SC_ARG(variant && us, "NULL argument");
    return wilson_tune_query(op, dtype == SC_C64, k, variant, us);
    SC_GUARD_END
}

sc_status sc_wilson_tune_set(const sc_op* op, sc_dtype dtype, int k, int variant) {
    SC_GUARD_BEGIN
    SC_ARG(op && has_links(op), "not a Wilson op");
    SC_ARG(dtype == SC_C128 || dtype == SC_C64, "dtype must be SC_C128 or SC_C64");
    SC_ARG(k >= 1 && variant >= -1 && variant < SC_WILSON_VARIANTS,
           "k must be >= 1 and variant in -1..SC_WILSON_VARIANTS-1");
    return wilson_tune_pin(op, dtype == SC_C64, k, variant);
    SC_GUARD_END
}

sc_status sc_wilson_range_check(const int* dims, int variant, int k, int64_t ldx, int64_t ldy, int64_t* accesses,
                                int64_t* outside) {
    SC_GUARD_BEGIN
    SC_ARG(dims && accesses && outside, "NULL argument");
    return wilson_tx_check(dims, variant, k, ldx, ldy, accesses, outside);
    SC_GUARD_END
}

sc_status sc_related_solve(const sc_op* op, int mixed, const void* B_dev, int64_t ldb, void* X_dev, int64_t ldx,
                           int k, int m, int reorth_freq, double tol, int maxit, int* iters, double* relres,
                           int* m_done, void* work_dev, size_t work_bytes, void* stream) {
    SC_GUARD_BEGIN
    SC_ARG(op, "op is NULL");
    SC_ARG(k >= 1 && m >= 1 && reorth_freq >= 0 && maxit >= 1, "need k >= 1, m >= 1, reorth_freq >= 0, maxit >= 1");
    SC_ARG(tol > 0.0 && std::isfinite(tol), "tol must be positive and finite");
    SC_ARG(B_dev && X_dev && work_dev, "NULL device pointer");
    SC_ARG(iters && relres && m_done, "NULL host pointer");
    SC_ARG(!(mixed && has_links(op) && !op->U32), "mixed precision needs U32 links");
    SC_ARG(ldb >= op->n && ldx >= op->n, "ldb or ldx smaller than n");
    SC_ARG(aligned(B_dev, dtype_bytes(op->dtype)) && aligned(X_dev, dtype_bytes(op->dtype)),
           "misaligned device pointer");
    if (work_bytes < related_workspace(op, k, m, mixed != 0) - 256) {
        set_error("related_solve: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    *m_done = 0;
    return related_solve(op, mixed, B_dev, ldb, X_dev, ldx, k, m, reorth_freq, tol, maxit, iters, relres, m_done,
                         work_dev, work_bytes, (hipStream_t)stream);
    SC_GUARD_END
}

sc_status sc_seeded_solve(const sc_op* op, int mixed, const void* B_dev, int64_t ldb, void* X_dev, int64_t ldx,
                          int k, int m, int reorth_freq, double tol, int maxit, int* iters, double* relres,
                          int* m_done, void* work_dev, size_t work_bytes, void* stream) {
    SC_GUARD_BEGIN
    SC_ARG(op, "op is NULL");
    SC_ARG(k >= 1 && m >= 1 && reorth_freq >= 0 && maxit >= 1, "need k >= 1, m >= 1, reorth_freq >= 0, maxit >= 1");
    SC_ARG(tol > 0.0 && std::isfinite(tol), "tol must be positive and finite");
    SC_ARG(B_dev && X_dev && work_dev, "NULL device pointer");
    SC_ARG(iters && relres && m_done, "NULL host pointer");
    SC_ARG(!(mixed && has_links(op) && !op->U32), "mixed precision needs U32 links");
    SC_ARG(ldb >= op->n && ldx >= op->n, "ldb or ldx smaller than n");
    SC_ARG(aligned(B_dev, dtype_bytes(op->dtype)) && aligned(X_dev, dtype_bytes(op->dtype)),
           "misaligned device pointer");
    if (work_bytes < seeded_workspace(op, k, m, mixed != 0) - 256) {
        set_error("seeded_solve: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    *m_done = 0;
    return seeded_solve(op, mixed, B_dev, ldb, X_dev, ldx, k, m, reorth_freq, tol, maxit, iters, relres, m_done,
                        work_dev, work_bytes, (hipStream_t)stream);
    SC_GUARD_END
}

sc_status sc_solve_minres(const sc_op* op, const void* B_dev, int64_t ldb, void* X_dev, int64_t ldx, int k,
                          double tol, int maxit, int* iters, double* relres, void* work_dev, size_t work_bytes,
                          void* stream) {
    SC_GUARD_BEGIN
    SC_ARG(op, "op is NULL");
    SC_ARG(k >= 1 && maxit >= 1, "need k >= 1 and maxit >= 1");
    SC_ARG(tol > 0.0 && std::isfinite(tol), "tol must be positive and finite");
    SC_ARG(B_dev && X_dev && work_dev, "NULL device pointer");
    SC_ARG(iters && relres, "NULL host pointer");
    SC_ARG(ldb >= op->n && ldx >= op->n, "ldb or ldx smaller than n");
    SC_ARG(aligned(B_dev, dtype_bytes(op->dtype)) && aligned(X_dev, dtype_bytes(op->dtype)),
           "misaligned device pointer");
    if (work_bytes < minres_workspace(op, k) - 256) {
        set_error("minres: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    return minres_solve(op, B_dev, ldb, X_dev, ldx, k, tol, maxit, iters, relres, work_dev, work_bytes,
                        (hipStream_t)stream);
    SC_GUARD_END
}

sc_status sc_indefinite_solve(const sc_op* op, const void* B_dev, int64_t ldb, void* X_dev, int64_t ldx, int k,
                              int m, int reorth_freq, double tol, int maxit, int* iters, double* relres, int* m_done,
                              void* work_dev, size_t work_bytes, void* stream) {
    SC_GUARD_BEGIN
    SC_ARG(op, "op is NULL");
    SC_ARG(k >= 1 && m >= 1 && reorth_freq >= 0 && maxit >= 1, "need k >= 1, m >= 1, reorth_freq >= 0, maxit >= 1");
    SC_ARG(tol > 0.0 && std::isfinite(tol), "tol must be positive and finite");
    SC_ARG(B_dev && X_dev && work_dev, "NULL device pointer");
    SC_ARG(iters && relres && m_done, "NULL host pointer");
    SC_ARG(ldb >= op->n && ldx >= op->n, "ldb or ldx smaller than n");
    SC_ARG(aligned(B_dev, dtype_bytes(op->dtype)) && aligned(X_dev, dtype_bytes(op->dtype)),
           "misaligned device pointer");
    if (work_bytes < indefinite_workspace(op, k, m) - 256) {
        set_error("indefinite_solve: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    *m_done = 0;
    return indefinite_solve(op, B_dev, ldb, X_dev, ldx, k, m, reorth_freq, tol, maxit, iters, relres, m_done,
                            work_dev, work_bytes, (hipStream_t)stream);
    SC_GUARD_END
}

sc_status sc_multiple_seed_solve(const sc_op* op, const void* B_dev, int64_t ldb, void* X_dev, int64_t ldx, int k,
                                 double tol, int maxit, int* iters, double* relres, void* work_dev, size_t work_bytes,
                                 void* stream) {
    SC_GUARD_BEGIN
    SC_ARG(op, "op is NULL");
    SC_ARG(k >= 1 && maxit >= 1, "need k >= 1 and maxit >= 1");
    SC_ARG(tol > 0.0 && std::isfinite(tol), "tol must be positive and finite");
    SC_ARG(B_dev && X_dev && work_dev, "NULL device pointer");
    SC_ARG(iters && relres, "NULL host pointer");
    SC_ARG(ldb >= op->n && ldx >= op->n, "ldb or ldx smaller than n");
    SC_ARG(aligned(B_dev, dtype_bytes(op->dtype)) && aligned(X_dev, dtype_bytes(op->dtype)),
           "misaligned device pointer");
    if (work_bytes < multiseed_workspace(op, k) - 256) {
        set_error("multiple_seed_solve: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    return multiseed_solve(op, B_dev, ldb, X_dev, ldx, k, tol, maxit, iters, relres, work_dev, work_bytes,
                           (hipStream_t)stream);
    SC_GUARD_END
}

sc_status sc_timer_enable(int every) {
    SC_GUARD_BEGIN
    return timer_enable(every);
    SC_GUARD_END
}

sc_status sc_timer_read(int cls, double* ms, int64_t* launches, double* bytes, double* flops) {
    SC_GUARD_BEGIN
    SC_ARG(cls >= 0 && cls < TC_COUNT, "unknown kernel class");
    SC_ARG(ms && launches && bytes && flops, "NULL argument");
    return timer_read(cls, ms, launches, bytes, flops);
    SC_GUARD_END
}

}  // extern "C"
