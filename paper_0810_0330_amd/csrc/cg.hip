// Batched CG (Hestenes-Stiefel) for the seeded systems (Section 2.2): every
// right-hand side runs its own recurrence with its own FP64 scalars, held on
// the device; converged columns are frozen by a per-column flag.  The host
// synchronises once per chunk of iterations to see whether any column is
// still active, then verifies the true residual b - A x of every column and
// restarts the ones still above tol.
//
// One iteration is four kernels: q = A p (the operator), partials of <p, q>,
// x += alpha p and r -= alpha q with partials of ||r||^2, and p = r + beta p.
// For the Wilson normal operator on a t-march stencil shape it is three: the
// D pass leaves the partials of <p, q> = ||D p||^2, the D^H pass applies
// r -= alpha q itself (q is never stored) and leaves those of ||r||^2, and one
// kernel does x += alpha p and p = r + beta p.  The formulas and their order
// are the same.
// Each consumer block re-adds the producer's per-block partials in a fixed
// order, so every block derives the same scalars.  The per-column state is
// double-buffered: the last kernel of an iteration reads one copy and writes
// the other, so no kernel reads a field that another of its blocks writes.
//
// mixed = 1: the vectors and the operator run in FP32; x and the true
// residual are FP64.  A reliable update (x64 += x32, r = b - A64 x64, r32 =
// r, x32 = 0) is made for every column whose FP32 residual norm has fallen by
// 1e4x since its last update, at the next host check (the column keeps
// iterating meanwhile, so no column idles; p is kept and CG continues with
// the true residual), and when the FP32 residual reaches tol (the column
// stops; CG restarts from the true residual if it is still above tol).
//
// A column whose residual has stalled stops early and is reported as not
// converged: its recursive residual norm has not fallen 1% below its smallest
// value within kStallWindow iterations (a breakdown of the recurrence, an
// operator that is not HPD, an inconsistent system), or,
// in mixed precision, a FP64 true residual that has not halved over
// kStallUpdates successive reliable updates (tol below what the FP64 residual
// can reach).  Its iteration limit is lowered to the count reached, so no
// restart takes it up again; in mixed precision it keeps x as of its last
// reliable update (the FP32 increment since then is dropped).  A reliable
// update whose true residual has not halved, or is more than twice the
// recursive residual norm, also restarts the direction (p = r): the kept p
// belongs to a recursion that has left the true residual behind, and
// continuing with it diverges.
#include "sc_internal.h"

#include <cmath>
#include <limits>
#include <memory>
#include <vector>

namespace sc {

// Mixed precision: a column's reliable update is due once its FP32 residual
// norm is 1e4 times below the largest since its last update (squared: 1e-8).
// The FP32 recurrence then still sits about three orders of magnitude above
// its rounding floor (single precision relative to that largest norm).
constexpr double kRelUpdate2 = 1e-8;
constexpr int kStallWindow = 1000;
constexpr int kStallUpdates = 3;

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
    c.beta = 0.0;
    c.flag = 0;
    c.active = (c.bnorm2 > 0.0) && (c.rho > c.tol2) && (c.iters < c.maxit) && isfinite(c.rho);
    st[j] = c;
}

// partials of Re<p, q>
template <typename R, bool VEC>
__global__ __launch_bounds__(kBlock) void k_cg_pq(const R* __restrict__ p, const R* __restrict__ q, int64_t ld,
                                                  int64_t N, const CGCol* st, double* part) {
    __shared__ double sh[kWaves];
    const int col = blockIdx.y;
    if (!st[col].active) return;
    constexpr int W = Pack<R>::W;
    const R* pc = p + col * ld;
    const R* qc = q + col * ld;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock * W;
    for (int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * W; i0 < N; i0 += stride) {
        if (VEC && i0 + W <= N) {
            const Pack<R> a = ldp(pc, i0), b = ldp(qc, i0);
#pragma unroll
            for (int e = 0; e < W; ++e) acc += (double)a.v[e] * (double)b.v[e];
        } else {
            for (int64_t j = i0; j < min(N, i0 + W); ++j) acc += (double)pc[j] * (double)qc[j];
        }
    }
    block_partial(acc, part + (int64_t)col * gridDim.x, sh);
}

// alpha = rho / <p, q>; x += alpha p; r -= alpha q; partials of ||r||^2
template <typename XT, typename R, bool VEC>
__global__ __launch_bounds__(kBlock) void k_cg_xr(XT* __restrict__ x, int64_t ldx, R* __restrict__ r,
                                                  const R* __restrict__ p, const R* __restrict__ q, int64_t ld,
                                                  int64_t N, const CGCol* st, const double* part_pq, int G,
                                                  double* part_rr) {
    __shared__ double sh[kWaves];
    const int col = blockIdx.y;
    if (!st[col].active) return;
    constexpr int W = Pack<R>::W;
    const double a = st[col].rho / sum_partials(part_pq + (int64_t)col * G, G, sh);
    const R aR = (R)a;
    XT* xc = x + col * ldx;
    R* rc = r + col * ld;
    const R* pc = p + col * ld;
    const R* qc = q + col * ld;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock * W;
    for (int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * W; i0 < N; i0 += stride) {
        if (VEC && sizeof(XT) == sizeof(R) && i0 + W <= N) {
            Pack<R> xv = ldp((R*)xc, i0), rv = ldp(rc, i0);
            const Pack<R> pv = ldp(pc, i0), qv = ldp(qc, i0);
#pragma unroll
            for (int e = 0; e < W; ++e) {
                xv.v[e] = xv.v[e] + aR * pv.v[e];
                rv.v[e] = rv.v[e] - aR * qv.v[e];
                acc += (double)rv.v[e] * (double)rv.v[e];
            }
            stp((R*)xc, i0, xv);
            stp(rc, i0, rv);
        } else {
            for (int64_t j = i0; j < min(N, i0 + W); ++j) {
                xc[j] = (XT)(xc[j] + (XT)aR * (XT)pc[j]);
                const R rv = rc[j] - aR * qc[j];
                rc[j] = rv;
                acc += (double)rv * (double)rv;
            }
        }
    }
    block_partial(acc, part_rr + (int64_t)col * gridDim.x, sh);
}

// rho_new from the partials, convergence / reliable-update decisions (the
// same in every block); p = r + beta p unless the column stops.  Block 0
// writes the next state copy.
template <typename R, bool VEC>
__global__ __launch_bounds__(kBlock) void k_cg_p(R* __restrict__ p, const R* __restrict__ r, int64_t ld, int64_t N,
                                                 const CGCol* st, CGCol* st_next, const double* part_rr, int G,
                                                 int mixed) {
    __shared__ double sh[kWaves];
    const int col = blockIdx.y;
    CGCol c = st[col];
    if (!c.active) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st_next[col] = c;
        return;
    }
    constexpr int W = Pack<R>::W;
    const double rr = sum_partials(part_rr + (int64_t)col * G, G, sh);
    c.iters += 1;
    c.rho_prev = c.rho;
    c.rho = rr;
    c.beta = rr / c.rho_prev;
    c.rmax2 = fmax(c.rmax2, rr);
    if (!(rr > c.tol2) || !isfinite(rr)) {
        c.flag = 1;
        c.active = 0;
    } else if (mixed && rr < kRelUpdate2 * c.rmax2) {
        c.flag = 2;  // reliable update due at the next host check; the column keeps iterating
    }
    if (c.iters >= c.maxit) c.active = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) st_next[col] = c;
    if (!c.active) return;
    const R b = (R)c.beta;
    R* pc = p + col * ld;
    const R* rc = r + col * ld;
    const int64_t stride = (int64_t)gridDim.x * kBlock * W;
    for (int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * W; i0 < N; i0 += stride) {
        if (VEC && i0 + W <= N) {
            Pack<R> pv = ldp(pc, i0);
            const Pack<R> rv = ldp(rc, i0);
#pragma unroll
            for (int e = 0; e < W; ++e) pv.v[e] = rv.v[e] + b * pv.v[e];
            stp(pc, i0, pv);
        } else {
            for (int64_t j = i0; j < min(N, i0 + W); ++j) pc[j] = rc[j] + b * pc[j];
        }
    }
}

// The fused iteration's last kernel: alpha = rho / <p, q> and the new rho from
// the stencil passes' partials; x += alpha p for the columns active at the
// start of the iteration, then the decisions of k_cg_p and p = r + beta p.
template <typename XT, typename R, bool VEC>
__global__ __launch_bounds__(kBlock) void k_cg_xp(XT* __restrict__ x, int64_t ldx, R* __restrict__ p,
                                                  const R* __restrict__ r, int64_t ld, int64_t N, const CGCol* st,
                                                  CGCol* st_next, const double* part_pq, const double* part_rr, int G,
                                                  int mixed) {
    __shared__ double sh[kWaves];
    const int col = blockIdx.y;
    CGCol c = st[col];
    if (!c.active) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st_next[col] = c;
        return;
    }
    constexpr int W = Pack<R>::W;
    const double a = c.rho / sum_partials(part_pq + (int64_t)col * G, G, sh);
    const double rr = sum_partials(part_rr + (int64_t)col * G, G, sh);
    c.iters += 1;
    c.rho_prev = c.rho;
    c.rho = rr;
    c.beta = rr / c.rho_prev;
    c.rmax2 = fmax(c.rmax2, rr);
    if (!(rr > c.tol2) || !isfinite(rr)) {
        c.flag = 1;
        c.active = 0;
    } else if (mixed && rr < kRelUpdate2 * c.rmax2) {
        c.flag = 2;  // reliable update due at the next host check; the column keeps iterating
    }
    if (c.iters >= c.maxit) c.active = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) st_next[col] = c;
    const bool cont = c.active != 0;
    const R aR = (R)a, b = (R)c.beta;
    XT* xc = x + col * ldx;
    R* pc = p + col * ld;
    const R* rc = r + col * ld;
    const int64_t stride = (int64_t)gridDim.x * kBlock * W;
    for (int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * W; i0 < N; i0 += stride) {
        if (VEC && sizeof(XT) == sizeof(R) && i0 + W <= N) {
            // r is loaded with x and p (cont is uniform over the block), so an
            // iteration waits on memory once, not once for x, p and again for r
            Pack<R> xv = ldp((R*)xc, i0), pv = ldp(pc, i0);
            Pack<R> rv;
            if (cont) rv = ldp(rc, i0);
#pragma unroll
            for (int e = 0; e < W; ++e) xv.v[e] = xv.v[e] + aR * pv.v[e];
            stp((R*)xc, i0, xv);
            if (cont) {
#pragma unroll
                for (int e = 0; e < W; ++e) pv.v[e] = rv.v[e] + b * pv.v[e];
                stp(pc, i0, pv);
            }
        } else {
            for (int64_t j = i0; j < min(N, i0 + W); ++j) {
                const R pj = pc[j];
                xc[j] = (XT)(xc[j] + (XT)aR * (XT)pj);
                if (cont) pc[j] = rc[j] + b * pj;
            }
        }
    }
}

// ---------------------------------------------------------------- reliable updates
// Batched over the flagged columns listed in cols[0..nu): gather, residual, direction.

// x64_j += xs_j; xs_j = 0; xg_c = x64_j
__global__ __launch_bounds__(kBlock) void k_ru_gather(const int* __restrict__ cols, double* __restrict__ X,
                                                      int64_t ldx, float* __restrict__ xs, double* __restrict__ xg,
                                                      int64_t N) {
    const int c = blockIdx.y;
    const int j = cols[c];
    double* x = X + j * ldx;
    float* a = xs + j * N;
    double* o = xg ? xg + c * N : nullptr;  // no copy when every column is updated (A x64 reads X itself)
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock) {
        const double v = x[i] + (double)a[i];
        x[i] = v;
        a[i] = 0.0f;
        if (o) o[i] = v;
    }
}

// r64_j = b_j - (A x)_c; r32_j = r64_j; partials of ||r64_j||^2
__global__ __launch_bounds__(kBlock) void k_ru_resid(const int* __restrict__ cols, const double* __restrict__ B,
                                                     int64_t ldb, const double* __restrict__ ax,
                                                     double* __restrict__ r64, float* __restrict__ r32, int64_t N,
                                                     double* part) {
    __shared__ double sh[kWaves];
    const int c = blockIdx.y;
    const int j = cols[c];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock) {
        const double v = B[j * ldb + i] - ax[c * N + i];
        r64[j * N + i] = v;
        r32[j * N + i] = (float)v;
        acc += v * v;
    }
    block_partial(acc, part + (int64_t)c * gridDim.x, sh);
}

// p_j = r_j + beta_c p_j for the listed columns (beta_c = 0 restarts the direction)
__global__ __launch_bounds__(kBlock) void k_ru_dir(const int* __restrict__ cols, const double* __restrict__ beta,
                                                   float* __restrict__ p, const float* __restrict__ r, int64_t N) {
    const int c = blockIdx.y;
    const int j = cols[c];
    const float b = (float)beta[c];
    float* pc = p + j * N;
    const float* rc = r + j * N;
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
    double* xg;    // gathered FP64 columns for partial true residuals (k x N2)
    void* tmp64;   // FP64 op scratch (k columns)
    double* part_pq;
    double* part_rr;
    double* part;
    CGCol* st[2];
    double* rho;
    double* bn;
    int* cols;        // reliable update: flagged column list (k)
    double* ru_beta;  // reliable update: per listed column beta (k)
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
        w.xg = c.take<double>(N2 * k);
    }
    w.ax64 = c.take<double>(N2 * k);
    w.tmp64 = c.take<double>(tmpn * k);
    w.part_pq = c.take<double>((size_t)kMaxRedBlocks * k);
    w.part_rr = c.take<double>((size_t)kMaxRedBlocks * k);
    w.part = c.take<double>((size_t)kMaxRedBlocks * k);
    w.st[0] = c.take<CGCol>(k);
    w.st[1] = c.take<CGCol>(k);
    w.rho = c.take<double>(k);
    w.bn = c.take<double>(k);
    w.cols = c.take<int>(k);
    w.ru_beta = c.take<double>(k);
    return w;
}

size_t cg_workspace(const sc_op* op, int k, bool mixed) {
    Carver c(nullptr, 0);
    carve_cg(c, op, k, mixed);
    return c.off + 256;
}

sc_status cg_pretune(const sc_op* op, int mixed, int k, void* work, size_t work_bytes, hipStream_t s) {
    Carver c(work, work_bytes);
    CGWork w = carve_cg(c, op, k, mixed != 0);
    if (!c.ok()) {
        set_error("cg_pretune: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    // q = A p on k columns of the workspace: the first pass of (lattice,
    // precision, k) runs the stencil autotuner, which the CG passes reuse
    const bool cpl = is_complex(op->dtype);
    const int64_t N2 = op->n * (cpl ? 2 : 1);
    if (mixed) SC_TRY(fill<float>((float*)w.p, N2 * k, 0.0f, s));
    else SC_TRY(fill<double>((double*)w.p, N2 * k, 0.0, s));
    return op_apply(op, mixed != 0, w.p, op->n, w.q, op->n, k, w.tmp, s);
}

// r64 = b - A x (FP64) for k columns, rr[j] = ||r64_j||^2
static sc_status true_residual(const sc_op* op, const double* B, int64_t ldb2, const double* X, int64_t ldx2, int k,
                               const CGWork& w, double* r64, int64_t ldr2, double* rr, hipStream_t s) {
    const bool cpl = is_complex(op->dtype);
    const int64_t N2 = op->n * (cpl ? 2 : 1);
    const int64_t div = cpl ? 2 : 1;
    SC_TRY(op_apply(op, false, X, ldx2 / div, w.ax64, op->n, k, w.tmp64, s));
    SC_TRY(lincomb(0, r64, ldr2, 0, B, ldb2, 0, w.ax64, N2, N2, k, 1.0, -1.0, s));
    SC_TRY(dot(0, r64, ldr2, 0, r64, ldr2, N2, k, rr, w.part, nullptr, s));
    return SC_OK;
}

// The batched CG of k columns as a steppable object: start() forms the
// residuals and column states (one host synchronisation); iterate(n) enqueues
// n iterations and nothing else (no host interaction, so a fixed n can be
// captured into a graph); check() reads the column states after iterations,
// applies the stall rules and makes the due reliable updates; verify() runs
// when no column is active: it checks every column's true residual and
// restarts the ones still above tol.  solve_cg drives it with host checks
// every chunk() iterations; the batch driver replays captured chunks of
// kGraphChunk iterations for many systems at once.
template <typename R, bool VEC>
class CGRunT final : public CGRun {
   public:
    CGRunT(const sc_op* op, bool mixed, const double* B, int64_t ldb, double* X, int64_t ldx, int k, double tol,
           int maxit, const CGWork& w, hipStream_t s)
        : op_(op), mixed_(mixed), B_(B), X_(X), k_(k), tol_(tol), maxit_(maxit), w_(w), s_(s) {
        const bool cpl = is_complex(op->dtype);
        N2_ = op->n * (cpl ? 2 : 1);
        const int64_t mul = cpl ? 2 : 1;
        ldb2_ = ldb * mul;
        ldx2_ = ldx * mul;
        ldx_ = ldx;
        g_ = red_grid(N2_);
        hst_.resize(k);
        hrr_.resize(k);
        chk_rho_.assign(k, 0.0);
        chk_it_.assign(k, -1);
        min_rho_.assign(k, kInf);
        best_true_.assign(k, kInf);
        it_min_.assign(k, 0);
        nstall_.assign(k, 0);
        relres_.assign(k, 0.0);
    }

    sc_status start() override {
        const int vt = mixed_ ? 1 : 0;
        R* r = (R*)w_.r;
        R* p = (R*)w_.p;
        hipStream_t s = s_;
        SC_TRY(dot(0, B_, ldb2_, 0, B_, ldb2_, N2_, k_, w_.bn, w_.part, nullptr, s));
        // r = b - A x; rho = ||r||^2
        double* r64 = mixed_ ? w_.r64 : (double*)r;
        SC_TRY(true_residual(op_, B_, ldb2_, X_, ldx2_, k_, w_, r64, N2_, w_.rho, s));
        if (mixed_) {
            SC_TRY(lincomb(1, r, N2_, 0, r64, N2_, 0, nullptr, 0, N2_, k_, 1.0, 0.0, s));
            SC_TRY(fill<float>((float*)w_.xs, N2_ * k_, 0.0f, s));
        }
        SC_TRY(lincomb(vt, p, N2_, vt, r, N2_, 0, nullptr, 0, N2_, k_, 1.0, 0.0, s));
        hipLaunchKernelGGL(k_cg_setup, dim3((k_ + 63) / 64), dim3(64), 0, s, w_.st[cur_], w_.rho, w_.bn, k_, tol_,
                           maxit_, 1);
        SC_LAUNCH_CHECK();
        // columns with b = 0 are solved by x = 0
        SC_HIP(hipMemcpyAsync(hst_.data(), w_.st[cur_], sizeof(CGCol) * k_, hipMemcpyDeviceToHost, s));
        SC_HIP(hipStreamSynchronize(s));
        for (int j = 0; j < k_; ++j)
            if (!(hst_[j].bnorm2 > 0.0))
                SC_TRY(lincomb(0, X_ + j * ldx2_, N2_, 0, X_ + j * ldx2_, N2_, 0, nullptr, 0, N2_, 1, 0.0, 0.0, s));
        return SC_OK;
    }

    bool any_active() const override {
        for (int j = 0; j < k_; ++j)
            if (hst_[j].active) return true;
        return false;
    }

    int chunk() const override { return chunk_; }
    int state_index() const override { return cur_; }
    hipStream_t stream() const override { return s_; }

    sc_status iterate(int n) override {
        R* r = (R*)w_.r;
        R* p = (R*)w_.p;
        R* q = (R*)w_.q;
        const dim3 blk(kBlock), grid(g_, k_);
        hipStream_t s = s_;
        for (int it = 0; it < n; ++it) {
            // fused form (Wilson, t-march shape): D pass with <p, A p> partials, D^H pass
            // finishing r -= alpha A p, then x += alpha p and p = r + beta p
            int gf = 0;
            SC_TRY(wilson_cg_fused(op_, mixed_, p, w_.tmp, k_, w_.st[cur_], w_.part_pq, r, op_->n, w_.part_rr,
                                   kMaxRedBlocks, &gf, s));
            if (gf > 0) {
                if (mixed_)
                    hipLaunchKernelGGL((k_cg_xp<float, R, VEC>), grid, blk, 0, s, (float*)w_.xs, N2_, p, r, N2_, N2_,
                                       w_.st[cur_], w_.st[1 - cur_], w_.part_pq, w_.part_rr, gf, 1);
                else
                    hipLaunchKernelGGL((k_cg_xp<double, R, VEC>), grid, blk, 0, s, X_, ldx2_, p, r, N2_, N2_,
                                       w_.st[cur_], w_.st[1 - cur_], w_.part_pq, w_.part_rr, gf, 0);
                SC_LAUNCH_CHECK();
                cur_ = 1 - cur_;
                continue;
            }
            // q = A p; for A = D^H D the D pass can also leave <p, q> = ||D p||^2
            int gpq = 0;
            SC_TRY(op_apply_norm(op_, mixed_, p, op_->n, q, op_->n, k_, w_.tmp, w_.part_pq, kMaxRedBlocks, &gpq, s));
            if (gpq == 0) {
                hipLaunchKernelGGL((k_cg_pq<R, VEC>), grid, blk, 0, s, p, q, N2_, N2_, w_.st[cur_], w_.part_pq);
                SC_LAUNCH_CHECK();
                gpq = g_;
            }
            if (mixed_)
                hipLaunchKernelGGL((k_cg_xr<float, R, VEC>), grid, blk, 0, s, (float*)w_.xs, N2_, r, p, q, N2_, N2_,
                                   w_.st[cur_], w_.part_pq, gpq, w_.part_rr);
            else
                hipLaunchKernelGGL((k_cg_xr<double, R, VEC>), grid, blk, 0, s, X_, ldx2_, r, p, q, N2_, N2_,
                                   w_.st[cur_], w_.part_pq, gpq, w_.part_rr);
            SC_LAUNCH_CHECK();
            hipLaunchKernelGGL((k_cg_p<R, VEC>), grid, blk, 0, s, p, r, N2_, N2_, w_.st[cur_], w_.st[1 - cur_],
                               w_.part_rr, g_, mixed_ ? 1 : 0);
            SC_LAUNCH_CHECK();
            cur_ = 1 - cur_;
        }
        return SC_OK;
    }

    sc_status check(bool* any_out) override {
        hipStream_t s = s_;
        R* r = (R*)w_.r;
        SC_HIP(hipMemcpyAsync(hst_.data(), w_.st[cur_], sizeof(CGCol) * k_, hipMemcpyDeviceToHost, s));
        SC_HIP(hipStreamSynchronize(s));
        bool any = false;
        std::vector<int> upd;
        int need = 0;        // iterations the slowest active column still needs, as estimated
        bool dirty = false;  // host-side state changes to copy back
        for (int j = 0; j < k_; ++j) {
            if (hst_[j].active) {
                if (hst_[j].rho < 0.98 * min_rho_[j]) {
                    min_rho_[j] = hst_[j].rho;
                    it_min_[j] = hst_[j].iters;
                } else if (hst_[j].iters - it_min_[j] >= kStallWindow) {
                    stop_stalled(j);
                    dirty = true;
                    // a recursion that stopped falling may have left the solution
                    // behind: the column keeps x as of its last reliable update
                    if (mixed_) SC_TRY(fill<float>((float*)w_.xs + (int64_t)j * N2_, N2_, 0.0f, s));
                }
            }
            any |= hst_[j].active != 0;
            if (mixed_ && hst_[j].flag != 0 && hst_[j].iters < hst_[j].maxit) upd.push_back(j);
            if (hst_[j].active) {
                const int di = hst_[j].iters - chk_it_[j];
                double est = kChunk;
                if (chk_it_[j] >= 0 && di > 0 && hst_[j].rho < chk_rho_[j] && hst_[j].rho > hst_[j].tol2) {
                    const double rate = std::log(hst_[j].rho / chk_rho_[j]) / di;  // < 0
                    est = std::ceil(std::log(hst_[j].tol2 / hst_[j].rho) / rate);
                }
                need = std::max(need, (int)std::min<double>(kChunk, std::max(1.0, est)));
            }
            chk_rho_[j] = hst_[j].rho;
            chk_it_[j] = hst_[j].iters;
        }
        chunk_ = need > 0 ? need : kChunk;
        if (dirty && upd.empty()) {
            SC_HIP(hipMemcpyAsync(w_.st[cur_], hst_.data(), sizeof(CGCol) * k_, hipMemcpyHostToDevice, s));
            SC_HIP(hipStreamSynchronize(s));
        }
        if (!upd.empty()) {
            // reliable update of the flagged columns (batched over the list):
            // x64 += xs; xs = 0; r64 = b - A64 x64; r = r64; then the direction
            const dim3 blk(kBlock);
            const int nu = (int)upd.size();
            const int gr = red_grid(N2_, 4);
            SC_HIP(hipMemcpyAsync(w_.cols, upd.data(), sizeof(int) * nu, hipMemcpyHostToDevice, s));
            const bool all = nu == k_;  // the list is then 0..k-1 in order
            hipLaunchKernelGGL(k_ru_gather, dim3(gr, nu), blk, 0, s, w_.cols, X_, ldx2_, (float*)w_.xs,
                               all ? nullptr : w_.xg, N2_);
            SC_LAUNCH_CHECK();
            if (all) SC_TRY(op_apply(op_, false, X_, ldx_, w_.ax64, op_->n, nu, w_.tmp64, s));
            else SC_TRY(op_apply(op_, false, w_.xg, op_->n, w_.ax64, op_->n, nu, w_.tmp64, s));
            hipLaunchKernelGGL(k_ru_resid, dim3(gr, nu), blk, 0, s, w_.cols, B_, ldb2_, w_.ax64, w_.r64, (float*)r,
                               N2_, w_.part);
            SC_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_dot_finish, dim3(nu), blk, 0, s, w_.part, gr, w_.rho);
            SC_LAUNCH_CHECK();
            SC_HIP(hipMemcpyAsync(hrr_.data(), w_.rho, sizeof(double) * nu, hipMemcpyDeviceToHost, s));
            SC_HIP(hipStreamSynchronize(s));
            std::vector<int> dl;
            std::vector<double> db;
            for (int c = 0; c < nu; ++c) {
                const int j = upd[c];
                CGCol& cc = hst_[j];
                const double rr = hrr_[c];
                const bool done = !(rr > cc.tol2);
                // the true residual should have fallen with the recursive one; if
                // it has not halved since the best one seen, or it is more than
                // twice the recursive residual norm (cc.rho is the recursion's
                // ||r||^2 at this check), the FP64 residual is at its rounding
                // floor and the kept direction no longer matches it
                const bool improved = rr < 0.5 * best_true_[j];
                const bool consistent = rr <= 4.0 * cc.rho;
                if (improved) {
                    best_true_[j] = rr;
                    nstall_[j] = 0;
                } else if (!done) {
                    ++nstall_[j];
                }
                if (!done && (cc.flag == 1 || !improved || !consistent)) {
                    // the FP32 recurrence reached tol but the true residual did not,
                    // or the true residual stopped following it: restart the
                    // direction from the true residual
                    dl.push_back(j);
                    db.push_back(0.0);
                }
                // otherwise (flag 2) p was formed from the recursive residual and is
                // kept; CG continues from the true residual (rho = ||r_true||^2)
                cc.rho = rr;
                cc.rho_prev = rr;
                cc.rmax2 = rr;
                cc.active = done ? 0 : 1;
                cc.flag = 0;
                min_rho_[j] = rr;
                it_min_[j] = cc.iters;
                if (!done && nstall_[j] >= kStallUpdates) stop_stalled(j);
                any |= cc.active != 0;
            }
            if (!dl.empty()) {
                SC_HIP(hipMemcpyAsync(w_.cols, dl.data(), sizeof(int) * dl.size(), hipMemcpyHostToDevice, s));
                SC_HIP(hipMemcpyAsync(w_.ru_beta, db.data(), sizeof(double) * db.size(), hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(k_ru_dir, dim3(gr, (unsigned)dl.size()), blk, 0, s, w_.cols, w_.ru_beta,
                                   (float*)w_.p, (const float*)r, N2_);
                SC_LAUNCH_CHECK();
            }
            SC_HIP(hipMemcpyAsync(w_.st[cur_], hst_.data(), sizeof(CGCol) * k_, hipMemcpyHostToDevice, s));
            SC_HIP(hipStreamSynchronize(s));
            // the updated columns measure their decay from the true residual on
            for (int c = 0; c < nu; ++c) {
                chk_rho_[upd[c]] = hst_[upd[c]].rho;
                chk_it_[upd[c]] = hst_[upd[c]].iters;
            }
        }
        *any_out = any;
        return SC_OK;
    }

    sc_status verify(bool* again_out) override {
        hipStream_t s = s_;
        const int vt = mixed_ ? 1 : 0;
        R* r = (R*)w_.r;
        R* p = (R*)w_.p;
        double* r64 = mixed_ ? w_.r64 : (double*)r;
        if (mixed_) {
            // fold any remaining FP32 increment into x
            SC_TRY(lincomb(0, X_, ldx2_, 0, X_, ldx2_, 1, w_.xs, N2_, N2_, k_, 1.0, 1.0, s));
            SC_TRY(fill<float>((float*)w_.xs, N2_ * k_, 0.0f, s));
        }
        // verify on the true residual
        SC_TRY(true_residual(op_, B_, ldb2_, X_, ldx2_, k_, w_, r64, N2_, w_.rho, s));
        SC_HIP(hipMemcpyAsync(hrr_.data(), w_.rho, sizeof(double) * k_, hipMemcpyDeviceToHost, s));
        SC_HIP(hipStreamSynchronize(s));
        bool again = false;
        for (int j = 0; j < k_; ++j) {
            const double bn = hst_[j].bnorm2;
            relres_[j] = bn > 0.0 ? std::sqrt(hrr_[j] / bn) : 0.0;
            if (bn > 0.0 && !(relres_[j] <= tol_) && hst_[j].iters < hst_[j].maxit) again = true;
        }
        *again_out = false;
        if (!again || restarts_ >= 5) return SC_OK;
        ++restarts_;
        // restart every column from its true residual (converged ones stay inactive)
        if (mixed_) SC_TRY(lincomb(1, r, N2_, 0, w_.r64, N2_, 0, nullptr, 0, N2_, k_, 1.0, 0.0, s));
        SC_TRY(lincomb(vt, p, N2_, vt, r, N2_, 0, nullptr, 0, N2_, k_, 1.0, 0.0, s));
        hipLaunchKernelGGL(k_cg_setup, dim3((k_ + 63) / 64), dim3(64), 0, s, w_.st[cur_], w_.rho, w_.bn, k_, tol_,
                           maxit_, 0);
        SC_LAUNCH_CHECK();
        SC_HIP(hipMemcpyAsync(hst_.data(), w_.st[cur_], sizeof(CGCol) * k_, hipMemcpyDeviceToHost, s));
        SC_HIP(hipStreamSynchronize(s));
        *again_out = true;
        return SC_OK;
    }

    void results(int* iters, double* relres, sc_status* result) const override {
        *result = SC_OK;
        for (int j = 0; j < k_; ++j) {
            iters[j] = hst_[j].iters;
            relres[j] = relres_[j];
            if (!(relres_[j] <= tol_)) *result = SC_NOT_CONVERGED;
        }
    }

   private:
    static constexpr double kInf = std::numeric_limits<double>::infinity();
    // iterations between host checks: at most kChunk, fewer when every active
    // column's residual decay since the previous check says it will reach tol
    // sooner (the check then comes when the last column converges)
    static constexpr int kChunk = 8;

    void stop_stalled(int j) {
        hst_[j].active = 0;
        hst_[j].flag = 0;
        hst_[j].maxit = hst_[j].iters;
    }

    const sc_op* op_;
    bool mixed_;
    const double* B_;
    double* X_;
    int k_;
    double tol_;
    int maxit_;
    CGWork w_;
    hipStream_t s_;
    int64_t N2_ = 0, ldb2_ = 0, ldx2_ = 0, ldx_ = 0;
    int g_ = 0;
    int cur_ = 0;  // index of the state copy the next iteration reads
    int chunk_ = kChunk;
    int restarts_ = 0;
    std::vector<CGCol> hst_;
    std::vector<double> hrr_, chk_rho_, min_rho_, best_true_, relres_;
    std::vector<int> chk_it_, it_min_, nstall_;
};

std::unique_ptr<CGRun> cg_make(const sc_op* op, int mixed, const void* B, int64_t ldb, void* X, int64_t ldx, int k,
                               double tol, int maxit, void* work, size_t work_bytes, hipStream_t s, sc_status* st) {
    Carver c(work, work_bytes);
    CGWork w = carve_cg(c, op, k, mixed != 0);
    *st = SC_OK;
    if (!c.ok()) {
        set_error("solve_cg: work buffer too small");
        *st = SC_ERR_WORKSPACE;
        return nullptr;
    }
    const bool cpl = is_complex(op->dtype);
    const int64_t N2 = op->n * (cpl ? 2 : 1);
    const int64_t mul = cpl ? 2 : 1;
    const double* Bd = (const double*)B;
    double* Xd = (double*)X;
    if (mixed) {
        // packs of 4 floats: columns of r, p, q, xs are N2 floats apart
        if ((N2 % 4) == 0) return std::make_unique<CGRunT<float, true>>(op, true, Bd, ldb, Xd, ldx, k, tol, maxit, w, s);
        return std::make_unique<CGRunT<float, false>>(op, true, Bd, ldb, Xd, ldx, k, tol, maxit, w, s);
    }
    const bool vec = (N2 % 2) == 0 && ((uintptr_t)X % 16) == 0 && ((ldx * mul) % 2) == 0;
    if (vec) return std::make_unique<CGRunT<double, true>>(op, false, Bd, ldb, Xd, ldx, k, tol, maxit, w, s);
    return std::make_unique<CGRunT<double, false>>(op, false, Bd, ldb, Xd, ldx, k, tol, maxit, w, s);
}

sc_status solve_cg(const sc_op* op, int mixed, const void* B, int64_t ldb, void* X, int64_t ldx, int k, double tol,
                   int maxit, int* iters, double* relres, void* work, size_t work_bytes, hipStream_t s) {
    sc_status st = SC_OK;
    std::unique_ptr<CGRun> cg = cg_make(op, mixed, B, ldb, X, ldx, k, tol, maxit, work, work_bytes, s, &st);
    if (!cg) return st;
    SC_TRY(cg->start());
    for (;;) {
        bool any = cg->any_active();
        while (any) {
            SC_TRY(cg->iterate(cg->chunk()));
            SC_TRY(cg->check(&any));
        }
        bool again = false;
        SC_TRY(cg->verify(&again));
        if (!again) break;
    }
    sc_status result = SC_OK;
    cg->results(iters, relres, &result);
    if (result == SC_NOT_CONVERGED)
        set_error("solve_cg: some right-hand side is above tol (iteration limit reached or residual stalled)");
    return result;
}

}  // namespace sc
