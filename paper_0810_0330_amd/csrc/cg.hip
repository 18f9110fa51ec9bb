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
            Pack<R> xv = ldp((R*)xc, i0), pv = ldp(pc, i0);
#pragma unroll
            for (int e = 0; e < W; ++e) xv.v[e] = xv.v[e] + aR * pv.v[e];
            stp((R*)xc, i0, xv);
            if (cont) {
                const Pack<R> rv = ldp(rc, i0);
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

template <typename R, bool VEC>
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
    // iterations between host checks: at most kChunk, fewer when every active
    // column's residual decay since the previous check says it will reach tol
    // sooner (the check then comes when the last column converges)
    constexpr int kChunk = 8;
    int chunk = kChunk;
    std::vector<double> chk_rho(k, 0.0);
    std::vector<int> chk_it(k, -1);
    int cur = 0;  // index of the state copy the next iteration reads
    // stall detection (see the file header)
    constexpr double kInf = std::numeric_limits<double>::infinity();
    std::vector<double> min_rho(k, kInf), best_true(k, kInf);
    std::vector<int> it_min(k, 0), nstall(k, 0);
    auto stop_stalled = [&](int j) {
        hst[j].active = 0;
        hst[j].flag = 0;
        hst[j].maxit = hst[j].iters;
    };

    SC_TRY(dot(0, B, ldb2, 0, B, ldb2, N2, k, w.bn, w.part, nullptr, s));
    // r = b - A x; rho = ||r||^2
    double* r64 = mixed ? w.r64 : (double*)r;
    SC_TRY(true_residual(op, B, ldb2, X, ldx2, k, w, r64, N2, w.rho, s));
    if (mixed) {
        SC_TRY(lincomb(1, r, N2, 0, r64, N2, 0, nullptr, 0, N2, k, 1.0, 0.0, s));
        SC_TRY(fill<float>((float*)w.xs, N2 * k, 0.0f, s));
    }
    SC_TRY(lincomb(vt, p, N2, vt, r, N2, 0, nullptr, 0, N2, k, 1.0, 0.0, s));
    hipLaunchKernelGGL(k_cg_setup, dim3((k + 63) / 64), dim3(64), 0, s, w.st[cur], w.rho, w.bn, k, tol, maxit, 1);
    SC_LAUNCH_CHECK();

    // columns with b = 0 are solved by x = 0
    SC_HIP(hipMemcpyAsync(hst.data(), w.st[cur], sizeof(CGCol) * k, hipMemcpyDeviceToHost, s));
    SC_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < k; ++j)
        if (!(hst[j].bnorm2 > 0.0)) SC_TRY(lincomb(0, X + j * ldx2, N2, 0, X + j * ldx2, N2, 0, nullptr, 0, N2, 1, 0.0, 0.0, s));

    int restarts = 0;
    for (;;) {
        bool any = false;
        for (int j = 0; j < k; ++j) any |= hst[j].active != 0;
        while (any) {
            for (int it = 0; it < chunk; ++it) {
                // fused form (Wilson, t-march shape): D pass with <p, A p> partials, D^H pass
                // finishing r -= alpha A p, then x += alpha p and p = r + beta p
                int gf = 0;
                SC_TRY(wilson_cg_fused(op, mixed, p, w.tmp, k, w.st[cur], w.part_pq, r, op->n, w.part_rr,
                                       kMaxRedBlocks, &gf, s));
                if (gf > 0) {
                    if (mixed)
                        hipLaunchKernelGGL((k_cg_xp<float, R, VEC>), grid, blk, 0, s, (float*)w.xs, N2, p, r, N2, N2,
                                           w.st[cur], w.st[1 - cur], w.part_pq, w.part_rr, gf, 1);
                    else
                        hipLaunchKernelGGL((k_cg_xp<double, R, VEC>), grid, blk, 0, s, X, ldx2, p, r, N2, N2,
                                           w.st[cur], w.st[1 - cur], w.part_pq, w.part_rr, gf, 0);
                    SC_LAUNCH_CHECK();
                    cur = 1 - cur;
                    continue;
                }
                // q = A p; for A = D^H D the D pass can also leave <p, q> = ||D p||^2
                int gpq = 0;
                SC_TRY(op_apply_norm(op, mixed, p, op->n, q, op->n, k, w.tmp, w.part_pq, kMaxRedBlocks, &gpq, s));
                if (gpq == 0) {
                    hipLaunchKernelGGL((k_cg_pq<R, VEC>), grid, blk, 0, s, p, q, N2, N2, w.st[cur], w.part_pq);
                    SC_LAUNCH_CHECK();
                    gpq = g;
                }
                if (mixed)
                    hipLaunchKernelGGL((k_cg_xr<float, R, VEC>), grid, blk, 0, s, (float*)w.xs, N2, r, p, q, N2, N2,
                                       w.st[cur], w.part_pq, gpq, w.part_rr);
                else
                    hipLaunchKernelGGL((k_cg_xr<double, R, VEC>), grid, blk, 0, s, X, ldx2, r, p, q, N2, N2,
                                       w.st[cur], w.part_pq, gpq, w.part_rr);
                SC_LAUNCH_CHECK();
                hipLaunchKernelGGL((k_cg_p<R, VEC>), grid, blk, 0, s, p, r, N2, N2, w.st[cur], w.st[1 - cur],
                                   w.part_rr, g, mixed ? 1 : 0);
                SC_LAUNCH_CHECK();
                cur = 1 - cur;
            }
            SC_HIP(hipMemcpyAsync(hst.data(), w.st[cur], sizeof(CGCol) * k, hipMemcpyDeviceToHost, s));
            SC_HIP(hipStreamSynchronize(s));
            any = false;
            std::vector<int> upd;
            int need = 0;  // iterations the slowest active column still needs, as estimated
            bool dirty = false;  // host-side state changes to copy back
            for (int j = 0; j < k; ++j) {
                if (hst[j].active) {
                    if (hst[j].rho < 0.98 * min_rho[j]) {
                        min_rho[j] = hst[j].rho;
                        it_min[j] = hst[j].iters;
                    } else if (hst[j].iters - it_min[j] >= kStallWindow) {
                        stop_stalled(j);
                        dirty = true;
                        // a recursion that stopped falling may have left the solution
                        // behind: the column keeps x as of its last reliable update
                        if (mixed) SC_TRY(fill<float>((float*)w.xs + (int64_t)j * N2, N2, 0.0f, s));
                    }
                }
                any |= hst[j].active != 0;
                if (mixed && hst[j].flag != 0 && hst[j].iters < hst[j].maxit) upd.push_back(j);
                if (hst[j].active) {
                    const int di = hst[j].iters - chk_it[j];
                    double est = kChunk;
                    if (chk_it[j] >= 0 && di > 0 && hst[j].rho < chk_rho[j] && hst[j].rho > hst[j].tol2) {
                        const double rate = std::log(hst[j].rho / chk_rho[j]) / di;  // < 0
                        est = std::ceil(std::log(hst[j].tol2 / hst[j].rho) / rate);
                    }
                    need = std::max(need, (int)std::min<double>(kChunk, std::max(1.0, est)));
                }
                chk_rho[j] = hst[j].rho;
                chk_it[j] = hst[j].iters;
            }
            chunk = need > 0 ? need : kChunk;
            if (dirty && upd.empty()) {
                SC_HIP(hipMemcpyAsync(w.st[cur], hst.data(), sizeof(CGCol) * k, hipMemcpyHostToDevice, s));
                SC_HIP(hipStreamSynchronize(s));
            }
            if (!upd.empty()) {
                // reliable update of the flagged columns (batched over the list):
                // x64 += xs; xs = 0; r64 = b - A64 x64; r = r64; then the direction
                const int nu = (int)upd.size();
                const int gr = red_grid(N2, 4);
                SC_HIP(hipMemcpyAsync(w.cols, upd.data(), sizeof(int) * nu, hipMemcpyHostToDevice, s));
                const bool all = nu == k;  // the list is then 0..k-1 in order
                hipLaunchKernelGGL(k_ru_gather, dim3(gr, nu), blk, 0, s, w.cols, X, ldx2, (float*)w.xs,
                                   all ? nullptr : w.xg, N2);
                SC_LAUNCH_CHECK();
                if (all) SC_TRY(op_apply(op, false, X, ldx, w.ax64, op->n, nu, w.tmp64, s));
                else SC_TRY(op_apply(op, false, w.xg, op->n, w.ax64, op->n, nu, w.tmp64, s));
                hipLaunchKernelGGL(k_ru_resid, dim3(gr, nu), blk, 0, s, w.cols, B, ldb2, w.ax64, w.r64, (float*)r, N2,
                                   w.part);
                SC_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_dot_finish, dim3(nu), blk, 0, s, w.part, gr, w.rho);
                SC_LAUNCH_CHECK();
                SC_HIP(hipMemcpyAsync(hrr.data(), w.rho, sizeof(double) * nu, hipMemcpyDeviceToHost, s));
                SC_HIP(hipStreamSynchronize(s));
                std::vector<double> hb(nu);
                std::vector<int> dl;
                std::vector<double> db;
                for (int c = 0; c < nu; ++c) {
                    const int j = upd[c];
                    CGCol& cc = hst[j];
                    const double rr = hrr[c];
                    const bool done = !(rr > cc.tol2);
                    // the true residual should have fallen with the recursive one; if
                    // it has not halved since the best one seen, or it is more than
                    // twice the recursive residual norm (cc.rho is the recursion's
                    // ||r||^2 at this check), the FP64 residual is at its rounding
                    // floor and the kept direction no longer matches it
                    const bool improved = rr < 0.5 * best_true[j];
                    const bool consistent = rr <= 4.0 * cc.rho;
                    if (improved) {
                        best_true[j] = rr;
                        nstall[j] = 0;
                    } else if (!done) {
                        ++nstall[j];
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
                    min_rho[j] = rr;
                    it_min[j] = cc.iters;
                    if (!done && nstall[j] >= kStallUpdates) stop_stalled(j);
                    any |= cc.active != 0;
                }
                if (!dl.empty()) {
                    SC_HIP(hipMemcpyAsync(w.cols, dl.data(), sizeof(int) * dl.size(), hipMemcpyHostToDevice, s));
                    SC_HIP(hipMemcpyAsync(w.ru_beta, db.data(), sizeof(double) * db.size(), hipMemcpyHostToDevice, s));
                    hipLaunchKernelGGL(k_ru_dir, dim3(gr, (unsigned)dl.size()), blk, 0, s, w.cols, w.ru_beta, (float*)p,
                                       (const float*)r, N2);
                    SC_LAUNCH_CHECK();
                }
                SC_HIP(hipMemcpyAsync(w.st[cur], hst.data(), sizeof(CGCol) * k, hipMemcpyHostToDevice, s));
                SC_HIP(hipStreamSynchronize(s));
                // the updated columns measure their decay from the true residual on
                for (int c = 0; c < nu; ++c) {
                    chk_rho[upd[c]] = hst[upd[c]].rho;
                    chk_it[upd[c]] = hst[upd[c]].iters;
                }
            }
        }
        if (mixed) {
            // fold any remaining FP32 increment into x
            SC_TRY(lincomb(0, X, ldx2, 0, X, ldx2, 1, w.xs, N2, N2, k, 1.0, 1.0, s));
            SC_TRY(fill<float>((float*)w.xs, N2 * k, 0.0f, s));
        }
        // verify on the true residual
        SC_TRY(true_residual(op, B, ldb2, X, ldx2, k, w, r64, N2, w.rho, s));
        SC_HIP(hipMemcpyAsync(hrr.data(), w.rho, sizeof(double) * k, hipMemcpyDeviceToHost, s));
        SC_HIP(hipStreamSynchronize(s));
        bool again = false;
        for (int j = 0; j < k; ++j) {
            const double bn = hst[j].bnorm2;
            relres[j] = bn > 0.0 ? std::sqrt(hrr[j] / bn) : 0.0;
            iters[j] = hst[j].iters;
            if (bn > 0.0 && !(relres[j] <= tol) && hst[j].iters < hst[j].maxit) again = true;
        }
        if (!again || restarts >= 5) break;
        ++restarts;
        // restart every column from its true residual (converged ones stay inactive)
        if (mixed) SC_TRY(lincomb(1, r, N2, 0, w.r64, N2, 0, nullptr, 0, N2, k, 1.0, 0.0, s));
        SC_TRY(lincomb(vt, p, N2, vt, r, N2, 0, nullptr, 0, N2, k, 1.0, 0.0, s));
        hipLaunchKernelGGL(k_cg_setup, dim3((k + 63) / 64), dim3(64), 0, s, w.st[cur], w.rho, w.bn, k, tol, maxit, 0);
        SC_LAUNCH_CHECK();
        SC_HIP(hipMemcpyAsync(hst.data(), w.st[cur], sizeof(CGCol) * k, hipMemcpyDeviceToHost, s));
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
    const bool cpl = is_complex(op->dtype);
    const int64_t N2 = op->n * (cpl ? 2 : 1);
    const int64_t mul = cpl ? 2 : 1;
    if (mixed) {
        // packs of 4 floats: columns of r, p, q, xs are N2 floats apart
        const bool vec = (N2 % 4) == 0;
        if (vec) SC_TRY((cg_run<float, true>(op, true, (const double*)B, ldb, (double*)X, ldx, k, tol, maxit, iters, relres, w, s, &result)));
        else SC_TRY((cg_run<float, false>(op, true, (const double*)B, ldb, (double*)X, ldx, k, tol, maxit, iters, relres, w, s, &result)));
    } else {
        const bool vec = (N2 % 2) == 0 && ((uintptr_t)X % 16) == 0 && ((ldx * mul) % 2) == 0;
        if (vec) SC_TRY((cg_run<double, true>(op, false, (const double*)B, ldb, (double*)X, ldx, k, tol, maxit, iters, relres, w, s, &result)));
        else SC_TRY((cg_run<double, false>(op, false, (const double*)B, ldb, (double*)X, ldx, k, tol, maxit, iters, relres, w, s, &result)));
    }
    if (result == SC_NOT_CONVERGED)
        set_error("solve_cg: some right-hand side is above tol (iteration limit reached or residual stalled)");
    return result;
}

}  // namespace sc
