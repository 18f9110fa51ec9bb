// MINRES (Paige and Saunders) for Hermitian, possibly indefinite A, batched
// over k columns with per-column scalars in device memory: the solver that
// finishes each system of the indefinite variant of the seed method (gamma_5 D:
// Section 4 names it as the alternative to A^H A; Section 3 names the QR
// factorization of the Lanczos tridiagonal matrix it needs).  FP64.
//
// Iteration k for one column (Lanczos on A, then the reflection of the
// previous step and a new one on column k of the tridiagonal matrix):
//   p = A v_k;  alpha_k = Re(v_k^H p);  p -= alpha_k v_k + beta_k v_{k-1};
//   beta_{k+1} = ||p||;  v_{k+1} = p / beta_{k+1}
//   delta2 = c' delta1 + s' alpha_k;  gamma1 = s' delta1 - c' alpha_k
//   eps' = s' beta_{k+1};  delta1' = -c' beta_{k+1}
//   gamma2 = |(gamma1, beta_{k+1})|;  c = gamma1 / gamma2;  s = beta_{k+1} / gamma2
//   tau = c phibar;  phibar = s phibar  (|phibar| = ||r_k||)
//   w_k = (v_k - delta2 w_{k-1} - eps w_{k-2}) / gamma2;  x += tau w_k
// It stops when |phibar| <= tol ||b||; the start (r = b - A x, beta_1 = ||r||)
// is also the true-residual check, so a finished batch is started again and
// the columns whose true residual is at tol stay inactive (at most 5 restarts,
// as the CG does).  A column stops early and is reported as not converged
// when its residual cannot reach tol: the rotated residual norm has not
// fallen by 1% within kStallWindow iterations (tol below the attainable
// residual), or ||A r_k|| has fallen to max(tol, sqrt(eps)) ||A|| ||r_k|| (the estimate of
// ||A|| being the Frobenius norm of the tridiagonal matrix so far), the
// least-squares stop of Paige and Saunders: r_k is then a null vector of A to
// that accuracy (an inconsistent system), and in finite precision the rotated
// residual keeps drifting down below the true one.  Its iteration limit is
// lowered to the count reached, so no restart takes it up again.
#include "sc_internal.h"

#include <cmath>
#include <vector>

namespace sc {

namespace {

constexpr int kStallWindow = 1000;
constexpr double kLsqFloor = 1.4901161193847656e-8;  // sqrt(DBL_EPSILON): least-squares stop (see k_mr_update)

struct MRCol {
    double beta;    // beta_k (the norm that scales v_k)
    double c, s;    // the previous reflection
    double delta1;  // delta_k^(1)
    double eps;     // epsilon_k^(1)
    double phibar;  // the rotated residual norm
    double alpha;   // alpha_k of the current iteration
    double bnorm;   // ||b||
    double tol;
    double relres;  // true relative residual at the last start
    double tnorm2;  // squared Frobenius norm of the tridiagonal matrix so far (estimate of ||A||^2)
    int active, iters, maxit, pad;
};

struct MRWork {
    double* v[2];   // v_{k-1}, v_k (swapped by the host)
    double* p;
    double* w[2];   // w_{k-2}, w_{k-1}
    double* ax;     // A x at a start
    double* tmp;    // operator scratch
    double* part_a;
    double* part_f;
    MRCol* st[2];
};

MRWork carve(Carver& c, const sc_op* op, int k) {
    const int64_t N2 = op->n * (is_complex(op->dtype) ? 2 : 1);
    MRWork w;
    for (int i = 0; i < 2; ++i) w.v[i] = c.take<double>((size_t)N2 * k);
    w.p = c.take<double>((size_t)N2 * k);
    for (int i = 0; i < 2; ++i) w.w[i] = c.take<double>((size_t)N2 * k);
    w.ax = c.take<double>((size_t)N2 * k);
    w.tmp = c.take<double>((size_t)std::max<int64_t>(op_apply_tmp_elems(op) * (is_complex(op->dtype) ? 2 : 1), 1) * k);
    w.part_a = c.take<double>((size_t)kMaxRedBlocks * k);
    w.part_f = c.take<double>((size_t)kMaxRedBlocks * k);
    for (int i = 0; i < 2; ++i) w.st[i] = c.take<MRCol>(k);
    return w;
}

// ||b||, tol and maxit of each column; everything else is set by k_mr_start
__global__ void k_mr_setup(MRCol* st, const double* part, int G, int k, double tol, int maxit) {
    __shared__ double sh[kWaves];
    const int j = blockIdx.x;
    if (j >= k) return;
    const double bb = sum_partials(part + (int64_t)j * G, G, sh);
    if (threadIdx.x == 0) {
        MRCol c{};
        c.bnorm = sqrt(bb);
        c.tol = tol;
        c.maxit = maxit;
        c.iters = 0;
        st[j] = c;
    }
}

// partials of ||x||^2 per block and column
__global__ __launch_bounds__(kBlock) void k_mr_norm(const double* __restrict__ x, int64_t ldx, int64_t N,
                                                    double* part) {
    __shared__ double sh[kWaves];
    const double* xc = x + blockIdx.y * ldx;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock)
        acc += xc[i] * xc[i];
    block_partial(acc, part + (int64_t)blockIdx.y * gridDim.x, sh);
}

// r = b - A x (already in v), beta_1 = ||r|| from the partials; columns at tol
// (or out of iterations) stay inactive; the others get v_1 = r / beta_1 and
// zero v_0, w_0, w_{-1}
__global__ __launch_bounds__(kBlock) void k_mr_start(MRCol* st, double* __restrict__ v, double* __restrict__ v0,
                                                     double* __restrict__ w0, double* __restrict__ w1, int64_t N,
                                                     const double* part, int G) {
    __shared__ double sh[kWaves];
    const int j = blockIdx.y;
    MRCol c = st[j];
    const double b1 = sqrt(sum_partials(part + (int64_t)j * G, G, sh));
    const bool run = c.bnorm > 0.0 && b1 > c.tol * c.bnorm && c.iters < c.maxit && isfinite(b1);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c.relres = c.bnorm > 0.0 ? b1 / c.bnorm : 0.0;
        c.active = run ? 1 : 0;
        c.beta = b1;
        c.phibar = b1;
        c.c = -1.0;
        c.s = 0.0;
        c.delta1 = 0.0;
        c.eps = 0.0;
        c.tnorm2 = 0.0;
        st[j] = c;
    }
    if (!run) return;
    const double inv = 1.0 / b1;
    double* vc = v + j * N;
    double* v0c = v0 + j * N;
    double* w0c = w0 + j * N;
    double* w1c = w1 + j * N;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock) {
        vc[i] = vc[i] * inv;
        v0c[i] = 0.0;
        w0c[i] = 0.0;
        w1c[i] = 0.0;
    }
}

// partials of Re(v^H p)
__global__ __launch_bounds__(kBlock) void k_mr_alpha(const MRCol* st, const double* __restrict__ v,
                                                     const double* __restrict__ p, int64_t N, double* part) {
    __shared__ double sh[kWaves];
    const int j = blockIdx.y;
    if (!st[j].active) return;
    const double* vc = v + j * N;
    const double* pc = p + j * N;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock)
        acc += vc[i] * pc[i];
    block_partial(acc, part + (int64_t)j * gridDim.x, sh);
}

// alpha_k from the partials; p -= alpha_k v_k + beta_k v_{k-1}; partials of ||p||^2
__global__ __launch_bounds__(kBlock) void k_mr_f(MRCol* st, const double* __restrict__ v,
                                                 const double* __restrict__ vprev, double* __restrict__ p, int64_t N,
                                                 const double* part_a, int G, double* part_f) {
    __shared__ double sh[kWaves];
    const int j = blockIdx.y;
    if (!st[j].active) return;
    const double a = sum_partials(part_a + (int64_t)j * G, G, sh);
    const double b = st[j].beta;
    if (blockIdx.x == 0 && threadIdx.x == 0) st[j].alpha = a;
    const double* vc = v + j * N;
    const double* vp = vprev + j * N;
    double* pc = p + j * N;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock) {
        const double f = pc[i] - a * vc[i] - b * vp[i];
        pc[i] = f;
        acc += f * f;
    }
    block_partial(acc, part_f + (int64_t)j * gridDim.x, sh);
}

// beta_{k+1}, the reflections, w_k into wnew (the buffer of w_{k-2}),
// x += tau w_k, v_{k+1} into vnext (the buffer of v_{k-1}); state into st_next
__global__ __launch_bounds__(kBlock) void k_mr_update(const MRCol* st, MRCol* st_next, const double* __restrict__ v,
                                                      double* __restrict__ vnext, const double* __restrict__ p,
                                                      const double* __restrict__ wprev, double* __restrict__ wnew,
                                                      double* __restrict__ X, int64_t ldx, int64_t N,
                                                      const double* part_f, int G) {
    __shared__ double sh[kWaves];
    const int j = blockIdx.y;
    MRCol c = st[j];
    if (!c.active) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st_next[j] = c;
        return;
    }
    const double bn = sqrt(sum_partials(part_f + (int64_t)j * G, G, sh));
    const double a = c.alpha;
    const double d2 = c.c * c.delta1 + c.s * a;
    const double g1 = c.s * c.delta1 - c.c * a;
    const double en = c.s * bn;
    const double d1n = -c.c * bn;
    const double g2 = sqrt(g1 * g1 + bn * bn);
    const double cc = g1 / g2, ss = bn / g2;
    const double tau = cc * c.phibar;
    const double ep = c.eps;
    const double inv_g2 = 1.0 / g2;
    const double inv_bn = bn > 0.0 ? 1.0 / bn : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        MRCol o = c;
        o.beta = bn;
        o.c = cc;
        o.s = ss;
        o.delta1 = d1n;
        o.eps = en;
        o.phibar = ss * c.phibar;
        o.iters = c.iters + 1;
        o.tnorm2 = c.tnorm2 + a * a + c.beta * c.beta + bn * bn;
        if (!(fabs(o.phibar) > c.tol * c.bnorm) || !(bn > 0.0) || !isfinite(o.phibar) || o.iters >= c.maxit)
            o.active = 0;
        // least-squares stop: ||A r|| / ||r|| = sqrt(g1^2 + d1n^2) has fallen to
        // max(tol, sqrt(eps)) times the estimate of ||A||, so r is a null vector of
        // A to that accuracy and no later iteration can reduce it.  In FP64 the
        // ratio bottoms out not far below sqrt(eps) = 1.5e-8 (about 1e-10 on an
        // inconsistent diagonal system), and the iterations after that point
        // let x grow without bound, so a smaller tol must not postpone the stop.
        if (o.active && !(sqrt(g1 * g1 + d1n * d1n) > fmax(c.tol, kLsqFloor) * sqrt(o.tnorm2))) {
            o.active = 0;
            o.maxit = o.iters;
        }
        st_next[j] = o;
    }
    const double* vc = v + j * N;
    double* vn = vnext + j * N;
    const double* pc = p + j * N;
    const double* wp = wprev + j * N;
    double* wn = wnew + j * N;  // holds w_{k-2} on entry
    double* xc = X + j * ldx;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock) {
        const double w = (vc[i] - d2 * wp[i] - ep * wn[i]) * inv_g2;
        wn[i] = w;
        xc[i] += tau * w;
        vn[i] = pc[i] * inv_bn;
    }
}

}  // namespace

size_t minres_workspace(const sc_op* op, int k) {
    Carver c(nullptr, 0);
    carve(c, op, std::max(k, 1));
    return c.off + 256;
}

sc_status minres_solve(const sc_op* op, const void* B, int64_t ldb, void* X, int64_t ldx, int k, double tol,
                       int maxit, int* iters, double* relres, void* work, size_t work_bytes, hipStream_t s) {
    Carver cv(work, work_bytes);
    MRWork w = carve(cv, op, k);
    if (!cv.ok()) {
        set_error("minres: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    const bool cpl = is_complex(op->dtype);
    const int64_t N2 = op->n * (cpl ? 2 : 1);
    const int64_t ldb2 = ldb * (cpl ? 2 : 1), ldx2 = ldx * (cpl ? 2 : 1);
    double* Xd = (double*)X;
    const int g = red_grid(N2);
    const dim3 grid(g, k), blk(kBlock);
    int cur = 0;   // state copy the next iteration reads
    int vi = 1;    // w.v[vi] is v_k, w.v[1 - vi] is v_{k-1}
    int wi = 1;    // w.w[wi] is w_{k-1}, w.w[1 - wi] is w_{k-2}
    std::vector<MRCol> hst(k);
    std::vector<double> mark(k, 0.0);  // rotated residual at the last 1% decrease
    std::vector<int> it_mark(k, 0);

    hipLaunchKernelGGL(k_mr_norm, grid, blk, 0, s, (const double*)B, ldb2, N2, w.part_a);
    SC_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mr_setup, dim3(k), blk, 0, s, w.st[cur], w.part_a, g, k, tol, maxit);
    SC_LAUNCH_CHECK();
    for (int restart = 0;; ++restart) {
        // start: r = b - A x in v_k, beta_1 = ||r|| (also the true-residual check)
        SC_TRY(op_apply(op, false, X, ldx, w.ax, op->n, k, w.tmp, s));
        SC_TRY(lincomb(0, w.v[vi], N2, 0, B, ldb2, 0, w.ax, N2, N2, k, 1.0, -1.0, s));
        hipLaunchKernelGGL(k_mr_norm, grid, blk, 0, s, w.v[vi], N2, N2, w.part_f);
        SC_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_mr_start, grid, blk, 0, s, w.st[cur], w.v[vi], w.v[1 - vi], w.w[0], w.w[1], N2,
                           w.part_f, g);
        SC_LAUNCH_CHECK();
        SC_HIP(hipMemcpyAsync(hst.data(), w.st[cur], sizeof(MRCol) * k, hipMemcpyDeviceToHost, s));
        SC_HIP(hipStreamSynchronize(s));
        bool any = false;
        for (int j = 0; j < k; ++j) any |= hst[j].active != 0;
        if (!any || restart > 5) break;
        // stall detection from this start on
        for (int j = 0; j < k; ++j) {
            mark[j] = std::fabs(hst[j].phibar);
            it_mark[j] = hst[j].iters;
        }
        while (any) {
            for (int it = 0; it < 8; ++it) {
                SC_TRY(op_apply(op, false, w.v[vi], op->n, w.p, op->n, k, w.tmp, s));
                hipLaunchKernelGGL(k_mr_alpha, grid, blk, 0, s, w.st[cur], w.v[vi], w.p, N2, w.part_a);
                SC_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_mr_f, grid, blk, 0, s, w.st[cur], w.v[vi], w.v[1 - vi], w.p, N2, w.part_a, g,
                                   w.part_f);
                SC_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_mr_update, grid, blk, 0, s, w.st[cur], w.st[1 - cur], w.v[vi], w.v[1 - vi],
                                   w.p, w.w[wi], w.w[1 - wi], Xd, ldx2, N2, w.part_f, g);
                SC_LAUNCH_CHECK();
                cur = 1 - cur;
                vi = 1 - vi;  // v_{k+1} was written over v_{k-1}
                wi = 1 - wi;  // w_k was written over w_{k-2}
            }
            SC_HIP(hipMemcpyAsync(hst.data(), w.st[cur], sizeof(MRCol) * k, hipMemcpyDeviceToHost, s));
            SC_HIP(hipStreamSynchronize(s));
            any = false;
            bool dirty = false;
            for (int j = 0; j < k; ++j) {
                if (hst[j].active) {
                    const double ph = std::fabs(hst[j].phibar);
                    if (ph <= 0.99 * mark[j]) {
                        mark[j] = ph;
                        it_mark[j] = hst[j].iters;
                    } else if (hst[j].iters - it_mark[j] >= kStallWindow) {
                        hst[j].active = 0;
                        hst[j].maxit = hst[j].iters;
                        dirty = true;
                    }
                }
                any |= hst[j].active != 0;
            }
            if (dirty) {
                SC_HIP(hipMemcpyAsync(w.st[cur], hst.data(), sizeof(MRCol) * k, hipMemcpyHostToDevice, s));
                SC_HIP(hipStreamSynchronize(s));
            }
        }
    }
    bool conv = true;
    for (int j = 0; j < k; ++j) {
        iters[j] = hst[j].iters;
        relres[j] = hst[j].relres;
        conv &= hst[j].bnorm == 0.0 || hst[j].relres <= tol;
    }
    // columns with b = 0 are solved by x = 0
    for (int j = 0; j < k; ++j)
        if (!(hst[j].bnorm > 0.0)) SC_TRY(lincomb(0, Xd + j * ldx2, N2, 0, Xd + j * ldx2, N2, 0, nullptr, 0, N2, 1, 0.0, 0.0, s));
    SC_HIP(hipStreamSynchronize(s));
    return conv ? SC_OK : SC_NOT_CONVERGED;
}

}  // namespace sc
