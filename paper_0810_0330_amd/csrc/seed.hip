// Seed phase: the Lanczos version of CG on right-hand side 1 (Section 3
// algorithm, steps 1-9), run for exactly m steps with periodic
// reorthogonalization.  All scalars (alpha_i, beta_i, the LU pivot delta_i used
// to detect an indefinite A) stay on the device; the host enqueues the whole
// phase without synchronising and reads the final state once.
//
// Steps 3, 4, 6 and 7 (the incremental w_i, x^1 and eta^j updates) are not
// formed per step: the seeded guesses are the Galerkin projection over the
// stored basis, X0 + V_m T_m^{-1} V_m^H R0, computed afterwards in one batched
// pass (two tall-skinny contractions and one tridiagonal solve).  x^1 is the
// same projection with V_m^H r0^1 = beta_0 e_1.
#include "sc_internal.h"

namespace sc {

constexpr double kBreakdownTol = 1e-12;  // beta_i <= kBreakdownTol * max |alpha_k|: invariant subspace

struct SeedState {
    double bsq;      // ||f||^2 of the current step
    double amax;     // max_k |alpha_k|
    double delta;    // LU pivot delta_i of T
    double vnorm2;   // ||v_i||^2 during reorthogonalization
    int halt;        // nonzero: stop every later kernel of the phase
    int halt_step;   // step at which halt was decided
    int status;      // sc_status of the halt
    int m_done;      // steps completed
};

__global__ void k_seed_init(SeedState* st) {
    st->bsq = 0.0;
    st->amax = 0.0;
    st->delta = 0.0;
    st->vnorm2 = 0.0;
    st->halt = 0;
    st->halt_step = 0;
    st->status = SC_OK;
    st->m_done = 0;
}

// beta_i = ||f|| after step 8 (step 9), with the breakdown and finiteness checks
__device__ void finish_beta(SeedState* st, double* beta, int i, double bsq) {
    const double b = sqrt(bsq);
    beta[i] = b;
    if (!isfinite(b)) {
        st->status = SC_ERR_NONFINITE;
        st->halt_step = i;
        st->m_done = i > 0 ? i - 1 : 0;
        st->halt = 1;
    } else if (i == 0 ? !(b > 0.0) : !(b > kBreakdownTol * st->amax)) {
        st->status = SC_BREAKDOWN;
        st->halt_step = i;
        st->m_done = i;
        st->halt = 1;
    } else {
        st->m_done = i;
    }
}

// ||x||^2 with the beta_i epilogue (i = 0: beta_0 of step 2)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_lz_norm(const R* __restrict__ x, int64_t N, double* beta, int i,
                                                    SeedState* st, double* part, unsigned* ctr) {
    __shared__ double sh[kWaves];
    if (st->halt) return;
    double acc = 0.0;
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < N; j += (int64_t)gridDim.x * kBlock) {
        const double v = (double)x[j];
        acc += v * v;
    }
    double tot;
    if (split_reduce(acc, part, ctr, &tot, sh) && threadIdx.x == 0) finish_beta(st, beta, i, tot);
}

// v_{i+1} = f / beta_i, stored as column i of V.  Runs after the halt decision of
// step i was taken by an earlier kernel, so it only reads the flags.
template <typename VT, typename FT>
__global__ __launch_bounds__(kBlock) void k_lz_next(VT* __restrict__ vnext, const FT* __restrict__ f, int64_t N,
                                                    const double* beta, int i, const SeedState* st) {
    const bool brk_here = st->halt && st->status == SC_BREAKDOWN && st->halt_step == i;
    if (st->halt && !brk_here) return;
    const FT b = (FT)beta[i];
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < N; j += (int64_t)gridDim.x * kBlock)
        vnext[j] = brk_here ? VT(0) : (VT)(f[j] / b);
}

// step 5, first half: f = A v_i - beta_{i-1} v_{i-1}; alpha_i = Re(v_i^H f)
// (+ the pivot delta_i = alpha_i - beta_{i-1}^2 / delta_{i-1} of step 6)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_lz_alpha(R* __restrict__ f, const R* __restrict__ Av,
                                                     const R* __restrict__ vi, const R* __restrict__ vprev,
                                                     int64_t N, const double* beta, double* alpha, int i,
                                                     SeedState* st, double* part, unsigned* ctr) {
    __shared__ double sh[kWaves];
    if (st->halt) return;
    const double bprev = i > 1 ? beta[i - 1] : 0.0;
    const R bp = (R)bprev;
    double acc = 0.0;
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < N; j += (int64_t)gridDim.x * kBlock) {
        const R fv = i > 1 ? Av[j] - bp * vprev[j] : Av[j];
        f[j] = fv;
        acc += (double)vi[j] * (double)fv;
    }
    double tot;
    if (split_reduce(acc, part, ctr, &tot, sh) && threadIdx.x == 0) {
        alpha[i - 1] = tot;
        const double d = (i == 1) ? tot : tot - bprev * bprev / st->delta;
        if (!isfinite(tot)) {
            st->status = SC_ERR_NONFINITE;
            st->halt_step = i;
            st->m_done = i - 1;
            st->halt = 1;
        } else if (!(d > 0.0)) {
            st->status = SC_ERR_NOT_PD;
            st->halt_step = i;
            st->m_done = i - 1;
            st->halt = 1;
        } else {
            st->delta = d;
            st->amax = fmax(st->amax, fabs(tot));
        }
    }
}

// step 5, second half: f -= alpha_i v_i (+ ||f||^2 and the beta_i epilogue
// when no reorthogonalization follows at this step)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_lz_f(R* __restrict__ f, const R* __restrict__ vi, int64_t N,
                                                 const double* alpha, double* beta, int i, int with_norm,
                                                 SeedState* st, double* part, unsigned* ctr) {
    __shared__ double sh[kWaves];
    if (st->halt) return;
    const R a = (R)alpha[i - 1];
    double acc = 0.0;
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < N; j += (int64_t)gridDim.x * kBlock) {
        const R fv = f[j] - a * vi[j];
        f[j] = fv;
        acc += (double)fv * (double)fv;
    }
    if (!with_norm) return;
    double tot;
    if (split_reduce(acc, part, ctr, &tot, sh) && threadIdx.x == 0) finish_beta(st, beta, i, tot);
}

// v /= sqrt(nrm2)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_scale_norm(R* __restrict__ v, int64_t N, const double* nrm2,
                                                       const int* halt) {
    if (*halt) return;
    const R nr = (R)sqrt(*nrm2);
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < N; j += (int64_t)gridDim.x * kBlock)
        v[j] = v[j] / nr;
}

// ----------------------------------------------------------------------------
struct SeedWork {
    void* av;        // A v_i          (vector precision)
    void* f;         // f              (vector precision)
    void* tmp;       // op scratch     (vector precision)
    double* r64;     // r0^1           (FP64)
    double* ax64;    // A x0           (FP64)
    void* tmp64;     // op scratch     (FP64)
    double* part;    // split-reduction partials
    unsigned* ctr;   // split-reduction counters (2)
    SeedState* st;
    double* G;       // reorthogonalization coefficients, (m) x 2 complex
    double* G2;      // one complex coefficient
    double* gpart;   // gemm_cn partials
    double* y;       // T^{-1} beta_0 e_1 (m complex)
    double* trid;    // LU work (2m)
};

static SeedWork carve_seed(Carver& c, const sc_op* op, int m, bool single) {
    const bool cpl = is_complex(op->dtype);
    const int64_t N2 = op->n * (cpl ? 2 : 1);
    const size_t vb = single ? 4 : 8;
    const int64_t tmpn = op_apply_tmp_elems(op) * (cpl ? 2 : 1);
    SeedWork w;
    w.av = c.take<char>(N2 * vb);
    w.f = c.take<char>(N2 * vb);
    w.tmp = c.take<char>(std::max<int64_t>(tmpn, 1) * vb);
    w.r64 = c.take<double>(N2);
    w.ax64 = c.take<double>(N2);
    w.tmp64 = c.take<double>(std::max<int64_t>(tmpn, 1));
    w.part = c.take<double>(kMaxRedBlocks);
    w.ctr = c.take<unsigned>(2);
    w.st = c.take<SeedState>(1);
    w.G = c.take<double>((size_t)std::max(m, 1) * 4);
    w.G2 = c.take<double>(4);
    w.gpart = c.take<double>(std::max(gemm_cn_part_doubles(op->n, std::max(m, 1), 2, cpl), (size_t)4 * 64));
    w.y = c.take<double>((size_t)std::max(m, 1) * 2);
    w.trid = c.take<double>((size_t)std::max(m, 1) * 2);
    return w;
}

size_t seed_workspace(const sc_op* op, int m, bool single) {
    Carver c(nullptr, 0);
    carve_seed(c, op, m, single);
    return c.off + 256;
}

template <typename R>
static sc_status seed_run(const sc_op* op, const void* b1, void* x1, int m, int freq, R* V, int64_t ldv,
                          double* alpha, double* beta, int* m_done, const SeedWork& w, hipStream_t s,
                          sc_status* result) {
    const bool single = sizeof(R) == 4;
    const bool cpl = is_complex(op->dtype);
    const int64_t N2 = op->n * (cpl ? 2 : 1);
    const int64_t ldv2 = ldv * (cpl ? 2 : 1);  // in reals
    const int rt = single ? 1 : 0;
    const int g = red_grid(N2);
    const dim3 blk(kBlock);
    R* f = (R*)w.f;
    R* av = (R*)w.av;
    int* halt = &w.st->halt;

    hipLaunchKernelGGL(k_seed_init, dim3(1), dim3(1), 0, s, w.st);
    SC_LAUNCH_CHECK();
    SC_TRY(fill<unsigned>(w.ctr, 2, 0u, s));

    // step 1: r0 = b1 - A x0 (FP64)
    SC_TRY(op_apply(op, false, x1, op->n, w.ax64, op->n, 1, w.tmp64, s));
    SC_TRY(lincomb(0, w.r64, N2, 0, b1, N2, 0, w.ax64, N2, N2, 1, 1.0, -1.0, s));
    // step 2: beta_0 = ||r0||, v_1 = r0 / beta_0
    hipLaunchKernelGGL(k_lz_norm<double>, dim3(g), blk, 0, s, w.r64, N2, beta, 0, w.st, w.part, w.ctr);
    SC_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_lz_next<R, double>), dim3(g), blk, 0, s, V, w.r64, N2, beta, 0, w.st);
    SC_LAUNCH_CHECK();

    for (int i = 1; i <= m; ++i) {
        R* vi = V + (int64_t)(i - 1) * ldv2;
        R* vprev = i > 1 ? V + (int64_t)(i - 2) * ldv2 : vi;
        R* vnext = V + (int64_t)i * ldv2;
        // step 5: f = A v_i - beta_{i-1} v_{i-1}; alpha_i; f -= alpha_i v_i
        SC_TRY(op_apply(op, single, vi, ldv, av, op->n, 1, w.tmp, s));
        hipLaunchKernelGGL(k_lz_alpha<R>, dim3(g), blk, 0, s, f, av, vi, vprev, N2, beta, alpha, i, w.st, w.part,
                           w.ctr);
        SC_LAUNCH_CHECK();
        const bool due = freq > 0 && i >= 2 && i % freq == 0;
        hipLaunchKernelGGL(k_lz_f<R>, dim3(g), blk, 0, s, f, vi, N2, alpha, beta, i, due ? 0 : 1, w.st, w.part,
                           w.ctr);
        SC_LAUNCH_CHECK();
        if (due) {
            // step 8: [v_i, f] -= V_{i-1} (V_{i-1}^H [v_i, f]); v_i /= ||v_i||; f -= v_i (v_i^H f)
            ColPtrs<const void> wc{};
            wc.p[0] = vi;
            wc.p[1] = f;
            ColPtrs<void> xc{};
            xc.p[0] = vi;
            xc.p[1] = f;
            SC_TRY(gemm_cn(cpl, single, V, ldv, op->n, i - 1, single, wc, 2, w.G, w.gpart, halt, s));
            SC_TRY(gemm_nn(cpl, single, V, ldv, op->n, i - 1, w.G, 2, single, xc, -1.0, halt, s));
            SC_TRY(dot(rt, vi, N2, rt, vi, N2, N2, 1, &w.st->vnorm2, w.part, w.ctr + 1, s));
            hipLaunchKernelGGL(k_scale_norm<R>, dim3(g), blk, 0, s, vi, N2, &w.st->vnorm2, halt);
            SC_LAUNCH_CHECK();
            ColPtrs<const void> fc{};
            fc.p[0] = f;
            ColPtrs<void> fo{};
            fo.p[0] = f;
            SC_TRY(gemm_cn(cpl, single, vi, ldv, op->n, 1, single, fc, 1, w.G2, w.gpart, halt, s));
            SC_TRY(gemm_nn(cpl, single, vi, ldv, op->n, 1, w.G2, 1, single, fo, -1.0, halt, s));
            hipLaunchKernelGGL(k_lz_norm<R>, dim3(g), blk, 0, s, f, N2, beta, i, w.st, w.part, w.ctr);
            SC_LAUNCH_CHECK();
        }
        // step 9: beta_i = ||f||, v_{i+1} = f / beta_i
        hipLaunchKernelGGL((k_lz_next<R, R>), dim3(g), blk, 0, s, vnext, f, N2, beta, i, w.st);
        SC_LAUNCH_CHECK();
    }

    SeedState hst;
    SC_HIP(hipMemcpyAsync(&hst, w.st, sizeof(SeedState), hipMemcpyDeviceToHost, s));
    SC_HIP(hipStreamSynchronize(s));
    *m_done = hst.m_done;
    *result = (sc_status)hst.status;
    // x^1 = x0 + V_md T_md^{-1} (beta_0 e_1)
    if (hst.m_done >= 1 && hst.status != SC_ERR_NONFINITE) {
        SC_TRY(tridiag_solve(alpha, beta, hst.m_done, w.y, 1, cpl, beta, w.trid, nullptr, s));
        ColPtrs<void> xc{};
        xc.p[0] = x1;
        SC_TRY(gemm_nn(cpl, single, V, ldv, op->n, hst.m_done, w.y, 1, false, xc, 1.0, nullptr, s));
    }
    return SC_OK;
}

sc_status seed_lanczos(const sc_op* op, const void* b1, void* x1, int m, int freq, void* V, int64_t ldv,
                       sc_dtype vdt, double* alpha, double* beta, int* m_done, void* work, size_t work_bytes,
                       hipStream_t s) {
    const bool single = is_single(vdt);
    Carver c(work, work_bytes);
    SeedWork w = carve_seed(c, op, m, single);
    if (!c.ok()) {
        set_error("seed_lanczos: work buffer too small");
        return SC_ERR_WORKSPACE;
    }
    sc_status result = SC_OK;
    if (single) SC_TRY(seed_run<float>(op, b1, x1, m, freq, (float*)V, ldv, alpha, beta, m_done, w, s, &result));
    else SC_TRY(seed_run<double>(op, b1, x1, m, freq, (double*)V, ldv, alpha, beta, m_done, w, s, &result));
    if (result == SC_ERR_NOT_PD) set_error("seed_lanczos: non-positive pivot, A is not positive definite");
    if (result == SC_ERR_NONFINITE) set_error("seed_lanczos: non-finite value in the Lanczos recurrence");
    return result;
}

}  // namespace sc
