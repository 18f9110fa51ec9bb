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
#include "sc_timer.h"
#include "wilson_dev.h"

namespace sc {

constexpr double kBreakdownTol = 1e-12;  // beta_i <= kBreakdownTol * max |alpha_k|: invariant subspace

// Device state of the phase.  Fields are written by block 0 of one kernel and
// read by later kernels only, except `halt`, which a kernel may set while its
// other blocks run: a block that already sees it skips work whose results the
// halt makes unused.
struct SeedState {
    double amax;     // max_k |alpha_k|
    int halt;        // nonzero: stop every later kernel of the phase
    int halt_step;   // step at which halt was decided
    int status;      // sc_status of the halt
    int m_done;      // steps completed
};

__global__ void k_seed_init(SeedState* st) {
    st->amax = 0.0;
    st->halt = 0;
    st->halt_step = 0;
    st->status = SC_OK;
    st->m_done = 0;
}

// partials of ||x||^2
template <typename R, bool VEC>
__global__ __launch_bounds__(kBlock) void k_norm_part(const R* __restrict__ x, int64_t N, double* part,
                                                      const int* halt) {
    __shared__ double sh[kWaves];
    if (halt && *halt) return;
    constexpr int W = Pack<R>::W;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock * W;
    for (int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * W; i0 < N; i0 += stride) {
        if (VEC && i0 + W <= N) {
            const Pack<R> a = ldp(x, i0);
#pragma unroll
            for (int e = 0; e < W; ++e) acc += (double)a.v[e] * (double)a.v[e];
        } else {
            for (int64_t j = i0; j < min(N, i0 + W); ++j) acc += (double)x[j] * (double)x[j];
        }
    }
    block_partial(acc, part, sh);
}

// step 9 (and step 2 for i = 0): beta_i = ||f|| from the partials, breakdown
// and finiteness checks, v_{i+1} = f / beta_i stored as column i of V
template <typename VT, typename FT, bool VEC>
__global__ __launch_bounds__(kBlock) void k_lz_next(VT* __restrict__ vnext, const FT* __restrict__ f, int64_t N,
                                                    double* beta, int i, SeedState* st, const double* part, int G) {
    __shared__ double sh[kWaves];
    if (st->halt) return;
    const double b = sqrt(sum_partials(part, G, sh));
    const bool fin = isfinite(b);
    const bool brk = fin && (i == 0 ? !(b > 0.0) : !(b > kBreakdownTol * st->amax));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        beta[i] = b;
        if (!fin) {
            st->status = SC_ERR_NONFINITE;
            st->halt_step = i;
            st->m_done = i > 0 ? i - 1 : 0;
            st->halt = 1;
        } else if (brk) {
            st->status = SC_BREAKDOWN;
            st->halt_step = i;
            st->m_done = i;
            st->halt = 1;
        } else {
            st->m_done = i;
        }
    }
    const FT bf = (FT)b;
    const bool zero = brk || !fin;
    if constexpr (VEC && sizeof(VT) == sizeof(FT)) {
        constexpr int W = Pack<FT>::W;
        const int64_t stride = (int64_t)gridDim.x * kBlock * W;
        for (int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * W; i0 < N; i0 += stride) {
            if (i0 + W <= N) {
                const Pack<FT> a = ldp(f, i0);
                Pack<FT> o;
#pragma unroll
                for (int e = 0; e < W; ++e) o.v[e] = zero ? FT(0) : a.v[e] / bf;
                stp((FT*)vnext, i0, o);
            } else {
                for (int64_t j = i0; j < N; ++j) vnext[j] = zero ? VT(0) : (VT)(f[j] / bf);
            }
        }
    } else {
        for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < N; j += (int64_t)gridDim.x * kBlock)
            vnext[j] = zero ? VT(0) : (VT)(f[j] / bf);
    }
}

// step 5, first half: f = A v_i - beta_{i-1} v_{i-1}; partials of Re(v_i^H f)
template <typename R, bool VEC>
__global__ __launch_bounds__(kBlock) void k_lz_alpha(R* __restrict__ f, const R* __restrict__ Av,
                                                     const R* __restrict__ vi, const R* __restrict__ vprev,
                                                     int64_t N, const double* beta, int i, const SeedState* st,
                                                     double* part) {
    __shared__ double sh[kWaves];
    if (st->halt) return;
    constexpr int W = Pack<R>::W;
    const R bp = (R)(i > 1 ? beta[i - 1] : 0.0);
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock * W;
    for (int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * W; i0 < N; i0 += stride) {
        if (VEC && i0 + W <= N) {
            const Pack<R> a = ldp(Av, i0), pv = ldp(vprev, i0), v = ldp(vi, i0);
            Pack<R> o;
#pragma unroll
            for (int e = 0; e < W; ++e) {
                o.v[e] = a.v[e] - bp * pv.v[e];
                acc += (double)v.v[e] * (double)o.v[e];
            }
            stp(f, i0, o);
        } else {
            for (int64_t j = i0; j < min(N, i0 + W); ++j) {
                const R fv = Av[j] - bp * vprev[j];
                f[j] = fv;
                acc += (double)vi[j] * (double)fv;
            }
        }
    }
    block_partial(acc, part, sh);
}

// step 5, second half: alpha_i from the partials (+ the LU pivot
// delta_i = alpha_i - beta_{i-1}^2 / delta_{i-1} of step 6, which must stay
// positive for an HPD A); f -= alpha_i v_i; partials of ||f||^2
template <typename R, bool VEC>
__global__ __launch_bounds__(kBlock) void k_lz_f(R* __restrict__ f, const R* __restrict__ vi, int64_t N,
                                                 double* alpha, const double* beta, double* delta, int i,
                                                 SeedState* st, const double* part_a, int G, double* part_f,
                                                 int indef) {
    __shared__ double sh[kWaves];
    if (st->halt) return;
    constexpr int W = Pack<R>::W;
    constexpr int UN = 8;  // packs per thread whose loads are issued before alpha is summed
    const int64_t stride = (int64_t)gridDim.x * kBlock * W;
    const int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * W;
    Pack<R> o[UN], v[UN];
    if constexpr (VEC) {
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int64_t j = i0 + u * stride;
            if (j + W <= N) {
                o[u] = ldp(f, j);
                v[u] = ldp(vi, j);
            }
        }
    }
    const double a = sum_partials(part_a, G, sh);
    // the LU pivot of step 6; an indefinite operator has no positive-pivot requirement
    const double d = (i == 1) ? a : a - beta[i - 1] * beta[i - 1] / delta[i - 1];
    const bool bad = !isfinite(a) || (!indef && !(d > 0.0));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        alpha[i - 1] = a;
        delta[i] = d;
        if (bad) {
            st->status = isfinite(a) ? SC_ERR_NOT_PD : SC_ERR_NONFINITE;
            st->halt_step = i;
            st->m_done = i - 1;
            st->halt = 1;
        } else {
            st->amax = fmax(st->amax, fabs(a));
        }
    }
    if (bad) return;
    const R aR = (R)a;
    double acc = 0.0;
    int64_t j = i0;
    if constexpr (VEC) {
        // the prefetched packs, in the order of the loop below
#pragma unroll
        for (int u = 0; u < UN; ++u, j += stride) {
            if (j + W > N) break;
#pragma unroll
            for (int e = 0; e < W; ++e) {
                o[u].v[e] = o[u].v[e] - aR * v[u].v[e];
                acc += (double)o[u].v[e] * (double)o[u].v[e];
            }
            stp(f, j, o[u]);
        }
    }
    for (; j < N; j += stride) {
        if (VEC && j + W <= N) {
            Pack<R> ov = ldp(f, j);
            const Pack<R> vv = ldp(vi, j);
#pragma unroll
            for (int e = 0; e < W; ++e) {
                ov.v[e] = ov.v[e] - aR * vv.v[e];
                acc += (double)ov.v[e] * (double)ov.v[e];
            }
            stp(f, j, ov);
        } else {
            for (int64_t q = j; q < min(N, j + W); ++q) {
                const R fv = f[q] - aR * vi[q];
                f[q] = fv;
                acc += (double)fv * (double)fv;
            }
        }
    }
    block_partial(acc, part_f, sh);
}

// ---------------------------------------------------------------- fused Wilson steps
// For the Wilson normal operator the two stencil passes of a Lanczos step carry
// the neighbouring vector work, on the direction-split launch shape (a block
// covers 64 sites, wave w the hops of direction w; partial results meet in
// LDS).  Two launches per step i >= 2:
//   D pass = step 9 of step i - 1 + the pass: beta_{i-1} = ||f|| from the
//     partials (the checks of k_lz_next), v_i = f / beta_{i-1} stored for the
//     block's sites, D v_i = (D f) / beta_{i-1}, and per 64-site tile its
//     share of alpha_i = ||D v_i||^2 - beta_{i-1} Re(v_i^H v_{i-1});
//   D^H pass = the pass + step 5: alpha_i as the sum of those shares (with
//     the LU pivot of step 6),
//     f = D^H (D v_i) - beta_{i-1} v_{i-1} - alpha_i v_i, and per tile the
//     partials of ||f||^2 for the next D pass.
// For A = D^H D, v^H A v = ||D v||^2, so this alpha_i is step 5's
// v_i^H (A v_i - beta_{i-1} v_{i-1}) in exact arithmetic; it is known before
// the D^H pass, which can then form the final f itself.  Step 1 (no v_0) takes
// the three-launch form: D^H pass with the partials of Re(v_1^H f), then
// k_lz_f.

// sum over the 4 direction waves of component j of spin mu, for lane l
template <typename R>
__device__ __forceinline__ cplx<R> dir_total(R (*red)[24][64], int mu, int cc, int l) {
    const int j = (mu * 3 + cc) * 2;
    return {red[0][j][l] + red[1][j][l] + red[2][j][l] + red[3][j][l],
            red[0][j + 1][l] + red[1][j + 1][l] + red[2][j + 1][l] + red[3][j + 1][l]};
}

template <typename R>
__device__ __forceinline__ void dir_stash(R (*red)[24][64], int mu, int l, const cplx<R> acc[4][3]) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            red[mu][(a * 3 + cc) * 2][l] = acc[a][cc].re;
            red[mu][(a * 3 + cc) * 2 + 1][l] = acc[a][cc].im;
        }
}

// The partials a fused pass needs, loaded into registers before its hops so
// that their latency overlaps the hops' own loads: the first kPre * kBlock of
// the G partials (the whole array up to 2048 tiles), the rest summed later.
// part_sum adds them in the order of sum_partials, so every block gets the
// same, deterministic total.
constexpr int kPre = 8;
template <int P = kPre>
struct PartPre {
    double v[P];
};
template <int P = kPre>
__device__ __forceinline__ PartPre<P> part_load(const double* __restrict__ part, int G) {
    PartPre<P> q;
#pragma unroll
    for (int u = 0; u < P; ++u) {
        const int j = (int)threadIdx.x + u * kBlock;
        q.v[u] = j < G ? part[j] : 0.0;
    }
    return q;
}
// The sum starts at -0.0, which the first addition absorbs exactly (x + -0.0 =
// x): with 0.0 the compiler moves that first addition into the conditional
// load of the first partial and waits for it there, before any other load of
// the kernel is issued.
template <int P>
__device__ __forceinline__ double part_sum(const PartPre<P>& q, const double* __restrict__ part, int G, double* sh) {
    double s = -0.0;
#pragma unroll
    for (int u = 0; u < P; ++u) s += q.v[u];
    for (int j = (int)threadIdx.x + P * kBlock; j < G; j += kBlock) s += part[j];
    return block_sum(s, sh);
}

template <typename R, typename VT, bool REC>
__global__ __launch_bounds__(kBlock) void k_lz_dnext(R* __restrict__ tmp, const R* __restrict__ f,
                                                     VT* __restrict__ vnext, const VT* __restrict__ vprev,
                                                     const R* __restrict__ U, Geom g, R kappa, R tsign, int ntile,
                                                     int per_xcd, double* beta, int im1, SeedState* st,
                                                     const double* part, int G, double* part_a) {
    __shared__ R red[4][24][64];
    __shared__ double sh[kWaves];
    const int b = blockIdx.x;
    const int L = (b % kXcd) * per_xcd + b / kXcd;
    if (L >= ntile) return;  // uniform over the block
    // the state is read here and acted on after every load of the pass has
    // been issued (the loads are in range whatever it says), so that its
    // latency is not one more round trip on the block's chain
    const int halted = st->halt;
    const double amax = st->amax;
    const int mu = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int s = L * 64 + l;
    const bool ok = s < (int)g.V;
    const unsigned uV = (unsigned)g.V;
    // the hops of D f first (they do not need beta), so that the latency of
    // the partial sum below overlaps their loads
    cplx<R> acc[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) acc[a][cc] = {R(0), R(0)};
    const PartPre<> pf = part_load(part, G);
    // the epilogue's own-site operands (f and v_{i-1} at the lane's 3
    // components), loaded with the partials so that the epilogue after the
    // barriers below waits on no memory
    cplx<R> fo[3];
    typename vec2<VT>::type po[3];
    if (ok)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            fo[cc] = ldc(f + 2 * (size_t)((mu * 3 + cc) * uV), (unsigned)s);
            po[cc] = reinterpret_cast<const typename vec2<VT>::type*>(vprev)[(mu * 3 + cc) * uV + s];
        }
    if (ok) {  // the x hops by DPP when a lane row is an x-row (X = 16)
        if (mu == 0 && g.X == 16) dir_hops_x16<false, R, REC>(acc, f, U, uV, s);
        else dir_hops<false, R, REC>(acc, f, U, g, uV, s, mu, tsign);
    }
    if (halted) return;  // uniform over the grid: an earlier step stopped the phase
    dir_stash(red, mu, l, acc);
    const double bn = sqrt(part_sum(pf, part, G, sh));  // its barriers also order the stash
    const bool fin = isfinite(bn);
    const bool brk = fin && !(bn > kBreakdownTol * amax);
    if (b == 0 && threadIdx.x == 0) {  // block 0 always holds a tile
        beta[im1] = bn;
        if (!fin) {
            st->status = SC_ERR_NONFINITE;
            st->halt_step = im1;
            st->m_done = im1 - 1;
            st->halt = 1;
        } else if (brk) {
            st->status = SC_BREAKDOWN;
            st->halt_step = im1;
            st->m_done = im1;
            st->halt = 1;
        } else {
            st->m_done = im1;
        }
    }
    if (brk || !fin) {  // the basis ends here: v_i = 0, as the separate step 9 stores
        if (ok)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                reinterpret_cast<typename vec2<VT>::type*>(vnext)[(mu * 3 + cc) * uV + s] =
                    typename vec2<VT>::type{VT(0), VT(0)};
        return;
    }
    const R rb = (R)(1.0 / bn);  // v_i = f / beta as f times 1 / beta (FP64 reciprocal, rounded once)
    // the lane's share of alpha_i = ||D v_i||^2 - beta_{i-1} Re(v_i^H v_{i-1}) over its 3 components
    double aacc = 0.0;
    if (ok) {
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            const cplx<R> h = dir_total(red, mu, cc, l);
            const size_t cb = 2 * (size_t)((mu * 3 + cc) * uV);
            const cplx<R> fv = fo[cc];
            const cplx<R> v = {fv.re * rb, fv.im * rb};                              // v_i
            const cplx<R> r = {(fv.re - kappa * h.re) * rb, (fv.im - kappa * h.im) * rb};  // D v_i
            const typename vec2<VT>::type vs{(VT)v.re, (VT)v.im};
            const typename vec2<VT>::type pv = po[cc];
            reinterpret_cast<typename vec2<R>::type*>(tmp + cb)[s] = typename vec2<R>::type{r.re, r.im};
            reinterpret_cast<typename vec2<VT>::type*>(vnext)[(mu * 3 + cc) * uV + s] = vs;
            aacc += (double)r.re * (double)r.re + (double)r.im * (double)r.im -
                    bn * ((double)vs.x * (double)pv.x + (double)vs.y * (double)pv.y);
        }
    }
    const double at = block_sum(aacc, sh);
    if (threadIdx.x == 0) part_a[L] = at;
}

template <typename R, bool REC>
__global__ __launch_bounds__(kBlock) void k_lz_dhalpha(R* __restrict__ f, const R* __restrict__ tmp,
                                                       const R* __restrict__ vi, const R* __restrict__ vprev,
                                                       const R* __restrict__ U, Geom g, R kappa, R tsign, int ntile,
                                                       int per_xcd, const double* beta, int i, const SeedState* st,
                                                       double* part) {
    __shared__ R red[4][24][64];
    __shared__ double sh[kWaves];
    if (st->halt) return;
    const int b = blockIdx.x;
    const int L = (b % kXcd) * per_xcd + b / kXcd;
    if (L >= ntile) return;  // uniform over the block
    const int mu = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int s = L * 64 + l;
    const bool ok = s < (int)g.V;
    const unsigned uV = (unsigned)g.V;
    cplx<R> acc[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) acc[a][cc] = {R(0), R(0)};
    if (ok) {  // the x hops by DPP when a lane row is an x-row (X = 16)
        if (mu == 0 && g.X == 16) dir_hops_x16<true, R, REC>(acc, tmp, U, uV, s);
        else dir_hops<true, R, REC>(acc, tmp, U, g, uV, s, mu, tsign);
    }
    dir_stash(red, mu, l, acc);
    __syncthreads();
    const R bp = (R)(i > 1 ? beta[i - 1] : 0.0);
    double dacc = 0.0;
    if (ok) {
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            const cplx<R> h = dir_total(red, mu, cc, l);
            const size_t cb = 2 * (size_t)((mu * 3 + cc) * uV);
            const cplx<R> t = ldc(tmp + cb, (unsigned)s);
            const cplx<R> av = {t.re - kappa * h.re, t.im - kappa * h.im};  // A v_i = D^H (D v_i)
            const cplx<R> pv = ldc(vprev + cb, (unsigned)s);
            const cplx<R> v = ldc(vi + cb, (unsigned)s);
            const cplx<R> fv = {av.re - bp * pv.re, av.im - bp * pv.im};
            reinterpret_cast<typename vec2<R>::type*>(f + cb)[s] = typename vec2<R>::type{fv.re, fv.im};
            dacc += (double)v.re * (double)fv.re + (double)v.im * (double)fv.im;
        }
    }
    const double tot = block_sum(dacc, sh);
    if (threadIdx.x == 0) part[L] = tot;
}

// D^H pass of step i >= 2: alpha_i from the D pass's partials, the pivot of
// step 6, and the final f = D^H (D v_i) - beta_{i-1} v_{i-1} - alpha_i v_i with
// the partials of ||f||^2
template <typename R, bool REC>
__global__ __launch_bounds__(kBlock) void k_lz_dhf(R* __restrict__ f, const R* __restrict__ tmp,
                                                   const R* __restrict__ vi, const R* __restrict__ vprev,
                                                   const R* __restrict__ U, Geom g, R kappa, R tsign, int ntile,
                                                   int per_xcd, double* alpha, const double* beta, double* delta,
                                                   int i, SeedState* st, const double* part_a, double* part_f,
                                                   int indef) {
    __shared__ R red[4][24][64];
    __shared__ double sh[kWaves];
    const int b = blockIdx.x;
    const int L = (b % kXcd) * per_xcd + b / kXcd;
    if (L >= ntile) return;  // uniform over the block
    // read here, acted on after the pass's loads are issued (as in k_lz_dnext)
    const int halted = st->halt;
    const double dprev = delta[i - 1];
    const int mu = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int s = L * 64 + l;
    const bool ok = s < (int)g.V;
    const unsigned uV = (unsigned)g.V;
    cplx<R> acc[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) acc[a][cc] = {R(0), R(0)};
    // 6 of the (up to) 8 partials per thread: the registers of the other 2
    // hold the epilogue's operands
    const PartPre<6> pa = part_load<6>(part_a, ntile);
    // the epilogue's own-site operands at the lane's 3 components, loaded with
    // the partials so that the epilogue after the barriers below waits on no
    // memory: D v_i - beta_{i-1} v_{i-1} (beta_{i-1} is known; the D pass
    // stored it) and v_i
    const double bp = beta[i - 1];
    const R bR = (R)bp;
    cplx<R> wo[3], vo[3];
    if (ok)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            const size_t cb = 2 * (size_t)((mu * 3 + cc) * uV);
            const cplx<R> t = ldc(tmp + cb, (unsigned)s);
            const cplx<R> pv = ldc(vprev + cb, (unsigned)s);
            wo[cc] = {t.re - bR * pv.re, t.im - bR * pv.im};
            vo[cc] = ldc(vi + cb, (unsigned)s);
        }
    if (ok) {  // the x hops by DPP when a lane row is an x-row (X = 16)
        if (mu == 0 && g.X == 16) dir_hops_x16<true, R, REC>(acc, tmp, U, uV, s);
        else dir_hops<true, R, REC>(acc, tmp, U, g, uV, s, mu, tsign);
    }
    if (halted) return;  // uniform over the grid: an earlier step stopped the phase
    dir_stash(red, mu, l, acc);
    // alpha_i from the D pass's per-tile shares (its barriers also order the
    // stash); every block adds the same partials in the same order, so every
    // block gets the same alpha
    const double a = part_sum(pa, part_a, ntile, sh);
    const double d = a - bp * bp / dprev;  // the LU pivot of step 6
    const bool bad = !isfinite(a) || (!indef && !(d > 0.0));
    if (b == 0 && threadIdx.x == 0) {  // block 0 always holds a tile
        alpha[i - 1] = a;
        delta[i] = d;
        if (bad) {
            st->status = isfinite(a) ? SC_ERR_NOT_PD : SC_ERR_NONFINITE;
            st->halt_step = i;
            st->m_done = i - 1;
            st->halt = 1;
        } else {
            st->amax = fmax(st->amax, fabs(a));
        }
    }
    if (bad) return;
    const R aR = (R)a;
    double facc = 0.0;
    if (ok) {
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            const cplx<R> h = dir_total(red, mu, cc, l);
            const size_t cb = 2 * (size_t)((mu * 3 + cc) * uV);
            const cplx<R> v = vo[cc];
            // f = A v_i - beta_{i-1} v_{i-1} - alpha_i v_i, A v_i = D^H (D v_i) = D v_i - kappa H (D v_i)
            const cplx<R> fv = {wo[cc].re - kappa * h.re - aR * v.re, wo[cc].im - kappa * h.im - aR * v.im};
            reinterpret_cast<typename vec2<R>::type*>(f + cb)[s] = typename vec2<R>::type{fv.re, fv.im};
            facc += (double)fv.re * (double)fv.re + (double)fv.im * (double)fv.im;
        }
    }
    const double tot = block_sum(facc, sh);
    if (threadIdx.x == 0) part_f[L] = tot;
}

// v /= ||v|| (norm from partials)
template <typename R>
__global__ __launch_bounds__(kBlock) void k_scale_norm(R* __restrict__ v, int64_t N, const double* part, int G,
                                                       const int* halt) {
    __shared__ double sh[kWaves];
    if (*halt) return;
    const R nr = (R)sqrt(sum_partials(part, G, sh));
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < N; j += (int64_t)gridDim.x * kBlock)
        v[j] = v[j] / nr;
}

// ----------------------------------------------------------------------------
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
    // per 64-site tile: its share of alpha from the fused D pass, of ||f||^2 from the fused D^H pass
    const int64_t ntile = (op->n / 12 + 63) / 64;
    w.part_a = c.take<double>(std::max<int64_t>(kMaxRedBlocks, ntile));
    w.part_f = c.take<double>(std::max<int64_t>(kMaxRedBlocks, ntile));
    w.part_v = c.take<double>(kMaxRedBlocks);
    w.delta = c.take<double>((size_t)m + 2);
    w.st = c.take<SeedState>(1);
    w.G = c.take<double>((size_t)std::max(m, 1) * 4);
    w.G2 = c.take<double>(4);
    w.gpart = c.take<double>(std::max(gemm_cn_part_doubles(op->n, std::max(m, 1), 2, cpl), (size_t)4 * 64));
    w.y = c.take<double>((size_t)(std::max(m, 1) + 1) * 2);
    w.trid = c.take<double>((size_t)std::max(m, 1) * 5);
    return w;
}

size_t seed_workspace(const sc_op* op, int m, bool single) {
    Carver c(nullptr, 0);
    carve_seed(c, op, m, single);
    return c.off + 256;
}

// Steps 1-9 for m steps, enqueued on `s` with no host synchronisation (the
// phase has static control flow, so it can be captured in a graph).
template <typename R, bool VEC>
static sc_status seed_enqueue(const sc_op* op, const void* b1, void* x1, int m, int freq, R* V, int64_t ldv,
                              double* alpha, double* beta, const SeedWork& w, hipStream_t s, bool indef_op) {
    const bool single = sizeof(R) == 4;
    const bool cpl = is_complex(op->dtype);
    const int64_t N2 = op->n * (cpl ? 2 : 1);
    const int64_t ldv2 = ldv * (cpl ? 2 : 1);  // in reals
    const int g = red_grid(N2);
    const dim3 blk(kBlock);
    R* f = (R*)w.f;
    R* av = (R*)w.av;
    int* halt = &w.st->halt;

    hipLaunchKernelGGL(k_seed_init, dim3(1), dim3(1), 0, s, w.st);
    SC_LAUNCH_CHECK();

    // step 1: r0 = b1 - A x0 (FP64); x1 == nullptr stands for x0 = 0, which is then not read
    if (x1) {
        SC_TRY(op_apply(op, false, x1, op->n, w.ax64, op->n, 1, w.tmp64, s));
        SC_TRY(lincomb(0, w.r64, N2, 0, b1, N2, 0, w.ax64, N2, N2, 1, 1.0, -1.0, s));
    } else {
        SC_TRY(lincomb(0, w.r64, N2, 0, b1, N2, 0, b1, N2, N2, 1, 1.0, 0.0, s));
    }
    // step 2: beta_0 = ||r0||, v_1 = r0 / beta_0
    hipLaunchKernelGGL((k_norm_part<double, VEC>), dim3(g), blk, 0, s, w.r64, N2, w.part_f, nullptr);
    SC_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_lz_next<R, double, false>), dim3(g), blk, 0, s, V, w.r64, N2, beta, 0, w.st, w.part_f, g);
    SC_LAUNCH_CHECK();

    // the fused Wilson form (direction-split passes carrying the vector work)
    const bool fused = op->kind == SC_OPK_WILSON && (!single || op->U32);
    const int indef = (indef_op || op->kind == SC_OPK_WILSON_G5) ? 1 : 0;  // Hermitian indefinite: no pivot check
    const Geom geo{op->dims[0], op->dims[1], op->dims[2], op->dims[3], op->vol};
    const int ntile = (int)((op->vol + 63) / 64);
    const int per_xcd = (ntile + kXcd - 1) / kXcd;
    const dim3 dgrid((unsigned)(per_xcd * kXcd));
    const R* U = fused ? (const R*)(single ? op->U32 : op->U64) : nullptr;
    const R kapR = (R)op->kappa;
    const R tsg = op->antiperiodic ? R(-1) : R(1);
    const double pass_bytes = (48.0 + 72.0) * sizeof(R) * (double)op->vol;
    const int tcls = single ? TC_WILSON_F32 : TC_WILSON_F64;
    // links in SU(3) and a single-precision pass: the fused kernels read rows
    // 0 and 1 of each link and rebuild row 2 (kRec is false for FP64, which
    // always reads the whole link)
    const bool rec = single && op->su3;
    constexpr bool kRec = sizeof(R) == 4;
    R* tmpv = (R*)w.tmp;
    int gf = g;  // partials of ||f||^2 left by the previous step

    for (int i = 1; i <= m; ++i) {
        R* vi = V + (int64_t)(i - 1) * ldv2;
        R* vprev = i > 1 ? V + (int64_t)(i - 2) * ldv2 : vi;
        R* vnext = V + (int64_t)i * ldv2;
        if (fused && i == 1) {
            // D pass, D^H pass with the partials of Re(v_1^H f), then k_lz_f applies alpha_1
            SC_TRY(wilson_pass(op, single, 0, vi, ldv, tmpv, op->n, 1, s));
            {
                TimerScope ts_(tcls, s, pass_bytes + 48.0 * sizeof(R) * op->vol, 1368.0 * op->vol);
#define SC_LZ_DHALPHA(REC_)                                                                               \
    SC_TLAUNCH((k_lz_dhalpha<R, REC_>), dgrid, blk, 0, s, f, (const R*)tmpv, (const R*)vi, (const R*)vprev, U, \
               geo, kapR, tsg, ntile, per_xcd, beta, i, w.st, w.part_a)
                if (rec) SC_LZ_DHALPHA(kRec);
                else SC_LZ_DHALPHA(false);
#undef SC_LZ_DHALPHA
                SC_LAUNCH_CHECK();
            }
            hipLaunchKernelGGL((k_lz_f<R, VEC>), dim3(g), blk, 0, s, f, vi, N2, alpha, beta, w.delta, i, w.st,
                               w.part_a, ntile, w.part_f, indef);
            SC_LAUNCH_CHECK();
            gf = g;
        } else if (fused) {
            // D pass with step 9 of step i - 1 and the partials of alpha_i, then the
            // D^H pass with step 5 (alpha_i, the pivot, the final f, its norm partials)
            {
                TimerScope ts_(tcls, s, pass_bytes + 48.0 * sizeof(R) * op->vol, 1368.0 * op->vol);
#define SC_LZ_DNEXT(REC_)                                                                                    \
    SC_TLAUNCH((k_lz_dnext<R, R, REC_>), dgrid, blk, 0, s, tmpv, (const R*)f, vi, (const R*)vprev, U, geo, kapR, \
               tsg, ntile, per_xcd, beta, i - 1, w.st, w.part_f, gf, w.part_a)
                if (rec) SC_LZ_DNEXT(kRec);
                else SC_LZ_DNEXT(false);
#undef SC_LZ_DNEXT
                SC_LAUNCH_CHECK();
            }
            {
                TimerScope ts_(tcls, s, pass_bytes + 48.0 * sizeof(R) * op->vol, 1416.0 * op->vol);
#define SC_LZ_DHF(REC_)                                                                                      \
    SC_TLAUNCH((k_lz_dhf<R, REC_>), dgrid, blk, 0, s, f, (const R*)tmpv, (const R*)vi, (const R*)vprev, U, geo, \
               kapR, tsg, ntile, per_xcd, alpha, beta, w.delta, i, w.st, w.part_a, w.part_f, indef)
                if (rec) SC_LZ_DHF(kRec);
                else SC_LZ_DHF(false);
#undef SC_LZ_DHF
                SC_LAUNCH_CHECK();
            }
            gf = ntile;
        } else {
            // step 5: f = A v_i - beta_{i-1} v_{i-1}; alpha_i; f -= alpha_i v_i
            SC_TRY(op_apply(op, single, vi, ldv, av, op->n, 1, w.tmp, s));
            hipLaunchKernelGGL((k_lz_alpha<R, VEC>), dim3(g), blk, 0, s, f, av, vi, vprev, N2, beta, i, w.st,
                               w.part_a);
            SC_LAUNCH_CHECK();
            hipLaunchKernelGGL((k_lz_f<R, VEC>), dim3(g), blk, 0, s, f, vi, N2, alpha, beta, w.delta, i, w.st,
                               w.part_a, g, w.part_f, indef);
            SC_LAUNCH_CHECK();
            gf = g;
        }
        if (freq > 0 && i >= 2 && i % freq == 0) {
            // step 8: [v_i, f] -= V_{i-1} (V_{i-1}^H [v_i, f]); v_i /= ||v_i||; f -= v_i (v_i^H f)
            ColPtrs<const void> wc{};
            wc.p[0] = vi;
            wc.p[1] = f;
            ColPtrs<void> xc{};
            xc.p[0] = vi;
            xc.p[1] = f;
            SC_TRY(gemm_cn(cpl, single, V, ldv, op->n, i - 1, single, wc, 2, w.G, w.gpart, halt, s));
            SC_TRY(gemm_nn(cpl, single, V, ldv, op->n, i - 1, w.G, 2, single, xc, -1.0, halt, s));
            hipLaunchKernelGGL((k_norm_part<R, VEC>), dim3(g), blk, 0, s, vi, N2, w.part_v, halt);
            SC_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_scale_norm<R>, dim3(g), blk, 0, s, vi, N2, w.part_v, g, halt);
            SC_LAUNCH_CHECK();
            ColPtrs<const void> fc{};
            fc.p[0] = f;
            ColPtrs<void> fo{};
            fo.p[0] = f;
            SC_TRY(gemm_cn(cpl, single, vi, ldv, op->n, 1, single, fc, 1, w.G2, w.gpart, halt, s));
            SC_TRY(gemm_nn(cpl, single, vi, ldv, op->n, 1, w.G2, 1, single, fo, -1.0, halt, s));
            hipLaunchKernelGGL((k_norm_part<R, VEC>), dim3(g), blk, 0, s, f, N2, w.part_f, halt);
            SC_LAUNCH_CHECK();
            gf = g;
        }
        // step 9: beta_i = ||f||, v_{i+1} = f / beta_i (the fused form does it in the next D pass)
        if (!fused || i == m) {
            hipLaunchKernelGGL((k_lz_next<R, R, VEC>), dim3(g), blk, 0, s, vnext, f, N2, beta, i, w.st, w.part_f,
                               gf);
            SC_LAUNCH_CHECK();
        }
    }
    return SC_OK;
}

// beta_0 e_1 as rows x es doubles
__global__ void k_e1(double* y, int rows, int es, const double* beta0) {
    for (int e = threadIdx.x; e < rows * es; e += blockDim.x) y[e] = e == 0 ? *beta0 : 0.0;
}

// Reads the phase's final state (one synchronisation) and forms x^1.
template <typename R>
static sc_status seed_finalize(const sc_op* op, void* x1, R* V, int64_t ldv, double* alpha, double* beta,
                               int* m_done, const SeedWork& w, hipStream_t s, sc_status* result, bool form_x1) {
    const bool single = sizeof(R) == 4;
    const bool cpl = is_complex(op->dtype);
    SeedState hst;
    SC_HIP(hipMemcpyAsync(&hst, w.st, sizeof(SeedState), hipMemcpyDeviceToHost, s));
    SC_HIP(hipStreamSynchronize(s));
    *m_done = hst.m_done;
    *result = (sc_status)hst.status;
    // x^1 = x0 + V_md T_md^{-1} (beta_0 e_1); for an indefinite op the minimum
    // residual x0 + V_md y, y = argmin || beta_0 e_1 - T~_md y || (QR of T~)
    if (form_x1 && hst.m_done >= 1 && hst.status != SC_ERR_NONFINITE) {
        if (op->kind == SC_OPK_WILSON_G5) {
            hipLaunchKernelGGL(k_e1, dim3(1), dim3(kBlock), 0, s, w.y, hst.m_done + 1, cpl ? 2 : 1, beta);
            SC_LAUNCH_CHECK();
            SC_TRY(tridiag_lsq(alpha, beta, hst.m_done, w.y, 1, cpl, w.trid, s));
        } else {
            SC_TRY(tridiag_solve(alpha, beta, hst.m_done, w.y, 1, cpl, beta, w.trid, nullptr, s));
        }
        ColPtrs<void> xc{};
        xc.p[0] = x1;
        SC_TRY(gemm_nn(cpl, single, V, ldv, op->n, hst.m_done, w.y, 1, false, xc, 1.0, nullptr, s));
    }
    return SC_OK;
}

sc_status seed_enqueue_any(const sc_op* op, const void* b1, void* x1, int m, int freq, void* V, int64_t ldv,
                           sc_dtype vdt, double* alpha, double* beta, const SeedWork& w, hipStream_t s,
                           bool indef) {
    const bool single = is_single(vdt);
    // 16-byte packs need 16-byte aligned columns
    const int64_t N2 = op->n * (is_complex(op->dtype) ? 2 : 1);
    const size_t rb = single ? 4 : 8;
    const bool vec = ((uintptr_t)V % 16 == 0) && ((ldv * (is_complex(vdt) ? 2 : 1) * rb) % 16 == 0) &&
                     ((N2 * rb) % 16 == 0);
    if (single) {
        if (vec) return seed_enqueue<float, true>(op, b1, x1, m, freq, (float*)V, ldv, alpha, beta, w, s, indef);
        return seed_enqueue<float, false>(op, b1, x1, m, freq, (float*)V, ldv, alpha, beta, w, s, indef);
    }
    if (vec) return seed_enqueue<double, true>(op, b1, x1, m, freq, (double*)V, ldv, alpha, beta, w, s, indef);
    return seed_enqueue<double, false>(op, b1, x1, m, freq, (double*)V, ldv, alpha, beta, w, s, indef);
}

sc_status seed_finalize_any(const sc_op* op, void* x1, void* V, int64_t ldv, sc_dtype vdt, double* alpha,
                            double* beta, int* m_done, const SeedWork& w, hipStream_t s, sc_status* result,
                            bool form_x1) {
    if (is_single(vdt))
        return seed_finalize<float>(op, x1, (float*)V, ldv, alpha, beta, m_done, w, s, result, form_x1);
    return seed_finalize<double>(op, x1, (double*)V, ldv, alpha, beta, m_done, w, s, result, form_x1);
}

SeedWork seed_carve(void* work, size_t work_bytes, const sc_op* op, int m, bool single, bool* ok) {
    Carver c(work, work_bytes);
    SeedWork w = carve_seed(c, op, m, single);
    *ok = c.ok();
    return w;
}

// Warm the stencil autotuner for the seed phase's shape (one column at the
// basis precision) outside any graph capture.
sc_status seed_pretune(const sc_op* op, bool single, const SeedWork& w, hipStream_t s) {
    return op_apply(op, single, w.f, op->n, w.av, op->n, 1, w.tmp, s);
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
    SC_TRY(seed_enqueue_any(op, b1, x1, m, freq, V, ldv, vdt, alpha, beta, w, s));
    if (single) SC_TRY(seed_finalize<float>(op, x1, (float*)V, ldv, alpha, beta, m_done, w, s, &result, true));
    else SC_TRY(seed_finalize<double>(op, x1, (double*)V, ldv, alpha, beta, m_done, w, s, &result, true));
    if (result == SC_ERR_NOT_PD) set_error("seed_lanczos: non-positive pivot, A is not positive definite");
    if (result == SC_ERR_NONFINITE) set_error("seed_lanczos: non-finite value in the Lanczos recurrence");
    return result;
}

}  // namespace sc
