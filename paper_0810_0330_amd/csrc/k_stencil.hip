// Operator applies: the 2D Laplacian, the diagonal matrix, and the Wilson-Dirac
// stencil D = 1 - kappa H, its adjoint, and the hopping term alone.
//
// The Wilson hopping term sums, over the four directions mu, a forward hop
// (1 - gamma_mu) U_mu(x) psi(x+mu) and a backward hop
// (1 + gamma_mu) U_mu(x-mu)^H psi(x-mu); the adjoint D^H swaps the two spin
// projectors.  In the chiral basis gamma_mu = [[0, A_mu], [A_mu^H, 0]] with
// A_k = -i sigma_k (k = x, y, z) and A_t = 1, so (1 + s gamma_mu) psi, s = +-1,
// is fixed by its upper half h = psi_up + s A_mu psi_down: the lower half is
// s A_mu^H h.  Each hop therefore projects the neighbour to a two-spin half
// spinor, multiplies the two colour vectors by the link, and reconstructs:
// 2 x (3x3 complex matrix-vector) per hop instead of 4.
#include "sc_internal.h"
#include "sc_timer.h"

namespace sc {

// ---------------------------------------------------------------- Laplacian
template <typename R>
__global__ __launch_bounds__(kBlock) void k_laplace2d(R* __restrict__ y, int64_t ldy, const R* __restrict__ x,
                                                      int64_t ldx, int nx, int ny) {
    const int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    const int64_t n = (int64_t)nx * ny;
    if (idx >= n) return;
    const R* xc = x + blockIdx.y * ldx;
    const int i = (int)(idx % nx);
    const int j = (int)(idx / nx);
    R v = R(4) * xc[idx];
    if (j > 0) v -= xc[idx - nx];
    if (j < ny - 1) v -= xc[idx + nx];
    if (i > 0) v -= xc[idx - 1];
    if (i < nx - 1) v -= xc[idx + 1];
    y[blockIdx.y * ldy + idx] = v;
}

// ---------------------------------------------------------------- diagonal
template <typename R>
__global__ __launch_bounds__(kBlock) void k_diag(R* __restrict__ y, int64_t ldy, const R* __restrict__ x,
                                                 int64_t ldx, const double* __restrict__ d, int64_t n) {
    const int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (idx >= n) return;
    y[blockIdx.y * ldy + idx] = R(d[idx]) * x[blockIdx.y * ldx + idx];
}

// ---------------------------------------------------------------- Wilson
struct Geom {
    int X, Y, Z, T;
    int64_t V;
};

template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }

// a + S*b
template <int S, typename R>
__device__ __forceinline__ cplx<R> adds(cplx<R> a, cplx<R> b) {
    if constexpr (S > 0) return {a.re + b.re, a.im + b.im};
    else return {a.re - b.re, a.im - b.im};
}
// a + S*i*b
template <int S, typename R>
__device__ __forceinline__ cplx<R> addis(cplx<R> a, cplx<R> b) {
    if constexpr (S > 0) return {a.re - b.im, a.im + b.re};
    else return {a.re + b.im, a.im - b.re};
}

// chi = U h (DAGU = false) or U^H h (DAGU = true) for one colour vector
template <bool DAGU, typename R>
__device__ __forceinline__ void su3_mul(const cplx<R> u[3][3], const cplx<R> h[3], cplx<R> chi[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R re = 0, im = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const cplx<R> m = DAGU ? u[b][a] : u[a][b];
            if constexpr (DAGU) {  // conj(m) * h
                re += m.re * h[b].re + m.im * h[b].im;
                im += m.re * h[b].im - m.im * h[b].re;
            } else {
                re += m.re * h[b].re - m.im * h[b].im;
                im += m.re * h[b].im + m.im * h[b].re;
            }
        }
        chi[a] = {re, im};
    }
}

// acc += (1 + SIG gamma_MU) (U or U^H) psi * bf
template <int MU, int SIG, bool DAGU, typename R>
__device__ __forceinline__ void hop(cplx<R> acc[4][3], const cplx<R> psi[4][3], const cplx<R> u[3][3], R bf) {
    cplx<R> h0[3], h1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if constexpr (MU == 0) {         // A = -i sigma_x: A psi_dn = (-i psi3, -i psi2)
            h0[c] = addis<-SIG>(psi[0][c], psi[3][c]);
            h1[c] = addis<-SIG>(psi[1][c], psi[2][c]);
        } else if constexpr (MU == 1) {  // A = -i sigma_y: A psi_dn = (-psi3, psi2)
            h0[c] = adds<-SIG>(psi[0][c], psi[3][c]);
            h1[c] = adds<SIG>(psi[1][c], psi[2][c]);
        } else if constexpr (MU == 2) {  // A = -i sigma_z: A psi_dn = (-i psi2, i psi3)
            h0[c] = addis<-SIG>(psi[0][c], psi[2][c]);
            h1[c] = addis<SIG>(psi[1][c], psi[3][c]);
        } else {                         // A = 1
            h0[c] = adds<SIG>(psi[0][c], psi[2][c]);
            h1[c] = adds<SIG>(psi[1][c], psi[3][c]);
        }
    }
    cplx<R> c0[3], c1[3];
    su3_mul<DAGU>(u, h0, c0);
    su3_mul<DAGU>(u, h1, c1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        c0[c].re *= bf; c0[c].im *= bf;
        c1[c].re *= bf; c1[c].im *= bf;
        acc[0][c] = cadd(acc[0][c], c0[c]);
        acc[1][c] = cadd(acc[1][c], c1[c]);
        // lower half: SIG * A^H chi
        if constexpr (MU == 0) {         // A^H = i sigma_x: (i chi1, i chi0)
            acc[2][c] = addis<SIG>(acc[2][c], c1[c]);
            acc[3][c] = addis<SIG>(acc[3][c], c0[c]);
        } else if constexpr (MU == 1) {  // A^H = i sigma_y: (chi1, -chi0)
            acc[2][c] = adds<SIG>(acc[2][c], c1[c]);
            acc[3][c] = adds<-SIG>(acc[3][c], c0[c]);
        } else if constexpr (MU == 2) {  // A^H = i sigma_z: (i chi0, -i chi1)
            acc[2][c] = addis<SIG>(acc[2][c], c0[c]);
            acc[3][c] = addis<-SIG>(acc[3][c], c1[c]);
        } else {
            acc[2][c] = adds<SIG>(acc[2][c], c0[c]);
            acc[3][c] = adds<SIG>(acc[3][c], c1[c]);
        }
    }
}

template <typename R>
__device__ __forceinline__ void load_spinor(const R* __restrict__ f, int64_t V, int64_t site, cplx<R> psi[4][3]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) psi[s][c] = ld2(f, (int64_t)(s * 3 + c) * V + site);
}

template <typename R>
__device__ __forceinline__ void load_link(const R* __restrict__ U, int64_t V, int mu, int64_t site, cplx<R> u[3][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) u[a][b] = ld2(U, (int64_t)((mu * 3 + a) * 3 + b) * V + site);
}

// MODE 0: out = in - kappa * H in (D or D^H);  MODE 1: out = H in (or H^H in)
template <typename R, bool DAG, int MODE>
__global__ __launch_bounds__(kBlock) void k_wilson(R* __restrict__ out, int64_t ldo, const R* __restrict__ in,
                                                   int64_t ldi, const R* __restrict__ U, Geom g, R kappa,
                                                   R tsign) {
    const int64_t s = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (s >= g.V) return;
    const R* src = in + blockIdx.y * ldi;
    R* dst = out + blockIdx.y * ldo;
    const int64_t XY = (int64_t)g.X * g.Y, XYZ = XY * g.Z;
    const int x = (int)(s % g.X);
    const int y = (int)((s / g.X) % g.Y);
    const int z = (int)((s / XY) % g.Z);
    const int t = (int)(s / XYZ);
    const int64_t nb_p[4] = {x == g.X - 1 ? s - (g.X - 1) : s + 1,
                             y == g.Y - 1 ? s - (int64_t)(g.Y - 1) * g.X : s + g.X,
                             z == g.Z - 1 ? s - (int64_t)(g.Z - 1) * XY : s + XY,
                             t == g.T - 1 ? s - (int64_t)(g.T - 1) * XYZ : s + XYZ};
    const int64_t nb_m[4] = {x == 0 ? s + (g.X - 1) : s - 1,
                             y == 0 ? s + (int64_t)(g.Y - 1) * g.X : s - g.X,
                             z == 0 ? s + (int64_t)(g.Z - 1) * XY : s - XY,
                             t == 0 ? s + (int64_t)(g.T - 1) * XYZ : s - XYZ};
    const R bf_p = (t == g.T - 1) ? tsign : R(1);
    const R bf_m = (t == 0) ? tsign : R(1);
    constexpr int SF = DAG ? 1 : -1;  // projector sign of the forward hop
    constexpr int SB = -SF;

    cplx<R> acc[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[a][c] = {R(0), R(0)};

    cplx<R> psi[4][3], u[3][3];
#define SC_WILSON_DIR(MU)                                                   \
    load_spinor(src, g.V, nb_p[MU], psi);                                   \
    load_link(U, g.V, MU, s, u);                                            \
    hop<MU, SF, false>(acc, psi, u, MU == 3 ? bf_p : R(1));                 \
    load_spinor(src, g.V, nb_m[MU], psi);                                   \
    load_link(U, g.V, MU, nb_m[MU], u);                                     \
    hop<MU, SB, true>(acc, psi, u, MU == 3 ? bf_m : R(1));
    SC_WILSON_DIR(0)
    SC_WILSON_DIR(1)
    SC_WILSON_DIR(2)
    SC_WILSON_DIR(3)
#undef SC_WILSON_DIR

#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t idx = (int64_t)(a * 3 + c) * g.V + s;
            cplx<R> r = acc[a][c];
            if constexpr (MODE == 0) {
                const cplx<R> p = ld2(src, idx);
                r = {p.re - kappa * r.re, p.im - kappa * r.im};
            }
            st2(dst, idx, r);
        }
}

// ---------------------------------------------------------------- launchers
template <typename R>
static sc_status wilson_launch(const sc_op* op, int which, const R* X, int64_t ldx, R* Y, int64_t ldy, int k,
                               const R* U, hipStream_t s) {
    Geom g{op->dims[0], op->dims[1], op->dims[2], op->dims[3], op->vol};
    dim3 grid((unsigned)((g.V + kBlock - 1) / kBlock), (unsigned)k);
    const R kap = (R)op->kappa;
    const R ts = op->antiperiodic ? R(-1) : R(1);
    // algorithmic traffic of one pass: each spinor read and written once per
    // column, the 4 links of a site read once per pass; 1320 flops of hopping
    // per site and column (+48 for psi - kappa H psi)
    const double bytes = (48.0 * k + 72.0) * sizeof(R) * (double)g.V;
    const double flops = (which < 2 ? 1368.0 : 1320.0) * k * (double)g.V;
    TimerScope ts_(sizeof(R) == 4 ? TC_WILSON_F32 : TC_WILSON_F64, s, bytes, flops);
    // ld arguments are in reals (2 per complex element)
    switch (which) {
        case 0: hipLaunchKernelGGL((k_wilson<R, false, 0>), grid, dim3(kBlock), 0, s, Y, 2 * ldy, X, 2 * ldx, U, g, kap, ts); break;
        case 1: hipLaunchKernelGGL((k_wilson<R, true, 0>), grid, dim3(kBlock), 0, s, Y, 2 * ldy, X, 2 * ldx, U, g, kap, ts); break;
        case 2: hipLaunchKernelGGL((k_wilson<R, false, 1>), grid, dim3(kBlock), 0, s, Y, 2 * ldy, X, 2 * ldx, U, g, kap, ts); break;
        default: hipLaunchKernelGGL((k_wilson<R, true, 1>), grid, dim3(kBlock), 0, s, Y, 2 * ldy, X, 2 * ldx, U, g, kap, ts); break;
    }
    SC_LAUNCH_CHECK();
    return SC_OK;
}

sc_status wilson_pass(const sc_op* op, bool single, int which, const void* X, int64_t ldx, void* Y, int64_t ldy,
                      int k, hipStream_t s) {
    if (k <= 0) return SC_OK;
    if (single) {
        if (!op->U32) {
            set_error("single-precision Wilson apply needs U32 links");
            return SC_ERR_ARG;
        }
        return wilson_launch<float>(op, which, (const float*)X, ldx, (float*)Y, ldy, k, (const float*)op->U32, s);
    }
    return wilson_launch<double>(op, which, (const double*)X, ldx, (double*)Y, ldy, k, (const double*)op->U64, s);
}

int64_t op_apply_tmp_elems(const sc_op* op) { return op->kind == SC_OPK_WILSON ? op->n : 0; }

sc_status op_apply(const sc_op* op, bool single, const void* X, int64_t ldx, void* Y, int64_t ldy, int k, void* tmp,
                   hipStream_t s) {
    if (k <= 0) return SC_OK;
    if (op->kind == SC_OPK_WILSON) {
        SC_TRY(wilson_pass(op, single, 0, X, ldx, tmp, op->n, k, s));
        return wilson_pass(op, single, 1, tmp, op->n, Y, ldy, k, s);
    }
    dim3 grid((unsigned)((op->n + kBlock - 1) / kBlock), (unsigned)k);
    if (op->kind == SC_OPK_LAPLACE2D) {
        if (single)
            hipLaunchKernelGGL(k_laplace2d<float>, grid, dim3(kBlock), 0, s, (float*)Y, ldy, (const float*)X, ldx, op->nx, op->ny);
        else
            hipLaunchKernelGGL(k_laplace2d<double>, grid, dim3(kBlock), 0, s, (double*)Y, ldy, (const double*)X, ldx, op->nx, op->ny);
    } else {
        if (single)
            hipLaunchKernelGGL(k_diag<float>, grid, dim3(kBlock), 0, s, (float*)Y, ldy, (const float*)X, ldx, op->d, op->n);
        else
            hipLaunchKernelGGL(k_diag<double>, grid, dim3(kBlock), 0, s, (double*)Y, ldy, (const double*)X, ldx, op->d, op->n);
    }
    SC_LAUNCH_CHECK();
    return SC_OK;
}

}  // namespace sc
