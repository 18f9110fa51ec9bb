// Device building blocks of the Wilson stencil, shared by the operator
// kernels and the fused Lanczos kernels of the seed phase.
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
#pragma once

#include "sc_common.h"

namespace sc {

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

template <typename R>
__device__ __forceinline__ R fmar(R a, R b, R c) {
    if constexpr (sizeof(R) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

// chi = U h (DAGU = false) or U^H h (DAGU = true) for one colour vector; four
// fused multiply-adds per complex product
template <bool DAGU, typename R>
__device__ __forceinline__ void su3_mul(const cplx<R> u[3][3], const cplx<R> h[3], cplx<R> chi[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R re, im;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const cplx<R> m = DAGU ? u[b][a] : u[a][b];
            const R mi = DAGU ? -m.im : m.im;  // conj(m) for U^H
            if (b == 0) {
                re = m.re * h[b].re;
                im = m.re * h[b].im;
            } else {
                re = fmar(m.re, h[b].re, re);
                im = fmar(m.re, h[b].im, im);
            }
            re = fmar(-mi, h[b].im, re);
            im = fmar(mi, h[b].re, im);
        }
        chi[a] = {re, im};
    }
}

// The two colour vectors of the half spinor h = psi_up + SIG A_mu psi_down.
template <int MU, int SIG, typename R>
__device__ __forceinline__ void project(const cplx<R> psi[4][3], cplx<R> h0[3], cplx<R> h1[3]) {
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
}

// One hop, acc += (1 + SIG gamma_MU) (U or U^H) psi (times bf for the time
// direction), in two halves: hop_half projects psi to the two colour vectors
// of the half spinor and multiplies them by the link; hop_acc rebuilds the
// four spin components from them and adds them to acc.
template <int MU, int SIG, bool DAGU, typename R>
__device__ __forceinline__ void hop_half(const cplx<R> psi[4][3], const cplx<R> u[3][3], R bf, cplx<R> c0[3],
                                         cplx<R> c1[3]) {
    cplx<R> h0[3], h1[3];
    project<MU, SIG>(psi, h0, h1);
    if constexpr (MU == 3) {  // (anti)periodic boundary factor of the time hops
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            h0[c].re *= bf; h0[c].im *= bf;
            h1[c].re *= bf; h1[c].im *= bf;
        }
    }
    su3_mul<DAGU>(u, h0, c0);
    su3_mul<DAGU>(u, h1, c1);
}

template <int MU, int SIG, typename R>
__device__ __forceinline__ void hop_acc(cplx<R> acc[4][3], const cplx<R> c0[3], const cplx<R> c1[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
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

template <int MU, int SIG, bool DAGU, typename R>
__device__ __forceinline__ void hop(cplx<R> acc[4][3], const cplx<R> psi[4][3], const cplx<R> u[3][3], R bf) {
    cplx<R> c0[3], c1[3];
    hop_half<MU, SIG, DAGU>(psi, u, bf, c0, c1);
    hop_acc<MU, SIG>(acc, c0, c1);
}

// Loads with a wave-uniform base (scalar registers) plus one unsigned 32-bit
// lane offset: the 12 components of a spinor and the 9 entries of a link are
// V elements apart, so every load of a site shares one offset register.
template <typename R>
__device__ __forceinline__ cplx<R> ldc(const R* __restrict__ base, unsigned site) {
    const typename vec2<R>::type v = reinterpret_cast<const typename vec2<R>::type*>(base)[site];
    return {v.x, v.y};
}

template <typename R>
__device__ __forceinline__ void load_spinor(const R* __restrict__ f, unsigned V, unsigned site, cplx<R> psi[4][3]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) psi[s][c] = ldc(f + 2 * (size_t)((s * 3 + c) * V), site);
}

// Row 2 of a matrix of SU(3) from rows 0 and 1: for a unitary matrix of
// determinant 1 it is the complex conjugate of their cross product.
template <typename R>
__device__ __forceinline__ void su3_row2(cplx<R> u[3][3]) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
        const cplx<R> p = u[0][b1], q = u[1][b2], r = u[0][b2], w = u[1][b1];
        const R re = (p.re * q.re - p.im * q.im) - (r.re * w.re - r.im * w.im);
        const R im = (p.re * q.im + p.im * q.re) - (r.re * w.im + r.im * w.re);
        u[2][b] = {re, -im};
    }
}

// The link U_mu(site).  REC (links known to be in SU(3)): rows 0 and 1 are
// read and row 2 is rebuilt from them, 12 of the 18 reals of the link.
template <typename R, bool REC = false>
__device__ __forceinline__ void load_link(const R* __restrict__ U, unsigned V, int mu, unsigned site, cplx<R> u[3][3]) {
#pragma unroll
    for (int a = 0; a < (REC ? 2 : 3); ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) u[a][b] = ldc(U + 2 * (size_t)(((mu * 3 + a) * 3 + b) * V), site);
    if constexpr (REC) su3_row2(u);
}


// Neighbours of site s in direction mu (forward np, backward nm) and the
// boundary factors of the two hops (tsign at the time boundary).
template <typename R>
__device__ __forceinline__ void neighbours(const Geom& g, int s, int mu, R tsign, int& np, int& nm, R& bfp, R& bfm) {
    const int XY = g.X * g.Y, XYZ = XY * g.Z;
    bfp = R(1);
    bfm = R(1);
    switch (mu) {
        case 0: {
            const int x = s % g.X;
            np = x == g.X - 1 ? s - (g.X - 1) : s + 1;
            nm = x == 0 ? s + (g.X - 1) : s - 1;
            break;
        }
        case 1: {
            const int y = (s / g.X) % g.Y;
            np = y == g.Y - 1 ? s - (g.Y - 1) * g.X : s + g.X;
            nm = y == 0 ? s + (g.Y - 1) * g.X : s - g.X;
            break;
        }
        case 2: {
            const int z = (s / XY) % g.Z;
            np = z == g.Z - 1 ? s - (g.Z - 1) * XY : s + XY;
            nm = z == 0 ? s + (g.Z - 1) * XY : s - XY;
            break;
        }
        default: {
            const int t = s / XYZ;
            np = t == g.T - 1 ? s - (g.T - 1) * XYZ : s + XYZ;
            nm = t == 0 ? s + (g.T - 1) * XYZ : s - XYZ;
            bfp = t == g.T - 1 ? tsign : R(1);
            bfm = t == 0 ? tsign : R(1);
            break;
        }
    }
}

// The value held by the lane one x-step up (x + 1) or down (x - 1) in this
// lane's row of 16 lanes, by DPP row rotation: for row_ror:n lane i reads lane
// (i - n) mod 16, so row_ror:15 gives x + 1 and row_ror:1 gives x - 1, wrapping
// exactly as the periodic x boundary does when a row holds one x-row of a
// lattice with X = 16.  FP64 values move as two 32-bit halves.
__device__ __forceinline__ float dpp_from_xp(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x12F, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_from_xm(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x121, 0xF, 0xF, false));
}
__device__ __forceinline__ double dpp_from_xp(double v) {
    int2 b = __builtin_bit_cast(int2, v);
    b.x = __builtin_amdgcn_update_dpp(0, b.x, 0x12F, 0xF, 0xF, false);
    b.y = __builtin_amdgcn_update_dpp(0, b.y, 0x12F, 0xF, 0xF, false);
    return __builtin_bit_cast(double, b);
}
__device__ __forceinline__ double dpp_from_xm(double v) {
    int2 b = __builtin_bit_cast(int2, v);
    b.x = __builtin_amdgcn_update_dpp(0, b.x, 0x121, 0xF, 0xF, false);
    b.y = __builtin_amdgcn_update_dpp(0, b.y, 0x121, 0xF, 0xF, false);
    return __builtin_bit_cast(double, b);
}

// The two x hops of site s when the wave's lanes hold whole x-rows of a
// lattice with X = 16 (lane l = site s mod 64, x = l mod 16): the lane loads
// only its own spinor and link, projects its spinor for both hops and forms
// U_x(s)^H P psi(s) itself; the forward hop takes the projection of lane x + 1
// and the backward hop the product of lane x - 1 through DPP.  Each quantity
// is the one the loading form computes from the neighbour's data, so the
// result is the same.
template <bool DAG, typename R, bool REC = false>
__device__ __forceinline__ void dir_hops_x16(cplx<R> acc[4][3], const R* __restrict__ src, const R* __restrict__ U,
                                             unsigned uV, int s) {
    constexpr int SF = DAG ? 1 : -1;
    constexpr int SB = -SF;
    cplx<R> u[3][3], psi[4][3];
    load_link<R, REC>(U, uV, 0, (unsigned)s, u);
    load_spinor(src, uV, (unsigned)s, psi);
    cplx<R> h0[3], h1[3], g0[3], g1[3], c0[3], c1[3];
    project<0, SF>(psi, h0, h1);  // what lane x - 1 needs for its forward hop
    project<0, SB>(psi, g0, g1);
    su3_mul<true>(u, g0, c0);     // what lane x + 1 needs for its backward hop
    su3_mul<true>(u, g1, c1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h0[c] = {dpp_from_xp(h0[c].re), dpp_from_xp(h0[c].im)};
        h1[c] = {dpp_from_xp(h1[c].re), dpp_from_xp(h1[c].im)};
        c0[c] = {dpp_from_xm(c0[c].re), dpp_from_xm(c0[c].im)};
        c1[c] = {dpp_from_xm(c1[c].re), dpp_from_xm(c1[c].im)};
    }
    hop_acc<0, SB>(acc, c0, c1);  // backward hop, from x - 1
    su3_mul<false>(u, h0, c0);
    su3_mul<false>(u, h1, c1);
    hop_acc<0, SF>(acc, c0, c1);  // forward hop, from x + 1
}

// acc += the forward and backward hops of direction mu at site s (one
// direction of the hopping term; mu wave-uniform)
template <bool DAG, typename R, bool REC = false>
__device__ __forceinline__ void dir_hops(cplx<R> acc[4][3], const R* __restrict__ src, const R* __restrict__ U,
                                         const Geom& g, unsigned uV, int s, int mu, R tsign) {
    constexpr int SF = DAG ? 1 : -1;
    constexpr int SB = -SF;
    int np, nm;
    R bfp, bfm;
    neighbours<R>(g, s, mu, tsign, np, nm, bfp, bfm);
    cplx<R> u[3][3], psi[4][3];
    load_link<R, REC>(U, uV, mu, (unsigned)s, u);
    load_spinor(src, uV, (unsigned)np, psi);
    switch (mu) {
        case 0: hop<0, SF, false>(acc, psi, u, bfp); break;
        case 1: hop<1, SF, false>(acc, psi, u, bfp); break;
        case 2: hop<2, SF, false>(acc, psi, u, bfp); break;
        default: hop<3, SF, false>(acc, psi, u, bfp); break;
    }
    load_link<R, REC>(U, uV, mu, (unsigned)nm, u);
    load_spinor(src, uV, (unsigned)nm, psi);
    switch (mu) {
        case 0: hop<0, SB, true>(acc, psi, u, bfm); break;
        case 1: hop<1, SB, true>(acc, psi, u, bfm); break;
        case 2: hop<2, SB, true>(acc, psi, u, bfm); break;
        default: hop<3, SB, true>(acc, psi, u, bfm); break;
    }
}

}  // namespace sc
