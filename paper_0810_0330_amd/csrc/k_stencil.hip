// Operator applies: the 2D Laplacian, the diagonal matrix, and the Wilson-Dirac
// stencil D = 1 - kappa H, its adjoint, and the hopping term alone, in several
// launch shapes chosen by an autotuner.  The hop arithmetic is in wilson_dev.h.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>

#include "sc_internal.h"
#include "sc_timer.h"
#include "wilson_dev.h"

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

// Block -> work mapping.  Workgroups are dispatched round-robin over the 8
// XCDs (block b runs on XCD b % 8), each with its own 4 MB L2.  Logical work
// item L = (b % 8) * per_xcd + b / 8 gives every XCD a contiguous range of L.
// L enumerates (site tile, column group) pairs chunk by chunk: a chunk holds G
// consecutive column groups, and within a chunk the G groups of one tile are
// consecutive in L.  G = all groups: a tile's links are reused from L2 by every
// column, but the t-neighbour tiles of all k columns must stay cached too;
// G = 1: one column group sweeps the lattice before the next, so its
// neighbour slices stay in L2 while the links are re-read once per group.
// Intermediate G trades the two.
//
// Tile order: zb = 1 takes tiles in site order, so a tile's t-neighbours are
// XYZ / 256 tiles away.  zb > 1 (when the tiles of a time slice split into
// blocks of zb) walks zb tiles along z, then the next time slice, and so on
// through all of t before the next block of z: the t-neighbours are then zb
// tiles away and the z-neighbours one, except across block edges.

__device__ __forceinline__ bool map_work(int ntiles, int ncg, int G, int per_xcd, int zb, int T, int& tile,
                                         int& cg) {
    const int b = blockIdx.x;
    const int L = (b % kXcd) * per_xcd + b / kXcd;
    if (L >= ntiles * ncg) return false;
    const int nfull = ncg / G;
    const int span = ntiles * G;
    const int c = L / span;
    if (c < nfull) {
        const int r = L - c * span;
        tile = r / G;
        cg = c * G + r % G;
    } else {  // last, partial chunk
        const int gl = ncg - nfull * G;
        const int r = L - nfull * span;
        tile = r / gl;
        cg = nfull * G + r % gl;
    }
    if (zb > 1) {  // tiles per time slice = ntiles / T, a multiple of zb (checked by the host)
        const int per_slab = T * zb;
        const int zblk = tile / per_slab, r = tile - zblk * per_slab;
        tile = (r / zb) * (ntiles / T) + zblk * zb + r % zb;
    }
    return true;
}

// Epilogues of the fused CG passes (the t-march and tiled forms; the partial
// sums of a block are left per column in e.part, see the kernels):
//   TM_NORM: out is written and the partials are of |out|^2 (for A = D^H D,
//     <p, A p> = ||D p||^2, so CG needs no separate reduction over p and A p);
//   TM_CG: out (= A p of a CG iteration) is not stored; for the columns active
//     in e.st, r -= alpha out with alpha = rho / (sum of e.pq's partials), and
//     the partials are of |r|^2.
enum { TM_PLAIN = 0, TM_NORM = 1, TM_CG = 2 };

struct TmEpi {
    double* part;
    const CGCol* st;
    const double* pq;
    void* r;
    int64_t ldr;  // reals
};

}  // namespace sc

#include "wilson_tx.h"

namespace sc {


// One output element of a tiled pass under epilogue EPI (see above): stored to
// out, or (TM_CG) applied to r in place, with its |.|^2 added to nacc.
template <typename R, int EPI>
__device__ __forceinline__ void epi_store(R* dst, R* rv, size_t cb, unsigned us, cplx<R> r, R alpha, double& nacc) {
    using V2 = typename vec2<R>::type;
    if constexpr (EPI == TM_CG) {
        V2 rr = reinterpret_cast<V2*>(rv + cb)[us];
        rr.x = rr.x - alpha * r.re;
        rr.y = rr.y - alpha * r.im;
        reinterpret_cast<V2*>(rv + cb)[us] = rr;
        nacc += (double)rr.x * (double)rr.x + (double)rr.y * (double)rr.y;
    } else {
        reinterpret_cast<V2*>(dst + cb)[us] = V2{r.re, r.im};
        if constexpr (EPI == TM_NORM) nacc += (double)r.re * (double)r.re + (double)r.im * (double)r.im;
    }
}

// alpha = rho / (sum of the TM_NORM partials) per column for TM_CG (block-uniform;
// the same sum, in the same order, as the CG kernel that follows), and which
// columns the pass updates
template <typename R, int EPI, int NC>
__device__ __forceinline__ void epi_setup(const TmEpi& e, const bool live[NC], int c0, int ntiles, double* sh,
                                          R alpha[NC], bool upd[NC], double nacc[NC]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        nacc[c] = 0.0;
        upd[c] = live[c];
        alpha[c] = R(0);
    }
    if constexpr (EPI == TM_CG) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int col = live[c] ? c0 + c : c0;
            const double pq = sum_partials(e.pq + (int64_t)col * ntiles, ntiles, sh);
            upd[c] = live[c] && e.st[col].active;
            alpha[c] = upd[c] ? (R)(e.st[col].rho / pq) : R(0);
        }
    }
}

// The block's partial of each live column at index column * ntiles + tile of e.part
template <int EPI, int NC>
__device__ __forceinline__ void epi_finish(const TmEpi& e, const bool live[NC], int c0, int ntiles, int tile,
                                           double* sh, const double nacc[NC]) {
    if constexpr (EPI != TM_PLAIN) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double tot = block_sum(nacc[c], sh);
            if (threadIdx.x == 0 && live[c]) e.part[(int64_t)(c0 + c) * ntiles + tile] = tot;
        }
    }
}

// MODE 0: out = in - kappa * H in (D or D^H);  MODE 1: out = H in (or H^H in).
// NC columns per thread: each link is loaded once and applied to NC spinors.
// With an epilogue (EPI != TM_PLAIN) every lane of a block stays for the block
// sums: a lane past the last site works on the last site and stores nothing.
template <typename R, bool DAG, int MODE, int NC, int MINW, bool BAR = false, int EPI = TM_PLAIN>
__global__ __launch_bounds__(kBlock, MINW) void k_wilson(R* __restrict__ out, int64_t ldo, const R* __restrict__ in,
                                                   int64_t ldi, const R* __restrict__ U, Geom g, R kappa, R tsign,
                                                   int k, int ncg, int ntiles, int per_xcd, int G, int zb, TmEpi e) {
    int tile, cgi;
    if (!map_work(ntiles, ncg, G, per_xcd, zb, g.T, tile, cgi)) return;
    const int c0 = cgi * NC;
    int s = tile * kBlock + threadIdx.x;
    const int V = (int)g.V;
    bool ok = true;
    if constexpr (EPI == TM_PLAIN) {
        if (s >= V) return;
    } else {
        ok = s < V;
        if (!ok) s = V - 1;
    }
    const int XY = g.X * g.Y, XYZ = XY * g.Z;
    const int x = s % g.X;
    const int y = (s / g.X) % g.Y;
    const int z = (s / XY) % g.Z;
    const int t = s / XYZ;
    const unsigned nb_p[4] = {(unsigned)(x == g.X - 1 ? s - (g.X - 1) : s + 1),
                              (unsigned)(y == g.Y - 1 ? s - (g.Y - 1) * g.X : s + g.X),
                              (unsigned)(z == g.Z - 1 ? s - (g.Z - 1) * XY : s + XY),
                              (unsigned)(t == g.T - 1 ? s - (g.T - 1) * XYZ : s + XYZ)};
    const unsigned nb_m[4] = {(unsigned)(x == 0 ? s + (g.X - 1) : s - 1),
                              (unsigned)(y == 0 ? s + (g.Y - 1) * g.X : s - g.X),
                              (unsigned)(z == 0 ? s + (g.Z - 1) * XY : s - XY),
                              (unsigned)(t == 0 ? s + (g.T - 1) * XYZ : s - XYZ)};
    const unsigned us = (unsigned)s, uV = (unsigned)V;
    const R bf_p = (t == g.T - 1) ? tsign : R(1);
    const R bf_m = (t == 0) ? tsign : R(1);
    constexpr int SF = DAG ? 1 : -1;  // projector sign of the forward hop
    constexpr int SB = -SF;

    const R* src[NC];
    bool live[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        live[c] = c0 + c < k;
        src[c] = in + (int64_t)(live[c] ? c0 + c : c0) * ldi;
    }
    [[maybe_unused]] double* esh = nullptr;
    R alpha[NC];
    bool upd[NC];
    double nacc[NC];
    if constexpr (EPI != TM_PLAIN) {
        __shared__ double esh_[kWaves];
        esh = esh_;
        epi_setup<R, EPI, NC>(e, live, c0, ntiles, esh, alpha, upd, nacc);
    }

    cplx<R> acc[NC][4][3];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) acc[c][a][cc] = {R(0), R(0)};

    cplx<R> psi[4][3], u[3][3];
    // The empty asm statements are compiler barriers: they keep the loads of
    // one hop from being hoisted above the previous hop, which bounds the
    // live registers to one hop's operands (several waves per SIMD then hide
    // the latency instead of one wave with every load in flight).
#define SC_WILSON_DIR(MU)                                                    \
    load_link(U, uV, MU, us, u);                                             \
    _Pragma("unroll") for (int c = 0; c < NC; ++c) {                         \
        load_spinor(src[c], uV, nb_p[MU], psi);                              \
        hop<MU, SF, false>(acc[c], psi, u, bf_p);                            \
        if (BAR) asm volatile("" ::: "memory");                              \
    }                                                                        \
    load_link(U, uV, MU, nb_m[MU], u);                                       \
    _Pragma("unroll") for (int c = 0; c < NC; ++c) {                         \
        load_spinor(src[c], uV, nb_m[MU], psi);                              \
        hop<MU, SB, true>(acc[c], psi, u, bf_m);                             \
        if (BAR) asm volatile("" ::: "memory");                              \
    }
    SC_WILSON_DIR(0)
    SC_WILSON_DIR(1)
    SC_WILSON_DIR(2)
    SC_WILSON_DIR(3)
#undef SC_WILSON_DIR

#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if constexpr (EPI == TM_PLAIN) {
            if (!live[c]) continue;
        } else {
            if (!ok || !upd[c]) continue;
        }
        R* dst = out + (int64_t)(c0 + c) * ldo;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                const size_t cb = 2 * (size_t)((a * 3 + cc) * uV);
                cplx<R> r = acc[c][a][cc];
                if constexpr (MODE == 0) {
                    const cplx<R> p = ldc(src[c] + cb, us);
                    r = {p.re - kappa * r.re, p.im - kappa * r.im};
                }
                if constexpr (EPI == TM_PLAIN)
                    reinterpret_cast<typename vec2<R>::type*>(dst + cb)[us] = typename vec2<R>::type{r.re, r.im};
                else
                    epi_store<R, EPI>(dst, (R*)e.r + (int64_t)(c0 + c) * e.ldr, cb, us, r, alpha[c], nacc[c]);
            }
    }
    if constexpr (EPI != TM_PLAIN) epi_finish<EPI, NC>(e, live, c0, ntiles, tile, esh, nacc);
}

// Rolled variant: a runtime loop over the 8 hops with a wave-uniform switch.
// Only one hop's operands are live at a time (low register use, high
// occupancy); the latency of a hop's loads is hidden by the other waves.
template <typename R, bool DAG, int MODE, int NC, int MINW, int EPI = TM_PLAIN>
__global__ __launch_bounds__(kBlock, MINW) void k_wilson_r(R* __restrict__ out, int64_t ldo, const R* __restrict__ in,
                                                         int64_t ldi, const R* __restrict__ U, Geom g, R kappa,
                                                         R tsign, int k, int ncg, int ntiles, int per_xcd, int G,
                                                         int zb, TmEpi e) {
    int tile, cgi;
    if (!map_work(ntiles, ncg, G, per_xcd, zb, g.T, tile, cgi)) return;
    const int c0 = cgi * NC;
    int s = tile * kBlock + threadIdx.x;
    const int V = (int)g.V;
    bool ok = true;  // as in k_wilson
    if constexpr (EPI == TM_PLAIN) {
        if (s >= V) return;
    } else {
        ok = s < V;
        if (!ok) s = V - 1;
    }
    const int XY = g.X * g.Y, XYZ = XY * g.Z;
    const int x = s % g.X;
    const int y = (s / g.X) % g.Y;
    const int z = (s / XY) % g.Z;
    const int t = s / XYZ;
    const unsigned us = (unsigned)s, uV = (unsigned)V;
    constexpr int SF = DAG ? 1 : -1;  // projector sign of the forward hop
    constexpr int SB = -SF;

    const R* src[NC];
    bool live[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        live[c] = c0 + c < k;
        src[c] = in + (int64_t)(live[c] ? c0 + c : c0) * ldi;
    }
    [[maybe_unused]] double* esh = nullptr;
    R alpha[NC];
    bool upd[NC];
    double nacc[NC];
    if constexpr (EPI != TM_PLAIN) {
        __shared__ double esh_[kWaves];
        esh = esh_;
        epi_setup<R, EPI, NC>(e, live, c0, ntiles, esh, alpha, upd, nacc);
    }
    cplx<R> acc[NC][4][3];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) acc[c][a][cc] = {R(0), R(0)};

#pragma unroll 1
    for (int d = 0; d < 8; ++d) {
        const int mu = d >> 1;
        const bool fwd = (d & 1) == 0;
        int nb;
        R bf = R(1);
        switch (mu) {
            case 0: nb = fwd ? (x == g.X - 1 ? s - (g.X - 1) : s + 1) : (x == 0 ? s + (g.X - 1) : s - 1); break;
            case 1: nb = fwd ? (y == g.Y - 1 ? s - (g.Y - 1) * g.X : s + g.X) : (y == 0 ? s + (g.Y - 1) * g.X : s - g.X); break;
            case 2: nb = fwd ? (z == g.Z - 1 ? s - (g.Z - 1) * XY : s + XY) : (z == 0 ? s + (g.Z - 1) * XY : s - XY); break;
            default:
                nb = fwd ? (t == g.T - 1 ? s - (g.T - 1) * XYZ : s + XYZ) : (t == 0 ? s + (g.T - 1) * XYZ : s - XYZ);
                bf = fwd ? ((t == g.T - 1) ? tsign : R(1)) : ((t == 0) ? tsign : R(1));
                break;
        }
        cplx<R> u[3][3], psi[4][3];
        load_link(U, uV, mu, fwd ? us : (unsigned)nb, u);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            load_spinor(src[c], uV, (unsigned)nb, psi);
            switch (d) {
                case 0: hop<0, SF, false>(acc[c], psi, u, bf); break;
                case 1: hop<0, SB, true>(acc[c], psi, u, bf); break;
                case 2: hop<1, SF, false>(acc[c], psi, u, bf); break;
                case 3: hop<1, SB, true>(acc[c], psi, u, bf); break;
                case 4: hop<2, SF, false>(acc[c], psi, u, bf); break;
                case 5: hop<2, SB, true>(acc[c], psi, u, bf); break;
                case 6: hop<3, SF, false>(acc[c], psi, u, bf); break;
                default: hop<3, SB, true>(acc[c], psi, u, bf); break;
            }
        }
    }

#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if constexpr (EPI == TM_PLAIN) {
            if (!live[c]) continue;
        } else {
            if (!ok || !upd[c]) continue;
        }
        R* dst = out + (int64_t)(c0 + c) * ldo;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                const size_t cb = 2 * (size_t)((a * 3 + cc) * uV);
                cplx<R> r = acc[c][a][cc];
                if constexpr (MODE == 0) {
                    const cplx<R> p = ldc(src[c] + cb, us);
                    r = {p.re - kappa * r.re, p.im - kappa * r.im};
                }
                if constexpr (EPI == TM_PLAIN)
                    reinterpret_cast<typename vec2<R>::type*>(dst + cb)[us] = typename vec2<R>::type{r.re, r.im};
                else
                    epi_store<R, EPI>(dst, (R*)e.r + (int64_t)(c0 + c) * e.ldr, cb, us, r, alpha[c], nacc[c]);
            }
    }
    if constexpr (EPI != TM_PLAIN) epi_finish<EPI, NC>(e, live, c0, ntiles, tile, esh, nacc);
}

// t-march form, for lattices whose xy-plane is one 256-site tile.  A block
// owns the xy-planes of NZ consecutive z (256 threads per plane) for NC
// columns and walks t through a segment of tlen time slices.  Per slice its
// spinors are staged in LDS, so the x and y hops read LDS, and so do the z
// hops between planes of the block; the +t neighbour is the same lane's next
// slice, loaded one slice ahead; the -t hop into the next slice,
// U_t^H (1 + SB gamma_t) psi(t), is formed while the slice is current (its
// link is the one the +t hop loads) and carried in registers as a half
// spinor.  Only the z hops out of the block's planes read other planes, from
// L2 or HBM: with one plane per block they re-read each spinor twice, and as
// a neighbour plane is next read a slice later by another block it has
// mostly left L2 by then; NZ planes cut that to 2 / NZ.  Work items
// enumerate (column group, segment, plane group) with the plane group
// fastest (CGMINOR = false: the planes of a segment run together on one XCD)
// or (segment, plane group, column group) with the column group fastest
// (CGMINOR = true: all column groups of a plane share its links through one
// L2).
//
// Epilogues (EPI, above), with the block's partial sums left per column at
// index column * (Z * nseg) + (segment * Z + z) of e.part.

// Sum over the 256 threads of plane zz of a block of NZ planes (the tree of
// block_sum, so the value is that of a one-plane block), and the index-order
// sum of a producer's partials taken the same way.
__device__ __forceinline__ double plane_sum(double v, double* sh /* kWaves per plane */, int zz) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = (threadIdx.x >> 6) & (kWaves - 1);
    __syncthreads();
    if (lane == 0) sh[zz * kWaves + w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) t += sh[zz * kWaves + i];
    return t;
}

__device__ __forceinline__ double plane_sum_partials(const double* __restrict__ part, int G, double* sh, int zz) {
    double s = 0.0;
    for (int i = threadIdx.x & (kBlock - 1); i < G; i += kBlock) s += part[i];
    return plane_sum(s, sh, zz);
}

template <typename R, bool DAG, int MODE, int NC, bool CGMINOR, int EPI = TM_PLAIN, int NZ = 1>
__global__ __launch_bounds__(kBlock * NZ) void k_wilson_tm(R* __restrict__ out, int64_t ldo, const R* __restrict__ in,
                                                           int64_t ldi, const R* __restrict__ U, Geom g, R kappa,
                                                           R tsign, int k, int ncg, int nseg, int tlen, int per_xcd,
                                                           TmEpi e = TmEpi{}) {
    using V2 = typename vec2<R>::type;
    __shared__ V2 pl[NZ][NC * 12][kBlock];
    __shared__ double nsh[kWaves * NZ];
    double nacc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) nacc[c] = 0.0;
    const int b = blockIdx.x;
    const int L = (b % kXcd) * per_xcd + b / kXcd;
    const int nzg = g.Z / NZ;  // groups of NZ consecutive planes
    if (g.X * g.Y != kBlock || g.Z % NZ != 0 || L >= ncg * nseg * nzg) return;  // uniform over the block
    const int Lp = CGMINOR ? L / ncg : L % (nzg * nseg);  // (segment, plane group) pair
    const int zz = threadIdx.x / kBlock;                   // this thread's plane in the group (wave-uniform)
    const int z = (Lp % nzg) * NZ + zz;
    const int seg = Lp / nzg;
    const int c0 = (CGMINOR ? L % ncg : L / (nzg * nseg)) * NC;
    const int t0 = seg * tlen;
    const int t1 = min(g.T, t0 + tlen);
    const int p = threadIdx.x % kBlock;  // x + X y
    const int x = p % g.X, y = p / g.X;
    const int XY = kBlock, XYZ = XY * g.Z;
    const unsigned uV = (unsigned)g.V;
    const int pxp = (x == g.X - 1 ? p - (g.X - 1) : p + 1), pxm = (x == 0 ? p + (g.X - 1) : p - 1);
    const int pyp = (y == g.Y - 1 ? p - (g.Y - 1) * g.X : p + g.X), pym = (y == 0 ? p + (g.Y - 1) * g.X : p - g.X);
    const int zoff_p = (z == g.Z - 1 ? -(g.Z - 1) * XY : XY), zoff_m = (z == 0 ? (g.Z - 1) * XY : -XY);
    constexpr int SF = DAG ? 1 : -1;
    constexpr int SB = -SF;

    const R* src[NC];
    bool live[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        live[c] = c0 + c < k;
        src[c] = in + (int64_t)(live[c] ? c0 + c : c0) * ldi;
    }
    R alpha[NC];
    bool upd[NC];
    if constexpr (EPI == TM_CG) {
        const int G = g.Z * nseg;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int col = live[c] ? c0 + c : c0;
            const double pq = plane_sum_partials(e.pq + (int64_t)col * G, G, nsh, zz);  // uniform
            upd[c] = live[c] && e.st[col].active;
            alpha[c] = upd[c] ? (R)(e.st[col].rho / pq) : R(0);
        }
    }

    // carry into slice t0 from slice t0 - 1
    cplx<R> cr0[NC][3], cr1[NC][3];
    {
        const int tm = (t0 == 0 ? g.T - 1 : t0 - 1);
        const unsigned sm = (unsigned)(p + XY * z + XYZ * tm);
        cplx<R> u[3][3], psi[4][3];
        load_link(U, uV, 3, sm, u);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            load_spinor(src[c], uV, sm, psi);
            hop_half<3, SB, true>(psi, u, t0 == 0 ? tsign : R(1), cr0[c], cr1[c]);
        }
    }
    cplx<R> cur[NC][4][3];
    {
        const unsigned s0 = (unsigned)(p + XY * z + XYZ * t0);
#pragma unroll
        for (int c = 0; c < NC; ++c) load_spinor(src[c], uV, s0, cur[c]);
    }

#pragma unroll 1
    for (int t = t0; t < t1; ++t) {
        const unsigned s = (unsigned)(p + XY * z + XYZ * t);
        __syncthreads();  // every lane is done reading the previous slice
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) pl[zz][c * 12 + a * 3 + cc][p] = V2{cur[c][a][cc].re, cur[c][a][cc].im};
        __syncthreads();

        cplx<R> acc[NC][4][3];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) acc[c][a][cc] = {R(0), R(0)};
            hop_acc<3, SB>(acc[c], cr0[c], cr1[c]);  // -t, carried
        }
        cplx<R> u[3][3], un[3][3], psi[4][3];
        // x, y hops from the staged slice (d = 0..3), then z hops (d = 4, 5)
        // from the neighbouring plane's staged slice where the block holds it,
        // else from L2; a rolled loop keeps one hop's operands live.  With
        // LPF the link of the next hop (after d = 5: of the +t hop) is loaded
        // while this one is computed (18 more registers per lane; only where
        // that does not lower the occupancy)
        constexpr bool LPF = sizeof(R) == 4 && NC == 2;
        auto lsite = [&](int d) -> unsigned {
            return (d & 1) == 0 ? s : (unsigned)((int)s + (d == 1 ? pxm - p : (d == 3 ? pym - p : zoff_m)));
        };
        if constexpr (LPF) load_link(U, uV, 0, s, un);
#pragma unroll 1
        for (int d = 0; d < 6; ++d) {
            const bool fwd = (d & 1) == 0;
            if constexpr (LPF) {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int bb = 0; bb < 3; ++bb) u[a][bb] = un[a][bb];
                if (d < 5) load_link(U, uV, (d + 1) >> 1, lsite(d + 1), un);
                else load_link(U, uV, 3, s, un);
            } else {
                load_link(U, uV, d >> 1, lsite(d), u);
            }
            if (d < 4) {
                const int pn = d == 0 ? pxp : (d == 1 ? pxm : (d == 2 ? pyp : pym));
#pragma unroll
                for (int c = 0; c < NC; ++c) {
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) {
                            const V2 v = pl[zz][c * 12 + a * 3 + cc][pn];
                            psi[a][cc] = {v.x, v.y};
                        }
                    switch (d) {
                        case 0: hop<0, SF, false>(acc[c], psi, u, R(1)); break;
                        case 1: hop<0, SB, true>(acc[c], psi, u, R(1)); break;
                        case 2: hop<1, SF, false>(acc[c], psi, u, R(1)); break;
                        default: hop<1, SB, true>(acc[c], psi, u, R(1)); break;
                    }
                }
            } else {
                const unsigned sn = (unsigned)((int)s + (fwd ? zoff_p : zoff_m));
                const int zn = fwd ? zz + 1 : zz - 1;  // the neighbour's plane in the group
                const bool staged = NZ > 1 && zn >= 0 && zn < NZ;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    if (staged) {
#pragma unroll
                        for (int a = 0; a < 4; ++a)
#pragma unroll
                            for (int cc = 0; cc < 3; ++cc) {
                                const V2 v = pl[zn][c * 12 + a * 3 + cc][p];
                                psi[a][cc] = {v.x, v.y};
                            }
                    } else {
                        load_spinor(src[c], uV, sn, psi);
                    }
                    if (fwd) hop<2, SF, false>(acc[c], psi, u, R(1));
                    else hop<2, SB, true>(acc[c], psi, u, R(1));
                }
            }
        }
        // +t hop with the next slice, which becomes current; carry the -t hop
        // of the next slice, formed from this one with the same link
        {
            const unsigned sp = (unsigned)(t == g.T - 1 ? (int)s - (g.T - 1) * XYZ : (int)s + XYZ);
            const R bfp = (t == g.T - 1) ? tsign : R(1);
            if constexpr (!LPF) load_link(U, uV, 3, s, un);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                load_spinor(src[c], uV, sp, psi);
                hop<3, SF, false>(acc[c], psi, un, bfp);
                hop_half<3, SB, true>(cur[c], un, R(1), cr0[c], cr1[c]);
                // write this slice's result, then advance
                if (EPI == TM_CG ? upd[c] : live[c]) {
                    R* dst = out + (int64_t)(c0 + c) * ldo;
                    R* rv = (R*)e.r + (int64_t)(c0 + c) * e.ldr;
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) {
                            cplx<R> r = acc[c][a][cc];
                            if constexpr (MODE == 0) r = {cur[c][a][cc].re - kappa * r.re, cur[c][a][cc].im - kappa * r.im};
                            const size_t off = 2 * (size_t)((a * 3 + cc) * uV);
                            if constexpr (EPI == TM_CG) {
                                V2 rr = reinterpret_cast<V2*>(rv + off)[s];
                                rr.x = rr.x - alpha[c] * r.re;
                                rr.y = rr.y - alpha[c] * r.im;
                                reinterpret_cast<V2*>(rv + off)[s] = rr;
                                nacc[c] += (double)rr.x * (double)rr.x + (double)rr.y * (double)rr.y;
                            } else {
                                reinterpret_cast<V2*>(dst + off)[s] = V2{r.re, r.im};
                                if constexpr (EPI == TM_NORM)
                                    nacc[c] += (double)r.re * (double)r.re + (double)r.im * (double)r.im;
                            }
                        }
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) cur[c][a][cc] = psi[a][cc];
            }
        }
    }
    if constexpr (EPI != TM_PLAIN) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double tot = plane_sum(nacc[c], nsh, zz);
            if (p == 0 && live[c]) e.part[(int64_t)(c0 + c) * (g.Z * nseg) + seg * g.Z + z] = tot;
        }
    }
}

// Direction-split form, for few columns: a block covers 64 sites of one
// column and its wave w takes the two hops of direction mu = w (wave-uniform,
// so no lane diverges); the four partial sums meet in LDS and wave w writes
// spin component w of the result.  Four times the waves of the one-site-per-
// thread form, each with a chain of two dependent hops instead of eight: for
// launches too small to hide memory latency otherwise.
template <typename R, bool DAG, int MODE, bool REC>
__global__ __launch_bounds__(kBlock) void k_wilson_dir(R* __restrict__ out, int64_t ldo, const R* __restrict__ in,
                                                       int64_t ldi, const R* __restrict__ U, Geom g, R kappa,
                                                       R tsign, int k, int ntile, int per_xcd) {
    __shared__ R red[4][24][64];
    const int b = blockIdx.x;
    const int L = (b % kXcd) * per_xcd + b / kXcd;
    if (L >= ntile * k) return;  // uniform over the block
    const int tile = L / k, col = L % k;
    const int mu = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int s = tile * 64 + l;
    const bool ok = s < (int)g.V;
    const unsigned uV = (unsigned)g.V;
    const R* src = in + (int64_t)col * ldi;
    cplx<R> acc[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) acc[a][cc] = {R(0), R(0)};
    if (ok) {  // the x hops by DPP when a lane row is an x-row (X = 16)
        if (mu == 0 && g.X == 16) dir_hops_x16<DAG, R, REC>(acc, src, U, uV, s);
        else dir_hops<DAG, R, REC>(acc, src, U, g, uV, s, mu, tsign);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            red[mu][(a * 3 + cc) * 2][l] = acc[a][cc].re;
            red[mu][(a * 3 + cc) * 2 + 1][l] = acc[a][cc].im;
        }
    __syncthreads();
    if (!ok) return;
    R* dst = out + (int64_t)col * ldo;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        const int j = (mu * 3 + cc) * 2;  // spin mu, colour cc
        cplx<R> r = {red[0][j][l] + red[1][j][l] + red[2][j][l] + red[3][j][l],
                     red[0][j + 1][l] + red[1][j + 1][l] + red[2][j + 1][l] + red[3][j + 1][l]};
        const size_t cb = 2 * (size_t)((mu * 3 + cc) * uV);
        if constexpr (MODE == 0) {
            const cplx<R> p = ldc(src + cb, (unsigned)s);
            r = {p.re - kappa * r.re, p.im - kappa * r.im};
        }
        reinterpret_cast<typename vec2<R>::type*>(dst + cb)[s] = typename vec2<R>::type{r.re, r.im};
    }
}

// ---------------------------------------------------------------- variants and autotuning
// A launch shape is (hop loop form x columns per thread), a column-chunk size
// G and a tile order; variant id = order * 16 + shape * 4 + chunk with chunk
// 0: G = all groups, 1: G = 1, 2: G = 2, 3: G = 4, and order 0: site order,
// 1: z-blocked by 4 tiles.  Ids 32..43 are the t-march form with one plane
// per block: 32 + 6 * order + 3 * (NC - 1) + {0, 1, 2} for segments of
// {4, 8, 16} time slices, order 0: column group slowest, 1: fastest.  Id 44
// is the direction-split form.  Ids 45..56 and 57..68 are the t-march form
// with 2 and 4 planes per block, numbered as 32..43 from 45 and 57.
enum WilsonShape { WS_UNROLLED_1 = 0, WS_ROLLED_1 = 1, WS_ROLLED_2 = 2, WS_ROLLED_4 = 3, WS_COUNT = 4 };
constexpr int kChunks = 4;
constexpr int kOrders = 2;
constexpr int kZBlock = 4;
constexpr int WV_TILED = kOrders * WS_COUNT * kChunks;
constexpr int WV_TMARCH = 12;
constexpr int WV_DIR = WV_TILED + WV_TMARCH;  // the direction-split form
constexpr int WV_TM2 = WV_DIR + 1;            // t-march, 2 and 4 planes per block
constexpr int WV_TX = WV_TM2 + 2 * WV_TMARCH;  // one column per thread, x hops by DPP (FP32, X = Y = 16)
constexpr int WV_NTX = 18;
constexpr int WV_COUNT = WV_TX + WV_NTX;
static_assert(WV_COUNT == SC_WILSON_VARIANTS, "variant count must match the header");

// The DPP form (wilson_tx.h): ids WV_TX + 6 * (nc - 1) + 3 * order + {0, 1, 2}
// for nc = 1, 2 columns per thread and segments of {4, 8, 16} time slices,
// order 0: the planes of a segment are consecutive work items, 1: the column
// groups of a plane are; ids WV_TX + 12 + 3 * (nc - 1) + {0, 1, 2}: order 2,
// quads of planes with the column groups of a quad consecutive (tx_item).
// FP32 D and D^H passes only, on
// lattices with X = Y = 16 (an x-row is a 16-lane DPP row, four y-rows a
// wave); its accumulator starts at -psi / kappa, so kappa must not be tiny.
static bool is_tx(int v) { return v >= WV_TX && v < WV_TX + WV_NTX; }
static bool tx_ok(const sc_op* op) {
    return op->dims[0] == 16 && op->dims[1] == 16 && std::fabs(op->kappa) >= 1e-6 &&
           288 * op->vol < (int64_t(1) << 31);  // FP32 links below 2^31 bytes (32-bit buffer offsets)
}
static int tx_tlen(const sc_op* op, int v) {
    const int i = (v - WV_TX) % 3;
    return std::max(1, std::min(i == 0 ? 4 : (i == 1 ? 8 : 16), op->dims[3]));
}
static int tx_nc(int v) {
    const int i = v - WV_TX;
    return i < 12 ? (i >= 6 ? 2 : 1) : (i >= 15 ? 2 : 1);
}
static int tx_order(int v) {
    const int i = v - WV_TX;
    return i < 12 ? ((i % 6) >= 3 ? 1 : 0) : 2;
}
static int tx_parts(const sc_op* op, int v) { return op->dims[2] * ((op->dims[3] + tx_tlen(op, v) - 1) / tx_tlen(op, v)); }

// launch geometry of a DPP-form pass (used by the launch and by its range check)
struct TxGeom {
    int nc, tlen, nseg, ncg, per_xcd, blocks, order;
};
static TxGeom tx_geom(const sc_op* op, int v, int k) {
    TxGeom q;
    q.nc = tx_nc(v);
    q.tlen = tx_tlen(op, v);
    q.nseg = (op->dims[3] + q.tlen - 1) / q.tlen;
    q.ncg = (k + q.nc - 1) / q.nc;
    q.per_xcd = (q.ncg * op->dims[2] * q.nseg + kXcd - 1) / kXcd;
    q.blocks = q.per_xcd * kXcd;
    q.order = tx_order(v);
    return q;
}

static void tx_launch(const sc_op* op, int v, bool dag, int epi, const float* X, int64_t ldx, float* Y, int64_t ldy,
                      int k, const float* U, const TmEpi& e, hipStream_t s) {
    Geom g{op->dims[0], op->dims[1], op->dims[2], op->dims[3], op->vol};
    const TxGeom q = tx_geom(op, v, k);
    const dim3 grid((unsigned)q.blocks), blk(kBlock);
    const float kap = (float)op->kappa, ts = op->antiperiodic ? -1.0f : 1.0f;
    // SU(3) links: rows 0 and 1 of each link read, row 2 rebuilt
#define SC_TX(DAG, EPI_, NC_)                                                                                         \
    do {                                                                                                              \
        if (op->su3)                                                                                                  \
            SC_TLAUNCH((k_wilson_tx<DAG, EPI_, NC_, true>), grid, blk, 0, s, Y, 2 * ldy, X, 2 * ldx, U, g, kap, ts, \
                       k, q.nseg, q.tlen, q.per_xcd, q.order, e);                                                     \
        else                                                                                                          \
            SC_TLAUNCH((k_wilson_tx<DAG, EPI_, NC_, false>), grid, blk, 0, s, Y, 2 * ldy, X, 2 * ldx, U, g, kap,    \
                       ts, k, q.nseg, q.tlen, q.per_xcd, q.order, e);                                                 \
    } while (0)
#define SC_TXE(NC_)                                 \
    if (epi == TM_NORM) SC_TX(false, TM_NORM, NC_); \
    else if (epi == TM_CG) SC_TX(true, TM_CG, NC_); \
    else if (dag) SC_TX(true, TM_PLAIN, NC_);       \
    else SC_TX(false, TM_PLAIN, NC_);
    if (tx_nc(v) == 1) {
        SC_TXE(1)
    } else {
        SC_TXE(2)
    }
#undef SC_TXE
#undef SC_TX
}

// Every buffer access of one DPP-form launch (any epilogue) on a lattice
// with these dims, k columns of leading dimensions ldx (source) and ldy
// (destination) in complex elements, walked on the host with the kernel's own
// index functions (wilson_tx.h): each load and store's byte offset against
// its descriptor's record (links 288 V bytes; a column 96 V bytes from the
// column's start, which must itself lie within the caller's k columns), and
// each partial-sum index against the k * parts of the caller's buffer.
// *accesses counts the checks, *outside the failures.
sc_status wilson_tx_check(const int dims[4], int v, int k, int64_t ldx, int64_t ldy, int64_t* accesses,
                          int64_t* outside) {
    sc_op op{};
    for (int i = 0; i < 4; ++i) op.dims[i] = dims[i];
    op.vol = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    op.n = 12 * op.vol;
    op.kappa = 0.12;
    if (!is_tx(v) || !tx_ok(&op) || k < 1 || dims[2] < 1 || dims[3] < 1) {
        set_error("wilson_tx_check: not a DPP-form shape for this lattice");
        return SC_ERR_ARG;
    }
    const TxGeom q = tx_geom(&op, v, k);
    const int Z = dims[2], T = dims[3];
    const int64_t V = op.vol;
    const unsigned uV = (unsigned)V;
    const int parts = Z * q.nseg;
    int64_t n = 0, bad = 0;
    // a load or store of site `site` with components up to `cmax` through a
    // descriptor of `rec` bytes: 32-bit offsets that the hardware adds, in range
    auto chk = [&](int64_t site, int cmax, int64_t rec) {
        ++n;
        const int64_t boff = (int64_t)tx_boff((unsigned)site), soff = (int64_t)tx_soff(cmax, uV);
        if (site < 0 || site >= V || boff + soff + 8 > rec || boff + soff + 8 > (int64_t(1) << 31)) ++bad;
    };
    // a column's descriptor: it starts col * ld complex elements in and spans 96 V
    // bytes, within the caller's k columns of ld elements (ld >= n)
    auto chk_col = [&](int col, int64_t ld) {
        ++n;
        const int64_t start = (int64_t)col * ld * 8, end = ((int64_t)(k - 1) * ld + op.n) * 8;
        if (col < 0 || col >= k || ld < op.n || start + (int64_t)kTxSpinorBytes * V > end) ++bad;
    };
    const int64_t lrec = (int64_t)kTxLinkBytes * V, srec = (int64_t)kTxSpinorBytes * V;
    for (int b = 0; b < q.blocks; ++b) {
        const int L = (b % kXcd) * q.per_xcd + b / kXcd;
        if (L >= q.ncg * Z * q.nseg) continue;  // the kernel returns
        const TxItem wi = tx_item(L, q.ncg, Z, q.nseg, q.order);
        const int t0 = wi.seg * q.tlen, t1 = std::min(T, t0 + q.tlen);
        ++n;
        if (wi.cg < 0 || wi.cg >= q.ncg || wi.z < 0 || wi.z >= Z || wi.seg < 0 || wi.seg >= q.nseg || t0 >= T) ++bad;
        for (int c = 0; c < q.nc; ++c) {
            const int col = tx_col(wi.cg, c, q.nc, k);
            chk_col(col, ldx);
            if (wi.cg * q.nc + c < k) {  // a column that stores (others get a zero-size record)
                chk_col(col, ldy);
                ++n;
                const int64_t pi = (int64_t)col * parts + (int64_t)wi.seg * Z + wi.z;
                if (pi < 0 || pi >= (int64_t)k * parts) ++bad;
            }
        }
        const int zp = tx_zstep(wi.z, Z, 1), zm = tx_zstep(wi.z, Z, -1);
        for (int p = 0; p < kTxPlane; ++p) {
            const int sm = tx_site(p, wi.z, tx_tprev(t0, T), Z);
            chk(sm, 3 * 9 + 8, lrec);  // U_t of the carried -t hop
            chk(sm, 11, srec);         // its spinor
            chk(tx_site(p, wi.z, t0, Z), 11, srec);
            for (int t = t0; t < t1; ++t) {
                const int s = tx_site(p, wi.z, t, Z);
                for (int mu = 0; mu < 4; ++mu) chk(s, mu * 9 + 8, lrec);
                chk(s + zm, 2 * 9 + 8, lrec);
                chk(s + zp, 11, srec);
                chk(s + zm, 11, srec);
                chk(tx_tnext_site(s, t, T, Z), 11, srec);
                chk(s, 11, srec);  // the store (and the TM_CG load of r)
            }
        }
    }
    *accesses = n;
    *outside = bad;
    return SC_OK;
}

static int chunk_groups(int chunk, int ncg) {
    const int g = chunk == 0 ? ncg : (chunk == 1 ? 1 : (chunk == 2 ? 2 : 4));
    return std::max(1, std::min(g, ncg));
}

// the z-blocked order needs whole tiles per time slice, in blocks of kZBlock
static bool zblock_ok(const sc_op* op) {
    const int64_t slice = (int64_t)op->dims[0] * op->dims[1] * op->dims[2];
    return slice % kBlock == 0 && (slice / kBlock) % kZBlock == 0 && slice / kBlock > kZBlock;
}

// the t-march form needs the xy-plane to be exactly one tile
static bool tmarch_ok(const sc_op* op) { return op->dims[0] * op->dims[1] == kBlock; }

template <typename R, int NC, bool CGMINOR, int NZ>
static void wilson_launch_tm(const sc_op* op, int which, const R* X, int64_t ldx, R* Y, int64_t ldy, int k,
                             const R* U, int tlen, hipStream_t s, int epi = TM_PLAIN, TmEpi e = TmEpi{}) {
    Geom g{op->dims[0], op->dims[1], op->dims[2], op->dims[3], op->vol};
    tlen = std::max(1, std::min(tlen, g.T));
    const int nseg = (g.T + tlen - 1) / tlen;
    const int ncg = (k + NC - 1) / NC;
    const int per_xcd = (ncg * nseg * (g.Z / NZ) + kXcd - 1) / kXcd;
    const dim3 grid((unsigned)(per_xcd * kXcd)), blk(kBlock * NZ);
    const R kap = (R)op->kappa;
    const R ts = op->antiperiodic ? R(-1) : R(1);
#define SC_WT(DAG, MODE)                                                                                   \
    SC_TLAUNCH((k_wilson_tm<R, DAG, MODE, NC, CGMINOR, TM_PLAIN, NZ>), grid, blk, 0, s, Y, 2 * ldy, X, \
               2 * ldx, U, g, kap, ts, k, ncg, nseg, tlen, per_xcd, TmEpi{});
    if (epi == TM_NORM) {  // D pass with the |D x|^2 partials
        SC_TLAUNCH((k_wilson_tm<R, false, 0, NC, CGMINOR, TM_NORM, NZ>), grid, blk, 0, s, Y, 2 * ldy, X,
                   2 * ldx, U, g, kap, ts, k, ncg, nseg, tlen, per_xcd, e);
        return;
    }
    if (epi == TM_CG) {  // D^H pass finishing r -= alpha A p
        SC_TLAUNCH((k_wilson_tm<R, true, 0, NC, CGMINOR, TM_CG, NZ>), grid, blk, 0, s, Y, 2 * ldy, X,
                   2 * ldx, U, g, kap, ts, k, ncg, nseg, tlen, per_xcd, e);
        return;
    }
    switch (which) {
        case 0: SC_WT(false, 0) break;
        case 1: SC_WT(true, 0) break;
        case 2: SC_WT(false, 1) break;
        default: SC_WT(true, 1) break;
    }
#undef SC_WT
}

// Effective t-march shape of variant v on this lattice and precision.  FP64
// has 1 column per thread (2 would spill); a block's staged planes must fit
// the 160 KB of LDS (at most 4 plane-columns of FP32 or 2 of FP64, 24 KB
// each) and the plane groups must tile Z; a pinned shape that does not fit
// takes the next smaller plane group.
struct TmShape {
    int tlen, nc, nz;
    bool cgminor;
};
static bool is_tmarch(int v) { return (v >= WV_TILED && v < WV_DIR) || (v >= WV_TM2 && v < WV_TX); }
static TmShape tm_shape(int v, bool single, int Z) {
    const int i = v < WV_DIR ? v - WV_TILED : (v - WV_TM2) % WV_TMARCH;
    TmShape t;
    t.nz = v < WV_DIR ? 1 : ((v - WV_TM2) < WV_TMARCH ? 2 : 4);
    t.tlen = i % 3 == 0 ? 4 : (i % 3 == 1 ? 8 : 16);
    t.nc = ((i / 3) % 2 == 1 && single) ? 2 : 1;
    t.cgminor = i >= 6;
    while (t.nz > 1 && (t.nz * t.nc * (single ? 1 : 2) > 4 || Z % t.nz != 0)) t.nz /= 2;
    return t;
}

template <typename R>
static void tm_launch(const sc_op* op, int which, const R* X, int64_t ldx, R* Y, int64_t ldy, int k, const R* U,
                      const TmShape& t, int epi, const TmEpi& e, hipStream_t s) {
#define SC_TMD(NC_, NZ_)                                                                                   \
    {                                                                                                      \
        if (t.cgminor) wilson_launch_tm<R, NC_, true, NZ_>(op, which, X, ldx, Y, ldy, k, U, t.tlen, s, epi, e); \
        else wilson_launch_tm<R, NC_, false, NZ_>(op, which, X, ldx, Y, ldy, k, U, t.tlen, s, epi, e);     \
    }
    if (t.nc == 1) {
        if (t.nz == 1) SC_TMD(1, 1)
        else if (t.nz == 2) SC_TMD(1, 2)
        else if constexpr (sizeof(R) == 4) SC_TMD(1, 4)
    } else if constexpr (sizeof(R) == 4) {
        if (t.nz == 1) SC_TMD(2, 1)
        else SC_TMD(2, 2)
    }
#undef SC_TMD
}

template <typename R>
static void wilson_launch_dir(const sc_op* op, int which, const R* X, int64_t ldx, R* Y, int64_t ldy, int k,
                              const R* U, hipStream_t s) {
    Geom g{op->dims[0], op->dims[1], op->dims[2], op->dims[3], op->vol};
    const int ntile = (int)((g.V + 63) / 64);
    const int per_xcd = (ntile * k + kXcd - 1) / kXcd;
    dim3 grid((unsigned)(per_xcd * kXcd));
    const R kap = (R)op->kappa;
    const R ts = op->antiperiodic ? R(-1) : R(1);
    // SU(3) links in a single-precision pass: rows 0 and 1 read, row 2 rebuilt
    constexpr bool kRec = sizeof(R) == 4;
    const bool rec = kRec && op->su3;
#define SC_WD(DAG, MODE)                                                                                           \
    if (rec)                                                                                                       \
        SC_TLAUNCH((k_wilson_dir<R, DAG, MODE, kRec>), grid, dim3(kBlock), 0, s, Y, 2 * ldy, X, 2 * ldx, U, g,  \
                   kap, ts, k, ntile, per_xcd);                                                                    \
    else                                                                                                           \
        SC_TLAUNCH((k_wilson_dir<R, DAG, MODE, false>), grid, dim3(kBlock), 0, s, Y, 2 * ldy, X, 2 * ldx, U, g, \
                   kap, ts, k, ntile, per_xcd);
    switch (which) {
        case 0: SC_WD(false, 0) break;
        case 1: SC_WD(true, 0) break;
        case 2: SC_WD(false, 1) break;
        default: SC_WD(true, 1) break;
    }
#undef SC_WD
}

template <typename R, int NC, bool ROLLED>
static void wilson_launch_v(const sc_op* op, int which, const R* X, int64_t ldx, R* Y, int64_t ldy, int k, const R* U,
                            int chunk, int order, hipStream_t s) {
    Geom g{op->dims[0], op->dims[1], op->dims[2], op->dims[3], op->vol};
    const int ntiles = (int)((g.V + kBlock - 1) / kBlock);
    const int ncg = (k + NC - 1) / NC;
    const int G = chunk_groups(chunk, ncg);
    const int zb = (order == 1 && zblock_ok(op)) ? kZBlock : 1;
    const int per_xcd = (ntiles * ncg + kXcd - 1) / kXcd;
    dim3 grid((unsigned)(per_xcd * kXcd));
    const R kap = (R)op->kappa;
    const R ts = op->antiperiodic ? R(-1) : R(1);
    // ld arguments are in reals (2 per complex element)
#define SC_WL(DAG, MODE)                                                                                       \
    if constexpr (ROLLED)                                                                                      \
        SC_TLAUNCH((k_wilson_r<R, DAG, MODE, NC, 1>), grid, dim3(kBlock), 0, s, Y, 2 * ldy, X,         \
                           2 * ldx, U, g, kap, ts, k, ncg, ntiles, per_xcd, G, zb, TmEpi{});                   \
    else                                                                                                       \
        SC_TLAUNCH((k_wilson<R, DAG, MODE, NC, 1, false>), grid, dim3(kBlock), 0, s, Y, 2 * ldy, X,    \
                           2 * ldx, U, g, kap, ts, k, ncg, ntiles, per_xcd, G, zb, TmEpi{});
    switch (which) {
        case 0: SC_WL(false, 0) break;
        case 1: SC_WL(true, 0) break;
        case 2: SC_WL(false, 1) break;
        default: SC_WL(true, 1) break;
    }
#undef SC_WL
}

// The fused CG passes on a tiled shape: epi TM_NORM is the D pass (partials of
// |D p|^2), TM_CG the D^H pass (r -= alpha A p); partials per column and tile.
template <typename R, int NC, bool ROLLED>
static void wilson_launch_v_epi(const sc_op* op, int epi, const R* X, int64_t ldx, R* Y, int64_t ldy, int k,
                                const R* U, int chunk, int order, const TmEpi& e, hipStream_t s) {
    Geom g{op->dims[0], op->dims[1], op->dims[2], op->dims[3], op->vol};
    const int ntiles = (int)((g.V + kBlock - 1) / kBlock);
    const int ncg = (k + NC - 1) / NC;
    const int G = chunk_groups(chunk, ncg);
    const int zb = (order == 1 && zblock_ok(op)) ? kZBlock : 1;
    const int per_xcd = (ntiles * ncg + kXcd - 1) / kXcd;
    dim3 grid((unsigned)(per_xcd * kXcd));
    const R kap = (R)op->kappa;
    const R ts = op->antiperiodic ? R(-1) : R(1);
#define SC_WLE(DAG, EPI_)                                                                                      \
    if constexpr (ROLLED)                                                                                      \
        SC_TLAUNCH((k_wilson_r<R, DAG, 0, NC, 1, EPI_>), grid, dim3(kBlock), 0, s, Y, 2 * ldy, X, 2 * ldx, U, \
                   g, kap, ts, k, ncg, ntiles, per_xcd, G, zb, e);                                             \
    else                                                                                                       \
        SC_TLAUNCH((k_wilson<R, DAG, 0, NC, 1, false, EPI_>), grid, dim3(kBlock), 0, s, Y, 2 * ldy, X,        \
                   2 * ldx, U, g, kap, ts, k, ncg, ntiles, per_xcd, G, zb, e);
    if (epi == TM_NORM) {
        SC_WLE(false, TM_NORM)
    } else {
        SC_WLE(true, TM_CG)
    }
#undef SC_WLE
}

template <typename R>
static void wilson_launch_variant_epi(int v, const sc_op* op, int epi, const R* X, int64_t ldx, R* Y, int64_t ldy,
                                      int k, const R* U, const TmEpi& e, hipStream_t s) {
    constexpr int N4 = sizeof(R) == 4 ? 4 : 2;
    const int chunk = v % kChunks, order = v / (WS_COUNT * kChunks);
    switch ((v / kChunks) % WS_COUNT) {
        case WS_UNROLLED_1: wilson_launch_v_epi<R, 1, false>(op, epi, X, ldx, Y, ldy, k, U, chunk, order, e, s); break;
        case WS_ROLLED_1: wilson_launch_v_epi<R, 1, true>(op, epi, X, ldx, Y, ldy, k, U, chunk, order, e, s); break;
        case WS_ROLLED_2: wilson_launch_v_epi<R, 2, true>(op, epi, X, ldx, Y, ldy, k, U, chunk, order, e, s); break;
        default: wilson_launch_v_epi<R, N4, true>(op, epi, X, ldx, Y, ldy, k, U, chunk, order, e, s); break;
    }
}

static int default_variant(bool single, int k) {
    return (k <= 1 ? WS_ROLLED_1 : (single ? WS_ROLLED_2 : WS_ROLLED_1)) * kChunks;
}

// FP64 has no 4-column shape (it would spill): it uses 2 columns there
template <typename R>
static void wilson_launch_variant(int v, const sc_op* op, int which, const R* X, int64_t ldx, R* Y, int64_t ldy, int k,
                                  const R* U, hipStream_t s) {
    if (is_tx(v)) {
        if constexpr (sizeof(R) == 4) {
            if (tx_ok(op) && which < 2) {
                tx_launch(op, v, which == 1, TM_PLAIN, X, ldx, Y, ldy, k, U, TmEpi{}, s);
                return;
            }
        }
        v = default_variant(sizeof(R) == 4, k);  // H passes, FP64 or another lattice
    }
    if (v == WV_DIR) {
        wilson_launch_dir<R>(op, which, X, ldx, Y, ldy, k, U, s);
        return;
    }
    if (is_tmarch(v) && !tmarch_ok(op)) v = default_variant(sizeof(R) == 4, k);  // not for this lattice
    if (is_tmarch(v)) {
        tm_launch<R>(op, which, X, ldx, Y, ldy, k, U, tm_shape(v, sizeof(R) == 4, op->dims[2]), TM_PLAIN, TmEpi{},
                     s);
        return;
    }
    constexpr int N4 = sizeof(R) == 4 ? 4 : 2;
    const int chunk = v % kChunks, order = v / (WS_COUNT * kChunks);
    switch ((v / kChunks) % WS_COUNT) {
        case WS_UNROLLED_1: wilson_launch_v<R, 1, false>(op, which, X, ldx, Y, ldy, k, U, chunk, order, s); break;
        case WS_ROLLED_1: wilson_launch_v<R, 1, true>(op, which, X, ldx, Y, ldy, k, U, chunk, order, s); break;
        case WS_ROLLED_2: wilson_launch_v<R, 2, true>(op, which, X, ldx, Y, ldy, k, U, chunk, order, s); break;
        default: wilson_launch_v<R, N4, true>(op, which, X, ldx, Y, ldy, k, U, chunk, order, s); break;
    }
}

// variants worth timing for this lattice, precision and column count
static bool variant_applies(const sc_op* op, int v, bool single, int k) {
    // (with one column group the orders 1 and 2 repeat order 0's work on other planes first: skipped)
    if (is_tx(v)) return single && tx_ok(op) && k > 1 && !(k <= tx_nc(v) && tx_order(v) != 0);
    if (v == WV_DIR) return k <= 4;
    if (is_tmarch(v)) {
        const int i = v < WV_DIR ? v - WV_TILED : (v - WV_TM2) % WV_TMARCH;
        const int nz = v < WV_DIR ? 1 : ((v - WV_TM2) < WV_TMARCH ? 2 : 4);
        if (!tmarch_ok(op)) return false;
        if ((i / 3) % 2 == 1 && (k == 1 || !single)) return false;  // 2 columns: FP64 would spill
        if (i >= 6 && k == 1) return false;                           // one column group: orders agree
        return tm_shape(v, single, op->dims[2]).nz == nz;             // else the same as a smaller group
    }
    const int shape = (v / kChunks) % WS_COUNT, chunk = v % kChunks, order = v / (WS_COUNT * kChunks);
    if (order == 1 && !zblock_ok(op)) return false;  // same as site order
    if (!single && shape == WS_ROLLED_4) return false;  // same as 2 columns in FP64
    const int nc = shape == WS_ROLLED_4 ? 4 : (shape == WS_ROLLED_2 ? 2 : 1);
    if (nc > 1 && k == 1) return false;
    const int ncg = (k + nc - 1) / nc;
    if (chunk != 0 && chunk_groups(chunk, ncg) == ncg) return false;  // same order as chunk 0
    return true;
}

namespace {
struct TuneKey {
    int dims[4];
    int single, k;
    int rec;  // single-precision passes rebuilding row 2 of SU(3) links (they move fewer bytes)
    bool operator<(const TuneKey& o) const {
        for (int i = 0; i < 4; ++i)
            if (dims[i] != o.dims[i]) return dims[i] < o.dims[i];
        if (single != o.single) return single < o.single;
        if (rec != o.rec) return rec < o.rec;
        return k < o.k;
    }
};
struct TuneRec {
    int best;
    float us[WV_COUNT];
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneRec> g_tune;
int g_tune_mode = -1;  // -1: read SEEDCG_TUNE on first use; 0: defaults only; 1: tune


}  // namespace

// Expected HBM traffic of a shape's work order, lowest first, from the
// FETCH_SIZE / WRITE_SIZE counters of the 24-column FP32 passes on 16^3 x 32
// (traffic over algorithmic bytes, class means): the DPP form in quads of
// planes, then the t-march forms with 2 or 4 planes per block (1.5x), the DPP
// form with column groups fastest (1.8x), the one-plane t-march forms
// (1.8-2.2x), the DPP form with planes fastest (2.4x), the direction-split form
// (one column: 1.3x, few columns), the tiled forms (site order, about 3x).
static int traffic_rank(int v) {
    if (is_tx(v)) return tx_order(v) == 2 ? 0 : (tx_order(v) == 1 ? 2 : 4);
    if (v >= WV_TM2 && v < WV_TX) return 1;
    if (v >= WV_TILED && v < WV_DIR) return 3;
    if (v == WV_DIR) return 5;
    return 6;
}
constexpr float kTuneTie = 1.03f;

// Time every variant on the caller's buffers (the output is rewritten by the
// real launch that follows) and keep the fastest for (lattice, precision, k),
// time ties going to the shape with the lower expected traffic.
// Returns false, with rec holding the default shape and no timings, when a HIP
// call fails; the caller does not cache that result.
template <typename R>
static bool tune_variants(const sc_op* op, int which, const R* X, int64_t ldx, R* Y, int64_t ldy, int k, const R* U,
                          hipStream_t s, TuneRec& rec) {
    const int dflt = default_variant(sizeof(R) == 4, k);
    rec.best = dflt;
    for (int v = 0; v < WV_COUNT; ++v) rec.us[v] = -1.0f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return false;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return false;
    }
    float best = 1e30f;
    bool ok = true;
    for (int v = 0; v < WV_COUNT && ok; ++v) {
        if (!variant_applies(op, v, sizeof(R) == 4, k)) continue;
        wilson_launch_variant<R>(v, op, which, X, ldx, Y, ldy, k, U, s);  // warm
        // median of 5 individually timed launches (robust to a stray slow one)
        float t[5];
        for (int r = 0; r < 5 && ok; ++r) {
            ok = hipEventRecord(e0, s) == hipSuccess;
            if (ok) wilson_launch_variant<R>(v, op, which, X, ldx, Y, ldy, k, U, s);
            ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                 hipEventElapsedTime(&t[r], e0, e1) == hipSuccess;
        }
        if (!ok) break;
        std::sort(t, t + 5);
        rec.us[v] = t[2] * 1000.0f;
        if (rec.us[v] < best) {
            best = rec.us[v];
            rec.best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // a time tie (within kTuneTie of the fastest, the spread of repeated
    // timings) goes to the shape that moves the fewest bytes past L2
    if (ok) {
        int pick = rec.best;
        for (int v = 0; v < WV_COUNT; ++v) {
            if (rec.us[v] < 0.0f || rec.us[v] > kTuneTie * best) continue;
            const int rv = traffic_rank(v), rp = traffic_rank(pick);
            if (rv < rp || (rv == rp && rec.us[v] < rec.us[pick])) pick = v;
        }
        rec.best = pick;
    }
    if (!ok) {
        rec.best = dflt;
        for (int v = 0; v < WV_COUNT; ++v) rec.us[v] = -1.0f;
    }
    return ok;
}

template <typename R>
static int choose_variant(const sc_op* op, int which, const R* X, int64_t ldx, R* Y, int64_t ldy, int k, const R* U,
                          hipStream_t s) {
    TuneKey key{{op->dims[0], op->dims[1], op->dims[2], op->dims[3]}, sizeof(R) == 4 ? 1 : 0, k,
                (sizeof(R) == 4 && op->su3) ? 1 : 0};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second.best;
    if (g_tune_mode < 0) {
        const char* e = getenv("SEEDCG_TUNE");
        g_tune_mode = (e && e[0] == '0') ? 0 : 1;
    }
    // no timing while the stream is captured into a graph (or when that cannot be asked)
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool capturing = hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
    if (g_tune_mode == 0 || capturing) return default_variant(sizeof(R) == 4, k);
    TuneRec rec;
    if (tune_variants<R>(op, which, X, ldx, Y, ldy, k, U, s, rec)) g_tune[key] = rec;
    return rec.best;
}

sc_status wilson_tune_pin(const sc_op* op, bool single, int k, int variant) {
    if (is_tmarch(variant) && !tmarch_ok(op)) {
        set_error("wilson_tune_set: the t-march shapes need an xy-plane of exactly 256 sites");
        return SC_ERR_ARG;
    }
    if (is_tx(variant) && !(single && tx_ok(op))) {
        set_error("wilson_tune_set: the DPP shapes need FP32, X = Y = 16 and |kappa| >= 1e-6");
        return SC_ERR_ARG;
    }
    TuneKey key{{op->dims[0], op->dims[1], op->dims[2], op->dims[3]}, single ? 1 : 0, k, (single && op->su3) ? 1 : 0};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (variant < 0) {
        g_tune.erase(key);
        return SC_OK;
    }
    TuneRec rec;
    rec.best = variant;
    for (int v = 0; v < WV_COUNT; ++v) rec.us[v] = -1.0f;
    g_tune[key] = rec;
    return SC_OK;
}

sc_status wilson_tune_query(const sc_op* op, bool single, int k, int* variant, float* us) {
    TuneKey key{{op->dims[0], op->dims[1], op->dims[2], op->dims[3]}, single ? 1 : 0, k, (single && op->su3) ? 1 : 0};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it == g_tune.end()) {
        *variant = -1;
        for (int v = 0; v < WV_COUNT; ++v) us[v] = -1.0f;
        return SC_OK;
    }
    *variant = it->second.best;
    for (int v = 0; v < WV_COUNT; ++v) us[v] = it->second.us[v];
    return SC_OK;
}

template <typename R>
static sc_status wilson_launch(const sc_op* op, int which, const R* X, int64_t ldx, R* Y, int64_t ldy, int k,
                               const R* U, hipStream_t s) {
    const int v = choose_variant<R>(op, which, X, ldx, Y, ldy, k, U, s);
    // algorithmic traffic of one pass: each spinor read and written once per
    // column, the 4 links of a site read once per pass; 1320 flops of hopping
    // per site and column (+48 for psi - kappa H psi)
    const double bytes = (48.0 * k + 72.0) * sizeof(R) * (double)op->vol;
    const double flops = (which < 2 ? 1368.0 : 1320.0) * k * (double)op->vol;
    const int cls = sizeof(R) == 4 ? (k == 1 ? TC_WILSON_F32 : TC_WILSON_F32_K) : (k == 1 ? TC_WILSON_F64 : TC_WILSON_F64_K);
    TimerScope ts_(cls, s, bytes, flops);
    wilson_launch_variant<R>(v, op, which, X, ldx, Y, ldy, k, U, s);
    SC_LAUNCH_CHECK();
    return SC_OK;
}

template <typename R>
static sc_status wilson_d_norm(const sc_op* op, const R* X, int64_t ldx, R* Y, int64_t ldy, int k, const R* U,
                               double* part, int max_parts, int* G, hipStream_t s) {
    *G = 0;
    const int v = choose_variant<R>(op, 0, X, ldx, Y, ldy, k, U, s);
    if constexpr (sizeof(R) == 4) {
        if (is_tx(v) && tx_ok(op) && tx_parts(op, v) <= max_parts) {
            const double bytes = (48.0 * k + 72.0) * 4.0 * (double)op->vol;
            TimerScope ts_(k == 1 ? TC_WILSON_F32 : TC_WILSON_F32_K, s, bytes, 1368.0 * k * (double)op->vol);
            TmEpi e{};
            e.part = part;
            tx_launch(op, v, false, TM_NORM, X, ldx, Y, ldy, k, U, e, s);
            SC_LAUNCH_CHECK();
            *G = tx_parts(op, v);
            return SC_OK;
        }
    }
    if (!is_tmarch(v) || !tmarch_ok(op)) return wilson_launch<R>(op, 0, X, ldx, Y, ldy, k, U, s);
    const TmShape t = tm_shape(v, sizeof(R) == 4, op->dims[2]);
    const int tlen = std::max(1, std::min(t.tlen, op->dims[3]));
    const int parts = op->dims[2] * ((op->dims[3] + tlen - 1) / tlen);
    if (parts > max_parts) return wilson_launch<R>(op, 0, X, ldx, Y, ldy, k, U, s);
    const double bytes = (48.0 * k + 72.0) * sizeof(R) * (double)op->vol;
    const int cls = sizeof(R) == 4 ? (k == 1 ? TC_WILSON_F32 : TC_WILSON_F32_K) : (k == 1 ? TC_WILSON_F64 : TC_WILSON_F64_K);
    TimerScope ts_(cls, s, bytes, 1368.0 * k * (double)op->vol);
    TmEpi e{};
    e.part = part;
    tm_launch<R>(op, 0, X, ldx, Y, ldy, k, U, t, TM_NORM, e, s);
    SC_LAUNCH_CHECK();
    *G = parts;
    return SC_OK;
}

template <typename R>
static sc_status wilson_cg_fused_t(const sc_op* op, const R* p, R* tmp, int k, const R* U, const CGCol* st,
                                   double* part_pq, R* r, int64_t ldr, double* part_rr, int max_parts, int* G,
                                   hipStream_t s) {
    *G = 0;
    // the t-march shapes (partials per plane and segment) and the tiled ones
    // (partials per 256-site tile); the direction-split shape has no epilogues
    const int v = choose_variant<R>(op, 0, p, op->n, tmp, op->n, k, U, s);
    if constexpr (sizeof(R) == 4) {
        if (is_tx(v) && tx_ok(op)) {
            const int parts = tx_parts(op, v);
            if (parts > max_parts) return SC_OK;
            const int cls = k == 1 ? TC_WILSON_F32 : TC_WILSON_F32_K;
            {
                TimerScope ts_(cls, s, (48.0 * k + 72.0) * 4.0 * (double)op->vol, 1368.0 * k * (double)op->vol);
                TmEpi e{};
                e.part = part_pq;
                e.st = st;  // columns no longer active are skipped
                tx_launch(op, v, false, TM_NORM, p, op->n, tmp, op->n, k, U, e, s);
                SC_LAUNCH_CHECK();
            }
            {
                TimerScope ts_(cls, s, (72.0 * k + 72.0) * 4.0 * (double)op->vol, 1368.0 * k * (double)op->vol);
                TmEpi e{};
                e.part = part_rr;
                e.st = st;
                e.pq = part_pq;
                e.r = r;
                e.ldr = 2 * ldr;
                tx_launch(op, v, true, TM_CG, tmp, op->n, tmp, op->n, k, U, e, s);
                SC_LAUNCH_CHECK();
            }
            *G = parts;
            return SC_OK;
        }
    }
    const bool tm = is_tmarch(v) && tmarch_ok(op);
    if (!tm && (v == WV_DIR || is_tmarch(v))) return SC_OK;
    TmShape t{};
    int parts;
    if (tm) {
        t = tm_shape(v, sizeof(R) == 4, op->dims[2]);
        const int tlen = std::max(1, std::min(t.tlen, op->dims[3]));
        parts = op->dims[2] * ((op->dims[3] + tlen - 1) / tlen);
    } else {
        parts = (int)((op->vol + kBlock - 1) / kBlock);
    }
    if (parts > max_parts) return SC_OK;
    const double bytes = (48.0 * k + 72.0) * sizeof(R) * (double)op->vol;
    const int cls = sizeof(R) == 4 ? (k == 1 ? TC_WILSON_F32 : TC_WILSON_F32_K) : (k == 1 ? TC_WILSON_F64 : TC_WILSON_F64_K);
    {
        TimerScope ts_(cls, s, bytes, 1368.0 * k * (double)op->vol);
        TmEpi e{};
        e.part = part_pq;
        if (tm)
            tm_launch<R>(op, 0, p, op->n, tmp, op->n, k, U, t, TM_NORM, e, s);
        else
            wilson_launch_variant_epi<R>(v, op, TM_NORM, p, op->n, tmp, op->n, k, U, e, s);
        SC_LAUNCH_CHECK();
    }
    {
        // D^H pass: reads tmp, reads and writes r (A p is not stored): 72k + 72 reals per site
        TimerScope ts_(cls, s, (72.0 * k + 72.0) * sizeof(R) * (double)op->vol, 1368.0 * k * (double)op->vol);
        TmEpi e{};
        e.part = part_rr;
        e.st = st;
        e.pq = part_pq;
        e.r = r;
        e.ldr = 2 * ldr;
        if (tm)
            tm_launch<R>(op, 1, tmp, op->n, tmp, op->n, k, U, t, TM_CG, e, s);
        else
            wilson_launch_variant_epi<R>(v, op, TM_CG, tmp, op->n, tmp, op->n, k, U, e, s);
        SC_LAUNCH_CHECK();
    }
    *G = parts;
    return SC_OK;
}

sc_status wilson_cg_fused(const sc_op* op, bool single, const void* p, void* tmp, int k, const CGCol* st,
                          double* part_pq, void* r, int64_t ldr, double* part_rr, int max_parts, int* G,
                          hipStream_t s) {
    *G = 0;
    if (op->kind != SC_OPK_WILSON || k <= 0) return SC_OK;
    if (single) {
        if (!op->U32) return SC_OK;
        return wilson_cg_fused_t<float>(op, (const float*)p, (float*)tmp, k, (const float*)op->U32, st, part_pq,
                                        (float*)r, ldr, part_rr, max_parts, G, s);
    }
    return wilson_cg_fused_t<double>(op, (const double*)p, (double*)tmp, k, (const double*)op->U64, st, part_pq,
                                     (double*)r, ldr, part_rr, max_parts, G, s);
}

sc_status op_apply_norm(const sc_op* op, bool single, const void* X, int64_t ldx, void* Y, int64_t ldy, int k,
                        void* tmp, double* part, int max_parts, int* G, hipStream_t s) {
    *G = 0;
    if (k <= 0) return SC_OK;
    if (op->kind != SC_OPK_WILSON) return op_apply(op, single, X, ldx, Y, ldy, k, tmp, s);
    if (single) {
        if (!op->U32) {
            set_error("single-precision Wilson apply needs U32 links");
            return SC_ERR_ARG;
        }
        SC_TRY(wilson_d_norm<float>(op, (const float*)X, ldx, (float*)tmp, op->n, k, (const float*)op->U32, part,
                                    max_parts, G, s));
    } else {
        SC_TRY(wilson_d_norm<double>(op, (const double*)X, ldx, (double*)tmp, op->n, k, (const double*)op->U64, part,
                                     max_parts, G, s));
    }
    return wilson_pass(op, single, 1, tmp, op->n, Y, ldy, k, s);
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

// gamma_5 = diag(1, 1, -1, -1) in spin: in the component-major layout the
// lower two spins are components 6..11, the second half of each column
template <typename R>
__global__ __launch_bounds__(kBlock) void k_gamma5(R* __restrict__ y, int64_t ldy, int64_t half) {
    R* c = y + blockIdx.y * ldy + half;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < half; i += (int64_t)gridDim.x * kBlock) c[i] = -c[i];
}

sc_status op_apply(const sc_op* op, bool single, const void* X, int64_t ldx, void* Y, int64_t ldy, int k, void* tmp,
                   hipStream_t s) {
    if (k <= 0) return SC_OK;
    if (op->kind == SC_OPK_WILSON) {
        SC_TRY(wilson_pass(op, single, 0, X, ldx, tmp, op->n, k, s));
        return wilson_pass(op, single, 1, tmp, op->n, Y, ldy, k, s);
    }
    if (op->kind == SC_OPK_WILSON_G5) {  // Q = gamma_5 D: one D pass, then the sign of the lower spins
        SC_TRY(wilson_pass(op, single, 0, X, ldx, Y, ldy, k, s));
        const int64_t half = 12 * op->vol;  // reals: 6 complex components of V sites
        const dim3 grid((unsigned)std::min<int64_t>((half + kBlock - 1) / kBlock, 1024), (unsigned)k);
        if (single) hipLaunchKernelGGL(k_gamma5<float>, grid, dim3(kBlock), 0, s, (float*)Y, 2 * ldy, half);
        else hipLaunchKernelGGL(k_gamma5<double>, grid, dim3(kBlock), 0, s, (double*)Y, 2 * ldy, half);
        SC_LAUNCH_CHECK();
        return SC_OK;
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
