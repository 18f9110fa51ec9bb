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
#include <cstdlib>
#include <map>
#include <mutex>

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

template <typename R>
__device__ __forceinline__ void load_link(const R* __restrict__ U, unsigned V, int mu, unsigned site, cplx<R> u[3][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) u[a][b] = ldc(U + 2 * (size_t)(((mu * 3 + a) * 3 + b) * V), site);
}

// Block -> work mapping.  Workgroups are dispatched round-robin over the 8
// XCDs (block b runs on XCD b % 8), each with its own L2.  Logical work item
// L = (b % 8) * per_xcd + b / 8 gives every XCD a contiguous range of L.  In
// tile-major order the column groups of one site tile are consecutive in L
// (a tile's links are reused from L2); in column-major order one column group
// sweeps the whole lattice before the next, so the t-neighbour slices of that
// group stay in L2 even when all k columns together exceed the caches (the
// links are then re-read once per group, from the 256 MB infinity cache).
constexpr int kXcd = 8;

// MODE 0: out = in - kappa * H in (D or D^H);  MODE 1: out = H in (or H^H in).
// NC columns per thread: each link is loaded once and applied to NC spinors.
template <typename R, bool DAG, int MODE, int NC, int MINW, bool BAR = false, bool COLMAJOR = false>
__global__ __launch_bounds__(kBlock, MINW) void k_wilson(R* __restrict__ out, int64_t ldo, const R* __restrict__ in,
                                                   int64_t ldi, const R* __restrict__ U, Geom g, R kappa, R tsign,
                                                   int k, int ncg, int ntiles, int per_xcd) {
    const int b = blockIdx.x;
    const int L = (b % kXcd) * per_xcd + b / kXcd;
    if (L >= ntiles * ncg) return;
    const int tile = COLMAJOR ? L % ntiles : L / ncg;
    const int c0 = (COLMAJOR ? L / ntiles : L % ncg) * NC;
    const int s = tile * kBlock + threadIdx.x;
    const int V = (int)g.V;
    if (s >= V) return;
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
        hop<MU, SF, false>(acc[c], psi, u, MU == 3 ? bf_p : R(1));           \
        if (BAR) asm volatile("" ::: "memory");                              \
    }                                                                        \
    load_link(U, uV, MU, nb_m[MU], u);                                       \
    _Pragma("unroll") for (int c = 0; c < NC; ++c) {                         \
        load_spinor(src[c], uV, nb_m[MU], psi);                              \
        hop<MU, SB, true>(acc[c], psi, u, MU == 3 ? bf_m : R(1));            \
        if (BAR) asm volatile("" ::: "memory");                              \
    }
    SC_WILSON_DIR(0)
    SC_WILSON_DIR(1)
    SC_WILSON_DIR(2)
    SC_WILSON_DIR(3)
#undef SC_WILSON_DIR

#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (!live[c]) continue;
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
                reinterpret_cast<typename vec2<R>::type*>(dst + cb)[us] = typename vec2<R>::type{r.re, r.im};
            }
    }
}

// Rolled variant: a runtime loop over the 8 hops with a wave-uniform switch.
// Only one hop's operands are live at a time (low register use, high
// occupancy); the latency of a hop's loads is hidden by the other waves.
template <typename R, bool DAG, int MODE, int NC, int MINW, bool COLMAJOR = false>
__global__ __launch_bounds__(kBlock, MINW) void k_wilson_r(R* __restrict__ out, int64_t ldo, const R* __restrict__ in,
                                                         int64_t ldi, const R* __restrict__ U, Geom g, R kappa,
                                                         R tsign, int k, int ncg, int ntiles, int per_xcd) {
    const int b = blockIdx.x;
    const int L = (b % kXcd) * per_xcd + b / kXcd;
    if (L >= ntiles * ncg) return;
    const int tile = COLMAJOR ? L % ntiles : L / ncg;
    const int c0 = (COLMAJOR ? L / ntiles : L % ncg) * NC;
    const int s = tile * kBlock + threadIdx.x;
    const int V = (int)g.V;
    if (s >= V) return;
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
        if (!live[c]) continue;
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
                reinterpret_cast<typename vec2<R>::type*>(dst + cb)[us] = typename vec2<R>::type{r.re, r.im};
            }
    }
}

// ---------------------------------------------------------------- launchers
// ---------------------------------------------------------------- variants and autotuning
// Candidate launch shapes of a stencil pass (columns per thread x loop form).
enum WilsonVariant {
    WV_UNROLLED_1 = 0,
    WV_ROLLED_1 = 1,
    WV_ROLLED_2 = 2,
    WV_ROLLED_4 = 3,
    WV_ROLLED_1_CM = 4,
    WV_ROLLED_2_CM = 5,
    WV_ROLLED_4_CM = 6,
    WV_COUNT = 7
};

template <typename R, int NC, bool ROLLED, bool CM>
static void wilson_launch_v(const sc_op* op, int which, const R* X, int64_t ldx, R* Y, int64_t ldy, int k, const R* U,
                            hipStream_t s) {
    Geom g{op->dims[0], op->dims[1], op->dims[2], op->dims[3], op->vol};
    const int ntiles = (int)((g.V + kBlock - 1) / kBlock);
    const int ncg = (k + NC - 1) / NC;
    const int per_xcd = (ntiles * ncg + kXcd - 1) / kXcd;
    dim3 grid((unsigned)(per_xcd * kXcd));
    const R kap = (R)op->kappa;
    const R ts = op->antiperiodic ? R(-1) : R(1);
    // ld arguments are in reals (2 per complex element)
#define SC_WL(DAG, MODE)                                                                                       \
    if (ROLLED)                                                                                                \
        hipLaunchKernelGGL((k_wilson_r<R, DAG, MODE, NC, 1, CM>), grid, dim3(kBlock), 0, s, Y, 2 * ldy, X,     \
                           2 * ldx, U, g, kap, ts, k, ncg, ntiles, per_xcd);                                   \
    else                                                                                                       \
        hipLaunchKernelGGL((k_wilson<R, DAG, MODE, NC, 1, false, CM>), grid, dim3(kBlock), 0, s, Y, 2 * ldy,   \
                           X, 2 * ldx, U, g, kap, ts, k, ncg, ntiles, per_xcd);
    switch (which) {
        case 0: SC_WL(false, 0) break;
        case 1: SC_WL(true, 0) break;
        case 2: SC_WL(false, 1) break;
        default: SC_WL(true, 1) break;
    }
#undef SC_WL
}

// FP64 has no 4-column shape (it would spill): those ids fall back to 2 columns
template <typename R>
static void wilson_launch_variant(int v, const sc_op* op, int which, const R* X, int64_t ldx, R* Y, int64_t ldy, int k,
                                  const R* U, hipStream_t s) {
    constexpr int N4 = sizeof(R) == 4 ? 4 : 2;
    switch (v) {
        case WV_UNROLLED_1: wilson_launch_v<R, 1, false, false>(op, which, X, ldx, Y, ldy, k, U, s); break;
        case WV_ROLLED_1: wilson_launch_v<R, 1, true, false>(op, which, X, ldx, Y, ldy, k, U, s); break;
        case WV_ROLLED_2: wilson_launch_v<R, 2, true, false>(op, which, X, ldx, Y, ldy, k, U, s); break;
        case WV_ROLLED_4: wilson_launch_v<R, N4, true, false>(op, which, X, ldx, Y, ldy, k, U, s); break;
        case WV_ROLLED_1_CM: wilson_launch_v<R, 1, true, true>(op, which, X, ldx, Y, ldy, k, U, s); break;
        case WV_ROLLED_2_CM: wilson_launch_v<R, 2, true, true>(op, which, X, ldx, Y, ldy, k, U, s); break;
        default: wilson_launch_v<R, N4, true, true>(op, which, X, ldx, Y, ldy, k, U, s); break;
    }
}

namespace {
struct TuneKey {
    int dims[4];
    int single, k;
    bool operator<(const TuneKey& o) const {
        for (int i = 0; i < 4; ++i)
            if (dims[i] != o.dims[i]) return dims[i] < o.dims[i];
        if (single != o.single) return single < o.single;
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

int default_variant(bool single, int k) { return k <= 1 ? WV_ROLLED_1 : (single ? WV_ROLLED_2 : WV_ROLLED_1); }
}  // namespace

// Time every variant on the caller's buffers (the output is rewritten by the
// real launch that follows) and keep the fastest for (lattice, precision, k).
template <typename R>
static TuneRec tune_variants(const sc_op* op, int which, const R* X, int64_t ldx, R* Y, int64_t ldy, int k, const R* U,
                             hipStream_t s) {
    TuneRec rec;
    rec.best = default_variant(sizeof(R) == 4, k);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return rec;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return rec;
    }
    float best = 1e30f;
    for (int v = 0; v < WV_COUNT; ++v) {
        rec.us[v] = -1.0f;
        if (sizeof(R) == 8 && (v == WV_ROLLED_4 || v == WV_ROLLED_4_CM)) continue;  // FP64 has no 4-column shape
        if (k == 1 && v >= WV_ROLLED_1_CM) continue;  // order is irrelevant for one column
        wilson_launch_variant<R>(v, op, which, X, ldx, Y, ldy, k, U, s);  // warm
        hipEventRecord(e0, s);
        for (int r = 0; r < 3; ++r) wilson_launch_variant<R>(v, op, which, X, ldx, Y, ldy, k, U, s);
        hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) break;
        float ms = 0.0f;
        hipEventElapsedTime(&ms, e0, e1);
        rec.us[v] = ms * 1000.0f / 3.0f;
        if (rec.us[v] < best) {
            best = rec.us[v];
            rec.best = v;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return rec;
}

template <typename R>
static int choose_variant(const sc_op* op, int which, const R* X, int64_t ldx, R* Y, int64_t ldy, int k, const R* U,
                          hipStream_t s) {
    TuneKey key{{op->dims[0], op->dims[1], op->dims[2], op->dims[3]}, sizeof(R) == 4 ? 1 : 0, k};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second.best;
    if (g_tune_mode < 0) {
        const char* e = getenv("SEEDCG_TUNE");
        g_tune_mode = (e && e[0] == '0') ? 0 : 1;
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipStreamIsCapturing(s, &cs);
    if (g_tune_mode == 0 || cs != hipStreamCaptureStatusNone) return default_variant(sizeof(R) == 4, k);
    TuneRec rec = tune_variants<R>(op, which, X, ldx, Y, ldy, k, U, s);
    g_tune[key] = rec;
    return rec.best;
}

sc_status wilson_tune_pin(const sc_op* op, bool single, int k, int variant) {
    TuneKey key{{op->dims[0], op->dims[1], op->dims[2], op->dims[3]}, single ? 1 : 0, k};
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
    TuneKey key{{op->dims[0], op->dims[1], op->dims[2], op->dims[3]}, single ? 1 : 0, k};
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
    TimerScope ts_(sizeof(R) == 4 ? TC_WILSON_F32 : TC_WILSON_F64, s, bytes, flops);
    wilson_launch_variant<R>(v, op, which, X, ldx, Y, ldy, k, U, s);
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
