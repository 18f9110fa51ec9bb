// Tall-skinny contractions with the stored Lanczos basis and the solve with the
// Lanczos tridiagonal matrix.
//
//   gemm_cn:  G = V^H W   (V: n x M basis, W: N <= 32 columns, G: M x N FP64)
//             used by step 8 (coefficients of v_i and f on v_1..v_{i-1}) and by
//             the projection (V^H R0).  Split over row chunks; each block
//             stages a KT x TM tile of V and a KT x N tile of W in LDS and
//             accumulates in FP64; the chunk partials are then added in chunk
//             order by a second kernel, so the result is deterministic.
//   gemm_nn:  X_j += scale * V Y_j  (thread per row, Y staged in LDS).
//   tridiag:  Y <- T^{-1} Y with T = L U, the factorization of the seed
//             algorithm's step 6 (pivots delta_i, multipliers gamma_{i-1}).
#include "sc_internal.h"
#include "sc_timer.h"

namespace sc {

template <typename R, bool CPLX>
__device__ __forceinline__ cplx<double> ld_elem(const R* p, int64_t idx) {
    if constexpr (CPLX) {
        cplx<R> c = ld2(p, idx);
        return {(double)c.re, (double)c.im};
    } else {
        return {(double)p[idx], 0.0};
    }
}

// ---------------------------------------------------------------- FP64 MFMA versions (complex)
// v_mfma_f64_16x16x4f64: D(16x16) += A(16x4) B(4x16); lane l supplies
// A[l%16][l/16] and B[l/16][l%16] and holds D[l/16 + 4v][l%16] in register v.
// A complex product is four real ones on the real and imaginary parts.
typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The complex right-hand block enters the MFMAs as one real matrix of 2N
// columns, [Re W | Im W] (padded with zeros to 16 NT columns, NT = ceil(N/8)),
// multiplied once by Re V and once by Im V: P = Re(V)^T [Re W | Im W] and
// Q = Im(V)^T [Re W | Im W].  The complex result is then
//   Re(V^H W)_j = P_j + Q_{N+j},  Im(V^H W)_j = P_{N+j} - Q_j,
//   Re(V Y)_j   = P_j - Q_{N+j},  Im(V Y)_j   = P_{N+j} + Q_j,
// which takes 2 NT MFMAs per 4-row step where four products per 16-column
// complex tile would take 8 ceil(N/16) (N = 23: 6 against 8).  Q is passed
// through LDS in the epilogue so that each lane holds one P and the Q it is
// combined with.

// G = V^H W: block = 4 waves over 64 basis columns (16 per wave), one row
// chunk; LDS stages of KR = 64 complex rows (measured 8% faster than 32 on
// the projection of the benchmark workload; the X += V Y kernel below keeps
// 32-column stages, which measured faster there).  The stages are software-pipelined:
// each thread holds its share of the next stage's V and W elements in
// registers, loaded before the current stage's MFMAs are issued and written to
// LDS after them, so the global-load latency of a stage hides behind the
// previous stage's compute.  V stays in its own precision in LDS and is
// widened when it is fed to the MFMA.
template <typename VR, typename WR, int NT, int KR = 64>
__global__ __launch_bounds__(kBlock) void k_cn_mfma(const VR* __restrict__ V, int64_t ldv, int64_t n, int M,
                                                    ColPtrs<const void> W, int N, double* __restrict__ part,
                                                    int64_t rows_per_chunk, int nchunk, const int* halt) {
    if (halt && *halt) return;
    constexpr int TA = 64;               // basis columns per block
    constexpr int TC = 16 * NT;          // real columns of [Re W | Im W], padded
    constexpr int EV = KR * TA / kBlock; // V elements per thread per stage
    constexpr int EW = (KR * TC / 2 + kBlock - 1) / kBlock;  // complex W elements per thread per stage
    union Lds {
        struct {
            VR vr[KR][TA + 1], vi[KR][TA + 1];
            double wb[KR][TC + 1];
        } st;
        double qs[TA][TC + 1];
    };
    __shared__ Lds lds;
    // work item L = (b % 8) * per_xcd + b / 8 over (row chunk, column block),
    // column blocks fastest: the blocks that read one chunk of W run together
    // on one XCD and share it through its L2
    const int mblk = (M + TA - 1) / TA;
    const int per_xcd = (nchunk * mblk + kXcd - 1) / kXcd;
    const int L = (blockIdx.x % kXcd) * per_xcd + blockIdx.x / kXcd;
    if (L >= nchunk * mblk) return;
    const int chunk = L / mblk;
    const int a0 = (L % mblk) * TA;
    const int64_t r0 = chunk * rows_per_chunk;
    const int64_t r1 = min(n, r0 + rows_per_chunk);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    d4_t accp[NT], accq[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) accp[t] = accq[t] = d4_t{0.0, 0.0, 0.0, 0.0};
    // columns 2N .. TC of the staged W block stay zero
    for (int e = threadIdx.x; e < KR * (TC + 1); e += kBlock) {
        const int c = e % (TC + 1);
        if (c >= 2 * N) lds.st.wb[e / (TC + 1)][c] = 0.0;
    }
    cplx<VR> pv[EV];
    cplx<double> pw[EW];
    // the W column each of the thread's W elements comes from is the same in
    // every stage: its pointer is read once here, not (with a wait) in every
    // stage's fetch
    const WR* wcol[EW];
#pragma unroll
    for (int q = 0; q < EW; ++q) {
        const int jj = (threadIdx.x + q * kBlock) / KR;
        wcol[q] = (const WR*)W.p[jj < N ? jj : 0];
    }
    // element e of a stage: V row e % KR of column e / KR; W row e % KR of complex column e / KR
    auto fetch = [&](int64_t rb) {
#pragma unroll
        for (int q = 0; q < EV; ++q) {
            const int e = threadIdx.x + q * kBlock;
            const int64_t r = rb + e % KR;
            const int a = a0 + e / KR;
            pv[q] = (r < r1 && a < M) ? ld2(V, (int64_t)a * ldv + r) : cplx<VR>{VR(0), VR(0)};
        }
#pragma unroll
        for (int q = 0; q < EW; ++q) {
            const int e = threadIdx.x + q * kBlock;
            const int64_t r = rb + e % KR;
            const int jj = e / KR;
            cplx<double> w{0.0, 0.0};
            if (r < r1 && jj < N) {
                const cplx<WR> c = ld2(wcol[q], r);
                w = {(double)c.re, (double)c.im};
            }
            pw[q] = w;
        }
    };
    if (r0 < r1) fetch(r0);
    for (int64_t rb = r0; rb < r1; rb += KR) {
        __syncthreads();  // the previous stage's MFMAs are done with the LDS tiles
#pragma unroll
        for (int q = 0; q < EV; ++q) {
            const int e = threadIdx.x + q * kBlock;
            lds.st.vr[e % KR][e / KR] = pv[q].re;
            lds.st.vi[e % KR][e / KR] = pv[q].im;
        }
#pragma unroll
        for (int q = 0; q < EW; ++q) {
            const int e = threadIdx.x + q * kBlock;
            const int jj = e / KR;
            if (jj < N) {
                lds.st.wb[e % KR][jj] = pw[q].re;
                lds.st.wb[e % KR][N + jj] = pw[q].im;
            }
        }
        __syncthreads();
        if (rb + KR < r1) fetch(rb + KR);  // in flight during this stage's MFMAs
#pragma unroll
        for (int ks = 0; ks < KR / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            const double ar = (double)lds.st.vr[kr][wv * 16 + (lane & 15)];
            const double ai = (double)lds.st.vi[kr][wv * 16 + (lane & 15)];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double bw = lds.st.wb[kr][t * 16 + (lane & 15)];
                accp[t] = mfma16(ar, bw, accp[t]);
                accq[t] = mfma16(ai, bw, accq[t]);
            }
        }
    }
    __syncthreads();  // the staging tiles are reused for Q
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) lds.qs[wv * 16 + (lane >> 4) + 4 * v][t * 16 + (lane & 15)] = accq[t][v];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = t * 16 + (lane & 15);
        if (c >= 2 * N) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int al = wv * 16 + (lane >> 4) + 4 * v;
            const int a = a0 + al;
            if (a >= M) continue;
            if (c < N) {  // Re G_{a,c}
                part[2 * (((int64_t)chunk * M + a) * N + c)] = accp[t][v] + lds.qs[al][N + c];
            } else {      // Im G_{a,c-N}
                part[2 * (((int64_t)chunk * M + a) * N + (c - N)) + 1] = accp[t][v] - lds.qs[al][c - N];
            }
        }
    }
}

// X_j += scale * V Y_j: block = 4 waves over 64 rows (16 per wave); LDS
// stages of 32 basis columns, software-pipelined like k_cn_mfma.
template <typename VR, typename XR, int NT, int KA = 32>
__global__ __launch_bounds__(kBlock) void k_nn_mfma(const VR* __restrict__ V, int64_t ldv, int64_t n, int M,
                                                    const double* __restrict__ Y, int N, ColPtrs<void> X,
                                                    double scale, const int* halt) {
    if (halt && *halt) return;
    constexpr int TR = 64;          // rows per block
    constexpr int TC = 16 * NT;     // real columns of [Re Y | Im Y], padded
    constexpr int EV = TR * KA / kBlock;
    constexpr int EY = (KA * TC / 2 + kBlock - 1) / kBlock;  // complex Y elements per thread per stage
    union Lds {
        struct {
            VR vr[TR][KA + 1], vi[TR][KA + 1];
            double yb[KA][TC + 1];
        } st;
        double qs[TR][TC + 1];
    };
    __shared__ Lds lds;
    const int64_t row0 = (int64_t)blockIdx.x * TR;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    d4_t accp[NT], accq[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) accp[t] = accq[t] = d4_t{0.0, 0.0, 0.0, 0.0};
    for (int e = threadIdx.x; e < KA * (TC + 1); e += kBlock) {
        const int c = e % (TC + 1);
        if (c >= 2 * N) lds.st.yb[e / (TC + 1)][c] = 0.0;
    }
    cplx<VR> pv[EV];
    cplx<double> py[EY];
    constexpr int YJ = TC / 2;  // complex Y columns a stage covers (>= N)
    // element e: V row e % TR of basis column e / TR; Y basis column e / YJ, right-hand column e % YJ
    auto fetch = [&](int ab) {
#pragma unroll
        for (int q = 0; q < EV; ++q) {
            const int e = threadIdx.x + q * kBlock;
            const int64_t r = row0 + e % TR;
            const int a = ab + e / TR;
            pv[q] = (r < n && a < M) ? ld2(V, (int64_t)a * ldv + r) : cplx<VR>{VR(0), VR(0)};
        }
#pragma unroll
        for (int q = 0; q < EY; ++q) {
            const int e = threadIdx.x + q * kBlock;
            const int a = ab + e / YJ, jj = e % YJ;
            py[q] = (e < KA * YJ && a < M && jj < N)
                        ? cplx<double>{Y[((int64_t)a * N + jj) * 2], Y[((int64_t)a * N + jj) * 2 + 1]}
                        : cplx<double>{0.0, 0.0};
        }
    };
    if (M > 0) fetch(0);
    for (int ab = 0; ab < M; ab += KA) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < EV; ++q) {
            const int e = threadIdx.x + q * kBlock;
            lds.st.vr[e % TR][e / TR] = pv[q].re;
            lds.st.vi[e % TR][e / TR] = pv[q].im;
        }
#pragma unroll
        for (int q = 0; q < EY; ++q) {
            const int e = threadIdx.x + q * kBlock;
            const int jj = e % YJ;
            if (e < KA * YJ && jj < N) {
                lds.st.yb[e / YJ][jj] = py[q].re;
                lds.st.yb[e / YJ][N + jj] = py[q].im;
            }
        }
        __syncthreads();
        if (ab + KA < M) fetch(ab + KA);
#pragma unroll
        for (int ks = 0; ks < KA / 4; ++ks) {
            const int ka = ks * 4 + (lane >> 4);
            const double ar = (double)lds.st.vr[wv * 16 + (lane & 15)][ka];
            const double ai = (double)lds.st.vi[wv * 16 + (lane & 15)][ka];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double by = lds.st.yb[ka][t * 16 + (lane & 15)];
                accp[t] = mfma16(ar, by, accp[t]);
                accq[t] = mfma16(ai, by, accq[t]);
            }
        }
    }
    __syncthreads();  // the staging tiles are reused for Q
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) lds.qs[wv * 16 + (lane >> 4) + 4 * v][t * 16 + (lane & 15)] = accq[t][v];
    __syncthreads();
    // every X element this lane updates is loaded (at clamped rows and
    // columns, so unconditionally) before any is stored: the output columns
    // are distinct, so no store changes a value loaded here, and the loads are
    // one round trip instead of one per element
    XR* xp[NT];
    XR xo[NT][4];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = min(t * 16 + (lane & 15), 2 * N - 1);
        const bool re = c < N;
        xp[t] = (XR*)X.p[re ? c : c - N] + (re ? 0 : 1);
#pragma unroll
        for (int v = 0; v < 4; ++v) xo[t][v] = xp[t][2 * min(row0 + wv * 16 + (lane >> 4) + 4 * v, n - 1)];
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int c = t * 16 + (lane & 15);
        if (c >= 2 * N) continue;
        const bool re = c < N;
        const int j = re ? c : c - N;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rl = wv * 16 + (lane >> 4) + 4 * v;
            const int64_t r = row0 + rl;
            if (r < n) {
                const double d = re ? accp[t][v] - lds.qs[rl][N + c] : accp[t][v] + lds.qs[rl][j];
                xp[t][2 * r] = (XR)((double)xo[t][v] + scale * d);
            }
        }
    }
}

// ---------------------------------------------------------------- G = V^H W, N <= 2 (reorthogonalization)
// Bandwidth kernel: a block owns a range of rows, in sub-chunks of
// kBlock * kSmallRPT rows, and 64 basis columns.  Per sub-chunk each thread
// holds its kSmallRPT rows of the (at most two) W columns in registers and
// streams the basis columns: all loads of a column are issued before they are
// used and the next column's loads are issued before the current column is
// reduced.  The four sums of a column (re, im for two W columns) are reduced
// over the wave by a reduce-scatter (7 exchanges instead of 24) and added to a
// block-private LDS slot; one partial per block and output is written at the
// end.  Rows past n are read from row n - 1 with a zero weight, so no lane
// branches.
constexpr int kSmallRPT = 8;     // rows per thread per sub-chunk
constexpr int kSmallCols = 64;   // basis columns per block
constexpr int kSmallSub = kBlock * kSmallRPT;

// v0..v3: this lane's four partial sums.  On return lanes 0, 16, 32, 48 hold
// the wave totals of sums 0, 1, 2, 3 (lane l: sum 2 * (l >= 32) + ((l >> 4) & 1)).
__device__ __forceinline__ double reduce_scatter4(double v0, double v1, double v2, double v3) {
    const int lane = threadIdx.x & 63;
    const bool hi32 = lane >= 32;
    // step 1 (xor 32): keep sums {2, 3} on the upper half, {0, 1} on the lower
    const double s0 = hi32 ? v0 : v2, s1 = hi32 ? v1 : v3;  // what the partner keeps
    const double k0 = hi32 ? v2 : v0, k1 = hi32 ? v3 : v1;
    const double a = k0 + __shfl_xor(s0, 32, 64);
    const double b = k1 + __shfl_xor(s1, 32, 64);
    // step 2 (xor 16): keep the second of the pair on odd 16-lane groups
    const bool hi16 = (lane >> 4) & 1;
    double t = (hi16 ? b : a) + __shfl_xor(hi16 ? a : b, 16, 64);
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    return t;
}

template <typename VR, typename WR>
__global__ __launch_bounds__(kBlock) void k_cn_small(const VR* __restrict__ V, int64_t ldv, int64_t n, int M,
                                                     ColPtrs<const void> W, int N, double* __restrict__ part,
                                                     int64_t rows_per_block, const int* halt) {
    if (halt && *halt) return;
    __shared__ double red[kSmallCols][kWaves][4];
    const int a0 = blockIdx.y * kSmallCols;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int na = min(kSmallCols, M - a0);
    for (int e = threadIdx.x; e < kSmallCols * kWaves * 4; e += kBlock) (&red[0][0][0])[e] = 0.0;
    __syncthreads();
    const int64_t rb0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t rb1 = min(n, rb0 + rows_per_block);
    const WR* W0 = (const WR*)W.p[0];
    const WR* W1 = (const WR*)W.p[N > 1 ? 1 : 0];
    const double w1on = N > 1 ? 1.0 : 0.0;
    for (int64_t rbase = rb0; rbase < rb1; rbase += kSmallSub) {
        int64_t rr[kSmallRPT];
        cplx<double> w0[kSmallRPT], w1[kSmallRPT];
#pragma unroll
        for (int t = 0; t < kSmallRPT; ++t) {
            const int64_t r = rbase + threadIdx.x + (int64_t)t * kBlock;
            const double on = r < rb1 ? 1.0 : 0.0;
            rr[t] = r < rb1 ? r : rb1 - 1;
            const cplx<WR> c0 = ld2(W0, rr[t]);
            const cplx<WR> c1 = ld2(W1, rr[t]);
            w0[t] = {on * (double)c0.re, on * (double)c0.im};
            w1[t] = {on * w1on * (double)c1.re, on * w1on * (double)c1.im};
        }
        cplx<VR> vb[kSmallRPT], vn[kSmallRPT];
#pragma unroll
        for (int t = 0; t < kSmallRPT; ++t) vb[t] = ld2(V + 2 * ((int64_t)a0 * ldv), rr[t]);
        for (int aa = 0; aa < na; ++aa) {
            const int an = aa + 1 < na ? aa + 1 : aa;  // prefetch the next column
#pragma unroll
            for (int t = 0; t < kSmallRPT; ++t) vn[t] = ld2(V + 2 * ((int64_t)(a0 + an) * ldv), rr[t]);
            double s0r = 0.0, s0i = 0.0, s1r = 0.0, s1i = 0.0;
#pragma unroll
            for (int t = 0; t < kSmallRPT; ++t) {
                const double vr = (double)vb[t].re, vi = (double)vb[t].im;
                s0r += vr * w0[t].re + vi * w0[t].im;  // conj(v) w
                s0i += vr * w0[t].im - vi * w0[t].re;
                s1r += vr * w1[t].re + vi * w1[t].im;
                s1i += vr * w1[t].im - vi * w1[t].re;
            }
            const double tot = reduce_scatter4(s0r, s0i, s1r, s1i);
            if ((lane & 15) == 0) red[aa][wv][lane >> 4] += tot;
#pragma unroll
            for (int t = 0; t < kSmallRPT; ++t) vb[t] = vn[t];
        }
    }
    __syncthreads();
    // one partial per (block, column, output), summed over the waves in order
    for (int e = threadIdx.x; e < na * 2 * N; e += kBlock) {
        const int aa = e / (2 * N), q = e % (2 * N);
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) v += red[aa][w][q];
        const int j = q >> 1;
        const int64_t o = ((int64_t)blockIdx.x * M + a0 + aa) * N + j;
        part[2 * o + (q & 1)] = v;
    }
}

// ---------------------------------------------------------------- G = V^H W
// TM basis columns per block, G_ = 256/TM thread groups, QN W-columns per thread.
template <typename VR, typename WR, bool CPLX, int TM, int QN, int KT>
__global__ __launch_bounds__(kBlock) void k_cn_partial(const VR* __restrict__ V, int64_t ldv, int64_t n, int M,
                                                       ColPtrs<const void> W, int N, double* __restrict__ part,
                                                       int64_t rows_per_chunk, const int* halt) {
    if (halt && *halt) return;
    constexpr int GR = kBlock / TM;
    constexpr int NT = GR * QN;
    __shared__ cplx<double> Vs[KT][TM + 1];
    __shared__ cplx<double> Ws[KT][NT];
    const int a0 = blockIdx.y * TM;
    const int64_t r0 = blockIdx.x * rows_per_chunk;
    const int64_t r1 = min(n, r0 + rows_per_chunk);
    const int ta = threadIdx.x % TM;
    const int tg = threadIdx.x / TM;
    cplx<double> acc[QN];
#pragma unroll
    for (int q = 0; q < QN; ++q) acc[q] = {0.0, 0.0};
    for (int64_t rb = r0; rb < r1; rb += KT) {
        __syncthreads();
        for (int e = threadIdx.x; e < KT * TM; e += kBlock) {
            const int rr = e % KT, aa = e / KT;
            const int64_t r = rb + rr;
            const int a = a0 + aa;
            Vs[rr][aa] = (r < r1 && a < M) ? ld_elem<VR, CPLX>(V, (int64_t)a * ldv + r) : cplx<double>{0.0, 0.0};
        }
        for (int e = threadIdx.x; e < KT * NT; e += kBlock) {
            const int rr = e % KT, jj = e / KT;
            const int64_t r = rb + rr;
            Ws[rr][jj] = (r < r1 && jj < N) ? ld_elem<WR, CPLX>((const WR*)W.p[jj], r) : cplx<double>{0.0, 0.0};
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < KT; ++rr) {
            const cplx<double> v = Vs[rr][ta];
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                const cplx<double> w = Ws[rr][tg + GR * q];
                acc[q].re += v.re * w.re + v.im * w.im;
                acc[q].im += v.re * w.im - v.im * w.re;
            }
        }
    }
    const int a = a0 + ta;
    if (a < M) {
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int j = tg + GR * q;
            if (j < N) {
                const int64_t o = ((int64_t)blockIdx.x * M + a) * N + j;
                part[2 * o] = acc[q].re;
                part[2 * o + 1] = acc[q].im;
            }
        }
    }
}

// G[o] = sum over chunks of the partials: a block takes 64 outputs, its 4
// waves sum interleaved quarters of the chunks, and the quarters are added in
// a fixed order (deterministic).
__global__ __launch_bounds__(kBlock) void k_cn_reduce(const double* __restrict__ part, int nchunk,
                                                      int64_t nout /* doubles */, double* __restrict__ G, bool cplx,
                                                      const int* halt) {
    if (halt && *halt) return;
    __shared__ double sh[kWaves][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t o = blockIdx.x * (int64_t)64 + lane;
    // wave wv adds chunks wv, wv + 4, ...: chunk wv + 4 (8 j + u) into
    // accumulator u, so eight loads are in flight at a time (a row chunk count
    // in the hundreds would otherwise be a chain of dependent loads); the
    // accumulators are then added in a fixed order
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    if (o < nout) {
        // partials keep (re, im) pairs for a real contraction; its result is the re part
        const int64_t stride = cplx ? nout : 2 * nout;
        const double* base = part + (cplx ? o : 2 * o);
        int c = wv;
        for (; c + 7 * kWaves < nchunk; c += 8 * kWaves)
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += base[(int64_t)(c + u * kWaves) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (c + u * kWaves < nchunk) acc[u] += base[(int64_t)(c + u * kWaves) * stride];
    }
    const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    sh[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && o < nout) G[o] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}

struct CnPlan {
    int tm, kt, nchunk;
    int64_t rows;
};

// Complex contractions use the MFMA kernel (64 basis columns x 32-row stages);
// real ones the vector kernel.
static CnPlan cn_plan(int64_t n, int M, int N, bool cplx = false) {
    CnPlan p;
    if (cplx && N <= 2) {  // k_cn_small: row ranges of whole sub-chunks, enough blocks to fill the chip
        p.tm = kSmallCols;
        p.kt = kSmallSub;
        const int mt = (M + kSmallCols - 1) / kSmallCols;
        const int64_t maxchunk = std::max<int64_t>(1, (n + kSmallSub - 1) / kSmallSub);
        const int64_t want = std::min<int64_t>(maxchunk, std::max<int64_t>(64, (2048 + mt - 1) / mt));
        const int64_t subs = (maxchunk + want - 1) / want;  // sub-chunks per block
        p.rows = subs * kSmallSub;
        p.nchunk = (int)std::max<int64_t>(1, (n + p.rows - 1) / p.rows);
        return p;
    }
    p.tm = cplx ? 64 : (N <= 2 ? 128 : 32);
    p.kt = cplx ? 64 : (N <= 2 ? 16 : 64);  // the complex MFMA kernel's stage depth (KR)
    const int mt = (M + p.tm - 1) / p.tm;
    int64_t want = std::max<int64_t>(1, (2048 + mt - 1) / mt);
    const int64_t maxchunk = std::max<int64_t>(1, (n + p.kt - 1) / p.kt);
    want = std::min(want, maxchunk);
    int64_t rows = (n + want - 1) / want;
    rows = (rows + p.kt - 1) / p.kt * p.kt;
    p.rows = std::max<int64_t>(rows, p.kt);
    p.nchunk = (int)std::max<int64_t>(1, (n + p.rows - 1) / p.rows);
    return p;
}

// Partials needed by any call with M' <= M basis columns and N' <= N columns:
// the split plan gives smaller M more row chunks, so the maximum is not at M.
size_t gemm_cn_part_doubles(int64_t n, int M, int N, bool cplx) {
    size_t best = 0;
    for (int nq = 1; nq <= N; ++nq)
        for (int mm = 1; mm <= M; ++mm) {
            const CnPlan p = cn_plan(n, mm, nq, cplx);
            best = std::max(best, (size_t)p.nchunk * mm * nq * 2);
        }
    return best;
}

template <typename VR, typename WR, bool CPLX>
static void cn_launch(const CnPlan& p, const VR* V, int64_t ldv, int64_t n, int M, const ColPtrs<const void>& W, int N,
                      double* part, const int* halt, hipStream_t s) {
    dim3 grid((unsigned)p.nchunk, (unsigned)((M + p.tm - 1) / p.tm));
    if (N <= 2)
        SC_TLAUNCH((k_cn_partial<VR, WR, CPLX, 128, 1, 16>), grid, dim3(kBlock), 0, s, V, ldv, n, M, W, N, part, p.rows, halt);
    else if (N <= 8)
        SC_TLAUNCH((k_cn_partial<VR, WR, CPLX, 32, 1, 64>), grid, dim3(kBlock), 0, s, V, ldv, n, M, W, N, part, p.rows, halt);
    else
        SC_TLAUNCH((k_cn_partial<VR, WR, CPLX, 32, 4, 64>), grid, dim3(kBlock), 0, s, V, ldv, n, M, W, N, part, p.rows, halt);
}

template <typename VR, typename WR>
static void cn_mfma_launch(const CnPlan& p, const VR* V, int64_t ldv, int64_t n, int M, const ColPtrs<const void>& W,
                           int N, double* part, const int* halt, hipStream_t s) {
    dim3 grid((unsigned)p.nchunk, (unsigned)((M + 63) / 64));
    const int mblk = (M + 63) / 64;
    const int per_xcd = (p.nchunk * mblk + kXcd - 1) / kXcd;
    dim3 grid1((unsigned)(per_xcd * kXcd));
#define SC_CNT(NT_) \
    SC_TLAUNCH((k_cn_mfma<VR, WR, NT_>), grid1, dim3(kBlock), 0, s, V, ldv, n, M, W, N, part, p.rows, p.nchunk, halt)
    if (N <= 2)
        SC_TLAUNCH((k_cn_small<VR, WR>), grid, dim3(kBlock), 0, s, V, ldv, n, M, W, N, part, p.rows, halt);
    else if (N <= 8)
        SC_CNT(1);
    else if (N <= 16)
        SC_CNT(2);
    else if (N <= 24)
        SC_CNT(3);
    else
        SC_CNT(4);
#undef SC_CNT
}

sc_status gemm_cn(bool cplx, bool vsingle, const void* V, int64_t ldv, int64_t n, int M, bool wsingle,
                  const ColPtrs<const void>& W, int N, double* G, double* part, const int* halt, hipStream_t s) {
    if (M <= 0 || N <= 0) return SC_OK;
    if (N > kMaxCols) {
        set_error("gemm_cn: too many columns");
        return SC_ERR_ARG;
    }
    CnPlan p = cn_plan(n, M, N, cplx);
    const double eb = (cplx ? 2.0 : 1.0);
    TimerScope ts_(TC_GEMM_CN, s,
                   (double)n * M * eb * (vsingle ? 4 : 8) + (double)n * N * eb * (wsingle ? 4 : 8) + (double)M * N * eb * 8,
                   (cplx ? 8.0 : 2.0) * n * M * N);
#define SC_CN(VR, WR, C) cn_launch<VR, WR, C>(p, (const VR*)V, ldv, n, M, W, N, part, halt, s)
#define SC_CNM(VR, WR) cn_mfma_launch<VR, WR>(p, (const VR*)V, ldv, n, M, W, N, part, halt, s)
    if (cplx) {
        if (vsingle) { if (wsingle) SC_CNM(float, float); else SC_CNM(float, double); }
        else { if (wsingle) SC_CNM(double, float); else SC_CNM(double, double); }
    } else {
        if (vsingle) { if (wsingle) SC_CN(float, float, false); else SC_CN(float, double, false); }
        else { if (wsingle) SC_CN(double, float, false); else SC_CN(double, double, false); }
    }
#undef SC_CN
#undef SC_CNM
    SC_LAUNCH_CHECK();
    const int64_t nout = (int64_t)M * N * (cplx ? 2 : 1);
    hipLaunchKernelGGL(k_cn_reduce, dim3((unsigned)((nout + 63) / 64)), dim3(kBlock), 0, s, part,
                       p.nchunk, cplx ? nout : (int64_t)M * N, G, cplx, halt);
    SC_LAUNCH_CHECK();
    return SC_OK;
}

// ---------------------------------------------------------------- X += scale V Y
template <typename VR, typename XR, bool CPLX, int NT>
__global__ __launch_bounds__(kBlock) void k_nn(const VR* __restrict__ V, int64_t ldv, int64_t n, int M,
                                               const double* __restrict__ Y, int N, ColPtrs<void> X, double scale,
                                               const int* halt) {
    if (halt && *halt) return;
    constexpr int AC = 64;
    constexpr int W = CPLX ? 2 : 1;
    __shared__ double Ys[AC * NT * W];
    const int64_t r = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    double ar[NT], ai[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) ar[j] = ai[j] = 0.0;
    for (int a0 = 0; a0 < M; a0 += AC) {
        const int na = min(AC, M - a0);
        __syncthreads();
        for (int e = threadIdx.x; e < AC * NT * W; e += kBlock) {
            const int aa = e / (NT * W);
            const int j = (e / W) % NT;
            const int pp = e % W;
            Ys[e] = (aa < na && j < N) ? Y[((int64_t)(a0 + aa) * N + j) * W + pp] : 0.0;
        }
        __syncthreads();
        if (r < n) {
            for (int aa = 0; aa < na; ++aa) {
                const cplx<double> v = ld_elem<VR, CPLX>(V, (int64_t)(a0 + aa) * ldv + r);
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    if constexpr (CPLX) {
                        const double yr = Ys[(aa * NT + j) * 2], yi = Ys[(aa * NT + j) * 2 + 1];
                        ar[j] += v.re * yr - v.im * yi;
                        ai[j] += v.re * yi + v.im * yr;
                    } else {
                        ar[j] += v.re * Ys[aa * NT + j];
                    }
                }
            }
        }
    }
    if (r >= n) return;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        if (j < N) {
            XR* x = (XR*)X.p[j];
            if constexpr (CPLX) {
                cplx<XR> c = ld2(x, r);
                c.re = (XR)((double)c.re + scale * ar[j]);
                c.im = (XR)((double)c.im + scale * ai[j]);
                st2(x, r, c);
            } else {
                x[r] = (XR)((double)x[r] + scale * ar[j]);
            }
        }
    }
}

// X += scale V Y for complex N <= 2 (reorthogonalization): each thread owns
// kNnRPT rows, the coefficients of 64 basis columns at a time are staged in
// LDS, and per column the thread's loads are issued together, the next
// column's before the current one is used.  Rows past n read row n - 1 and
// are not written.
constexpr int kNnRPT = 8;  // 8 rows per thread: 7% faster than 4 and 2 on the 16^3 x 32 reorthogonalization

template <typename VR, typename XR>
__global__ __launch_bounds__(kBlock) void k_nn_small(const VR* __restrict__ V, int64_t ldv, int64_t n, int M,
                                                     const double* __restrict__ Y, int N, ColPtrs<void> X,
                                                     double scale, const int* halt) {
    if (halt && *halt) return;
    constexpr int AC = 64;
    __shared__ double Ys[AC * 4];  // [column][y0.re, y0.im, y1.re, y1.im]
    const int64_t r0 = (int64_t)blockIdx.x * kBlock * kNnRPT + threadIdx.x;
    int64_t rr[kNnRPT];
#pragma unroll
    for (int t = 0; t < kNnRPT; ++t) rr[t] = min(r0 + (int64_t)t * kBlock, n - 1);
    double a0r[kNnRPT], a0i[kNnRPT], a1r[kNnRPT], a1i[kNnRPT];
#pragma unroll
    for (int t = 0; t < kNnRPT; ++t) a0r[t] = a0i[t] = a1r[t] = a1i[t] = 0.0;
    for (int c0 = 0; c0 < M; c0 += AC) {
        const int na = min(AC, M - c0);
        __syncthreads();
        for (int e = threadIdx.x; e < AC * 4; e += kBlock) {
            const int aa = e >> 2, j = (e >> 1) & 1, pp = e & 1;
            Ys[e] = (aa < na && j < N) ? Y[((int64_t)(c0 + aa) * N + j) * 2 + pp] : 0.0;
        }
        __syncthreads();
        cplx<VR> vb[kNnRPT], vn[kNnRPT];
#pragma unroll
        for (int t = 0; t < kNnRPT; ++t) vb[t] = ld2(V + 2 * ((int64_t)c0 * ldv), rr[t]);
        for (int aa = 0; aa < na; ++aa) {
            const int an = aa + 1 < na ? aa + 1 : aa;
#pragma unroll
            for (int t = 0; t < kNnRPT; ++t) vn[t] = ld2(V + 2 * ((int64_t)(c0 + an) * ldv), rr[t]);
            const double y0r = Ys[aa * 4], y0i = Ys[aa * 4 + 1], y1r = Ys[aa * 4 + 2], y1i = Ys[aa * 4 + 3];
#pragma unroll
            for (int t = 0; t < kNnRPT; ++t) {
                const double vr = (double)vb[t].re, vi = (double)vb[t].im;
                a0r[t] += vr * y0r - vi * y0i;
                a0i[t] += vr * y0i + vi * y0r;
                a1r[t] += vr * y1r - vi * y1i;
                a1i[t] += vr * y1i + vi * y1r;
            }
#pragma unroll
            for (int t = 0; t < kNnRPT; ++t) vb[t] = vn[t];
        }
    }
    // every X element of the thread's rows is loaded (at the clamped rows, so
    // unconditionally) before any is stored: the output columns are distinct,
    // so no store changes a value loaded here, and the loads are one round
    // trip instead of one per row and column
    XR* x0 = (XR*)X.p[0];
    XR* x1 = (XR*)X.p[N > 1 ? 1 : 0];  // column 0 again when there is one (loaded, not stored)
    cplx<XR> xa[kNnRPT], xb[kNnRPT];
#pragma unroll
    for (int t = 0; t < kNnRPT; ++t) {
        xa[t] = ld2(x0, rr[t]);
        xb[t] = ld2(x1, rr[t]);
    }
#pragma unroll
    for (int t = 0; t < kNnRPT; ++t) {
        const int64_t r = r0 + (int64_t)t * kBlock;
        if (r >= n) continue;
        cplx<XR> c = xa[t];
        c.re = (XR)((double)c.re + scale * a0r[t]);
        c.im = (XR)((double)c.im + scale * a0i[t]);
        st2(x0, r, c);
        if (N > 1) {
            cplx<XR> d = xb[t];
            d.re = (XR)((double)d.re + scale * a1r[t]);
            d.im = (XR)((double)d.im + scale * a1i[t]);
            st2(x1, r, d);
        }
    }
}

template <typename VR, typename XR, bool CPLX>
static void nn_launch(const VR* V, int64_t ldv, int64_t n, int M, const double* Y, int N, const ColPtrs<void>& X,
                      double scale, const int* halt, hipStream_t s) {
    if (CPLX && N > 2) {
        dim3 gm((unsigned)((n + 63) / 64));
#define SC_NNT(NT_) SC_TLAUNCH((k_nn_mfma<VR, XR, NT_>), gm, dim3(kBlock), 0, s, V, ldv, n, M, Y, N, X, scale, halt)
        if (N <= 8)
            SC_NNT(1);
        else if (N <= 16)
            SC_NNT(2);
        else if (N <= 24)
            SC_NNT(3);
        else
            SC_NNT(4);
#undef SC_NNT
        return;
    }
    if (CPLX && N <= 2) {
        dim3 gs((unsigned)((n + kBlock * kNnRPT - 1) / (kBlock * kNnRPT)));
        SC_TLAUNCH((k_nn_small<VR, XR>), gs, dim3(kBlock), 0, s, V, ldv, n, M, Y, N, X, scale, halt);
        return;
    }
    dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
    if (N <= 2)
        SC_TLAUNCH((k_nn<VR, XR, CPLX, 2>), grid, dim3(kBlock), 0, s, V, ldv, n, M, Y, N, X, scale, halt);
    else if (N <= 8)
        SC_TLAUNCH((k_nn<VR, XR, CPLX, 8>), grid, dim3(kBlock), 0, s, V, ldv, n, M, Y, N, X, scale, halt);
    else
        SC_TLAUNCH((k_nn<VR, XR, CPLX, 32>), grid, dim3(kBlock), 0, s, V, ldv, n, M, Y, N, X, scale, halt);
}

sc_status gemm_nn(bool cplx, bool vsingle, const void* V, int64_t ldv, int64_t n, int M, const double* Y, int N,
                  bool xsingle, const ColPtrs<void>& X, double scale, const int* halt, hipStream_t s) {
    if (M <= 0 || N <= 0 || n <= 0) return SC_OK;
    if (N > kMaxCols) {
        set_error("gemm_nn: too many columns");
        return SC_ERR_ARG;
    }
    const double eb = (cplx ? 2.0 : 1.0);
    TimerScope ts_(TC_GEMM_NN, s, (double)n * M * eb * (vsingle ? 4 : 8) + 2.0 * n * N * eb * (xsingle ? 4 : 8),
                   (cplx ? 8.0 : 2.0) * n * M * N);
#define SC_NN(VR, XR, C) nn_launch<VR, XR, C>((const VR*)V, ldv, n, M, Y, N, X, scale, halt, s)
    if (cplx) {
        if (vsingle) { if (xsingle) SC_NN(float, float, true); else SC_NN(float, double, true); }
        else { if (xsingle) SC_NN(double, float, true); else SC_NN(double, double, true); }
    } else {
        if (vsingle) { if (xsingle) SC_NN(float, float, false); else SC_NN(float, double, false); }
        else { if (xsingle) SC_NN(double, float, false); else SC_NN(double, double, false); }
    }
#undef SC_NN
    SC_LAUNCH_CHECK();
    return SC_OK;
}

// ---------------------------------------------------------------- T^{-1}
// T is real, so a complex right-hand side is two real ones: Y is an M x nc
// row-major real matrix (nc = N or 2N, at most 2 kMaxCols).  One block: the
// pivots of T = L U (step 6) are formed on thread 0 from tiles of alpha and
// beta staged in LDS; then the forward and backward sweeps run with thread t
// on column t over tiles of kTriT rows staged in LDS (one coalesced load and
// store per tile instead of a global round trip per row).  The arithmetic and
// its order are those of the plain sweeps.
constexpr int kTriT = 128;

__global__ __launch_bounds__(kBlock) void k_tridiag(const double* __restrict__ alpha, const double* __restrict__ beta,
                                                    int M, double* __restrict__ Y, int nc, const double* e1_beta0,
                                                    double* __restrict__ work, const int* halt) {
    if (halt && *halt) return;
    __shared__ double yt[kTriT][2 * kMaxCols + 1];
    __shared__ double at[kTriT], bt[kTriT];
    double* gam = work;
    double* del = work + M;
    const int t = threadIdx.x;
    double dprev = 0.0;
    for (int a0 = 0; a0 < M; a0 += kTriT) {
        const int na = min(kTriT, M - a0);
        __syncthreads();
        for (int i = t; i < na; i += blockDim.x) {
            at[i] = alpha[a0 + i];
            bt[i] = beta[a0 + i];
        }
        __syncthreads();
        if (t == 0) {
            for (int i = 0; i < na; ++i) {
                const int a = a0 + i;
                if (a == 0) {
                    del[0] = at[0];
                    dprev = at[0];
                } else {
                    const double g = bt[i] / dprev;
                    const double d = at[i] - g * bt[i];
                    gam[a] = g;
                    del[a] = d;
                    dprev = d;
                }
            }
        }
    }
    if (e1_beta0) {
        for (int64_t e = t; e < (int64_t)M * nc; e += blockDim.x) Y[e] = (e == 0) ? *e1_beta0 : 0.0;
    }
    // forward: y_a -= gam_a y_{a-1}
    double prev = 0.0;
    for (int a0 = 0; a0 < M; a0 += kTriT) {
        const int na = min(kTriT, M - a0);
        __syncthreads();
        for (int e = t; e < na * nc; e += blockDim.x) yt[e / nc][e % nc] = Y[(int64_t)a0 * nc + e];
        for (int i = t; i < na; i += blockDim.x) at[i] = gam[a0 + i];
        __syncthreads();
        if (t < nc) {
            int i = 0;
            if (a0 == 0) {
                prev = yt[0][t];
                i = 1;
            }
            for (; i < na; ++i) {
                const double y = yt[i][t] - at[i] * prev;
                yt[i][t] = y;
                prev = y;
            }
        }
        __syncthreads();
        for (int e = t; e < na * nc; e += blockDim.x) Y[(int64_t)a0 * nc + e] = yt[e / nc][e % nc];
    }
    // backward: y_a = (y_a - beta_{a+1} y_{a+1}) / del_a
    double next = 0.0;
    for (int a1 = M; a1 > 0; a1 -= kTriT) {
        const int a0 = max(0, a1 - kTriT), na = a1 - a0;
        __syncthreads();
        for (int e = t; e < na * nc; e += blockDim.x) yt[e / nc][e % nc] = Y[(int64_t)a0 * nc + e];
        for (int i = t; i < na; i += blockDim.x) {
            at[i] = del[a0 + i];
            bt[i] = (a0 + i + 1 < M) ? beta[a0 + i + 1] : 0.0;
        }
        __syncthreads();
        if (t < nc) {
            int i = na - 1;
            if (a1 == M) {
                next = yt[i][t] / at[i];
                yt[i][t] = next;
                --i;
            }
            for (; i >= 0; --i) {
                const double y = (yt[i][t] - bt[i] * next) / at[i];
                yt[i][t] = y;
                next = y;
            }
        }
        __syncthreads();
        for (int e = t; e < na * nc; e += blockDim.x) Y[(int64_t)a0 * nc + e] = yt[e / nc][e % nc];
    }
}

// Least squares with the (M+1) x M tridiagonal T~ (T with the row beta_M e_M^T
// appended): C (M+1 x nc, row-major, real) is overwritten so that its first M
// rows hold y = argmin || C - T~ y || per column.  A QR factorization of T~
// by M reflections G_k on rows (k, k+1), [u; w] -> [c u + s w; s u - c w],
// the recurrences of MINRES (Paige and Saunders): thread 0 forms the
// rotations and the three diagonals of R (r_kk, r_{k-1,k}, r_{k-2,k}); then
// each column is rotated and back-substituted by one thread, over tiles of
// rows staged in LDS.
__global__ __launch_bounds__(kBlock) void k_tridiag_lsq(const double* __restrict__ alpha,
                                                        const double* __restrict__ beta, int M, double* __restrict__ C,
                                                        int nc, double* __restrict__ work) {
    __shared__ double yt[kTriT + 1][2 * kMaxCols + 1];
    __shared__ double ct[kTriT], st[kTriT], r0t[kTriT + 2], r1t[kTriT + 2], r2t[kTriT + 2];
    double* cs = work;
    double* sn = work + M;
    double* rd = work + 2 * M;   // r_kk
    double* ru1 = work + 3 * M;  // r_{k-1,k}
    double* ru2 = work + 4 * M;  // r_{k-2,k}
    const int t = threadIdx.x;
    if (t == 0) {
        double cp = -1.0, sp = 0.0, d1 = 0.0, ep = 0.0;
        for (int k = 0; k < M; ++k) {
            const double a = alpha[k], bn = beta[k + 1];
            const double d2 = cp * d1 + sp * a;
            const double g1 = sp * d1 - cp * a;
            const double en = sp * bn;
            const double d1n = -cp * bn;
            const double g2 = sqrt(g1 * g1 + bn * bn);
            const double c = g1 / g2, sv = bn / g2;
            cs[k] = c;
            sn[k] = sv;
            rd[k] = g2;
            ru1[k] = d2;
            ru2[k] = ep;
            cp = c;
            sp = sv;
            d1 = d1n;
            ep = en;
        }
    }
    __syncthreads();
    // the reflections, in order, on each column (row k is final after G_k)
    double carry = 0.0;
    for (int a0 = 0; a0 < M; a0 += kTriT) {
        const int na = min(kTriT, M - a0);
        __syncthreads();
        for (int e = t; e < (na + 1) * nc; e += blockDim.x) yt[e / nc][e % nc] = C[(int64_t)a0 * nc + e];
        for (int i = t; i < na; i += blockDim.x) {
            ct[i] = cs[a0 + i];
            st[i] = sn[a0 + i];
        }
        __syncthreads();
        if (t < nc) {
            double u = a0 == 0 ? yt[0][t] : carry;
            for (int i = 0; i < na; ++i) {
                const double w = yt[i + 1][t];
                yt[i][t] = ct[i] * u + st[i] * w;
                u = st[i] * u - ct[i] * w;
            }
            carry = u;
            yt[na][t] = u;
        }
        __syncthreads();
        for (int e = t; e < (na + 1) * nc; e += blockDim.x) C[(int64_t)a0 * nc + e] = yt[e / nc][e % nc];
    }
    // back substitution: y_k = (u_k - r_{k,k+1} y_{k+1} - r_{k,k+2} y_{k+2}) / r_kk
    double y1 = 0.0, y2 = 0.0;  // y_{k+1}, y_{k+2}
    for (int a1 = M; a1 > 0; a1 -= kTriT) {
        const int a0 = max(0, a1 - kTriT), na = a1 - a0;
        __syncthreads();
        for (int e = t; e < na * nc; e += blockDim.x) yt[e / nc][e % nc] = C[(int64_t)a0 * nc + e];
        for (int i = t; i < na; i += blockDim.x) r0t[i] = rd[a0 + i];
        for (int i = t; i < na + 2; i += blockDim.x) {
            r1t[i] = a0 + i < M ? ru1[a0 + i] : 0.0;
            r2t[i] = a0 + i < M ? ru2[a0 + i] : 0.0;
        }
        __syncthreads();
        if (t < nc) {
            for (int i = na - 1; i >= 0; --i) {
                // r_{k,k+1} is the entry above the diagonal in column k+1, r_{k,k+2} two above in column k+2
                const double y = (yt[i][t] - r1t[i + 1] * y1 - r2t[i + 2] * y2) / r0t[i];
                yt[i][t] = y;
                y2 = y1;
                y1 = y;
            }
        }
        __syncthreads();
        for (int e = t; e < na * nc; e += blockDim.x) C[(int64_t)a0 * nc + e] = yt[e / nc][e % nc];
    }
}

sc_status tridiag_lsq(const double* alpha, const double* beta, int M, double* C, int N, bool cplx, double* work,
                      hipStream_t s) {
    if (M <= 0 || N <= 0) return SC_OK;
    const int nc = N * (cplx ? 2 : 1);
    if (nc > 2 * kMaxCols) {
        set_error("tridiag_lsq: too many columns");
        return SC_ERR_ARG;
    }
    hipLaunchKernelGGL(k_tridiag_lsq, dim3(1), dim3(kBlock), 0, s, alpha, beta, M, C, nc, work);
    SC_LAUNCH_CHECK();
    return SC_OK;
}

sc_status tridiag_solve(const double* alpha, const double* beta, int M, double* Y, int N, bool cplx,
                        const double* e1_beta0, double* work, const int* halt, hipStream_t s) {
    if (M <= 0 || N <= 0) return SC_OK;
    const int nc = N * (cplx ? 2 : 1);
    if (nc > 2 * kMaxCols) {
        set_error("tridiag_solve: too many columns");
        return SC_ERR_ARG;
    }
    hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(kBlock), 0, s, alpha, beta, M, Y, nc, e1_beta0, work, halt);
    SC_LAUNCH_CHECK();
    return SC_OK;
}

}  // namespace sc
