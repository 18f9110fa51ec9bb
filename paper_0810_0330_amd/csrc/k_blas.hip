// Streaming vector kernels on real views (a complex column of n elements is
// 2n reals): linear combinations with precision conversion, and dot products
// accumulated in FP64 (per-block partials, then a fixed-order finish).
#include "sc_internal.h"

namespace sc {

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
sc_status fill(T* p, int64_t n, T v, hipStream_t s) {
    if (n <= 0) return SC_OK;
    int g = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_fill<T>, dim3(g), dim3(kBlock), 0, s, p, n, v);
    SC_LAUNCH_CHECK();
    return SC_OK;
}
template sc_status fill<double>(double*, int64_t, double, hipStream_t);
template sc_status fill<unsigned>(unsigned*, int64_t, unsigned, hipStream_t);
template sc_status fill<int>(int*, int64_t, int, hipStream_t);
template sc_status fill<float>(float*, int64_t, float, hipStream_t);

// z = a x + b y: four elements per thread and trip, a grid stride apart, so
// every load instruction of a wave covers 64 consecutive elements and four of
// them are in flight before the first is used
template <typename ZT, typename XT, typename YT>
__global__ __launch_bounds__(kBlock) void k_lincomb(ZT* __restrict__ z, int64_t ldz, const XT* __restrict__ x,
                                                    int64_t ldx, const YT* __restrict__ y, int64_t ldy, int64_t N,
                                                    double a, double b) {
    const int col = blockIdx.y;
    ZT* zc = z + col * ldz;
    const XT* xc = x + col * ldx;
    const YT* yc = y ? y + col * ldy : nullptr;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + 3 * stride < N; i += 4 * stride) {
        double xv[4], yv[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = (double)xc[i + u * stride];
        if (yc) {
#pragma unroll
            for (int u = 0; u < 4; ++u) yv[u] = (double)yc[i + u * stride];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double v = a * xv[u];
            if (yc) v += b * yv[u];
            zc[i + u * stride] = (ZT)v;
        }
    }
    for (; i < N; i += stride) {
        double v = a * (double)xc[i];
        if (yc) v += b * (double)yc[i];
        zc[i] = (ZT)v;
    }
}

template <typename ZT, typename XT>
static void lincomb_y(int yt, ZT* z, int64_t ldz, const XT* x, int64_t ldx, const void* y, int64_t ldy, int64_t N,
                      int k, double a, double b, hipStream_t s) {
    dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((N + 4 * kBlock - 1) / (4 * kBlock), 2048)), (unsigned)k);
    if (yt == 0)
        hipLaunchKernelGGL((k_lincomb<ZT, XT, double>), grid, dim3(kBlock), 0, s, z, ldz, x, ldx, (const double*)y, ldy, N, a, b);
    else
        hipLaunchKernelGGL((k_lincomb<ZT, XT, float>), grid, dim3(kBlock), 0, s, z, ldz, x, ldx, (const float*)y, ldy, N, a, b);
}

template <typename ZT>
static void lincomb_x(int xt, ZT* z, int64_t ldz, const void* x, int64_t ldx, int yt, const void* y, int64_t ldy,
                      int64_t N, int k, double a, double b, hipStream_t s) {
    if (xt == 0) lincomb_y<ZT, double>(yt, z, ldz, (const double*)x, ldx, y, ldy, N, k, a, b, s);
    else lincomb_y<ZT, float>(yt, z, ldz, (const float*)x, ldx, y, ldy, N, k, a, b, s);
}

sc_status lincomb(int zt, void* z, int64_t ldz, int xt, const void* x, int64_t ldx, int yt, const void* y,
                  int64_t ldy, int64_t N, int k, double a, double b, hipStream_t s) {
    if (N <= 0 || k <= 0) return SC_OK;
    if (zt == 0) lincomb_x<double>(xt, (double*)z, ldz, x, ldx, yt, y, ldy, N, k, a, b, s);
    else lincomb_x<float>(xt, (float*)z, ldz, x, ldx, yt, y, ldy, N, k, a, b, s);
    SC_LAUNCH_CHECK();
    return SC_OK;
}

// partial sums of x*y per block and column
template <typename XT, typename YT>
__global__ __launch_bounds__(kBlock) void k_dot_part(const XT* __restrict__ x, int64_t ldx, const YT* __restrict__ y,
                                                     int64_t ldy, int64_t N, double* part) {
    __shared__ double sh[kWaves];
    const int col = blockIdx.y;
    const XT* xc = x + col * ldx;
    const YT* yc = y + col * ldy;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock)
        acc += (double)xc[i] * (double)yc[i];
    block_partial(acc, part + (int64_t)col * gridDim.x, sh);
}

__global__ __launch_bounds__(kBlock) void k_dot_finish(const double* part, int G, double* res) {
    __shared__ double sh[kWaves];
    const double s = sum_partials(part + (int64_t)blockIdx.x * G, G, sh);
    if (threadIdx.x == 0) res[blockIdx.x] = s;
}

template <typename XT>
static void dot_y(int yt, const XT* x, int64_t ldx, const void* y, int64_t ldy, int64_t N, int k, double* res,
                  double* part, hipStream_t s) {
    const int g = red_grid(N, 4);
    dim3 grid((unsigned)g, (unsigned)k);
    if (yt == 0)
        hipLaunchKernelGGL((k_dot_part<XT, double>), grid, dim3(kBlock), 0, s, x, ldx, (const double*)y, ldy, N, part);
    else
        hipLaunchKernelGGL((k_dot_part<XT, float>), grid, dim3(kBlock), 0, s, x, ldx, (const float*)y, ldy, N, part);
    hipLaunchKernelGGL(k_dot_finish, dim3(k), dim3(kBlock), 0, s, part, g, res);
}

sc_status dot(int xt, const void* x, int64_t ldx, int yt, const void* y, int64_t ldy, int64_t N, int k, double* res,
              double* part, unsigned* /*unused*/, hipStream_t s) {
    if (k <= 0) return SC_OK;
    if (xt == 0) dot_y<double>(yt, (const double*)x, ldx, y, ldy, N, k, res, part, s);
    else dot_y<float>(yt, (const float*)x, ldx, y, ldy, N, k, res, part, s);
    SC_LAUNCH_CHECK();
    return SC_OK;
}

}  // namespace sc
