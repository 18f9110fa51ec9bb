// Whether the links of a Wilson operator are in SU(3): the condition under
// which a link's third row is the complex conjugate of the cross product of
// its first two, so that the single-precision passes may read two rows of each
// link and rebuild the third (12 of the 18 reals of a link).
#include <algorithm>
#include <cmath>
#include <vector>

#include "sc_internal.h"

namespace sc {

namespace {

constexpr int kLinkBlock = 256;

// Largest over the 4V links of the entrywise moduli of U U^H - 1 and of
// |det U - 1|, in FP64; +inf when a link holds a value that is not finite.
// One maximum per block (an LDS tree), taken over the blocks on the host.
__global__ __launch_bounds__(kLinkBlock) void k_su3_dev(const double* __restrict__ U, int64_t V, double* out) {
    __shared__ double sm[kLinkBlock];
    double dev = 0.0;
    bool bad = false;
    const int64_t nl = 4 * V;
    for (int64_t l = (int64_t)blockIdx.x * kLinkBlock + threadIdx.x; l < nl; l += (int64_t)gridDim.x * kLinkBlock) {
        const int64_t mu = l / V, x = l % V;
        cplx<double> u[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const int64_t e = ((mu * 3 + a) * 3 + b) * V + x;
                u[a][b] = {U[2 * e], U[2 * e + 1]};
                bad |= !isfinite(u[a][b].re) || !isfinite(u[a][b].im);
            }
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {  // (U U^H)_{ac} = sum_b u_ab conj(u_cb)
                double re = a == c ? -1.0 : 0.0, im = 0.0;
                for (int b = 0; b < 3; ++b) {
                    re += u[a][b].re * u[c][b].re + u[a][b].im * u[c][b].im;
                    im += u[a][b].im * u[c][b].re - u[a][b].re * u[c][b].im;
                }
                const double m = sqrt(re * re + im * im);
                bad |= isnan(m);  // an overflow in the products
                dev = fmax(dev, m);
            }
        // det U by the first row's cofactors
        auto mul = [](cplx<double> p, cplx<double> q) { return cplx<double>{p.re * q.re - p.im * q.im, p.re * q.im + p.im * q.re}; };
        auto sub = [](cplx<double> p, cplx<double> q) { return cplx<double>{p.re - q.re, p.im - q.im}; };
        const cplx<double> c0 = sub(mul(u[1][1], u[2][2]), mul(u[1][2], u[2][1]));
        const cplx<double> c1 = sub(mul(u[1][2], u[2][0]), mul(u[1][0], u[2][2]));
        const cplx<double> c2 = sub(mul(u[1][0], u[2][1]), mul(u[1][1], u[2][0]));
        const cplx<double> d0 = mul(u[0][0], c0), d1 = mul(u[0][1], c1), d2 = mul(u[0][2], c2);
        const double dre = d0.re + d1.re + d2.re - 1.0, dim = d0.im + d1.im + d2.im;
        const double m = sqrt(dre * dre + dim * dim);
        bad |= isnan(m);
        dev = fmax(dev, m);
    }
    sm[threadIdx.x] = (bad || !isfinite(dev)) ? INFINITY : dev;
    __syncthreads();
    for (int h = kLinkBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

}  // namespace

sc_status wilson_check_su3(sc_op* op, hipStream_t s, double* deviation, int* rebuild) {
    const int64_t nl = 4 * op->vol;
    const int grid = (int)std::min<int64_t>((nl + kLinkBlock - 1) / kLinkBlock, 1024);
    double* d = nullptr;
    SC_HIP(hipMalloc((void**)&d, grid * sizeof(double)));
    std::vector<double> h(grid, 0.0);
    hipLaunchKernelGGL(k_su3_dev, dim3(grid), dim3(kLinkBlock), 0, s, (const double*)op->U64, op->vol, d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, grid * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    const hipError_t ef = hipFree(d);
    SC_HIP(e);
    SC_HIP(ef);
    double dev = 0.0;
    for (double v : h) dev = std::max(dev, v);  // no NaN: the kernel maps non-finite values to +inf
    op->su3 = (op->U32 && dev <= kSu3Tol) ? 1 : 0;
    if (deviation) *deviation = dev;
    if (rebuild) *rebuild = op->su3;
    return SC_OK;
}

}  // namespace sc
