// order.hip -- relative 2-norm of the difference between two potentials,
// for the measured choice of the expansion order (fmm_choose_order): the
// truncation error of an expansion falls geometrically in p at fixed theta
// (Sec. 2.3), so the order is the smallest one whose result agrees with a
// high-order evaluation to the requested accuracy.
#include <algorithm>
#include <cmath>
#include <vector>

#include "fmm_internal.h"

namespace fmm {

constexpr int kErrBlocks = 512;

// per-block sums of |a - ref|^2 and |ref|^2 over a grid-stride range
__global__ void __launch_bounds__(256)
k_err_partial(const double2* __restrict__ a, const double2* __restrict__ ref, int64_t n, double2* part)
{
    __shared__ double sn[4], sd[4];
    double num = 0.0, den = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double2 r = ref[i], x = a[i];
        const double dx = x.x - r.x, dy = x.y - r.y;
        num = fma(dx, dx, fma(dy, dy, num));
        den = fma(r.x, r.x, fma(r.y, r.y, den));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        num += __shfl_xor(num, o, 64);
        den += __shfl_xor(den, o, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { sn[w] = num; sd[w] = den; }
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(sn[0] + sn[1] + sn[2] + sn[3], sd[0] + sd[1] + sd[2] + sd[3]);
}

// ||a - ref||_2 / ||ref||_2 over n complex values (device arrays, [n][2]);
// waits for `s`.  The block sums are added on the host in a fixed order.
double rel_err2_device(const double* a, const double* ref, int64_t n, hipStream_t s)
{
    if (n <= 0) return 0.0;
    const int nb = (int)std::min<int64_t>(kErrBlocks, (n + 255) / 256);
    DBuf<double> part;
    part.alloc(2 * (size_t)nb, s);
    k_err_partial<<<nb, 256, 0, s>>>((const double2*)a, (const double2*)ref, n, (double2*)part.p);
    check_launch("error norm");
    std::vector<double> h(2 * (size_t)nb);
    FMM_HIP(hipMemcpyAsync(h.data(), part.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    FMM_HIP(hipStreamSynchronize(s));
    double num = 0.0, den = 0.0;
    for (int b = 0; b < nb; ++b) { num += h[2 * b]; den += h[2 * b + 1]; }
    if (den == 0.0) return num == 0.0 ? 0.0 : INFINITY;
    return std::sqrt(num / den);
}

}  // namespace fmm
