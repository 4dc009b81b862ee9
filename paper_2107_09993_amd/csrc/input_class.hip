// Input class for the autotuner's table: whether the attributes of the input
// rise together (correlated), trade off against each other (anti-correlated)
// or neither.  The skyline's size and the cost of each grid and refine form
// depend mostly on this, so the tuning table can hold one row per class.
//
// A strided sample of at most kClassSample points gives, per dimension, the
// sums of x and x^2 and, per point, the sum s of its coordinates: with v_k the
// variance of dimension k and V the variance of s,
//   V = sum_k v_k + 2 sum_{k<l} cov(k, l),
// so the mean correlation of two dimensions is about
//   rho = (V - sum_k v_k) / ((d - 1) sum_k v_k).
// Points spread near a plane sum = const give V ~ 0 and rho ~ -1/(d-1); points
// along the diagonal give rho ~ 1; independent attributes rho ~ 0.
#include "common.h"
#include "../../include/skycell.h"

namespace skycell {

constexpr int kClassThreads = 256;
constexpr int kClassBlocks = 64;
constexpr uint32_t kClassSample = 1u << 16;

// Per block: the sums over its sample points of x_k and x_k^2 (k < D), of s
// and of s^2, in binary64, at out[block * (2D + 2) + ...].
template <typename T, int D>
__global__ __launch_bounds__(kClassThreads) void k_class_moments(const T *__restrict__ pts, uint32_t n,
                                                                 uint32_t stride, uint32_t samples,
                                                                 double *__restrict__ out)
{
    constexpr int kV = 2 * D + 2;
    double acc[kV];
#pragma unroll
    for (int v = 0; v < kV; ++v) acc[v] = 0.0;
    for (uint32_t j = blockIdx.x * kClassThreads + threadIdx.x; j < samples; j += kClassBlocks * kClassThreads) {
        const uint32_t i = j * stride;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double x = (double)pts[(size_t)k * n + i];
            acc[k] += x;
            acc[D + k] += x * x;
            s += x;
        }
        acc[2 * D] += s;
        acc[2 * D + 1] += s * s;
    }
    __shared__ double s_part[kClassThreads / kWave][kV];
#pragma unroll
    for (int v = 0; v < kV; ++v) {
        double a = acc[v];
        for (int off = kWave / 2; off > 0; off >>= 1) a += __shfl_xor(a, off);
        if (__lane_id() == 0) s_part[threadIdx.x / kWave][v] = a;
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)kV) {
        double a = 0.0;
        for (int w = 0; w < kClassThreads / kWave; ++w) a += s_part[w][threadIdx.x];
        out[(size_t)blockIdx.x * kV + threadIdx.x] = a;
    }
}

template <typename T>
static hipError_t launch_moments_t(const T *pts, uint32_t n, int d, uint32_t stride, uint32_t samples, double *out,
                                   hipStream_t st)
{
    switch (d) {
#define SKYCELL_CLASS_CASE(DD)                                                                                 \
    case DD:                                                                                                   \
        hipLaunchKernelGGL((k_class_moments<T, DD>), dim3(kClassBlocks), dim3(kClassThreads), 0, st, pts, n, stride, \
                           samples, out);                                                                      \
        return hipGetLastError();
        SKYCELL_CLASS_CASE(1)
        SKYCELL_CLASS_CASE(2)
        SKYCELL_CLASS_CASE(3)
        SKYCELL_CLASS_CASE(4)
        SKYCELL_CLASS_CASE(5)
        SKYCELL_CLASS_CASE(6)
        SKYCELL_CLASS_CASE(7)
        SKYCELL_CLASS_CASE(8)
        SKYCELL_CLASS_CASE(9)
        SKYCELL_CLASS_CASE(10)
        SKYCELL_CLASS_CASE(11)
        SKYCELL_CLASS_CASE(12)
        SKYCELL_CLASS_CASE(13)
        SKYCELL_CLASS_CASE(14)
        SKYCELL_CLASS_CASE(15)
        SKYCELL_CLASS_CASE(16)
#undef SKYCELL_CLASS_CASE
    default:
        return hipErrorInvalidValue;
    }
}

size_t class_moments_bytes(int d) { return sizeof(double) * (size_t)kClassBlocks * (size_t)(2 * d + 2); }

hipError_t launch_class_moments(const void *pts, int dtype, int64_t n, int d, double *out, hipStream_t st)
{
    const uint32_t samples = (uint64_t)n < kClassSample ? (uint32_t)n : kClassSample;
    const uint32_t stride = (uint32_t)((uint64_t)n / samples);
    if (dtype == SKYCELL_DTYPE_F32) return launch_moments_t((const float *)pts, (uint32_t)n, d, stride, samples, out, st);
    return launch_moments_t((const uint16_t *)pts, (uint32_t)n, d, stride, samples, out, st);
}

int class_from_moments(const double *part, int d, int64_t n)
{
    if (d < 2 || n < 2) return SKYCELL_CLASS_INDEPENDENT;
    const uint64_t samples = (uint64_t)n < kClassSample ? (uint64_t)n : kClassSample;
    const int kv = 2 * d + 2;
    double sum[2 * SKYCELL_MAX_D + 2] = {};
    for (int b = 0; b < kClassBlocks; ++b)
        for (int v = 0; v < kv; ++v) sum[v] += part[(size_t)b * kv + v];
    const double m = (double)samples;
    double var_sum = 0.0;
    for (int k = 0; k < d; ++k) {
        const double mean = sum[k] / m;
        var_sum += sum[d + k] / m - mean * mean;
    }
    const double smean = sum[2 * d] / m;
    const double svar = sum[2 * d + 1] / m - smean * smean;
    if (!(var_sum > 0.0)) return SKYCELL_CLASS_INDEPENDENT;
    const double rho = (svar - var_sum) / ((double)(d - 1) * var_sum);
    if (rho > 0.3) return SKYCELL_CLASS_CORRELATED;
    if (rho < -0.3 / (double)(d - 1)) return SKYCELL_CLASS_ANTICORRELATED;
    return SKYCELL_CLASS_INDEPENDENT;
}

}  // namespace skycell
