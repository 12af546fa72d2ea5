// tb_readback.hip -- significance of the candidate records, on the device,
// before they are copied to the host (the readback step of the threshold
// search, Sec. 2.1).
//
// Whitened noise powers are unit exponentials, so a fold of h of them has the
// upper tail Q(h, S) = exp(-S) sum_{k<h} S^k / k!; a record's significance is
// the z with one-sided Gaussian tail Q(z) = Q(h, S), found in FP64.  Each
// record {template, bin, series << 8 | log2 h, S} is rewritten in place as
// {template, bin | log2 h << 28, sigma (FP32 bits), S}: bins stay below 2^24,
// and the host knows a request's series.
#include <hip/hip_runtime.h>

#include "tb_internal.h"

namespace tb {
namespace {

constexpr double kHalfLog2PiD = 0.91893853320467274178;  // log sqrt(2 pi)
constexpr double kRsqrt2D = 0.70710678118654752440;

// log Q(h, x): the sum relative to its largest term k* = min(h - 1, floor x),
// neighbouring terms by the ratios x / k and k / x.
__device__ double log_q_dev(int h, double x)
{
    if (x <= 0.0) return 0.0;
    const int ks = (int)fmin((double)(h - 1), floor(x));
    double acc = 1.0, r = 1.0;
    for (int k = ks; k >= 1; --k) {
        r *= (double)k / x;
        acc += r;
    }
    r = 1.0;
    for (int k = ks + 1; k < h; ++k) {
        r *= x / (double)k;
        acc += r;
    }
    return -x + ks * log(x) - lgamma((double)ks + 1.0) + log(acc);
}

// log of the one-sided Gaussian tail; from z = 37 on (erfc nears the bottom
// of the double range) by the continued fraction of the Mills ratio.
__device__ double log_gauss_sf_dev(double z)
{
    if (z < 37.0) return log(0.5 * erfc(z * kRsqrt2D));
    double f = z;
    for (int k = 80; k >= 1; --k) f = z + (double)k / f;
    return -0.5 * z * z - kHalfLog2PiD - log(f);
}

// z with log_gauss_sf(z) = log Q(h, s), z >= -30.  log_gauss_sf is concave
// and decreasing, so after the first Newton step every step approaches the
// root from above; the start is the tail expansion
// log Q(z) ~ -z^2/2 - log z - log sqrt(2 pi), refined twice.
__device__ double fold_sigma_dev(int h, double s)
{
    const double target = log_q_dev(h, s);
    if (target >= log_gauss_sf_dev(-30.0)) return -30.0;
    double z = sqrt(fmax(0.0, -2.0 * target));
    if (z > 2.0)
        for (int i = 0; i < 2; ++i) z = sqrt(fmax(0.0, -2.0 * (target + kHalfLog2PiD + log(z))));
    double lo = -30.0, hi = HUGE_VAL;
    for (int it = 0; it < 100; ++it) {
        const double lz = log_gauss_sf_dev(z);
        const double g = lz - target;
        if (g > 0)
            lo = z;
        else
            hi = z;
        const double dg = -exp(-0.5 * z * z - kHalfLog2PiD - lz);
        double nz = z - g / dg;
        if (!(nz > lo && nz < hi)) nz = hi < HUGE_VAL ? 0.5 * (lo + hi) : z + fmax(1.0, fabs(z));
        if (fabs(nz - z) < 1e-12 * fmax(1.0, fabs(z))) return nz;
        z = nz;
    }
    return z;
}

// The first min(*counter, cap) records of a ring, grid-stride.
__global__ __launch_bounds__(256) void k_significance(uint4* __restrict__ ring, const uint32_t* __restrict__ counter,
                                                      uint32_t cap)
{
    const uint32_t n = min(*counter, cap);
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
        const uint4 q = ring[i];
        const uint32_t l = q.z & 0xffu;
        const float sg = (float)fold_sigma_dev(1 << l, (double)__uint_as_float(q.w));
        ring[i] = make_uint4(q.x, q.y | (l << 28), __float_as_uint(sg), q.w);
    }
}

}  // namespace

hipError_t launch_significance(uint4* ring, const uint32_t* counter, uint64_t cap, hipStream_t s)
{
    if (cap == 0) return hipSuccess;
    const uint32_t c = (uint32_t)(cap < 0xffffffffull ? cap : 0xffffffffull);
    const uint32_t blocks = (uint32_t)((cap + 255) / 256 < 256 ? (cap + 255) / 256 : 256);
    hipLaunchKernelGGL(k_significance, dim3(blocks), dim3(256), 0, s, ring, counter, c);
    return hipGetLastError();
}

}  // namespace tb
