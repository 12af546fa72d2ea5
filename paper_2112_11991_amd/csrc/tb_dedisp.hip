// tb_dedisp.hip -- incoherent dedispersion of an 8-bit filterbank, the step
// before the search (App. A, Sec. 5.2): for DM trial d, output sample t is
// the sum over channels c of x_c[t + s_dc], s_dc the channel's dispersion
// delay in samples relative to the highest frequency.
//
// The filterbank arrives time-major (all channels of a sample together) and
// is transposed once to channel-major bytes.  A workgroup then owns TT
// output samples of DT consecutive DM trials: for each channel it stages the
// bytes [t0 + min_d s_dc, t0 + TT + max_d s_dc) in LDS and every thread adds
// the 4 x DT samples it owns.  Sums of bytes over up to 8192 channels stay
// below 2^31, so they accumulate exactly in 32-bit integers and are converted
// once.  A channel whose delay spread within the DM tile exceeds the staging
// room is read straight from global memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "tb_internal.h"

namespace tb {
namespace {

constexpr int DD_NT = 256;              // threads per workgroup
constexpr int DD_TT = 1024;             // output samples per workgroup (4 per thread)
constexpr int DD_DT = 16;               // DM trials per workgroup
constexpr int DD_SPAN = 3072;           // delay spread a staged channel may have
constexpr int DD_SEG = DD_TT + DD_SPAN; // staged bytes per channel

// 64 x 64 byte tiles: in[t][c] (time-major) -> out[c][t].
__global__ __launch_bounds__(256) void k_fb_transpose(const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                      int nchan, int64_t nsamp)
{
    __shared__ uint8_t tile[64][65];
    const int64_t t0 = (int64_t)blockIdx.x * 64;
    const int c0 = (int)blockIdx.y * 64;
    const int tx = (int)threadIdx.x & 63, ty = (int)threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int64_t t = t0 + r;
        const int c = c0 + tx;
        tile[r][tx] = (t < nsamp && c < nchan) ? in[t * nchan + c] : (uint8_t)0;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int c = c0 + r;
        const int64_t t = t0 + tx;
        if (c < nchan && t < nsamp) out[(int64_t)c * nsamp + t] = tile[tx][r];
    }
}

// delay[c * ldd + d]: delay of channel c at DM trial d (ldd = DM trials
// rounded up to DD_DT); lo[c * ntile + g], span in hi: the smallest delay and
// the spread over tile g's trials.
__global__ __launch_bounds__(DD_NT) void k_dedisperse(const uint8_t* __restrict__ x, int nchan, int64_t nsamp,
                                                      const int32_t* __restrict__ delay, int ldd,
                                                      const int2* __restrict__ lospan, int ntile, int ndm,
                                                      int64_t nout, float* __restrict__ out)
{
    __shared__ __align__(16) uint8_t seg[DD_SEG];
    const int64_t t0 = (int64_t)blockIdx.x * DD_TT;
    const int g = (int)blockIdx.y, d0 = g * DD_DT;
    const int tid = (int)threadIdx.x;
    uint32_t acc[4][DD_DT];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < DD_DT; ++j) acc[k][j] = 0u;

    for (int c = 0; c < nchan; ++c) {
        const int2 ls = lospan[(int64_t)c * ntile + g];  // uniform
        const int32_t* dc = delay + (int64_t)c * ldd + d0;
        const uint8_t* xc = x + (int64_t)c * nsamp;
        if (ls.y <= DD_SPAN) {
            // stage [t0 + lo, t0 + lo + TT + span), clipped to the series
            const int64_t a = t0 + ls.x;
            const int n = DD_TT + ls.y;
            __syncthreads();
            for (int i = tid; i < n; i += DD_NT) {
                const int64_t t = a + i;
                seg[i] = t < nsamp ? xc[t] : (uint8_t)0;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < DD_DT; ++j) {
                const int o = dc[j] - ls.x + tid;
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[k][j] += seg[o + k * DD_NT];
            }
        } else {
#pragma unroll
            for (int j = 0; j < DD_DT; ++j) {
                const int64_t a = t0 + dc[j] + tid;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int64_t t = a + k * DD_NT;
                    acc[k][j] += t < nsamp ? xc[t] : 0u;
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < DD_DT; ++j) {
        if (d0 + j >= ndm) break;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t t = t0 + tid + k * DD_NT;
            if (t < nout) out[(int64_t)(d0 + j) * nout + t] = (float)acc[k][j];
        }
    }
}

}  // namespace

int64_t dedisp_delays(int nchan, double fch1, double foff, double tsamp, const double* dm, int ndm,
                      std::vector<int32_t>& delay, int& ldd)
{
    const double flast = fch1 + (nchan - 1) * foff;
    const double ftop = fch1 > flast ? fch1 : flast;
    ldd = (ndm + DD_DT - 1) / DD_DT * DD_DT;
    delay.assign((size_t)nchan * ldd, 0);
    int64_t smax = 0;
    for (int d = 0; d < ndm; ++d)
        for (int c = 0; c < nchan; ++c) {
            const double f = fch1 + c * foff;
            const double dl = 4.148808e3 * dm[d] * (1.0 / (f * f) - 1.0 / (ftop * ftop));
            const int64_t v = (int64_t)std::rint(dl / tsamp);
            delay[(size_t)c * ldd + d] = (int32_t)v;
            smax = std::max(smax, v);
        }
    // padding trials repeat the last real one (never stored)
    for (int c = 0; c < nchan; ++c)
        for (int d = ndm; d < ldd; ++d) delay[(size_t)c * ldd + d] = delay[(size_t)c * ldd + ndm - 1];
    return smax;
}

hipError_t launch_dedisperse(const uint8_t* d_tm, uint8_t* d_cm, int nchan, int64_t nsamp, const int32_t* d_delay,
                             int ldd, const int2* d_lospan, int ndm, int64_t nout, float* out, hipStream_t s)
{
    if (d_tm) {
        const dim3 tg((unsigned)((nsamp + 63) / 64), (unsigned)((nchan + 63) / 64));
        hipLaunchKernelGGL(k_fb_transpose, tg, dim3(256), 0, s, d_tm, d_cm, nchan, nsamp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int ntile = ldd / DD_DT;
    const dim3 grid((unsigned)((nout + DD_TT - 1) / DD_TT), (unsigned)ntile);
    hipLaunchKernelGGL(k_dedisperse, grid, dim3(DD_NT), 0, s, d_cm, nchan, nsamp, d_delay, ldd, d_lospan, ntile, ndm,
                       nout, out);
    return hipGetLastError();
}

int dedisp_tile() { return DD_DT; }

}  // namespace tb
