// tb_dedisp.hip -- incoherent dedispersion of an 8-bit filterbank, the step
// before the search (App. A, Sec. 5.2): for DM trial d, output sample t is
// the sum over channels c of x_c[t + s_dc], s_dc the channel's dispersion
// delay in samples relative to the highest frequency.
//
// The filterbank arrives time-major (all channels of a sample together) and
// is transposed once to channel-major bytes.  A workgroup then owns TT
// output samples of DT consecutive DM trials: for each channel it stages the
// bytes [t0 + min_d s_dc, t0 + TT + max_d s_dc) in LDS (four channels per
// step, double-buffered) and every thread adds the 4 x DT samples it owns.
// Sums of bytes over up to 8192 channels stay below 2^31, so they accumulate
// exactly in 32-bit integers and are converted once.  A channel whose delay spread within the DM tile exceeds the staging
// room is read straight from global memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "tb_internal.h"

namespace tb {
namespace {

constexpr int DD_NT = 256;               // threads per workgroup
constexpr int DD_TT = 1024;              // output samples per workgroup (4 per thread)
constexpr int DD_DT = 16;                // DM trials per workgroup
constexpr int DD_CH = 4;                 // channels staged per step
constexpr int DD_SEGD = 1024;            // staged dwords per channel (4096 bytes)
constexpr int DD_SPAN = 4 * DD_SEGD - DD_TT - 8;  // delay spread a staged channel may have (3064)

// 64 x 64 sample tiles: in (time-major, 8-bit samples or 4-bit pairs with
// the even channel in the low nibble) -> out[c][t] bytes with rows of ldx
// bytes; the row padding beyond nsamp is zeroed.
template <int NBITS>
__global__ __launch_bounds__(256) void k_fb_transpose(const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                      int nchan, int64_t nsamp, int64_t ldx)
{
    __shared__ uint8_t tile[64][65];
    const int64_t t0 = (int64_t)blockIdx.x * 64;
    const int c0 = (int)blockIdx.y * 64;
    const int tx = (int)threadIdx.x & 63, ty = (int)threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int64_t t = t0 + r;
        const int c = c0 + tx;
        uint8_t v = 0;
        if (t < nsamp && c < nchan) {
            if constexpr (NBITS == 8) {
                v = in[t * nchan + c];
            } else {
                const uint8_t b = in[(t * nchan + c) >> 1];
                v = (c & 1) ? (uint8_t)(b >> 4) : (uint8_t)(b & 15u);
            }
        }
        tile[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int c = c0 + r;
        const int64_t t = t0 + tx;
        if (c < nchan && t < ldx) out[(int64_t)c * ldx + t] = tile[tx][r];
    }
}

// delay[c * ldd + d]: delay of channel c at DM trial d (ldd = DM trials
// rounded up to DD_DT); lospan[c * ntile + g] = (smallest delay, spread) over
// tile g's trials.  Channel rows are ldx bytes (a multiple of 16), zero
// beyond nsamp.  Channels are taken DD_CH at a time: while one group is
// summed from LDS, the next group's aligned dwords are already loading into
// registers, then stored to the other LDS buffer (one barrier per group).
__global__ __launch_bounds__(DD_NT) void k_dedisperse(const uint8_t* __restrict__ x, int nchan, int64_t ldx,
                                                      const int32_t* __restrict__ delay, int ldd,
                                                      const int2* __restrict__ lospan, int ntile, int ndm,
                                                      int64_t nout, float* __restrict__ out)
{
    __shared__ __align__(16) uint32_t sbuf[2][DD_CH][DD_SEGD];
    const int64_t t0 = (int64_t)blockIdx.x * DD_TT;
    const int g = (int)blockIdx.y, d0 = g * DD_DT;
    const int tid = (int)threadIdx.x;
    const int ngrp = (nchan + DD_CH - 1) / DD_CH;
    uint32_t acc[4][DD_DT];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < DD_DT; ++j) acc[k][j] = 0u;

    uint32_t pf[DD_CH][4];
    // dwords of channel c's segment [t0 + lo, t0 + lo + TT + span) from the
    // aligned start a0 = (t0 + lo) & ~3; none for channels read from global
    auto fetch = [&](int grp) {
#pragma unroll
        for (int q = 0; q < DD_CH; ++q) {
            const int c = grp * DD_CH + q;
            int2 ls = make_int2(0, DD_SPAN + 1);
            if (c < nchan) ls = lospan[(int64_t)c * ntile + g];
            const int64_t a0 = (t0 + ls.x) & ~(int64_t)3;
            const uint32_t* row = reinterpret_cast<const uint32_t*>(x + (int64_t)(c < nchan ? c : 0) * ldx);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int64_t byte = a0 + 4 * (int64_t)(tid + m * DD_NT);
                pf[q][m] = (ls.y <= DD_SPAN && byte + 4 <= ldx) ? row[byte >> 2] : 0u;
            }
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < DD_CH; ++q)
#pragma unroll
            for (int m = 0; m < 4; ++m) sbuf[buf][q][tid + m * DD_NT] = pf[q][m];
    };

    fetch(0);
    stash(0);
    __syncthreads();
    for (int grp = 0; grp < ngrp; ++grp) {
        const int buf = grp & 1;
        if (grp + 1 < ngrp) fetch(grp + 1);
#pragma unroll
        for (int q = 0; q < DD_CH; ++q) {
            const int c = grp * DD_CH + q;
            if (c >= nchan) break;
            const int2 ls = lospan[(int64_t)c * ntile + g];  // uniform
            const int32_t* dc = delay + (int64_t)c * ldd + d0;
            if (ls.y <= DD_SPAN) {
                const uint8_t* seg = reinterpret_cast<const uint8_t*>(sbuf[buf][q]);
                const int shift = (int)((t0 + ls.x) & 3);
#pragma unroll
                for (int j = 0; j < DD_DT; ++j) {
                    const int o = shift + dc[j] - ls.x + tid;
#pragma unroll
                    for (int k = 0; k < 4; ++k) acc[k][j] += seg[o + k * DD_NT];
                }
            } else {
                const uint8_t* xc = x + (int64_t)c * ldx;
#pragma unroll
                for (int j = 0; j < DD_DT; ++j) {
                    const int64_t a = t0 + dc[j] + tid;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int64_t t = a + k * DD_NT;
                        acc[k][j] += t < ldx ? xc[t] : 0u;
                    }
                }
            }
        }
        if (grp + 1 < ngrp) stash(buf ^ 1);
        __syncthreads();
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

hipError_t launch_dedisperse(const uint8_t* d_tm, int nbits, uint8_t* d_cm, int nchan, int64_t nsamp, int64_t ldx,
                             const int32_t* d_delay, int ldd, const int2* d_lospan, int ndm, int64_t nout, float* out,
                             hipStream_t s)
{
    if (d_tm) {
        const dim3 tg((unsigned)((ldx + 63) / 64), (unsigned)((nchan + 63) / 64));
        if (nbits == 4)
            hipLaunchKernelGGL(k_fb_transpose<4>, tg, dim3(256), 0, s, d_tm, d_cm, nchan, nsamp, ldx);
        else
            hipLaunchKernelGGL(k_fb_transpose<8>, tg, dim3(256), 0, s, d_tm, d_cm, nchan, nsamp, ldx);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int ntile = ldd / DD_DT;
    const dim3 grid((unsigned)((nout + DD_TT - 1) / DD_TT), (unsigned)ntile);
    hipLaunchKernelGGL(k_dedisperse, grid, dim3(DD_NT), 0, s, d_cm, nchan, ldx, d_delay, ldd, d_lospan, ntile, ndm,
                       nout, out);
    return hipGetLastError();
}

int dedisp_tile() { return DD_DT; }

}  // namespace tb
