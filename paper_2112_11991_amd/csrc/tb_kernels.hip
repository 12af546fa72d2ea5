// tb_kernels.hip -- gfx950 kernels of the per-template coherent orbital
// search (arXiv:2112.11991): Roemer-delay resampling fused into the first FFT
// pass, second FFT pass with the real-to-complex split and power, block
// medians of the whitening, and harmonic sum with threshold and wave-ballot
// compaction of the peaks.
//
// Wave64 throughout; LDS-staged Stockham transforms; no MFMA (nothing here is
// a dense contraction).  Workgroup ids are remapped so that each of the eight
// XCDs (which the hardware feeds round-robin) walks a contiguous range of
// tiles and its L2 sees neighbouring addresses.
#include <hip/hip_runtime.h>

#include "tb_internal.h"

namespace tb {
namespace {

constexpr int NT = 256;   // threads per workgroup
constexpr int PAD = 1;    // LDS column padding (complex elements)

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // -i * a

// The hardware hands workgroup b to XCD b % 8; give XCD x the contiguous
// logical tiles [x*n/8, (x+1)*n/8) of the first 8*floor(n/8) workgroups.
__device__ __forceinline__ int xcd_remap(int bid, int n)
{
    int full = n & ~7;
    if (bid >= full) return bid;
    return (bid & 7) * (full >> 3) + (bid >> 3);
}

// ------------------------------------------------------------------------
// Kepler's equation E - e sin E = M (Sec. 2.1) by Newton from E0 = M, and
// the BT Roemer delay tau[(cos E - e) sin w + sqrt(1-e^2) sin E cos w]
// (App. A.1), all in FP64: absolute sample times reach 2^24 tsamp, where FP32
// would lose the sub-sample delay.
__device__ __forceinline__ double kepler_E(double M, double e)
{
    if (e == 0.0) return M;
    double E = M;
    for (int it = 0; it < 64; ++it) {
        double s, c;
        sincos(E, &s, &c);
        double step = (E - e * s - M) / (1.0 - e * c);
        E -= step;
        if (fabs(step) < 1e-12) break;
    }
    return E;
}

__device__ __forceinline__ double roemer(const TmplDev& p, double t)
{
    double M = p.omega * t + p.alpha;
    double E = kepler_E(M, p.ecc);
    double s, c;
    sincos(E, &s, &c);
    return p.tau * ((c - p.ecc) * p.sinw + p.beta * s * p.cosw);
}

// Input index read by output sample j (Algorithm 1 with the zero offset
// removed): j - nearest_integer((Delta(j tsamp) - Delta(0)) / tsamp).
__device__ __forceinline__ int64_t source_index(const TmplDev& p, int64_t j, double tsamp)
{
    double d = (roemer(p, (double)j * tsamp) - p.d0) / tsamp;
    return j - (int64_t)rint(d);
}

__global__ void k_template_prep(const tb_template* __restrict__ t, uint32_t count, TmplDev* __restrict__ out)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    tb_template a = t[i];
    TmplDev d;
    d.omega = 2.0 * M_PI / a.porb_s;
    d.alpha = a.alpha_rad;
    d.tau = a.tau_lts;
    d.ecc = a.ecc;
    d.sinw = sin(a.omega_rad);
    d.cosw = cos(a.omega_rad);
    d.beta = sqrt(1.0 - a.ecc * a.ecc);
    d.d0 = 0.0;
    d.d0 = roemer(d, 0.0);
    out[i] = d;
}

// ------------------------------------------------------------------------
// Mean removal on load: FP64 partial sums per workgroup, then one workgroup
// adds them in a fixed order and subtracts.
__global__ __launch_bounds__(NT) void k_partial_sum(const float* __restrict__ x, int64_t n,
                                                     double* __restrict__ partial)
{
    __shared__ double red[NT];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        acc += (double)x[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NT) void k_finish_mean(double* __restrict__ partial, int nparts, int64_t n)
{
    __shared__ double red[NT];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += NT) acc += partial[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[nparts] = red[0] / (double)n;
}

__global__ __launch_bounds__(NT) void k_subtract(const float* __restrict__ in, float* __restrict__ out, int64_t n,
                                                  const double* __restrict__ mean)
{
    double m = *mean;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        out[i] = (float)((double)in[i] - m);
}

// Plain streaming copy: the practical HBM ceiling and the reference for
// scaling memory counters.
__global__ __launch_bounds__(NT) void k_copy(float4* __restrict__ dst, const float4* __restrict__ src, size_t count)
{
    for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < count; i += (size_t)gridDim.x * NT) dst[i] = src[i];
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t count)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// ------------------------------------------------------------------------
// Stockham autosort FFT of C columns of length L held in LDS (column c at
// buf + c*LS), forward sign, natural order in and out.  Each stage loads its
// butterflies into registers, synchronises, and writes back, so it runs in
// place.  Twiddles W_L^r come from an FP64-built table.
template <int L>
struct Log2 {
    static constexpr int value = 1 + Log2<L / 2>::value;
};
template <>
struct Log2<1> {
    static constexpr int value = 0;
};

template <int L, int C, int LS>
__device__ __forceinline__ void radix2_first(float2* buf)
{
    constexpr int H = L / 2, NB = C * H, PER = (NB + NT - 1) / NT;
    float2 a[PER], b[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        int bi = threadIdx.x + i * NT;
        if (NB % NT == 0 || bi < NB) {
            int c = bi / H, j = bi % H;
            a[i] = buf[c * LS + j];
            b[i] = buf[c * LS + j + H];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        int bi = threadIdx.x + i * NT;
        if (NB % NT == 0 || bi < NB) {
            int c = bi / H, j = bi % H;
            buf[c * LS + 2 * j] = cadd(a[i], b[i]);
            buf[c * LS + 2 * j + 1] = csub(a[i], b[i]);
        }
    }
    __syncthreads();
}

template <int L, int C, int LS>
__device__ __forceinline__ void radix4_stage(float2* buf, const float2* __restrict__ tw, int ns_log)
{
    constexpr int Q = L / 4, NB = C * Q, PER = (NB + NT - 1) / NT, LG = Log2<L>::value;
    const int Ns = 1 << ns_log;
    float2 v[PER][4];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        int bi = threadIdx.x + i * NT;
        if (NB % NT == 0 || bi < NB) {
            int c = bi / Q, j = bi % Q, k = j & (Ns - 1);
            const float2* src = buf + c * LS + j;
            float2 v0 = src[0], v1 = src[Q], v2 = src[2 * Q], v3 = src[3 * Q];
            if (ns_log > 0) {
                int sh = LG - 2 - ns_log;
                v1 = cmul(v1, tw[k << sh]);
                v2 = cmul(v2, tw[(2 * k) << sh]);
                v3 = cmul(v3, tw[(3 * k) << sh]);
            }
            float2 t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = mul_mi(csub(v1, v3));
            v[i][0] = cadd(t0, t2);
            v[i][1] = cadd(t1, t3);
            v[i][2] = csub(t0, t2);
            v[i][3] = csub(t1, t3);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        int bi = threadIdx.x + i * NT;
        if (NB % NT == 0 || bi < NB) {
            int c = bi / Q, j = bi % Q, k = j & (Ns - 1);
            float2* dst = buf + c * LS + ((j >> ns_log) << (ns_log + 2)) + k;
            dst[0] = v[i][0];
            dst[Ns] = v[i][1];
            dst[2 * Ns] = v[i][2];
            dst[3 * Ns] = v[i][3];
        }
    }
    __syncthreads();
}

template <int L, int C, int LS>
__device__ __forceinline__ void fft_columns(float2* buf, const float2* __restrict__ tw)
{
    constexpr int LG = Log2<L>::value;
    int ns_log = 0;
    if (LG & 1) {
        radix2_first<L, C, LS>(buf);
        ns_log = 1;
    }
    for (; ns_log < LG; ns_log += 2) radix4_stage<L, C, LS>(buf, tw, ns_log);
}

__device__ __forceinline__ float2 twiddle2(const float2* __restrict__ lo, const float2* __restrict__ hi, uint32_t q)
{
    return cmul(hi[q >> TW_LO_BITS], lo[q & ((1u << TW_LO_BITS) - 1)]);
}

// ------------------------------------------------------------------------
// Pass 1: for complex point m = n1 + R*n2 (n1 < R, n2 < S) the packed value
// z_m = y_{2m} + i y_{2m+1} of the demodulated series, y_j = x0[src_j], is
// gathered straight from the resident series; S-point transforms over n2;
// the inter-pass twiddle W_M^{n1 k2}.  Output tile of workgroup w (columns
// n1 in [w*C1, (w+1)*C1)) is the contiguous block Y[w][k2][c].
template <int S, int C1>
__global__ __launch_bounds__(NT) void k_pass1(const float* __restrict__ x, int64_t n, int R, double tsamp,
                                              const TmplDev* __restrict__ tm, float2* __restrict__ Y,
                                              size_t y_stride, const float2* __restrict__ twS,
                                              const float2* __restrict__ twM_lo, const float2* __restrict__ twM_hi,
                                              int32_t* __restrict__ src_out)
{
    constexpr int LS = S + PAD;
    __shared__ float2 buf[C1 * LS];
    const TmplDev p = tm[blockIdx.y];
    const int ntiles = R / C1;
    const int tile = xcd_remap(blockIdx.x, ntiles);
    const int c0 = tile * C1;

    for (int e = threadIdx.x; e < C1 * S; e += NT) {
        int s = e / C1, c = e % C1;
        int64_t j = 2 * ((int64_t)c0 + c + (int64_t)R * s);
        int64_t i0 = source_index(p, j, tsamp);
        int64_t i1 = source_index(p, j + 1, tsamp);
        float y0 = (i0 >= 0 && i0 < n) ? x[i0] : 0.0f;
        float y1 = (i1 >= 0 && i1 < n) ? x[i1] : 0.0f;
        if (src_out) {
            src_out[j] = (int32_t)i0;
            src_out[j + 1] = (int32_t)i1;
        }
        buf[c * LS + s] = make_float2(y0, y1);
    }
    __syncthreads();
    fft_columns<S, C1, LS>(buf, twS);

    float2* out = Y + blockIdx.y * y_stride + (size_t)tile * S * C1;
    for (int e = threadIdx.x; e < C1 * S; e += NT) {
        int k2 = e / C1, c = e % C1;
        uint32_t q = (uint32_t)(c0 + c) * (uint32_t)k2;
        out[e] = cmul(buf[c * LS + k2], twiddle2(twM_lo, twM_hi, q));
    }
}

// Real-to-complex split of the packed transform Z (length M) of a real series
// of length N = 2M: X_k = (Z_k + Z*_{M-k})/2 - i W_N^k (Z_k - Z*_{M-k})/2.
__device__ __forceinline__ float power_of(float2 z, float2 zm, float2 w)
{
    float ax = z.x + zm.x, ay = z.y - zm.y;
    float bx = z.x - zm.x, by = z.y + zm.y;
    float xr = 0.5f * (ax + w.x * by + w.y * bx);
    float xi = 0.5f * (ay - w.x * bx + w.y * by);
    return xr * xr + xi * xi;
}

// Pass 2: workgroup g owns columns k2 in A = [gD, gD+D) and their mirrors
// S - k2 (column 0 pairs with itself, so its mirror slot carries the other
// self-paired column S/2).  R-point transforms over n1 give Z at
// k = k2 + S k1; Z_{M-k} sits in the mirror column at k1' = R-1-k1.
template <int R, int D>
__global__ __launch_bounds__(NT) void k_pass2(const float2* __restrict__ Y, size_t y_stride, int S, int C1,
                                              float* __restrict__ P, size_t p_stride, int64_t M,
                                              const float2* __restrict__ twR, const float2* __restrict__ tw2M_lo,
                                              const float2* __restrict__ tw2M_hi)
{
    constexpr int LS = R + PAD;
    __shared__ float2 buf[2 * D * LS];
    const int ngroups = S / (2 * D);
    const int g = xcd_remap(blockIdx.x, ngroups);
    const float2* Ys = Y + blockIdx.y * y_stride;
    float* Ps = P + blockIdx.y * p_stride;

    for (int e = threadIdx.x; e < 2 * D * R; e += NT) {
        int c = e % C1;
        int q = (e / C1) % (2 * D);
        int w = e / (C1 * 2 * D);
        int col;
        if (q < D) {
            col = g * D + q;
        } else {
            int a = g * D + (q - D);
            col = (a == 0) ? S / 2 : S - a;
        }
        buf[q * LS + w * C1 + c] = Ys[((size_t)w * S + col) * C1 + c];
    }
    __syncthreads();
    fft_columns<R, 2 * D, LS>(buf, twR);

    for (int e = threadIdx.x; e < D * R; e += NT) {
        int d = e % D, k1 = e / D;
        int a = g * D + d;
        if (a == 0) {
            float2 z = buf[k1];
            if (k1 == 0) {
                float s0 = z.x + z.y, sm = z.x - z.y;
                Ps[0] = s0 * s0;
                Ps[M] = sm * sm;
            } else {
                uint32_t k = (uint32_t)S * (uint32_t)k1;
                Ps[k] = power_of(z, buf[R - k1], twiddle2(tw2M_lo, tw2M_hi, k));
            }
            float2 zh = buf[D * LS + k1], zhm = buf[D * LS + R - 1 - k1];
            uint32_t kh = (uint32_t)(S / 2) + (uint32_t)S * (uint32_t)k1;
            Ps[kh] = power_of(zh, zhm, twiddle2(tw2M_lo, tw2M_hi, kh));
        } else {
            float2 za = buf[d * LS + k1];
            float2 zb = buf[(D + d) * LS + R - 1 - k1];
            uint32_t k = (uint32_t)a + (uint32_t)S * (uint32_t)k1;
            float2 w = twiddle2(tw2M_lo, tw2M_hi, k);
            Ps[k] = power_of(za, zb, w);
            // W_N^{M-k} = -conj(W_N^k)
            Ps[M - k] = power_of(zb, za, make_float2(-w.x, w.y));
        }
    }
}

// ------------------------------------------------------------------------
// Whitening block medians: element of rank floor((n_b-1)/2) of bins
// [1 + bW, 1 + bW + n_b), by radix selection on the IEEE bits (powers are
// non-negative, so unsigned order is numeric order).
__global__ __launch_bounds__(NT) void k_median(const float* __restrict__ P, size_t p_stride, int64_t M, int W,
                                               float* __restrict__ med, size_t med_stride)
{
    extern __shared__ uint32_t vals[];
    __shared__ uint32_t hist[256];
    __shared__ uint32_t s_prefix, s_rank;
    const int b = blockIdx.x;
    const float* Ps = P + blockIdx.y * p_stride;
    const int64_t start = 1 + (int64_t)b * W;
    const int cnt = (int)((M - (int64_t)b * W) < W ? (M - (int64_t)b * W) : W);
    for (int i = threadIdx.x; i < cnt; i += NT) vals[i] = __float_as_uint(Ps[start + i]);
    if (threadIdx.x == 0) {
        s_prefix = 0;
        s_rank = (uint32_t)(cnt - 1) / 2;
    }
    uint32_t mask = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
        hist[threadIdx.x] = 0;
        __syncthreads();
        uint32_t prefix = s_prefix;
        for (int i = threadIdx.x; i < cnt; i += NT) {
            uint32_t v = vals[i];
            if ((v & mask) == prefix) atomicAdd(&hist[(v >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t r = s_rank, acc = 0;
            int dd = 0;
            for (; dd < 255; ++dd) {
                if (acc + hist[dd] > r) break;
                acc += hist[dd];
            }
            s_rank = r - acc;
            s_prefix = prefix | ((uint32_t)dd << shift);
        }
        mask |= 255u << shift;
        __syncthreads();
    }
    if (threadIdx.x == 0) med[blockIdx.y * med_stride + b] = __uint_as_float(s_prefix);
}

// ------------------------------------------------------------------------
// Harmonic sum (Sec. 2.1, 16 harmonics) with whitening applied as the
// spectrum is staged, threshold and wave-ballot compaction.
//
// Bin k of fold h adds harmonic m at bin floor((2mk + h)/(2h)); with
// j = 16 m / h that is floor((jk + 8)/16), so an output tile [k0, k0+T)
// needs, for each j = 1..16, the contiguous input run
// [floor((j k0 + 8)/16), floor((j (k0+T-1) + 8)/16)], about 8.5 T bins in
// all.  Each run is loaded once into LDS, whitened P ln2 / m(q) on the way
// (m the linear interpolation between block-median centres), and the folds
// are formed incrementally: fold 2h adds the odd m of the new fold.
constexpr int HT = 1024;                 // output bins per workgroup
constexpr int HSEG = (17 * HT) / 2 + 64; // LDS floats for the 16 runs

__device__ __forceinline__ float whitened(const float* __restrict__ Ps, const float* __restrict__ med, int q,
                                          int W, int nblk, int64_t M)
{
    if (q == 0) return 0.0f;
    // twice the block centres: 2c_b = 2bW + n_b + 1
    int n0 = (int)(M < W ? M : W);
    int two_c0 = n0 + 1;
    int nlast = (int)(M - (int64_t)(nblk - 1) * W);
    int two_cl = 2 * (nblk - 1) * W + nlast + 1;
    int two_q = 2 * q;
    float level;
    if (two_q <= two_c0) {
        level = med[0];
    } else if (two_q >= two_cl) {
        level = med[nblk - 1];
    } else {
        int b = (two_q - (W + 1)) / (2 * W);
        if (b > nblk - 2) b = nblk - 2;
        int two_cb = 2 * b * W + W + 1;
        int two_cn = (b + 1 == nblk - 1) ? two_cl : two_cb + 2 * W;
        float f = (float)(two_q - two_cb) / (float)(two_cn - two_cb);
        level = med[b] + (med[b + 1] - med[b]) * f;
    }
    return level > 0.0f ? (Ps[q] * 0.69314718055994530942f) / level : 0.0f;
}

__global__ __launch_bounds__(NT) void k_harmsum(const float* __restrict__ P, size_t p_stride,
                                                const float* __restrict__ med, size_t med_stride, int64_t M, int W,
                                                int nblk, int tmpl_base, PeakParams pp, uint4* __restrict__ ring,
                                                uint32_t* __restrict__ counter, float* __restrict__ sums_out)
{
    __shared__ float seg[HSEG];
    __shared__ int s_off[17], s_lo[17];
    const int ntile = gridDim.x;
    const int tile = xcd_remap(blockIdx.x, ntile);
    const int k0 = tile * HT;
    const int kend = (int)(((int64_t)k0 + HT - 1) < M ? (int64_t)k0 + HT - 1 : M);
    const float* Ps = P + blockIdx.y * p_stride;
    const float* meds = med + blockIdx.y * med_stride;
    const int jstep = 16 >> (pp.nfold - 1);  // runs needed: multiples of 16/harm_max

    if (threadIdx.x == 0) {
        int off = 0;
        for (int j = jstep; j <= 16; j += jstep) {
            int lo = (j * k0 + 8) >> 4, hi = (j * kend + 8) >> 4;
            s_off[j] = off;
            s_lo[j] = lo;
            off += hi - lo + 1;
        }
    }
    __syncthreads();
    for (int j = jstep; j <= 16; j += jstep) {
        int lo = s_lo[j], len = ((j * kend + 8) >> 4) - lo + 1;
        float* dst = seg + s_off[j];
        for (int i = threadIdx.x; i < len; i += NT) dst[i] = whitened(Ps, meds, lo + i, W, nblk, M);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t tid = pp.first_template_id + (uint32_t)(tmpl_base + (int)blockIdx.y);
    for (int r = 0; r < HT / NT; ++r) {
        int k = k0 + r * NT + threadIdx.x;
        bool in = k <= kend;
        float acc = in ? seg[s_off[16] + k - s_lo[16]] : 0.0f;
        for (int l = 0; l < pp.nfold; ++l) {
            if (l > 0 && in) {
                int h = 1 << l;
                for (int m = 1; m < h; m += 2) {
                    int j = m << (4 - l);
                    acc += seg[s_off[j] + ((j * k + 8) >> 4) - s_lo[j]];
                }
            }
            if (sums_out && in) sums_out[(size_t)l * (M + 1) + k] = acc;
            bool hit = in && k >= pp.klo[l] && k <= pp.khi[l] && acc > pp.thr[l];
            uint64_t mask = __ballot(hit);
            if (mask) {
                int leader = __ffsll((unsigned long long)mask) - 1;
                uint32_t base = 0;
                if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
                base = __shfl(base, leader);
                if (hit) {
                    uint32_t idx = base + (uint32_t)__popcll(mask & below);
                    if (idx < pp.capacity)
                        ring[idx] = make_uint4(tid, (uint32_t)k, (pp.series_id << 8) | (uint32_t)l,
                                               __float_as_uint(acc));
                }
            }
        }
    }
}

// ------------------------------------------------------------------------
template <int S>
constexpr int c1_of()
{
    return (8192 / S) < 16 ? (8192 / S) : 16;
}
template <int R>
constexpr int d_of()
{
    return (4096 / R) < 16 ? (4096 / R) : 16;
}

template <int S>
hipError_t pass1_launch(const Geometry& g, const float* x, double tsamp, const TmplDev* tm, int nslots,
                        const Slots& ws, int32_t* src_out, hipStream_t s)
{
    constexpr int C1 = c1_of<S>();
    dim3 grid(g.R / C1, nslots);
    hipLaunchKernelGGL((k_pass1<S, C1>), grid, dim3(NT), 0, s, x, g.n, g.R, tsamp, tm, ws.Y, ws.y_stride,
                       g.twS, g.twM_lo, g.twM_hi, src_out);
    return hipGetLastError();
}

template <int R>
hipError_t pass2_launch(const Geometry& g, int nslots, const Slots& ws, hipStream_t s)
{
    constexpr int D = d_of<R>();
    dim3 grid(g.S / (2 * D), nslots);
    hipLaunchKernelGGL((k_pass2<R, D>), grid, dim3(NT), 0, s, ws.Y, ws.y_stride, g.S, g.C1, ws.P, ws.p_stride,
                       g.M, g.twR, g.tw2M_lo, g.tw2M_hi);
    return hipGetLastError();
}

}  // namespace

int pass1_columns(int S)
{
    int c = 8192 / S;
    return c < 16 ? c : 16;
}
int pass2_pairs(int R)
{
    int d = 4096 / R;
    return d < 16 ? d : 16;
}
int harmsum_tile() { return HT; }

hipError_t launch_template_prep(const tb_template* t, uint32_t count, TmplDev* out, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_template_prep, dim3((count + 127) / 128), dim3(128), 0, s, t, count, out);
    return hipGetLastError();
}

hipError_t launch_mean_subtract(const float* in, float* out, int64_t n, double* partial, hipStream_t s)
{
    const int parts = 1024;
    hipLaunchKernelGGL(k_partial_sum, dim3(parts), dim3(NT), 0, s, in, n, partial);
    hipLaunchKernelGGL(k_finish_mean, dim3(1), dim3(NT), 0, s, partial, parts, n);
    int64_t blocks = (n + NT - 1) / NT;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_subtract, dim3((unsigned)blocks), dim3(NT), 0, s, in, out, n, partial + parts);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}

hipError_t launch_copy(float4* dst, const float4* src, size_t count, hipStream_t s)
{
    size_t blocks = (count + NT - 1) / NT;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(NT), 0, s, dst, src, count);
    return hipGetLastError();
}

hipError_t launch_wave(const Geometry& g, const float* x, double tsamp, const TmplDev* tm, int tmpl_base,
                       int nslots, const Slots& ws, const PeakParams& pp, uint4* ring, uint32_t* counter,
                       const Inspect& ins, hipStream_t s, hipEvent_t* ev)
{
    hipError_t e;
    const TmplDev* tmw = tm + tmpl_base;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    switch (g.S) {
    case 32: e = pass1_launch<32>(g, x, tsamp, tmw, nslots, ws, ins.src, s); break;
    case 64: e = pass1_launch<64>(g, x, tsamp, tmw, nslots, ws, ins.src, s); break;
    case 128: e = pass1_launch<128>(g, x, tsamp, tmw, nslots, ws, ins.src, s); break;
    case 256: e = pass1_launch<256>(g, x, tsamp, tmw, nslots, ws, ins.src, s); break;
    case 512: e = pass1_launch<512>(g, x, tsamp, tmw, nslots, ws, ins.src, s); break;
    case 1024: e = pass1_launch<1024>(g, x, tsamp, tmw, nslots, ws, ins.src, s); break;
    case 2048: e = pass1_launch<2048>(g, x, tsamp, tmw, nslots, ws, ins.src, s); break;
    case 4096: e = pass1_launch<4096>(g, x, tsamp, tmw, nslots, ws, ins.src, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    switch (g.R) {
    case 16: e = pass2_launch<16>(g, nslots, ws, s); break;
    case 32: e = pass2_launch<32>(g, nslots, ws, s); break;
    case 64: e = pass2_launch<64>(g, nslots, ws, s); break;
    case 128: e = pass2_launch<128>(g, nslots, ws, s); break;
    case 256: e = pass2_launch<256>(g, nslots, ws, s); break;
    case 512: e = pass2_launch<512>(g, nslots, ws, s); break;
    case 1024: e = pass2_launch<1024>(g, nslots, ws, s); break;
    case 2048: e = pass2_launch<2048>(g, nslots, ws, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_median, dim3(g.nblk, nslots), dim3(NT), sizeof(uint32_t) * (size_t)g.W, s, ws.P,
                       ws.p_stride, g.M, g.W, ws.med, ws.med_stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[3], s)) != hipSuccess) return e;
    int ntile = (int)((g.M + 1 + HT - 1) / HT);
    hipLaunchKernelGGL(k_harmsum, dim3(ntile, nslots), dim3(NT), 0, s, ws.P, ws.p_stride, ws.med, ws.med_stride,
                       g.M, g.W, g.nblk, tmpl_base, pp, ring, counter, ins.sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[4], s)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace tb
