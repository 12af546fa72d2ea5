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

#include <algorithm>

#include "tb_internal.h"

namespace tb {
namespace {

constexpr int NT = 256;   // threads per workgroup

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

// The same delay through the App. B series (model 1): sum over k of
// sin(psi) C_k cos kM + cos(psi) S_k sin kM, minus e sin(psi); no Kepler solve.
__device__ __forceinline__ double series_F(const TmplDev& p, double M)
{
    double F = p.ca[0] - p.ecc * p.sinw;
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        double s, c;
        sincos((double)k * M, &s, &c);
        F += p.ca[k] * c + p.sb[k] * s;
    }
    return F;
}

__device__ __forceinline__ double roemer(const TmplDev& p, double t)
{
    double M = p.omega * t + p.alpha;
    if (p.model) return p.tau * series_F(p, M);
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

// Nearest integer of d (ties to even, as rint) for |d| < 2^31: adding
// 1.5 * 2^52 leaves the rounded value in the low mantissa bits.
__device__ __forceinline__ int rint_i32(double d)
{
    const double t = d + 6755399441055744.0;
    return __double2loint(t);
}

__global__ void k_template_prep(const tb_template* __restrict__ t, uint32_t count, TmplDev* __restrict__ out,
                                int model)
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
    d.model = model;
    d.pad = 0;
    double C[8], S[8];
    series_coefficients(a.ecc, C, S);
    d.g5 = 0.0;
    for (int k = 0; k < 8; ++k) {
        d.ca[k] = d.sinw * C[k];
        d.sb[k] = d.cosw * S[k];
        const double k5 = (double)(k * k * k * k * k);
        d.g5 += k5 * (fabs(C[k]) + fabs(S[k]));
    }
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
// LDS-staged Stockham FFTs of C columns of length L (C L = TE <= 16384
// complex points per workgroup, T = TE/16 threads, 16 points per thread).
// Stages are radix 16 (the first one radix 2, 4 or 8 when log2 L is not a
// multiple of 4); each stage reads its butterflies from LDS into registers,
// transforms them there and writes them back in Stockham order, so two LDS
// passes per stage.  Columns are padded by one element every 16 so that the
// strided stores of the early stages spread over the banks.  Forward sign,
// natural order in and out.  Twiddles come from an FP64-built table.
template <int L>
struct Log2 {
    static constexpr int value = 1 + Log2<L / 2>::value;
};
template <>
struct Log2<1> {
    static constexpr int value = 0;
};

__device__ __forceinline__ int pidx(int i) { return i + (i >> 4); }

__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3)
{
    float2 t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = mul_mi(csub(v1, v3));
    v0 = cadd(t0, t2);
    v1 = cadd(t1, t3);
    v2 = csub(t0, t2);
    v3 = csub(t1, t3);
}

template <int RAD>
__device__ __forceinline__ void dft(float2* v);

template <>
__device__ __forceinline__ void dft<2>(float2* v)
{
    float2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
}

template <>
__device__ __forceinline__ void dft<4>(float2* v)
{
    dft4(v[0], v[1], v[2], v[3]);
}

// 8 = 2 x 4: even/odd 4-point transforms joined with W_8^k.
template <>
__device__ __forceinline__ void dft<8>(float2* v)
{
    constexpr float H = 0.70710678118654752440f;
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    o1 = make_float2(H * (o1.x + o1.y), H * (o1.y - o1.x));   // * W8^1
    o2 = mul_mi(o2);                                          // * W8^2
    o3 = make_float2(H * (o3.y - o3.x), -H * (o3.x + o3.y));  // * W8^3
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

// 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2.
template <>
__device__ __forceinline__ void dft<16>(float2* v)
{
    constexpr float C1 = 0.92387953251128675613f, S1 = 0.38268343236508977173f, H = 0.70710678118654752440f;
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // v[n2 + 4 k1] *= W16^(n2 k1)
    v[5] = cmul(v[5], make_float2(C1, -S1));
    v[6] = cmul(v[6], make_float2(H, -H));
    v[7] = cmul(v[7], make_float2(S1, -C1));
    v[9] = cmul(v[9], make_float2(H, -H));
    v[10] = mul_mi(v[10]);
    v[11] = cmul(v[11], make_float2(-H, -H));
    v[13] = cmul(v[13], make_float2(S1, -C1));
    v[14] = cmul(v[14], make_float2(-H, -H));
    v[15] = cmul(v[15], make_float2(-C1, S1));
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // X[k1 + 4 k2] sits in v[4 k1 + k2]: transpose back to natural order
    float2 t[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) t[i] = v[4 * (i & 3) + (i >> 2)];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = t[i];
}

// Radix-16 stage twiddles W_{16 NS}^{r k} (r = 1..15, k < NS) for every
// stride NS = 2, 4, ..., TWST_NS_MAX of a Stockham stage, 15 consecutive
// entries per k and the tables of successive NS back to back.  They depend
// only on NS, so one table serves every transform length.
__device__ __forceinline__ constexpr int twst_offset(int NS) { return 15 * (NS - 2); }

// From stride 32 on, lanes hold so many different k that per-k records would
// spread a wave's load over tens of cache lines; those stages read W^k, W^2k,
// W^4k and W^8k from a table of W_{16 NS}^i (i < 16 NS, consecutive i) and
// form the other eleven powers by products (at most three roundings deep).
constexpr int TWST_RECORDS = 15 * (2 + 4 + 8 + 16);  // record tables of NS = 2..16
__device__ __forceinline__ constexpr int twpow_offset(int NS) { return TWST_RECORDS + 16 * (NS - 32); }

// W_32^r = exp(-2 pi i r / 32), r < 16, as the host's FP64-built stage table
// rounds them to FP32 (the entry for r = 8 keeps cos's 6.1e-17).
__device__ constexpr float kW32c[16] = {
    1.0f, 0.9807852506637573f, 0.9238795042037964f, 0.8314695954322815f, 0.7071067690849304f,
    0.5555702447891235f, 0.3826834261417389f, 0.19509032368659973f, 6.123234262925839e-17f,
    -0.19509032368659973f, -0.3826834261417389f, -0.5555702447891235f, -0.7071067690849304f,
    -0.8314695954322815f, -0.9238795042037964f, -0.9807852506637573f};
__device__ constexpr float kW32s[16] = {
    -0.0f, -0.19509032368659973f, -0.3826834261417389f, -0.5555702447891235f, -0.7071067690849304f,
    -0.8314695954322815f, -0.9238795042037964f, -0.9807852506637573f, -1.0f, -0.9807852506637573f,
    -0.9238795042037964f, -0.8314695954322815f, -0.7071067690849304f, -0.5555702447891235f,
    -0.3826834261417389f, -0.19509032368659973f};

// Stage twiddles of a radix-16 Stockham stage of stride NS: v[r] *= W_{16 NS}^{r k}.
// Stride 2 has k in {0, 1}, whose twiddles are 1 and the constants above: no
// table loads to wait for after the stage's barrier.
template <int RAD, int NS>
__device__ __forceinline__ void stage_twiddle(float2* v, const float2* __restrict__ twst, int k)
{
    if (NS == 2) {
        const bool odd = (k & 1) != 0;
#pragma unroll
        for (int r = 1; r < RAD; ++r)
            v[r] = cmul(v[r], odd ? make_float2(kW32c[r], kW32s[r]) : make_float2(1.0f, -0.0f));
    } else if (NS > 1 && NS < 32) {
        const float2* tw = twst + twst_offset(NS) + 15 * k;
#pragma unroll
        for (int r = 1; r < RAD; ++r) v[r] = cmul(v[r], tw[r - 1]);
    } else if (NS >= 32) {
        const float2* T = twst + twpow_offset(NS);
        float2 w[16];
        w[1] = T[k];
        w[2] = T[2 * k];
        w[4] = T[4 * k];
        w[8] = T[8 * k];
        w[3] = cmul(w[1], w[2]);
        w[5] = cmul(w[1], w[4]);
        w[6] = cmul(w[2], w[4]);
        w[7] = cmul(w[3], w[4]);
#pragma unroll
        for (int r = 9; r < 16; ++r) w[r] = cmul(w[r - 8], w[8]);
#pragma unroll
        for (int r = 1; r < RAD; ++r) v[r] = cmul(v[r], w[r]);
    }
}

// One Stockham stage.  Element addresses are pidx(a) + pidx(b) with a < b's
// stride (both powers of two), which equals pidx(a + b); writing them that way
// leaves one address per butterfly and compile-time offsets for the rest.
template <int L, int C, int RAD, int NS>
__device__ __forceinline__ void fft_stage(float2* lds, const float2* __restrict__ twst)
{
    static_assert(NS == 1 || RAD == 16, "only radix-16 stages carry twiddles");
    constexpr int T = C * L / 16, BPT = 16 / RAD, LR = L / RAD, LSP = L + L / 16 + 1;
    float2 v[16];
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int bi = threadIdx.x + u * T;
        const int c = bi / LR, j = bi % LR, k = j % NS;
        const float2* src = lds + c * LSP + pidx(j);
#pragma unroll
        for (int r = 0; r < RAD; ++r) v[u * RAD + r] = src[pidx(r * LR)];
        stage_twiddle<RAD, NS>(v + u * RAD, twst, k);
        dft<RAD>(v + u * RAD);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int bi = threadIdx.x + u * T;
        const int c = bi / LR, j = bi % LR, k = j % NS;
        float2* dst = lds + c * LSP + pidx((j / NS) * RAD * NS + k);
#pragma unroll
        for (int r = 0; r < RAD; ++r) dst[pidx(r * NS)] = v[u * RAD + r];
    }
    __syncthreads();
}

// Radix-16 stages of strides NS, 16 NS, ... below END.
template <int L, int C, int NS, int END = L>
struct Radix16Stages {
    static __device__ __forceinline__ void run(float2* lds, const float2* __restrict__ twst)
    {
        fft_stage<L, C, 16, NS>(lds, twst);
        Radix16Stages<L, C, NS * 16, END>::run(lds, twst);
    }
};
template <int L, int C, int END>
struct Radix16Stages<L, C, END, END> {
    static __device__ __forceinline__ void run(float2*, const float2* __restrict__) {}
};

// Radix of the first stage of an L-point transform (the rest are radix 16).
template <int L>
struct FirstRadix {
    static constexpr int value = (Log2<L>::value % 4) ? (1 << (Log2<L>::value % 4)) : 16;
};

// First stage (stride 1) from registers: the caller holds the 16 points
// row0 + (L/16) i of column c of the tile, and the points a first-stage
// butterfly joins (L/R0 apart) are all among them, so the butterflies run
// before anything is written; the results go to their Stockham places
// R0 j + r.  A barrier must separate these writes from later reads.
template <int L>
__device__ __forceinline__ void first_stage_from_regs(float2* col_lds, int row0, const float2 (&z)[16])
{
    constexpr int R0 = FirstRadix<L>::value, G = 16 / R0, RS = L / 16;
#pragma unroll
    for (int i = 0; i < G; ++i) {
        float2 a[R0];
#pragma unroll
        for (int r = 0; r < R0; ++r) a[r] = z[i + G * r];
        dft<R0>(a);
        float2* dst = col_lds + pidx((row0 + RS * i) * R0);
#pragma unroll
        for (int r = 0; r < R0; ++r) dst[r] = a[r];  // R0 consecutive points share one padding group
    }
}

// Last stage (stride L/16) of a one-column tile into registers: thread t
// reads points t + (L/16) r and leaves output t + (L/16) r in v[r], the
// points the caller stores next, so the result never returns to LDS.
template <int L>
__device__ __forceinline__ void last_stage_to_regs(const float2* lds, const float2* __restrict__ twst, float2 (&v)[16])
{
    constexpr int NS = L / 16;
    const int k = threadIdx.x;
    const float2* src = lds + pidx(k);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = src[pidx(r * NS)];
    stage_twiddle<16, NS>(v, twst, k);
    dft<16>(v);
}

template <int L, int C>
__device__ __forceinline__ void fft_tile(float2* lds, const float2* __restrict__ twst)
{
    constexpr int R0 = FirstRadix<L>::value;
    static_assert(L / 16 <= TWST_NS_MAX, "stage twiddle table too short");
    fft_stage<L, C, R0, 1>(lds, twst);
    Radix16Stages<L, C, R0>::run(lds, twst);
}

__device__ __forceinline__ float2 twiddle2(const float2* __restrict__ lo, const float2* __restrict__ hi, uint32_t q)
{
    return cmul(hi[q >> TW_LO_BITS], lo[q & ((1u << TW_LO_BITS) - 1)]);
}

// ------------------------------------------------------------------------
// Local delay expansion.  A thread's 16 consecutive points of a pass-1 tile
// cover a short run of sample indices; around its midpoint j_c the delay
// delta(j) = (Delta(j tsamp) - Delta(0)) / tsamp is expanded to fourth order
// in u = j - j_c from the exact Kepler solution there and the analytic
// derivatives of the BT delay (App. A.1) with respect to the mean anomaly
// (Faa di Bruno, q = E' = 1/(1 - e cos E)):
//   E'' = -e sE q^3,  E''' = -e cE q^4 + 3 e^2 sE^2 q^5,
//   E'''' = e sE q^5 + 10 e^2 sE cE q^6 - 15 e^3 sE^3 q^7.
// The remainder is at most A W'^5 g5(e) U^5 / 120 samples (A = tau/tsamp,
// W' = Omega tsamp, U the largest |u|, |F^(5)| <= g5 = 3 (1+e)^2/(1-e)^9);
// when that exceeds 1e-11 the delay is solved exactly at every sample.
struct DelayPoly {
    double c0, c1, c2, c3, c4;
};

__device__ __forceinline__ bool poly_ok(const TmplDev& p, double tsamp, double U)
{
    const double A = p.tau / tsamp, Wp = p.omega * tsamp, e = p.ecc, om = 1.0 - e;
    const double om3 = om * om * om;
    // |F^(5)| in M: the BT bound, or sum k^5 (|C_k| + |S_k|) for the series
    const double g5 = p.model ? p.g5 : 3.0 * (1.0 + e) * (1.0 + e) / (om3 * om3 * om3);
    const double w5 = Wp * Wp * Wp * Wp * Wp, u5 = U * U * U * U * U;
    return A * w5 * g5 * u5 / 120.0 <= 1e-11;
}

// Series model: F^(m)(M) = sum_k k^m [a_k cos^(m)(kM) + b_k sin^(m)(kM)] with
// a_k = sin(psi) C_k, b_k = cos(psi) S_k.
__device__ __forceinline__ void series_derivatives(const TmplDev& p, double M, double (&F)[5])
{
    F[0] = p.ca[0] - p.ecc * p.sinw;
    F[1] = F[2] = F[3] = F[4] = 0.0;
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        double s, c;
        sincos((double)k * M, &s, &c);
        const double a = p.ca[k], b = p.sb[k], kk = (double)k;
        const double ac = a * c, as = a * s, bc = b * c, bs = b * s;
        F[0] += ac + bs;
        F[1] += kk * (bc - as);
        F[2] -= kk * kk * (ac + bs);
        F[3] += kk * kk * kk * (as - bc);
        F[4] += kk * kk * kk * kk * (ac + bs);
    }
}

__device__ __forceinline__ DelayPoly delay_poly(const TmplDev& p, double tsamp, int64_t jc)
{
    const double e = p.ecc;
    const double M = p.omega * ((double)jc * tsamp) + p.alpha;
    const double w = p.omega, ts = tsamp;
    DelayPoly r;
    if (p.model) {
        double F[5];
        series_derivatives(p, M, F);
        r.c0 = (p.tau * F[0] - p.d0) / ts;
        r.c1 = p.tau * w * F[1];
        r.c2 = p.tau * w * w * ts * F[2] * 0.5;
        r.c3 = p.tau * w * w * w * ts * ts * F[3] * (1.0 / 6.0);
        r.c4 = p.tau * w * w * w * w * ts * ts * ts * F[4] * (1.0 / 24.0);
        return r;
    }
    const double E = kepler_E(M, e);
    double sE, cE;
    sincos(E, &sE, &cE);
    const double F = (cE - e) * p.sinw + p.beta * sE * p.cosw;
    const double FE = -sE * p.sinw + p.beta * cE * p.cosw;
    const double FEE = -cE * p.sinw - p.beta * sE * p.cosw;
    const double q = 1.0 / (1.0 - e * cE), q2 = q * q, q3 = q2 * q, q4 = q2 * q2;
    const double E1 = q;
    const double E2 = -e * sE * q3;
    const double E3 = -e * cE * q4 + 3.0 * e * e * sE * sE * q4 * q;
    const double E4 = e * sE * q4 * q + 10.0 * e * e * sE * cE * q3 * q3 - 15.0 * e * e * e * sE * sE * sE * q4 * q3;
    // F_EEE = -F_E, F_EEEE = -F_EE
    const double F1 = FE * E1;
    const double F2 = FEE * E1 * E1 + FE * E2;
    const double F3 = -FE * E1 * E1 * E1 + 3.0 * FEE * E1 * E2 + FE * E3;
    const double F4 = -FEE * E1 * E1 * E1 * E1 - 6.0 * FE * E1 * E1 * E2 + FEE * (3.0 * E2 * E2 + 4.0 * E1 * E3) +
                      FE * E4;
    r.c0 = (p.tau * F - p.d0) / ts;
    r.c1 = p.tau * w * F1;
    r.c2 = p.tau * w * w * ts * F2 * 0.5;
    r.c3 = p.tau * w * w * w * ts * ts * F3 * (1.0 / 6.0);
    r.c4 = p.tau * w * w * w * w * ts * ts * ts * F4 * (1.0 / 24.0);
    return r;
}

__device__ __forceinline__ int64_t source_from_poly(const DelayPoly& d, int64_t j, int64_t jc)
{
    const double u = (double)(j - jc);
    const double dl = d.c0 + u * (d.c1 + u * (d.c2 + u * (d.c3 + u * d.c4)));
    return j - (int64_t)rint(dl);
}

// ------------------------------------------------------------------------
// Resident series layout.  The mean-removed series is stored as complex
// pairs z_m = (x_2m, x_2m+1) in the tile order of pass 1: point m = n1 + R s
// (n1 < R, s < S) sits at ((n1 / C1) (S + P) + P + s) C1 + n1 % C1, so each
// block of C1 columns runs down all S rows and is followed by P zero rows,
// and P zero rows precede the first block.  Pass-1 workgroup w reads columns
// n1 in [w C1, (w+1) C1) down all rows; a delayed read lands in the same or
// a neighbouring column a few rows away, so consecutive lanes (consecutive
// rows) read neighbouring pairs, and the two samples of a point usually share
// one pair.  A sample index outside [0, n) by less than P - 1 rows (2R
// samples each) falls on zero rows, so the gather needs no range test: it
// works on i' = i + 2PR >= 0, which has the same column n1 and parity as i and
// row s + P.
__device__ __forceinline__ uint32_t bit_insert_low(uint32_t hi, uint32_t lo)
{
    uint32_t r;  // (hi & ~1) | (lo & 1)
    asm("v_bfi_b32 %0, 1, %1, %2" : "=v"(r) : "v"(lo), "v"(hi));
    return r;
}

template <int C1>
__device__ __forceinline__ uint32_t padded_index(uint32_t ip, int lgR, uint32_t SP)
{
    constexpr int LC = Log2<C1>::value;
    const uint32_t n1 = __builtin_amdgcn_ubfe(ip, 1u, (uint32_t)lgR);
    if constexpr (C1 == 1) {
        // float offset 2 (n1 (S + P) + s + P) + parity; i' >> lgR is
        // 2 (s + P) plus one bit of n1, replaced by the parity
        return __umul24(n1, 2 * SP) + bit_insert_low(ip >> lgR, ip);
    } else {
        const uint32_t blk = __umul24(n1 >> LC, SP) + (ip >> (lgR + 1));
        return (((blk << LC) | (n1 & (C1 - 1))) << 1) | (ip & 1u);
    }
}

// Sample at shifted index i' (see above; zero outside the series); the load
// uses a 32-bit byte offset from the series base.
template <int C1>
__device__ __forceinline__ float load_sample(const float* __restrict__ x, int ip, int lgR, uint32_t SP)
{
    const uint32_t a = padded_index<C1>((uint32_t)ip, lgR, SP);
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(x) + (a << 2));
}

// Pass-1 gather for templates whose delay polynomial would not meet the
// accuracy bound: Kepler solve at every sample, written straight to the tile.
// Kept out of line so that its FP64 code does not crowd the common path.
// Any delay: indices outside the series read element 0, a zero row.
template <int S, int C1>
__device__ __attribute__((noinline)) void gather_exact(const float* __restrict__ x, int n, int c0, int R, int lgR,
                                                       int P, double tsamp, const TmplDev* __restrict__ tp,
                                                       float2* lds, int32_t* __restrict__ src_out)
{
    constexpr int T = C1 * S / 16, LSP = S + S / 16 + 1;
    const TmplDev& p = *tp;
    const uint32_t SP = (uint32_t)(S + P);
    const int jsh = 2 * P * R;
#pragma unroll 1
    for (int e = threadIdx.x; e < C1 * S; e += T) {
        const int j = 2 * (c0 + (e % C1) + R * (e / C1));
        const int i0 = (int)source_index(p, j, tsamp), i1 = (int)source_index(p, j + 1, tsamp);
        const uint32_t a0 = (unsigned)i0 < (unsigned)n ? padded_index<C1>(i0 + jsh, lgR, SP) : 0u;
        const uint32_t a1 = (unsigned)i1 < (unsigned)n ? padded_index<C1>(i1 + jsh, lgR, SP) : 0u;
        if (src_out) {
            src_out[j] = i0;
            src_out[j + 1] = i1;
        }
        lds[(e % C1) * LSP + pidx(e / C1)] = make_float2(x[a0], x[a1]);
    }
}

// Natural order -> the padded tile order above (the zero rows are cleared
// beforehand).
__global__ __launch_bounds__(NT) void k_tile_series(const float* __restrict__ in, float* __restrict__ out, int64_t M,
                                                    int lgR, int S, int C1, int P)
{
    for (int64_t m = (int64_t)blockIdx.x * NT + threadIdx.x; m < M; m += (int64_t)gridDim.x * NT) {
        const int64_t n1 = m & ((1ll << lgR) - 1), s = m >> lgR;
        const int64_t d = ((n1 / C1) * (S + P) + P + s) * C1 + (n1 % C1);
        reinterpret_cast<float2*>(out)[d] = reinterpret_cast<const float2*>(in)[m];
    }
}

// Delay polynomials of a template, shared by every pass-1 workgroup.  Tile
// points are grouped in chunks of 16 consecutive points e (row s = e / C1,
// column c = e % C1), or of 8 when 16 would miss the accuracy bound; in the
// tile of column offset c0, point e carries the samples j = 2 (c0 + c + R s)
// and j + 1.  Chunk g is expanded around the middle sample jmid of its
// samples in the tile with c0 = 0; a tile with another offset evaluates the
// same polynomial at u = j - jmid, at most 2 (R - C1) further out, and the
// accuracy bound covers that full reach.  Every chunk of a size spans the
// same samples, so one word per template gives log2 of the chunk size used
// (4 or 3), or 0 for the exact per-sample solve.
__global__ __launch_bounds__(NT) void k_chunk_polys(const TmplDev* __restrict__ tm, double tsamp, int R, int C1,
                                                    int P, int64_t n, int npts, ChunkPoly* __restrict__ polys,
                                                    size_t poly_stride, int32_t* __restrict__ pok)
{
    const int g = (int)(blockIdx.x * NT + threadIdx.x);
    const TmplDev p = tm[blockIdx.y];
    auto jof = [&](int e) -> int { return 2 * (e % C1 + R * (e / C1)); };
    auto reach = [&](int len) -> double {
        const int lo = jof(0), hi = jof(len - 1) + 1, mid = lo + (hi - lo) / 2;
        return (double)(hi - mid) + 2.0 * (double)(R - C1);
    };
    // Delay swing: delta is taken relative to sample 0, so over the n samples
    // |delta| <= tau min(2 max|F|, Omega n tsamp max|dF/dM|) / tsamp; for the
    // BT delay max|F| <= 1 + e and max|dF/dM| <= 1 / (1 - e), for the series
    // the sums of |coefficient| and k |coefficient|.  A swing that could leave
    // the zero rows of the resident series takes the exact path, which tests
    // every index.
    double fmax = 1.0 + p.ecc, dfmax = 1.0 / (1.0 - p.ecc);
    if (p.model) {
        fmax = fabs(p.ca[0] - p.ecc * p.sinw);
        dfmax = 0.0;
        for (int k = 1; k < 8; ++k) {
            fmax += fabs(p.ca[k]) + fabs(p.sb[k]);
            dfmax += k * (fabs(p.ca[k]) + fabs(p.sb[k]));
        }
    }
    const double swing = p.tau * fmin(2.0 * fmax, p.omega * (double)n * tsamp * dfmax) / tsamp;
    const bool in_pad = swing + 1.0 <= 2.0 * (double)R * (double)(P - 1);
    const int shift = !in_pad ? 0 : poly_ok(p, tsamp, reach(16)) ? 4 : poly_ok(p, tsamp, reach(8)) ? 3 : 0;
    if (g == 0) pok[blockIdx.y] = shift;
    if (shift == 0 || g >= (npts >> shift)) return;
    const int len = 1 << shift;
    const int lo = jof(len * g), hi = jof(len * g + len - 1) + 1, mid = lo + (hi - lo) / 2;
    const DelayPoly d = delay_poly(p, tsamp, mid);
    ChunkPoly c;
    c.c0 = d.c0;
    c.c1 = d.c1;
    c.c2 = d.c2;
    c.c3 = d.c3;
    c.c4 = d.c4;
    c.jmid = mid + 2 * P * R;  // in the shifted indices of the gather
    c.pad = 0;
    polys[blockIdx.y * poly_stride + g] = c;
}

// ------------------------------------------------------------------------
// Pass 1: for complex point m = n1 + R*n2 (n1 < R, n2 < S) the packed value
// z_m = y_{2m} + i y_{2m+1} of the demodulated series, y_j = x0[src_j], is
// gathered straight from the resident series; S-point transforms over n2;
// the inter-pass twiddle W_M^{n1 k2}.  Workgroup w owns columns
// n1 in [w C1, (w+1) C1) and writes them as the contiguous block Y[w][k2][c].
// Thread t handles points e = t + T i (i < 16): column t % C1, row
// t / C1 + (S/16) i, so a wave's loads are consecutive rows.
template <int S, int C1>
__global__ __launch_bounds__(C1 * S / 16, 4) void k_fft1(const float* __restrict__ x, int64_t n, int R, int lgR,
                                                      int P, double tsamp, const TmplDev* __restrict__ tm,
                                                      const ChunkPoly* __restrict__ polys, size_t poly_stride,
                                                      const int32_t* __restrict__ pok,
                                                      float2* __restrict__ Y, size_t y_stride,
                                                      const float2* __restrict__ twst,
                                                      const float2* __restrict__ twM_lo,
                                                      const float2* __restrict__ twM_hi, int32_t* __restrict__ src_out)
{
    constexpr int T = C1 * S / 16, LSP = S + S / 16 + 1, RS = S / 16;
    __shared__ __align__(16) float2 lds[C1 * LSP];
    static_assert(sizeof(ChunkPoly) * 2 * T <= sizeof(float2) * C1 * LSP, "polynomials must fit in the tile");
    static_assert(T % 16 == 0, "chunks of 16 points must not straddle a thread's rows");
    const int tile = xcd_remap(blockIdx.x, R / C1);
    const int c0 = tile * C1;
    const int c = (int)threadIdx.x % C1, row0 = (int)threadIdx.x / C1;
    const uint32_t n32 = (uint32_t)n;

    const int shift = pok[blockIdx.y];  // log2 points per polynomial chunk, 0 = exact solve
    float2 zv[16];  // points row0 + RS i of column c
    if (shift) {
        // Sample indices fit in 32 bits: n <= 2^24 and the host bounds the delay;
        // this path's delays stay within the zero rows (checked per template).
        // The template's chunk polynomials (T of them for 16-point chunks, 2T
        // for 8-point ones) are parked in the (not yet used) tile memory, so
        // that their reads wait on LDS only and the series loads of earlier
        // points stay in flight.
        ChunkPoly* cp = reinterpret_cast<ChunkPoly*>(lds);
        for (int c = (int)threadIdx.x; c < (C1 * S) >> shift; c += T) cp[c] = polys[blockIdx.y * poly_stride + c];
        __syncthreads();
        // Indices are shifted by P rows (jsh samples), the chunk centres too.
        // T is a multiple of 16, so point t + T i lies in chunk
        // (t >> shift) + i (T >> shift).
        const int jsh = 2 * P * R;
        const int jbase = 2 * (c0 + c + R * row0) + jsh, jstep = 2 * R * RS;
        const ChunkPoly* cpt = cp + ((int)threadIdx.x >> shift);
        const int cstep = T >> shift;
        auto sources = [&](int i, int& jp, int& ip0, int& ip1) {
            const ChunkPoly d = cpt[i * cstep];
            jp = jbase + i * jstep;
            const double u = (double)(jp - d.jmid), u1 = u + 1.0;
            const double d0 = d.c0 + u * (d.c1 + u * (d.c2 + u * (d.c3 + u * d.c4)));
            const double d1 = d.c0 + u1 * (d.c1 + u1 * (d.c2 + u1 * (d.c3 + u1 * d.c4)));
            ip0 = jp - rint_i32(d0);
            ip1 = jp + 1 - rint_i32(d1);
        };
        const uint32_t SP = (uint32_t)(S + P);
        float v[32];
        // The gather's waves issue at raised priority, so that a CU's other
        // workgroup, busy with its transform, yields issue slots until these
        // loads are in flight.
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            int jp, ip0, ip1;
            sources(i, jp, ip0, ip1);
            v[2 * i] = load_sample<C1>(x, ip0, lgR, SP);
            v[2 * i + 1] = load_sample<C1>(x, ip1, lgR, SP);
        }
        __builtin_amdgcn_s_setprio(0);
        if (src_out) {
            for (int i = 0; i < 16; ++i) {
                int jp, ip0, ip1;
                sources(i, jp, ip0, ip1);
                src_out[jp - jsh] = ip0 - jsh;
                src_out[jp - jsh + 1] = ip1 - jsh;
            }
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) zv[i] = make_float2(v[2 * i], v[2 * i + 1]);
    } else {
        // the exact gather fills the tile in natural order; each thread
        // takes back its own points
        gather_exact<S, C1>(x, (int)n32, c0, R, lgR, P, tsamp, tm + blockIdx.y, lds, src_out);
        __syncthreads();
        const float2* own = lds + c * LSP + pidx(row0);
#pragma unroll
        for (int i = 0; i < 16; ++i) zv[i] = own[pidx(RS * i)];
    }
    __syncthreads();  // the polynomials (or the exact gather's tile) are no longer read
    first_stage_from_regs<S>(lds + c * LSP, row0, zv);
    __syncthreads();

    // W_M^{(c0+c) k2} for k2 = row0 + RS i: start value times W_M^{(c0+c) RS}
    // per step (a recurrence of at most 15 products).
    float2* out = Y + blockIdx.y * y_stride + (size_t)tile * S * C1 + threadIdx.x;
    const uint32_t col = (uint32_t)(c0 + c);
    float2 w = twiddle2(twM_lo, twM_hi, col * (uint32_t)row0);
    const float2 z = twiddle2(twM_lo, twM_hi, col * (uint32_t)RS);
    if constexpr (C1 == 1) {
        // the last stage leaves each thread exactly the points it stores
        Radix16Stages<S, 1, FirstRadix<S>::value, S / 16>::run(lds, twst);
        float2 y[16];
        last_stage_to_regs<S>(lds, twst, y);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            out[i * T] = cmul(y[i], w);
            w = cmul(w, z);
        }
    } else {
        Radix16Stages<S, C1, FirstRadix<S>::value>::run(lds, twst);
        const float2* src = lds + c * LSP + pidx(row0);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            out[i * T] = cmul(src[pidx(RS * i)], w);
            w = cmul(w, z);
        }
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

// Pass 2: workgroup g owns the D2/2 columns k2 in A = [g D, g D + D) and
// their mirrors S - k2 (column 0 pairs with itself, so its mirror slot
// carries the other self-paired column S/2).  R-point transforms over n1 give
// Z at k = k2 + S k1, and Z_{M-k} sits in the mirror slot at k1' = R-1-k1
// (in column 0 at (R - k1) mod R).  Each slot emits |X|^2 for its own bins:
// runs of D consecutive bins per k1, ascending for A, descending for mirrors.
//
// When every pass-1 workgroup held one column (C1 = 1, R > 16), thread t
// loads slot q = t % D2 of blocks w = t / D2 + RK i, so all of its addresses
// are a per-thread base plus compile-time steps; other geometries take the
// general index arithmetic.  Thread t emits bins k1 = t / D2 + RK i of slot q.
//
// With fac (a series whitened once, bins 0..M like one power row), every bin
// is stored as |X_k|^2 fac_k, the whitened power; without it fac_k = 1 and
// the raw power is stored.  The factors are loaded before the transform so
// that their latency hides behind it.
template <int R, int D2>
__global__ __launch_bounds__(D2 * R / 16) void k_fft2(const float2* __restrict__ Y, size_t y_stride, int S, int lgS,
                                                      int lgC1, float* __restrict__ P, size_t p_stride, int64_t M,
                                                      const float2* __restrict__ twst,
                                                      const float2* __restrict__ tw2M_lo,
                                                      const float2* __restrict__ tw2M_hi,
                                                      const float* __restrict__ fac)
{
    constexpr int T = D2 * R / 16, LSP = R + R / 16 + 1, D = D2 / 2, RK = R / 16, LD2 = Log2<D2>::value;
    // R > 16 with one pass-1 column per workgroup (the plan's geometries)
    const bool one_column = R > 16 && lgC1 == 0;
    __shared__ float2 lds[D2 * LSP];
    const int g = xcd_remap(blockIdx.x, S / D2);
    const float2* Ys = Y + blockIdx.y * y_stride;
    float* Ps = P + blockIdx.y * p_stride;
    const int q = (int)threadIdx.x & (D2 - 1), k1t = (int)threadIdx.x >> LD2;
    const int a = g * D + (q < D ? q : q - D);
    const int col = q < D ? a : (a == 0 ? S / 2 : S - a);

    float2 v[16];
    if (one_column) {
        // element i: block w = k1t + RK i, column col (the first stage runs
        // on these registers below)
        const uint32_t off0 = ((((uint32_t)k1t << lgS) + (uint32_t)col) << 3);
        const uint32_t step = (uint32_t)RK << (lgS + 3);
#pragma unroll
        for (int i = 0; i < 16; ++i)
            v[i] = *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(Ys) + (off0 + step * (uint32_t)i));
    } else {
        // element e = (w, q, c): block w of pass 1, slot q, column c (C1 = 2^lgC1)
        const int cmask = (1 << lgC1) - 1;
        int laddr[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = (int)threadIdx.x + i * T;
            const int c = e & cmask, qe = (e >> lgC1) & (D2 - 1), w = e >> (lgC1 + LD2);
            const int ae = g * D + (qe < D ? qe : qe - D);
            const int cole = qe < D ? ae : (ae == 0 ? S / 2 : S - ae);
            const uint32_t src = ((((uint32_t)w << lgS) + (uint32_t)cole) << lgC1) | (uint32_t)c;
            v[i] = Ys[src];
            laddr[i] = qe * LSP + pidx((w << lgC1) | c);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) lds[laddr[i]] = v[i];
    }
    const uint32_t soff0 = ((uint32_t)col + ((uint32_t)k1t << lgS)) << 2;
    const uint32_t sstep = (uint32_t)RK << (lgS + 2);
    float fv[16];
    if (fac) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            fv[i] = *reinterpret_cast<const float*>(reinterpret_cast<const char*>(fac) + (soff0 + sstep * (uint32_t)i));
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) fv[i] = 1.0f;
    }
    if (one_column) {
        first_stage_from_regs<R>(lds + q * LSP, k1t, v);
        __syncthreads();
        Radix16Stages<R, D2, FirstRadix<R>::value>::run(lds, twst);
    } else {
        __syncthreads();
        fft_tile<R, D2>(lds, twst);
    }

    // Thread t emits slot q at k1 = k1t + RK i.  The split twiddle
    // W_2M^{col + S k1} advances by W_2M^{S RK} = W_32 per step.
    const int pq = (a == 0) ? q : (q < D ? q + D : q - D);
    const bool self = q < D && a == 0;  // column 0: Z_{M-k} at k1' = (R - k1) mod R
    float2 w = twiddle2(tw2M_lo, tw2M_hi, (uint32_t)col + (uint32_t)S * (uint32_t)k1t);
    const float2 z = make_float2(0.98078528040323044913f, -0.19509032201612826785f);
    auto store = [&](int i, float v) {
        *reinterpret_cast<float*>(reinterpret_cast<char*>(Ps) + (soff0 + sstep * (uint32_t)i)) = v * fv[i];
    };
    if (self && k1t == 0) {
        // bins k1 = RK i of column 0; bin 0 pairs with itself, and the
        // Nyquist bin M comes from Z_0 as well
        const float2* own = lds + q * LSP;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int k1 = RK * i;
            const float2 zo = own[pidx(k1)];
            const float2 zm = own[pidx((R - k1) & (R - 1))];
            store(i, power_of(zo, zm, w));
            w = cmul(w, z);
            if (i == 0) {
                const float sm = zo.x - zo.y;
                Ps[M] = sm * sm * (fac ? fac[M] : 1.0f);
            }
        }
    } else {
        // mirror index R-1-k1 (R-k1 in column 0) = RK (15 - i) + m0 with m0 < RK
        const int m0 = self ? RK - k1t : RK - 1 - k1t;
        const float2* own = lds + q * LSP + pidx(k1t);
        const float2* mir = lds + pq * LSP + pidx(m0);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float2 zo = own[pidx(RK * i)];
            const float2 zm = mir[pidx(RK * (15 - i))];
            store(i, power_of(zo, zm, w));
            w = cmul(w, z);
        }
    }
}

// ------------------------------------------------------------------------
// Whitening block medians: element of rank floor((n_b-1)/2) of bins
// [1 + bW, 1 + bW + n_b), by radix selection on the IEEE bits (powers are
// non-negative, so unsigned order is numeric order).  Three digits: bits
// 30..20 (the exponent and three mantissa bits, so that the few exponents a
// block spans spread over many histogram bins), then 19..10 and 9..0.  The
// block's values stay in registers (VPT per thread).  Counting uses LDS
// atomics into one histogram (NC copies are summed; one measured fastest:
// the smaller LDS footprint and clearing outweigh the extra contention);
// thread t owns the NBIN/NT consecutive bins from t NBIN/NT on, sums and
// clears them, and a block-wide prefix sum over the threads finds the digit
// holding the rank.
constexpr int MED_BINS = 2048;  // first-digit histogram (bits 30..20)

// Lower median (rank floor((cnt-1)/2)) of a block's values v (IEEE bits,
// absent entries 0xffffffff), by the three-digit radix selection above.
// Every thread of the workgroup calls it and gets the median.  hist must be
// zero on entry and is zero again on return (every pass clears the bins it
// sums, and later passes only count into bins the first one cleared).
template <int VPT>
__device__ __forceinline__ float block_median(const uint32_t (&v)[VPT], int cnt, uint32_t* hist, uint32_t* wsum,
                                              uint32_t& s_digit, uint32_t& s_rank)
{
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t rank = (uint32_t)(cnt - 1) / 2, prefix = 0, mask = 0x80000000u;
#pragma unroll
    for (int pass = 0; pass < 3; ++pass) {
        const int shift = pass == 0 ? 20 : pass == 1 ? 10 : 0;
        const int nbin = pass == 0 ? MED_BINS : 1024;
        const uint32_t dmask = (uint32_t)nbin - 1;
        const int per = nbin / NT;  // bins per thread: 8, then 4
        if (pass == 0 && cnt == VPT * NT) {
            // a whole block: every value counts in the first digit, with no
            // per-value predicate
#pragma unroll
            for (int i = 0; i < VPT; ++i) atomicAdd(&hist[(v[i] >> shift) & dmask], 1u);
        } else {
#pragma unroll
            for (int i = 0; i < VPT; ++i)
                if ((v[i] & mask) == prefix) atomicAdd(&hist[(v[i] >> shift) & dmask], 1u);
        }
        __syncthreads();
        uint32_t cnts[8];
        uint32_t tot = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            cnts[k] = 0;
            if (k < per) {
                const int bin = (int)threadIdx.x * per + k;
                cnts[k] = hist[bin];
                hist[bin] = 0;
                tot += cnts[k];
            }
        }
        uint32_t inc = tot;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(inc, d);
            if (lane >= d) inc += o;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        uint32_t excl = inc - tot;
#pragma unroll
        for (int w = 0; w < NW; ++w)
            if (w < wave) excl += wsum[w];
        if (excl <= rank && rank < excl + tot) {
            uint32_t run = excl;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (k < per && cnts[k] && run <= rank && rank < run + cnts[k]) {
                    s_digit = (uint32_t)((int)threadIdx.x * per + k);
                    s_rank = rank - run;
                }
                run += cnts[k];
            }
        }
        __syncthreads();
        prefix |= s_digit << shift;
        mask |= dmask << shift;
        rank = s_rank;
    }
    return __uint_as_float(prefix);
}

// The values of block b (bins [1 + bW, 1 + bW + n_b)): thread t holds bins
// t + NT i; absent entries get the largest key, which never matches a prefix
// of a real one.  Returns n_b.
template <int VPT>
__device__ __forceinline__ int load_block(const float* __restrict__ Ps, int64_t M, int W, int b, uint32_t (&v)[VPT])
{
    const int64_t start = 1 + (int64_t)b * W;
    const int cnt = (int)((M - (int64_t)b * W) < W ? (M - (int64_t)b * W) : W);
    if (cnt == VPT * NT) {
        const float* row = Ps + start + threadIdx.x;
#pragma unroll
        for (int i = 0; i < VPT; ++i) v[i] = __float_as_uint(row[i * NT]);
        return cnt;
    }
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
        const int q = (int)threadIdx.x + i * NT;
        v[i] = q < cnt ? __float_as_uint(Ps[start + q]) : 0xffffffffu;
    }
    return cnt;
}

// Whitening block medians: element of rank floor((n_b-1)/2) of bins
// [1 + bW, 1 + bW + n_b), by radix selection on the IEEE bits (powers are
// non-negative, so unsigned order is numeric order).  Three digits: bits
// 30..20 (the exponent and three mantissa bits, so that the few exponents a
// block spans spread over many histogram bins), then 19..10 and 9..0.  The
// block's values stay in registers (VPT per thread).  Counting uses LDS
// atomics into one histogram (copies per wave measured slower: the smaller
// LDS footprint and clearing outweigh the extra contention); thread t owns
// the NBIN/NT consecutive bins from t NBIN/NT on, sums and clears them, and a
// block-wide prefix sum over the threads finds the digit holding the rank.
template <int VPT>
__global__ __launch_bounds__(NT) void k_median(const float* __restrict__ P, size_t p_stride, int64_t M, int W,
                                               float* __restrict__ med, size_t med_stride)
{
    __shared__ uint32_t hist[MED_BINS];
    __shared__ uint32_t wsum[NT / 64];
    __shared__ uint32_t s_digit, s_rank;
    uint32_t v[VPT];
    const int cnt = load_block<VPT>(P + blockIdx.y * p_stride, M, W, blockIdx.x, v);
#pragma unroll
    for (int i = 0; i < MED_BINS / NT; ++i) hist[threadIdx.x + i * NT] = 0;
    __syncthreads();
    const float m = block_median<VPT>(v, cnt, hist, wsum, s_digit, s_rank);
    if (threadIdx.x == 0) med[blockIdx.y * med_stride + blockIdx.x] = m;
}

// Whitening: P^_k = P_k ln2 / m(k), m the straight line between neighbouring
// block-median centres c_b = start_b + (n_b - 1)/2, held constant before the
// first and after the last centre; P^_0 = 0.  One workgroup per block.
// Centres are kept doubled so that they stay integers (below 2^24, so exact
// in FP32); the line is evaluated as m_left + slope (2q - 2c_left).
struct WhitenLine {
    int start, cnt;
    float s_l, s_r, base_l, ml0, fc, m_here;
    __device__ __forceinline__ float level(int q) const
    {
        const float x = (float)(2 * q);
        return x < fc ? fmaf(s_l, x - base_l, ml0) : fmaf(s_r, x - fc, m_here);
    }
};

// The line of block b from its own median and its neighbours' (m_l, m_r are
// not used where block b is the first or the last).
__device__ __forceinline__ WhitenLine whiten_line_of(int b, int Mi, int W, int nblk, float m_l, float m_here,
                                                     float m_r)
{
    auto two_c = [&](int bb) -> int {
        const int n_b = (bb == nblk - 1) ? (Mi - bb * W) : W;
        return 2 * bb * W + n_b + 1;
    };
    WhitenLine L;
    L.start = 1 + b * W;
    L.cnt = (Mi - b * W) < W ? (Mi - b * W) : W;
    const int c_here = two_c(b);
    L.m_here = m_here;
    // left segment [c_{b-1}, c_b), right [c_b, c_{b+1}); flat outside the first/last centre
    const bool has_l = b > 0, has_r = b + 1 < nblk;
    const int c_l = has_l ? two_c(b - 1) : c_here, c_r = has_r ? two_c(b + 1) : c_here;
    if (!has_l) m_l = m_here;
    if (!has_r) m_r = m_here;
    L.s_l = has_l ? (L.m_here - m_l) / (float)(c_here - c_l) : 0.0f;
    L.s_r = has_r ? (m_r - L.m_here) / (float)(c_r - c_here) : 0.0f;
    L.base_l = has_l ? (float)c_l : (float)c_here;
    L.ml0 = has_l ? m_l : L.m_here;
    L.fc = (float)c_here;
    return L;
}

__device__ __forceinline__ WhitenLine whiten_line(const float* __restrict__ md, int b, int Mi, int W, int nblk)
{
    const float m_l = b > 0 ? md[b - 1] : 0.0f, m_r = b + 1 < nblk ? md[b + 1] : 0.0f;
    return whiten_line_of(b, Mi, W, nblk, m_l, md[b], m_r);
}

constexpr float LN2F = 0.69314718055994530942f;

// First of the sorted, disjoint bin ranges zap[0..nzap) that ends at or
// after bin q (nzap if none).
__device__ __forceinline__ int first_zap(const int2* __restrict__ zap, int nzap, int q)
{
    int lo = 0, hi = nzap;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (zap[mid].y < q) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Block medians and whitening in one pass over the spectrum: power P in,
// whitened power Q out (a separate array: neighbouring workgroups read the
// raw power of the blocks next to theirs).  Workgroup g owns the mw
// consecutive blocks [b0, b1) of one template and walks them in order with
// two blocks' values in registers: the median of block b + 1 is taken, then
// block b (still in registers) is whitened with the line through the medians
// of b - 1, b and b + 1 and stored.  The medians of the blocks just outside
// [b0, b1) are recomputed here rather than waited for (two extra medians per
// mw blocks), so workgroups never wait on each other.  The medians
// are k_median's; each bin is whitened as P^ = P ln2 rcp(m(k)), m(k) the line
// of WhitenLine (0 where m(k) <= 0, in birdie ranges, and at k = 0).  A
// median pass followed by a separate whitening pass, which reads the spectrum
// twice, was measured slower.
template <int VPT>
__global__ __launch_bounds__(NT) void k_median_whiten(const float* __restrict__ P, float* __restrict__ Q,
                                                      size_t p_stride, int64_t M, int W, int nblk, int mw,
                                                      float* __restrict__ med, size_t med_stride,
                                                      const int2* __restrict__ zap, int nzap)
{
    __shared__ uint32_t hist[MED_BINS];
    __shared__ uint32_t wsum[NT / 64];
    __shared__ uint32_t s_digit, s_rank;
    const float* Ps = P + blockIdx.y * p_stride;
    float* Qs = Q + blockIdx.y * p_stride;
    float* md = med + blockIdx.y * med_stride;
    const int b0 = (int)blockIdx.x * mw, b1 = min(b0 + mw, nblk);
#pragma unroll
    for (int i = 0; i < MED_BINS / NT; ++i) hist[threadIdx.x + i * NT] = 0;
    __syncthreads();
    uint32_t cur[VPT], nxt[VPT];
    float m_l = 0.0f;
    if (b0 > 0) {
        const int c = load_block<VPT>(Ps, M, W, b0 - 1, nxt);
        m_l = block_median<VPT>(nxt, c, hist, wsum, s_digit, s_rank);
    }
    int cnt = load_block<VPT>(Ps, M, W, b0, cur);
    float m_c = block_median<VPT>(cur, cnt, hist, wsum, s_digit, s_rank);
    for (int b = b0; b < b1; ++b) {
        float m_r = 0.0f;
        int cnt_n = 0;
        if (b + 1 < nblk) {
            cnt_n = load_block<VPT>(Ps, M, W, b + 1, nxt);
            m_r = block_median<VPT>(nxt, cnt_n, hist, wsum, s_digit, s_rank);
        }
        if (threadIdx.x == 0) md[b] = m_c;
        const WhitenLine L = whiten_line_of(b, (int)M, W, nblk, m_l, m_c, m_r);
        int r = nzap ? first_zap(zap, nzap, L.start) : 0;
        if (cnt == VPT * NT && !nzap) {
            float* qrow = Qs + L.start + threadIdx.x;
#pragma unroll
            for (int i = 0; i < VPT; ++i) {
                const int q = L.start + (int)threadIdx.x + i * NT;
                const float level = L.level(q);
                const float p = __uint_as_float(cur[i]);
                qrow[i * NT] = level > 0.0f ? p * (LN2F * __builtin_amdgcn_rcpf(level)) : 0.0f;
            }
        } else
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
            const int qi = (int)threadIdx.x + i * NT;
            if (qi < cnt) {
                const int q = L.start + qi;
                bool zapped = false;
                if (nzap) {
                    while (r < nzap && zap[r].y < q) ++r;
                    zapped = r < nzap && zap[r].x <= q;
                }
                const float level = L.level(q);
                const float p = __uint_as_float(cur[i]);
                Qs[q] = (level > 0.0f && !zapped) ? p * (LN2F * __builtin_amdgcn_rcpf(level)) : 0.0f;
            }
        }
        if (b == 0 && threadIdx.x == 0) Qs[0] = 0.0f;
        m_l = m_c;
        m_c = m_r;
        cnt = cnt_n;
#pragma unroll
        for (int i = 0; i < VPT; ++i) cur[i] = nxt[i];
    }
}

// Zeroes the bins of the birdie ranges in a series' whitening factors; one
// workgroup per range.
__global__ __launch_bounds__(NT) void k_zap_factors(float* __restrict__ fac, const int2* __restrict__ zap)
{
    const int2 z = zap[blockIdx.x];
    for (int q = z.x + (int)threadIdx.x; q <= z.y; q += NT) fac[q] = 0.0f;
}

// Once per series: the factor ln2 / m(k) (0 where m(k) <= 0, and at k = 0)
// that pass 2 applies to every template's power, the same float the
// per-template whitening multiplies by.
__global__ __launch_bounds__(NT) void k_series_factor(const float* __restrict__ med, int64_t M, int W, int nblk,
                                                      float* __restrict__ fac)
{
    const int b = blockIdx.x;
    const WhitenLine L = whiten_line(med, b, (int)M, W, nblk);
    for (int i = threadIdx.x; i < L.cnt; i += NT) {
        const int q = L.start + i;
        const float level = L.level(q);
        fac[q] = level > 0.0f ? LN2F * __builtin_amdgcn_rcpf(level) : 0.0f;
    }
    if (b == 0 && threadIdx.x == 0) fac[0] = 0.0f;
}

// ------------------------------------------------------------------------
// Harmonic sum (Sec. 2.1, up to 16 harmonics), threshold and wave-ballot
// compaction, on the whitened spectrum.
//
// Bin k of fold h adds harmonic m at bin floor((2mk + h)/(2h)); with
// j = 16 m / h that is floor((jk + 8)/16).  A workgroup handles the HT bins
// [k0, k0 + HT), thread t the bins k0 + t + NT r (r < HT/NT); moving r by one
// moves every harmonic index by exactly 16 j, so each thread computes one
// index per j and reads the rest at compile-time offsets.  Lanes of a wave
// hold consecutive bins, so a wave's read of harmonic j covers about 4j
// consecutive floats: the loads go straight to L2 (no LDS staging, no
// barrier), which leaves occupancy to the register count.  Fold 2h adds the
// odd m of the new fold to fold h (ascending m), the order the oracle uses.
constexpr int HT = 1024;  // output bins per workgroup

// One fold's threshold test and wave-ballot append of the bins above it.
__device__ __forceinline__ void emit(bool hit, int lane, uint64_t below, uint32_t* __restrict__ counter,
                                     uint4* __restrict__ ring, uint32_t capacity, uint32_t tid, int k,
                                     uint32_t series_fold, float acc)
{
    const uint64_t mask = __ballot(hit);
    if (mask) {
        const int leader = __ffsll((unsigned long long)mask) - 1;
        uint32_t rbase = 0;
        if (lane == leader) rbase = atomicAdd(counter, (uint32_t)__popcll(mask));
        rbase = __shfl(rbase, leader);
        if (hit) {
            const uint32_t idx = rbase + (uint32_t)__popcll(mask & below);
            if (idx < capacity) ring[idx] = make_uint4(tid, (uint32_t)k, series_fold, __float_as_uint(acc));
        }
    }
}

// Fold sums of a thread's R4 bins.  FULL tiles end at or below M, so no
// index can pass it; the last tile clamps its indices (bins beyond M are not
// reported).
template <int NF, bool FULL>
__device__ __forceinline__ void fold_sums(const float* __restrict__ Ps, int kt, int M, float (&acc)[NF][HT / NT])
{
    constexpr int R4 = HT / NT;
    auto at = [&](int j, int r) -> float {
        if (FULL) return (Ps + ((j * kt + 8) >> 4))[16 * j * r];  // one address per j, immediate offsets
        const int i = ((j * kt + 8) >> 4) + 16 * j * r;
        return Ps[i < M ? i : M];
    };
#pragma unroll
    for (int r = 0; r < R4; ++r) acc[0][r] = at(16, r);
#pragma unroll
    for (int l = 1; l < NF; ++l) {
#pragma unroll
        for (int r = 0; r < R4; ++r) acc[l][r] = acc[l - 1][r];
#pragma unroll
        for (int m = 1; m < (1 << l); m += 2) {
            const int j = m << (4 - l);
#pragma unroll
            for (int r = 0; r < R4; ++r) acc[l][r] += at(j, r);
        }
    }
}

// Tile order: the grid's x extent is a multiple of 8, so workgroup x runs on
// XCD x % 8, and tile_of[x] is the tile it takes (-1: none).  The table puts
// each binary subtree {t, 2t, 2t+1, 4t, ...} of tiles on one XCD, parent
// first: runs j <= 8 of tiles 2t and 2t+1 lie inside run 2j of tile t, so
// they are read while still in that XCD's L2.
template <int NF>
__global__ __launch_bounds__(NT) void k_harmsum(const float* __restrict__ P, size_t p_stride, int64_t M,
                                                int tmpl_base, PeakParams pp, uint4* __restrict__ ring,
                                                uint32_t* __restrict__ counter, float* __restrict__ sums_out,
                                                const int32_t* __restrict__ tile_of)
{
    constexpr int R4 = HT / NT;
    const int tile = tile_of[blockIdx.x];
    if (tile < 0) return;
    const int k0 = tile * HT;
    const int Mi = (int)M;
    const int kend = k0 + HT - 1 < Mi ? k0 + HT - 1 : Mi;
    const float* Ps = P + blockIdx.y * p_stride;
    const uint32_t tid = pp.first_template_id + (uint32_t)(tmpl_base + (int)blockIdx.y);
    const int kt = k0 + (int)threadIdx.x;
    const int lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const bool full = kend == k0 + HT - 1;
    bool inside = full && !sums_out;
#pragma unroll
    for (int l = 0; l < NF; ++l) inside = inside && k0 >= pp.klo[l] && kend <= pp.khi[l];

    float acc[NF][R4];
    if (full)
        fold_sums<NF, true>(Ps, kt, Mi, acc);
    else
        fold_sums<NF, false>(Ps, kt, Mi, acc);

    if (inside) {
        // one comparison per fold (the largest of a thread's bins) and one
        // ballot decide whether the wave has anything to report
        bool any = false;
#pragma unroll
        for (int l = 0; l < NF; ++l) {
            float mx = acc[l][0];
#pragma unroll
            for (int r = 1; r < R4; ++r) mx = fmaxf(mx, acc[l][r]);
            any = any || mx > pp.thr[l];
        }
        if (!__ballot(any)) return;
    }
#pragma unroll
    for (int l = 0; l < NF; ++l)
#pragma unroll
        for (int r = 0; r < R4; ++r) {
            const int k = kt + NT * r;
            const bool in = k <= kend;
            if (sums_out && in) sums_out[(size_t)l * (M + 1) + k] = acc[l][r];
            const bool hit = in && k >= pp.klo[l] && k <= pp.khi[l] && acc[l][r] > pp.thr[l];
            emit(hit, lane, below, counter, ring, pp.capacity, tid, k, (pp.series_id << 8) | (uint32_t)l, acc[l][r]);
        }
}

// ------------------------------------------------------------------------
int ilog2i(int v)
{
    int r = 0;
    while ((1 << (r + 1)) <= v) ++r;
    return r;
}

template <int S, int C1>
hipError_t fft1_launch(const Geometry& g, const float* x, double tsamp, const TmplDev* tm, int nslots,
                       const Slots& ws, int32_t* src_out, hipStream_t s)
{
    dim3 grid(g.R / C1, nslots);
    hipLaunchKernelGGL((k_fft1<S, C1>), grid, dim3(C1 * S / 16), 0, s, x, g.n, g.R, g.lgR, g.P, tsamp, tm, ws.poly,
                       ws.poly_stride, ws.pok, ws.Y, ws.y_stride, g.twst, g.twM_lo, g.twM_hi, src_out);
    return hipGetLastError();
}

template <int R, int D2>
hipError_t fft2_launch(const Geometry& g, int nslots, const Slots& ws, const float* fac, hipStream_t s)
{
    dim3 grid(g.S / D2, nslots);
    hipLaunchKernelGGL((k_fft2<R, D2>), grid, dim3(D2 * R / 16), 0, s, ws.Y, ws.y_stride, g.S, ilog2i(g.S),
                       ilog2i(g.C1), ws.P,
                       ws.p_stride, g.M, g.twst, g.tw2M_lo, g.tw2M_hi, fac);
    return hipGetLastError();
}

template <int A, int B>
struct Shape {
    static constexpr int a = A, b = B;
};

// Pass-1 shapes (S, C1) and pass-2 shapes (R, D2) of the 16384- and
// 8192-point tiles, n = 2^10 .. 2^24.
template <class... K>
hipError_t fft1_dispatch(const Geometry& g, const float* x, double tsamp, const TmplDev* tm, int nslots,
                         const Slots& ws, int32_t* src_out, hipStream_t s)
{
    hipError_t e = hipErrorInvalidValue;
    (void)((g.S == K::a && g.C1 == K::b ? (e = fft1_launch<K::a, K::b>(g, x, tsamp, tm, nslots, ws, src_out, s),
                                           true)
                                        : false) ||
           ...);
    return e;
}
template <class... K>
hipError_t fft2_dispatch(const Geometry& g, int nslots, const Slots& ws, const float* fac, hipStream_t s)
{
    hipError_t e = hipErrorInvalidValue;
    (void)((g.R == K::a && g.D2 == K::b ? (e = fft2_launch<K::a, K::b>(g, nslots, ws, fac, s), true) : false) ||
           ...);
    return e;
}

hipError_t launch_fft1(const Geometry& g, const float* x, double tsamp, const TmplDev* tm, int nslots,
                       const Slots& ws, int32_t* src_out, hipStream_t s)
{
    return fft1_dispatch<Shape<32, 16>, Shape<64, 16>, Shape<128, 16>, Shape<256, 16>, Shape<512, 16>,
                         Shape<1024, 16>, Shape<1024, 8>, Shape<2048, 8>, Shape<2048, 4>, Shape<4096, 4>,
                         Shape<4096, 2>, Shape<8192, 2>, Shape<8192, 1>, Shape<16384, 1>>(g, x, tsamp, tm, nslots,
                                                                                         ws, src_out, s);
}

hipError_t launch_fft2(const Geometry& g, int nslots, const Slots& ws, const float* fac, hipStream_t s)
{
    return fft2_dispatch<Shape<16, 32>, Shape<16, 64>, Shape<16, 128>, Shape<16, 256>, Shape<16, 512>,
                         Shape<16, 1024>, Shape<32, 512>, Shape<64, 256>, Shape<128, 128>, Shape<256, 64>,
                         Shape<512, 32>, Shape<32, 256>, Shape<64, 128>, Shape<128, 64>, Shape<256, 32>,
                         Shape<512, 16>, Shape<1024, 8>>(g, nslots, ws, fac, s);
}

}  // namespace

int harmsum_tile() { return HT; }

hipError_t launch_template_prep(const tb_template* t, uint32_t count, TmplDev* out, int model, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_template_prep, dim3((count + 127) / 128), dim3(128), 0, s, t, count, out, model);
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

hipError_t launch_tile_series(const Geometry& g, const float* in, float* out, hipStream_t s)
{
    int64_t blocks = (g.M + NT - 1) / NT;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_tile_series, dim3((unsigned)blocks), dim3(NT), 0, s, in, out, g.M, g.lgR, g.S, g.C1, g.P);
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

namespace {

// Records an event of kernel class cls on s into marks (none without marks).
hipError_t mark(Marks* marks, int cls, hipStream_t s)
{
    if (!marks) return hipSuccess;
    hipEvent_t ev = nullptr;
    hipError_t r = hipEventCreate(&ev);
    if (r != hipSuccess) return r;
    marks->emplace_back(cls, ev);
    return hipEventRecord(ev, s);
}

// Delay polynomials, then passes 1 and 2 in groups of ws.BY templates: the
// power (whitened by fac when given) of nslots templates in ws.P.
hipError_t launch_power(const Geometry& g, const float* x, double tsamp, const TmplDev* tmw, int nslots,
                        const Slots& ws, const float* fac, int32_t* src_out, hipStream_t s, Marks* marks)
{
    hipError_t e;
    if ((e = mark(marks, K_POLY, s)) != hipSuccess) return e;
    const int npts = (int)std::min<int64_t>(g.TE, g.M), nchunk = npts / 8;
    hipLaunchKernelGGL(k_chunk_polys, dim3((nchunk + NT - 1) / NT, nslots), dim3(NT), 0, s, tmw, tsamp, g.R, g.C1,
                       g.P, g.n, npts, ws.poly, ws.poly_stride, ws.pok);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int q0 = 0; q0 < nslots; q0 += ws.BY) {
        const int nq = std::min(ws.BY, nslots - q0);
        Slots grp = ws;
        grp.poly = ws.poly + (size_t)q0 * ws.poly_stride;
        grp.pok = ws.pok + q0;
        grp.P = ws.P + (size_t)q0 * ws.p_stride;
        if ((e = mark(marks, K_PASS1, s)) != hipSuccess) return e;
        if ((e = launch_fft1(g, x, tsamp, tmw + q0, nq, grp, q0 == 0 ? src_out : nullptr, s)) != hipSuccess)
            return e;
        if ((e = mark(marks, K_PASS2, s)) != hipSuccess) return e;
        if ((e = launch_fft2(g, nq, grp, fac, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_median(const Geometry& g, int nslots, const Slots& ws, float* med, size_t med_stride,
                         hipStream_t s)
{
    if (g.W <= 16 * NT)
        hipLaunchKernelGGL((k_median<16>), dim3(g.nblk, nslots), dim3(NT), 0, s, ws.P, ws.p_stride, g.M, g.W, med,
                           med_stride);
    else
        hipLaunchKernelGGL((k_median<32>), dim3(g.nblk, nslots), dim3(NT), 0, s, ws.P, ws.p_stride, g.M, g.W, med,
                           med_stride);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_series_levels(const Geometry& g, const float* x, double tsamp, const TmplDev* tm, const Slots& ws,
                                float* med, float* fac, hipStream_t s)
{
    hipError_t e;
    if ((e = launch_power(g, x, tsamp, tm, 1, ws, nullptr, nullptr, s, nullptr)) != hipSuccess) return e;
    if ((e = launch_median(g, 1, ws, med, 0, s)) != hipSuccess) return e;
    return launch_series_factors(g, med, fac, nullptr, 0, s);
}

hipError_t launch_series_factors(const Geometry& g, const float* med, float* fac, const int2* zap, int nzap,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(k_series_factor, dim3(g.nblk), dim3(NT), 0, s, med, g.M, g.W, g.nblk, fac);
    if (nzap) hipLaunchKernelGGL(k_zap_factors, dim3(nzap), dim3(NT), 0, s, fac, zap);
    return hipGetLastError();
}

hipError_t launch_wave(const Geometry& g, const float* x, double tsamp, const TmplDev* tm, int tmpl_base,
                       int nslots, const Slots& ws, const float* fac, const int2* zap, int nzap, const PeakParams& pp,
                       uint4* ring, uint32_t* counter, const Inspect& ins, hipStream_t s, Marks* marks)
{
    hipError_t e;
    if ((e = launch_power(g, x, tsamp, tm + tmpl_base, nslots, ws, fac, ins.src, s, marks)) != hipSuccess) return e;
    if (ins.power &&
        (e = hipMemcpyAsync(ins.power, ws.P, sizeof(float) * (size_t)(g.M + 1), hipMemcpyDeviceToDevice, s)) !=
            hipSuccess)
        return e;
    if (!fac) {
        // block medians and whitening in one kernel (the whitening class of
        // the profile then has no launches of its own)
        if ((e = mark(marks, K_MEDIAN, s)) != hipSuccess) return e;
        // as many blocks per workgroup as keep about 1024 workgroups (four per
        // compute unit, one round at this kernel's occupancy), at most 64: each
        // workgroup recomputes the medians of the two blocks just outside its
        // run, so longer runs re-read less of the spectrum
        const int mw = std::max(2, std::min(64, g.nblk * nslots / 1024));
        const dim3 grid((g.nblk + mw - 1) / mw, nslots);
        if (g.W <= 16 * NT)
            hipLaunchKernelGGL((k_median_whiten<16>), grid, dim3(NT), 0, s, ws.P, ws.Q, ws.p_stride, g.M, g.W,
                               g.nblk, mw, ws.med, ws.med_stride, zap, nzap);
        else
            hipLaunchKernelGGL((k_median_whiten<32>), grid, dim3(NT), 0, s, ws.P, ws.Q, ws.p_stride, g.M, g.W,
                               g.nblk, mw, ws.med, ws.med_stride, zap, nzap);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = mark(marks, K_HARMSUM, s)) != hipSuccess) return e;
    const float* spec = fac ? ws.P : ws.Q;  // whitened power
    dim3 hg(g.hgrid, nslots);
    switch (pp.nfold) {
    case 1: hipLaunchKernelGGL((k_harmsum<1>), hg, dim3(NT), 0, s, spec, ws.p_stride, g.M, tmpl_base, pp, ring, counter, ins.sums, g.tile_of); break;
    case 2: hipLaunchKernelGGL((k_harmsum<2>), hg, dim3(NT), 0, s, spec, ws.p_stride, g.M, tmpl_base, pp, ring, counter, ins.sums, g.tile_of); break;
    case 3: hipLaunchKernelGGL((k_harmsum<3>), hg, dim3(NT), 0, s, spec, ws.p_stride, g.M, tmpl_base, pp, ring, counter, ins.sums, g.tile_of); break;
    case 4: hipLaunchKernelGGL((k_harmsum<4>), hg, dim3(NT), 0, s, spec, ws.p_stride, g.M, tmpl_base, pp, ring, counter, ins.sums, g.tile_of); break;
    case 5: hipLaunchKernelGGL((k_harmsum<5>), hg, dim3(NT), 0, s, spec, ws.p_stride, g.M, tmpl_base, pp, ring, counter, ins.sums, g.tile_of); break;
    default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return mark(marks, -1, s);
}

}  // namespace tb
