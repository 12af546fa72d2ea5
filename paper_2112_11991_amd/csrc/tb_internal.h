// tb_internal.h -- declarations shared by the kernels and the engine of the
// gfx950 template-bank search library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

#include "../../include/tb.h"

namespace tb {

// Per-template constants, prepared on the device from a tb_template:
// Omega = 2 pi / P_orb, the Roemer-delay factors of the BT model (App. A.1)
// and the zero offset Delta(0) of Algorithm 1.  With the series delay
// (model 1) also sin(psi) C_k and cos(psi) S_k of the App. B expansion and
// sum_k k^5 (|C_k| + |S_k|), the bound on the fifth derivative in M.
struct TmplDev {
    double omega, alpha, tau, ecc;
    double sinw, cosw, beta, d0;
    double ca[8], sb[8];
    double g5;
    int32_t model, pad;
};
static_assert(sizeof(TmplDev) == 208, "TmplDev layout");

// App. B coefficients C_0..C_7 and S_0..S_7 (S_0 = 0) of
//   cos E = sum C_k(e) cos kM,  sqrt(1-e^2) sin E = sum S_k(e) sin kM,
// complete through e^6.
__host__ __device__ inline void series_coefficients(double e, double* C, double* S)
{
    const double e2 = e * e, e3 = e2 * e, e4 = e3 * e, e5 = e4 * e, e6 = e5 * e;
    C[0] = -e / 2.0;
    C[1] = 1.0 - (3.0 / 8.0) * e2 + (5.0 / 192.0) * e4 - (7.0 / 9216.0) * e6;
    C[2] = e / 2.0 - e3 / 3.0 + e5 / 16.0;
    C[3] = (3.0 / 8.0) * e2 - (45.0 / 128.0) * e4 + (567.0 / 5120.0) * e6;
    C[4] = e3 / 3.0 - (2.0 / 5.0) * e5;
    C[5] = (125.0 / 384.0) * e4 - (4375.0 / 9216.0) * e6;
    C[6] = (27.0 / 80.0) * e5;
    C[7] = (16807.0 / 46080.0) * e6;
    S[0] = 0.0;
    S[1] = 1.0 - (5.0 / 8.0) * e2 - (11.0 / 192.0) * e4 - (457.0 / 9216.0) * e6;
    S[2] = e / 2.0 - (5.0 / 12.0) * e3 + e5 / 24.0;
    S[3] = (3.0 / 8.0) * e2 - (51.0 / 128.0) * e4 + (543.0 / 5120.0) * e6;
    S[4] = e3 / 3.0 - (13.0 / 30.0) * e5;
    S[5] = (125.0 / 384.0) * e4 - (4625.0 / 9216.0) * e6;
    S[6] = (27.0 / 80.0) * e5;
    S[7] = (16807.0 / 46080.0) * e6;
}

// Two-pass FFT geometry of a real series of n = 2M samples packed as M
// complex points, M = R * S.  Each workgroup holds min(TE, M) points, TE the
// tile size (16384, or 8192 for two workgroups per CU): pass 1 does S-point
// transforms over the strided index (C1 = TE/S columns per workgroup), pass 2
// R-point transforms over D2 = TE/R columns (D2/2 mirrored pairs) followed by
// the real-to-complex split and |X|^2.
struct Geometry {
    int log2n = 0;
    int64_t n = 0, M = 0;
    int TE = 0;
    int S = 0, R = 0, C1 = 0, D2 = 0, lgR = 0;
    int P = 0;             // zero rows before and after every pass-1 column block of a resident series
    int W = 0;             // whitening window (bins per median block)
    int nblk = 0;          // whitening blocks
    int htile = 0;         // harmonic-sum output bins per workgroup
    float2* twst = nullptr;                        // radix-16 stage twiddles, every stride
    float2* twM_lo = nullptr, *twM_hi = nullptr;   // W_M^q split in 2^10 x rest
    float2* tw2M_lo = nullptr, *tw2M_hi = nullptr; // W_2M^k likewise
    int32_t* tile_of = nullptr;                    // harmonic-sum tile per workgroup (XCD-aware order)
    int hgrid = 0;                                 // harmonic-sum workgroups per template (multiple of 8)
};

constexpr int TW_LO_BITS = 10;
constexpr int TWST_NS_MAX = 1024;           // largest stage stride (16384-point transforms)
constexpr int PAD_REACH_LOG2 = 20;          // largest delay swing (samples) the zero rows of a series cover

// Floats of a resident series: R columns of S complex points in blocks of
// C1, each block with P zero rows after it and P before the first.
inline size_t series_floats(const Geometry& g)
{
    return 2 * ((size_t)g.R * (size_t)(g.S + g.P) + (size_t)g.P * (size_t)g.C1);
}

// Fourth-order expansion of the sample delay around the middle sample of a
// chunk of 16 or 8 pass-1 tile points, 48 bytes so that records stay 16-B
// aligned.  jmid is that sample plus 2PR, in the shifted indices the pass-1
// gather works with (P zero rows of 2R samples precede a resident series).
struct ChunkPoly {
    double c0, c1, c2, c3, c4;
    int32_t jmid, pad;
};
static_assert(sizeof(ChunkPoly) == 48, "ChunkPoly layout");

// Per-launch search parameters of the harmonic sum / threshold stage.
struct PeakParams {
    float thr[5];      // S_h threshold per fold, h = 1, 2, 4, 8, 16
    int32_t klo[5];    // first bin searched per fold (h * kmin)
    int32_t khi[5];    // last bin searched per fold
    int32_t nfold;     // log2(harm_max) + 1
    uint32_t series_id;
    uint32_t first_template_id;
    uint32_t capacity; // ring records
};

// Device workspace for B templates in flight at one series length.
struct Slots {
    int B = 0;             // templates per wave (power, medians, harmonic sum)
    int BY = 0;            // exchange slots: passes 1 and 2 run in groups of BY templates
    float2* Y = nullptr;   // exchange buffer, BY x M complex
    size_t y_stride = 0;   // complex per slot
    float* P = nullptr;    // power, B x (M + 1), padded
    float* Q = nullptr;    // whitened power (per-template whitening), same layout as P
    size_t p_stride = 0;
    float* med = nullptr;  // block medians, B x nblk
    size_t med_stride = 0;
    ChunkPoly* poly = nullptr;  // delay polynomials, B x (tile points / 8)
    size_t poly_stride = 0;
    int32_t* pok = nullptr;     // per slot: log2 points per chunk (4 or 3), 0 = exact solve
};

// Optional per-stage outputs (template slot 0 only).
struct Inspect {
    int32_t* src = nullptr;  // n
    float* power = nullptr;  // M + 1, copied before whitening overwrites it
    float* sums = nullptr;   // nfold x (M + 1)
};

// model: 0 BT with the Newton Kepler solve, 1 the App. B series.
hipError_t launch_template_prep(const tb_template* t, uint32_t count, TmplDev* out, int model, hipStream_t s);
hipError_t launch_mean_subtract(const float* in, float* out, int64_t n, double* partial, hipStream_t s);
// Kernel classes timed by the plan's profiler, in launch order.
enum { K_POLY = 0, K_PASS1 = 1, K_PASS2 = 2, K_MEDIAN = 3, K_WHITEN = 4, K_HARMSUM = 5, K_CLASSES = 6 };

// Timing marks of one wave: (kernel class, event recorded before its kernel),
// closed by (-1, event after the last kernel).
using Marks = std::vector<std::pair<int, hipEvent_t>>;

// Queues the kernels of one wave of nslots templates (passes 1 and 2 in
// groups of ws.BY, so that a group's exchange buffer is still cached when
// pass 2 reads it).  fac: whitening factors of a series whitened once (M + 1
// floats), applied by pass 2 in place of the per-template medians and
// whitening; nullptr for per-template whitening.  zap[0..nzap): the series'
// birdie bin ranges (inclusive, sorted, disjoint), zeroed by the per-template
// whitening (a series whitened once carries them in fac).  With marks, an
// event is recorded before every kernel.
hipError_t launch_wave(const Geometry& g, const float* x, double tsamp, const TmplDev* tm, int tmpl_base,
                       int nslots, const Slots& ws, const float* fac, const int2* zap, int nzap, const PeakParams& pp,
                       uint4* ring, uint32_t* counter, const Inspect& ins, hipStream_t s, Marks* marks = nullptr);
// The power spectrum of the series x read through template tm (one without
// orbit reads it as loaded), its block medians into med (nblk floats) and the
// whitening factors ln2 / m(k) into fac (M + 1 floats).  Uses slot 0 of ws.
hipError_t launch_series_levels(const Geometry& g, const float* x, double tsamp, const TmplDev* tm,
                                const Slots& ws, float* med, float* fac, hipStream_t s);
// Factors ln2 / m(k) from the series medians, then 0 over the birdie ranges.
hipError_t launch_series_factors(const Geometry& g, const float* med, float* fac, const int2* zap, int nzap,
                                 hipStream_t s);
hipError_t launch_copy(float4* dst, const float4* src, size_t count, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t count, hipStream_t s);
// Rewrites a mean-removed series into the tile order pass 1 reads.
hipError_t launch_tile_series(const Geometry& g, const float* in, float* out, hipStream_t s);
int harmsum_tile();
// Rewrites the first min(*counter, cap) candidate records in place with their
// significance: {template, bin | log2 h << 28, sigma bits, S} (tb_readback.hip).
hipError_t launch_significance(uint4* ring, const uint32_t* counter, uint64_t cap, hipStream_t s);
// Candidate records a request's device ring holds (the plan's ring_capacity).
uint64_t plan_ring_capacity(tb_plan_t p);
// Dedispersion: integer delays delay[c * ldd + d] (ldd = ndm rounded up to the
// DM tile) of every channel and trial; returns the largest.
int64_t dedisp_delays(int nchan, double fch1, double foff, double tsamp, const double* dm, int ndm,
                      std::vector<int32_t>& delay, int& ldd);
// Transposes d_tm (time-major, nbits 8 or 4) into d_cm (channel-major bytes,
// rows of ldx bytes, a multiple of 16, zero beyond nsamp), then dedisperses
// into out (ndm x nout floats).
hipError_t launch_dedisperse(const uint8_t* d_tm, int nbits, uint8_t* d_cm, int nchan, int64_t nsamp, int64_t ldx,
                             const int32_t* d_delay, int ldd, const int2* d_lospan, int ndm, int64_t nout, float* out,
                             hipStream_t s);
int dedisp_tile();
// Bank density of count points (device arrays); kind 0 circular, 1 elliptical;
// waits for the stream; *ms (may be null) receives the kernel time.
hipError_t launch_bank_density(int kind, int nodes, double T, double fmax, const tb_template* d_pts, uint32_t count,
                               double* d_out, hipStream_t s, double* ms);

}  // namespace tb
