/*
 * tb.h -- C ABI of the MI355X (gfx950) template-bank coherent orbital search.
 *
 * The library implements the per-template search of Balakrishnan et al.,
 * "Coherent Search for Binary Pulsars across all Five Keplerian Parameters in
 * Radio Observations using the template-bank algorithm" (arXiv:2112.11991):
 * for every Keplerian orbital template it removes the Roemer delay from a
 * dedispersed time series by nearest-sample resampling (App. A.1, Algorithm
 * 1), takes a real-to-complex FFT (the spin-frequency grid of Sec. 2.4), forms
 * and whitens the power spectrum ("Fourier de-reddening", Sec. 5.2), sums up
 * to 16 harmonics (Sec. 2.1) and keeps every bin above a false-alarm
 * threshold (Sec. 2.1).  All of it runs in hand-written HIP kernels.
 *
 * Conventions
 *  - Every call returns a tb_status; errors are negative.  Nothing is thrown
 *    across the ABI.  tb_strerror() names a status.
 *  - Host buffers passed in are owned by the caller and only read or written
 *    during the call.  Device pointers (TB_MEM_DEVICE) must stay valid until
 *    the call returns.  Everything the plan allocates it owns and frees in
 *    tb_destroy().
 *  - One plan may be used from several host threads; calls are serialised by
 *    a mutex inside the plan.
 *  - Series length n must be a power of two in [2^10, 2^max_log2n],
 *    max_log2n <= 24.
 */
#ifndef TB_H
#define TB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tb_plan_s* tb_plan_t;

typedef enum {
    TB_OK = 0,
    TB_ERR_INVALID_ARG = -1, /* bad argument: NULL, non-power-of-two n, e >= 1, tau < 0, ... */
    TB_ERR_OOM = -2,         /* device or host allocation failed */
    TB_ERR_BUDGET = -3,      /* the plan's HBM budget would be exceeded */
    TB_ERR_DEVICE = -4,      /* a HIP runtime call failed */
    TB_ERR_OVERFLOW = -5,    /* more candidates than the request's ring holds; the
                                count is still exact and the first ring_capacity
                                records found are returned */
    TB_ERR_NOT_READY = -6,   /* tb_poll / non-blocking tb_get_candidates: still running */
    TB_ERR_UNKNOWN_ID = -7,  /* no such series or request */
    TB_ERR_TOO_LARGE = -8    /* tb_search_templates_noalloc: the work does not fit its fixed scratch */
} tb_status;

/* tb_config.flags.  TB_DELAY_SERIES: the Roemer delay of every template is
 * taken from the series of cos E and sqrt(1-e^2) sin E in the mean anomaly
 * with the App. B coefficients (complete through e^6; the ELL7 model of Sec.
 * 2.2 and App. A.1) instead of the BT delay with a Newton solve of Kepler's
 * equation.  It differs from the BT delay by O(e^7) of tau (about 1.3 e^7 tau
 * at most; 1e-7 tau at e = 0.1) and equals it for e = 0. */
enum { TB_DELAY_SERIES = 1 };

/* tb_load_series flags: where data lives (one of the two), optionally ORed
 * with TB_SERIES_WHITENING. */
enum { TB_MEM_HOST = 0, TB_MEM_DEVICE = 1, TB_SERIES_WHITENING = 2 };

typedef struct {
    uint32_t max_log2n;        /* largest series accepted, log2 samples, 10..24 */
    uint32_t harm_max;         /* harmonics summed: 1, 2, 4, 8 or 16 (Sec. 2.1; 16 in Sec. 5.2) */
    uint32_t whiten_window;    /* W, spectral bins per median block of the whitening, 1..8192 */
    uint32_t batch_templates;  /* templates in flight per wave; 0 = the plan's choice, 2^28 / (n/2)
                                  clamped to 4..256 (64 at n = 2^23) */
    double threshold_sigma;    /* one-sided Gaussian-equivalent false-alarm threshold (Sec. 2.1) */
    double fmin_hz;            /* lowest fundamental searched (default 1 Hz) */
    double fmax_hz;            /* highest fundamental searched; 0 = Nyquist */
    uint64_t hbm_budget_bytes; /* device memory the plan may hold; 0 = no limit */
    uint64_t ring_capacity;    /* candidate records kept per request (default 1<<20) */
    void* stream;              /* hipStream_t the plan launches on; NULL = a stream of its own */
    int32_t device;            /* HIP device ordinal; the plan makes it current on each call */
    uint32_t lanes;            /* streams requests are spread over (1..16); work on different
                                  lanes overlaps on the device.  Lane 0 is `stream`. */
    uint32_t flags;            /* 0, or TB_DELAY_SERIES */
    uint32_t tile_points;      /* FFT points per workgroup: 8192 (two workgroups per compute
                                  unit) or 16384 (one); 0 = the plan's choice (8192, and
                                  16384 for series of 2^24 samples) */
} tb_config;

/* One Keplerian orbital template (Sec. 2.1): P_orb = 2 pi / Omega, tau = a sin(eps)/c,
 * alpha the initial orbital phase (M = Omega t + alpha), e the eccentricity,
 * omega (psi in the paper) the longitude of periastron.  Circular: ecc = omega_rad = 0. */
typedef struct {
    double porb_s;
    double tau_lts;
    double alpha_rad;
    double ecc;
    double omega_rad;
} tb_template;

/* One bin of a harmonic fold above threshold (App. A "peak detection"). */
typedef struct {
    uint32_t series_id;
    uint32_t template_id;  /* first_template_id + index within the request */
    uint32_t bin;          /* k: the h-th harmonic bin, fundamental at k/h bins */
    uint8_t log2_harm;     /* h = 2^log2_harm harmonics summed */
    uint8_t reserved[3];
    float power;           /* S_h[k], sum of h whitened powers */
    float sigma;           /* Gaussian-equivalent significance of S_h[k] (Sec. 2.1) */
    double freq_hz;        /* fundamental frequency k / (h T), T = n tsamp */
} tb_candidate;

/* Fills cfg with the defaults: max_log2n 24, harm_max 16, whiten_window 4096,
 * threshold_sigma 6, fmin_hz 1, fmax_hz 0, no budget, ring 1<<20, own stream,
 * device 0, one lane. */
void tb_default_config(tb_config* cfg);

/* Creates a plan: checks cfg, makes device cfg->device current, creates or
 * adopts the stream, and fixes the search parameters every request uses: the
 * number of harmonics summed and the false-alarm threshold of Sec. 2.1
 * (harmonic sums up to 16 and the search set-up of Sec. 5.2), the whitening
 * window of the Fourier de-reddening (Sec. 5.2, App. A) and the searched
 * frequency band (the uniform frequency grid of Sec. 2.4).  Returns
 * TB_ERR_INVALID_ARG for a bad cfg, TB_ERR_DEVICE if the device cannot be
 * used. */
tb_status tb_plan(const tb_config* cfg, tb_plan_t* out);

/* Waits for the plan's work, frees everything it owns.  NULL is a no-op.
 * Resource management only: the paper defines no such step. */
tb_status tb_destroy(tb_plan_t plan);

/* Copies a dedispersed series S_i, i = 0..n-1 at times i*tsamp (App. A.1),
 * into plan memory (from host, or device-to-device on the plan stream for
 * TB_MEM_DEVICE) and removes its mean in double precision.  Returns the new
 * id in *series_id.  TB_ERR_BUDGET if it does not fit the HBM budget.  A
 * series occupies 4n bytes plus about 4 min(n/8, 2^20) bytes of zero padding
 * that reads before or after it land on (counted by tb_memory).
 *
 * With TB_SERIES_WHITENING the Fourier de-reddening (App. A, Sec. 5.2) is done
 * once for the series instead of once per template: the block medians of the
 * power spectrum of the series as loaded (no demodulation) give the level
 * m(k), and every template searched on the series has P^_k = P_k ln2 / m(k)
 * (0 where m(k) <= 0; P^_0 = 0).  The per-template block-median and whitening
 * kernels then do not run.  The series holds 4 (n/2 + 1) more bytes, and
 * loading it allocates the search workspace of its length if the plan does not
 * hold it yet. */
tb_status tb_load_series(tb_plan_t plan, const float* data, uint64_t n, double tsamp_s,
                         uint32_t flags, int32_t* series_id);

/* Launch shape for series of 2^log2n samples: FFT points per workgroup
 * (8192 or 16384; 0 = the plan's choice) and templates per wave (1..4096;
 * 0 = the plan's choice), e.g. as chosen by an autotuner measuring each on
 * the device.  Must be set before the plan first uses that length (a series
 * of it loaded or searched): TB_ERR_INVALID_ARG afterwards, or for values
 * outside those sets or log2n outside 10..max_log2n. */
tb_status tb_set_shape(tb_plan_t plan, uint32_t log2n, uint32_t tile_points, uint32_t batch_templates);

/* Birdie zapping (App. A and Sec. 5.2 name Fourier birdie zapping among the
 * per-series steps): replaces the series' list of interference intervals.
 * For every template searched on the series afterwards, the whitened power of
 * each bin k with lo_hz[i] <= k / T <= hi_hz[i] (T = n tsamp; bins
 * ceil(lo T) .. floor(hi T) within 1 .. n/2) is 0 before the harmonic sum.
 * count = 0 clears the list; at most TB_ZAP_MAX intervals; empty intervals
 * (lo > hi) are ignored.  Waits for the plan's queued work first.  The raw
 * powers and medians that tb_inspect_template reports are not affected.
 * TB_ERR_INVALID_ARG for NULL arrays with count > 0, non-finite ends or too
 * many intervals; TB_ERR_UNKNOWN_ID for an unknown series. */
enum { TB_ZAP_MAX = 65536 };
tb_status tb_zap_series(tb_plan_t plan, int32_t series_id, const double* lo_hz, const double* hi_hz,
                        uint32_t count);

/* Frees a series; requests already submitted on it complete first. */
tb_status tb_unload_series(tb_plan_t plan, int32_t series_id);

/* Searches count templates of t over one resident series (Algorithm 1, then
 * FFT, power, whitening, harmonic sum, threshold).  Asynchronous: the
 * templates are copied before return and the work is queued on the plan's
 * stream; *request_id names it for tb_poll / tb_get_candidates / tb_release.
 * TB_ERR_INVALID_ARG for P_orb <= 0, tau < 0, e outside [0, 1) or
 * non-finite values. */
tb_status tb_search_templates(tb_plan_t plan, int32_t series_id, const tb_template* t,
                              uint32_t count, uint32_t first_template_id, int64_t* request_id);

/* Allocation-free search, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): tb_search_templates followed by a blocking tb_get_candidates,
 * with the same kernels and results, that calls no hipMalloc, hipFree or
 * other allocator.  Everything the search needs beyond the resident series
 * and the plan's tables (the templates, the FFT exchange buffer, powers,
 * block medians, delay polynomials, the candidate counter and a ring of
 * capacity records) is carved from one fixed device array of
 * TB_NOALLOC_SCRATCH_BYTES (160 MiB) per GPU, set up when the first plan on
 * that GPU is created and held until the process ends (not counted by
 * tb_memory).  The work runs on the plan's first lane; templates per launch
 * are reduced (down to one) until the workspace fits.  Returns when the
 * candidates are in out (host, capacity records; NULL if capacity is 0),
 * sorted by (series, template, log2_harm, bin), and *n_total holds the
 * exact count.  TB_ERR_TOO_LARGE if count templates, capacity ring records
 * and one template's workspace exceed the array (the workspace alone takes
 * about 128 MiB at 2^24 samples); TB_ERR_OVERFLOW if more than capacity
 * candidates were found (the first capacity found are returned); otherwise
 * the errors of tb_search_templates.  Every call on one GPU shares that
 * GPU's array, which keeps the last call's contents: calls that overlap on
 * one GPU (from different plans or host threads) race. */
enum { TB_NOALLOC_SCRATCH_BYTES = 160 << 20 };
tb_status tb_search_templates_noalloc(tb_plan_t plan, int32_t series_id, const tb_template* t, uint32_t count,
                                      uint32_t first_template_id, tb_candidate* out, uint64_t capacity,
                                      uint64_t* n_total);

/* TB_OK once the request's device work has finished (its threshold step of
 * Sec. 2.1 and peak detection of App. A included), TB_ERR_NOT_READY before;
 * TB_ERR_UNKNOWN_ID for an unknown request, TB_ERR_DEVICE if the device
 * reported an error. */
tb_status tb_poll(tb_plan_t plan, int64_t request_id);

/* The candidates of a request: every bin of every harmonic fold whose sum
 * exceeds the fold's false-alarm threshold (the threshold step of Sec. 2.1;
 * the peak detection of App. A, read as every bin above threshold), with the
 * Gaussian-equivalent significance and fundamental frequency of each.
 * Copies up to capacity candidates of a request into out (host), sorted by
 * (series, template, log2_harm, bin), and the full count into *n_total
 * (out may be NULL to query the count).  blocking != 0 waits for the request;
 * otherwise TB_ERR_NOT_READY is returned while it runs.  TB_ERR_OVERFLOW if
 * the device ring overflowed (ring_capacity records are kept). */
tb_status tb_get_candidates(tb_plan_t plan, int64_t request_id, tb_candidate* out,
                            uint64_t capacity, uint64_t* n_total, int blocking);

/* Waits for and forgets a request.  Its device buffer and pinned template
 * copy go back to the plan, which keeps up to 32 of each for later requests
 * (so that steady-state submits allocate nothing) and frees them in
 * tb_destroy.  Resource management only: the paper defines no such step.
 * TB_ERR_UNKNOWN_ID for an unknown request. */
tb_status tb_release(tb_plan_t plan, int64_t request_id);

/* Blocks until every queued request of the plan has finished. */
tb_status tb_synchronize(tb_plan_t plan);

/* Device memory the plan holds (series, workspaces, tables, requests not yet
 * released; the idle request buffers it keeps for reuse are not counted) and
 * its current HBM budget (0 = none).  Either pointer may be NULL. */
tb_status tb_memory(tb_plan_t plan, uint64_t* held_bytes, uint64_t* budget_bytes);

/* Changes the admission budget; 0 removes it.  Memory already held is kept;
 * later allocations that would exceed the budget fail with TB_ERR_BUDGET. */
tb_status tb_set_budget(tb_plan_t plan, uint64_t budget_bytes);

/* Continuous-batching service of a request stream (the per-DM-trial x
 * template workload of Sec. 5 arriving over time; the paper states no
 * scheduling, so this is the library's own).  Each request is a resident
 * series and a chunk of templates that becomes available at t_arrival_s
 * (seconds after the call starts, times time_scale).  The calling thread
 * admits requests in arrival order as soon as they have arrived and the
 * plan's HBM budget allows (a request refused with TB_ERR_BUDGET waits for
 * running ones to finish), lets tb_search_templates spread them over the
 * plan's lanes, polls the running ones without sleeping and copies each
 * request's candidates (sorted as by tb_get_candidates) into out the moment
 * its device work has finished, then releases it.  With TB_SERVE_SATURATE
 * every request counts as arrived at t = 0.
 *   req     count requests, any order; templates are read during the call
 *   out     host array of capacity records shared by all requests, filled in
 *           completion order; NULL with capacity 0 keeps counts only
 *   res     host array of count results, in req's order: admission and
 *           completion times (seconds after the call started), where the
 *           request's records start in out, how many were copied, the exact
 *           count, and TB_OK or TB_ERR_OVERFLOW (the device ring or out held
 *           fewer than the count)
 *   stats   may be NULL: [0] most requests in flight at once, [1] admissions
 *           deferred by the budget
 * TB_ERR_BUDGET if a request does not fit the budget with nothing running;
 * TB_ERR_INVALID_ARG for bad arguments (checked before anything is queued);
 * otherwise the first error of an underlying call, after the requests in
 * flight have been waited for and released (requests not served keep status
 * TB_ERR_NOT_READY and times -1; the failing one carries the error). */
typedef struct {
    double t_arrival_s;
    int32_t series_id;
    uint32_t count;               /* templates */
    const tb_template* templates; /* host */
    uint32_t first_template_id;
    uint32_t reserved;
} tb_serve_request;

typedef struct {
    double t_admit_s;
    double t_done_s;
    uint64_t cand_offset;
    uint64_t n_copied;
    uint64_t n_total;
    int32_t status;
    uint32_t reserved;
} tb_serve_result;

enum { TB_SERVE_SATURATE = 1 };
tb_status tb_serve(tb_plan_t plan, const tb_serve_request* req, uint32_t count, double time_scale, uint32_t flags,
                   tb_candidate* out, uint64_t capacity, tb_serve_result* res, uint32_t stats[2]);

/* Static description of a status (a utility; the paper defines nothing here). */
const char* tb_strerror(tb_status status);

/* Per-stage outputs of one template, for checking the stages one by one
 * (same kernels as tb_search_templates).  Host buffers, any may be NULL:
 *   src    int32[n]      input index read for output sample j (Algorithm 1)
 *   power  float[n/2+1]  P_k = |X_k|^2 of the demodulated series
 *   medians float[ceil((n/2)/W)]  whitening block medians (of the series itself
 *                        for a series loaded with TB_SERIES_WHITENING)
 *   sums   float[(log2(harm_max)+1) * (n/2+1)]  S_h[k] per fold
 * Candidates of this template are not kept. */
tb_status tb_inspect_template(tb_plan_t plan, int32_t series_id, const tb_template* t,
                              int32_t* src, float* power, float* medians, float* sums);

/* Per-fold power thresholds the plan compares S_h against (float), for
 * h = 1, 2, 4, 8, 16 (entries beyond harm_max are 0). */
tb_status tb_thresholds(tb_plan_t plan, float out[5]);

/* Milliseconds of device time of the last completed request's kernels, as
 * measured with HIP events on the plan stream (0 if none). */
tb_status tb_last_request_ms(tb_plan_t plan, int64_t request_id, double* ms);

/* Per-kernel device timing: with profiling on, HIP events are recorded on a
 * wave's stream before, between and after its kernels, for every `every`-th
 * wave queued (1 = all; a sample keeps the events' own cost out of the
 * measured throughput).  every > 0 clears earlier measurements and starts a
 * new one; 0 stops.  Negative values are rejected. */
tb_status tb_profile(tb_plan_t plan, int every);

/* Waits for queued work and reports, per kernel class, the summed device
 * milliseconds and launch counts of the timed waves since profiling started:
 *   [0] delay polynomials, [1] resample + FFT pass 1, [2] FFT pass 2 + power,
 *   [3] block medians and whitening (one kernel), [4] no longer used (0),
 *   [5] harmonic sum + threshold + compaction.
 * *templates receives the number of templates the timed waves processed.
 * Any output pointer may be NULL. */
tb_status tb_profile_read(tb_plan_t plan, double ms[6], uint64_t launches[6], uint64_t* templates);

/* Streaming copy of bytes (a multiple of 16) between two device buffers on the
 * plan stream, repeated reps times; *ms receives the mean device time of one
 * copy.  A measurement utility: the practical HBM ceiling. */
tb_status tb_stream_copy(tb_plan_t plan, void* dst, const void* src, uint64_t bytes, uint32_t reps, double* ms);

/* Incoherent dedispersion, the step that produces the searched series (App.
 * A.1 and Sec. 5.2 run it before the orbital search; no formula is given).
 * data: 8- or 4-bit filterbank, time-major (sample t's channels together),
 * host or device memory (flags TB_MEM_HOST / TB_MEM_DEVICE).  Channel c is at
 * fch1 + c foff MHz (foff may be negative).  For each DM dm[d] (pc cm^-3, >= 0)
 * the series out[d * nout + t] = sum_c x_c[t + s_dc], s_dc = rint(4.148808e3
 * dm (f_c^-2 - f_top^-2) / tsamp) samples behind the highest frequency f_top,
 * nout = nsamp - max s_dc (the samples every channel covers).  out is a
 * device array of ndm * nout floats owned by the caller (pass NULL to get
 * *nout only); the sums are exact.  The call allocates scratch of about
 * nchan * nsamp bytes (plus the packed input for host data) for its duration
 * and waits for the result; *kernel_ms (may be NULL) receives the device
 * time.
 * TB_ERR_INVALID_ARG for bad sizes (nchan 1..8192, nsamp < 2^31, ndm 1..2^20),
 * negative or non-finite DMs, a band reaching 0 Hz, or delays beyond the data. */
typedef struct {
    uint32_t nchan;
    uint32_t nbits;    /* 8, or 4: two channels per byte, the even channel in the low nibble
                          (nchan even); 0 means 8 */
    uint64_t nsamp;
    double fch1_mhz;
    double foff_mhz;
    double tsamp_s;
} tb_filterbank;
tb_status tb_dedisperse(tb_plan_t plan, const tb_filterbank* fb, const uint8_t* data, uint32_t flags, const double* dm,
                        uint32_t ndm, float* out, uint64_t* nout, double* kernel_ms);

/* Random template bank (Secs. 2.3-2.7).  Proper-volume density of the bank
 * at the given points: the square root of the determinant of the phase
 * metric (Sec. 2.2: time averages of products of phase derivatives, minus the
 * products of their averages) projected to constant spin frequency (Sec.
 * 2.5), times (2 pi f_max T)^n (Sec. 2.6), per unit of the bank's coordinates
 *   TB_BANK_CIRCULAR   (P_orb [s], tau [lt-s], alpha)            n = 3
 *   TB_BANK_ELLIPTICAL (P_orb, tau, alpha, e, psi = omega_rad)   n = 5.
 * The volume of a prior region is the integral of this density; the number
 * of random templates for coverage eta and mismatch m is
 * ln(1 - eta) / ln(1 - m^(n/2) C_n / V), C_n the unit n-ball volume, and the
 * templates are drawn with probability proportional to it.  Averages use
 * `nodes` Gauss-Legendre nodes over the observation (8..8192; 128 resolves
 * up to about 10 orbits).  points and out are host arrays of count entries
 * (templates must be valid: P_orb > 0, tau >= 0, 0 <= e < 1; e and psi are
 * ignored for circular banks); *kernel_ms (may be NULL) receives the device
 * time of the kernel.  FP64 throughout. */
enum { TB_BANK_CIRCULAR = 0, TB_BANK_ELLIPTICAL = 1 };
typedef struct {
    uint32_t kind;    /* TB_BANK_CIRCULAR or TB_BANK_ELLIPTICAL */
    uint32_t nodes;   /* quadrature nodes over the observation */
    double tobs_s;    /* observation time T */
    double fmax_hz;   /* highest spin frequency the bank is built for */
} tb_bank_metric;
tb_status tb_bank_density(tb_plan_t plan, const tb_bank_metric* m, const tb_template* points, uint64_t count,
                          double* out, double* kernel_ms);

/* Prior region of a random bank (Table 1): P_orb uniform in [porb_min_s, porb_max_s]; tau uniform below the
 * Kepler limit tau_max(P_orb) = (G M_sun / c^3)^(1/3) (2 pi / P_orb)^(-2/3) m_c / (m_p + m_c)^(2/3) lt-s for a
 * pulsar of at least m_pulsar_min_msun and a companion of at most m_comp_max_msun solar masses (Sec. 2.7); alpha
 * (and psi) uniform in [0, 2 pi); e uniform in [0, ecc_max) (elliptical banks, ecc_max > 0). */
typedef struct {
    double porb_min_s, porb_max_s;
    double m_pulsar_min_msun, m_comp_max_msun;
    double ecc_max;
} tb_bank_priors;

/* Proposals of a random bank (Secs. 2.5-2.7): maps count rows of uniform draws u (host, row-major, d = 3
 * values in [0, 1) per row for TB_BANK_CIRCULAR, d = 5 for TB_BANK_ELLIPTICAL, in the order P_orb, tau / tau_max,
 * alpha, e, psi) to points of the prior region, takes their proper-volume densities as tb_bank_density does, and
 * weighs each by density / proposal pdf.  points and weights (host, count entries) may be NULL.  stats[0] receives
 * the Monte-Carlo volume (the mean weight: the integral of the density over the region), stats[1] its standard
 * error, stats[2] the largest weight.  The caller draws u, so banks are reproducible from its generator.
 * TB_ERR_INVALID_ARG for a bad metric (as tb_bank_density) or priors (porb_min_s <= 0 or > porb_max_s, masses
 * <= 0, ecc_max outside (0, 1) for elliptical banks), count < 2 with stats. */
tb_status tb_bank_propose(tb_plan_t plan, const tb_bank_metric* m, const tb_bank_priors* priors, const double* u,
                          uint64_t count, tb_template* points, double* weights, double* stats, double* kernel_ms);

/* Number of random templates for coverage eta and maximal mismatch mu in a bank of proper volume V and dimension
 * n (Sec. 2.7): ln(1 - eta) / ln(1 - mu^(n/2) C_n / V), C_n = pi^(n/2) / Gamma(n/2 + 1) the volume of the unit
 * n-ball.  TB_ERR_INVALID_ARG unless V > 0, 0 < eta < 1, mu > 0, 1 <= n <= 16 and mu^(n/2) C_n < V. */
tb_status tb_bank_count(double volume, uint32_t n, double coverage, double mismatch, double* count);

/* Rejection step of the random bank: proposal i is kept (keep[i] = 1) when u[i] * wmax < weights[i], so kept
 * points are distributed as the density (Sec. 2.5).  *n_keep (may be NULL) receives the number kept, *n_above
 * (may be NULL) the number of weights above wmax (kept regardless; a scale that is too small shows there).
 * Host arrays of count entries.  TB_ERR_INVALID_ARG for NULL arrays with count > 0 or wmax <= 0. */
tb_status tb_bank_select(const double* weights, const double* u, uint64_t count, double wmax, uint8_t* keep,
                         uint64_t* n_keep, uint64_t* n_above);

/* Candidate grouping (App. A: the search software groups repeated detections
 * of the same signal and keeps the strongest; the paper gives no rule, this
 * is the library's).  Host arrays, no plan or device needed.
 *   F = bin * 16 / 2^log2_harm: the fundamental in sixteenths of a bin.
 *   Candidates are taken from the strongest (sigma descending, then series,
 *   template, log2_harm, bin ascending).  One that no stronger kept candidate
 *   has absorbed is kept, and absorbs every weaker, unabsorbed candidate of
 *   the same series_id whose F is within tol + ppm 1e-6 (p/q) F_kept of
 *   (p/q) F_kept for some integers 1 <= p, q <= max_ratio (1 = same frequency
 *   only), decided exactly: 1e6 |q F - p F_kept| <= 1e6 q tol + ppm p F_kept.
 *   tol is in sixteenths of a fundamental bin 1/T (16 = one bin).
 * out (n records, must not overlap in) receives the kept candidates in
 * strength order, group_size (may be NULL; n entries) how many candidates
 * each one's group holds (itself included), *n_kept their number.  Any input
 * order gives the same result.  TB_ERR_INVALID_ARG for NULL pointers with
 * n > 0, n >= 2^32, max_ratio outside 1..64, tol > 2^20, ppm > 1e6, a
 * log2_harm above 4 or a NaN sigma. */
tb_status tb_distill(const tb_candidate* in, uint64_t n, uint32_t max_ratio, uint32_t tol, uint32_t ppm,
                     tb_candidate* out, uint32_t* group_size, uint64_t* n_kept);

#ifdef __cplusplus
}
#endif
#endif
