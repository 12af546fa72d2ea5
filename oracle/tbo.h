/*
 * tbo.h -- CPU oracle for the per-template coherent orbital search of
 * Balakrishnan et al., "Coherent Search for Binary Pulsars across all Five
 * Keplerian Parameters in Radio Observations using the template-bank
 * algorithm" (arXiv:2112.11991).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, double-precision C
 * restatement of what the search computes, written so that each step can be
 * checked against the paper by eye.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  The product library
 * (include/tb.h) never links, calls or includes anything here, and the two
 * share no code, tables or constants.
 *
 * Steps and the passages they follow:
 *   O0 dedispersion ......... incoherent shift-and-add over channels, the
 *                             step before the search (App. A, Sec. 5.2;
 *                             the paper names it without a formula)
 *   O1 mean removal ......... zero-mean convention of the mean-padding remark
 *                             (Sec. 2.8, Template Bank Verification)
 *   O2 mean anomaly ......... Kepler equation, Sec. 2.1 (M = Omega t + alpha)
 *   O3 Kepler + Roemer delay  Sec. 2.1 Kepler equation; App. A.1 eq.
 *                             "romer delay bt" (BT model)
 *   O4 nearest-neighbour index App. A.1 and Algorithm 1 (zero offset at t=0)
 *   O5 DFT .................. Sec. 2.4 (uniform spin-frequency grid by FFT)
 *   O6 power ................ Sec. 2.1, equation of the power statistic
 *   O7 whitening ............ "Fourier de-reddening", Sec. 5.2 / App. A
 *                             (method not given by the paper: block medians,
 *                             linear interpolation, normalised so that noise
 *                             powers follow the chi^2 law of Sec. 2.1), per
 *                             template or once per series
 *   O8 harmonic sum ......... Sec. 2.1 (S_L = sum_{n<=2^L} P_n), 16 harmonics
 *                             (Sec. 5.2)
 *   O9 thresholds ........... Sec. 2.1 (chi^2 with 2^(L+1) dof, false alarm)
 *   O10 candidates .......... peak detection, App. A
 *   O11 grouping ............ candidate reduction by grouping repeated
 *                             detections, App. A (method not given by the
 *                             paper: greedy harmonic grouping, see tbo.c)
 */
#ifndef TBO_H
#define TBO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One orbital template (Sec. 2.1: tau = a sin(eps)/c, Omega = 2 pi / P_orb,
 * alpha initial orbital phase, e eccentricity, psi longitude of periastron).
 * A circular template has ecc = 0 and omega_rad = 0. */
typedef struct {
    double porb_s;
    double tau_lts;
    double alpha_rad;
    double ecc;
    double omega_rad;
} tbo_template;

typedef struct {
    int64_t n;               /* samples, power of two */
    double  tsamp;           /* sampling time [s] */
    int32_t harm_max;        /* 1, 2, 4, 8 or 16 */
    int64_t whiten_window;   /* W, bins per median block */
    double  threshold_sigma; /* one-sided Gaussian-equivalent threshold */
    double  fmin_hz;         /* lowest fundamental searched */
    double  fmax_hz;         /* highest fundamental searched; 0 = Nyquist */
    int32_t series_whitening; /* 0: each template whitened by its own block
                                 medians; 1: levels taken once from the
                                 series' own spectrum (tbo_series_levels) */
    int32_t delay_model;      /* 0: BT with the Newton Kepler solve; 1: the
                                 App. B series (tbo_roemer_delay_series) */
    int32_t nzap;             /* birdies: whitened powers of bins k with    */
    const double* zap_lo_hz;  /* zap_lo_hz[i] <= k / T <= zap_hi_hz[i]      */
    const double* zap_hi_hz;  /* are set to 0 (tbo_zap); nzap = 0: none     */
} tbo_config;

typedef struct {
    uint32_t series_id;
    uint32_t template_id;
    uint32_t bin;        /* bin index k of the harmonic-summed spectrum */
    int32_t  log2_harm;  /* fold: h = 2^log2_harm harmonics summed */
    double   power;      /* S_h[k] */
    double   sigma;      /* Gaussian-equivalent significance */
    double   freq_hz;    /* fundamental frequency k / (h T) */
} tbo_candidate;

/* O1 */
void tbo_mean_subtract(const float* x, int64_t n, float* x0);

/* O3: Newton solve of E - e sin E = M from E0 = M; returns E, *iters (may be
 * NULL) receives the number of updates made. */
double tbo_kepler(double M, double e, int32_t* iters);

/* O2-O3: Roemer delay Delta(t) [s] of a template at time t [s]. */
double tbo_roemer_delay(const tbo_template* t, double time_s);

/* O4: delta_j = (Delta(j tsamp) - Delta(0)) / tsamp for j < n (may be NULL)
 * and src_j = j - rint(delta_j). */
void tbo_resample_index(const tbo_template* t, int64_t n, double tsamp,
                        double* delta, int64_t* src);

/* O3 through the App. B series of cos E and sqrt(1-e^2) sin E in the mean
 * anomaly (complete through e^6, the paper's ELL7), no Kepler solve. */
double tbo_roemer_delay_series(const tbo_template* t, double time_s);

/* O4 with the delay of model 0 (BT, Newton) or 1 (App. B series). */
void tbo_resample_index_model(const tbo_template* t, int64_t n, double tsamp, int32_t model,
                              double* delta, int64_t* src);

/* O4: y_j = x0[src_j] inside [0, n), else 0. */
void tbo_resample(const float* x0, int64_t n, const int64_t* src, double* y);

/* O5: X_k = sum_n y_n exp(-2 pi i k n / n), k = 0..n/2.  The naive version
 * is O(n^2); the radix-2 version is the oracle's own FFT. */
void tbo_dft_naive(const double* y, int64_t n, double* re, double* im);
void tbo_fft(const double* y, int64_t n, double* re, double* im);

/* O6: P_k = Re^2 + Im^2, k = 0..n/2. */
void tbo_power(const double* re, const double* im, int64_t nbins, double* p);

/* O7: nbins = n/2 + 1.  med receives the block medians (ceil((nbins-1)/W)
 * values; may be NULL), phat the whitened spectrum. */
void tbo_whiten(const double* p, int64_t nbins, int64_t w, double* med, double* phat);

/* O7 once per series: block medians (ceil((nbins-1)/W) values, may be NULL)
 * and the interpolated level m(k), k = 0..n/2 (lev[0] = 0), of the spectrum
 * of x0 itself.  A template searched with cfg->series_whitening = 1 has
 * P^_k = P_k ln2 / m(k).  Returns 0, or -1 on allocation failure. */
int tbo_series_levels(const float* x0, const tbo_config* cfg, double* med, double* lev);

/* O7b birdie zapping: phat_k = 0 for every bin k (1..nbins-1) with
 * lo_hz[i] <= k / T <= hi_hz[i] for some i, T = n tsamp; i.e. k from
 * ceil(lo T) to floor(hi T). */
void tbo_zap(double* phat, int64_t nbins, double T, const double* lo_hz, const double* hi_hz, int32_t count);

/* O8: all folds 1..harm_max.  s has (log2(harm_max)+1) * nbins doubles,
 * fold l at s + l*nbins. */
void tbo_harmsum(const double* phat, int64_t nbins, int32_t harm_max, double* s);

/* O9: threshold on S_h so that one bin exceeds it by chance with the
 * one-sided Gaussian tail probability of sigma. */
double tbo_threshold(int32_t h, double sigma);
/* log of the chi^2 tail, log Q(h, S) with Q the regularised upper incomplete
 * gamma of integer order h. */
double tbo_log_tail(int32_t h, double s);
/* O10: Gaussian-equivalent significance of S_h = s. */
double tbo_sigma(int32_t h, double s);

/* Per-stage outputs for one template (any pointer may be NULL except x0). */
int tbo_template_stages(const float* x0, const tbo_config* cfg, const tbo_template* t,
                        int64_t* src, double* p, double* med, double* phat, double* s);

/* O1-O10 for count templates of one mean-subtracted series, spread over
 * nthreads host threads.  Candidates are sorted by (template, fold, bin);
 * *n_total receives the full count even when it exceeds capacity.
 * Returns 0, or -1 on bad arguments / allocation failure. */
int tbo_search(const float* x0, const tbo_config* cfg, const tbo_template* t,
               uint32_t count, uint32_t first_template_id, uint32_t series_id,
               int32_t nthreads, tbo_candidate* out, int64_t capacity, int64_t* n_total);

/* O0 dedispersion (upstream of the search; App. A, Sec. 5.2): the series for
 * dispersion measure dm[d] is out[d * nout + t] = sum over channels c of
 * x[t + s_dc][c] for t < nout, x time-major 8-bit samples (or 4-bit: two
 * channels per byte, the even channel in the low nibble), channel c
 * at f_c = fch1 + c foff [MHz], s_dc = rint(K_DM dm[d] (f_c^-2 - f_top^-2) / tsamp)
 * with f_top the highest channel frequency and K_DM the dispersion constant
 * (tbo_dispersion_constant); nout = nsamp - max over d, c of s_dc.
 * Returns nout, or -1 on bad arguments (nout < 1 included). */
double tbo_dispersion_constant(void);
int64_t tbo_dedisperse(const uint8_t* data, int32_t nbits, int32_t nchan, int64_t nsamp, double fch1_mhz,
                       double foff_mhz, double tsamp, const double* dm, int32_t ndm, float* out);

/* O11 candidate grouping: the kept candidates (strongest of each group) in
 * strength order into out (n records), their group sizes into group (may be
 * NULL), their count into *n_kept.  max_ratio (1..64) bounds p and q of the
 * harmonic ratios p/q; the tolerance is tol (0..2^20) sixteenths of a
 * fundamental bin (1/(16 T)) plus ppm (0..1e6) parts per million of the
 * target (p/q) F.  Returns 0, or -1 on bad arguments / allocation failure. */
int tbo_distill(const tbo_candidate* in, int64_t n, int32_t max_ratio, int64_t tol, int64_t ppm,
                tbo_candidate* out, int64_t* group, int64_t* n_kept);

#ifdef __cplusplus
}
#endif
#endif
