/*
 * tbo.c -- CPU oracle for the per-template coherent orbital search
 * (arXiv:2112.11991).  TEST INFRASTRUCTURE ONLY: see tbo.h.
 *
 * Everything is double precision and written in the order the method states
 * it.  Library routines used as single steps: libm sin/cos/sqrt/erfc/lgamma,
 * qsort.  No blocking, fusion or reordering beyond what is written here.
 */
#define _GNU_SOURCE
#include "tbo.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------- O1 ---- */
/* The series is taken with its mean removed: samples the resampler reads from
 * outside the observation then count as the mean (the mean-padding remark of
 * Sec. 2.8), and the DC bin carries no power. */
void tbo_mean_subtract(const float* x, int64_t n, float* x0)
{
    double sum = 0.0;
    for (int64_t i = 0; i < n; ++i) sum += (double)x[i];
    double mean = sum / (double)n;
    for (int64_t i = 0; i < n; ++i) x0[i] = (float)((double)x[i] - mean);
}

/* ------------------------------------------------------------- O2-O3 ---- */
/* Kepler's equation E - e sin E = M (Sec. 2.1), solved iteratively as the
 * resampling algorithm requires (Algorithm 1): Newton from E0 = M, stop once
 * the update is below 1e-12 rad, at most 64 updates. */
double tbo_kepler(double M, double e, int32_t* iters)
{
    int32_t it = 0;
    double E = M;
    if (e != 0.0) {
        for (it = 0; it < 64;) {
            double step = (E - e * sin(E) - M) / (1.0 - e * cos(E));
            E -= step;
            ++it;
            if (fabs(step) < 1e-12) break;
        }
    }
    if (iters) *iters = it;
    return E;
}

/* Roemer delay of the BT model (App. A.1, the equation of the BT Roemer delay):
 *   Delta = tau [ (cos E - e) sin psi + sqrt(1 - e^2) sin E cos psi ],
 * with the mean anomaly M = Omega t + alpha of the Kepler equation in Sec. 2.1
 * (Omega = 2 pi / P_orb, the mean angular velocity). */
double tbo_roemer_delay(const tbo_template* t, double time_s)
{
    double Omega = 2.0 * M_PI / t->porb_s;
    double M = Omega * time_s + t->alpha_rad;
    double E = tbo_kepler(M, t->ecc, NULL);
    double e = t->ecc;
    return t->tau_lts * ((cos(E) - e) * sin(t->omega_rad)
                         + sqrt(1.0 - e * e) * sin(E) * cos(t->omega_rad));
}

/* Nearest-neighbour demodulation (App. A.1, Algorithm 1).  The zero offset
 * Delta(0) (mean anomaly alpha at t = 0) is subtracted from the delay so that
 * output sample 0 reads input sample 0; output sample j reads input sample
 * j - [delta_j], [.] the nearest integer (ties to even), with the delay
 * evaluated at t_j = j tsamp. */
void tbo_resample_index(const tbo_template* t, int64_t n, double tsamp,
                        double* delta, int64_t* src)
{
    double d0 = tbo_roemer_delay(t, 0.0);
    for (int64_t j = 0; j < n; ++j) {
        double tj = (double)j * tsamp;
        double dj = (tbo_roemer_delay(t, tj) - d0) / tsamp;
        if (delta) delta[j] = dj;
        if (src) src[j] = j - (int64_t)rint(dj);
    }
}

/* O3 with the App. B expansion (the paper's ELL7): cos E and sqrt(1-e^2) sin E
 * replaced by their series in the mean anomaly, complete through e^6,
 *   cos E = sum_{k=0..7} C_k(e) cos kM,  sqrt(1-e^2) sin E = sum_{k=1..7} S_k(e) sin kM,
 * in the BT delay tau[(cos E - e) sin psi + sqrt(1-e^2) sin E cos psi].  No
 * Kepler solve; the truncation leaves O(e^7) of tau. */
static void appb_coefficients(double e, double* C, double* S)
{
    double e2 = e * e, e3 = e2 * e, e4 = e3 * e, e5 = e4 * e, e6 = e5 * e;
    C[0] = -0.5 * e;
    C[1] = 1.0 - 3.0 / 8.0 * e2 + 5.0 / 192.0 * e4 - 7.0 / 9216.0 * e6;
    C[2] = 0.5 * e - 1.0 / 3.0 * e3 + 1.0 / 16.0 * e5;
    C[3] = 3.0 / 8.0 * e2 - 45.0 / 128.0 * e4 + 567.0 / 5120.0 * e6;
    C[4] = 1.0 / 3.0 * e3 - 2.0 / 5.0 * e5;
    C[5] = 125.0 / 384.0 * e4 - 4375.0 / 9216.0 * e6;
    C[6] = 27.0 / 80.0 * e5;
    C[7] = 16807.0 / 46080.0 * e6;
    S[0] = 0.0;
    S[1] = 1.0 - 5.0 / 8.0 * e2 - 11.0 / 192.0 * e4 - 457.0 / 9216.0 * e6;
    S[2] = 0.5 * e - 5.0 / 12.0 * e3 + 1.0 / 24.0 * e5;
    S[3] = 3.0 / 8.0 * e2 - 51.0 / 128.0 * e4 + 543.0 / 5120.0 * e6;
    S[4] = 1.0 / 3.0 * e3 - 13.0 / 30.0 * e5;
    S[5] = 125.0 / 384.0 * e4 - 4625.0 / 9216.0 * e6;
    S[6] = 27.0 / 80.0 * e5;
    S[7] = 16807.0 / 46080.0 * e6;
}

double tbo_roemer_delay_series(const tbo_template* t, double time_s)
{
    double C[8], S[8];
    appb_coefficients(t->ecc, C, S);
    double Omega = 2.0 * M_PI / t->porb_s;
    double M = Omega * time_s + t->alpha_rad;
    double cosE = 0.0, sinE_b = 0.0;
    for (int k = 0; k <= 7; ++k) {
        cosE += C[k] * cos((double)k * M);
        sinE_b += S[k] * sin((double)k * M);
    }
    return t->tau_lts * ((cosE - t->ecc) * sin(t->omega_rad) + sinE_b * cos(t->omega_rad));
}

void tbo_resample_index_model(const tbo_template* t, int64_t n, double tsamp, int32_t model,
                              double* delta, int64_t* src)
{
    if (model == 0) {
        tbo_resample_index(t, n, tsamp, delta, src);
        return;
    }
    double d0 = tbo_roemer_delay_series(t, 0.0);
    for (int64_t j = 0; j < n; ++j) {
        double dj = (tbo_roemer_delay_series(t, (double)j * tsamp) - d0) / tsamp;
        if (delta) delta[j] = dj;
        if (src) src[j] = j - (int64_t)rint(dj);
    }
}

/* Samples the demodulated series needs from before the start or after the end
 * of the observation are zero, i.e. the (removed) mean. */
void tbo_resample(const float* x0, int64_t n, const int64_t* src, double* y)
{
    for (int64_t j = 0; j < n; ++j) {
        int64_t s = src[j];
        y[j] = (s >= 0 && s < n) ? (double)x0[s] : 0.0;
    }
}

/* ---------------------------------------------------------------- O5 ---- */
/* X_k = sum_n y_n exp(-2 pi i k n / N) for k = 0..N/2 by the definition, with
 * the exponent reduced exactly: k n mod N. */
void tbo_dft_naive(const double* y, int64_t n, double* re, double* im)
{
    double* c = (double*)malloc(sizeof(double) * (size_t)n);
    double* s = (double*)malloc(sizeof(double) * (size_t)n);
    for (int64_t r = 0; r < n; ++r) {
        c[r] = cos(2.0 * M_PI * (double)r / (double)n);
        s[r] = sin(2.0 * M_PI * (double)r / (double)n);
    }
    for (int64_t k = 0; k <= n / 2; ++k) {
        double ar = 0.0, ai = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            int64_t r = (k * j) % n;
            ar += y[j] * c[r];
            ai -= y[j] * s[r];
        }
        re[k] = ar;
        im[k] = ai;
    }
    free(c);
    free(s);
}

/* Iterative radix-2 decimation-in-time FFT of the full length-N complex
 * sequence y + 0i: bit-reversal permutation, then log2 N butterfly stages
 * with twiddles exp(-2 pi i r / N) taken from a cos/sin table. */
void tbo_fft(const double* y, int64_t n, double* re, double* im)
{
    double* ar = (double*)malloc(sizeof(double) * (size_t)n);
    double* ai = (double*)malloc(sizeof(double) * (size_t)n);
    double* c = (double*)malloc(sizeof(double) * (size_t)(n / 2 + 1));
    double* s = (double*)malloc(sizeof(double) * (size_t)(n / 2 + 1));
    int lg = 0;
    while (((int64_t)1 << lg) < n) ++lg;
    for (int64_t j = 0; j < n; ++j) {
        int64_t r = 0;
        for (int b = 0; b < lg; ++b)
            if (j & ((int64_t)1 << b)) r |= (int64_t)1 << (lg - 1 - b);
        ar[r] = y[j];
        ai[r] = 0.0;
    }
    for (int64_t r = 0; r <= n / 2; ++r) {
        c[r] = cos(2.0 * M_PI * (double)r / (double)n);
        s[r] = sin(2.0 * M_PI * (double)r / (double)n);
    }
    for (int64_t len = 2; len <= n; len <<= 1) {
        int64_t half = len / 2, step = n / len;
        for (int64_t base = 0; base < n; base += len) {
            for (int64_t q = 0; q < half; ++q) {
                double wr = c[q * step], wi = -s[q * step];
                int64_t u = base + q, v = base + q + half;
                double tr = ar[v] * wr - ai[v] * wi;
                double ti = ar[v] * wi + ai[v] * wr;
                ar[v] = ar[u] - tr;
                ai[v] = ai[u] - ti;
                ar[u] += tr;
                ai[u] += ti;
            }
        }
    }
    for (int64_t k = 0; k <= n / 2; ++k) {
        re[k] = ar[k];
        im[k] = ai[k];
    }
    free(ar);
    free(ai);
    free(c);
    free(s);
}

/* ---------------------------------------------------------------- O6 ---- */
/* Power |X_k|^2: the detection statistic P_n of Sec. 2.1 evaluated on the
 * FFT frequency grid of the demodulated series. */
void tbo_power(const double* re, const double* im, int64_t nbins, double* p)
{
    for (int64_t k = 0; k < nbins; ++k) p[k] = re[k] * re[k] + im[k] * im[k];
}

/* ---------------------------------------------------------------- O7 ---- */
static int cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

/* Red-noise removal ("Fourier de-reddening").  Bins 1..N/2 are cut into
 * consecutive blocks of W bins (the last may be short).  Each block's median
 * is its element of 0-based rank floor((n_b - 1)/2) in ascending order,
 * placed at the block centre start + (n_b - 1)/2.  The local level m(k) is
 * the straight line between neighbouring centres, held constant beyond the
 * first and last centre.  The whitened power is P_k ln2 / m(k), so that noise
 * powers have median ln 2 and mean 1, i.e. follow the exponential law behind
 * the chi^2 statistics of Sec. 2.1.  The DC bin is set to zero. */
/* The whitening level m(k) of every bin k >= 1 (lev[0] = 0): block medians
 * of p, joined by straight lines between block centres. */
static void whiten_levels(const double* p, int64_t nbins, int64_t w, double* med, double* lev)
{
    int64_t m = nbins - 1; /* bins 1..m */
    int64_t nb = (m + w - 1) / w;
    double* meds = (double*)malloc(sizeof(double) * (size_t)nb);
    double* cent = (double*)malloc(sizeof(double) * (size_t)nb);
    double* tmp = (double*)malloc(sizeof(double) * (size_t)w);
    for (int64_t b = 0; b < nb; ++b) {
        int64_t start = 1 + b * w;
        int64_t cnt = (m - b * w) < w ? (m - b * w) : w;
        memcpy(tmp, p + start, sizeof(double) * (size_t)cnt);
        qsort(tmp, (size_t)cnt, sizeof(double), cmp_double);
        meds[b] = tmp[(cnt - 1) / 2];
        cent[b] = (double)start + (double)(cnt - 1) / 2.0;
        if (med) med[b] = meds[b];
    }
    lev[0] = 0.0;
    int64_t b = 0;
    for (int64_t k = 1; k < nbins; ++k) {
        double level;
        double kk = (double)k;
        if (kk <= cent[0]) {
            level = meds[0];
        } else if (kk >= cent[nb - 1]) {
            level = meds[nb - 1];
        } else {
            while (!(cent[b] <= kk && kk < cent[b + 1])) ++b;
            double f = (kk - cent[b]) / (cent[b + 1] - cent[b]);
            level = meds[b] + (meds[b + 1] - meds[b]) * f;
        }
        lev[k] = level;
    }
    free(meds);
    free(cent);
    free(tmp);
}

/* P^_k = P_k ln2 / m(k) for k >= 1 (0 where m(k) is not positive), P^_0 = 0. */
static void whiten_apply(const double* p, int64_t nbins, const double* lev, double* phat)
{
    phat[0] = 0.0;
    for (int64_t k = 1; k < nbins; ++k) {
        double level = lev[k];
        phat[k] = (level > 0.0) ? p[k] * M_LN2 / level : 0.0;
    }
}

void tbo_whiten(const double* p, int64_t nbins, int64_t w, double* med, double* phat)
{
    double* lev = (double*)malloc(sizeof(double) * (size_t)nbins);
    whiten_levels(p, nbins, w, med, lev);
    whiten_apply(p, nbins, lev, phat);
    free(lev);
}

/* O7, once per series: the levels come from the spectrum of the mean-removed
 * series as loaded (no demodulation, y_j = x0_j) and serve every template
 * searched on it. */
int tbo_series_levels(const float* x0, const tbo_config* cfg, double* med, double* lev)
{
    int64_t n = cfg->n, nb = n / 2 + 1;
    double* y = (double*)malloc(sizeof(double) * (size_t)n);
    double* re = (double*)malloc(sizeof(double) * (size_t)nb);
    double* im = (double*)malloc(sizeof(double) * (size_t)nb);
    double* p = (double*)malloc(sizeof(double) * (size_t)nb);
    int rc = (y && re && im && p) ? 0 : -1;
    if (rc == 0) {
        for (int64_t j = 0; j < n; ++j) y[j] = (double)x0[j];
        if (n <= 4096) tbo_dft_naive(y, n, re, im);
        else tbo_fft(y, n, re, im);
        tbo_power(re, im, nb, p);
        whiten_levels(p, nb, cfg->whiten_window, med, lev);
    }
    free(y);
    free(re);
    free(im);
    free(p);
    return rc;
}

/* Birdie zapping (App. A and Sec. 5.2 list Fourier birdie zapping among the
 * per-series steps; no rule is given): known interference frequencies are
 * removed from the search by zeroing the whitened power of the bins whose
 * frequency k / T lies in a listed interval, before the harmonic sum. */
void tbo_zap(double* phat, int64_t nbins, double T, const double* lo_hz, const double* hi_hz, int32_t count)
{
    for (int32_t i = 0; i < count; ++i) {
        double lo = ceil(lo_hz[i] * T), hi = floor(hi_hz[i] * T);
        for (int64_t k = 1; k < nbins; ++k)
            if ((double)k >= lo && (double)k <= hi) phat[k] = 0.0;
    }
}

/* ---------------------------------------------------------------- O8 ---- */
/* Incoherent harmonic sum S_L = sum_{n <= 2^L} P_n (Sec. 2.1) on the bin grid:
 * bin k of fold h holds the h-th harmonic of a fundamental at k/h bins, and
 * harmonic m of it sits at bin round_half_up(m k / h).  Folding doubles h each
 * time, adding only the odd m of the new fold (the even ones are exactly the
 * previous fold's terms):
 *   S_1[k] = P[k],  S_2h[k] = S_h[k] + sum_{m = 1,3,...,2h-1} P[floor((2mk + 2h)/(4h))]. */
void tbo_harmsum(const double* phat, int64_t nbins, int32_t harm_max, double* s)
{
    int nf = 0;
    while ((1 << nf) < harm_max) ++nf;
    memcpy(s, phat, sizeof(double) * (size_t)nbins);
    for (int l = 1; l <= nf; ++l) {
        int64_t h2 = (int64_t)1 << l; /* the new fold 2h */
        int64_t h = h2 / 2;
        double* prev = s + (l - 1) * nbins;
        double* cur = s + l * nbins;
        for (int64_t k = 0; k < nbins; ++k) {
            double acc = prev[k];
            for (int64_t mm = 1; mm < h2; mm += 2) acc += phat[(2 * mm * k + 2 * h) / (4 * h)];
            cur[k] = acc;
        }
    }
}

/* ------------------------------------------------------------ O9-O10 ---- */
/* With whitened noise powers exponential of unit mean, S_h is a sum of h of
 * them: 2 S_h is chi^2 with 2h degrees of freedom (Sec. 2.1) and its tail is
 * Q(h, S) = exp(-S) sum_{k<h} S^k / k!. */
double tbo_log_tail(int32_t h, double s)
{
    if (s <= 0.0) return 0.0;
    double mx = -INFINITY;
    for (int32_t k = 0; k < h; ++k) {
        double t = (double)k * log(s) - lgamma((double)k + 1.0);
        if (t > mx) mx = t;
    }
    double acc = 0.0;
    for (int32_t k = 0; k < h; ++k) acc += exp((double)k * log(s) - lgamma((double)k + 1.0) - mx);
    return -s + mx + log(acc);
}

/* log of the one-sided Gaussian tail 0.5 erfc(z / sqrt 2); for z >= 30 the
 * asymptotic (Laplace) series of the Mills ratio. */
static double log_gauss_tail(double z)
{
    if (z < 30.0) return log(0.5 * erfc(z / sqrt(2.0)));
    double z2 = z * z;
    double series = 1.0 - 1.0 / z2 + 3.0 / (z2 * z2) - 15.0 / (z2 * z2 * z2)
                    + 105.0 / (z2 * z2 * z2 * z2);
    return -0.5 * z2 - log(z) - 0.5 * log(2.0 * M_PI) + log(series);
}

/* Power threshold with the same false-alarm probability per bin as a
 * one-sided Gaussian at sigma (bisection on log Q). */
double tbo_threshold(int32_t h, double sigma)
{
    double target = log_gauss_tail(sigma);
    double lo = 0.0, hi = 1.0;
    while (tbo_log_tail(h, hi) > target) hi *= 2.0;
    for (int i = 0; i < 200; ++i) {
        double mid = 0.5 * (lo + hi);
        if (tbo_log_tail(h, mid) > target) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Gaussian-equivalent significance of S_h = s (bisection in log space). */
double tbo_sigma(int32_t h, double s)
{
    double target = tbo_log_tail(h, s);
    double lo = -40.0, hi = 1e5;
    for (int i = 0; i < 300; ++i) {
        double mid = 0.5 * (lo + hi);
        if (log_gauss_tail(mid) > target) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------ pipeline -- */
typedef struct {
    int64_t* src;
    double* y;
    double* re;
    double* im;
    double* p;
    double* phat;
    double* s; /* running fold, nbins */
} work_t;

static int work_alloc(work_t* w, int64_t n)
{
    int64_t nb = n / 2 + 1;
    w->src = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    w->y = (double*)malloc(sizeof(double) * (size_t)n);
    w->re = (double*)malloc(sizeof(double) * (size_t)nb);
    w->im = (double*)malloc(sizeof(double) * (size_t)nb);
    w->p = (double*)malloc(sizeof(double) * (size_t)nb);
    w->phat = (double*)malloc(sizeof(double) * (size_t)nb);
    w->s = (double*)malloc(sizeof(double) * (size_t)nb);
    return (w->src && w->y && w->re && w->im && w->p && w->phat && w->s) ? 0 : -1;
}

static void work_free(work_t* w)
{
    free(w->src);
    free(w->y);
    free(w->re);
    free(w->im);
    free(w->p);
    free(w->phat);
    free(w->s);
}

static int valid_cfg(const tbo_config* c)
{
    if (c->n < 16 || (c->n & (c->n - 1))) return 0;
    if (!(c->tsamp > 0.0) || c->whiten_window < 1) return 0;
    if (c->harm_max != 1 && c->harm_max != 2 && c->harm_max != 4 && c->harm_max != 8
        && c->harm_max != 16)
        return 0;
    if (c->series_whitening != 0 && c->series_whitening != 1) return 0;
    if (c->delay_model != 0 && c->delay_model != 1) return 0;
    if (c->nzap < 0 || (c->nzap > 0 && (!c->zap_lo_hz || !c->zap_hi_hz))) return 0;
    return 1;
}

/* Demodulate, transform, power and whiten one template: with series levels
 * (lev non-NULL) those are applied, otherwise the template's own block
 * medians (into med, may be NULL). */
static void front_end(const float* x0, const tbo_config* c, const tbo_template* t, const double* lev,
                      double* med, work_t* w)
{
    int64_t n = c->n, nb = n / 2 + 1;
    tbo_resample_index_model(t, n, c->tsamp, c->delay_model, NULL, w->src);
    tbo_resample(x0, n, w->src, w->y);
    if (n <= 4096) tbo_dft_naive(w->y, n, w->re, w->im);
    else tbo_fft(w->y, n, w->re, w->im);
    tbo_power(w->re, w->im, nb, w->p);
    if (lev) whiten_apply(w->p, nb, lev, w->phat);
    else tbo_whiten(w->p, nb, c->whiten_window, med, w->phat);
    tbo_zap(w->phat, nb, (double)n * c->tsamp, c->zap_lo_hz, c->zap_hi_hz, c->nzap);
}

int tbo_template_stages(const float* x0, const tbo_config* cfg, const tbo_template* t,
                        int64_t* src, double* p, double* med, double* phat, double* s)
{
    if (!valid_cfg(cfg)) return -1;
    int64_t n = cfg->n, nb = n / 2 + 1;
    work_t w;
    double* lev = cfg->series_whitening ? (double*)malloc(sizeof(double) * (size_t)nb) : NULL;
    if (work_alloc(&w, n) || (cfg->series_whitening && (!lev || tbo_series_levels(x0, cfg, med, lev)))) {
        work_free(&w);
        free(lev);
        return -1;
    }
    front_end(x0, cfg, t, lev, lev ? NULL : med, &w);
    if (src) memcpy(src, w.src, sizeof(int64_t) * (size_t)n);
    if (p) memcpy(p, w.p, sizeof(double) * (size_t)nb);
    if (phat) memcpy(phat, w.phat, sizeof(double) * (size_t)nb);
    if (s) tbo_harmsum(w.phat, nb, cfg->harm_max, s);
    work_free(&w);
    free(lev);
    return 0;
}

typedef struct {
    tbo_candidate* v;
    int64_t n, cap;
} cand_list;

static int cand_push(cand_list* l, const tbo_candidate* c)
{
    if (l->n == l->cap) {
        int64_t nc = l->cap ? 2 * l->cap : 64;
        tbo_candidate* nv = (tbo_candidate*)realloc(l->v, sizeof(tbo_candidate) * (size_t)nc);
        if (!nv) return -1;
        l->v = nv;
        l->cap = nc;
    }
    l->v[l->n++] = *c;
    return 0;
}

typedef struct {
    const float* x0;
    const tbo_config* cfg;
    const tbo_template* t;
    const double* lev; /* series levels, or NULL for per-template whitening */
    uint32_t count, first_id, series_id;
    double thr[5];
    int64_t kmin;
    cand_list* lists;
    int64_t next; /* shared template counter */
    int failed;
} job_t;

/* Keep every (fold, bin) whose harmonic sum exceeds the fold's threshold,
 * for fundamentals in [fmin, fmax]: bins h*kmin .. min(N/2, floor(h fmax T)). */
static int pick(job_t* J, work_t* w, uint32_t ti)
{
    const tbo_config* c = J->cfg;
    int64_t nb = c->n / 2 + 1, m = nb - 1;
    double T = (double)c->n * c->tsamp;
    int nf = 0;
    while ((1 << nf) < c->harm_max) ++nf;
    memcpy(w->s, w->phat, sizeof(double) * (size_t)nb);
    for (int l = 0; l <= nf; ++l) {
        int64_t h = (int64_t)1 << l;
        if (l > 0) {
            int64_t hp = h / 2;
            for (int64_t k = 0; k < nb; ++k) {
                double acc = w->s[k];
                for (int64_t mm = 1; mm < h; mm += 2) acc += w->phat[(2 * mm * k + 2 * hp) / (4 * hp)];
                w->s[k] = acc;
            }
        }
        int64_t klo = h * J->kmin;
        int64_t khi = m;
        if (c->fmax_hz > 0.0) {
            int64_t kf = (int64_t)floor((double)h * c->fmax_hz * T);
            if (kf < khi) khi = kf;
        }
        for (int64_t k = klo; k <= khi; ++k) {
            if (w->s[k] > J->thr[l]) {
                tbo_candidate cd;
                cd.series_id = J->series_id;
                cd.template_id = J->first_id + ti;
                cd.bin = (uint32_t)k;
                cd.log2_harm = l;
                cd.power = w->s[k];
                cd.sigma = tbo_sigma((int32_t)h, w->s[k]);
                cd.freq_hz = (double)k / ((double)h * T);
                if (cand_push(&J->lists[ti], &cd)) return -1;
            }
        }
    }
    return 0;
}

static void* worker(void* arg)
{
    job_t* J = (job_t*)arg;
    work_t w;
    if (work_alloc(&w, J->cfg->n)) {
        __atomic_store_n(&J->failed, 1, __ATOMIC_SEQ_CST);
        work_free(&w);
        return NULL;
    }
    for (;;) {
        int64_t i = __atomic_fetch_add(&J->next, 1, __ATOMIC_SEQ_CST);
        if (i >= (int64_t)J->count) break;
        front_end(J->x0, J->cfg, &J->t[i], J->lev, NULL, &w);
        if (pick(J, &w, (uint32_t)i)) __atomic_store_n(&J->failed, 1, __ATOMIC_SEQ_CST);
    }
    work_free(&w);
    return NULL;
}

int tbo_search(const float* x0, const tbo_config* cfg, const tbo_template* t,
               uint32_t count, uint32_t first_template_id, uint32_t series_id,
               int32_t nthreads, tbo_candidate* out, int64_t capacity, int64_t* n_total)
{
    if (!x0 || !cfg || !valid_cfg(cfg) || (count && !t) || !n_total) return -1;
    job_t J;
    memset(&J, 0, sizeof(J));
    J.x0 = x0;
    J.cfg = cfg;
    J.t = t;
    J.count = count;
    J.first_id = first_template_id;
    J.series_id = series_id;
    for (int l = 0; l < 5; ++l) J.thr[l] = tbo_threshold(1 << l, cfg->threshold_sigma);
    double T = (double)cfg->n * cfg->tsamp;
    J.kmin = (int64_t)ceil(cfg->fmin_hz * T);
    if (J.kmin < 1) J.kmin = 1;
    double* lev = NULL;
    if (cfg->series_whitening) {
        lev = (double*)malloc(sizeof(double) * (size_t)(cfg->n / 2 + 1));
        if (!lev || tbo_series_levels(x0, cfg, NULL, lev)) {
            free(lev);
            return -1;
        }
        J.lev = lev;
    }
    J.lists = (cand_list*)calloc(count ? count : 1, sizeof(cand_list));
    if (!J.lists) {
        free(lev);
        return -1;
    }
    if (nthreads < 1) nthreads = 1;
    if ((uint32_t)nthreads > count && count > 0) nthreads = (int32_t)count;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    int started = 0;
    for (int i = 0; i < nthreads; ++i)
        if (pthread_create(&th[i], NULL, worker, &J) == 0) ++started;
    if (started == 0) worker(&J);
    for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
    free(th);
    int64_t tot = 0;
    for (uint32_t i = 0; i < count; ++i) {
        for (int64_t q = 0; q < J.lists[i].n; ++q) {
            if (out && tot < capacity) out[tot] = J.lists[i].v[q];
            ++tot;
        }
        free(J.lists[i].v);
    }
    free(J.lists);
    free(lev);
    *n_total = tot;
    return J.failed ? -1 : 0;
}

/* ----------------------------------------------------------- O11 -------- */
/* Candidate grouping (App. A: detections of the same signal are grouped and
 * the strongest kept; the paper gives no algorithm, so this is a definition).
 * Position of a candidate's fundamental in 1/16 fundamental bins:
 * F = 16 k / h = k * 2^(4 - log2_harm), an integer.  Strength order: sigma
 * descending, then series, template, fold, bin ascending.  A candidate b is
 * related to a stronger one a when they share the series and, for some
 * integers 1 <= p, q <= max_ratio, F_b lies within tol + ppm 1e-6 (p/q) F_a of
 * (p/q) F_a; times 1e6 q, in integers:
 *   1e6 |q F_b - p F_a| <= 1e6 q tol + ppm p F_a.
 * Walking the strength order, a candidate nobody
 * stronger has absorbed is kept and absorbs every weaker, not yet absorbed
 * candidate related to it. */
static int64_t cand_F(const tbo_candidate* c)
{
    return (int64_t)c->bin << (4 - c->log2_harm);
}

static int stronger(const tbo_candidate* a, const tbo_candidate* b)
{
    if (a->sigma != b->sigma) return a->sigma > b->sigma;
    if (a->series_id != b->series_id) return a->series_id < b->series_id;
    if (a->template_id != b->template_id) return a->template_id < b->template_id;
    if (a->log2_harm != b->log2_harm) return a->log2_harm < b->log2_harm;
    return a->bin < b->bin;
}

static const tbo_candidate* g_sort_base; /* qsort context (the oracle's grouping is not reentrant) */
static int cmp_strength(const void* x, const void* y)
{
    const tbo_candidate* a = &g_sort_base[*(const int64_t*)x];
    const tbo_candidate* b = &g_sort_base[*(const int64_t*)y];
    if (stronger(a, b)) return -1;
    if (stronger(b, a)) return 1;
    return 0;
}

static int related(const tbo_candidate* a, const tbo_candidate* b, int32_t max_ratio, int64_t tol, int64_t ppm)
{
    if (a->series_id != b->series_id) return 0;
    int64_t fa = cand_F(a), fb = cand_F(b);
    for (int64_t p = 1; p <= max_ratio; ++p)
        for (int64_t q = 1; q <= max_ratio; ++q) {
            int64_t d = q * fb - p * fa;
            if (d < 0) d = -d;
            if (1000000 * d <= 1000000 * q * tol + ppm * p * fa) return 1;
        }
    return 0;
}

int tbo_distill(const tbo_candidate* in, int64_t n, int32_t max_ratio, int64_t tol, int64_t ppm,
                tbo_candidate* out, int64_t* group, int64_t* n_kept)
{
    if (n < 0 || (n > 0 && (!in || !out)) || !n_kept || max_ratio < 1 || max_ratio > 64 || tol < 0 ||
        tol > (1 << 20) || ppm < 0 || ppm > 1000000)
        return -1;
    for (int64_t i = 0; i < n; ++i)
        if (in[i].log2_harm < 0 || in[i].log2_harm > 4 || in[i].sigma != in[i].sigma) return -1;
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    char* absorbed = (char*)calloc((size_t)(n ? n : 1), 1);
    if (!order || !absorbed) {
        free(order);
        free(absorbed);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) order[i] = i;
    g_sort_base = in;
    qsort(order, (size_t)n, sizeof(int64_t), cmp_strength);
    int64_t kept = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t a = order[i];
        if (absorbed[a]) continue;
        int64_t members = 1;
        for (int64_t j = i + 1; j < n; ++j) {
            int64_t b = order[j];
            if (!absorbed[b] && related(&in[a], &in[b], max_ratio, tol, ppm)) {
                absorbed[b] = 1;
                ++members;
            }
        }
        out[kept] = in[a];
        if (group) group[kept] = members;
        ++kept;
    }
    *n_kept = kept;
    free(order);
    free(absorbed);
    return 0;
}

/* ----------------------------------------------------------- O0 --------- */
/* Cold-plasma dispersion: a pulse at frequency f arrives K_DM DM / f^2 later
 * than at infinite frequency, K_DM = e^2 / (2 pi m_e c) in units of
 * s MHz^2 pc^-1 cm^3 (the paper names dedispersion without a formula). */
double tbo_dispersion_constant(void) { return 4.148808e3; }

/* Sample (t, c) of a time-major filterbank of 8-bit values, or of 4-bit
 * values packed two channels per byte with the even channel in the low
 * nibble. */
static unsigned fb_sample(const uint8_t* data, int32_t nbits, int32_t nchan, int64_t t, int32_t c)
{
    if (nbits == 8) return data[(size_t)t * nchan + c];
    uint8_t b = data[((size_t)t * nchan + c) / 2];
    return (c % 2 == 0) ? (b & 15u) : (b >> 4);
}

int64_t tbo_dedisperse(const uint8_t* data, int32_t nbits, int32_t nchan, int64_t nsamp, double fch1_mhz,
                       double foff_mhz, double tsamp, const double* dm, int32_t ndm, float* out)
{
    if (!data || nchan < 1 || nsamp < 1 || !(tsamp > 0.0) || !dm || ndm < 1 || !(fch1_mhz > 0.0)) return -1;
    if (nbits != 8 && !(nbits == 4 && nchan % 2 == 0)) return -1;
    double ftop = fch1_mhz > fch1_mhz + (nchan - 1) * foff_mhz ? fch1_mhz : fch1_mhz + (nchan - 1) * foff_mhz;
    double fbot = fch1_mhz < fch1_mhz + (nchan - 1) * foff_mhz ? fch1_mhz : fch1_mhz + (nchan - 1) * foff_mhz;
    if (!(fbot > 0.0)) return -1;
    int64_t* s = (int64_t*)malloc(sizeof(int64_t) * (size_t)ndm * (size_t)nchan);
    if (!s) return -1;
    int64_t smax = 0;
    for (int32_t d = 0; d < ndm; ++d) {
        if (!(dm[d] >= 0.0)) {
            free(s);
            return -1;
        }
        for (int32_t c = 0; c < nchan; ++c) {
            double f = fch1_mhz + c * foff_mhz;
            double delay = tbo_dispersion_constant() * dm[d] * (1.0 / (f * f) - 1.0 / (ftop * ftop));
            int64_t v = (int64_t)rint(delay / tsamp);
            s[(size_t)d * nchan + c] = v;
            if (v > smax) smax = v;
        }
    }
    int64_t nout = nsamp - smax;
    if (nout < 1) {
        free(s);
        return -1;
    }
    if (out)
        for (int32_t d = 0; d < ndm; ++d)
            for (int64_t t = 0; t < nout; ++t) {
                double acc = 0.0;
                for (int32_t c = 0; c < nchan; ++c) acc += (double)fb_sample(data, nbits, nchan, t + s[(size_t)d * nchan + c], c);
                out[(size_t)d * nout + t] = (float)acc;
            }
    free(s);
    return nout;
}
