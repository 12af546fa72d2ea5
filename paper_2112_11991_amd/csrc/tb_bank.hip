// tb_bank.hip -- proper-volume density of the random template bank
// (Secs. 2.3-2.7): for each point of the orbital parameter space, the square
// root of the determinant of the phase metric projected to constant spin
// frequency, scaled by (2 pi f_max T)^n and expressed per unit of the bank's
// coordinates (P_orb, tau, alpha) or (P_orb, tau, alpha, e, psi).
//
// Phase (dimensionless, Sec. 2.6): kappa u + X cos E + Y sqrt(1-e^2) sin E with
// u = t/T, X = tau sin(psi)/T, Y = tau cos(psi)/T, M = Omega T u + alpha; a
// circular orbit has kappa u + tau' sin(M), tau' = tau/T.  Metric (Sec. 2.2):
// g_ab = <d_a Phi d_b Phi> - <d_a Phi><d_b Phi> over u in [0, 1]; projection
// (Sec. 2.5): gamma_ab = g_ab - g_ka g_kb / g_kk with d_kappa Phi = u.
//
// One thread per point makes three quadrature passes in FP64 registers
// (the averages are smooth integrals; Gauss-Legendre nodes come from the
// host), then takes the determinant by elimination with partial pivoting.
// FP64 throughout: the elliptical metric is nearly singular for small e.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "tb_internal.h"

namespace tb {
namespace {

template <int N>
__device__ __forceinline__ double det_pivot(double (&a)[N][N])
{
    double det = 1.0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        int p = c;
        double best = fabs(a[c][c]);
#pragma unroll
        for (int r = c + 1; r < N; ++r)
            if (fabs(a[r][c]) > best) {
                best = fabs(a[r][c]);
                p = r;
            }
        if (best == 0.0) return 0.0;
        if (p != c) {
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const double t = a[c][k];
                a[c][k] = a[p][k];
                a[p][k] = t;
            }
            det = -det;
        }
        det *= a[c][c];
#pragma unroll
        for (int r = c + 1; r < N; ++r) {
            const double f = a[r][c] / a[c][c];
#pragma unroll
            for (int k = c; k < N; ++k) a[r][k] -= f * a[c][k];
        }
    }
    return det;
}

__device__ __forceinline__ double kepler_newton(double M, double e)
{
    double E = M;
    for (int it = 0; it < 64; ++it) {
        double s, c;
        sincos(E, &s, &c);
        const double step = (E - e * s - M) / (1.0 - e * c);
        E -= step;
        if (fabs(step) < 1e-15) break;
    }
    return E;
}

// N = 3 (circular) or 5 (elliptical) parameters.
template <int N>
__global__ __launch_bounds__(256) void k_bank_density(const tb_template* __restrict__ pts, uint32_t count,
                                                      const double2* __restrict__ gl, int nodes, double T,
                                                      double chi_n, double* __restrict__ out)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= count) return;
    const tb_template t = pts[i];
    const double Op = 2.0 * M_PI / t.porb_s * T;
    const double e = t.ecc, b = sqrt(1.0 - e * e);
    const double X = t.tau_lts * sin(t.omega_rad) / T, Y = t.tau_lts * cos(t.omega_rad) / T, tp = t.tau_lts / T;
    // d Phi~ / d lambda at u: circular (tau', Omega', alpha), elliptical (X, Y, e, Omega', alpha)
    auto derivs = [&](double u, double (&d)[N]) {
        const double M = Op * u + t.alpha_rad;
        if constexpr (N == 3) {
            double s, c;
            sincos(M, &s, &c);
            d[0] = s;
            d[1] = tp * u * c;
            d[2] = tp * c;
        } else {
            const double E = kepler_newton(M, e);
            double sE, cE;
            sincos(E, &sE, &cE);
            const double q = 1.0 / (1.0 - e * cE);  // dE/dM; dE/de = sin E q
            const double A = -X * sE + Y * b * cE;  // d/dE of X cos E + Y b sin E
            d[0] = cE;
            d[1] = b * sE;
            d[2] = A * (sE * q) - Y * e / b * sE;
            d[3] = A * q * u;
            d[4] = A * q;
        }
    };
    // Two passes: the weighted means and slopes in u of the derivatives, then
    // the average products of their residuals after that straight-line fit.
    // This is g_ab - g_ka g_kb / g_kk (d_kappa Phi~ = u) without subtracting
    // nearly equal terms when the orbital arc is short.
    double S[N], Su[N];
    double su = 0.0, suu = 0.0;
#pragma unroll
    for (int a = 0; a < N; ++a) S[a] = Su[a] = 0.0;
    for (int j = 0; j < nodes; ++j) {
        const double2 uw = gl[j];
        double d[N];
        derivs(uw.x, d);
        su += uw.y * uw.x;
#pragma unroll
        for (int a = 0; a < N; ++a) S[a] += uw.y * d[a];
    }
    for (int j = 0; j < nodes; ++j) {
        const double2 uw = gl[j];
        const double uc = uw.x - su;
        double d[N];
        derivs(uw.x, d);
        suu += uw.y * uc * uc;
#pragma unroll
        for (int a = 0; a < N; ++a) Su[a] += uw.y * (d[a] - S[a]) * uc;
    }
    double slope[N];
#pragma unroll
    for (int a = 0; a < N; ++a) slope[a] = Su[a] / suu;
    double gam[N][N];
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int c = 0; c < N; ++c) gam[a][c] = 0.0;
    for (int j = 0; j < nodes; ++j) {
        const double2 uw = gl[j];
        const double uc = uw.x - su;
        double d[N], r[N];
        derivs(uw.x, d);
#pragma unroll
        for (int a = 0; a < N; ++a) r[a] = d[a] - S[a] - slope[a] * uc;
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
            for (int c = 0; c <= a; ++c) gam[a][c] += uw.y * r[a] * r[c];
    }
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int c = 0; c < a; ++c) gam[c][a] = gam[a][c];
    const double det = det_pivot<N>(gam);
    // per unit of (P_orb, tau, alpha[, e, psi])
    const double jac = N == 3 ? 2.0 * M_PI / (t.porb_s * t.porb_s)
                              : t.tau_lts * 2.0 * M_PI / (T * t.porb_s * t.porb_s);
    out[i] = sqrt(det > 0.0 ? det : 0.0) * chi_n * jac;
}

// Gauss-Legendre nodes and weights on [0, 1] (Newton on P_n from the
// Chebyshev-like first guesses).
std::vector<double2> gauss_legendre(int n)
{
    std::vector<double2> r(n);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        const double w = 2.0 / ((1.0 - x * x) * dp * dp);
        r[i] = make_double2(0.5 * (1.0 - x), 0.5 * w);
        r[n - 1 - i] = make_double2(0.5 * (1.0 + x), 0.5 * w);
    }
    return r;
}

}  // namespace

hipError_t launch_bank_density(int kind, int nodes, double T, double fmax, const tb_template* d_pts, uint32_t count,
                               double* d_out, hipStream_t s, double* ms)
{
    std::vector<double2> gl = gauss_legendre(nodes);
    double2* d_gl = nullptr;
    hipError_t e = hipMalloc(&d_gl, sizeof(double2) * nodes);
    if (e != hipSuccess) return e;
    hipEvent_t ev[2] = {nullptr, nullptr};
    e = hipMemcpyAsync(d_gl, gl.data(), sizeof(double2) * nodes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && ms) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess && ms) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess && ms) e = hipEventRecord(ev[0], s);
    const double chi = 2.0 * M_PI * fmax * T;
    const dim3 grid((count + 255) / 256);
    if (e == hipSuccess && count) {
        if (kind == 0)
            hipLaunchKernelGGL(k_bank_density<3>, grid, dim3(256), 0, s, d_pts, count, d_gl, nodes, T, chi * chi * chi,
                               d_out);
        else
            hipLaunchKernelGGL(k_bank_density<5>, grid, dim3(256), 0, s, d_pts, count, d_gl, nodes, T,
                               chi * chi * chi * chi * chi, d_out);
        e = hipGetLastError();
    }
    if (e == hipSuccess && ms) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && ms) {
        float f = 0.0f;
        e = hipEventElapsedTime(&f, ev[0], ev[1]);
        *ms = f;
    }
    for (hipEvent_t x : ev)
        if (x) hipEventDestroy(x);
    hipFree(d_gl);
    return e;
}

}  // namespace tb
