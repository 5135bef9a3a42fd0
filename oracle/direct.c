/*
 * Acquisition oracle: plain FP64 time-domain cross-correlation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the bench's CPU
 * baseline leg may load this library.  It shares no code, header, table or
 * helper with the GPU path.
 *
 * Definition followed (the searching step of the paper, Section 3, steps 7-8:
 * cross-correlate the received samples with each stored replica; the paper's
 * correlation is extended here to complex baseband with a grid of carrier
 * offset hypotheses):
 *
 *   c[t][k][tau] = sum_{n=0}^{L-1} x[tau+n] * s_t[n] * exp(-j 2 pi f_k (tau+n) / Fs)
 *   P[t][k][tau] = |c[t][k][tau]|^2,     tau = 0 .. N-L   (valid lags only)
 *
 * with s_t the real +/-1 replica of tag t.  The exponential depends only on the
 * absolute sample index, so each bin mixes the block once,
 * x_k[i] = x[i] * exp(-j 2 pi f_k i / Fs), and then correlates x_k with the
 * real template; this is the same sum, term by term.
 *
 * Everything is double precision; the block arrives as complex64 and is
 * promoted exactly.  OpenMP splits the lag loop; each lag's sum runs over n in
 * increasing order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static const double kTwoPi = 6.283185307179586476925286766559;

/* x_k[i] = x[i] * exp(-j 2 pi f i / fs), i < n; x is complex64 interleaved. */
static void mix_block(const float* x, int64_t n, double f, double fs, double* re, double* im)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double ph = -kTwoPi * f * (double)i / fs;
        double c = cos(ph), s = sin(ph);
        double xr = (double)x[2 * i], xi = (double)x[2 * i + 1];
        re[i] = xr * c - xi * s;
        im[i] = xr * s + xi * c;
    }
}

/*
 * Full power array.  x: complex64 [n]; tmpl: double [T][L]; freqs: double [K];
 * P: double [T][K][n-L+1].  Returns 0, or -1 on bad sizes / allocation.
 */
int oracle_corr_power(const float* x, int64_t n, const double* tmpl, int32_t T, int64_t L,
                      const double* freqs, int32_t K, double fs, double* P)
{
    if (n < L || L <= 0 || T <= 0 || K <= 0) return -1;
    const int64_t lags = n - L + 1;
    double* re = (double*)malloc(sizeof(double) * (size_t)n);
    double* im = (double*)malloc(sizeof(double) * (size_t)n);
    if (!re || !im) { free(re); free(im); return -1; }
    for (int32_t k = 0; k < K; ++k) {
        mix_block(x, n, freqs[k], fs, re, im);
        for (int32_t t = 0; t < T; ++t) {
            const double* s = tmpl + (size_t)t * (size_t)L;
            double* out = P + ((size_t)t * (size_t)K + (size_t)k) * (size_t)lags;
#pragma omp parallel for schedule(static)
            for (int64_t tau = 0; tau < lags; ++tau) {
                double cr = 0.0, ci = 0.0;
                for (int64_t i = 0; i < L; ++i) {
                    cr += re[tau + i] * s[i];
                    ci += im[tau + i] * s[i];
                }
                out[tau] = cr * cr + ci * ci;
            }
        }
    }
    free(re);
    free(im);
    return 0;
}

/*
 * The same definition evaluated at an explicit list of points (t, k, tau), with
 * the exponential taken per term.  Used where the full array is too large.
 */
int oracle_corr_power_at(const float* x, int64_t n, const double* tmpl, int32_t T, int64_t L,
                         const double* freqs, int32_t K, double fs, int64_t npts,
                         const int32_t* tt, const int32_t* kk, const int64_t* taus, double* out)
{
    if (n < L || L <= 0) return -1;
    for (int64_t p = 0; p < npts; ++p)
        if (tt[p] < 0 || tt[p] >= T || kk[p] < 0 || kk[p] >= K || taus[p] < 0 || taus[p] > n - L)
            return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < npts; ++p) {
        const double* s = tmpl + (size_t)tt[p] * (size_t)L;
        const double f = freqs[kk[p]];
        const int64_t tau = taus[p];
        double cr = 0.0, ci = 0.0;
        for (int64_t i = 0; i < L; ++i) {
            int64_t idx = tau + i;
            double ph = -kTwoPi * f * (double)idx / fs;
            double c = cos(ph), sn = sin(ph);
            double xr = (double)x[2 * idx], xi = (double)x[2 * idx + 1];
            cr += (xr * c - xi * sn) * s[i];
            ci += (xr * sn + xi * c) * s[i];
        }
        out[p] = cr * cr + ci * ci;
    }
    return 0;
}

/* Number of threads the OpenMP runtime will use (for reporting). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the following calls (timing the oracle on fewer cores);
 * n < 1 restores the runtime's default.  Returns the count now in effect. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    static int dflt = 0;
    if (dflt == 0) dflt = omp_get_max_threads();
    omp_set_num_threads(n >= 1 ? n : dflt);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
