/*
 * Plain FP64 CPU oracle of the polyphase-filter-bank spectrometer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may build, load or run
 * it; the product path never does.  It shares no code, header, table or
 * constant with the GPU library.
 *
 * What it computes (paper, Section 4):
 *   - unpack: two's-complement 8-bit complex samples -> double (exact);
 *   - pre-filter (polyphase filter bank, weighted overlap-add): spectrum j is
 *       y_j[n] = sum_{p=0}^{P-1} h[p*N + n] * x[(j+p)*N + n],   n in [0, N),
 *     i.e. P consecutive N-sample frames weighted by the prototype filter h
 *     (the paper's 8-tap PFB); direct-FFT mode is y_j[n] = x[j*N + n];
 *   - DFT of each y_j, forward, unnormalised, natural bin order:
 *       X_j[k] = sum_n y_j[n] exp(-2 pi i k n / N),
 *     computed by an iterative radix-2 decimation-in-time FFT whose twiddles
 *     are evaluated per index (no recurrences), plus a brute-force O(N^2) DFT;
 *   - polarisation products |X|^2, |Y|^2, Re(X Y*), Im(X Y*);
 *   - accumulation of the products over consecutive spectra, summed
 *     sequentially in spectrum order.
 *
 * Readings where the paper is silent (each one is listed with its reason in
 * the design notes of the repository):
 *   - prototype filter: h[m] = sinc((m - P*N/2)/N) * w[m], m in [0, P*N),
 *     sinc(u) = sin(pi u)/(pi u), sinc(0) = 1, periodic Hann
 *     w[m] = 1/2 - 1/2 cos(2 pi m / (P*N)), no gain normalisation;
 *   - h[p*N + n] multiplies frame j+p (correlation form), hop = N;
 *   - the first spectrum needs P frames (no zero-padded warm-up);
 *   - cross product is X * conj(Y): Re = XrYr + XiYi, Im = XiYr - XrYi.
 *
 * Sample layout: int8 x[T][n_pol][2] (time-major; re, im per polarisation).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_WINDOW_HANN_SINC 0
#define ORC_WINDOW_RECT 1

static const double ORC_PI = 3.14159265358979323846264338327950288;

/* ---- unpack ------------------------------------------------------------ */

/* Two's-complement int8 to double.  Exact for every byte, -128 included. */
void orc_unpack(const int8_t *in, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = (double)in[i];
}

/* ---- prototype filter ---------------------------------------------------- */

static double orc_sinc(double u)
{
    if (u == 0.0)
        return 1.0;
    return sin(ORC_PI * u) / (ORC_PI * u);
}

/* Filter taps h[0 .. P*N).  Returns 0 on success, -1 on a bad argument. */
int orc_taps(int64_t N, int32_t P, int32_t window, double *h)
{
    if (N < 1 || P < 1)
        return -1;
    const int64_t L = (int64_t)P * N;
    for (int64_t m = 0; m < L; ++m) {
        if (window == ORC_WINDOW_RECT) {
            h[m] = 1.0;
        } else if (window == ORC_WINDOW_HANN_SINC) {
            double u = (double)(m - L / 2) / (double)N;
            double w = 0.5 - 0.5 * cos(2.0 * ORC_PI * (double)m / (double)L);
            h[m] = orc_sinc(u) * w;
        } else {
            return -1;
        }
    }
    return 0;
}

/* ---- transforms -------------------------------------------------------- */

/* Brute-force DFT, forward, unnormalised: O(N^2).  The angle of every term is
 * reduced exactly (k*n mod N) before the trigonometric call. */
void orc_dft(const double *re, const double *im, int64_t N, double *ore, double *oim)
{
    for (int64_t k = 0; k < N; ++k) {
        double sr = 0.0, si = 0.0;
        for (int64_t n = 0; n < N; ++n) {
            int64_t r = (int64_t)(((__int128)k * n) % N);
            double a = -2.0 * ORC_PI * (double)r / (double)N;
            double c = cos(a), s = sin(a);
            sr += re[n] * c - im[n] * s;
            si += re[n] * s + im[n] * c;
        }
        ore[k] = sr;
        oim[k] = si;
    }
}

static int orc_is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

/* In-place iterative radix-2 decimation-in-time FFT (forward, unnormalised,
 * natural order out).  N must be a power of two.  Returns -1 otherwise. */
int orc_fft(double *re, double *im, int64_t N)
{
    if (!orc_is_pow2(N))
        return -1;
    /* bit-reversal permutation of the input */
    int bits = 0;
    while (((int64_t)1 << bits) < N)
        ++bits;
    for (int64_t i = 0; i < N; ++i) {
        int64_t r = 0;
        for (int b = 0; b < bits; ++b)
            if (i & ((int64_t)1 << b))
                r |= (int64_t)1 << (bits - 1 - b);
        if (r > i) {
            double t = re[i]; re[i] = re[r]; re[r] = t;
            t = im[i]; im[i] = im[r]; im[r] = t;
        }
    }
    /* butterflies: merge pairs of length-(len/2) transforms */
    for (int64_t len = 2; len <= N; len <<= 1) {
        int64_t half = len >> 1;
        for (int64_t s = 0; s < N; s += len) {
            for (int64_t t = 0; t < half; ++t) {
                /* twiddle W_len^t = exp(-2 pi i t / len), evaluated directly */
                double a = -2.0 * ORC_PI * (double)t / (double)len;
                double wr = cos(a), wi = sin(a);
                int64_t u = s + t, v = s + t + half;
                double br = re[v] * wr - im[v] * wi;
                double bi = re[v] * wi + im[v] * wr;
                re[v] = re[u] - br;
                im[v] = im[u] - bi;
                re[u] = re[u] + br;
                im[u] = im[u] + bi;
            }
        }
    }
    return 0;
}

/* ---- pre-filter ---------------------------------------------------------- */

/* PFB output of spectrum j for every polarisation, from double samples
 * xs[T][n_pol][2].  y[n_pol][N][2].  direct != 0: y_j = frame j (no filter;
 * P is then ignored).  The caller guarantees (j+P)*N <= T. */
void orc_pfb_f64(const double *xs, int32_t n_pol, int64_t N, int32_t P,
                 const double *h, int32_t direct, int64_t j, double *y)
{
    for (int32_t pol = 0; pol < n_pol; ++pol) {
        for (int64_t n = 0; n < N; ++n) {
            double ar = 0.0, ai = 0.0;
            if (direct) {
                int64_t t = j * N + n;
                ar = xs[(t * n_pol + pol) * 2 + 0];
                ai = xs[(t * n_pol + pol) * 2 + 1];
            } else {
                for (int32_t p = 0; p < P; ++p) {
                    int64_t t = (j + p) * N + n;
                    double c = h[(int64_t)p * N + n];
                    ar += c * xs[(t * n_pol + pol) * 2 + 0];
                    ai += c * xs[(t * n_pol + pol) * 2 + 1];
                }
            }
            y[((int64_t)pol * N + n) * 2 + 0] = ar;
            y[((int64_t)pol * N + n) * 2 + 1] = ai;
        }
    }
}

/* Same, from int8 samples x[T][n_pol][2] (unpacked first). */
void orc_pfb(const int8_t *x, int32_t n_pol, int64_t N, int32_t P,
             const double *h, int32_t direct, int64_t j, double *y)
{
    int64_t frames = direct ? 1 : P;
    int64_t cnt = frames * N * n_pol * 2;
    double *xs = (double *)malloc((size_t)cnt * sizeof(double));
    orc_unpack(x + j * N * n_pol * 2, cnt, xs);
    /* xs now holds frames j .. j+frames-1; index them from 0 */
    orc_pfb_f64(xs, n_pol, N, P, h, direct, 0, y);
    free(xs);
}

/* ---- products ------------------------------------------------------------ */

/* Products of one spectrum.  X[n_pol][N][2] -> prod[n_prod][N] with
 * n_prod = 1 (|X|^2) for one polarisation, 4 (|X|^2, |Y|^2, Re XY*, Im XY*)
 * for two. */
void orc_products(const double *X, int32_t n_pol, int64_t N, double *prod)
{
    for (int64_t k = 0; k < N; ++k) {
        double xr = X[2 * k], xi = X[2 * k + 1];
        prod[k] = xr * xr + xi * xi;
        if (n_pol == 2) {
            double yr = X[(N + k) * 2], yi = X[(N + k) * 2 + 1];
            prod[N + k] = yr * yr + yi * yi;
            prod[2 * N + k] = xr * yr + xi * yi;
            prod[3 * N + k] = xi * yr - xr * yi;
        }
    }
}

/* One spectrum's products from the int8 stream: pre-filter, FFT, products. */
static void orc_one_spectrum(const int8_t *x, int32_t n_pol, int64_t N, int32_t P,
                             const double *h, int32_t direct, int64_t j,
                             double *work /* 8*N */, double *prod)
{
    double *y = work;                 /* [n_pol][N][2] */
    double *re = work + 2 * N * 2;    /* N */
    double *im = re + N;              /* N */
    orc_pfb(x, n_pol, N, P, h, direct, j, y);
    double *spec = (double *)malloc((size_t)n_pol * N * 2 * sizeof(double));
    for (int32_t pol = 0; pol < n_pol; ++pol) {
        for (int64_t n = 0; n < N; ++n) {
            re[n] = y[((int64_t)pol * N + n) * 2];
            im[n] = y[((int64_t)pol * N + n) * 2 + 1];
        }
        orc_fft(re, im, N);
        for (int64_t k = 0; k < N; ++k) {
            spec[((int64_t)pol * N + k) * 2] = re[k];
            spec[((int64_t)pol * N + k) * 2 + 1] = im[k];
        }
    }
    orc_products(spec, n_pol, N, prod);
    free(spec);
}

/* Integrated products over spectra [j0, j1):
 *   out[q][k] = sum_{j=j0}^{j1-1} prod_q(j, k),
 * summed sequentially in j.  Spectra are computed in parallel batches
 * (independent work), then added in order, so the sum order is the plain
 * sequential one.  Returns 0, or -1 on a bad argument. */
int orc_integrate(const int8_t *x, int64_t T, int32_t n_pol, int64_t N, int32_t P,
                  const double *h, int32_t direct, int64_t j0, int64_t j1,
                  double *out, int32_t n_threads)
{
    if (!orc_is_pow2(N) || (n_pol != 1 && n_pol != 2) || j0 < 0 || j1 < j0)
        return -1;
    int64_t frames = direct ? 1 : P;
    if ((j1 - 1 + frames) * N > T && j1 > j0)
        return -1;
    const int32_t n_prod = n_pol == 2 ? 4 : 1;
    memset(out, 0, (size_t)n_prod * N * sizeof(double));
#ifdef _OPENMP
    if (n_threads < 1)
        n_threads = omp_get_max_threads();
#else
    n_threads = 1;
#endif
    const int64_t batch = 64;
    double *prods = (double *)malloc((size_t)batch * n_prod * N * sizeof(double));
    for (int64_t b0 = j0; b0 < j1; b0 += batch) {
        int64_t nb = j1 - b0 < batch ? j1 - b0 : batch;
#ifdef _OPENMP
#pragma omp parallel for num_threads(n_threads) schedule(dynamic, 1)
#endif
        for (int64_t i = 0; i < nb; ++i) {
            double *work = (double *)malloc((size_t)(4 * N + 4 * N) * sizeof(double));
            orc_one_spectrum(x, n_pol, N, P, h, direct, b0 + i, work,
                             prods + i * n_prod * N);
            free(work);
        }
        for (int64_t i = 0; i < nb; ++i)
            for (int64_t e = 0; e < n_prod * N; ++e)
                out[e] += prods[i * n_prod * N + e];
    }
    free(prods);
    return 0;
}

/* Number of valid spectra in a stream of T time samples. */
int64_t orc_num_spectra(int64_t T, int64_t N, int32_t P, int32_t direct)
{
    int64_t frames = T / N;
    int64_t need = direct ? 1 : P;
    return frames >= need ? frames - need + 1 : 0;
}
