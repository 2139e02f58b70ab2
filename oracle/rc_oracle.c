/*
 * rc_oracle.c -- plain, slow, double-precision reference ("the oracle") for the
 * Doppler and ionospheric correction of sampled arbitrary waveforms described in
 * Vickers, Mack & Osaretin, "Real-Time Doppler and Ionospheric Distortion
 * Correction Techniques for Arbitrary Waveforms Utilizing GPU Compute"
 * (arXiv 2508.04951).
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links, includes or calls
 * this file.  Only the tests, the package smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or constant generator
 * with the GPU path.
 *
 * Every routine writes the plain definition out in float64, in the order the
 * paper states it:
 *   alpha         Eq (1)-(2): alpha = (1 + v_r/c) / (1 - v_r/c), v_r > 0 approaching
 *   resampling    Eq (2) and Eq (17): y[m] = S(alpha * m) by a windowed
 *                 Whittaker-Shannon (sinc) sum (Sec. III-B, App. C)
 *   iono delay    Eq (3) / App. A: tau(f) = K2/(c f^2), K2 = e^2 E / (8 pi^2 m_e eps0)
 *   iono operator Eq (15) (distort, +) and Eq (16) (correct, -), discretised as an
 *                 N-point DFT, per-bin phase exp(-/+ 4 pi i K2 / (c f_k)), inverse DFT
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - time origin: output m samples the input at t = alpha * m (in input samples);
 *   - x[n] = 0 outside [0, n_in);
 *   - window: sum over the 2H inputs n = floor(t)-H+1 .. floor(t)+H with a Kaiser
 *     taper K((t-n)/H); "rect" drops the taper; "paper mode" uses the 2H+1 inputs
 *     centred on the nearest input sample (App. C, Fig. 10) with no taper;
 *     half_width 0 means the full (unwindowed) sum over every input;
 *   - an output at an exact integer t is the input sample itself (sinc(0) = 1,
 *     sinc(k) = 0 for every other integer k);
 *   - f_k = carrier + fs * fftfreq(N)[k] (numpy convention, bin N/2 negative);
 *     at f_k == 0 the response is 1;
 *   - the phase 4 pi K2 / (c f_k) is a function of the double inputs (fs, carrier,
 *     E) and of the CODATA constants as decimal numbers.  With a carrier below
 *     fs/2 it reaches ~1e12 rad, where a float64 quotient is already uncertain by
 *     ~1e-4 rad, so the phase alone is evaluated in long double (64-bit
 *     significand) and reduced by cosl/sinl;
 *   - forward DFT unnormalised, inverse scaled by 1/N;
 *   - batch: Doppler first, then the ionosphere on the resampled samples.
 *
 * Complex arrays are interleaved (re, im) pairs of doubles.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Exact SI value of the speed of light. */
#define RCO_C 299792458.0
/* CODATA 2022 recommended values (elementary charge exact in the 2019 SI). */
#define RCO_E_CHARGE 1.602176634e-19
#define RCO_M_E 9.1093837139e-31
#define RCO_EPS0 8.8541878188e-12
#define RCO_PI 3.14159265358979323846
/* The same constants as long double literals, for the dispersive phase. */
#define RCO_CL 299792458.0L
#define RCO_E_CHARGEL 1.602176634e-19L
#define RCO_M_EL 9.1093837139e-31L
#define RCO_EPS0L 8.8541878188e-12L
#define RCO_PIL 3.141592653589793238462643383279502884L

enum { RCO_WIN_KAISER = 0, RCO_WIN_RECT = 1, RCO_WIN_PAPER = 2 };
enum { RCO_CORRECT = 0, RCO_DISTORT = 1 };

int rco_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Eq (1): alpha = (1 + v_r/c)/(1 - v_r/c).  NaN unless |v_r| < c. */
double rco_alpha_from_vr(double v_r)
{
    if (!(fabs(v_r) < RCO_C))
        return NAN;
    return (1.0 + v_r / RCO_C) / (1.0 - v_r / RCO_C);
}

/* Eq (3) / App. A: K2 / E = e^2 / (8 pi^2 m_e eps0), in m^3 s^-2. */
double rco_k2_per_tec(void)
{
    return RCO_E_CHARGE * RCO_E_CHARGE / (8.0 * RCO_PI * RCO_PI * RCO_M_E * RCO_EPS0);
}

/* Modified Bessel function of the first kind, order 0, by its power series
 * I0(z) = sum_k ((z/2)^k / k!)^2, summed until a term drops below 1e-17 of the sum. */
double rco_bessel_i0(double z)
{
    double q = 0.25 * z * z, term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < 1e-17 * sum)
            break;
    }
    return sum;
}

/* Kaiser taper on [-1, 1]: I0(beta sqrt(1 - x^2)) / I0(beta); 0 outside. */
double rco_kaiser(double x, double beta)
{
    if (!(fabs(x) <= 1.0))
        return 0.0;
    return rco_bessel_i0(beta * sqrt(1.0 - x * x)) / rco_bessel_i0(beta);
}

/* Normalised sinc: sin(pi u)/(pi u), 1 at u = 0. */
double rco_sinc(double u)
{
    if (u == 0.0)
        return 1.0;
    return sin(RCO_PI * u) / (RCO_PI * u);
}

/* One output of the windowed Whittaker-Shannon sum, Eq (17), at t = alpha*m. */
static void doppler_one(const double *x, int64_t n_in, double t, int half_width, int window,
                        double beta, double *out)
{
    double re = 0.0, im = 0.0;
    double f = floor(t);
    if (t == f) { /* exact sample instant: sinc(0) = 1, sinc(k) = 0 */
        if (f >= 0.0 && f < (double)n_in) {
            int64_t k = (int64_t)f;
            re = x[2 * k];
            im = x[2 * k + 1];
        }
        out[0] = re;
        out[1] = im;
        return;
    }
    int64_t lo, hi; /* inclusive input range of the window */
    if (half_width == 0) {
        lo = 0;
        hi = n_in - 1;
    } else if (window == RCO_WIN_PAPER) {
        int64_t c = (int64_t)floor(t + 0.5); /* nearest input sample */
        lo = c - half_width;
        hi = c + half_width;
    } else {
        lo = (int64_t)f - half_width + 1;
        hi = (int64_t)f + half_width;
    }
    if (lo < 0)
        lo = 0;
    if (hi > n_in - 1)
        hi = n_in - 1;
    for (int64_t n = lo; n <= hi; ++n) {
        double u = t - (double)n;
        double w = rco_sinc(u);
        if (half_width != 0 && window == RCO_WIN_KAISER)
            w *= rco_kaiser(u / (double)half_width, beta);
        re += x[2 * n] * w;
        im += x[2 * n + 1] * w;
    }
    out[0] = re;
    out[1] = im;
}

/* Doppler resampling, Eq (2): y[m] = S(alpha m), m = 0 .. n_out-1. */
int rco_doppler(const double *x, int64_t n_in, double *y, int64_t n_out, double alpha,
                int half_width, int window, double beta)
{
    if (!x || !y || n_in <= 0 || n_out < 0 || !(alpha > 0.0) || !isfinite(alpha) ||
        half_width < 0 || !(beta >= 0.0))
        return 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < n_out; ++m)
        doppler_one(x, n_in, alpha * (double)m, half_width, window, beta, y + 2 * m);
    return 0;
}

/* The same sum at selected output indices only: y[i] = S(alpha * idx[i]). */
int rco_doppler_at(const double *x, int64_t n_in, const int64_t *idx, int64_t count, double *y,
                   double alpha, int half_width, int window, double beta)
{
    if (!x || !y || !idx || n_in <= 0 || count < 0 || !(alpha > 0.0) || half_width < 0)
        return 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < count; ++i)
        doppler_one(x, n_in, alpha * (double)idx[i], half_width, window, beta, y + 2 * i);
    return 0;
}

/* Naive DFT: X[k] = sum_n x[n] exp(sign * 2 pi i ((k n) mod N) / N).
 * The product k*n is reduced modulo N in integers so every angle is exact. */
int rco_dft(const double *x, double *X, int64_t n, int sign)
{
    if (!x || !X || n <= 0)
        return 1;
    double *cs = malloc(sizeof(double) * 2 * (size_t)n);
    if (!cs)
        return 2;
    for (int64_t j = 0; j < n; ++j) {
        double a = 2.0 * RCO_PI * (double)j / (double)n;
        cs[2 * j] = cos(a);
        cs[2 * j + 1] = (double)sign * sin(a);
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double re = 0.0, im = 0.0;
        for (int64_t m = 0; m < n; ++m) {
            int64_t j = (int64_t)(((__int128)k * m) % n);
            double c = cs[2 * j], s = cs[2 * j + 1];
            re += x[2 * m] * c - x[2 * m + 1] * s;
            im += x[2 * m] * s + x[2 * m + 1] * c;
        }
        X[2 * k] = re;
        X[2 * k + 1] = im;
    }
    free(cs);
    return 0;
}

/* Radix-2 decimation in time.  X[0..n) = DFT of x[0], x[xs], .., x[(n-1) xs]
 * (strides in complex elements), with twiddles w[j*ws] = exp(sign 2 pi i j ws / N). */
static void fft2_rec(const double *x, int64_t xs, double *X, int64_t n, const double *w, int64_t ws)
{
    if (n == 1) {
        X[0] = x[0];
        X[1] = x[1];
        return;
    }
    int64_t h = n / 2;
    fft2_rec(x, 2 * xs, X, h, w, 2 * ws);              /* even samples -> X[0..h) */
    fft2_rec(x + 2 * xs, 2 * xs, X + 2 * h, h, w, 2 * ws); /* odd samples -> X[h..n) */
    for (int64_t k = 0; k < h; ++k) {
        double er = X[2 * k], ei = X[2 * k + 1];
        double orr = X[2 * (k + h)], oi = X[2 * (k + h) + 1];
        double wr = w[2 * k * ws], wi = w[2 * k * ws + 1];
        double tr = wr * orr - wi * oi, ti = wr * oi + wi * orr;
        X[2 * k] = er + tr;
        X[2 * k + 1] = ei + ti;
        X[2 * (k + h)] = er - tr;
        X[2 * (k + h) + 1] = ei - ti;
    }
}

static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

static int fft_pow2(const double *x, double *X, int64_t n, int sign)
{
    double *w = malloc(sizeof(double) * 2 * (size_t)(n > 1 ? n / 2 : 1));
    if (!w)
        return 2;
    for (int64_t j = 0; j < n / 2; ++j) {
        double a = 2.0 * RCO_PI * (double)j / (double)n;
        w[2 * j] = cos(a);
        w[2 * j + 1] = (double)sign * sin(a);
    }
    fft2_rec(x, 1, X, n, w, 1);
    free(w);
    return 0;
}

/* DFT of any length.  Powers of two use radix 2; other lengths use Bluestein's
 * chirp-z identity nk = (n^2 + k^2 - (k-n)^2)/2 with a power-of-two circular
 * convolution of length M >= 2N-1.  n^2 is reduced modulo 2N in integers. */
int rco_fft(const double *x, double *X, int64_t n, int sign)
{
    if (!x || !X || n <= 0 || (sign != 1 && sign != -1))
        return 1;
    if (is_pow2(n))
        return fft_pow2(x, X, n, sign);
    int64_t M = 1;
    while (M < 2 * n - 1)
        M <<= 1;
    double *c = malloc(sizeof(double) * 2 * (size_t)n); /* c[j] = exp(sign pi i j^2 / N) */
    double *a = calloc(2 * (size_t)M, sizeof(double));
    double *b = calloc(2 * (size_t)M, sizeof(double));
    double *A = malloc(sizeof(double) * 2 * (size_t)M);
    double *B = malloc(sizeof(double) * 2 * (size_t)M);
    if (!c || !a || !b || !A || !B) {
        free(c); free(a); free(b); free(A); free(B);
        return 2;
    }
    for (int64_t j = 0; j < n; ++j) {
        int64_t q = (int64_t)(((__int128)j * j) % (2 * n));
        double ang = RCO_PI * (double)q / (double)n;
        c[2 * j] = cos(ang);
        c[2 * j + 1] = (double)sign * sin(ang);
    }
    for (int64_t j = 0; j < n; ++j) { /* a = x * c */
        a[2 * j] = x[2 * j] * c[2 * j] - x[2 * j + 1] * c[2 * j + 1];
        a[2 * j + 1] = x[2 * j] * c[2 * j + 1] + x[2 * j + 1] * c[2 * j];
    }
    for (int64_t j = 0; j < n; ++j) { /* b = conj(c), wrapped for negative lags */
        b[2 * j] = c[2 * j];
        b[2 * j + 1] = -c[2 * j + 1];
        if (j > 0) {
            b[2 * (M - j)] = c[2 * j];
            b[2 * (M - j) + 1] = -c[2 * j + 1];
        }
    }
    fft_pow2(a, A, M, -1);
    fft_pow2(b, B, M, -1);
    for (int64_t j = 0; j < M; ++j) {
        double ar = A[2 * j], ai = A[2 * j + 1], br = B[2 * j], bi = B[2 * j + 1];
        A[2 * j] = ar * br - ai * bi;
        A[2 * j + 1] = ar * bi + ai * br;
    }
    fft_pow2(A, a, M, +1); /* a = M * (a (*) b) */
    for (int64_t k = 0; k < n; ++k) {
        double vr = a[2 * k] / (double)M, vi = a[2 * k + 1] / (double)M;
        X[2 * k] = vr * c[2 * k] - vi * c[2 * k + 1];
        X[2 * k + 1] = vr * c[2 * k + 1] + vi * c[2 * k];
    }
    free(c); free(a); free(b); free(A); free(B);
    return 0;
}

/* Physical (RF) frequency of DFT bin k: carrier + fs * fftfreq(N)[k]. */
double rco_bin_frequency(int64_t k, int64_t n, double fs, double carrier)
{
    int64_t kk = (k < (n + 1) / 2) ? k : k - n;
    return carrier + fs * (double)kk / (double)n;
}

/* Per-bin response of Eq (15) (distort, +) or Eq (16) (correct, -):
 * H_k = exp(+/- i 4 pi K2 / (c f_k)), H_k = 1 where f_k == 0. */
int rco_iono_response(int64_t n, double fs, double carrier, double tec, int direction, double *H)
{
    if (!H || n <= 0 || !(fs > 0.0) || !isfinite(carrier) || !isfinite(tec))
        return 1;
    /* K2 = e^2 E / (8 pi^2 m_e eps0) and f_k in long double: see the header note. */
    long double k2 = RCO_E_CHARGEL * RCO_E_CHARGEL / (8.0L * RCO_PIL * RCO_PIL * RCO_M_EL * RCO_EPS0L)
                     * (long double)tec;
    long double s = (direction == RCO_DISTORT) ? 1.0L : -1.0L;
    for (int64_t k = 0; k < n; ++k) {
        int64_t kk = (k < (n + 1) / 2) ? k : k - n;
        long double f = (long double)carrier + (long double)fs * (long double)kk / (long double)n;
        if (f == 0.0L) {
            H[2 * k] = 1.0;
            H[2 * k + 1] = 0.0;
            continue;
        }
        long double phi = s * 4.0L * RCO_PIL * k2 / (RCO_CL * f);
        H[2 * k] = (double)cosl(phi);
        H[2 * k + 1] = (double)sinl(phi);
    }
    return 0;
}

/* Eq (15)/(16): y = IDFT( DFT(x) * H ).  naive != 0 uses the O(N^2) DFT. */
int rco_ionosphere(const double *x, double *y, int64_t n, double fs, double carrier, double tec,
                   int direction, int naive)
{
    if (!x || !y || n <= 0)
        return 1;
    double *X = malloc(sizeof(double) * 2 * (size_t)n);
    double *H = malloc(sizeof(double) * 2 * (size_t)n);
    if (!X || !H) {
        free(X); free(H);
        return 2;
    }
    int rc = naive ? rco_dft(x, X, n, -1) : rco_fft(x, X, n, -1);
    if (!rc)
        rc = rco_iono_response(n, fs, carrier, tec, direction, H);
    if (!rc) {
        for (int64_t k = 0; k < n; ++k) {
            double xr = X[2 * k], xi = X[2 * k + 1], hr = H[2 * k], hi = H[2 * k + 1];
            X[2 * k] = xr * hr - xi * hi;
            X[2 * k + 1] = xr * hi + xi * hr;
        }
        rc = naive ? rco_dft(X, y, n, +1) : rco_fft(X, y, n, +1);
    }
    if (!rc)
        for (int64_t j = 0; j < 2 * n; ++j)
            y[j] /= (double)n;
    free(X);
    free(H);
    return rc;
}

/* Pulse compression with the ionospheric operator in the same frequency-domain pass (Sec. II-B
 * bundles Eq (15)/(16) with pulse compression; Sec. II-D times it).  The matched filter is read
 * as the circular cross-correlation with the replica r zero-padded to n (n_rep <= n):
 *     y = IDFT( DFT(x) * conj(DFT(r)) * H ),  i.e.  y[m] = sum_j x_c[(j + m) mod n] conj(r[j])
 * where x_c is the ionosphere-corrected (or distorted) x.  naive != 0 uses the O(N^2) DFT. */
int rco_compress(const double *x, const double *r, int64_t n_rep, double *y, int64_t n, double fs,
                 double carrier, double tec, int direction, int naive)
{
    if (!x || !r || !y || n <= 0 || n_rep <= 0 || n_rep > n)
        return 1;
    double *X = malloc(sizeof(double) * 2 * (size_t)n);
    double *R = malloc(sizeof(double) * 2 * (size_t)n);
    double *rp = calloc(2 * (size_t)n, sizeof(double));
    double *H = malloc(sizeof(double) * 2 * (size_t)n);
    if (!X || !R || !rp || !H) {
        free(X); free(R); free(rp); free(H);
        return 2;
    }
    for (int64_t j = 0; j < 2 * n_rep; ++j)
        rp[j] = r[j];
    int rc = naive ? rco_dft(x, X, n, -1) : rco_fft(x, X, n, -1);
    if (!rc)
        rc = naive ? rco_dft(rp, R, n, -1) : rco_fft(rp, R, n, -1);
    if (!rc)
        rc = rco_iono_response(n, fs, carrier, tec, direction, H);
    if (!rc) {
        for (int64_t k = 0; k < n; ++k) {
            /* X * conj(R) */
            const double xr = X[2 * k], xi = X[2 * k + 1], rr = R[2 * k], ri = R[2 * k + 1];
            const double pr = xr * rr + xi * ri, pi = xi * rr - xr * ri;
            const double hr = H[2 * k], hi = H[2 * k + 1];
            X[2 * k] = pr * hr - pi * hi;
            X[2 * k + 1] = pr * hi + pi * hr;
        }
        rc = naive ? rco_dft(X, y, n, +1) : rco_fft(X, y, n, +1);
    }
    if (!rc)
        for (int64_t j = 0; j < 2 * n; ++j)
            y[j] /= (double)n;
    free(X); free(R); free(rp); free(H);
    return rc;
}

/* One pulse of a batch: Doppler resampling (if do_doppler), then the ionospheric
 * operator on the resampled samples (if do_iono).  y holds n_out samples. */
int rco_pulse(const double *x, int64_t n_in, double *y, int64_t n_out, double fs, double alpha,
              double tec, double carrier, int do_doppler, int do_iono, int direction,
              int half_width, int window, double beta, int naive)
{
    if (!x || !y || n_in <= 0 || n_out <= 0)
        return 1;
    double *r = malloc(sizeof(double) * 2 * (size_t)n_out);
    if (!r)
        return 2;
    int rc = 0;
    if (do_doppler) {
        rc = rco_doppler(x, n_in, r, n_out, alpha, half_width, window, beta);
    } else {
        for (int64_t j = 0; j < n_out; ++j) {
            r[2 * j] = j < n_in ? x[2 * j] : 0.0;
            r[2 * j + 1] = j < n_in ? x[2 * j + 1] : 0.0;
        }
    }
    if (!rc) {
        if (do_iono)
            rc = rco_ionosphere(r, y, n_out, fs, carrier, tec, direction, naive);
        else
            memcpy(y, r, sizeof(double) * 2 * (size_t)n_out);
    }
    free(r);
    return rc;
}

/* ---------------------------------------------------------------------------------------
 * The paper's other resampling methods (Sec. I list of methods, Table I, Sec. III-A, App. C),
 * kept as references for the baseline engines.
 * --------------------------------------------------------------------------------------- */

/* App. C, Alg. 2: the paper's window (N_w = 2h + 1 inputs centred on the nearest input
 * sample, untapered) with sinc taken from a table of its positive half.  The table holds
 * lut_size values sinc(i dx), i = 0 .. lut_size-1, spanning the window's largest distance
 * u_max = h + 1/2, so dx = u_max / (lut_size - 1); a tap at distance u = |t - n| takes entry
 * floor(u / dx + 1/2) (nearest), computed as floor(u * inv_dx + 0.5) with inv_dx = 1 / dx.
 * No exact-instant special case: the table sum is the method. */
int rco_doppler_lut(const double *x, int64_t n_in, double *y, int64_t n_out, double alpha,
                    int h, int lut_size)
{
    if (!x || !y || n_in <= 0 || n_out < 0 || !(alpha > 0.0) || !isfinite(alpha) || h < 0 ||
        lut_size < 2)
        return 1;
    double *lut = malloc(sizeof(double) * (size_t)lut_size);
    if (!lut)
        return 2;
    const double u_max = (double)h + 0.5;
    const double dx = u_max / (double)(lut_size - 1);
    const double inv_dx = (double)(lut_size - 1) / u_max;
    for (int i = 0; i < lut_size; ++i)
        lut[i] = rco_sinc((double)i * dx);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < n_out; ++m) {
        double t = alpha * (double)m;
        int64_t c = (int64_t)floor(t + 0.5);
        double re = 0.0, im = 0.0;
        for (int64_t n = c - h; n <= c + h; ++n) {
            if (n < 0 || n >= n_in)
                continue;
            double u = fabs(t - (double)n);
            int64_t i = (int64_t)floor(u * inv_dx + 0.5);
            double w = (i < lut_size) ? lut[i] : 0.0;
            re += x[2 * n] * w;
            im += x[2 * n + 1] * w;
        }
        y[2 * m] = re;
        y[2 * m + 1] = im;
    }
    free(lut);
    return 0;
}

/* Linear interpolation (Sec. I, Table I): y[m] = (1 - mu) x[f] + mu x[f + 1] with
 * t = alpha m, f = floor(t), mu = t - f; x[n] = 0 outside [0, n_in). */
int rco_doppler_linear(const double *x, int64_t n_in, double *y, int64_t n_out, double alpha)
{
    if (!x || !y || n_in <= 0 || n_out < 0 || !(alpha > 0.0) || !isfinite(alpha))
        return 1;
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < n_out; ++m) {
        double t = alpha * (double)m;
        double f = floor(t), mu = t - f;
        int64_t k = (int64_t)f;
        double a_re = (k >= 0 && k < n_in) ? x[2 * k] : 0.0;
        double a_im = (k >= 0 && k < n_in) ? x[2 * k + 1] : 0.0;
        double b_re = (k + 1 >= 0 && k + 1 < n_in) ? x[2 * (k + 1)] : 0.0;
        double b_im = (k + 1 >= 0 && k + 1 < n_in) ? x[2 * (k + 1) + 1] : 0.0;
        y[2 * m] = (1.0 - mu) * a_re + mu * b_re;
        y[2 * m + 1] = (1.0 - mu) * a_im + mu * b_im;
    }
    return 0;
}

/* Frequency conversion (Sec. I, Table I): the dilation of Eq (2) replaced by the frequency
 * shift it causes at one reference frequency f_ref (Hz, on the samples' own frequency axis):
 * y[m] = x[m] exp(2 pi i (alpha - 1) f_ref m / fs).  Exact for a tone at f_ref only. */
int rco_doppler_tone(const double *x, int64_t n, double *y, double fs, double alpha, double f_ref)
{
    if (!x || !y || n < 0 || !(fs > 0.0) || !(alpha > 0.0) || !isfinite(alpha) || !isfinite(f_ref))
        return 1;
    const double nu = (alpha - 1.0) * f_ref / fs; /* cycles per sample */
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < n; ++m) {
        double cyc = nu * (double)m;
        cyc -= floor(cyc); /* whole cycles dropped exactly */
        double c = cos(2.0 * RCO_PI * cyc), s = sin(2.0 * RCO_PI * cyc);
        double re = x[2 * m], im = x[2 * m + 1]; /* y may be x */
        y[2 * m] = re * c - im * s;
        y[2 * m + 1] = re * s + im * c;
    }
    return 0;
}

/* FFT P/Q resampling (Sec. I, Sec. III-A): the DFT of the n_in samples has bins removed or
 * zero bins added to reach n_out bins, then the inverse DFT of length n_out is taken:
 *   y[m] = (1/n_in) sum_j Y_j exp(2 pi i j m / n_out),
 * i.e. the samples' trigonometric interpolant, limited to the band both lengths hold, at
 * t = m n_in / n_out input samples.  With K = min(n_in, n_out), signed bins |k| < K/2 are
 * copied; for even K the bin k = K/2 is, when removing bins, the sum of the input bins +K/2
 * and -K/2 (both alias onto the output's Nyquist bin), and, when adding bins, the input
 * Nyquist bin split in halves between output bins +K/2 and -K/2. */
int rco_resample_fft(const double *x, int64_t n_in, double *y, int64_t n_out)
{
    if (!x || !y || n_in <= 0 || n_out <= 0)
        return 1;
    double *X = malloc(sizeof(double) * 2 * (size_t)n_in);
    double *Y = calloc(2 * (size_t)n_out, sizeof(double));
    if (!X || !Y) {
        free(X); free(Y);
        return 2;
    }
    int rc = rco_fft(x, X, n_in, -1);
    if (!rc) {
        int64_t K = n_in < n_out ? n_in : n_out;
        int64_t half = (K - 1) / 2; /* bins with |k| <= half are copied */
        for (int64_t k = -half; k <= half; ++k) {
            int64_t si = (k + n_in) % n_in, di = (k + n_out) % n_out;
            Y[2 * di] = X[2 * si];
            Y[2 * di + 1] = X[2 * si + 1];
        }
        if (K % 2 == 0) {
            int64_t k = K / 2;
            if (n_out < n_in) { /* output Nyquist bin: input bins +K/2 and -K/2 */
                int64_t a = k % n_in, b = (n_in - k) % n_in;
                Y[2 * k] = X[2 * a] + X[2 * b];
                Y[2 * k + 1] = X[2 * a + 1] + X[2 * b + 1];
            } else if (n_out > n_in) { /* input Nyquist bin split between +K/2 and -K/2 */
                int64_t d1 = k, d2 = n_out - k;
                Y[2 * d1] = 0.5 * X[2 * k];
                Y[2 * d1 + 1] = 0.5 * X[2 * k + 1];
                Y[2 * d2] = 0.5 * X[2 * k];
                Y[2 * d2 + 1] = 0.5 * X[2 * k + 1];
            } else { /* same length: the bin itself */
                Y[2 * k] = X[2 * k];
                Y[2 * k + 1] = X[2 * k + 1];
            }
        }
        rc = rco_fft(Y, y, n_out, +1);
        if (!rc)
            for (int64_t j = 0; j < 2 * n_out; ++j)
                y[j] /= (double)n_in;
    }
    free(X); free(Y);
    return rc;
}

/* The P/Q length for a dilation alpha (Sec. III-A): the n_in / alpha samples the dilated
 * record spans, rounded so that an even number of samples is removed or added,
 * n_i = n_in - 2 round((n_in - n_in / alpha) / 2) (half-way cases away from zero).
 * Then alpha_eff = n_in / n_i is the dilation P/Q performs exactly. */
int64_t rco_pq_length(int64_t n_in, double alpha)
{
    double d = ((double)n_in - (double)n_in / alpha) / 2.0;
    return n_in - 2 * (int64_t)llround(d);
}

/* Doppler correction by FFT P/Q resampling (Sec. III-A): y[m] = P/Q resample of x to
 * n_i = rco_pq_length(n_in, alpha) samples for m < min(n_i, n_out), 0 beyond (past the end of
 * the dilated record).  With tone != 0 (P/Q "with frequency conversion"), the remaining
 * dilation alpha / alpha_eff is then applied as frequency conversion at the reference
 * frequency, which P/Q has moved to alpha_eff f_ref. */
int rco_doppler_pq(const double *x, int64_t n_in, double *y, int64_t n_out, double fs, double alpha,
                   double f_ref, int tone)
{
    if (!x || !y || n_in <= 0 || n_out < 0 || !(alpha > 0.0) || !isfinite(alpha) || !(fs > 0.0))
        return 1;
    int64_t ni = rco_pq_length(n_in, alpha);
    if (ni <= 0)
        return 1;
    double *r = malloc(sizeof(double) * 2 * (size_t)ni);
    if (!r)
        return 2;
    int rc = rco_resample_fft(x, n_in, r, ni);
    if (!rc && tone) {
        double a_eff = (double)n_in / (double)ni;
        rc = rco_doppler_tone(r, ni, r, fs, alpha / a_eff, a_eff * f_ref);
    }
    if (!rc)
        for (int64_t m = 0; m < n_out; ++m) {
            y[2 * m] = m < ni ? r[2 * m] : 0.0;
            y[2 * m + 1] = m < ni ? r[2 * m + 1] : 0.0;
        }
    free(r);
    return rc;
}
