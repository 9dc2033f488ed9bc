/*
 * CPU FP64 oracle for the NFFT and its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file: only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code with the HIP library.
 *
 * Everything here is plain, serial (except the direct NDFT, which uses OpenMP
 * over independent output entries) and computed in double precision.
 *
 * Sources (arXiv:1810.09891, "NFFT Interface for Julia"):
 *   - Sec. 1 eq. (1.2) / (1.3) and Sec. 2 eq. (2.1)-(2.2): the trigonometric
 *     polynomial, the index set I_N and the adjoint sum (direct NDFT below).
 *   - Sec. 2 Algorithm 2.1 (NFFT: deconvolve, FFT, interpolate) and
 *     Algorithm 2.2 (adjoint NFFT: spread, inverse FFT, deconvolve).
 *   - Sec. 2 eq. (2.9): the deconvolution by the Fourier coefficients of the
 *     periodised window; eq. (2.13): the stencil index set.
 *   - Sec. 2 eq. (2.15) / (2.16): the error measures E_2 and E_inf.
 *   - Sec. 4: the Kaiser-Bessel window (named, formula not printed).
 *   - Sec. 1: the NNFFT (nonequispaced in both domains), named only; its direct sums
 *     (or_nndft_*) are the definition with real frequencies in eq. (1.2) / (1.3).
 *
 * Readings where the paper is silent or garbled (each also listed in the
 * design notes):
 *   R1 Kaiser-Bessel pair in the grid variable z = n*x - l:
 *        phi(z)   = sinh(b*sqrt(m^2-z^2)) / (pi*sqrt(m^2-z^2))     |z| < m
 *                 = sin (b*sqrt(z^2-m^2)) / (pi*sqrt(z^2-m^2))     |z| > m
 *                 = b/pi                                           |z| = m
 *        phihat(k) = (1/n) * I0(m*sqrt(b^2 - (2*pi*k/n)^2)),   b = pi*(2 - 1/sigma),
 *      sigma = n/N per dimension, tensor product over dimensions.
 *   R2 The stencil of node x is l = u-m, ..., u+m+1 with u = floor(n*x) in
 *      double precision (2m+2 points per dimension), evaluated with the
 *      formula of R1 at every point (no zeroing outside |z| <= m).
 *   R3 Grid indices are taken modulo n (true modulo for negatives).
 *   R4 Forward FFT sign -, adjoint FFT sign +, both unnormalised, the factor
 *      1/|I_n| is part of the deconvolution.
 *   R5 Multi-dimensional arrays are row-major (last index fastest); the
 *      coefficient array is centred: position i_t holds k_t = i_t - N_t/2.
 *   R6 Nodes are accepted anywhere on the real line and treated periodically.
 */
#include <complex.h>
#include <omp.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846264338327950288

typedef double complex cplx;

/* ------------------------------------------------------------------------- */
/* Modified Bessel function I0 from its power series                          */
/*   I0(x) = sum_{i>=0} ((x/2)^i / i!)^2.  All terms are positive, so the sum  */
/*   is accurate to rounding; stop when a term no longer changes the sum.     */
/* ------------------------------------------------------------------------- */
double or_bessel_i0(double x)
{
    double half = 0.5 * x;
    double term = 1.0; /* ((x/2)^i / i!) for the current i */
    double sum = 1.0;
    for (int i = 1; i < 500; ++i) {
        term *= half / (double)i;
        double t2 = term * term;
        sum += t2;
        if (t2 < 1e-17 * sum)
            break;
    }
    return sum;
}

/* Shape parameter of the Kaiser-Bessel window for oversampling sigma = n/N (R1). */
double or_kb_b(long N, long n)
{
    double sigma = (double)n / (double)N;
    return OR_PI * (2.0 - 1.0 / sigma);
}

/* Kaiser-Bessel window in the grid variable z (R1), textbook form. */
double or_kb_phi(double z, int m, double b)
{
    double a = (double)m * (double)m - z * z;
    if (a > 0.0) {
        double s = sqrt(a);
        return sinh(b * s) / (OR_PI * s);
    }
    if (a < 0.0) {
        double s = sqrt(-a);
        return sin(b * s) / (OR_PI * s);
    }
    return b / OR_PI;
}

/* Derivative d phi / d z of the window above (used only by the gradient checks). */
double or_kb_dphi(double z, int m, double b)
{
    double a = (double)m * (double)m - z * z;
    if (a > 0.0) {
        double s = sqrt(a);
        double bs = b * s;
        if (bs < 1e-3) /* series of (bs cosh bs - sinh bs)/s^3 = b^3/3 (1 + (bs)^2/10 + ...) */
            return -(z / OR_PI) * b * b * b / 3.0 * (1.0 + bs * bs / 10.0);
        return -(z / OR_PI) * (bs * cosh(bs) - sinh(bs)) / (s * s * s);
    }
    if (a < 0.0) {
        double s = sqrt(-a);
        double bs = b * s;
        if (bs < 1e-3) /* (bs cos bs - sin bs)/s^3 = -b^3/3 (1 - (bs)^2/10 + ...) */
            return -(z / OR_PI) * b * b * b / 3.0 * (1.0 - bs * bs / 10.0);
        return (z / OR_PI) * (bs * cos(bs) - sin(bs)) / (s * s * s);
    }
    return -(z / OR_PI) * b * b * b / 3.0;
}

/* Fourier transform of the window at integer frequency k for grid length n (R1). */
double or_kb_phihat(long k, long n, int m, double b)
{
    double w = 2.0 * OR_PI * (double)k / (double)n;
    double a = b * b - w * w;
    if (a < 0.0)
        return 0.0;
    return or_bessel_i0((double)m * sqrt(a)) / (double)n;
}

/* ------------------------------------------------------------------------- */
/* One-dimensional DFT                                                        */
/*   out[l] = sum_k in[k] * exp(sign * 2 pi i k l / n), unnormalised (R4).    */
/* ------------------------------------------------------------------------- */

/* Direct O(n^2) sum; angles reduced exactly through (k*l mod n). */
/* Gaussian window (one of the windows the NFFT library of Sec. 3 can be configured with;
 * its formulas are not printed in the paper -- the standard pair of the NFFT literature):
 * in the grid variable z,
 *   phi(z) = (pi b)^{-1/2} exp(-z^2 / b),   b = 2 sigma m / ((2 sigma - 1) pi),
 *   phihat(k) = (1/n) exp(-b (pi k / n)^2),  sigma = n / N,
 * so that n phihat(k) is the Fourier transform of phi at frequency k/n. */
double or_gauss_b(long N, long n, int m)
{
    const double sigma = (double)n / (double)N;
    return 2.0 * sigma * (double)m / ((2.0 * sigma - 1.0) * 3.14159265358979323846);
}

double or_gauss_phi(double z, double b)
{
    return exp(-z * z / b) / sqrt(3.14159265358979323846 * b);
}

double or_gauss_dphi(double z, double b) { return -2.0 * z / b * or_gauss_phi(z, b); }

double or_gauss_phihat(long k, long n, double b)
{
    const double a = 3.14159265358979323846 * (double)k / (double)n;
    return exp(-b * a * a) / (double)n;
}

/* Cardinal B-spline N_k of order k (degree k - 1, knots 0, 1, ..., k) at x, by the
 * recursion N_q(x) = (x N_{q-1}(x) + (q - x) N_{q-1}(x - 1)) / (q - 1) with N_1 the indicator
 * of [0, 1), run over the k values N_q(t + j), j = 0..q-1, that are nonzero at the
 * fractional part t of x (de Boor's triangle; every term is a nonnegative combination, so
 * there is no cancellation). */
#define OR_MAXK 64
double or_bspline_n(int k, double x)
{
    if (!(x >= 0.0) || x >= (double)k || k < 1 || k > OR_MAXK)
        return 0.0;
    const double fl = floor(x);
    const double t = x - fl;
    const int j = (int)fl;
    double b[OR_MAXK + 1];
    for (int i = 0; i <= k; ++i)
        b[i] = 0.0;
    b[0] = 1.0;
    for (int q = 2; q <= k; ++q) {
        double nb[OR_MAXK + 1];
        for (int i = 0; i < q; ++i) {
            const double cur = i < q - 1 ? b[i] : 0.0;
            const double prev = i > 0 ? b[i - 1] : 0.0;
            nb[i] = ((t + (double)i) * cur + ((double)q - t - (double)i) * prev) / (double)(q - 1);
        }
        for (int i = 0; i < q; ++i)
            b[i] = nb[i];
    }
    return b[j];
}

/* B-spline window (another window the NFFT library of Sec. 3 can be configured with; the
 * standard pair of the NFFT literature): in the grid variable z,
 *   phi(z) = M_2m(z) = N_2m(z + m)  (centred B-spline of order 2m, support [-m, m]),
 *   phihat(k) = (1/n) (sin(pi k / n) / (pi k / n))^(2m). */
double or_bspline_phi(double z, int m) { return or_bspline_n(2 * m, z + (double)m); }
double or_bspline_dphi(double z, int m)
{
    /* d/dx N_k(x) = N_{k-1}(x) - N_{k-1}(x - 1) */
    return or_bspline_n(2 * m - 1, z + (double)m) - or_bspline_n(2 * m - 1, z + (double)m - 1.0);
}
double or_bspline_phihat(long k, long n, int m)
{
    if (k == 0)
        return 1.0 / (double)n;
    const double a = 3.14159265358979323846 * (double)k / (double)n;
    return pow(sin(a) / a, 2.0 * (double)m) / (double)n;
}

/* Sinc window (the fourth configurable window; standard pair): with
 * a = pi (2 - 1/sigma) / (2m), sigma = n / N,
 *   phi(z) = (sin(a z) / (a z))^(2m),
 *   phihat(k) = (1/n) (pi / a) M_2m(pi k / (n a)),
 * the 2m-fold convolution of the box that is the transform of sin(a z)/(a z). */
double or_sinc_a(long N, long n, int m)
{
    const double sigma = (double)n / (double)N;
    return 3.14159265358979323846 * (2.0 - 1.0 / sigma) / (2.0 * (double)m);
}
static double or_sinc1(double x) { return fabs(x) < 1e-8 ? 1.0 - x * x / 6.0 : sin(x) / x; }
double or_sinc_phi(double z, int m, double a) { return pow(or_sinc1(a * z), 2.0 * (double)m); }
/* d/dx sin(x)/x: the series sum_{n>=1} (-1)^n 2n x^(2n-1) / (2n+1)! for |x| < 1 (the
 * closed form (x cos x - sin x) / x^2 loses digits to cancellation there), the closed form
 * beyond. */
static double or_dsinc1(double x)
{
    if (fabs(x) >= 1.0)
        return (x * cos(x) - sin(x)) / (x * x);
    double term = -x / 3.0, sum = 0.0; /* n = 1: -2x/3! */
    for (int n = 1; n < 14; ++n) {
        sum += term;
        /* term_{n+1} / term_n = -x^2 (n+1) / (n (2n+2)(2n+3)) */
        term *= -x * x * (double)(n + 1) / ((double)n * (2.0 * n + 2.0) * (2.0 * n + 3.0));
    }
    return sum;
}
double or_sinc_dphi(double z, int m, double a)
{
    const double x = a * z;
    const double ds = or_dsinc1(x);
    return 2.0 * (double)m * pow(or_sinc1(x), 2.0 * (double)m - 1.0) * ds * a;
}
double or_sinc_phihat(long k, long n, int m, double a)
{
    const double u = 3.14159265358979323846 * (double)k / ((double)n * a);
    return (3.14159265358979323846 / a) * or_bspline_n(2 * m, u + (double)m) / (double)n;
}

/* Window used by the NFFT functions below: 0 Kaiser-Bessel (R1), 1 Gaussian, 2 B-spline,
 * 3 sinc. */
static int or_window = 0;
void or_set_window(int w) { or_window = w; }
int or_get_window(void) { return or_window; }

static double win_b(long N, long n, int m)
{
    switch (or_window) {
    case 1: return or_gauss_b(N, n, m);
    case 2: return 0.0;
    case 3: return or_sinc_a(N, n, m);
    default: return or_kb_b(N, n);
    }
}
static double win_phi(double z, int m, double b)
{
    switch (or_window) {
    case 1: return or_gauss_phi(z, b);
    case 2: return or_bspline_phi(z, m);
    case 3: return or_sinc_phi(z, m, b);
    default: return or_kb_phi(z, m, b);
    }
}
static double win_dphi(double z, int m, double b)
{
    switch (or_window) {
    case 1: return or_gauss_dphi(z, b);
    case 2: return or_bspline_dphi(z, m);
    case 3: return or_sinc_dphi(z, m, b);
    default: return or_kb_dphi(z, m, b);
    }
}
static double win_phihat(long k, long n, int m, double b)
{
    switch (or_window) {
    case 1: return or_gauss_phihat(k, n, b);
    case 2: return or_bspline_phihat(k, n, m);
    case 3: return or_sinc_phihat(k, n, m, b);
    default: return or_kb_phihat(k, n, m, b);
    }
}

void or_dft_naive(const cplx *in, cplx *out, long n, int sign)
{
    for (long l = 0; l < n; ++l) {
        cplx acc = 0.0;
        for (long k = 0; k < n; ++k) {
            long r = (k * l) % n;
            double ang = (double)sign * 2.0 * OR_PI * (double)r / (double)n;
            acc += in[k] * (cos(ang) + I * sin(ang));
        }
        out[l] = acc;
    }
}

static int is_pow2(long n) { return n > 0 && (n & (n - 1)) == 0; }

/* Iterative radix-2 decimation-in-time FFT, in place, n a power of two.
 * Twiddles are evaluated directly with cos/sin of the exact angle each stage. */
static void fft_radix2(cplx *a, long n, int sign)
{
    /* bit-reversal permutation */
    for (long i = 1, j = 0; i < n; ++i) {
        long bit = n >> 1;
        for (; j & bit; bit >>= 1)
            j ^= bit;
        j ^= bit;
        if (i < j) {
            cplx t = a[i];
            a[i] = a[j];
            a[j] = t;
        }
    }
    for (long len = 2; len <= n; len <<= 1) {
        long half = len >> 1;
        for (long k = 0; k < half; ++k) {
            double ang = (double)sign * 2.0 * OR_PI * (double)k / (double)len;
            cplx w = cos(ang) + I * sin(ang);
            for (long i = 0; i < n; i += len) {
                cplx u = a[i + k];
                cplx v = a[i + k + half] * w;
                a[i + k] = u + v;
                a[i + k + half] = u - v;
            }
        }
    }
}

/* 1-D transform of length n: radix-2 when n is a power of two, else the direct sum. */
void or_fft_1d(cplx *a, long n, int sign)
{
    if (is_pow2(n)) {
        fft_radix2(a, n, sign);
    } else {
        cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        or_dft_naive(a, tmp, n, sign);
        memcpy(a, tmp, sizeof(cplx) * (size_t)n);
        free(tmp);
    }
}

/* d-variate unnormalised DFT of a row-major array of shape n[0..d-1], done
 * dimension by dimension (Algorithm 2.1 step 2 / Algorithm 2.2 step 2). */
void or_fft_d(int d, const long *n, cplx *a, int sign)
{
    long total = 1;
    for (int t = 0; t < d; ++t)
        total *= n[t];
    for (int t = 0; t < d; ++t) {
        long len = n[t];
        long inner = 1; /* stride of dimension t */
        for (int q = t + 1; q < d; ++q)
            inner *= n[q];
        long outer = total / (len * inner);
        cplx *line = (cplx *)malloc(sizeof(cplx) * (size_t)len);
        for (long o = 0; o < outer; ++o) {
            for (long i = 0; i < inner; ++i) {
                cplx *base = a + o * len * inner + i;
                for (long k = 0; k < len; ++k)
                    line[k] = base[k * inner];
                or_fft_1d(line, len, sign);
                for (long k = 0; k < len; ++k)
                    base[k * inner] = line[k];
            }
        }
        free(line);
    }
}

/* ------------------------------------------------------------------------- */
/* Direct NDFT, eq. (1.2) and eq. (1.3)                                       */
/* ------------------------------------------------------------------------- */

static long prod_l(int d, const long *v)
{
    long p = 1;
    for (int t = 0; t < d; ++t)
        p *= v[t];
    return p;
}

/* Frequency vector of centred row-major position idx (R5). */
static void centred_k(int d, const long *N, long idx, long *k)
{
    for (int t = d - 1; t >= 0; --t) {
        long i = idx % N[t];
        idx /= N[t];
        k[t] = i - N[t] / 2;
    }
}

/* exp(sign * 2 pi i k x) for one dimension.  The product k*x is formed in long
 * double, which holds it exactly for |k| <= 2^11, so the fractional part of the
 * phase is exact before it is rounded to double and the angle stays in [0, 2 pi). */
static cplx expo1(long k, double x, int sign)
{
    long double p = (long double)k * (long double)x;
    double fr = (double)(p - floorl(p));
    double ang = (double)sign * 2.0 * OR_PI * fr;
    return cos(ang) + I * sin(ang);
}

/* Per-node tables E_t[i] = exp(sign 2 pi i k_t x_t), k_t = i - N_t/2, so that
 * exp(sign 2 pi i k.x) = prod_t E_t[k_t + N_t/2] (an identity of the exponential). */
static void node_tables(int d, const long *N, const double *xj, int sign, cplx **E)
{
    for (int t = 0; t < d; ++t)
        for (long i = 0; i < N[t]; ++i)
            E[t][i] = expo1(i - N[t] / 2, xj[t], sign);
}

static cplx **alloc_tables(int d, const long *N)
{
    cplx **E = (cplx **)malloc(sizeof(cplx *) * 3);
    for (int t = 0; t < d; ++t)
        E[t] = (cplx *)malloc(sizeof(cplx) * (size_t)N[t]);
    return E;
}

static void free_tables(int d, cplx **E)
{
    for (int t = 0; t < d; ++t)
        free(E[t]);
    free(E);
}

/* exp(sign 2 pi i k.x) for the centred row-major position idx, from the tables. */
static cplx table_expo(int d, const long *N, long idx, cplx *const *E)
{
    cplx e = 1.0;
    for (int t = d - 1; t >= 0; --t) {
        long i = idx % N[t];
        idx /= N[t];
        e *= E[t][i];
    }
    return e;
}

/* f_j = sum_{k in I_N} fhat_k exp(-2 pi i k.x_j) */
void or_ndft_trafo(int d, const long *N, long M, const double *x, const cplx *fhat, cplx *f)
{
    long nk = prod_l(d, N);
#pragma omp parallel
    {
        cplx **E = alloc_tables(d, N);
#pragma omp for schedule(dynamic, 16)
        for (long j = 0; j < M; ++j) {
            node_tables(d, N, x + j * d, -1, E);
            cplx acc = 0.0;
            for (long idx = 0; idx < nk; ++idx)
                acc += fhat[idx] * table_expo(d, N, idx, E);
            f[j] = acc;
        }
        free_tables(d, E);
    }
}

/* hhat_k = sum_j f_j exp(+2 pi i k.x_j).  Parallel over blocks of nodes would
 * change nothing in the arithmetic per entry, so the loop is over k outright:
 * each k runs the node sum in node order. */
void or_ndft_adjoint(int d, const long *N, long M, const double *x, const cplx *f, cplx *fhat)
{
    long nk = prod_l(d, N);
#pragma omp parallel for schedule(dynamic, 64)
    for (long idx = 0; idx < nk; ++idx) {
        long k[3];
        centred_k(d, N, idx, k);
        cplx acc = 0.0;
        for (long j = 0; j < M; ++j) {
            cplx e = 1.0;
            for (int t = 0; t < d; ++t)
                e *= expo1(k[t], x[j * d + t], +1);
            acc += f[j] * e;
        }
        fhat[idx] = acc;
    }
}

/* NNDFT, the transform with nonequispaced nodes in both domains that Sec. 1 names as a
 * generalisation of the NFFT, written out as its definition: real frequencies v_k (K x d)
 * in place of the integer k of eq. (1.2),
 *   f_j    = sum_k fhat_k exp(-2 pi i v_k.x_j),   j < M,
 *   hhat_k = sum_j f_j    exp(+2 pi i v_k.x_j),   k < K.
 * The phase v_k.x_j is accumulated in long double and reduced modulo 1 before the
 * exponential, as in expo1. */
static cplx expo_real(int d, const double *v, const double *x, int sign)
{
    long double p = 0.0L;
    for (int t = 0; t < d; ++t)
        p += (long double)v[t] * (long double)x[t];
    double fr = (double)(p - floorl(p));
    double ang = (double)sign * 2.0 * OR_PI * fr;
    return cos(ang) + I * sin(ang);
}

void or_nndft_trafo(int d, long K, long M, const double *v, const double *x, const cplx *fhat, cplx *f)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (long j = 0; j < M; ++j) {
        cplx acc = 0.0;
        for (long k = 0; k < K; ++k)
            acc += fhat[k] * expo_real(d, v + k * d, x + j * d, -1);
        f[j] = acc;
    }
}

void or_nndft_adjoint(int d, long K, long M, const double *v, const double *x, const cplx *f, cplx *hhat)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (long k = 0; k < K; ++k) {
        cplx acc = 0.0;
        for (long j = 0; j < M; ++j)
            acc += f[j] * expo_real(d, v + k * d, x + j * d, +1);
        hhat[k] = acc;
    }
}

/* Gradient of L(x, fhat) = || A(x) fhat - y ||_2^2 for the direct NDFT, given the
 * residual r = A(x) fhat - y:
 *   dL/dx_{j,t} = 2 Re( conj(r_j) * sum_k fhat_k (-2 pi i k_t) exp(-2 pi i k.x_j) ).
 * grad is [M][d]. */
void or_ndft_grad_x(int d, const long *N, long M, const double *x, const cplx *fhat, const cplx *r,
                    double *grad)
{
    long nk = prod_l(d, N);
#pragma omp parallel
    {
        cplx **E = alloc_tables(d, N);
#pragma omp for schedule(dynamic, 16)
        for (long j = 0; j < M; ++j) {
            node_tables(d, N, x + j * d, -1, E);
            long k[3];
            cplx acc[3] = {0.0, 0.0, 0.0};
            for (long idx = 0; idx < nk; ++idx) {
                centred_k(d, N, idx, k);
                cplx e = fhat[idx] * table_expo(d, N, idx, E);
                for (int t = 0; t < d; ++t)
                    acc[t] += e * (-2.0 * OR_PI * I * (double)k[t]);
            }
            for (int t = 0; t < d; ++t)
                grad[j * d + t] = 2.0 * creal(conj(r[j]) * acc[t]);
        }
        free_tables(d, E);
    }
}

/* ------------------------------------------------------------------------- */
/* NFFT, Algorithm 2.1 and Algorithm 2.2, step by step                        */
/* ------------------------------------------------------------------------- */

/* Step 1 of Algorithm 2.1 (with the window selected by or_set_window):
 * ghat[k mod n] = fhat_k / (|I_n| prod_t phihat_t(k_t))
 * for k in I_N, zero elsewhere on I_n.  ghat has shape n (row-major). */
void or_nfft_deconv(int d, const long *N, const long *n, int m, const cplx *fhat, cplx *ghat)
{
    long nn = prod_l(d, n), nk = prod_l(d, N);
    double b[3];
    for (int t = 0; t < d; ++t)
        b[t] = win_b(N[t], n[t], m);
    memset(ghat, 0, sizeof(cplx) * (size_t)nn);
    for (long idx = 0; idx < nk; ++idx) {
        long k[3];
        centred_k(d, N, idx, k);
        double c = (double)nn;
        long pos = 0;
        for (int t = 0; t < d; ++t) {
            c *= win_phihat(k[t], n[t], m, b[t]);
            long l = ((k[t] % n[t]) + n[t]) % n[t];
            pos = pos * n[t] + l;
        }
        ghat[pos] = fhat[idx] / c;
    }
}

/* Step 3 of Algorithm 2.2: hhat_k = ghat[k mod n] / (|I_n| prod_t phihat_t(k_t)). */
void or_nfft_deconv_adj(int d, const long *N, const long *n, int m, const cplx *ghat, cplx *fhat)
{
    long nn = prod_l(d, n), nk = prod_l(d, N);
    double b[3];
    for (int t = 0; t < d; ++t)
        b[t] = win_b(N[t], n[t], m);
    for (long idx = 0; idx < nk; ++idx) {
        long k[3];
        centred_k(d, N, idx, k);
        double c = (double)nn;
        long pos = 0;
        for (int t = 0; t < d; ++t) {
            c *= win_phihat(k[t], n[t], m, b[t]);
            long l = ((k[t] % n[t]) + n[t]) % n[t];
            pos = pos * n[t] + l;
        }
        fhat[idx] = ghat[pos] / c;
    }
}

/* Stencil of one node (R2): y_t = n_t x_t, u_t = floor(y_t); stencil point
 * s = 0..2m+1 is grid index l = u_t + s - m (taken mod n_t) at offset
 * z = y_t - l.  The window is a tensor product (the PRE_PSI structure of
 * Table 3.2), so its d*(2m+2) one-dimensional factors are tabulated per node:
 * phi[t][s] = phi_t(y_t - (u_t + s - m)), and dphi likewise for the derivative. */
#define OR_MAXW 64
static void node_factors(int d, const long *N, const long *n, int m, const double *xj, long *u,
                         double phi[3][OR_MAXW], double dphi[3][OR_MAXW])
{
    int W = 2 * m + 2;
    for (int t = 0; t < d; ++t) {
        double b = win_b(N[t], n[t], m);
        double y = (double)n[t] * xj[t];
        u[t] = (long)floor(y);
        for (int s = 0; s < W; ++s) {
            double z = y - (double)(u[t] + s - m);
            phi[t][s] = win_phi(z, m, b);
            if (dphi)
                dphi[t][s] = win_dphi(z, m, b);
        }
    }
}

static long wrap(long l, long n)
{
    long r = l % n;
    return r < 0 ? r + n : r;
}

/* Row-major grid position and window weight of stencil point c (flat over
 * {0..W-1}^d, last dimension fastest). */
static long stencil_point(int d, const long *n, int m, int W, long c, const long *u, int *s)
{
    long pos = 0;
    for (int t = d - 1; t >= 0; --t) {
        s[t] = (int)(c % W);
        c /= W;
    }
    for (int t = 0; t < d; ++t)
        pos = pos * n[t] + wrap(u[t] + s[t] - m, n[t]);
    return pos;
}

static double weight(int d, double phi[3][OR_MAXW], const int *s)
{
    double w = 1.0;
    for (int t = 0; t < d; ++t)
        w *= phi[t][s[t]];
    return w;
}

static long stencil_size(int d, int W)
{
    long cnt = 1;
    for (int t = 0; t < d; ++t)
        cnt *= W;
    return cnt;
}

/* Step 3 of Algorithm 2.1: f_j = sum over the stencil of g_l * prod_t phi_t(n_t x_t - l_t). */
void or_nfft_interp(int d, const long *N, const long *n, int m, long M, const double *x, const cplx *g,
                    cplx *f)
{
    int W = 2 * m + 2;
    long cnt = stencil_size(d, W);
    /* every f_j is its own sum: nodes are shared out among threads */
#pragma omp parallel for schedule(dynamic, 64)
    for (long j = 0; j < M; ++j) {
        double phi[3][OR_MAXW];
        long u[3];
        int s[3];
        node_factors(d, N, n, m, x + j * d, u, phi, NULL);
        cplx acc = 0.0;
        for (long c = 0; c < cnt; ++c) {
            long pos = stencil_point(d, n, m, W, c, u, s);
            acc += g[pos] * weight(d, phi, s);
        }
        f[j] = acc;
    }
}

/* Step 1 of Algorithm 2.2: g_l = sum_j f_j prod_t phi_t(n_t x_{j,t} - l_t), every g_l summed
 * over the nodes in node order.  Threads own disjoint ranges of the first grid index; each
 * walks all nodes in order and adds only into its own range, so every g_l receives exactly
 * the additions of a serial loop over j, in the same order (the result does not depend on
 * the thread count). */
void or_nfft_spread(int d, const long *N, const long *n, int m, long M, const double *x, const cplx *f,
                    cplx *g)
{
    int W = 2 * m + 2;
    long inner = stencil_size(d - 1, W); /* stencil points per first-dimension point */
    memset(g, 0, sizeof(cplx) * (size_t)prod_l(d, n));
#pragma omp parallel
    {
        int nt = omp_get_num_threads(), id = omp_get_thread_num();
        long lo = n[0] * id / nt, hi = n[0] * (id + 1) / nt;
        double phi[3][OR_MAXW];
        for (long j = 0; j < M; ++j) {
            long u[3];
            int s[3];
            /* does the node's stencil reach this thread's range of the first index? */
            long u0 = (long)floor((double)n[0] * x[j * d]);
            int hit = 0;
            for (int s0 = 0; s0 < W && !hit; ++s0) {
                long l0 = wrap(u0 + s0 - m, n[0]);
                hit = l0 >= lo && l0 < hi;
            }
            if (!hit)
                continue;
            node_factors(d, N, n, m, x + j * d, u, phi, NULL);
            for (int s0 = 0; s0 < W; ++s0) {
                long l0 = wrap(u[0] + s0 - m, n[0]);
                if (l0 < lo || l0 >= hi)
                    continue;
                for (long c = s0 * inner; c < (s0 + 1) * inner; ++c) {
                    long pos = stencil_point(d, n, m, W, c, u, s);
                    g[pos] += f[j] * weight(d, phi, s);
                }
            }
        }
    }
}

/* Gradient of f_j = NFFT(x, fhat)_j with respect to x_{j,t}, through the window only:
 * df_j/dx_{j,t} = n_t * sum over the stencil of g_l * phi'_t(.) * prod_{t' != t} phi_t'(.).
 * out is [M][d] complex. */
void or_nfft_interp_dx(int d, const long *N, const long *n, int m, long M, const double *x, const cplx *g,
                       cplx *out)
{
    int W = 2 * m + 2;
    long cnt = stencil_size(d, W);
    double phi[3][OR_MAXW], dphi[3][OR_MAXW];
    for (long j = 0; j < M; ++j) {
        long u[3];
        int s[3];
        node_factors(d, N, n, m, x + j * d, u, phi, dphi);
        cplx acc[3] = {0.0, 0.0, 0.0};
        for (long c = 0; c < cnt; ++c) {
            long pos = stencil_point(d, n, m, W, c, u, s);
            for (int t = 0; t < d; ++t) {
                double w = (double)n[t] * dphi[t][s[t]];
                for (int q = 0; q < d; ++q)
                    if (q != t)
                        w *= phi[q][s[q]];
                acc[t] += g[pos] * w;
            }
        }
        for (int t = 0; t < d; ++t)
            out[j * d + t] = acc[t];
    }
}

/* Algorithm 2.1: f = B F D fhat. */
void or_nfft_trafo(int d, const long *N, const long *n, int m, long M, const double *x, const cplx *fhat,
                   cplx *f)
{
    long nn = prod_l(d, n);
    cplx *g = (cplx *)malloc(sizeof(cplx) * (size_t)nn);
    or_nfft_deconv(d, N, n, m, fhat, g);
    or_fft_d(d, n, g, -1);
    or_nfft_interp(d, N, n, m, M, x, g, f);
    free(g);
}

/* Algorithm 2.2: hhat = D^H F^H B^T f. */
void or_nfft_adjoint(int d, const long *N, const long *n, int m, long M, const double *x, const cplx *f,
                     cplx *fhat)
{
    long nn = prod_l(d, n);
    cplx *g = (cplx *)malloc(sizeof(cplx) * (size_t)nn);
    or_nfft_spread(d, N, n, m, M, x, f, g);
    or_fft_d(d, n, g, +1);
    or_nfft_deconv_adj(d, N, n, m, g, fhat);
    free(g);
}

/* Grid produced by steps 1-2 of Algorithm 2.1 (exposed for step-level checks). */
void or_nfft_grid(int d, const long *N, const long *n, int m, const cplx *fhat, cplx *g)
{
    or_nfft_deconv(d, N, n, m, fhat, g);
    or_fft_d(d, n, g, -1);
}

/* Steps 2-3 of Algorithm 2.2 applied to a given grid (exposed for step-level checks). */
void or_nfft_adjoint_from_grid(int d, const long *N, const long *n, int m, const cplx *g_in, cplx *fhat)
{
    long nn = prod_l(d, n);
    cplx *g = (cplx *)malloc(sizeof(cplx) * (size_t)nn);
    memcpy(g, g_in, sizeof(cplx) * (size_t)nn);
    or_fft_d(d, n, g, +1);
    or_nfft_deconv_adj(d, N, n, m, g, fhat);
    free(g);
}

/* Relative errors, eq. (2.15) and eq. (2.16):
 *   E2   = ||f - ft||_2 / ||f||_2
 *   Einf = ||f - ft||_inf / ||fhat||_1   (norm1 passed in as ref_l1). */
double or_err_l2(const cplx *ref, const cplx *approx, long len)
{
    double num = 0.0, den = 0.0;
    for (long i = 0; i < len; ++i) {
        cplx e = ref[i] - approx[i];
        num += creal(e) * creal(e) + cimag(e) * cimag(e);
        den += creal(ref[i]) * creal(ref[i]) + cimag(ref[i]) * cimag(ref[i]);
    }
    return sqrt(num) / sqrt(den);
}

double or_err_inf(const cplx *ref, const cplx *approx, long len, double ref_l1)
{
    double mx = 0.0;
    for (long i = 0; i < len; ++i) {
        double e = cabs(ref[i] - approx[i]);
        if (e > mx)
            mx = e;
    }
    return mx / ref_l1;
}

/* Thread count used by the OpenMP loops of the direct NDFT (the serial NFFT
 * routines never use more than one). */
#ifdef _OPENMP
#include <omp.h>
void or_set_threads(int nt) { omp_set_num_threads(nt); }
int or_get_threads(void) { return omp_get_max_threads(); }
#else
void or_set_threads(int nt) { (void)nt; }
int or_get_threads(void) { return 1; }
#endif

/* hhat_k of eq. (1.3) for the `nsel` centred row-major positions listed in sel
 * (for checks of single outputs of a large transform). */
void or_ndft_adjoint_at(int d, const long *N, long M, const double *x, const cplx *f, long nsel, const long *sel,
                        cplx *out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (long q = 0; q < nsel; ++q) {
        long k[3];
        centred_k(d, N, sel[q], k);
        cplx acc = 0.0;
        for (long j = 0; j < M; ++j) {
            cplx e = 1.0;
            for (int t = 0; t < d; ++t)
                e *= expo1(k[t], x[j * d + t], +1);
            acc += f[j] * e;
        }
        out[q] = acc;
    }
}
