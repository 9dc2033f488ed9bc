/*
 * Driver for the sanitizer run of the CPU oracle (tests/test_oracle_sanitize.py): every
 * exported routine of oracle/nfft_oracle.c on small inputs -- every window, d = 1..3,
 * power-of-two and other grid lengths (the latter take the naive DFT), nodes inside and
 * outside [-1/2, 1/2) -- so that AddressSanitizer and UndefinedBehaviorSanitizer see each
 * code path once.  Test infrastructure: built and run only by that test.  Prints one line
 * per case and "done"; a sanitizer finding aborts the run.
 */
#include <complex.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef double complex cplx;

double or_bessel_i0(double x);
double or_kb_b(long N, long n);
double or_kb_phi(double z, int m, double b);
double or_kb_dphi(double z, int m, double b);
double or_kb_phihat(long k, long n, int m, double b);
double or_gauss_b(long N, long n, int m);
double or_gauss_phi(double z, double b);
double or_gauss_dphi(double z, double b);
double or_gauss_phihat(long k, long n, double b);
double or_bspline_n(int k, double x);
double or_bspline_phi(double z, int m);
double or_bspline_dphi(double z, int m);
double or_bspline_phihat(long k, long n, int m);
double or_sinc_a(long N, long n, int m);
double or_sinc_phi(double z, int m, double a);
double or_sinc_dphi(double z, int m, double a);
double or_sinc_phihat(long k, long n, int m, double a);
void or_set_window(int w);
int or_get_window(void);
void or_dft_naive(const cplx *in, cplx *out, long n, int sign);
void or_fft_1d(cplx *a, long n, int sign);
void or_fft_d(int d, const long *n, cplx *a, int sign);
void or_ndft_trafo(int d, const long *N, long M, const double *x, const cplx *fhat, cplx *f);
void or_ndft_adjoint(int d, const long *N, long M, const double *x, const cplx *f, cplx *fhat);
void or_nndft_trafo(int d, long K, long M, const double *v, const double *x, const cplx *fhat, cplx *f);
void or_nndft_adjoint(int d, long K, long M, const double *v, const double *x, const cplx *f, cplx *hhat);
void or_ndft_grad_x(int d, const long *N, long M, const double *x, const cplx *fhat, const cplx *r, double *g);
void or_nfft_deconv(int d, const long *N, const long *n, int m, const cplx *fhat, cplx *ghat);
void or_nfft_deconv_adj(int d, const long *N, const long *n, int m, const cplx *ghat, cplx *fhat);
void or_nfft_interp(int d, const long *N, const long *n, int m, long M, const double *x, const cplx *g, cplx *f);
void or_nfft_spread(int d, const long *N, const long *n, int m, long M, const double *x, const cplx *f, cplx *g);
void or_nfft_interp_dx(int d, const long *N, const long *n, int m, long M, const double *x, const cplx *g,
                       cplx *dfdx);
void or_nfft_trafo(int d, const long *N, const long *n, int m, long M, const double *x, const cplx *fhat, cplx *f);
void or_nfft_adjoint(int d, const long *N, const long *n, int m, long M, const double *x, const cplx *f,
                     cplx *fhat);
void or_nfft_grid(int d, const long *N, const long *n, int m, const cplx *fhat, cplx *g);
void or_nfft_adjoint_from_grid(int d, const long *N, const long *n, int m, const cplx *g_in, cplx *fhat);
double or_err_l2(const cplx *ref, const cplx *approx, long len);
double or_err_inf(const cplx *ref, const cplx *approx, long len, double ref_l1);

static unsigned long long rng = 88172645463325252ull;
static double urand(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static long prod(int d, const long *v)
{
    long p = 1;
    for (int t = 0; t < d; ++t)
        p *= v[t];
    return p;
}

static void *xmalloc(size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

/* one plan shape: every transform, step and error routine; returns E_2 of the NFFT */
static double run_case(int d, const long *N, const long *n, int m, long M, double spread_x)
{
    const long nN = prod(d, N), nn = prod(d, n);
    double *x = xmalloc(sizeof(double) * (size_t)(M * d));
    cplx *fhat = xmalloc(sizeof(cplx) * (size_t)nN), *f = xmalloc(sizeof(cplx) * (size_t)M);
    cplx *fref = xmalloc(sizeof(cplx) * (size_t)M), *fin = xmalloc(sizeof(cplx) * (size_t)M);
    cplx *h = xmalloc(sizeof(cplx) * (size_t)nN), *href = xmalloc(sizeof(cplx) * (size_t)nN);
    cplx *g = xmalloc(sizeof(cplx) * (size_t)nn), *g2 = xmalloc(sizeof(cplx) * (size_t)nn);
    cplx *ghat = xmalloc(sizeof(cplx) * (size_t)nn), *dfdx = xmalloc(sizeof(cplx) * (size_t)(M * d));
    double *grad = xmalloc(sizeof(double) * (size_t)(M * d));
    for (long i = 0; i < M * d; ++i)
        x[i] = (urand() - 0.5) * spread_x;
    for (long i = 0; i < nN; ++i)
        fhat[i] = (urand() - 0.5) + I * (urand() - 0.5);
    for (long j = 0; j < M; ++j)
        fin[j] = (urand() - 0.5) + I * (urand() - 0.5);
    or_ndft_trafo(d, N, M, x, fhat, fref);
    or_ndft_adjoint(d, N, M, x, fin, href);
    or_ndft_grad_x(d, N, M, x, fhat, fin, grad);
    or_nfft_trafo(d, N, n, m, M, x, fhat, f);
    or_nfft_adjoint(d, N, n, m, M, x, fin, h);
    or_nfft_deconv(d, N, n, m, fhat, ghat);
    or_nfft_deconv_adj(d, N, n, m, ghat, h);
    or_nfft_grid(d, N, n, m, fhat, g);
    or_nfft_interp(d, N, n, m, M, x, g, f);
    or_nfft_interp_dx(d, N, n, m, M, x, g, dfdx);
    or_nfft_spread(d, N, n, m, M, x, fin, g2);
    or_nfft_adjoint_from_grid(d, N, n, m, g2, h);
    or_fft_d(d, n, g2, -1);
    double l1 = 0.0;
    for (long i = 0; i < nN; ++i)
        l1 += cabs(fhat[i]);
    (void)or_err_inf(fref, f, M, l1);
    const double e2 = or_err_l2(fref, f, M);
    free(x); free(fhat); free(f); free(fref); free(fin); free(h); free(href);
    free(g); free(g2); free(ghat); free(dfdx); free(grad);
    return e2;
}

int main(void)
{
    /* scalar window routines at and around the stencil edge */
    (void)or_bessel_i0(0.0);
    (void)or_bessel_i0(40.0);
    for (int m = 1; m <= 8; m += 7) {
        const double b = or_kb_b(16, 32), bg = or_gauss_b(16, 32, m), a = or_sinc_a(16, 32, m);
        for (int i = -2 * m - 2; i <= 2 * m + 2; ++i) {
            const double z = 0.5 * i;
            (void)or_kb_phi(z, m, b); (void)or_kb_dphi(z, m, b);
            (void)or_gauss_phi(z, bg); (void)or_gauss_dphi(z, bg);
            (void)or_bspline_phi(z, m); (void)or_bspline_dphi(z, m); (void)or_bspline_n(2 * m, z + m);
            (void)or_sinc_phi(z, m, a); (void)or_sinc_dphi(z, m, a);
        }
        for (long k = -16; k < 16; ++k) {
            (void)or_kb_phihat(k, 32, m, b); (void)or_gauss_phihat(k, 32, bg);
            (void)or_bspline_phihat(k, 32, m); (void)or_sinc_phihat(k, 32, m, a);
        }
    }
    /* FFTs: power of two, odd prime, mixed */
    const long lens[] = {1, 2, 8, 7, 30, 64};
    for (int i = 0; i < 6; ++i) {
        const long L = lens[i];
        cplx *a = xmalloc(sizeof(cplx) * (size_t)L), *o = xmalloc(sizeof(cplx) * (size_t)L);
        for (long j = 0; j < L; ++j)
            a[j] = urand() + I * urand();
        or_dft_naive(a, o, L, 1);
        or_fft_1d(a, L, -1);
        free(a); free(o);
    }
    /* nonequispaced in both domains */
    {
        const long K = 37, M = 41;
        double *v = xmalloc(sizeof(double) * 2 * K), *xx = xmalloc(sizeof(double) * 2 * M);
        cplx *fh = xmalloc(sizeof(cplx) * K), *ff = xmalloc(sizeof(cplx) * M), *hh = xmalloc(sizeof(cplx) * K);
        for (long i = 0; i < 2 * K; ++i) v[i] = (urand() - 0.5) * 20.0;
        for (long i = 0; i < 2 * M; ++i) xx[i] = urand() - 0.5;
        for (long i = 0; i < K; ++i) fh[i] = urand() + I * urand();
        or_nndft_trafo(2, K, M, v, xx, fh, ff);
        or_nndft_adjoint(2, K, M, v, xx, ff, hh);
        free(v); free(xx); free(fh); free(ff); free(hh);
    }
    /* plan shapes for every window */
    struct { int d; long N[3], n[3]; int m; long M; double spread; } cases[] = {
        {1, {16}, {32}, 4, 40, 1.0},
        {1, {10}, {14}, 3, 25, 3.0},          /* odd factor 7: naive DFT; nodes outside [-1/2, 1/2) */
        {2, {8, 12}, {16, 24}, 2, 60, 1.0},
        {2, {6, 8}, {10, 18}, 3, 30, 1.0},   /* 5 and 9 */
        {3, {4, 6, 8}, {8, 12, 16}, 2, 50, 1.0},
        {3, {4, 4, 4}, {8, 8, 8}, 6, 20, 1.0}, /* stencil wider than the grid */
    };
    for (int w = 0; w < 4; ++w) {
        or_set_window(w);
        if (or_get_window() != w)
            return 3;
        for (size_t c = 0; c < sizeof(cases) / sizeof(cases[0]); ++c) {
            const double e2 = run_case(cases[c].d, cases[c].N, cases[c].n, cases[c].m, cases[c].M, cases[c].spread);
            printf("window %d case %zu E2 %.3e\n", w, c, e2);
        }
    }
    or_set_window(0);
    printf("done\n");
    return 0;
}
