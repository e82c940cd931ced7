/*
 * fft_oracle.c -- plain, slow, obviously correct CPU reference for the
 * batched complex-to-complex DFT (TEST INFRASTRUCTURE ONLY).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library.  The GPU library shares no code, header, table or
 * constant generator with it.
 *
 * What it computes (TurboFFT, Sec. 2.2 "DFT and FFT"):
 *   forward  y_k = sum_n x_n * exp(-2*pi*i*k*n/N)
 *   inverse  x_k = (1/N) sum_n y_n * exp(+2*pi*i*k*n/N)
 * i.e. y = W x with W = (w_N^{jk}), w_N = exp(-2*pi*i/N).  The FFT reaches the
 * same result up to rounding, so the oracle is that definition written out:
 *   - oracle_dft : the O(N^2) matrix-vector product, exponent index (j*k) mod N
 *                  reduced exactly in integers;
 *   - oracle_fft : the textbook recursive decimation-in-time factorisation
 *                  (split by 2, else by 3, else fall back to the DFT), which the
 *                  paper cites as the sparse factorisation of W (Van Loan).
 * All arithmetic is IEEE binary64.  Complex numbers are interleaved (re, im).
 *
 * Twiddles exp(sign*2*pi*i*m/N) are evaluated accurately: m is reduced modulo N
 * in integers, folded into the first octant by symmetry, and std cos/sin is
 * called on an angle of at most pi/4 whose numerator is an exact integer.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double re, im; } cd;

/* exp(sign * 2*pi*i * m / N), sign = -1 (forward) or +1 (inverse). */
void oracle_twiddle(long long N, long long m, int sign, double* out_re, double* out_im)
{
    const long double PI_L = 3.141592653589793238462643383279502884L;
    long long r = m % N;
    if (r < 0) r += N;
    int mirrored = 0;                 /* w^r = conj(w^(N-r)) */
    if (2 * r > N) { r = N - r; mirrored = 1; }
    /* now 0 <= r <= N/2, theta = 2*pi*r/N in [0, pi] */
    double c, s;
    long long e8 = 8 * r;
    if (e8 <= N) {                    /* theta <= pi/4 */
        long double th = 2.0L * PI_L * (long double)r / (long double)N;
        c = (double)cosl(th); s = (double)sinl(th);
    } else if (e8 <= 2 * N) {         /* theta = pi/2 - phi, phi in [0, pi/4] */
        long double ph = PI_L * (long double)(N - 4 * r) / (2.0L * (long double)N);
        c = (double)sinl(ph); s = (double)cosl(ph);
    } else if (e8 <= 3 * N) {         /* theta = pi/2 + phi */
        long double ph = PI_L * (long double)(4 * r - N) / (2.0L * (long double)N);
        c = -(double)sinl(ph); s = (double)cosl(ph);
    } else {                          /* theta = pi - phi, phi = pi*(N-2r)/N */
        long double ph = PI_L * (long double)(N - 2 * r) / (long double)N;
        c = -(double)cosl(ph); s = (double)sinl(ph);
    }
    /* exp(i*theta) = (c, s); exp(-i*theta) = (c, -s); mirroring conjugates. */
    double sign_im = (double)sign * (mirrored ? -1.0 : 1.0);
    *out_re = c;
    *out_im = sign_im * s;
}

/* O(N^2) DFT of one signal.  sign = -1 forward, +1 inverse (unscaled). */
void oracle_dft(const double* x, double* y, long long N, int sign)
{
    const cd* xc = (const cd*)x;
    cd* yc = (cd*)y;
    cd* w = (cd*)malloc(sizeof(cd) * (size_t)N);
    for (long long m = 0; m < N; ++m) oracle_twiddle(N, m, sign, &w[m].re, &w[m].im);
    for (long long k = 0; k < N; ++k) {
        double sr = 0.0, si = 0.0;
        for (long long n = 0; n < N; ++n) {
            long long idx = (long long)(((unsigned long long)k * (unsigned long long)n) % (unsigned long long)N);
            sr += xc[n].re * w[idx].re - xc[n].im * w[idx].im;
            si += xc[n].re * w[idx].im + xc[n].im * w[idx].re;
        }
        yc[k].re = sr; yc[k].im = si;
    }
    free(w);
}

/*
 * Recursive DIT: X[k] = sum_{r<p} w_N^{r k} * S_r[k mod (N/p)], where S_r is
 * the length-N/p DFT of x[r], x[r+p], x[r+2p], ...  The table wtop holds
 * w_Ntop^j for the top-level length; a sub-length M uses w_M^j = w_Ntop^{j*Ntop/M}.
 */
static void fft_rec(const cd* x, long long stride, cd* y, long long M,
                    const cd* wtop, long long Ntop)
{
    if (M == 1) { y[0] = x[0]; return; }
    int p = (M % 2 == 0) ? 2 : ((M % 3 == 0) ? 3 : 0);
    long long step = Ntop / M;        /* w_M^j = wtop[j * step] */
    if (p == 0) {                     /* no small factor left: plain DFT */
        for (long long k = 0; k < M; ++k) {
            double sr = 0.0, si = 0.0;
            for (long long n = 0; n < M; ++n) {
                long long j = (k * n) % M;
                const cd w = wtop[j * step];
                const cd v = x[n * stride];
                sr += v.re * w.re - v.im * w.im;
                si += v.re * w.im + v.im * w.re;
            }
            y[k].re = sr; y[k].im = si;
        }
        return;
    }
    long long m = M / p;
    cd* sub = (cd*)malloc(sizeof(cd) * (size_t)M);
    for (int r = 0; r < p; ++r) fft_rec(x + r * stride, stride * p, sub + r * m, m, wtop, Ntop);
    for (long long k = 0; k < M; ++k) {
        double sr = 0.0, si = 0.0;
        for (int r = 0; r < p; ++r) {
            long long j = ((long long)r * k) % M;
            const cd w = wtop[j * step];
            const cd v = sub[r * m + (k % m)];
            sr += v.re * w.re - v.im * w.im;
            si += v.re * w.im + v.im * w.re;
        }
        y[k].re = sr; y[k].im = si;
    }
    free(sub);
}

/* One signal, recursive FFT.  sign = -1 forward, +1 inverse (unscaled). */
void oracle_fft(const double* x, double* y, long long N, int sign)
{
    cd* w = (cd*)malloc(sizeof(cd) * (size_t)N);
    for (long long m = 0; m < N; ++m) oracle_twiddle(N, m, sign, &w[m].re, &w[m].im);
    fft_rec((const cd*)x, 1, (cd*)y, N, w, N);
    free(w);
}

/*
 * Batched transform of `count` signals of length N stored back to back
 * ([count][N] interleaved).  dir = -1 forward, +1 inverse; every output is
 * multiplied by `scale` (the caller passes 1 or 1/N).  use_dft selects the
 * O(N^2) definition instead of the recursive factorisation.
 */
void oracle_batch(const double* x, double* y, long long N, long long count,
                  int dir, double scale, int use_dft)
{
    cd* w = (cd*)malloc(sizeof(cd) * (size_t)N);
    for (long long m = 0; m < N; ++m) oracle_twiddle(N, m, dir, &w[m].re, &w[m].im);
    for (long long b = 0; b < count; ++b) {
        const double* xb = x + 2 * N * b;
        double* yb = y + 2 * N * b;
        if (use_dft) oracle_dft(xb, yb, N, dir);
        else fft_rec((const cd*)xb, 1, (cd*)yb, N, w, N);
        if (scale != 1.0)
            for (long long k = 0; k < 2 * N; ++k) yb[k] *= scale;
    }
    free(w);
}

/*
 * Single output bins y_k for a list of k (O(N) each): the DFT row k applied
 * to x, used to check a sample of outputs of very long transforms.
 */
void oracle_dft_bins(const double* x, long long N, const long long* ks, long long nk,
                     int dir, double* out)
{
    for (long long q = 0; q < nk; ++q) {
        long long k = ks[q];
        double sr = 0.0, si = 0.0;
        for (long long n = 0; n < N; ++n) {
            double wr, wi;
            long long j = (long long)(((unsigned long long)k * (unsigned long long)n) % (unsigned long long)N);
            oracle_twiddle(N, j, dir, &wr, &wi);
            sr += x[2 * n] * wr - x[2 * n + 1] * wi;
            si += x[2 * n] * wi + x[2 * n + 1] * wr;
        }
        out[2 * q] = sr; out[2 * q + 1] = si;
    }
}
