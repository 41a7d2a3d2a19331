/*
 * FP64 CPU oracle of the wide-field measurement operator Phi = G F Z
 * (paper: eq. 1 and its description of G, F and Z in the introduction;
 * appendix E for the w-term and the row-wise w-kernel convolution in G).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
 * GPU library is checked against. Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it. It shares no code, header, table
 * or helper with the GPU library; the only inputs both sides share are the
 * seeded draws of the `synth` module and the per-plane w-kernel taps computed
 * by the oracle's own Python layer (least-squares fit in phi.py).
 *
 * Conventions (readings of passages the paper leaves open):
 *   - forward Fourier kernel exp(-i ...), adjoint exp(+i ...); the DFT is
 *     unnormalised both ways;
 *   - centred pixel indices n in [-N/2, N/2)^2, stored at [n_y+N/2][n_x+N/2];
 *   - zero padding is wrap-centred: pixel n sits at grid cell (n mod N');
 *   - grid position of a visibility p = omega N' / (2 pi) (cells), its window
 *     centre c = floor(p + 1/2) and fraction f = p - c in [-1/2, 1/2);
 *   - the Kaiser-Bessel kernel has odd width J with taps j = -(J-1)/2 .. (J-1)/2
 *     relative to c, weight kappa(f - j).
 * Complex arrays are interleaved (re, im) double pairs, i.e. C99 double complex.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cpx;

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* Kaiser-Bessel interpolation kernel (the paper cites Fessler2003 for the   */
/* NUFFT interpolation kernels of G and the matching correction in Z).       */
/* ------------------------------------------------------------------------ */

/* Modified Bessel function of the first kind, order 0, by its power series
 * I0(x) = sum_k (x^2/4)^k / (k!)^2, summed until the terms stop mattering. */
double or_i0(double x)
{
    double q = 0.25 * x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 1000; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term <= 1e-18 * sum) break;
    }
    return sum;
}

/* Shape parameter of Beatty et al. (2005) for width J and oversampling sigma. */
double or_kb_beta(int J, double sigma)
{
    double a = (double)J / sigma * (sigma - 0.5);
    return M_PI * sqrt(a * a - 0.8);
}

/* kappa(t) = I0(beta sqrt(1 - (2t/J)^2)) / I0(beta) for |t| <= J/2, else 0. */
double or_kb(double t, int J, double beta)
{
    double u = 2.0 * t / (double)J;
    if (fabs(u) > 1.0) return 0.0;
    return or_i0(beta * sqrt(1.0 - u * u)) / or_i0(beta);
}

/* Continuous Fourier transform of kappa, kappa_hat(nu) = int kappa(t) e^{-2 pi i nu t} dt
 * = (J / I0(beta)) sinh(a)/a with a = sqrt(beta^2 - (pi J nu)^2) (sin for a^2 < 0). */
double or_kb_hat(double nu, int J, double beta)
{
    double z = M_PI * (double)J * nu;
    double a2 = beta * beta - z * z, r;
    if (a2 > 0.0) { double a = sqrt(a2); r = sinh(a) / a; }
    else if (a2 < 0.0) { double a = sqrt(-a2); r = sin(a) / a; }
    else r = 1.0;
    return (double)J * r / or_i0(beta);
}

/* ------------------------------------------------------------------------ */
/* F: unnormalised DFT by an iterative radix-2 Cooley-Tukey FFT.             */
/* sign = -1: forward, X[k] = sum_j x[j] e^{-2 pi i jk/n}; sign = +1: adjoint. */
/* ------------------------------------------------------------------------ */
void or_fft1d(cpx *a, int n, int sign)
{
    if (n < 1 || (n & (n - 1))) abort();            /* radix 2 only */
    for (int i = 1, j = 0; i < n; ++i) {            /* bit-reversal permutation */
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cpx t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len >> 1;
        for (int k = 0; k < half; ++k) {
            double ang = (double)sign * 2.0 * M_PI * (double)k / (double)len;
            cpx w = cos(ang) + I * sin(ang);
            for (int i = 0; i < n; i += len) {
                cpx u = a[i + k], v = a[i + k + half] * w;
                a[i + k] = u + v;
                a[i + k + half] = u - v;
            }
        }
    }
}

/* 2D transform of an n x n row-major array: rows, then columns. */
void or_fft2d(cpx *a, int n, int sign)
{
    #pragma omp parallel for schedule(static)
    for (int r = 0; r < n; ++r) or_fft1d(a + (size_t)r * n, n, sign);
    #pragma omp parallel
    {
        cpx *col = (cpx *)malloc(sizeof(cpx) * (size_t)n);
        #pragma omp for schedule(static)
        for (int c = 0; c < n; ++c) {
            for (int r = 0; r < n; ++r) col[r] = a[(size_t)r * n + c];
            or_fft1d(col, n, sign);
            for (int r = 0; r < n; ++r) a[(size_t)r * n + c] = col[r];
        }
        free(col);
    }
}

/* ------------------------------------------------------------------------ */
/* Z and its adjoint (zero-padding to the N' grid with the kappa_hat         */
/* correction, wrap-centred placement).                                      */
/* ------------------------------------------------------------------------ */
static inline int64_t wrap(int64_t i, int64_t n) { i %= n; return i < 0 ? i + n : i; }

void or_zpad(int N, int Np, int J, double beta, const double *x, cpx *X0)
{
    memset(X0, 0, sizeof(cpx) * (size_t)Np * Np);
    double *corr = (double *)malloc(sizeof(double) * N);
    for (int i = 0; i < N; ++i) corr[i] = or_kb_hat((double)(i - N / 2) / Np, J, beta);
    for (int iy = 0; iy < N; ++iy)
        for (int ix = 0; ix < N; ++ix) {
            int64_t gy = wrap(iy - N / 2, Np), gx = wrap(ix - N / 2, Np);
            X0[gy * Np + gx] = x[(size_t)iy * N + ix] / (corr[ix] * corr[iy]);
        }
    free(corr);
}

/* Real part of Z^dagger: x_n = Re{Y[n mod N']} / (kappa_hat(n_x/N') kappa_hat(n_y/N')). */
void or_zpad_adj(int N, int Np, int J, double beta, const cpx *Y, double *x)
{
    double *corr = (double *)malloc(sizeof(double) * N);
    for (int i = 0; i < N; ++i) corr[i] = or_kb_hat((double)(i - N / 2) / Np, J, beta);
    for (int iy = 0; iy < N; ++iy)
        for (int ix = 0; ix < N; ++ix) {
            int64_t gy = wrap(iy - N / 2, Np), gx = wrap(ix - N / 2, Np);
            x[(size_t)iy * N + ix] = creal(Y[gy * Np + gx]) / (corr[ix] * corr[iy]);
        }
    free(corr);
}

/* ------------------------------------------------------------------------ */
/* G: one sparse row per visibility. Per axis, the w-kernel taps k[q]        */
/* (|q| <= h) are convolved with the J Kaiser-Bessel taps:                   */
/*   g[a] = sum_q k[q] kappa(f - a - q),  |a + q| <= (J-1)/2,                */
/*   a in [-(h + (J-1)/2), h + (J-1)/2],                                     */
/* and G_{m,(ky,kx)} = g_v[ay] g_u[ax] at cell (c_v + ay, c_u + ax) mod N'.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int N, Np, J, hmax;
    double beta;
    int64_t M;
    const double *pu, *pv;      /* grid positions p = omega N'/(2 pi), FP64 */
    const int32_t *plane;       /* per-visibility w-plane index */
    const int32_t *plane_h;     /* per-plane half-support h */
    const cpx *plane_k;         /* per-plane taps, stride 2*hmax+1, q = -hmax..hmax */
} or_op;

static void axis_weights(double f, const cpx *k /* k[q], q in [-h,h] */, int h,
                         int J, double beta, cpx *g /* 2h+J entries */)
{
    int jh = (J - 1) / 2;
    double kb[64];
    for (int j = -jh; j <= jh; ++j) kb[j + jh] = or_kb(f - (double)j, J, beta);
    for (int a = -h - jh; a <= h + jh; ++a) {
        cpx s = 0.0;
        for (int q = -h; q <= h; ++q) {
            int j = a + q;
            if (j < -jh || j > jh) continue;
            s += k[q] * kb[j + jh];
        }
        g[a + h + jh] = s;
    }
}

static void row_setup(const or_op *op, int64_t m, int64_t *cu, int64_t *cv, int *h,
                      cpx *gu, cpx *gv)
{
    double fcu = floor(op->pu[m] + 0.5), fcv = floor(op->pv[m] + 0.5);
    double fu = op->pu[m] - fcu, fv = op->pv[m] - fcv;
    int pl = op->plane[m];
    *h = op->plane_h[pl];
    const cpx *k = op->plane_k + (size_t)pl * (2 * op->hmax + 1) + op->hmax;
    axis_weights(fu, k, *h, op->J, op->beta, gu);
    axis_weights(fv, k, *h, op->J, op->beta, gv);
    *cu = (int64_t)fcu;
    *cv = (int64_t)fcv;
}

/* y = G X */
void or_degrid(const or_op *op, const cpx *X, cpx *y)
{
    const int jh = (op->J - 1) / 2;
    #pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t m = 0; m < op->M; ++m) {
        int64_t cu, cv; int h;
        cpx gu[64], gv[64];
        row_setup(op, m, &cu, &cv, &h, gu, gv);
        int S = 2 * h + op->J, off = h + jh;
        cpx acc = 0.0;
        for (int ay = 0; ay < S; ++ay) {
            int64_t ky = wrap(cv + ay - off, op->Np);
            for (int ax = 0; ax < S; ++ax) {
                int64_t kx = wrap(cu + ax - off, op->Np);
                acc += gv[ay] * gu[ax] * X[ky * op->Np + kx];
            }
        }
        y[m] = acc;
    }
}

/* Y = G^H r (Y is overwritten). Each thread owns a band of grid rows and
 * walks all visibilities in order, so every cell sums its contributions in
 * visibility order (deterministic for a fixed thread count). */
void or_grid(const or_op *op, const cpx *r, cpx *Y)
{
    const int64_t Np = op->Np;
    const int jh = (op->J - 1) / 2;
    memset(Y, 0, sizeof(cpx) * (size_t)Np * Np);
    int nb = 1;
#ifdef _OPENMP
    nb = omp_get_max_threads();
#endif
    if (nb > Np) nb = (int)Np;
    #pragma omp parallel for schedule(static, 1)
    for (int b = 0; b < nb; ++b) {
        int64_t r0 = Np * b / nb, r1 = Np * (b + 1) / nb;
        for (int64_t m = 0; m < op->M; ++m) {
            double fcv = floor(op->pv[m] + 0.5);
            int h = op->plane_h[op->plane[m]];
            int S = 2 * h + op->J, off = h + jh;
            /* does any window row fall into [r0, r1)? */
            int hit = 0;
            for (int ay = 0; ay < S && !hit; ++ay) {
                int64_t ky = wrap((int64_t)fcv + ay - off, Np);
                hit = (ky >= r0 && ky < r1);
            }
            if (!hit) continue;
            int64_t cu, cv;
            cpx gu[64], gv[64];
            row_setup(op, m, &cu, &cv, &h, gu, gv);
            for (int ay = 0; ay < S; ++ay) {
                int64_t ky = wrap(cv + ay - off, Np);
                if (ky < r0 || ky >= r1) continue;
                for (int ax = 0; ax < S; ++ax) {
                    int64_t kx = wrap(cu + ax - off, Np);
                    Y[ky * Np + kx] += conj(gv[ay] * gu[ax]) * r[m];
                }
            }
        }
    }
}

/* Dense G row values of visibility m in window order (row-major over (ay, ax)),
 * and the flat grid index of every entry. Returns the window side S. */
int or_g_row(const or_op *op, int64_t m, cpx *vals, int64_t *cols)
{
    const int jh = (op->J - 1) / 2;
    int64_t cu, cv; int h;
    cpx gu[64], gv[64];
    row_setup(op, m, &cu, &cv, &h, gu, gv);
    int S = 2 * h + op->J, off = h + jh;
    for (int ay = 0; ay < S; ++ay)
        for (int ax = 0; ax < S; ++ax) {
            vals[ay * S + ax] = gv[ay] * gu[ax];
            cols[ay * S + ax] = wrap(cv + ay - off, op->Np) * op->Np + wrap(cu + ax - off, op->Np);
        }
    return S;
}

/* ------------------------------------------------------------------------ */
/* Phi = G F Z and Re{Phi^dagger}                                            */
/* ------------------------------------------------------------------------ */
void or_phi(const or_op *op, const double *x, cpx *y)
{
    size_t ng = (size_t)op->Np * op->Np;
    cpx *X = (cpx *)malloc(sizeof(cpx) * ng);
    or_zpad(op->N, op->Np, op->J, op->beta, x, X);
    or_fft2d(X, op->Np, -1);
    or_degrid(op, X, y);
    free(X);
}

void or_phi_adj(const or_op *op, const cpx *y, double *x)
{
    size_t ng = (size_t)op->Np * op->Np;
    cpx *Y = (cpx *)malloc(sizeof(cpx) * ng);
    or_grid(op, y, Y);
    or_fft2d(Y, op->Np, +1);
    or_zpad_adj(op->N, op->Np, op->J, op->beta, Y, x);
    free(Y);
}

/* Exported entry points with plain arguments (for ctypes). */
#define OP_ARGS int N, int Np, int J, double beta, int hmax, int64_t M,            \
                const double *pu, const double *pv, const int32_t *plane,          \
                const int32_t *plane_h, const double *plane_k
#define OP_INIT or_op op = { N, Np, J, hmax, beta, M, pu, pv, plane, plane_h,      \
                             (const cpx *)plane_k }

void or_phi_c(OP_ARGS, const double *x, double *y)            { OP_INIT; or_phi(&op, x, (cpx *)y); }
void or_phi_adj_c(OP_ARGS, const double *y, double *x)        { OP_INIT; or_phi_adj(&op, (const cpx *)y, x); }
void or_degrid_c(OP_ARGS, const double *X, double *y)         { OP_INIT; or_degrid(&op, (const cpx *)X, (cpx *)y); }
void or_grid_c(OP_ARGS, const double *r, double *Y)           { OP_INIT; or_grid(&op, (const cpx *)r, (cpx *)Y); }
int  or_g_row_c(OP_ARGS, int64_t m, double *vals, int64_t *cols) { OP_INIT; return or_g_row(&op, m, (cpx *)vals, cols); }

/* Re{Phi^dagger (Phi x - y)} with the residual squared norm (y may be NULL). */
double or_grad_c(OP_ARGS, const double *x, const double *y, double *g)
{
    OP_INIT;
    cpx *r = (cpx *)malloc(sizeof(cpx) * (size_t)M);
    or_phi(&op, x, r);
    double rr = 0.0;
    for (int64_t m = 0; m < M; ++m) {
        if (y) r[m] -= ((const cpx *)y)[m];
        rr += creal(r[m]) * creal(r[m]) + cimag(r[m]) * cimag(r[m]);
    }
    or_phi_adj(&op, r, g);
    free(r);
    return rr;
}

void or_fft2d_c(double *a, int n, int sign) { or_fft2d((cpx *)a, n, sign); }
void or_fft1d_c(double *a, int n, int sign) { or_fft1d((cpx *)a, n, sign); }
void or_zpad_c(int N, int Np, int J, double beta, const double *x, double *X0) { or_zpad(N, Np, J, beta, x, (cpx *)X0); }
void or_zpad_adj_c(int N, int Np, int J, double beta, const double *Y, double *x) { or_zpad_adj(N, Np, J, beta, (const cpx *)Y, x); }

/* ------------------------------------------------------------------------ */
/* Brute-force direct model (paper eq. 1 with the closed-form w-term of      */
/* appendix E): y_m = sum_n x_n exp(-i omega_m . n)                          */
/*                        exp(-2 pi i w_m (sqrt(1 - l^2 - m^2) - 1)),        */
/* l = n_x delta, m = n_y delta. paraxial != 0 replaces sqrt(1-s)-1 by -s/2. */
/* ------------------------------------------------------------------------ */
static inline double wphase(double w, double l, double mm, int paraxial)
{
    double s = l * l + mm * mm;
    double d = paraxial ? -0.5 * s : sqrt(1.0 - s) - 1.0;
    return -2.0 * M_PI * w * d;
}

void or_dft_c(int N, int64_t M, const double *uvw, double cell, int paraxial,
              const double *x, double *y_out)
{
    cpx *y = (cpx *)y_out;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t m = 0; m < M; ++m) {
        double ou = uvw[3 * m], ov = uvw[3 * m + 1], w = uvw[3 * m + 2];
        cpx acc = 0.0;
        for (int iy = 0; iy < N; ++iy) {
            int ny = iy - N / 2;
            for (int ix = 0; ix < N; ++ix) {
                int nx = ix - N / 2;
                double ph = -(ou * nx + ov * ny) + wphase(w, nx * cell, ny * cell, paraxial);
                acc += x[(size_t)iy * N + ix] * (cos(ph) + I * sin(ph));
            }
        }
        y[m] = acc;
    }
}

/* Real-image adjoint of the direct model: x_n = Re sum_m conj(phase_mn) y_m. */
void or_dft_adj_c(int N, int64_t M, const double *uvw, double cell, int paraxial,
                  const double *y_in, double *x)
{
    const cpx *y = (const cpx *)y_in;
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < (int64_t)N * N; ++p) {
        int ny = (int)(p / N) - N / 2, nx = (int)(p % N) - N / 2;
        double acc = 0.0;
        for (int64_t m = 0; m < M; ++m) {
            double ph = -(uvw[3 * m] * nx + uvw[3 * m + 1] * ny)
                        + wphase(uvw[3 * m + 2], nx * cell, ny * cell, paraxial);
            acc += creal((cos(ph) - I * sin(ph)) * y[m]);
        }
        x[p] = acc;
    }
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel regions, for timing: every sum above is
 * taken in the same order whatever the thread count (per visibility, per FFT
 * row or column, and per grid cell in visibility order), so results do not
 * depend on it. */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
