/*
 * claire_oracle.c -- slow, plain FP64 CPU oracle for stationary-velocity
 * Gauss-Newton-Krylov image registration (Himthani et al., "CLAIRE --
 * Parallelized Diffeomorphic Image Registration for Large-Scale Biomedical
 * Imaging Applications", arXiv 2209.08189).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant with the HIP implementation.
 *
 * Every array is FP64, C order [x1][x2][x3] with x3 fastest; vector fields
 * are three such arrays back to back.  Indices wrap periodically.  Nothing
 * here is blocked, fused or reordered beyond what the paper's equations and
 * the readings listed per function state.  OpenMP only splits independent
 * output points over x1; every sum is serial, in index order.
 *
 * What is pinned and what is not: every function here is exercised by a pin
 * (closed form, exact special case, library routine or brute force) in the
 * CPU test suite, except the GN iterate sequence on general images, whose
 * only check is consistency of its parts (adjoint identity under refinement,
 * FD gradient check): "parity unpinned" for the outer-iterate sequence.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559

/* ------------------------------------------------------------------ grid */

static long wrapi(long i, long n) { long r = i % n; return r < 0 ? r + n : r; }

static long at(int n1, int n2, int n3, long i, long j, long k)
{
    return (wrapi(i, n1) * n2 + wrapi(j, n2)) * (long)n3 + wrapi(k, n3);
}

/* ---------------------------------------------- cubic Lagrange weights
 * Section 2.2 / Section 3 (IP kernel): cubic Lagrange interpolation.  The
 * four nodes are base-1, base, base+1, base+2 with base = floor(p) and
 * f = p - base in [0,1); weight of node base+a is the Lagrange basis
 * polynomial of that node evaluated at f.                                 */
static void lagrange4(double f, double w[4])
{
    w[0] = -f * (f - 1.0) * (f - 2.0) / 6.0;
    w[1] = (f + 1.0) * (f - 1.0) * (f - 2.0) / 2.0;
    w[2] = -(f + 1.0) * f * (f - 2.0) / 2.0;
    w[3] = (f + 1.0) * f * (f - 1.0) / 6.0;
}

/* Tricubic Lagrange value of u at node (i,j,k) displaced by (d1,d2,d3)
 * index units.  The integer part of the foot is node + floor(d) and the
 * fraction is d - floor(d), both taken from the displacement alone.     */
static double interp_node(int n1, int n2, int n3, const double *u,
                          long i, long j, long k, double d1, double d2, double d3)
{
    double f1 = floor(d1), f2 = floor(d2), f3 = floor(d3);
    long b1 = i + (long)f1, b2 = j + (long)f2, b3 = k + (long)f3;
    double w1[4], w2[4], w3[4];
    lagrange4(d1 - f1, w1);
    lagrange4(d2 - f2, w2);
    lagrange4(d3 - f3, w3);
    double s = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c)
                s += w1[a] * w2[b] * w3[c] *
                     u[at(n1, n2, n3, b1 + a - 1, b2 + b - 1, b3 + c - 1)];
    return s;
}

/* Trilinear value (the paper's linear interpolation option, Section 3.3
 * and Section 3): nodes base and base + 1 per axis with weights 1 - f and
 * f, base = node + floor(d), f = d - floor(d).                            */
static double interp_node_lin(int n1, int n2, int n3, const double *u,
                              long i, long j, long k, double d1, double d2, double d3)
{
    double f1 = floor(d1), f2 = floor(d2), f3 = floor(d3);
    long b1 = i + (long)f1, b2 = j + (long)f2, b3 = k + (long)f3;
    double w1[2] = {1.0 - (d1 - f1), d1 - f1}, w2[2] = {1.0 - (d2 - f2), d2 - f2}, w3[2] = {1.0 - (d3 - f3), d3 - f3};
    double s = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c)
                s += w1[a] * w2[b] * w3[c] * u[at(n1, n2, n3, b1 + a, b2 + b, b3 + c)];
    return s;
}

/* order 1: trilinear, otherwise tricubic Lagrange */
static double interp_node_ord(int order, int n1, int n2, int n3, const double *u,
                              long i, long j, long k, double d1, double d2, double d3)
{
    return order == 1 ? interp_node_lin(n1, n2, n3, u, i, j, k, d1, d2, d3)
                      : interp_node(n1, n2, n3, u, i, j, k, d1, d2, d3);
}

/* out(x_ijk) = I[u](x_ijk + d_ijk), d in index units (3 arrays), with the
 * interpolation of the given order (1 trilinear, 3 tricubic Lagrange). */
void orc_interp_order(int n1, int n2, int n3, int order, const double *u, const double *d, double *out)
{
    long N = (long)n1 * n2 * n3;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n1; ++i)
        for (long j = 0; j < n2; ++j)
            for (long k = 0; k < n3; ++k) {
                long p = (i * n2 + j) * n3 + k;
                out[p] = interp_node_ord(order, n1, n2, n3, u, i, j, k, d[p], d[N + p], d[2 * N + p]);
            }
}

/* out(x_ijk) = I[u](x_ijk + d_ijk), tricubic Lagrange. */
void orc_interp(int n1, int n2, int n3, const double *u, const double *d, double *out)
{
    orc_interp_order(n1, n2, n3, 3, u, d, out);
}

/* Value of I[u] at an arbitrary point p (index units, any real). */
double orc_interp_point(int n1, int n2, int n3, const double *u, double p1, double p2, double p3)
{
    return interp_node(n1, n2, n3, u, 0, 0, 0, p1, p2, p3);
}

double orc_interp_point_lin(int n1, int n2, int n3, const double *u, double p1, double p2, double p3)
{
    return interp_node_lin(n1, n2, n3, u, 0, 0, 0, p1, p2, p3);
}

/* ------------------------------------------------ 8th-order central FD
 * Section 2.2 and Section 3 (FD kernel): first derivatives by the explicit
 * central 9-point stencil of order 8,
 *   du/dx ~ (1/h) sum_{j=1..4} c_j (u[+j] - u[-j]),
 *   c = (4/5, -1/5, 4/105, -1/280).                                    */
static const double FD8[4] = {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};

static double dx_axis(int n1, int n2, int n3, const double *u, long i, long j, long k, int axis)
{
    double s = 0.0;
    for (int q = 1; q <= 4; ++q) {
        double up, um;
        if (axis == 0) { up = u[at(n1, n2, n3, i + q, j, k)]; um = u[at(n1, n2, n3, i - q, j, k)]; }
        else if (axis == 1) { up = u[at(n1, n2, n3, i, j + q, k)]; um = u[at(n1, n2, n3, i, j - q, k)]; }
        else { up = u[at(n1, n2, n3, i, j, k + q)]; um = u[at(n1, n2, n3, i, j, k - q)]; }
        s += FD8[q - 1] * (up - um);
    }
    int n = axis == 0 ? n1 : (axis == 1 ? n2 : n3);
    return s / (TWO_PI / n);
}

void orc_grad(int n1, int n2, int n3, const double *u, double *g)
{
    long N = (long)n1 * n2 * n3;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n1; ++i)
        for (long j = 0; j < n2; ++j)
            for (long k = 0; k < n3; ++k) {
                long p = (i * n2 + j) * n3 + k;
                for (int a = 0; a < 3; ++a) g[a * N + p] = dx_axis(n1, n2, n3, u, i, j, k, a);
            }
}

void orc_div(int n1, int n2, int n3, const double *v, double *out)
{
    long N = (long)n1 * n2 * n3;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n1; ++i)
        for (long j = 0; j < n2; ++j)
            for (long k = 0; k < n3; ++k) {
                long p = (i * n2 + j) * n3 + k;
                out[p] = dx_axis(n1, n2, n3, v, i, j, k, 0) +
                         dx_axis(n1, n2, n3, v + N, i, j, k, 1) +
                         dx_axis(n1, n2, n3, v + 2 * N, i, j, k, 2);
            }
}

/* ------------------------------------------------------------ FFT
 * Textbook iterative radix-2 Cooley-Tukey on one complex line (length a
 * power of two), X[k] = sum_n x[n] exp(sign * 2 pi i n k / L), unscaled.  */
static void fft_line(double *re, double *im, int L, int sign)
{
    for (int i = 1, j = 0; i < L; ++i) {          /* bit reversal */
        int bit = L >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    for (int len = 2; len <= L; len <<= 1) {
        for (int s = 0; s < L; s += len) {
            for (int q = 0; q < len / 2; ++q) {
                double ang = sign * TWO_PI * q / len;
                double wr = cos(ang), wi = sin(ang);
                int a = s + q, b = s + q + len / 2;
                double xr = re[b] * wr - im[b] * wi;
                double xi = re[b] * wi + im[b] * wr;
                re[b] = re[a] - xr; im[b] = im[a] - xi;
                re[a] += xr; im[a] += xi;
            }
        }
    }
}

/* In-place unscaled 3D DFT of a complex array (re, im) with sign +-1.
 * Every extent must be a power of two (radix-2 lines); anything else stops
 * the process with a message rather than running past the line buffers.  */
void orc_fft3(int n1, int n2, int n3, double *re, double *im, int sign)
{
    int dims_chk[3] = {n1, n2, n3};
    for (int a = 0; a < 3; ++a)
        if (dims_chk[a] < 1 || (dims_chk[a] & (dims_chk[a] - 1)) != 0) {
            fprintf(stderr, "orc_fft3: extent %d is not a power of two\n", dims_chk[a]);
            abort();
        }
    int dims[3] = {n1, n2, n3};
    long strides[3] = {(long)n2 * n3, n3, 1};
    long N = (long)n1 * n2 * n3;
    for (int ax = 0; ax < 3; ++ax) {
        int L = dims[ax];
        long st = strides[ax];
        long nlines = N / L;
#pragma omp parallel
        {
            double *br = malloc(sizeof(double) * L), *bi = malloc(sizeof(double) * L);
#pragma omp for schedule(static)
            for (long ln = 0; ln < nlines; ++ln) {
                /* base offset of line ln: enumerate all index tuples with axis index 0 */
                long base;
                if (ax == 0) base = ln;                                   /* (j,k) */
                else if (ax == 1) base = (ln / n3) * (long)n2 * n3 + (ln % n3); /* (i,k) */
                else base = ln * (long)n3;                                /* (i,j) */
                for (int q = 0; q < L; ++q) { br[q] = re[base + q * st]; bi[q] = im[base + q * st]; }
                fft_line(br, bi, L, sign);
                for (int q = 0; q < L; ++q) { re[base + q * st] = br[q]; im[base + q * st] = bi[q]; }
            }
            free(br); free(bi);
        }
    }
}

/* Integer wavenumber of DFT index q on an axis of n points: 0..n/2-1 are
 * non-negative, n/2..n-1 map to -n/2..-1 (the Nyquist index is -n/2).   */
static double wavenum(int q, int n) { return q < n / 2 ? (double)q : (double)(q - n); }

/* Spectral operators (Section 2.2: "two FFTs and one Hadamard product").
 *   kind 0: beta * A,     A = -Laplacian, symbol |k|^2 (H1 seminorm)
 *   kind 1: (beta * A)^-1 with |k|^2 replaced by max(|k|^2, 1)
 *   kind 2: identity (FFT round trip)
 * Applied to ncomp consecutive scalar fields.                           */
void orc_spectral(int n1, int n2, int n3, const double *in, double *out, int ncomp, int kind, double beta)
{
    long N = (long)n1 * n2 * n3;
    double *re = malloc(sizeof(double) * N), *im = malloc(sizeof(double) * N);
    for (int c = 0; c < ncomp; ++c) {
        for (long p = 0; p < N; ++p) { re[p] = in[c * N + p]; im[p] = 0.0; }
        orc_fft3(n1, n2, n3, re, im, -1);
        for (long i = 0; i < n1; ++i)
            for (long j = 0; j < n2; ++j)
                for (long k = 0; k < n3; ++k) {
                    long p = (i * n2 + j) * n3 + k;
                    double k1 = wavenum((int)i, n1), k2 = wavenum((int)j, n2), k3 = wavenum((int)k, n3);
                    double ksq = k1 * k1 + k2 * k2 + k3 * k3;
                    double s;
                    if (kind == 0) s = beta * ksq;
                    else if (kind == 1) s = 1.0 / (beta * (ksq > 1.0 ? ksq : 1.0));
                    else s = 1.0;
                    re[p] *= s; im[p] *= s;
                }
        orc_fft3(n1, n2, n3, re, im, +1);
        for (long p = 0; p < N; ++p) out[c * N + p] = re[p] / (double)N;
    }
    free(re); free(im);
}

/* ------------------------------------------ near-incompressible part
 * The objective of Section 2.1 with beta_w > 0: w = div v is penalised by
 * its H1 norm, so the regularisation is
 *   R(v) = beta_v/2 <A v, v> + beta_w/2 (<w, w> + <A w, w>),
 * the H1 norm written with A = -Laplacian (symbol |k|^2), as the H1
 * seminorm of v is.  Reading: div is spectral, with the derivative
 * wavenumber kappa_d = k_d except at the Nyquist index, where kappa_d = 0
 * (the odd derivative of a real field has no Nyquist component); |k|^2
 * keeps the Nyquist wavenumber, as in A.                                */
static double dwavenum(int q, int n) { return q == n / 2 ? 0.0 : wavenum(q, n); }

/* w = div v by spectral derivatives (sum_d i kappa_d v_d^). */
void orc_spec_div(int n1, int n2, int n3, const double *v, double *w)
{
    long N = (long)n1 * n2 * n3;
    double *re = malloc(sizeof(double) * N), *im = malloc(sizeof(double) * N);
    double *ar = calloc(N, sizeof(double)), *ai = calloc(N, sizeof(double));
    for (int c = 0; c < 3; ++c) {
        for (long p = 0; p < N; ++p) { re[p] = v[c * N + p]; im[p] = 0.0; }
        orc_fft3(n1, n2, n3, re, im, -1);
        for (long i = 0; i < n1; ++i)
            for (long j = 0; j < n2; ++j)
                for (long k = 0; k < n3; ++k) {
                    long p = (i * n2 + j) * n3 + k;
                    double kap = c == 0 ? dwavenum((int)i, n1) : c == 1 ? dwavenum((int)j, n2) : dwavenum((int)k, n3);
                    ar[p] += -kap * im[p];      /* i kappa (re + i im) */
                    ai[p] += kap * re[p];
                }
    }
    orc_fft3(n1, n2, n3, ar, ai, +1);
    for (long p = 0; p < N; ++p) w[p] = ar[p] / (double)N;
    free(re); free(im); free(ar); free(ai);
}

/* g = grad u by spectral derivatives (i kappa_d u^). */
void orc_spec_grad(int n1, int n2, int n3, const double *u, double *g)
{
    long N = (long)n1 * n2 * n3;
    double *re = malloc(sizeof(double) * N), *im = malloc(sizeof(double) * N);
    double *br = malloc(sizeof(double) * N), *bi = malloc(sizeof(double) * N);
    for (long p = 0; p < N; ++p) { re[p] = u[p]; im[p] = 0.0; }
    orc_fft3(n1, n2, n3, re, im, -1);
    for (int c = 0; c < 3; ++c) {
        for (long i = 0; i < n1; ++i)
            for (long j = 0; j < n2; ++j)
                for (long k = 0; k < n3; ++k) {
                    long p = (i * n2 + j) * n3 + k;
                    double kap = c == 0 ? dwavenum((int)i, n1) : c == 1 ? dwavenum((int)j, n2) : dwavenum((int)k, n3);
                    br[p] = -kap * im[p];
                    bi[p] = kap * re[p];
                }
        orc_fft3(n1, n2, n3, br, bi, +1);
        for (long p = 0; p < N; ++p) g[c * N + p] = br[p] / (double)N;
    }
    free(re); free(im); free(br); free(bi);
}

/* Solve the real 3x3 system M x = b (Gaussian elimination with partial
 * pivoting); M is overwritten.                                          */
static void solve3(double M[3][3], double b[3], double x[3])
{
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
        if (piv != c) {
            for (int q = 0; q < 3; ++q) { double t = M[c][q]; M[c][q] = M[piv][q]; M[piv][q] = t; }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < 3; ++r) {
            double f = M[r][c] / M[c][c];
            for (int q = c; q < 3; ++q) M[r][q] -= f * M[c][q];
            b[r] -= f * b[c];
        }
    }
    for (int r = 2; r >= 0; --r) {
        double t = b[r];
        for (int q = r + 1; q < 3; ++q) t -= M[r][q] * x[q];
        x[r] = t / M[r][r];
    }
}

/* Operators on a vector field (3 consecutive fields) that act on each
 * Fourier mode's 3-vector.  L is the Hessian of R (the first variation of
 * the regularisation): per mode L = beta_v |k|^2 I + beta_w (1 + |k|^2)
 * kappa kappa^T, the second term being -grad (1 - Laplacian) div.
 *   kind 0: L
 *   kind 1: preconditioner, L^-1 on k != 0 (3x3 solve), 1/beta_v at k = 0
 *   kind 3: K = beta_v A L^-1 (3x3 solve, then beta_v |k|^2), I at k = 0;
 *           with it the reduced gradient beta_v A v + K b is beta_v A L^-1
 *           applied to the L2 gradient L v + b (the Leray-like operator of
 *           the reduced-gradient equation, Section 2.2)
 * With beta_w = 0 these are beta_v A, (beta_v A)^-1 and I.              */
void orc_reg_op(int n1, int n2, int n3, const double *in, double *out, int kind, double beta_v, double beta_w)
{
    long N = (long)n1 * n2 * n3;
    double *re[3], *im[3];
    for (int c = 0; c < 3; ++c) {
        re[c] = malloc(sizeof(double) * N);
        im[c] = malloc(sizeof(double) * N);
        for (long p = 0; p < N; ++p) { re[c][p] = in[c * N + p]; im[c][p] = 0.0; }
        orc_fft3(n1, n2, n3, re[c], im[c], -1);
    }
    for (long i = 0; i < n1; ++i)
        for (long j = 0; j < n2; ++j)
            for (long k = 0; k < n3; ++k) {
                long p = (i * n2 + j) * n3 + k;
                double kk[3] = {wavenum((int)i, n1), wavenum((int)j, n2), wavenum((int)k, n3)};
                double ka[3] = {dwavenum((int)i, n1), dwavenum((int)j, n2), dwavenum((int)k, n3)};
                double ksq = kk[0] * kk[0] + kk[1] * kk[1] + kk[2] * kk[2];
                double L[3][3];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        L[a][b] = (a == b ? beta_v * ksq : 0.0) + beta_w * (1.0 + ksq) * ka[a] * ka[b];
                double xr[3] = {re[0][p], re[1][p], re[2][p]}, xi[3] = {im[0][p], im[1][p], im[2][p]};
                double yr[3], yi[3];
                if (kind == 0) {
                    for (int a = 0; a < 3; ++a) {
                        yr[a] = L[a][0] * xr[0] + L[a][1] * xr[1] + L[a][2] * xr[2];
                        yi[a] = L[a][0] * xi[0] + L[a][1] * xi[1] + L[a][2] * xi[2];
                    }
                } else if (ksq == 0.0) {
                    double s = kind == 1 ? 1.0 / beta_v : 1.0;
                    for (int a = 0; a < 3; ++a) { yr[a] = s * xr[a]; yi[a] = s * xi[a]; }
                } else {
                    double M[3][3];
                    memcpy(M, L, sizeof(M));
                    solve3(M, xr, yr);
                    memcpy(M, L, sizeof(M));
                    solve3(M, xi, yi);
                    if (kind == 3)
                        for (int a = 0; a < 3; ++a) { yr[a] *= beta_v * ksq; yi[a] *= beta_v * ksq; }
                }
                for (int a = 0; a < 3; ++a) { re[a][p] = yr[a]; im[a][p] = yi[a]; }
            }
    for (int c = 0; c < 3; ++c) {
        orc_fft3(n1, n2, n3, re[c], im[c], +1);
        for (long p = 0; p < N; ++p) out[c * N + p] = re[c][p] / (double)N;
        free(re[c]); free(im[c]);
    }
}

/* Spectral prolongation (coarse nc -> fine nf grid) or restriction (fine
 * -> coarse): copy the Fourier modes with |k_d| < nc_d/2 on every axis,
 * zero everything else (the coarse Nyquist planes included), rescale by
 * the voxel-count ratio.  Section 5.3 uses spectral prolongation of v.  */
void orc_spectral_resample(int a1, int a2, int a3, const double *in, int b1, int b2, int b3, double *out)
{
    long Na = (long)a1 * a2 * a3, Nb = (long)b1 * b2 * b3;
    double *re = malloc(sizeof(double) * Na), *im = malloc(sizeof(double) * Na);
    double *ore = calloc(Nb, sizeof(double)), *oim = calloc(Nb, sizeof(double));
    for (long p = 0; p < Na; ++p) { re[p] = in[p]; im[p] = 0.0; }
    orc_fft3(a1, a2, a3, re, im, -1);
    int c1 = a1 < b1 ? a1 : b1, c2 = a2 < b2 ? a2 : b2, c3 = a3 < b3 ? a3 : b3;
    for (int i = 0; i < a1; ++i)
        for (int j = 0; j < a2; ++j)
            for (int k = 0; k < a3; ++k) {
                double k1 = wavenum(i, a1), k2 = wavenum(j, a2), k3 = wavenum(k, a3);
                if (fabs(k1) >= c1 / 2.0 || fabs(k2) >= c2 / 2.0 || fabs(k3) >= c3 / 2.0) continue;
                long q = ((long)wrapi((long)k1, b1) * b2 + wrapi((long)k2, b2)) * b3 + wrapi((long)k3, b3);
                long p = ((long)i * a2 + j) * a3 + k;
                ore[q] = re[p]; oim[q] = im[p];
            }
    orc_fft3(b1, b2, b3, ore, oim, +1);
    for (long q = 0; q < Nb; ++q) out[q] = ore[q] / (double)Na;
    free(re); free(im); free(ore); free(oim);
}

/* ------------------------------------------------ characteristics (RK2)
 * Section 2.2: semi-Lagrangian steps with a second-order Runge-Kutta
 * backtrace of the characteristics; the velocity is stationary, so the
 * feet are computed once per velocity.  Reading: Heun's method, with the
 * velocity at the predictor point taken by the same tricubic interpolant.
 *   forward (state):    X_f = x - dt/2 [v(x) + v(x - dt v(x))]
 *   backward (adjoint): X_b = x + dt/2 [v(x) + v(x + dt v(x))]
 * Stored as displacements from the node in index units.                  */
void orc_feet_order(int n1, int n2, int n3, int nt, int order, const double *v, double *df, double *db)
{
    long N = (long)n1 * n2 * n3;
    double dt = 1.0 / nt;
    double h[3] = {TWO_PI / n1, TWO_PI / n2, TWO_PI / n3};
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n1; ++i)
        for (long j = 0; j < n2; ++j)
            for (long k = 0; k < n3; ++k) {
                long p = (i * n2 + j) * n3 + k;
                double pf[3], pb[3];
                for (int a = 0; a < 3; ++a) {
                    pf[a] = -dt * v[a * N + p] / h[a];
                    pb[a] = dt * v[a * N + p] / h[a];
                }
                for (int a = 0; a < 3; ++a) {
                    double vf = interp_node_ord(order, n1, n2, n3, v + a * N, i, j, k, pf[0], pf[1], pf[2]);
                    double vb = interp_node_ord(order, n1, n2, n3, v + a * N, i, j, k, pb[0], pb[1], pb[2]);
                    df[a * N + p] = -0.5 * dt * (v[a * N + p] + vf) / h[a];
                    db[a * N + p] = 0.5 * dt * (v[a * N + p] + vb) / h[a];
                }
            }
}

void orc_feet(int n1, int n2, int n3, int nt, const double *v, double *df, double *db)
{
    orc_feet_order(n1, n2, n3, nt, 3, v, df, db);
}

/* Adjoint transport -d_t lambda - div(lambda v) = 0 (eq. of the adjoint)
 * written along the backward characteristic: d lambda / d tau = lambda *
 * div v.  Heun along that path gives lambda^j = c * lambda^{j+1}(X_b) with
 *   c = 1 + dt/2 (dbar + d + dt dbar d),  d = div_h v,  dbar = d(X_b).   */
void orc_adjoint_factor_order(int n1, int n2, int n3, int nt, int order, const double *v, const double *db,
                              double *c)
{
    long N = (long)n1 * n2 * n3;
    double dt = 1.0 / nt;
    double *d = malloc(sizeof(double) * N), *dbar = malloc(sizeof(double) * N);
    orc_div(n1, n2, n3, v, d);
    orc_interp_order(n1, n2, n3, order, d, db, dbar);
    for (long p = 0; p < N; ++p) c[p] = 1.0 + 0.5 * dt * (dbar[p] + d[p] + dt * dbar[p] * d[p]);
    free(d); free(dbar);
}

void orc_adjoint_factor(int n1, int n2, int n3, int nt, const double *v, const double *db, double *c)
{
    orc_adjoint_factor_order(n1, n2, n3, nt, 3, v, db, c);
}

/* ------------------------------------------------------------ context */

typedef struct orc_ctx {
    int n1, n2, n3, nt;
    long N;
    double beta, hv;        /* hv = h1 h2 h3, weight of the discrete L2 product */
    double *m0, *m1, *v;
    double *df, *db, *c;    /* feet (index-unit displacements) and adjoint factor */
    double *m, *lam;        /* state and adjoint at t_j, j = 0..nt */
    double *mt, *lamt;      /* incremental state and adjoint of the last matvec */
    double *work3a, *work3b;
    double beta_w;          /* divergence regularisation (0: K = I) */
    int interp;             /* interpolation order: 3 tricubic (default), 1 trilinear */
    int precond;            /* 0: spectral L^-1; 1: zero-velocity Hessian H0; 2: its two-level variant */
    int precond_inner;      /* inner CG iterations of the H0 preconditioner */
    int have_feet, have_state;
    /* sensitivity probe (tests only): relative perturbation of every PCG
     * matvec output, see orc_set_matvec_perturbation */
    double pert_eps;
    unsigned long long pert_seed, pert_calls;
} orc_ctx;

orc_ctx *orc_create(int n1, int n2, int n3, int nt, double beta)
{
    orc_ctx *o = calloc(1, sizeof(orc_ctx));
    o->n1 = n1; o->n2 = n2; o->n3 = n3; o->nt = nt; o->beta = beta;
    o->interp = 3;
    o->N = (long)n1 * n2 * n3;
    o->hv = (TWO_PI / n1) * (TWO_PI / n2) * (TWO_PI / n3);
    long N = o->N;
    o->m0 = calloc(N, sizeof(double)); o->m1 = calloc(N, sizeof(double));
    o->v = calloc(3 * N, sizeof(double));
    o->df = calloc(3 * N, sizeof(double)); o->db = calloc(3 * N, sizeof(double));
    o->c = calloc(N, sizeof(double));
    o->m = calloc((nt + 1) * N, sizeof(double)); o->lam = calloc((nt + 1) * N, sizeof(double));
    o->mt = calloc((nt + 1) * N, sizeof(double)); o->lamt = calloc((nt + 1) * N, sizeof(double));
    o->work3a = calloc(3 * N, sizeof(double)); o->work3b = calloc(3 * N, sizeof(double));
    return o;
}

void orc_set_beta_w(orc_ctx *o, double beta_w) { o->beta_w = beta_w; }

/* Interpolation order of every SL step of the context (3 tricubic, 1
 * trilinear); the feet of the current velocity are recomputed.            */
void orc_set_velocity(orc_ctx *o, const double *v);

void orc_set_interp(orc_ctx *o, int order)
{
    o->interp = order == 1 ? 1 : 3;
    if (o->have_feet) {
        double *v = malloc(sizeof(double) * 3 * o->N);
        memcpy(v, o->v, sizeof(double) * 3 * o->N);
        orc_set_velocity(o, v);
        free(v);
    }
}

void orc_destroy(orc_ctx *o)
{
    if (!o) return;
    free(o->m0); free(o->m1); free(o->v); free(o->df); free(o->db); free(o->c);
    free(o->m); free(o->lam); free(o->mt); free(o->lamt); free(o->work3a); free(o->work3b);
    free(o);
}

static double dot(const double *a, const double *b, long n, double w)
{
    double s = 0.0;
    for (long p = 0; p < n; ++p) s += a[p] * b[p];
    return w * s;
}

void orc_set_images(orc_ctx *o, const double *m0, const double *m1)
{
    memcpy(o->m0, m0, sizeof(double) * o->N);
    memcpy(o->m1, m1, sizeof(double) * o->N);
    o->have_state = 0;
}

void orc_set_velocity(orc_ctx *o, const double *v)
{
    memcpy(o->v, v, sizeof(double) * 3 * o->N);
    orc_feet_order(o->n1, o->n2, o->n3, o->nt, o->interp, o->v, o->df, o->db);
    orc_adjoint_factor_order(o->n1, o->n2, o->n3, o->nt, o->interp, o->v, o->db, o->c);
    o->have_feet = 1;
    o->have_state = 0;
}

/* State equation d_t m + v.grad m = 0, m(0) = m0, one SL step per dt:
 * m^{j+1}(x) = m^j(X_f).                                                 */
void orc_state(orc_ctx *o)
{
    long N = o->N;
    memcpy(o->m, o->m0, sizeof(double) * N);
    for (int j = 0; j < o->nt; ++j)
        orc_interp_order(o->n1, o->n2, o->n3, o->interp, o->m + j * N, o->df, o->m + (j + 1) * N);
    o->have_state = 1;
}

/* J = 1/2 <m(1)-m1, m(1)-m1> + beta/2 <A v, v>
 *     + beta_w/2 (<w, w> + <A w, w>), w = div v,
 * <a,b> = h1h2h3 sum a b (objective of the optimal-control problem,
 * Section 2.1; the beta_w term is the H1 norm of w).                      */
void orc_objective(orc_ctx *o, double *J, double *mis, double *reg)
{
    long N = o->N;
    if (!o->have_state) orc_state(o);
    double s = 0.0;
    const double *mN = o->m + o->nt * N;
    for (long p = 0; p < N; ++p) { double r = mN[p] - o->m1[p]; s += r * r; }
    double mm = 0.5 * o->hv * s;
    orc_spectral(o->n1, o->n2, o->n3, o->v, o->work3a, 3, 0, o->beta);
    double rr = 0.5 * dot(o->work3a, o->v, 3 * N, o->hv);
    if (o->beta_w != 0.0) {
        double *w = malloc(sizeof(double) * N), *Aw = malloc(sizeof(double) * N);
        orc_spec_div(o->n1, o->n2, o->n3, o->v, w);
        orc_spectral(o->n1, o->n2, o->n3, w, Aw, 1, 0, 1.0);
        rr += 0.5 * o->beta_w * (dot(w, w, N, o->hv) + dot(Aw, w, N, o->hv));
        free(w); free(Aw);
    }
    if (mis) *mis = mm;
    if (reg) *reg = rr;
    if (J) *J = mm + rr;
}

/* Trapezoid quadrature of int_0^1 lam grad m dt on the nt+1 time points. */
static void quadrature(orc_ctx *o, const double *lamj, double *b)
{
    long N = o->N;
    double dt = 1.0 / o->nt;
    double *gm = o->work3b;
    memset(b, 0, sizeof(double) * 3 * N);
    for (int j = 0; j <= o->nt; ++j) {
        double w = (j == 0 || j == o->nt) ? 0.5 * dt : dt;
        orc_grad(o->n1, o->n2, o->n3, o->m + j * N, gm);
        for (int a = 0; a < 3; ++a)
            for (long p = 0; p < N; ++p) b[a * N + p] += w * lamj[j * N + p] * gm[a * N + p];
    }
}

/* Adjoint solve (final condition lam(1) = m1 - m(1)) and the data part
 * b = int lam grad m dt of the reduced gradient.                         */
static void data_gradient(orc_ctx *o, double *b)
{
    long N = o->N;
    int nt = o->nt;
    if (!o->have_state) orc_state(o);
    double *lamN = o->lam + nt * N;
    for (long p = 0; p < N; ++p) lamN[p] = o->m1[p] - o->m[nt * N + p];
    for (int j = nt - 1; j >= 0; --j) {
        orc_interp_order(o->n1, o->n2, o->n3, o->interp, o->lam + (j + 1) * N, o->db, o->lam + j * N);
        for (long p = 0; p < N; ++p) o->lam[j * N + p] *= o->c[p];
    }
    quadrature(o, o->lam, b);
}

/* Both gradients at the current v: the reduced gradient of Section 2.2,
 * g = beta A v + K b (g may be NULL), and the L2 gradient of J,
 * g_l2 = L v + b (may be NULL); with beta_w = 0 both are beta A v + b.  */
static void gradients(orc_ctx *o, double *g, double *g_l2, double *J, double *mis, double *reg)
{
    long N = o->N;
    double *b = malloc(sizeof(double) * 3 * N);
    data_gradient(o, b);
    orc_objective(o, J, mis, reg);          /* leaves beta A v in work3a */
    if (o->beta_w == 0.0) {
        for (long p = 0; p < 3 * N; ++p) {
            if (g) g[p] = o->work3a[p] + b[p];
            if (g_l2) g_l2[p] = o->work3a[p] + b[p];
        }
    } else {
        double *t = malloc(sizeof(double) * 3 * N);
        if (g) {
            orc_reg_op(o->n1, o->n2, o->n3, b, t, 3, o->beta, o->beta_w);
            for (long p = 0; p < 3 * N; ++p) g[p] = o->work3a[p] + t[p];
        }
        if (g_l2) {
            orc_reg_op(o->n1, o->n2, o->n3, o->v, t, 0, o->beta, o->beta_w);
            for (long p = 0; p < 3 * N; ++p) g_l2[p] = t[p] + b[p];
        }
        free(t);
    }
    free(b);
}

/* Reduced gradient g = beta A v + K int lam grad m dt (eq. of the reduced
 * gradient).                                                              */
void orc_gradient(orc_ctx *o, double *g, double *J, double *mis, double *reg)
{
    gradients(o, g, NULL, J, mis, reg);
}

/* L2 gradient of the objective, L v + int lam grad m dt. */
void orc_gradient_l2(orc_ctx *o, double *g_l2)
{
    gradients(o, NULL, g_l2, NULL, NULL, NULL);
}

/* Data part of the Gauss-Newton Hessian matvec:
 *   incremental state  d_t mt + v.grad mt = -vt.grad m,  mt(0) = 0
 *   incremental adjoint as the adjoint, lamt(1) = -mt(1)
 *   b~ = int lamt grad m dt.
 * The source s^j = -vt.grad_h m^j is integrated by the trapezoid rule along
 * the characteristic: mt^{j+1} = I[mt^j + dt/2 s^j](X_f) + dt/2 s^{j+1}. */
static void data_matvec(orc_ctx *o, const double *vt, double *bt)
{
    long N = o->N;
    int nt = o->nt;
    double dt = 1.0 / nt;
    if (!o->have_state) orc_state(o);
    double *s = malloc(sizeof(double) * (nt + 1) * N);
    double *gm = malloc(sizeof(double) * 3 * N), *q = malloc(sizeof(double) * N);
    for (int j = 0; j <= nt; ++j) {
        orc_grad(o->n1, o->n2, o->n3, o->m + j * N, gm);
        for (long p = 0; p < N; ++p)
            s[j * N + p] = -(vt[p] * gm[p] + vt[N + p] * gm[N + p] + vt[2 * N + p] * gm[2 * N + p]);
    }
    memset(o->mt, 0, sizeof(double) * N);
    for (int j = 0; j < nt; ++j) {
        for (long p = 0; p < N; ++p) q[p] = o->mt[j * N + p] + 0.5 * dt * s[j * N + p];
        orc_interp_order(o->n1, o->n2, o->n3, o->interp, q, o->df, o->mt + (j + 1) * N);
        for (long p = 0; p < N; ++p) o->mt[(j + 1) * N + p] += 0.5 * dt * s[(j + 1) * N + p];
    }
    for (long p = 0; p < N; ++p) o->lamt[nt * N + p] = -o->mt[nt * N + p];
    for (int j = nt - 1; j >= 0; --j) {
        orc_interp_order(o->n1, o->n2, o->n3, o->interp, o->lamt + (j + 1) * N, o->db, o->lamt + j * N);
        for (long p = 0; p < N; ++p) o->lamt[j * N + p] *= o->c[p];
    }
    quadrature(o, o->lamt, bt);
    free(s); free(gm); free(q);
}

/* Gauss-Newton Hessian matvec of the reduced gradient (Section 2.2):
 * H vt = beta A vt + K b~.                                               */
void orc_matvec(orc_ctx *o, const double *vt, double *Hvt)
{
    long N = o->N;
    double *b = malloc(sizeof(double) * 3 * N);
    data_matvec(o, vt, b);
    orc_spectral(o->n1, o->n2, o->n3, vt, Hvt, 3, 0, o->beta);
    if (o->beta_w != 0.0) {
        double *t = malloc(sizeof(double) * 3 * N);
        orc_reg_op(o->n1, o->n2, o->n3, b, t, 3, o->beta, o->beta_w);
        memcpy(b, t, sizeof(double) * 3 * N);
        free(t);
    }
    for (long p = 0; p < 3 * N; ++p) Hvt[p] += b[p];
    free(b);
}

/* The same operator in its L2-symmetric form, L vt + b~ = K^-1 H vt: the
 * Hessian of J itself (equal to H when beta_w = 0).                      */
void orc_matvec_sym(orc_ctx *o, const double *vt, double *Hvt)
{
    long N = o->N;
    if (o->beta_w == 0.0) {
        orc_matvec(o, vt, Hvt);
        return;
    }
    double *b = malloc(sizeof(double) * 3 * N);
    data_matvec(o, vt, b);
    orc_reg_op(o->n1, o->n2, o->n3, vt, Hvt, 0, o->beta, o->beta_w);
    for (long p = 0; p < 3 * N; ++p) Hvt[p] += b[p];
    free(b);
}

/* Spectral preconditioner: (beta A)^-1 with the k = 0 mode mapped to
 * 1/beta; with beta_w > 0 the inverse of L (same k = 0 rule).           */
static void precond_spectral(orc_ctx *o, const double *r, double *z)
{
    if (o->beta_w == 0.0)
        orc_spectral(o->n1, o->n2, o->n3, r, z, 3, 1, o->beta);
    else
        orc_reg_op(o->n1, o->n2, o->n3, r, z, 1, o->beta, o->beta_w);
}

/* Zero-velocity Hessian preconditioner (Section 2.2 names the zero
 * velocity approximation of H as a preconditioner; its construction is in
 * a cited paper that is not at hand).  Reading: at v = 0 the state is m0
 * for all t, the incremental state is -t vt.grad m0 and the incremental
 * adjoint is constant, so the Gauss-Newton Hessian of J is
 *   H0 vt = L vt + (grad_h m0 . vt) grad_h m0,
 * a pointwise rank-one data term.  z ~ H0^-1 r by precond_inner steps of
 * CG from z = 0, preconditioned by the spectral L^-1; the k = 0 mode of L
 * is taken as beta_v (L_0), the preconditioner's own convention, so that
 * the inner operator stays definite where the data term vanishes.        */
/* Spectral L^-1 and L_0 on a given grid. */
static void grid_precond(int n1, int n2, int n3, double bv, double bw, const double *r, double *z)
{
    if (bw == 0.0) orc_spectral(n1, n2, n3, r, z, 3, 1, bv);
    else orc_reg_op(n1, n2, n3, r, z, 1, bv, bw);
}

/* L_0 = L with the k = 0 mode mapped by beta_v (the spectral
 * preconditioner's convention), which keeps L_0 + g g^T definite even when
 * the data term vanishes: y = L x + beta_v mean(x) per component.        */
static void grid_reg0(int n1, int n2, int n3, double bv, double bw, const double *x, double *y)
{
    long N = (long)n1 * n2 * n3;
    if (bw == 0.0) orc_spectral(n1, n2, n3, x, y, 3, 0, bv);
    else orc_reg_op(n1, n2, n3, x, y, 0, bv, bw);
    for (int a = 0; a < 3; ++a) {
        double mean = 0.0;
        for (long q = 0; q < N; ++q) mean += x[a * N + q];
        mean /= (double)N;
        for (long q = 0; q < N; ++q) y[a * N + q] += bv * mean;
    }
}

/* iters CG steps from z = 0 on (L_0 + g g^T) z = r over an n1 x n2 x n3
 * grid (g = grad m0 on that grid), preconditioned by the grid's spectral
 * L^-1 (= L_0^-1).                                                       */
static void h0_cg(int n1, int n2, int n3, double bv, double bw, int iters, const double *gm, const double *r,
                  double *z)
{
    long N = (long)n1 * n2 * n3, n = 3 * N;
    double w = (TWO_PI / n1) * (TWO_PI / n2) * (TWO_PI / n3);
    double *ri = malloc(sizeof(double) * n), *zi = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *Hp = malloc(sizeof(double) * n);
    memset(z, 0, sizeof(double) * n);
    memcpy(ri, r, sizeof(double) * n);
    grid_precond(n1, n2, n3, bv, bw, ri, zi);
    memcpy(p, zi, sizeof(double) * n);
    double rz = dot(ri, zi, n, w);
    for (int it = 0; it < iters && rz > 0.0; ++it) {
        grid_reg0(n1, n2, n3, bv, bw, p, Hp);
        for (long q = 0; q < N; ++q) {
            double gp = gm[q] * p[q] + gm[N + q] * p[N + q] + gm[2 * N + q] * p[2 * N + q];
            for (int a = 0; a < 3; ++a) Hp[a * N + q] += gp * gm[a * N + q];
        }
        double pHp = dot(p, Hp, n, w);
        if (!(pHp > 0.0)) break;
        double alpha = rz / pHp;
        for (long q = 0; q < n; ++q) { z[q] += alpha * p[q]; ri[q] -= alpha * Hp[q]; }
        if (it == iters - 1) break;
        grid_precond(n1, n2, n3, bv, bw, ri, zi);
        double rzn = dot(ri, zi, n, w);
        double b = rzn / rz;
        rz = rzn;
        for (long q = 0; q < n; ++q) p[q] = zi[q] + b * p[q];
    }
    free(ri); free(zi); free(p); free(Hp);
}

static void precond_h0(orc_ctx *o, const double *r, double *z)
{
    double *gm = malloc(sizeof(double) * 3 * o->N);
    orc_grad(o->n1, o->n2, o->n3, o->m0, gm);
    h0_cg(o->n1, o->n2, o->n3, o->beta, o->beta_w, o->precond_inner, gm, r, z);
    free(gm);
}

/* Two-level coarse-grid variant (Section 2.2 names it as the default and
 * defers its construction to a cited paper).  Reading: the Fourier modes
 * that a half-resolution grid represents (|k_d| < n_d/4 on every axis, the
 * band kept by spectral restriction) get the zero-velocity Hessian inverted
 * on that grid, the modes above the band get the spectral L^-1:
 *   r_c = R r,  z_c = iters CG steps on (L_0 + g_c g_c^T) z_c = r_c,
 *   z   = P z_c + L^-1 (r - P R r),
 * with R / P spectral restriction / prolongation (orc_spectral_resample),
 * g_c = grad_h of the restricted template R m0 on the coarse grid (FD8 with
 * the coarse spacing) and L^-1 the spectral preconditioner (k = 0 mode by
 * 1/beta_v; r - P R r has no k = 0 mode).                                 */
static void resample3(int a1, int a2, int a3, const double *in, int b1, int b2, int b3, double *out)
{
    long Na = (long)a1 * a2 * a3, Nb = (long)b1 * b2 * b3;
    for (int c = 0; c < 3; ++c) orc_spectral_resample(a1, a2, a3, in + c * Na, b1, b2, b3, out + c * Nb);
}

static void precond_h0_2level(orc_ctx *o, const double *r, double *z)
{
    int n1 = o->n1, n2 = o->n2, n3 = o->n3, c1 = n1 / 2, c2 = n2 / 2, c3 = n3 / 2;
    long N = o->N, Nc = (long)c1 * c2 * c3;
    double *m0c = malloc(sizeof(double) * Nc), *gc = malloc(sizeof(double) * 3 * Nc);
    double *rc = malloc(sizeof(double) * 3 * Nc), *zc = malloc(sizeof(double) * 3 * Nc);
    double *lowr = malloc(sizeof(double) * 3 * N), *zl = malloc(sizeof(double) * 3 * N);
    orc_spectral_resample(n1, n2, n3, o->m0, c1, c2, c3, m0c);
    orc_grad(c1, c2, c3, m0c, gc);
    resample3(n1, n2, n3, r, c1, c2, c3, rc);                 /* R r */
    h0_cg(c1, c2, c3, o->beta, o->beta_w, o->precond_inner, gc, rc, zc);
    resample3(c1, c2, c3, rc, n1, n2, n3, lowr);             /* P R r */
    for (long q = 0; q < 3 * N; ++q) lowr[q] = r[q] - lowr[q];   /* r - P R r */
    grid_precond(n1, n2, n3, o->beta, o->beta_w, lowr, z);   /* L^-1 of the high band */
    resample3(c1, c2, c3, zc, n1, n2, n3, zl);               /* P z_c */
    for (long q = 0; q < 3 * N; ++q) z[q] += zl[q];
    free(m0c); free(gc); free(rc); free(zc); free(lowr); free(zl);
}

void orc_set_precond(orc_ctx *o, int kind, int inner)
{
    o->precond = kind;
    o->precond_inner = inner;
}

/* The solver's preconditioner: spectral, or the H0 inner solve.           */
void orc_precond(orc_ctx *o, const double *r, double *z)
{
    if (o->precond == 1)
        precond_h0(o, r, z);
    else if (o->precond == 2)
        precond_h0_2level(o, r, z);
    else
        precond_spectral(o, r, z);
}

/* Jacobian determinant J = det grad y of the map y with m(x, 1) =
 * m0(y(x)) (Section 3.4, the bounds [J_min, 1/J_min] of the parameter
 * search).  Reading (the paper does not say how J is computed): grad y
 * transported by v gives d_t J + v.grad J = -(div v) J, J(x, 0) = 1,
 * solved with the state's semi-Lagrangian step and Heun's rule for the
 * source along the characteristic from X_f (time t_j) to x (time t_j+1):
 *   J^{j+1}(x) = J^j(X_f) (1 - dt/2 (d_f + d - dt d_f d)),
 * d = div_h v at x and d_f = d interpolated at X_f.                      */
void orc_jacobian_det(orc_ctx *o, double *J)
{
    long N = o->N;
    double dt = 1.0 / o->nt;
    double *d = malloc(sizeof(double) * N), *dfo = malloc(sizeof(double) * N);
    double *f = malloc(sizeof(double) * N), *cur = malloc(sizeof(double) * N);
    orc_div(o->n1, o->n2, o->n3, o->v, d);
    orc_interp_order(o->n1, o->n2, o->n3, o->interp, d, o->df, dfo);
    for (long p = 0; p < N; ++p) {
        f[p] = 1.0 - 0.5 * dt * (dfo[p] + d[p] - dt * dfo[p] * d[p]);
        cur[p] = 1.0;
    }
    for (int j = 0; j < o->nt; ++j) {
        orc_interp_order(o->n1, o->n2, o->n3, o->interp, cur, o->df, J);
        for (long p = 0; p < N; ++p) J[p] *= f[p];
        memcpy(cur, J, sizeof(double) * N);
    }
    free(d); free(dfo); free(f); free(cur);
}

/* Read back an internal field: which = 0 state m^j, 1 adjoint lam^j,
 * 2 incremental state mt^j, 3 incremental adjoint lamt^j, 4 forward feet
 * (3N), 5 backward feet (3N), 6 adjoint factor c.                         */
void orc_get_field(orc_ctx *o, int which, int j, double *out)
{
    long N = o->N;
    switch (which) {
    case 0: memcpy(out, o->m + j * N, sizeof(double) * N); break;
    case 1: memcpy(out, o->lam + j * N, sizeof(double) * N); break;
    case 2: memcpy(out, o->mt + j * N, sizeof(double) * N); break;
    case 3: memcpy(out, o->lamt + j * N, sizeof(double) * N); break;
    case 4: memcpy(out, o->df, sizeof(double) * 3 * N); break;
    case 5: memcpy(out, o->db, sizeof(double) * 3 * N); break;
    case 6: memcpy(out, o->c, sizeof(double) * N); break;
    default: break;
    }
}

/* -------------------------------------------------------- PCG and GN
 * Section 2.2 (Gauss-Newton-Krylov solver): v_{k+1} = v_k + alpha_k vt_k,
 * H vt_k = -g_k solved by matrix-free PCG, Armijo line search.  Readings:
 *  - PCG from x0 = 0, preconditioner (beta A)^-1 (k = 0 mode 1/beta), stop
 *    when ||r_i|| <= eta ||r_0|| or after max_pcg iterations, or on
 *    p.Hp <= 0 (then return x, or z_0 if that happens at i = 0);
 *  - forcing eta = min(0.5, sqrt(||g|| / g_ref));
 *  - Armijo: alpha = 1, halve while J(v + alpha vt) > J(v) + 1e-4 alpha
 *    <g, vt>, at most 10 trials;
 *  - g_ref = ||g(v = 0)||, stop when ||g|| <= gtol g_ref.
 *  - with the H0 preconditioner (an inner Krylov solve, not a fixed linear
 *    operator) PCG is flexible: beta = <r_new, z_new - z_old> / <r, z>.
 *  - beta_w > 0: g and H are the reduced gradient and Hessian, K times the
 *    L2 gradient and Hessian of J.  PCG runs on the L2-symmetric form
 *    (L + B) x = -g_l2 with the preconditioner L^-1, which is PCG on
 *    H x = -g with K as a left preconditioner: the same Newton step; its
 *    residual test is on the symmetric system.  Armijo uses <g_l2, vt>,
 *    the directional derivative of J; the stopping test and the forcing
 *    term use ||g||.
 * A forced run (forced_pcg / forced_alpha non-NULL) takes exactly the given
 * PCG iteration counts and step lengths instead of testing them.
 * log is [max_outer + 1][8]: k, J, mismatch, reg, ||g||, pcg iterations,
 * alpha, line-search trials (the last row is the final iterate).         */
/* Sensitivity probe for the tests (not part of the method): with eps > 0,
 * every matvec inside PCG is multiplied elementwise by (1 + eps xi), xi
 * uniform in [-1, 1) from the splitmix64 hash (Steele, Lea and Flood 2014)
 * of (seed, call number, index).  eps ~ 1e-6 mimics the relative rounding
 * error of a single-precision matvec; eps = 0 switches it off.           */
static unsigned long long splitmix64(unsigned long long x)
{
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

void orc_set_matvec_perturbation(orc_ctx *o, double eps, unsigned long long seed)
{
    o->pert_eps = eps;
    o->pert_seed = seed;
    o->pert_calls = 0;
}

static void perturb(orc_ctx *o, double *y, long n)
{
    if (o->pert_eps == 0.0) return;
    unsigned long long key = splitmix64(o->pert_seed ^ splitmix64(o->pert_calls++));
    for (long q = 0; q < n; ++q) {
        double xi = (double)(splitmix64(key + (unsigned long long)q) >> 11) * 0x1.0p-53 * 2.0 - 1.0;
        y[q] *= 1.0 + o->pert_eps * xi;
    }
}

int orc_pcg(orc_ctx *o, const double *rhs, double *x, int max_pcg, double eta, int forced_iters, int *iters_out)
{
    long n = 3 * o->N;
    double w = o->hv;
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *Hp = malloc(sizeof(double) * n);
    memset(x, 0, sizeof(double) * n);
    memcpy(r, rhs, sizeof(double) * n);
    orc_precond(o, r, z);
    memcpy(p, z, sizeof(double) * n);
    double rz = dot(r, z, n, w);
    double r0 = sqrt(dot(r, r, n, w));
    int limit = forced_iters >= 0 ? forced_iters : max_pcg;
    int it = 0, negcurv = 0;
    while (it < limit) {
        orc_matvec_sym(o, p, Hp);
        perturb(o, Hp, n);
        double pHp = dot(p, Hp, n, w);
        if (pHp <= 0.0) {
            negcurv = 1;
            if (it == 0) memcpy(x, z, sizeof(double) * n);
            break;
        }
        double alpha = rz / pHp;
        for (long q = 0; q < n; ++q) { x[q] += alpha * p[q]; r[q] -= alpha * Hp[q]; }
        ++it;
        double rn = sqrt(dot(r, r, n, w));
        if (forced_iters < 0 && rn <= eta * r0) break;
        if (it >= limit) break;
        double rz_old = 0.0;
        if (o->precond != 0) rz_old = dot(r, z, n, w);
        orc_precond(o, r, z);
        double rz_new = dot(r, z, n, w);
        double bt = (rz_new - rz_old) / rz;
        rz = rz_new;
        for (long q = 0; q < n; ++q) p[q] = z[q] + bt * p[q];
    }
    if (iters_out) *iters_out = it;
    free(r); free(z); free(p); free(Hp);
    return negcurv;
}

int orc_solve(orc_ctx *o, int max_outer, int max_pcg, double gtol,
              const int *forced_pcg, const double *forced_alpha,
              double *log, int *n_outer, double *gref_out)
{
    long n = 3 * o->N;
    double w = o->hv;
    double *v = malloc(sizeof(double) * n), *g = malloc(sizeof(double) * n);
    double *gl = malloc(sizeof(double) * n);
    double *vt = malloc(sizeof(double) * n), *rhs = malloc(sizeof(double) * n);
    double *vtrial = malloc(sizeof(double) * n);
    memcpy(v, o->v, sizeof(double) * n);

    /* g_ref at v = 0 */
    memset(vtrial, 0, sizeof(double) * n);
    orc_set_velocity(o, vtrial);
    orc_gradient(o, g, NULL, NULL, NULL);
    double gref = sqrt(dot(g, g, n, w));
    if (gref_out) *gref_out = gref;
    orc_set_velocity(o, v);

    int status = 1, k = 0;
    double J, mis, reg;
    for (k = 0; k < max_outer; ++k) {
        gradients(o, g, gl, &J, &mis, &reg);
        double gn = sqrt(dot(g, g, n, w));
        double *row = log ? log + 8 * k : NULL;
        if (row) { row[0] = k; row[1] = J; row[2] = mis; row[3] = reg; row[4] = gn; row[5] = 0; row[6] = 0; row[7] = 0; }
        if (!forced_pcg && gn <= gtol * gref) { status = 0; break; }
        double eta = sqrt(gn / gref);
        if (eta > 0.5) eta = 0.5;
        for (long q = 0; q < n; ++q) rhs[q] = -gl[q];
        int its = 0;
        orc_pcg(o, rhs, vt, max_pcg, eta, forced_pcg ? forced_pcg[k] : -1, &its);
        double gvt = dot(gl, vt, n, w);
        double alpha = 1.0;
        int trials = 0, ok = 0;
        if (forced_alpha) {
            alpha = forced_alpha[k];
            ok = 1;
        } else {
            for (trials = 1; trials <= 10; ++trials) {
                for (long q = 0; q < n; ++q) vtrial[q] = v[q] + alpha * vt[q];
                orc_set_velocity(o, vtrial);
                double Jt;
                orc_objective(o, &Jt, NULL, NULL);
                if (Jt <= J + 1e-4 * alpha * gvt) { ok = 1; break; }
                alpha *= 0.5;
            }
        }
        if (!forced_alpha && !ok) trials = 10;   /* every one of the 10 trials failed */
        if (row) { row[5] = its; row[6] = ok ? alpha : 0.0; row[7] = trials; }
        if (!ok) {
            orc_set_velocity(o, v);
            status = 2;
            ++k;
            break;
        }
        if (forced_alpha) {
            for (long q = 0; q < n; ++q) v[q] += alpha * vt[q];
            orc_set_velocity(o, v);
        } else {
            /* the accepted trial v + alpha vt is already loaded */
            memcpy(v, vtrial, sizeof(double) * n);
        }
    }
    if (status != 0) {
        orc_gradient(o, g, &J, &mis, &reg);
        double gn = sqrt(dot(g, g, n, w));
        if (log) {
            double *row = log + 8 * k;
            row[0] = k; row[1] = J; row[2] = mis; row[3] = reg; row[4] = gn; row[5] = 0; row[6] = 0; row[7] = 0;
        }
        if (status == 1 && gn <= gtol * gref) status = 0;
    }
    if (n_outer) *n_outer = k;
    free(v); free(g); free(gl); free(vt); free(rhs); free(vtrial);
    return status;
}

/* ------------------------------------------ parameter identification
 * Section 3.4.  A trial sets (beta_v, beta_w), runs the GN solve from the
 * current velocity (the previous trial's result) and tests the bounds
 * J_min <= det grad y <= 1/J_min.  Each trial appends a log row: beta_v,
 * beta_w, min J, max J, valid, GN iterations, PCG iterations, status,
 * final mismatch, 0.                                                     */
void orc_set_beta(orc_ctx *o, double beta_v, double beta_w)
{
    o->beta = beta_v;
    o->beta_w = beta_w;
}

typedef struct {
    int max_outer, max_pcg;
    double gtol, jmin;
    double *log;
    int max_rows, rows;
    double *best;           /* velocity of the last valid trial (3N) */
    int last_ok;
} search_run;

static int search_trial(orc_ctx *o, search_run *sr, double bv, double bw)
{
    orc_set_beta(o, bv, bw);
    double *log = malloc(sizeof(double) * 8 * (sr->max_outer + 1));
    int nout = 0;
    double gref;
    int st = orc_solve(o, sr->max_outer, sr->max_pcg, sr->gtol, NULL, NULL, log, &nout, &gref);
    int pcg = 0;
    for (int k = 0; k < nout; ++k) pcg += (int)log[8 * k + 5];
    double mis = log[8 * nout + 2];
    free(log);
    double *J = malloc(sizeof(double) * o->N);
    orc_jacobian_det(o, J);
    double lo = J[0], hi = J[0];
    for (long p = 1; p < o->N; ++p) {
        if (J[p] < lo) lo = J[p];
        if (J[p] > hi) hi = J[p];
    }
    free(J);
    int ok = isfinite(lo) && isfinite(hi) && lo >= sr->jmin && hi <= 1.0 / sr->jmin;
    if (ok && sr->best) memcpy(sr->best, o->v, sizeof(double) * 3 * o->N);
    sr->last_ok = ok;
    if (sr->rows < sr->max_rows) {
        double *row = sr->log + 10 * sr->rows;
        row[0] = bv; row[1] = bw; row[2] = lo; row[3] = hi; row[4] = ok;
        row[5] = nout; row[6] = pcg; row[7] = st; row[8] = mis; row[9] = 0.0;
    }
    sr->rows++;
    return ok;
}

/* Parameter search: (i) beta_w = beta_w_max; beta_v = beta_v_max and then
 * one decade smaller per trial while the bounds hold (never below
 * beta_v_min); after the first breach, bisection between the last valid
 * value and the breaching one until the next midpoint would move beta_v by
 * less than rel_change of the valid value; beta_v* is the last valid value.
 * (ii) beta_v = beta_v*; beta_w one decade smaller per trial from
 * beta_w_max while the bounds hold (never below beta_w_min); beta_w* is the
 * last valid value.  Decade steps below a minimum are compared with a
 * relative slack of 1e-9.  The context ends at the solution of the last
 * valid trial, the one for (beta_v*, beta_w*), restored when a later trial
 * breached the bounds.  Returns 0, or 3 when beta_v_max already breaches
 * the bounds.                                                             */
int orc_param_search(orc_ctx *o, double jmin, double bv_max, double bv_min, double bw_max, double bw_min,
                     double rel_change, int search_bw, int max_outer, int max_pcg, double gtol,
                     double *log, int max_rows, int *n_rows, double *bv_star, double *bw_star)
{
    double *best = malloc(sizeof(double) * 3 * o->N);
    search_run sr = {max_outer, max_pcg, gtol, jmin, log, max_rows, 0, best, 0};
    double valid_bv = -1.0, breach_bv = -1.0;
    double bv = bv_max;
    while (1) {
        if (!search_trial(o, &sr, bv, bw_max)) { breach_bv = bv; break; }
        valid_bv = bv;
        if (bv / 10.0 < bv_min * (1.0 - 1e-9)) break;
        bv = bv / 10.0;
    }
    int status = 0;
    if (valid_bv < 0.0) {
        status = 3;
        valid_bv = bv_max;
    } else if (breach_bv > 0.0) {
        while (1) {
            double mid = 0.5 * (valid_bv + breach_bv);
            if (valid_bv - mid < rel_change * valid_bv) break;
            if (search_trial(o, &sr, mid, bw_max)) valid_bv = mid;
            else breach_bv = mid;
        }
    }
    double bw_valid = bw_max;
    if (status == 0 && search_bw && bw_max > 0.0) {
        double bw = bw_max;
        while (bw / 10.0 >= bw_min * (1.0 - 1e-9)) {
            bw = bw / 10.0;
            if (!search_trial(o, &sr, valid_bv, bw)) break;
            bw_valid = bw;
        }
    }
    if (status == 0 && !sr.last_ok) {
        orc_set_velocity(o, best);
        orc_set_beta(o, valid_bv, bw_valid);
    }
    free(best);
    if (n_rows) *n_rows = sr.rows;
    if (bv_star) *bv_star = valid_bv;
    if (bw_star) *bw_star = bw_valid;
    return status;
}

/* Parameter continuation toward (bv_target, bw_target): beta_w = bw_max
 * with beta_v = bv_max, bv_max/10, ... down to 10^ceil(log10 bv_target),
 * then bv_target; then beta_v = bv_target with beta_w one decade smaller
 * per solve from bw_max down to bw_target.  No bounds test (jmin = 0 in
 * the valid column).                                                     */
int orc_param_continuation(orc_ctx *o, double bv_max, double bw_max, double bv_target, double bw_target,
                           int max_outer, int max_pcg, double gtol, double *log, int max_rows, int *n_rows)
{
    search_run sr = {max_outer, max_pcg, gtol, 0.0, log, max_rows, 0, NULL, 0};
    double stop = pow(10.0, ceil(log10(bv_target)));
    double bv = bv_max;
    while (bv > stop * (1.0 + 1e-9)) {
        search_trial(o, &sr, bv, bw_max);
        bv = bv / 10.0;
    }
    search_trial(o, &sr, bv, bw_max);
    if (fabs(bv - bv_target) > 1e-9 * bv_target) search_trial(o, &sr, bv_target, bw_max);
    if (bw_target <= 0.0) {
        if (bw_max > 0.0) search_trial(o, &sr, bv_target, 0.0);
    } else {
        double bw = bw_max;
        while (bw > bw_target * (1.0 + 1e-9)) {
            bw = bw / 10.0 > bw_target ? bw / 10.0 : bw_target;
            search_trial(o, &sr, bv_target, bw);
        }
    }
    if (n_rows) *n_rows = sr.rows;
    return 0;
}

void orc_get_velocity(orc_ctx *o, double *v) { memcpy(v, o->v, sizeof(double) * 3 * o->N); }

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
