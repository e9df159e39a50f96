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

/* out(x_ijk) = I[u](x_ijk + d_ijk), d in index units (3 arrays). */
void orc_interp(int n1, int n2, int n3, const double *u, const double *d, double *out)
{
    long N = (long)n1 * n2 * n3;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n1; ++i)
        for (long j = 0; j < n2; ++j)
            for (long k = 0; k < n3; ++k) {
                long p = (i * n2 + j) * n3 + k;
                out[p] = interp_node(n1, n2, n3, u, i, j, k, d[p], d[N + p], d[2 * N + p]);
            }
}

/* Value of I[u] at an arbitrary point p (index units, any real). */
double orc_interp_point(int n1, int n2, int n3, const double *u, double p1, double p2, double p3)
{
    return interp_node(n1, n2, n3, u, 0, 0, 0, p1, p2, p3);
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

/* In-place unscaled 3D DFT of a complex array (re, im) with sign +-1. */
void orc_fft3(int n1, int n2, int n3, double *re, double *im, int sign)
{
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
void orc_feet(int n1, int n2, int n3, int nt, const double *v, double *df, double *db)
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
                    double vf = interp_node(n1, n2, n3, v + a * N, i, j, k, pf[0], pf[1], pf[2]);
                    double vb = interp_node(n1, n2, n3, v + a * N, i, j, k, pb[0], pb[1], pb[2]);
                    df[a * N + p] = -0.5 * dt * (v[a * N + p] + vf) / h[a];
                    db[a * N + p] = 0.5 * dt * (v[a * N + p] + vb) / h[a];
                }
            }
}

/* Adjoint transport -d_t lambda - div(lambda v) = 0 (eq. of the adjoint)
 * written along the backward characteristic: d lambda / d tau = lambda *
 * div v.  Heun along that path gives lambda^j = c * lambda^{j+1}(X_b) with
 *   c = 1 + dt/2 (dbar + d + dt dbar d),  d = div_h v,  dbar = d(X_b).   */
void orc_adjoint_factor(int n1, int n2, int n3, int nt, const double *v, const double *db, double *c)
{
    long N = (long)n1 * n2 * n3;
    double dt = 1.0 / nt;
    double *d = malloc(sizeof(double) * N), *dbar = malloc(sizeof(double) * N);
    orc_div(n1, n2, n3, v, d);
    orc_interp(n1, n2, n3, d, db, dbar);
    for (long p = 0; p < N; ++p) c[p] = 1.0 + 0.5 * dt * (dbar[p] + d[p] + dt * dbar[p] * d[p]);
    free(d); free(dbar);
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
    int have_feet, have_state;
} orc_ctx;

orc_ctx *orc_create(int n1, int n2, int n3, int nt, double beta)
{
    orc_ctx *o = calloc(1, sizeof(orc_ctx));
    o->n1 = n1; o->n2 = n2; o->n3 = n3; o->nt = nt; o->beta = beta;
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
    orc_feet(o->n1, o->n2, o->n3, o->nt, o->v, o->df, o->db);
    orc_adjoint_factor(o->n1, o->n2, o->n3, o->nt, o->v, o->db, o->c);
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
        orc_interp(o->n1, o->n2, o->n3, o->m + j * N, o->df, o->m + (j + 1) * N);
    o->have_state = 1;
}

/* J = 1/2 <m(1)-m1, m(1)-m1> + beta/2 <A v, v>, <a,b> = h1h2h3 sum a b
 * (objective of the optimal-control problem, Section 2.1).              */
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

/* Reduced gradient g = beta A v + int lam grad m dt (eq. of the reduced
 * gradient, K = I), adjoint final condition lam(1) = m1 - m(1).         */
void orc_gradient(orc_ctx *o, double *g, double *J, double *mis, double *reg)
{
    long N = o->N;
    int nt = o->nt;
    if (!o->have_state) orc_state(o);
    double *lamN = o->lam + nt * N;
    for (long p = 0; p < N; ++p) lamN[p] = o->m1[p] - o->m[nt * N + p];
    for (int j = nt - 1; j >= 0; --j) {
        orc_interp(o->n1, o->n2, o->n3, o->lam + (j + 1) * N, o->db, o->lam + j * N);
        for (long p = 0; p < N; ++p) o->lam[j * N + p] *= o->c[p];
    }
    double *b = malloc(sizeof(double) * 3 * N);
    quadrature(o, o->lam, b);
    orc_objective(o, J, mis, reg);          /* leaves beta A v in work3a */
    for (long p = 0; p < 3 * N; ++p) g[p] = o->work3a[p] + b[p];
    free(b);
}

/* Gauss-Newton Hessian matvec (eq. of the matvec, K = I):
 *   incremental state  d_t mt + v.grad mt = -vt.grad m,  mt(0) = 0
 *   incremental adjoint as the adjoint, lamt(1) = -mt(1)
 *   H vt = beta A vt + int lamt grad m dt.
 * The source s^j = -vt.grad_h m^j is integrated by the trapezoid rule along
 * the characteristic: mt^{j+1} = I[mt^j + dt/2 s^j](X_f) + dt/2 s^{j+1}. */
void orc_matvec(orc_ctx *o, const double *vt, double *Hvt)
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
        orc_interp(o->n1, o->n2, o->n3, q, o->df, o->mt + (j + 1) * N);
        for (long p = 0; p < N; ++p) o->mt[(j + 1) * N + p] += 0.5 * dt * s[(j + 1) * N + p];
    }
    for (long p = 0; p < N; ++p) o->lamt[nt * N + p] = -o->mt[nt * N + p];
    for (int j = nt - 1; j >= 0; --j) {
        orc_interp(o->n1, o->n2, o->n3, o->lamt + (j + 1) * N, o->db, o->lamt + j * N);
        for (long p = 0; p < N; ++p) o->lamt[j * N + p] *= o->c[p];
    }
    double *b = malloc(sizeof(double) * 3 * N);
    quadrature(o, o->lamt, b);
    orc_spectral(o->n1, o->n2, o->n3, vt, Hvt, 3, 0, o->beta);
    for (long p = 0; p < 3 * N; ++p) Hvt[p] += b[p];
    free(b); free(s); free(gm); free(q);
}

void orc_precond(orc_ctx *o, const double *r, double *z)
{
    orc_spectral(o->n1, o->n2, o->n3, r, z, 3, 1, o->beta);
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
 * A forced run (forced_pcg / forced_alpha non-NULL) takes exactly the given
 * PCG iteration counts and step lengths instead of testing them.
 * log is [max_outer + 1][8]: k, J, mismatch, reg, ||g||, pcg iterations,
 * alpha, line-search trials (the last row is the final iterate).         */
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
        orc_matvec(o, p, Hp);
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
        orc_precond(o, r, z);
        double rz_new = dot(r, z, n, w);
        double bt = rz_new / rz;
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
        orc_gradient(o, g, &J, &mis, &reg);
        double gn = sqrt(dot(g, g, n, w));
        double *row = log ? log + 8 * k : NULL;
        if (row) { row[0] = k; row[1] = J; row[2] = mis; row[3] = reg; row[4] = gn; row[5] = 0; row[6] = 0; row[7] = 0; }
        if (!forced_pcg && gn <= gtol * gref) { status = 0; break; }
        double eta = sqrt(gn / gref);
        if (eta > 0.5) eta = 0.5;
        for (long q = 0; q < n; ++q) rhs[q] = -g[q];
        int its = 0;
        orc_pcg(o, rhs, vt, max_pcg, eta, forced_pcg ? forced_pcg[k] : -1, &its);
        double gvt = dot(g, vt, n, w);
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
    free(v); free(g); free(vt); free(rhs); free(vtrial);
    return status;
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
