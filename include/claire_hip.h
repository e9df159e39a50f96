/*
 * claire_hip.h -- C ABI of the MI355X (gfx950) implementation of the
 * Gauss-Newton-Krylov hot path of stationary-velocity diffeomorphic image
 * registration (Himthani et al., CLAIRE, arXiv 2209.08189).
 *
 * Problem (Section 2.1, optimal-control problem): given a template image m0
 * and a reference image m1 on the periodic domain [0, 2pi)^3, find a
 * stationary velocity v minimising
 *     1/2 ||m(1) - m1||^2 + beta_v/2 <A v, v> + beta_w/2 (<w, w> + <A w, w>),
 * where m solves the transport equation d_t m + v . grad m = 0, m(0) = m0,
 * A = -Laplacian (H1 seminorm of v) and w = div v, penalised by its H1 norm
 * (Section 2.1; beta_w = 0 drops the term).  The regularisation's Hessian is
 * L = beta_v A + beta_w (-grad)(1 + A) div; the Leray-like operator of the
 * reduced gradient (Section 2.2) is K = beta_v A L^-1, the identity when
 * beta_w = 0.  Spectral first derivatives (div, and grad in L) use
 * wavenumber 0 at the Nyquist index; A keeps it.
 *
 * Conventions that hold for every entry point:
 *   - Grid: n1 x n2 x n3 nodes x_i = 2 pi i / n, each n_d a power of two,
 *     16 <= n_d <= 1024.  Fields are C order [x1][x2][x3] (x3 fastest);
 *     vector fields are three such arrays back to back ([3][n1][n2][n3]).
 *   - Every buffer argument is a DEVICE pointer owned by the caller.  The
 *     library copies inputs at the set_* calls and never keeps a caller
 *     pointer.  Input and output buffers of one call must not overlap
 *     (CL_ERR_ALIAS).  All library memory is allocated in cl_create.
 *   - All device work is enqueued on the stream given in cl_options (NULL =
 *     the default stream).  Calls returning host scalars synchronise that
 *     stream; cl_hessian_matvec, cl_precond_apply, cl_set_* and the field
 *     accessors only enqueue.
 *   - Return value: CL_OK (0), a negative error code, or a positive
 *     non-fatal status.  No exception, abort or exit crosses this boundary;
 *     the message of the last error of a context is cl_last_error(ctx).
 *   - A context is not thread safe: one context per host thread.
 */
#ifndef CLAIRE_HIP_H
#define CLAIRE_HIP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CL_OPTIONS_VERSION 5

typedef struct cl_ctx cl_ctx;

/* Storage precision of the scalar fields (images, state, adjoint and
 * incremental fields).  Arithmetic is FP32; Krylov dot products, norms and
 * the objective are reduced in FP64 whatever the storage. */
typedef enum { CL_F32 = 0, CL_BF16 = 1, CL_F16 = 2 } cl_dtype;

enum {
    CL_OK = 0,
    CL_ERR_ARG = -1,          /* NULL pointer, bad option value */
    CL_ERR_SHAPE = -2,        /* n_d not a power of two in [16, 1024] */
    CL_ERR_DTYPE = -3,        /* unsupported cl_dtype */
    CL_ERR_OOM = -4,          /* device allocation failed or workspace cap exceeded */
    CL_ERR_HIP = -5,          /* a HIP runtime call failed */
    CL_ERR_NONFINITE = -6,    /* NaN or Inf found in an input */
    CL_ERR_UNSUPPORTED = -7,  /* option combination the library does not implement */
    CL_ERR_STATE = -8,        /* call order violated (e.g. gradient before set_images) */
    CL_ERR_ALIAS = -9,        /* input and output buffers overlap */
    CL_STATUS_MAXIT = 1,      /* solve stopped at max_outer */
    CL_STATUS_LINESEARCH_FAIL = 2, /* Armijo found no step; last accepted v kept */
    CL_STATUS_BOUNDS = 3      /* parameter search: beta_v_max already breaches the J bounds */
};

typedef struct {
    int struct_version;       /* must be CL_OPTIONS_VERSION */
    int nt;                   /* semi-Lagrangian time steps, >= 1 (default 4) */
    double beta_v;            /* H1-seminorm regularisation weight, > 0 (default 5e-4) */
    double beta_w;            /* H1-norm weight of div v, >= 0 (default 0: K = I) */
    double gtol;              /* stop when ||g|| <= gtol ||g(v=0)|| (default 1e-2) */
    int max_outer;            /* Gauss-Newton iteration limit (default 50) */
    int max_pcg;              /* PCG iteration limit per GN step (default 10) */
    int forcing;              /* 1: eta = min(0.5, sqrt(||g||/||g(0)||)); 0: eta = eta_fixed */
    double eta_fixed;
    int storage_state;        /* cl_dtype of m0, m1 and the state m^j (default CL_F32) */
    int storage_adjoint;      /* cl_dtype of the adjoint and incremental fields (default CL_F32) */
    void *stream;             /* hipStream_t; NULL = default stream */
    unsigned long long workspace_cap_bytes; /* device memory the context may take: when the full layout
                                                exceeds it (0: exceeds 15/16 of the free device memory), the
                                                lean layout is used (see cl_layout); cl_create fails with
                                                CL_ERR_OOM when a nonzero cap is below even that */
    int precond;              /* CL_PRECOND_SPECTRAL (default), CL_PRECOND_H0 or CL_PRECOND_H0_2LEVEL */
    int precond_inner;        /* inner CG iterations of the H0 preconditioners, 1..100 (default 5) */
    int interp_order;         /* interpolation of every SL step: 3 tricubic Lagrange (default),
                                 1 trilinear (the paper's choice above 256^3, Section 3.3) */
    int overlap_spectral;     /* 1: cl_hessian_matvec computes its beta_v A vt term on a side stream
                                 that the context owns (default priority), beside the transport
                                 sweeps, and joins it to `stream` before the term is used, so the
                                 call keeps the semantics of one stream; results are bitwise those
                                 of 0.  0: one stream (default) */
    int fault_flip_direction; /* failure injection for tests of the line-search failure path: 1 makes
                                 cl_solve step along -vt (an ascent direction), so every Armijo trial
                                 fails and the solve returns CL_STATUS_LINESEARCH_FAIL with the last
                                 accepted v kept.  0: off (default) */
} cl_options;

/* Preconditioners of the GN system (Section 2.2).
 *   CL_PRECOND_SPECTRAL: L^-1, i.e. (beta_v A)^-1 (k = 0 -> 1/beta_v) when
 *     beta_w = 0; one FFT pair.
 *   CL_PRECOND_H0: the zero-velocity approximation of the Hessian.  At
 *     v = 0 the Gauss-Newton Hessian of J is H0 vt = L vt + (grad_h m0 .
 *     vt) grad_h m0 (state m0 at all times, incremental adjoint constant);
 *     z ~ H0^-1 r by precond_inner steps of CG from z = 0 preconditioned
 *     by L^-1, at full resolution, with the k = 0 mode of L taken as beta_v
 *     (the preconditioner's convention) so the inner operator stays
 *     definite where the data term vanishes.  The outer PCG is then flexible
 *     (beta = <r_new, z_new - z_old> / <r, z>).  Needs the full memory
 *     layout (stored grad_h m^j) and six more vector fields of workspace;
 *     cl_create returns CL_ERR_UNSUPPORTED in the lean layout.
 *   CL_PRECOND_H0_2LEVEL: the two-level coarse-grid variant that Section
 *     2.2 names as the default.  The Fourier band a half-resolution grid
 *     represents (|k_d| < n_d / 4) gets H0 inverted on that grid by
 *     precond_inner CG steps (H0 of the spectrally restricted template,
 *     FD8 with the coarse spacing), the modes above it get L^-1:
 *     z = P z_c + L^-1 (r - P R r), z_c ~ H0_c^-1 R r, with R / P spectral
 *     restriction / prolongation.  Flexible outer PCG as for CL_PRECOND_H0.
 *     Needs n_d >= 32 (CL_ERR_SHAPE) and the full layout. */
enum { CL_PRECOND_SPECTRAL = 0, CL_PRECOND_H0 = 1, CL_PRECOND_H0_2LEVEL = 2 };

typedef struct {
    int status;               /* CL_OK (converged), CL_STATUS_MAXIT or CL_STATUS_LINESEARCH_FAIL */
    int outer_iters;          /* GN steps taken */
    int pcg_iters_total;
    int linesearch_trials;    /* objective evaluations in the line searches */
    double J0, J;             /* objective at the start and at the final v */
    double mismatch, reg;     /* parts of the final J */
    double gnorm0, gnorm;     /* ||g|| at the start and at the final v */
    double gref;              /* ||g(v = 0)||, the reference of the stopping test */
    double ms;                /* wall time of the solve */
} cl_solve_report;

/* Fill *opt with the defaults listed above. */
void cl_default_options(cl_options *opt);

/* Device bytes cl_create would allocate for this grid and options (host-only query; with
 * workspace_cap_bytes = 0 it reports the full layout). */
int cl_query_workspace(int n1, int n2, int n3, const cl_options *opt, unsigned long long *bytes);

/* Create a context on the current HIP device; allocates all workspace. */
int cl_create(cl_ctx **out, int n1, int n2, int n3, const cl_options *opt);

/* Memory layout of a context: 0 = full (every incremental source field is kept; the state gradients
 * grad_h m^j are stored once per velocity where a kernel reads them: all nt+1 levels, (nt+1) x 3 FP32
 * fields, on grids with n3 < 64 or n2 < 8 or with nt > 4, level 0 for CL_PRECOND_H0, none
 * otherwise, since the marching kernels take the stencil of m^j on the fly),
 * 1 = lean (no stored gradients and one source field, computed level by level: slower).  Same results
 * up to FP32 rounding order.  Negative: error code (NULL context). */
int cl_layout(const cl_ctx *ctx);
void cl_destroy(cl_ctx *ctx);

/* Template m0 and reference m1 (Section 2.1), each n1*n2*n3 values of type
 * dt (CL_F32 only) on the device; copied and converted to the
 * context's storage precision.  Rejects NaN/Inf (CL_ERR_NONFINITE). */
int cl_set_images(cl_ctx *ctx, const void *m0, const void *m1, int dt);

/* Stationary velocity v, FP32 [3][n1][n2][n3] on the device (copied).
 * Recomputes the RK2 characteristic feet of both directions and the adjoint
 * divergence factor (Section 2.2, semi-Lagrangian scheme). */
int cl_set_velocity(cl_ctx *ctx, const float *v);
int cl_get_velocity(cl_ctx *ctx, float *v_out);

/* Objective J = mismatch + reg at the current v (Section 2.1); synchronises. */
int cl_objective(cl_ctx *ctx, double *J, double *mismatch, double *reg);

/* Reduced gradient g = beta_v A v + K int_0^1 lambda grad m dt (Section
 * 2.2, reduced gradient) at the current v.  g_out (FP32 [3][n1][n2][n3], may
 * be NULL) receives g; *gnorm (may be NULL) receives sqrt(h1h2h3 sum g.g);
 * J (may be NULL) the objective.  g = K times the L2 gradient of J; the two
 * coincide when beta_w = 0.  Synchronises. */
int cl_gradient(cl_ctx *ctx, float *g_out, double *gnorm, double *J);

/* Gauss-Newton Hessian matvec H vt = beta_v A vt + K int lambda~ grad m dt
 * (Section 2.2, Hessian matvec; two transport solves) at the current v; K
 * times the L2 Hessian of J, which the solver's PCG uses (K acts there as a
 * left preconditioner, so the Newton step is the same).
 * Needs the state of the current v (computed by cl_gradient or
 * cl_objective).  vt and Hvt must be 16-byte aligned (CL_ERR_ARG).
 * Enqueued only, no synchronisation. */
int cl_hessian_matvec(cl_ctx *ctx, const float *vt, float *Hvt);

/* The context's preconditioner applied to r (3 fields): the spectral
 * z = (beta_v A)^-1 r with the k = 0 mode scaled by 1/beta_v (with beta_w >
 * 0, z = L^-1 r, i.e. (beta_v A)^-1 K r), or the zero-velocity inner solve
 * (CL_PRECOND_H0; needs the images).  Enqueued only. */
int cl_precond_apply(cl_ctx *ctx, const float *r, float *z);

/* Gauss-Newton-Krylov solve with Armijo line search from the current v
 * (Section 2.2, Gauss-Newton-Krylov solver); on return the context holds
 * the final v.  rep may be NULL. */
int cl_solve(cl_ctx *ctx, cl_solve_report *rep);

/* Same, but replaying given decisions: step k runs exactly forced_pcg[k]
 * PCG iterations (fewer only on negative curvature) and takes the step
 * length forced_alpha[k], for n_outer steps, with no stopping test. */
int cl_solve_forced(cl_ctx *ctx, const int *forced_pcg, const double *forced_alpha,
                    int n_outer, cl_solve_report *rep);

/* Per-iteration log of the last solve: rows of 8 doubles (k, J, mismatch,
 * reg, ||g||, pcg iterations, alpha, line-search trials); the last row is
 * the final iterate.  Copies min(*n_rows, max_rows) rows. */
int cl_get_solve_log(cl_ctx *ctx, double *rows, int max_rows, int *n_rows);

/* Deformed template m(t = 1) at the current v, FP32 on the device. */
int cl_deformed_template(cl_ctx *ctx, float *m_out);

/* Read an internal field into an FP32 device buffer (inspection and
 * parity tests): which = CL_FIELD_*, j = time index 0..nt where relevant. */
enum {
    CL_FIELD_STATE = 0,       /* m^j, last objective/gradient */
    CL_FIELD_ADJOINT = 1,     /* lambda^j, last gradient */
    CL_FIELD_INC_STATE = 2,   /* mt^nt of the last matvec (only j = nt is kept) */
    CL_FIELD_INC_ADJOINT = 3, /* lambda~^j, last matvec */
    CL_FIELD_FEET_F = 4,      /* forward feet, index-unit displacements, 3 fields */
    CL_FIELD_FEET_B = 5,      /* backward feet, 3 fields */
    CL_FIELD_ADJ_FACTOR = 6   /* adjoint divergence factor c */
};
int cl_get_field(cl_ctx *ctx, int which, int j, float *out);

/* ---------------------------------------------------------------------
 * Parameter identification (Section 3.4).
 *
 * J = det grad y, y the map with m(1) = m0 o y, bounded by [J_min, 1/J_min]
 * (Section 3.4).  The paper does not say how J is computed; here grad y is
 * transported by v: d_t J + v.grad J = -(div v) J, J(0) = 1, with the
 * state's semi-Lagrangian step and Heun's rule for the source along the
 * characteristic, J^{j+1}(x) = J^j(X_f) (1 - dt/2 (d_f + d - dt d_f d)),
 * d = div_h v, d_f = d at the foot X_f.
 */

/* New regularisation weights for the following solves (beta_v > 0,
 * beta_w >= 0; CL_ERR_ARG otherwise).  Host only. */
int cl_set_regularization(cl_ctx *ctx, double beta_v, double beta_w);

/* J at the current v: *jmin, *jmax (may be NULL) receive its extremes (NaN
 * if any value is not finite); J_out (device, n1 n2 n3 FP32, may be NULL)
 * receives the field.  Synchronises. */
int cl_jacobian_det(cl_ctx *ctx, float *J_out, double *jmin, double *jmax);

typedef struct {
    double jmin;              /* J_min in (0, 1): bounds [J_min, 1/J_min] (default 0.25) */
    double beta_v_max;        /* first beta_v (default 1) */
    double beta_v_min;        /* lowest beta_v tried (default 1e-5) */
    double beta_w_max;        /* beta_w of the first stage, start of the second (default 1e-5) */
    double beta_w_min;        /* lowest beta_w tried (default 1e-7) */
    double rel_change;        /* bisection stop: relative change of beta_v (default 0.1) */
    int search_beta_w;        /* 1: run the beta_w stage (default 1) */
    int verbose;              /* 1: one line per trial on stderr (default 0) */
} cl_search_options;

typedef struct {
    double beta_v, beta_w;    /* beta_v*, beta_w* */
    double jmin, jmax;        /* J extremes of the final solution */
    int status;               /* CL_OK or CL_STATUS_BOUNDS */
    int solves, gn_total, pcg_total;
    double ms;                /* wall time */
} cl_search_report;

void cl_default_search_options(cl_search_options *so);

/* Parameter search from the current v (Section 3.4, two stages):
 *  (i)  beta_w = beta_w_max; beta_v = beta_v_max, then down by decades
 *       (not below beta_v_min) while J stays within bounds; at the first
 *       breach a bisection between the last valid and the breaching value,
 *       stopped when the next midpoint would change beta_v by less than
 *       rel_change times the valid value; beta_v* = the last valid value.
 *  (ii) beta_v = beta_v*; beta_w down by decades from beta_w_max (not below
 *       beta_w_min) while J stays within bounds; beta_w* = the last valid.
 * Every trial is a cl_solve warm-started from the previous trial's v.  On
 * return the context holds the solution for (beta_v*, beta_w*) and those
 * weights.  CL_STATUS_BOUNDS if beta_v_max already breaches the bounds
 * (then beta_v* = beta_v_max).  Each trial is logged (cl_get_search_log). */
int cl_param_search(cl_ctx *ctx, const cl_search_options *so, cl_search_report *rep);

/* Parameter continuation toward known weights (Section 3.4): solves at
 * beta_w = beta_w_max for beta_v = beta_v_max, beta_v_max / 10, ... down to
 * 10^ceil(log10 beta_v*), then beta_v*; then at beta_v* for beta_w from
 * beta_w_max down by decades to beta_w* (beta_w_target <= beta_w_max).
 * No bounds test; every solution's J extremes are logged. */
int cl_param_continuation(cl_ctx *ctx, const cl_search_options *so, double beta_v_target, double beta_w_target,
                          cl_search_report *rep);

/* Trials of the last search or continuation, 10 doubles per row: beta_v,
 * beta_w, J min, J max, within bounds (1/0), GN iterations, PCG iterations,
 * solve status, final mismatch, solve ms.  rows may be NULL (count only). */
int cl_get_search_log(cl_ctx *ctx, double *rows, int max_rows, int *n_rows);

/* Building blocks on the context's grid (parity tests of single kernels):
 *   cl_interp:   out(x) = I[u](x + d(x)) with the context's interpolation (tricubic
 *                Lagrange, or trilinear with interp_order = 1), d in index units (3 fields)
 *   cl_fd_grad:  g = grad_h u, 8th-order central differences (3 fields out)
 *   cl_fd_div:   out = div_h v (3 fields in)
 *   cl_spectral: kind 0: beta_v A, 1: (beta_v A)^-1 (k = 0 -> 1/beta_v),
 *                2: identity through the FFT, 3: K; ncomp fields in and
 *                out.  With beta_w > 0 and ncomp = 3, kinds 0, 1 and 3
 *                are L, L^-1 (k = 0 -> 1/beta_v) and K, which couple the
 *                three components per Fourier mode. */
int cl_interp(cl_ctx *ctx, const float *u, const float *d, float *out);
int cl_fd_grad(cl_ctx *ctx, const float *u, float *g);
int cl_fd_div(cl_ctx *ctx, const float *v, float *out);
int cl_spectral(cl_ctx *ctx, int kind, int ncomp, const float *in, float *out);

/* cl_interp without a context, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): out(x) = I[u](x + d(x)) on an n1 x n2 x n3 grid
 * (powers of two in [16, 1024]) with tricubic Lagrange (interp_order = 3)
 * or trilinear (1) interpolation; u, out: n1 n2 n3 FP32 values, d: three
 * such fields of index-unit displacements, all device pointers owned by
 * the caller, C order, x3 fastest.  Enqueued on `stream` (hipStream_t,
 * NULL = default), no synchronisation.  The per-tile stencil boxes live in
 * a library-held device array of CL_NOALLOC_BOX_INTS ints per GPU (4 MiB;
 * grids of more than 2^28 voxels return CL_ERR_OOM); calls that overlap on
 * one GPU share it and race.  No device or host memory is allocated.
 * Errors: CL_ERR_ARG (NULL pointer, bad order), CL_ERR_SHAPE, CL_ERR_ALIAS
 * (out overlaps u or d), CL_ERR_OOM, CL_ERR_HIP. */
#define CL_NOALLOC_BOX_INTS (1 << 20)
int cl_interp_noalloc(int n1, int n2, int n3, int interp_order, const float *u, const float *d, float *out,
                      void *stream);

/* FP64 inner product h1h2h3 sum a.b of two FP32 device vectors of n values;
 * synchronises. */
int cl_dot(cl_ctx *ctx, const float *a, const float *b, size_t n, double *out);

/* Plain device copy of n floats on the context stream (bandwidth
 * calibration of the memory counters). */
int cl_copy_f32(cl_ctx *ctx, const float *src, float *dst, size_t n);

/* Per-kernel timing with HIP events on the context stream.  mask selects
 * kernel classes (bit = 1 << CL_K_*); 0 disables.  cl_profile_query returns
 * the summed milliseconds and launch count of one class since the last
 * enable; synchronises. */
enum {
    CL_K_FEET = 0, CL_K_SL_STATE = 1, CL_K_SL_ADJOINT = 2, CL_K_SL_INC = 3,
    CL_K_FD = 4, CL_K_QUAD = 5, CL_K_FFT = 6, CL_K_VEC = 7, CL_K_COUNT = 8
};
int cl_profile_enable(cl_ctx *ctx, unsigned mask);
int cl_profile_query(cl_ctx *ctx, int kclass, double *ms_total, long long *launches);
const char *cl_kernel_class_name(int kclass);

const char *cl_status_string(int status);
const char *cl_last_error(const cl_ctx *ctx);

/* ---------------------------------------------------------------------
 * Learned warm start.  A 3D convolutional encoder-decoder (4 levels with
 * 16/32/64/128 channels, two 3x3x3 convolutions with LeakyReLU per level,
 * 2x average pooling down, nearest 2x upsampling and skip concatenation up,
 * 1x1x1 FP32 head) maps (m0, m1) on an in_n^3 grid to a velocity on that
 * grid.  Convolutions run in BF16 on the matrix cores with FP32
 * accumulation; parameters are FP32 (Adam).  It only proposes an initial
 * velocity: the Gauss-Newton solve above remains the judge of its error
 * (a prediction is used only if it lowers the objective below J(0)).
 * Same conventions as above: device pointers, caller-owned, one stream.
 * ------------------------------------------------------------------- */
#define CL_NET_OPTIONS_VERSION 1
typedef struct cl_net cl_net;
typedef struct {
    int struct_version;       /* must be CL_NET_OPTIONS_VERSION */
    int in_n;                 /* network grid: power of two in [32, 256] (default 128) */
    int base_channels;        /* 16 (the only width built) */
    float slope;              /* LeakyReLU slope (0.2) */
    float lr, beta1, beta2, eps;   /* Adam (1e-3, 0.9, 0.999, 1e-8) */
    unsigned long long seed;  /* parameter initialisation */
    void *stream;             /* hipStream_t; NULL = default stream */
} cl_net_options;

void cl_net_default_options(cl_net_options *opt);
int cl_net_create(cl_net **out, const cl_net_options *opt);
void cl_net_destroy(cl_net *net);
int cl_net_num_params(cl_net *net, size_t *n);
/* copy the FP32 parameter vector to / from a device buffer of num_params values */
int cl_net_get_params(cl_net *net, float *dst);
int cl_net_set_params(cl_net *net, const float *src);
/* v_out [3][in_n^3] FP32 = network(m0, m1), inputs FP32 [in_n^3] each */
int cl_net_forward(cl_net *net, const float *m0, const float *m1, float *v_out);
/* loss = (1/2) mean (v - label)^2 over the 3 in_n^3 values and its gradient
 * w.r.t. every parameter (grad_out: num_params FP32, may be NULL); no update */
int cl_net_loss_grad(cl_net *net, const float *m0, const float *m1, const float *v_label, float *grad_out,
                     double *loss);
/* one Adam step on the mean loss of `batch` samples stored back to back
 * (m0, m1: batch x in_n^3; v_label: batch x 3 x in_n^3); *loss = mean loss */
int cl_net_train_step(cl_net *net, const float *m0, const float *m1, const float *v_label, int batch, double *loss);
const char *cl_net_last_error(const cl_net *net);

/* Spectral resampling between two periodic grids (Section 5.3 prolongs
 * velocities spectrally): Fourier modes with |k_d| < min(n_a, n_b)/2 are
 * kept (coarse Nyquist planes dropped), all others are zero, so
 * band-limited fields are reproduced.  in: ncomp fields on grid a, out:
 * ncomp fields on grid b (FP32, device). */
typedef struct cl_resampler cl_resampler;
int cl_resampler_create(cl_resampler **out, int a1, int a2, int a3, int b1, int b2, int b3, void *stream);
void cl_resampler_destroy(cl_resampler *r);
int cl_resample(cl_resampler *r, const float *in, float *out, int ncomp);

/* Warm start of a registration context from the network: restrict the
 * context's images to the network grid, predict v there, prolong it to the
 * context grid, and keep it as the context's velocity only if it lowers the
 * objective below J(v = 0) (else v = 0).  *used = 1 if the prediction was
 * kept.  The context and the network must share one stream. */
int cl_warm_start(cl_ctx *ctx, cl_net *net, int *used, double *J_pred, double *J_zero);

/* Single layers (parity tests).  Tensors channels-last [D][H][W][C] BF16;
 * w FP32 [27][Ci][Co] with tap (tz * 3 + ty) * 3 + tx; zero padding.
 *   cl_nn_conv3: transpose = 0: out[.., Co] = act(conv(in[.., Ci]) + b)
 *                transpose = 1: out[.., Ci] = conv^T(in[.., Co]) (no bias/act)
 *     out is FP32 if out_f32 else BF16; wpack: device scratch of
 *     28 * Ci * Co * 2 bytes (the 27 taps packed in pairs with a zero
 *     tap).  Ci, Co multiples of 16.
 *   cl_nn_conv3_dw: gw[t][i][o] = sum_p x[p + t - 1][i] dz[p][o], gb[o] =
 *     sum_p dz[p][o] (gb may be NULL); workspace from cl_nn_conv3_dw_workspace. */
int cl_nn_conv3(const void *in, const float *w, const float *b, void *out, int out_f32, int D, int H, int W, int Ci,
                int Co, int act, float slope, int transpose, void *wpack, void *stream);
int cl_nn_conv3_dw_workspace(int D, int H, int W, int Ci, int Co, size_t *bytes);
int cl_nn_conv3_dw(const void *x, const void *dz, float *gw, float *gb, void *workspace, int D, int H, int W, int Ci,
                   int Co, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CLAIRE_HIP_H */
