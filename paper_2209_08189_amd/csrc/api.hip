// api.hip -- context, operator composition and Gauss-Newton-Krylov control
// (host C++) behind the C ABI of include/claire_hip.h.
//
// Every field operation is a HIP kernel on the context stream; the host only
// sequences launches and reads FP64 scalars (dot products, norms, objective
// parts) back, one synchronisation per scalar.
#include "internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

using namespace clh;

namespace {

constexpr double TWO_PI = 6.283185307179586476925286766559;

struct Prof {
    unsigned mask = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[CL_K_COUNT];
    double ms[CL_K_COUNT] = {};
    long long n[CL_K_COUNT] = {};
    std::vector<hipEvent_t> pool;
};

} // namespace

struct cl_ctx {
    Grid g{};
    cl_options opt{};
    hipStream_t s = nullptr;
    // side stream (default priority, non-blocking) for the beta A vt term of
    // a Hessian matvec with overlap_spectral, which runs beside the transport
    // sweeps; fork / join events order it against s
    hipStream_t s2 = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    int nt = 4;
    float dt = 0.25f;
    double hv = 0.0;             // h1 h2 h3
    int dts = CL_F32, dta = CL_F32;
    size_t N = 0;

    std::vector<void *> allocs;
    void *m0 = nullptr, *m1 = nullptr;      // state dtype
    void *m = nullptr;                      // (nt+1) N, state dtype
    void *lam = nullptr;                    // (nt+1) N, adjoint dtype
    void *q[2] = {nullptr, nullptr};        // adjoint dtype
    float *G = nullptr;                     // grad_h m^j, (nt+1) x 3N FP32
    float *S = nullptr;                     // incremental sources s^1..s^nt, nt x N FP32 (or one field)
    bool lean = false;                      // lean layout: one source field, no stored gradients
    bool S_all = true;                      // S holds every level (the full layout)
    int G_levels = 0;                       // levels of grad_h m^j kept in G (0, 1 or nt + 1)
    int *box_f = nullptr, *box_b = nullptr, *box_t = nullptr;  // tile stencil boxes: X_f, X_b, scratch
    float *v = nullptr, *vtrial = nullptr;  // 3N
    float *df = nullptr, *db = nullptr;     // 3N
    float *c = nullptr, *divv = nullptr;    // N
    float *grad = nullptr, *Av = nullptr, *tmp3 = nullptr;  // 3N
    float *fscr = nullptr;                  // 3N workspace of the feet computation
    float *px = nullptr, *pr = nullptr, *pz = nullptr, *pp = nullptr, *pHp = nullptr;  // 3N
    double *partials = nullptr, *dscal = nullptr, *hscal = nullptr;
    double *qparts = nullptr;                // partials of the fused PCG reductions
    int nqparts = 1;
    double *pscal = nullptr;                 // PCG device scalars (PCG_* slots)
    // zero-velocity preconditioner: inner CG vectors, L z of its result, the
    // previous outer z (flexible PCG); 3N each, allocated with that option
    float *ir = nullptr, *izi = nullptr, *ip = nullptr, *iLp = nullptr, *ih = nullptr, *ilz = nullptr,
          *zold = nullptr;
    // two-level variant: the half-resolution grid, its FFT plan, the
    // restricted template's FD8 gradient, the restricted residual and its
    // inner solution, and the inner CG vectors on that grid
    struct Coarse {
        Grid g{};
        FFTPlan fft{};
        size_t N = 0;
        double hv = 0.0;
        float *m0 = nullptr, *G0 = nullptr, *r = nullptr, *z = nullptr;
        float *ir = nullptr, *izi = nullptr, *ip = nullptr, *iLp = nullptr, *ih = nullptr;
        bool valid = false;                 // G0 matches the current images
    } cz;
    int nparts = 1;
    FFTPlan fft{};

    bool images = false, vel = false, feet_f = false, feet_b = false, state = false, av = false;
    bool sgrad = false;                     // G valid for the current state
    bool gref_valid = false;
    double gref = 0.0;
    std::vector<std::vector<double>> log;
    std::vector<std::vector<double>> slog;  // parameter search / continuation trials
    std::string err;
    Prof prof;
};

namespace {

struct Fail {
    int code;
};

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);              \
            throw Fail{CL_ERR_HIP};                                                     \
        }                                                                               \
    } while (0)

int fail(cl_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

bool pow2_ok(int n) { return n >= 16 && n <= 1024 && (n & (n - 1)) == 0; }

int ilog2i(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

Grid make_grid(int n1, int n2, int n3, int interp)
{
    Grid g{};
    g.n1 = n1; g.n2 = n2; g.n3 = n3;
    g.l1 = ilog2i(n1); g.l2 = ilog2i(n2); g.l3 = ilog2i(n3);
    g.N = n1 * n2 * n3;
    g.ih1 = (float)(n1 / TWO_PI); g.ih2 = (float)(n2 / TWO_PI); g.ih3 = (float)(n3 / TWO_PI);
    g.h1 = (float)(TWO_PI / n1); g.h2 = (float)(TWO_PI / n2); g.h3 = (float)(TWO_PI / n3);
    g.interp = interp;
    return g;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

// ---- profiling: HIP events around launches of selected kernel classes
hipEvent_t prof_event(cl_ctx *ctx)
{
    if (!ctx->prof.pool.empty()) {
        hipEvent_t e = ctx->prof.pool.back();
        ctx->prof.pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
}

void prof_drain(cl_ctx *ctx)
{
    HIPCHK(hipStreamSynchronize(ctx->s));
    if (ctx->s2) HIPCHK(hipStreamSynchronize(ctx->s2));   // a side launch may not be joined yet
    for (int k = 0; k < CL_K_COUNT; ++k) {
        for (auto &pr : ctx->prof.pending[k]) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
            ctx->prof.ms[k] += ms;
            ctx->prof.n[k] += 1;
            ctx->prof.pool.push_back(pr.first);
            ctx->prof.pool.push_back(pr.second);
        }
        ctx->prof.pending[k].clear();
    }
}

// launches of f on stream st (ctx->s or the side stream; prof_drain
// synchronizes both)
template <typename F> void run_on(cl_ctx *ctx, hipStream_t st, int kclass, F &&f)
{
    const bool on = (ctx->prof.mask >> kclass) & 1u;
    hipEvent_t a = nullptr, b = nullptr;
    if (on) {
        a = prof_event(ctx);
        HIPCHK(hipEventRecord(a, st));
    }
    f();
    HIPCHK(hipGetLastError());
    if (on) {
        b = prof_event(ctx);
        HIPCHK(hipEventRecord(b, st));
        ctx->prof.pending[kclass].push_back({a, b});
        if (ctx->prof.pending[kclass].size() > 4096) prof_drain(ctx);
    }
}

template <typename F> void run(cl_ctx *ctx, int kclass, F &&f) { run_on(ctx, ctx->s, kclass, std::forward<F>(f)); }

// ---- helpers
void *slot(cl_ctx *ctx, void *base, int dt, int j) { return (char *)base + (size_t)j * ctx->N * dtype_size(dt); }

double read_scalar(cl_ctx *ctx)
{
    HIPCHK(hipMemcpyAsync(ctx->hscal, ctx->dscal, sizeof(double), hipMemcpyDeviceToHost, ctx->s));
    HIPCHK(hipStreamSynchronize(ctx->s));
    return *ctx->hscal;
}

// h-weighted FP64 inner product of two FP32 vectors of n values
double dotw(cl_ctx *ctx, const float *a, const float *b, size_t n)
{
    run(ctx, CL_K_VEC, [&] {
        launch_dot(a, b, n, ctx->partials, ctx->nparts, ctx->s);
        launch_finalize(ctx->partials, ctx->nparts, ctx->hv, ctx->dscal, ctx->s);
    });
    return read_scalar(ctx);
}

double count_nonfinite(cl_ctx *ctx, const float *a, size_t n)
{
    run(ctx, CL_K_VEC, [&] {
        launch_count_nonfinite(a, n, ctx->partials, ctx->nparts, ctx->s);
        launch_finalize(ctx->partials, ctx->nparts, 1.0, ctx->dscal, ctx->s);
    });
    return read_scalar(ctx);
}

void spectral(cl_ctx *ctx, int kind, int ncomp, const float *in, float *out, const float *add)
{
    run(ctx, CL_K_FFT, [&] {
        spectral_apply(ctx->fft, kind, (float)ctx->opt.beta_v, (float)ctx->opt.beta_w, ncomp, in, out, add, ctx->s);
    });
}

// the same without the divergence term: beta_v A, (beta_v A)^-1, identity
void spectral_scalar(cl_ctx *ctx, int kind, int ncomp, const float *in, float *out)
{
    run(ctx, CL_K_FFT, [&] {
        spectral_apply(ctx->fft, kind, (float)ctx->opt.beta_v, 0.f, ncomp, in, out, nullptr, ctx->s);
    });
}

// ---- operator layer

// RK2 feet for the current v (forward always, backward + adjoint factor on request)
void ensure_feet(cl_ctx *ctx, bool backward)
{
    if (!ctx->feet_f || (backward && !ctx->feet_b)) {
        if (backward) run(ctx, CL_K_FD, [&] { launch_fd_div(ctx->g, ctx->v, ctx->divv, ctx->s); });
        run(ctx, CL_K_FEET, [&] {
            launch_feet(ctx->g, ctx->dt, ctx->v, ctx->df, backward ? ctx->db : nullptr,
                        backward ? ctx->divv : nullptr, backward ? ctx->c : nullptr, ctx->box_f, ctx->box_b,
                        ctx->fscr, ctx->s);
        });
        ctx->feet_f = true;
        if (backward) ctx->feet_b = true;
    }
}

// state m^0..m^nt (Section 2.1 transport equation, one SL step per dt)
void ensure_state(cl_ctx *ctx)
{
    ensure_feet(ctx, false);
    if (ctx->state) return;
    ctx->sgrad = false;
    const size_t bytes = ctx->N * dtype_size(ctx->dts);
    HIPCHK(hipMemcpyAsync(ctx->m, ctx->m0, bytes, hipMemcpyDeviceToDevice, ctx->s));
    for (int j = 0; j < ctx->nt; ++j)
        run(ctx, CL_K_SL_STATE, [&] {
            launch_sl_state(ctx->g, ctx->dts, slot(ctx, ctx->m, ctx->dts, j), ctx->df, ctx->box_f, ctx->dts,
                            slot(ctx, ctx->m, ctx->dts, j + 1), ctx->s);
        });
    ctx->state = true;
}

// G^j = grad_h m^j for the current state (used by the gradient and every
// Hessian matvec at this velocity)
void ensure_sgrad(cl_ctx *ctx)
{
    ensure_state(ctx);
    if (ctx->sgrad || ctx->G_levels == 0) return;
    StateGradArgs a{};
    for (int j = 0; j < ctx->G_levels; ++j) {
        a.m[j] = slot(ctx, ctx->m, ctx->dts, j);
        a.G[j] = ctx->G + (size_t)j * 3 * ctx->N;
    }
    run(ctx, CL_K_FD, [&] { launch_state_grad(ctx->g, ctx->dts, a, ctx->G_levels, ctx->s); });
    ctx->sgrad = true;
}

double mismatch_only(cl_ctx *ctx)
{
    run(ctx, CL_K_VEC, [&] {
        launch_sq_diff(ctx->g, ctx->dts, ctx->m1, slot(ctx, ctx->m, ctx->dts, ctx->nt), ctx->partials, ctx->nparts,
                       ctx->s);
        launch_finalize(ctx->partials, ctx->nparts, 0.5 * ctx->hv, ctx->dscal, ctx->s);
    });
    return read_scalar(ctx);
}

double regulariser(cl_ctx *ctx)
{
    if (!ctx->av) {
        spectral(ctx, 0, 3, ctx->v, ctx->Av, nullptr);
        ctx->av = true;
    }
    return 0.5 * dotw(ctx, ctx->Av, ctx->v, 3 * ctx->N);
}

void objective(cl_ctx *ctx, double *J, double *mis, double *reg)
{
    ensure_state(ctx);
    const double a = mismatch_only(ctx);
    const double r = regulariser(ctx);
    if (mis) *mis = a;
    if (reg) *reg = r;
    if (J) *J = a + r;
}

QuadArgs quad_args(cl_ctx *ctx)
{
    QuadArgs qa{};
    qa.count = ctx->nt + 1;
    qa.lean = ctx->G_levels == ctx->nt + 1 ? 0 : 1;   // 0: the per-node kernels read G
    qa.dt_m = ctx->dts;
    for (int j = 0; j <= ctx->nt; ++j) {
        qa.lam[j] = slot(ctx, ctx->lam, ctx->dta, j);
        qa.m[j] = slot(ctx, ctx->m, ctx->dts, j);
        qa.G[j] = j < ctx->G_levels ? ctx->G + (size_t)j * 3 * ctx->N : nullptr;
        qa.w[j] = (j == 0 || j == ctx->nt) ? 0.5f * ctx->dt : ctx->dt;
    }
    return qa;
}

// adjoint lam^j = c I[lam^{j+1}](X_b), j = nt-1 .. 0
void adjoint_sweep(cl_ctx *ctx)
{
    for (int j = ctx->nt - 1; j >= 0; --j)
        run(ctx, CL_K_SL_ADJOINT, [&] {
            launch_sl_adjoint(ctx->g, ctx->dta, slot(ctx, ctx->lam, ctx->dta, j + 1), ctx->db, ctx->box_b, ctx->c, ctx->dta,
                              slot(ctx, ctx->lam, ctx->dta, j), ctx->s);
        });
}

// Gradient at the current v.  ctx->grad receives the L2 gradient of J,
// L v + b (the PCG right-hand side and the Armijo slope); the reduced
// gradient of Section 2.2, g = beta_v A v + K b = K (L v + b), is returned
// by reduced_grad() and its norm by this function.  With beta_w = 0 the two
// coincide (K = I, L = beta_v A).
double gradient(cl_ctx *ctx, double *J, double *mis_out, double *reg_out)
{
    ensure_feet(ctx, true);
    ensure_sgrad(ctx);
    run(ctx, CL_K_VEC, [&] {
        launch_residual(ctx->g, ctx->dts, ctx->m1, slot(ctx, ctx->m, ctx->dts, ctx->nt), ctx->dta,
                        slot(ctx, ctx->lam, ctx->dta, ctx->nt), ctx->partials, ctx->nparts, ctx->s);
        launch_finalize(ctx->partials, ctx->nparts, 0.5 * ctx->hv, ctx->dscal, ctx->s);
    });
    const double mis = read_scalar(ctx);
    adjoint_sweep(ctx);
    if (!ctx->av) {
        spectral(ctx, 0, 3, ctx->v, ctx->Av, nullptr);
        ctx->av = true;
    }
    const QuadArgs qa = quad_args(ctx);
    const size_t n3 = 3 * ctx->N;
    if (ctx->opt.beta_w == 0.0) {
        run(ctx, CL_K_QUAD, [&] { launch_quadrature(ctx->g, ctx->dta, qa, ctx->Av, ctx->grad, ctx->s); });
    } else {
        // b into the PCG z vector (free outside PCG; the feet scratch that
        // may share it is consumed by now), L v + b into ctx->grad, and the
        // reduced gradient beta_v A v + K b in z, each term formed directly
        run(ctx, CL_K_QUAD, [&] { launch_quadrature(ctx->g, ctx->dta, qa, nullptr, ctx->pz, ctx->s); });
        run(ctx, CL_K_VEC, [&] { launch_axpy(ctx->grad, ctx->Av, ctx->pz, 1.0f, n3, ctx->s); });
        spectral(ctx, 3, 3, ctx->pz, ctx->pz, nullptr);
        spectral_scalar(ctx, 0, 3, ctx->v, ctx->tmp3);
        run(ctx, CL_K_VEC, [&] { launch_axpy(ctx->pz, ctx->pz, ctx->tmp3, 1.0f, n3, ctx->s); });
    }
    const double reg = 0.5 * dotw(ctx, ctx->Av, ctx->v, 3 * ctx->N);
    if (mis_out) *mis_out = mis;
    if (reg_out) *reg_out = reg;
    if (J) *J = mis + reg;
    const float *g = ctx->opt.beta_w != 0.0 ? ctx->pz : ctx->grad;
    return std::sqrt(dotw(ctx, g, g, 3 * ctx->N));
}

// the reduced gradient after gradient(): beta_v A v + K b, or ctx->grad
const float *reduced_grad(cl_ctx *ctx) { return ctx->opt.beta_w != 0.0 ? ctx->pz : ctx->grad; }

// GN Hessian matvec (incremental state, incremental adjoint, quadrature,
// beta A vt); needs feet of both directions and the state of the current v.
// dot_out (device, optional): <vt, Hvt> (weighted by h1 h2 h3), fused into
// the quadrature that produces Hvt.
// data_only: Hvt = the data term b~ alone (no regularisation term added).
void matvec(cl_ctx *ctx, const float *vt, float *Hvt, const float *Avt_known = nullptr, double *dot_out = nullptr,
            bool data_only = false)
{
    ensure_feet(ctx, true);
    ensure_sgrad(ctx);
    const float dt = ctx->dt;
    const int nt = ctx->nt;
    // beta A vt: on the side stream beside the sweeps (overlap_spectral; it
    // needs only vt, and the sweeps touch neither tmp3 nor the FFT work
    // space; s joins it before the quadrature), else after them on s
    const float *Avt = Avt_known;
    const bool side = !Avt && !data_only && ctx->opt.overlap_spectral;
    if (side) {
        HIPCHK(hipEventRecord(ctx->fork, ctx->s));
        HIPCHK(hipStreamWaitEvent(ctx->s2, ctx->fork, 0));
        run_on(ctx, ctx->s2, CL_K_FFT, [&] {
            spectral_apply(ctx->fft, 0, (float)ctx->opt.beta_v, (float)ctx->opt.beta_w, 3, vt, ctx->tmp3, nullptr,
                           ctx->s2);
        });
        HIPCHK(hipEventRecord(ctx->join, ctx->s2));
        Avt = ctx->tmp3;
    }
    // sources s^j = -vt . grad_h m^j, q^0 = dt/2 s^0: all levels at once (by
    // the marching FD8 kernel or from the stored gradients), or one time
    // level at a time by FD8 (lean layout with one source field)
    const bool per_level = !ctx->S_all;
    if (per_level) {
        run(ctx, CL_K_VEC, [&] {
            launch_inc_source_fd(ctx->g, ctx->dts, slot(ctx, ctx->m, ctx->dts, 0), vt, 0.5f * dt, ctx->dta,
                                 ctx->q[0], ctx->s);
        });
    } else if (sources_march(ctx->g, nt)) {
        const QuadArgs qa = quad_args(ctx);
        run(ctx, CL_K_VEC, [&] {
            launch_inc_sources_march(ctx->g, ctx->dts, qa, vt, nt, 0.5f * dt, ctx->dta, ctx->q[0], ctx->S, ctx->s);
        });
    } else {
        run(ctx, CL_K_VEC, [&] {
            launch_inc_sources(ctx->g, ctx->G, vt, nt, 0.5f * dt, ctx->dta, ctx->q[0], ctx->S, ctx->s);
        });
    }
    for (int j = 0; j < nt; ++j) {
        const bool last = j == nt - 1;
        void *out = last ? slot(ctx, ctx->lam, ctx->dta, nt) : ctx->q[(j + 1) & 1];
        const float *Sj = per_level ? ctx->S : ctx->S + (size_t)j * ctx->N;
        if (per_level)
            run(ctx, CL_K_VEC, [&] {
                launch_inc_source_fd(ctx->g, ctx->dts, slot(ctx, ctx->m, ctx->dts, j + 1), vt, 1.0f, CL_F32,
                                     ctx->S, ctx->s);
            });
        run(ctx, CL_K_SL_INC, [&] {
            launch_sl_inc(ctx->g, ctx->dta, ctx->q[j & 1], ctx->df, ctx->box_f, Sj, last ? -1.0f : 1.0f,
                          last ? -0.5f * dt : dt, ctx->dta, out, ctx->s);
        });
    }
    adjoint_sweep(ctx);
    if (side) {
        HIPCHK(hipStreamWaitEvent(ctx->s, ctx->join, 0));
    } else if (!Avt && !data_only) {
        spectral(ctx, 0, 3, vt, ctx->tmp3, nullptr);
        Avt = ctx->tmp3;
    }
    const QuadArgs qa = quad_args(ctx);
    if (dot_out) {
        run(ctx, CL_K_QUAD, [&] {
            launch_quadrature_dot(ctx->g, ctx->dta, qa, Avt, Hvt, vt, ctx->qparts, ctx->s);
            launch_finalize(ctx->qparts, quadrature_blocks(ctx->g, qa), ctx->hv, dot_out, ctx->s);
        });
    } else {
        run(ctx, CL_K_QUAD, [&] { launch_quadrature(ctx->g, ctx->dta, qa, Avt, Hvt, ctx->s); });
    }
}

// One grid of the zero-velocity inner solve: its geometry, FFT plan,
// grad_h m0 on that grid and the inner CG vectors.
struct H0Level {
    const Grid *g;
    const FFTPlan *fft;
    size_t N;
    double hv;
    const float *G0;
    float *ir, *izi, *ip, *iLp, *ih;
};

void level_spectral(cl_ctx *ctx, const H0Level &L, int kind, const float *in, float *out)
{
    run(ctx, CL_K_FFT, [&] {
        spectral_apply(*L.fft, kind, (float)ctx->opt.beta_v, (float)ctx->opt.beta_w, 3, in, out, nullptr, ctx->s);
    });
}

// z ~ H0^-1 r (zero-velocity Hessian) on grid L by opt.precond_inner CG
// steps from z = 0 with the spectral preconditioner.  The inner operator
// is L_0 + G G^T with L_0 = L except that the k = 0 mode is mapped by
// beta_v (the preconditioner's convention, definite where the data term
// vanishes); L_0 p of the inner directions is carried by the recurrence
// L_0 p = r + beta L_0 p (L_0 P_s = I), so the only FFT pair per step is
// the spectral preconditioner.  Each step after the first updates the
// direction and applies the operator in one pass.
void h0_inner(cl_ctx *ctx, const H0Level &L, const float *r, float *z)
{
    const size_t N = L.N, n = 3 * N;
    double *sc = ctx->pscal + PCG_INNER;
    const int nb = std::min(ctx->nparts, reduce_blocks(n));
    HIPCHK(hipMemcpyAsync(L.ir, r, n * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
    run(ctx, CL_K_VEC, [&] { launch_fill_f32(z, 0.0f, n, ctx->s); });
    level_spectral(ctx, L, 1, L.ir, L.izi);
    HIPCHK(hipMemcpyAsync(L.ip, L.izi, n * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
    HIPCHK(hipMemcpyAsync(L.iLp, L.ir, n * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
    run(ctx, CL_K_VEC, [&] {
        launch_dot(L.ir, L.izi, n, ctx->partials, nb, ctx->s);
        launch_finalize(ctx->partials, nb, L.hv, sc + PCG_RZ, ctx->s);
    });
    const int inner = ctx->opt.precond_inner;
    for (int it = 0; it < inner; ++it) {
        run(ctx, CL_K_VEC, [&] {
            if (it == 0)
                launch_h0_apply(L.ip, L.iLp, L.G0, L.ih, N, ctx->partials, nb, ctx->s);
            else
                launch_h0_direction_apply(L.ip, L.iLp, L.izi, L.ir, L.G0, L.ih, sc, N, ctx->partials, nb, ctx->s);
            launch_finalize(ctx->partials, nb, L.hv, sc + PCG_PHP, ctx->s);
            launch_pcg_alpha(sc, ctx->s);
            launch_h0_update(z, L.ir, L.ip, L.ih, sc, N, ctx->s);
        });
        if (it == inner - 1) break;
        level_spectral(ctx, L, 1, L.ir, L.izi);
        run(ctx, CL_K_VEC, [&] {
            launch_dot(L.ir, L.izi, n, ctx->partials, nb, ctx->s);
            launch_finalize(ctx->partials, nb, L.hv, sc + PCG_RZNEW, ctx->s);
            launch_pcg_beta(sc, ctx->s);
        });
    }
}

// Full resolution: grad_h m0 is the stored G^0; ctx->ilz receives L z (one
// spectral operation) for the outer recurrence.
void precond_h0(cl_ctx *ctx, const float *r, float *z)
{
    ensure_sgrad(ctx);
    const H0Level L{&ctx->g, &ctx->fft, ctx->N, ctx->hv, ctx->G, ctx->ir, ctx->izi, ctx->ip, ctx->iLp, ctx->ih};
    h0_inner(ctx, L, r, z);
    spectral(ctx, 0, 3, z, ctx->ilz, nullptr);
}

// Two-level variant (Section 2.2 names the two-level coarse-grid
// approximation as the default; reading): the Fourier band a half-resolution
// grid represents (|k_d| < n_d / 4) gets H0 inverted on that grid, the modes
// above it get the spectral L^-1:
//   z = P z_c + L^-1 (r - P R r),  z_c ~ H0_c^-1 R r,
// R / P spectral restriction / prolongation, H0_c = L_0 + g_c g_c^T with g_c
// = grad_h (R m0) on the coarse grid.  ctx->ilz receives L z.
void ensure_coarse(cl_ctx *ctx)
{
    auto &c = ctx->cz;
    if (c.valid) return;
    // R m0 (FP32 copy of the stored template into the fine work vector first)
    run(ctx, CL_K_VEC, [&] { launch_to_f32(ctx->dts, ctx->m0, ctx->ir, ctx->N, ctx->s); });
    run(ctx, CL_K_FFT, [&] { spectral_resample(ctx->fft, c.fft, 1, ctx->ir, c.m0, ctx->s); });
    run(ctx, CL_K_FD, [&] { launch_fd_grad(c.g, c.m0, c.G0, ctx->s); });
    c.valid = true;
}

void precond_h0_2level(cl_ctx *ctx, const float *r, float *z)
{
    ensure_coarse(ctx);
    auto &c = ctx->cz;
    const size_t n = 3 * ctx->N;
    run(ctx, CL_K_FFT, [&] { spectral_resample(ctx->fft, c.fft, 3, r, c.r, ctx->s); });        // R r
    run(ctx, CL_K_FFT, [&] { spectral_resample(c.fft, ctx->fft, 3, c.r, ctx->ir, ctx->s); });  // P R r
    run(ctx, CL_K_VEC, [&] { launch_axpy(ctx->ir, r, ctx->ir, -1.0f, n, ctx->s); });           // r - P R r
    spectral(ctx, 1, 3, ctx->ir, z, nullptr);                                                  // L^-1 (r - P R r)
    const H0Level L{&c.g, &c.fft, c.N, c.hv, c.G0, c.ir, c.izi, c.ip, c.iLp, c.ih};
    h0_inner(ctx, L, c.r, c.z);
    run(ctx, CL_K_FFT, [&] { spectral_resample(c.fft, ctx->fft, 3, c.z, ctx->ir, ctx->s); });  // P z_c
    run(ctx, CL_K_VEC, [&] { launch_axpy(z, z, ctx->ir, 1.0f, n, ctx->s); });
    spectral(ctx, 0, 3, z, ctx->ilz, nullptr);
}

void precond(cl_ctx *ctx, const float *r, float *z)
{
    if (ctx->opt.precond == CL_PRECOND_H0)
        precond_h0(ctx, r, z);
    else if (ctx->opt.precond == CL_PRECOND_H0_2LEVEL)
        precond_h0_2level(ctx, r, z);
    else
        spectral(ctx, 1, 3, r, z, nullptr);
}

void load_velocity(cl_ctx *ctx, const float *src_dev)
{
    HIPCHK(hipMemcpyAsync(ctx->v, src_dev, 3 * ctx->N * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
    ctx->vel = true;
    ctx->feet_f = ctx->feet_b = ctx->state = ctx->av = false;
}

// PCG on H x = rhs (rhs in ctx->pr on entry); solution in ctx->px.
int pcg(cl_ctx *ctx, int max_pcg, double eta, int forced, int *iters)
{
    // Scalars stay on the device (PCG_* slots of pscal): alpha, beta and the
    // curvature test are formed there, and the host reads ||r|| and the
    // curvature flag once per iteration for the stopping test.
    const size_t n = 3 * ctx->N;
    double *sc = ctx->pscal;
    const int nbc = reduce_blocks(ctx->N);
    run(ctx, CL_K_VEC, [&] { launch_fill_f32(ctx->px, 0.0f, n, ctx->s); });
    precond(ctx, ctx->pr, ctx->pz);
    HIPCHK(hipMemcpyAsync(ctx->pp, ctx->pz, n * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
    run(ctx, CL_K_VEC, [&] {
        launch_dot(ctx->pr, ctx->pz, n, ctx->partials, ctx->nparts, ctx->s);
        launch_finalize(ctx->partials, ctx->nparts, ctx->hv, sc + PCG_RZ, ctx->s);
    });
    const double r0 = std::sqrt(dotw(ctx, ctx->pr, ctx->pr, n));
    // beta A p by recurrence: p = z + b p and beta A z = r - mean(r) (A has
    // no k = 0 mode, the preconditioner maps it by 1/beta), so the matvecs
    // inside PCG need no FFT pair of their own.  With the zero-velocity
    // preconditioner L z comes from its inner solve.
    const bool h0 = ctx->opt.precond == CL_PRECOND_H0 || ctx->opt.precond == CL_PRECOND_H0_2LEVEL;
    float *pAp = ctx->tmp3;
    if (h0) {
        HIPCHK(hipMemcpyAsync(pAp, ctx->ilz, n * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
    } else {
        run(ctx, CL_K_VEC, [&] {
            launch_fill_f32(pAp, 0.0f, n, ctx->s);
            launch_comp_sums3(ctx->pr, ctx->N, ctx->partials, ctx->nparts / 3, sc + PCG_SUMR, ctx->s);
            launch_mean_free_axpy(pAp, ctx->pr, sc + PCG_SUMR, 0.0f, ctx->N, ctx->s);
        });
    }
    const int limit = forced >= 0 ? forced : max_pcg;
    int it = 0, neg = 0;
    while (it < limit) {
        matvec(ctx, ctx->pp, ctx->pHp, pAp, sc + PCG_PHP);
        run(ctx, CL_K_VEC, [&] {
            launch_pcg_alpha(sc, ctx->s);
            launch_pcg_update3(ctx->px, ctx->pr, ctx->pp, ctx->pHp, sc, ctx->N, ctx->qparts, nbc, ctx->hv, ctx->s);
        });
        HIPCHK(hipMemcpyAsync(ctx->hscal, sc, sizeof(double) * PCG_NSCAL, hipMemcpyDeviceToHost, ctx->s));
        HIPCHK(hipStreamSynchronize(ctx->s));
        if (ctx->hscal[PCG_NEG] != 0.0) {
            neg = 1;
            if (it == 0) HIPCHK(hipMemcpyAsync(ctx->px, ctx->pz, n * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
            break;
        }
        const double rn = std::sqrt(ctx->hscal[PCG_RR]);
        ++it;
        if (forced < 0 && rn <= eta * r0) break;
        if (it >= limit) break;
        if (h0) {
            // flexible PCG: beta = <r, z_new - z_old> / <r_old, z_old>
            HIPCHK(hipMemcpyAsync(ctx->zold, ctx->pz, n * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
            precond(ctx, ctx->pr, ctx->pz);
            run(ctx, CL_K_VEC, [&] {
                launch_dot(ctx->pr, ctx->pz, n, ctx->partials, ctx->nparts, ctx->s);
                launch_finalize(ctx->partials, ctx->nparts, ctx->hv, sc + PCG_RZNEW, ctx->s);
                launch_dot(ctx->pr, ctx->zold, n, ctx->partials, ctx->nparts, ctx->s);
                launch_finalize(ctx->partials, ctx->nparts, ctx->hv, sc + PCG_RZOLD, ctx->s);
                launch_pcg_beta_flex(sc, ctx->s);
                launch_pcg_direction_lz(ctx->pp, pAp, ctx->pz, ctx->ilz, sc, ctx->N, ctx->s);
            });
            continue;
        }
        precond(ctx, ctx->pr, ctx->pz);
        run(ctx, CL_K_VEC, [&] {
            launch_dot(ctx->pr, ctx->pz, n, ctx->partials, ctx->nparts, ctx->s);
            launch_finalize(ctx->partials, ctx->nparts, ctx->hv, sc + PCG_RZNEW, ctx->s);
            launch_pcg_beta(sc, ctx->s);
            launch_pcg_direction(ctx->pp, pAp, ctx->pz, ctx->pr, sc, ctx->N, ctx->s);
        });
    }
    if (iters) *iters = it;
    return neg;
}

double compute_gref(cl_ctx *ctx)
{
    if (ctx->gref_valid) return ctx->gref;
    // g(v = 0): swap in a zero velocity, evaluate, restore
    const size_t n = 3 * ctx->N;
    std::swap(ctx->v, ctx->vtrial);
    run(ctx, CL_K_VEC, [&] { launch_fill_f32(ctx->v, 0.0f, n, ctx->s); });
    ctx->feet_f = ctx->feet_b = ctx->state = ctx->av = false;
    ctx->gref = gradient(ctx, nullptr, nullptr, nullptr);
    ctx->gref_valid = true;
    std::swap(ctx->v, ctx->vtrial);
    ctx->feet_f = ctx->feet_b = ctx->state = ctx->av = false;
    return ctx->gref;
}

int solve(cl_ctx *ctx, const int *forced_pcg, const double *forced_alpha, int forced_n, cl_solve_report *rep)
{
    const auto t0 = std::chrono::steady_clock::now();
    const size_t n = 3 * ctx->N;
    const bool forced = forced_pcg != nullptr;
    const int max_outer = forced ? forced_n : ctx->opt.max_outer;
    const double gref = compute_gref(ctx);
    ctx->log.clear();
    cl_solve_report R{};
    R.gref = gref;
    int status = CL_STATUS_MAXIT, k = 0;
    double J = 0, mis = 0, reg = 0, gn = 0;
    for (k = 0; k < max_outer; ++k) {
        gn = gradient(ctx, &J, &mis, &reg);
        if (k == 0) { R.J0 = J; R.gnorm0 = gn; }
        ctx->log.push_back({(double)k, J, mis, reg, gn, 0.0, 0.0, 0.0});
        if (!forced && gn <= ctx->opt.gtol * gref) { status = CL_OK; break; }
        double eta = ctx->opt.forcing ? std::min(0.5, std::sqrt(gn / gref)) : ctx->opt.eta_fixed;
        run(ctx, CL_K_VEC, [&] { launch_scale(ctx->pr, ctx->grad, -1.0f, n, ctx->s); });   // rhs = -g
        int its = 0;
        pcg(ctx, ctx->opt.max_pcg, eta, forced ? forced_pcg[k] : -1, &its);
        R.pcg_iters_total += its;
        if (ctx->opt.fault_flip_direction)   // failure injection: an ascent direction
            run(ctx, CL_K_VEC, [&] { launch_scale(ctx->px, ctx->px, -1.0f, n, ctx->s); });
        const double gvt = dotw(ctx, ctx->grad, ctx->px, n);
        double alpha = 1.0;
        int trials = 0;
        bool ok = false;
        if (forced) {
            alpha = forced_alpha[k];
            run(ctx, CL_K_VEC, [&] { launch_axpy(ctx->vtrial, ctx->v, ctx->px, (float)alpha, n, ctx->s); });
            std::swap(ctx->v, ctx->vtrial);
            ctx->feet_f = ctx->feet_b = ctx->state = ctx->av = false;
            ok = true;
        } else {
            for (trials = 1; trials <= 10; ++trials) {
                run(ctx, CL_K_VEC, [&] { launch_axpy(ctx->vtrial, ctx->v, ctx->px, (float)alpha, n, ctx->s); });
                std::swap(ctx->v, ctx->vtrial);
                ctx->feet_f = ctx->feet_b = ctx->state = ctx->av = false;
                double Jt;
                objective(ctx, &Jt, nullptr, nullptr);
                R.linesearch_trials++;
                if (Jt <= J + 1e-4 * alpha * gvt) { ok = true; break; }
                std::swap(ctx->v, ctx->vtrial);   // back to the accepted v
                ctx->feet_f = ctx->feet_b = ctx->state = ctx->av = false;
                alpha *= 0.5;
            }
        }
        if (!forced && !ok) trials = 10;   // every one of the 10 trials failed
        ctx->log.back()[5] = its;
        ctx->log.back()[6] = ok ? alpha : 0.0;
        ctx->log.back()[7] = trials;
        if (!ok) {
            status = CL_STATUS_LINESEARCH_FAIL;
            ++k;
            break;
        }
    }
    if (status != CL_OK) {
        gn = gradient(ctx, &J, &mis, &reg);
        ctx->log.push_back({(double)k, J, mis, reg, gn, 0.0, 0.0, 0.0});
        if (status == CL_STATUS_MAXIT && gn <= ctx->opt.gtol * gref) status = CL_OK;
        if (k == 0) { R.J0 = J; R.gnorm0 = gn; }
    }
    R.status = status;
    R.outer_iters = k;
    R.J = J; R.mismatch = mis; R.reg = reg; R.gnorm = gn;
    HIPCHK(hipStreamSynchronize(ctx->s));
    R.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = R;
    return status;
}

// Levels of grad_h m^j a context stores: every level where a kernel reads
// them (grids the marching FD8 kernels do not cover, or more time steps than
// the all-level source pass takes), level 0 for the full-resolution
// zero-velocity preconditioner (the two-level one takes the gradient of its
// coarse template), none otherwise (and none in the lean layout)
int grad_levels(int n1, int n2, int n3, const cl_options &o, bool lean)
{
    if (lean) return 0;
    const Grid g = make_grid(n1, n2, n3, o.interp_order);
    QuadArgs qa{};
    qa.count = o.nt + 1;
    if (!quadrature_marches(g, qa) || !sources_march(g, o.nt)) return o.nt + 1;
    return o.precond == CL_PRECOND_H0 ? 1 : 0;
}

size_t workspace_bytes(int n1, int n2, int n3, const cl_options &o, bool lean)
{
    const size_t N = (size_t)n1 * n2 * n3;
    const size_t es = dtype_size(o.storage_state), ea = dtype_size(o.storage_adjoint);
    size_t b = 0;
    b += 2 * N * es;                         // m0, m1
    b += (size_t)(o.nt + 1) * N * es;        // m^j
    b += (size_t)(o.nt + 1) * N * ea;        // lam^j / lam~^j
    b += 2 * N * ea;                         // q ping-pong
    b += (size_t)grad_levels(n1, n2, n3, o, lean) * 3 * N * sizeof(float);   // grad_h m^j
    b += (size_t)(lean ? 1 : o.nt) * N * sizeof(float);   // incremental sources s^j
    b += 3 * (N / 2048 + 1) * 8 * sizeof(int);  // tile stencil boxes
    b += 2 * N * sizeof(float);              // c, div v
    b += 12 * 3 * N * sizeof(float);         // v, vtrial, df, db, g, Av, tmp3, PCG x r z p Hp
    if (o.precond == CL_PRECOND_H0) b += 7 * 3 * N * sizeof(float);   // inner CG, L z, previous z
    if (o.precond == CL_PRECOND_H0_2LEVEL) {
        const size_t Nc = N / 8;
        b += 3 * 3 * N * sizeof(float);                                   // fine work vector, L z, previous z
        b += (1 + 3 + 2 * 3 + 5 * 3) * Nc * sizeof(float);                // R m0, g_c, r_c, z_c, inner CG
        b += fft_spec_bytes(n1 / 2, n2 / 2, n3 / 2, 3) + 4 * 513 * sizeof(float2);
    }
    b += fft_spec_bytes(n1, n2, n3, 3);
    b += 4 * 1025 * sizeof(float2) + 4096 * sizeof(double) + 256;   // FFT tables, reduction partials, scalars
    b += (std::max<size_t>((N / 4 + 255) / 256, 6 * (size_t)reduce_blocks(N)) + PCG_NSCAL) * sizeof(double);
    return b;
}

// J = det grad y at the current v: min and max, and the field (N floats,
// device) if J_out is given.  Uses the feet of the current v and tmp3.
void jacobian(cl_ctx *ctx, double *jmin, double *jmax, float *J_out)
{
    ensure_feet(ctx, true);
    float *J = ctx->tmp3 + 2 * ctx->N;
    run(ctx, CL_K_SL_STATE, [&] {
        launch_jacobian(ctx->g, ctx->dt, ctx->nt, ctx->divv, ctx->df, ctx->box_f, ctx->tmp3, J, ctx->s);
    });
    run(ctx, CL_K_VEC, [&] { launch_minmax(J, ctx->N, ctx->partials, ctx->nparts / 2, ctx->dscal, ctx->s); });
    HIPCHK(hipMemcpyAsync(ctx->hscal, ctx->dscal, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->s));
    if (J_out) HIPCHK(hipMemcpyAsync(J_out, J, ctx->N * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
    HIPCHK(hipStreamSynchronize(ctx->s));
    *jmin = ctx->hscal[0];
    *jmax = ctx->hscal[1];
}

// new regularisation weights: the cached beta A v and g_ref depend on them
void set_regularization(cl_ctx *ctx, double beta_v, double beta_w)
{
    ctx->opt.beta_v = beta_v;
    ctx->opt.beta_w = beta_w;
    ctx->av = false;
    ctx->gref_valid = false;
}

// Parameter search (Section 3.4, parameter identification).  Every trial
// is a GN solve warm-started from the previous trial's velocity, followed
// by the bounds test J_min <= det grad y <= 1/J_min.
//  (i)  beta_w = beta_w_max; beta_v from beta_v_max down by decades while
//       the bounds hold (not below beta_v_min); on the first breach a
//       bisection between the last valid and the breaching value, stopped
//       when the next step would change beta_v by less than rel_change of
//       the valid value; beta_v* = the last valid value.
//  (ii) beta_v = beta_v*; beta_w from beta_w_max down by decades while the
//       bounds hold (not below beta_w_min); beta_w* = the last valid value.
// The velocity of the last valid trial, the solution for (beta_v*,
// beta_w*), is kept in host memory and restored at the end when a later
// trial breached the bounds.
struct Search {
    cl_ctx *ctx;
    const cl_search_options &so;
    cl_search_report R{};
    std::vector<float> best;     // v of the last valid trial (host)
    double best_jmin = 0, best_jmax = 0;

    bool trial(double bv, double bw)
    {
        set_regularization(ctx, bv, bw);
        cl_solve_report sr{};
        solve(ctx, nullptr, nullptr, 0, &sr);
        double jl = 0, jh = 0;
        jacobian(ctx, &jl, &jh, nullptr);
        const bool ok = std::isfinite(jl) && std::isfinite(jh) && jl >= so.jmin && jh <= 1.0 / so.jmin;
        R.solves++;
        R.gn_total += sr.outer_iters;
        R.pcg_total += sr.pcg_iters_total;
        R.jmin = jl;
        R.jmax = jh;
        ctx->slog.push_back({bv, bw, jl, jh, ok ? 1.0 : 0.0, (double)sr.outer_iters, (double)sr.pcg_iters_total,
                             (double)sr.status, sr.mismatch, sr.ms});
        if (so.verbose) {
            std::fprintf(stderr, "[claire] trial beta_v %.6g beta_w %.3g: J [%.4f, %.4f] %s, %d GN, %d PCG, %.1f s\n",
                         bv, bw, jl, jh, so.jmin > 0.0 ? (ok ? "within bounds" : "breach") : "", sr.outer_iters,
                         sr.pcg_iters_total, sr.ms / 1e3);
            std::fflush(stderr);
        }
        if (ok && so.jmin > 0.0) {
            best.resize(3 * ctx->N);
            HIPCHK(hipMemcpy(best.data(), ctx->v, best.size() * sizeof(float), hipMemcpyDeviceToHost));
            best_jmin = jl;
            best_jmax = jh;
        }
        return ok;
    }

    // back to the last valid trial's solution and weights
    void restore(double bv, double bw)
    {
        HIPCHK(hipMemcpy(ctx->v, best.data(), best.size() * sizeof(float), hipMemcpyHostToDevice));
        ctx->vel = true;
        ctx->feet_f = ctx->feet_b = ctx->state = ctx->av = false;
        set_regularization(ctx, bv, bw);
        R.jmin = best_jmin;
        R.jmax = best_jmax;
    }
};

constexpr double DECADE_SLACK = 1e-9;   // decade steps compared with a relative slack

int param_search(cl_ctx *ctx, const cl_search_options &so, cl_search_report *rep)
{
    const auto t0 = std::chrono::steady_clock::now();
    ctx->slog.clear();
    Search S{ctx, so};
    const double bw = so.beta_w_max;
    double bv = so.beta_v_max, good = -1.0, bad = -1.0;
    for (;;) {
        if (!S.trial(bv, bw)) {
            bad = bv;
            break;
        }
        good = bv;
        const double next = bv / 10.0;
        if (next < so.beta_v_min * (1.0 - DECADE_SLACK)) break;
        bv = next;
    }
    int status = CL_OK;
    if (good < 0.0) {
        status = CL_STATUS_BOUNDS;
        good = so.beta_v_max;
    } else if (bad > 0.0) {
        for (;;) {
            const double mid = 0.5 * (good + bad);
            if (good - mid < so.rel_change * good) break;
            if (S.trial(mid, bw))
                good = mid;
            else
                bad = mid;
        }
    }
    double bw_star = bw;
    if (status == CL_OK && so.search_beta_w && bw > 0.0) {
        for (double b = bw;;) {
            const double next = b / 10.0;
            if (next < so.beta_w_min * (1.0 - DECADE_SLACK)) break;
            if (!S.trial(good, next)) break;
            bw_star = b = next;
        }
    }
    const auto &last = ctx->slog.back();
    if (status == CL_OK && last[4] != 1.0) S.restore(good, bw_star);
    S.R.beta_v = good;
    S.R.beta_w = bw_star;
    S.R.status = status;
    S.R.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = S.R;
    return status;
}

// Parameter continuation (Section 3.4): the search's solve sequence toward
// known targets without bounds tests or bisection.  (i) beta_w = beta_w_max,
// beta_v = beta_v_max, beta_v_max / 10, ... down to 10^k, k = ceil(log10
// beta_v*), then beta_v*; (ii) beta_v = beta_v*, beta_w from beta_w_max down
// by decades to beta_w*.  Each solve is warm-started from the previous one;
// J bounds of every solution are logged.
int param_continuation(cl_ctx *ctx, const cl_search_options &so, double bv_star, double bw_star,
                       cl_search_report *rep)
{
    const auto t0 = std::chrono::steady_clock::now();
    ctx->slog.clear();
    cl_search_options loose = so;
    loose.jmin = 0.0;   // the log's valid column then only flags finite J
    Search S{ctx, loose};
    const double stop = std::pow(10.0, std::ceil(std::log10(bv_star)));
    double bv = so.beta_v_max;
    for (; bv > stop * (1.0 + DECADE_SLACK); bv /= 10.0) S.trial(bv, so.beta_w_max);
    S.trial(bv, so.beta_w_max);
    if (std::fabs(bv - bv_star) > DECADE_SLACK * bv_star) S.trial(bv_star, so.beta_w_max);
    if (bw_star <= 0.0) {
        if (so.beta_w_max > 0.0) S.trial(bv_star, 0.0);
    } else {
        for (double b = so.beta_w_max; b > bw_star * (1.0 + DECADE_SLACK);) {
            b = std::max(b / 10.0, bw_star);
            S.trial(bv_star, b);
        }
    }
    S.R.beta_v = bv_star;
    S.R.beta_w = bw_star;
    S.R.status = CL_OK;
    S.R.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = S.R;
    return CL_OK;
}

int check_reg(double beta_v, double beta_w, cl_ctx *ctx)
{
    if (!(beta_v > 0.0) || !std::isfinite(beta_v)) return fail(ctx, CL_ERR_ARG, "beta_v must be > 0");
    if (!(beta_w >= 0.0) || !std::isfinite(beta_w)) return fail(ctx, CL_ERR_ARG, "beta_w must be >= 0");
    return CL_OK;
}

int check_search(const cl_search_options *so, cl_ctx *ctx)
{
    if (!so) return fail(ctx, CL_ERR_ARG, "search options pointer is NULL");
    if (!(so->jmin > 0.0 && so->jmin < 1.0)) return fail(ctx, CL_ERR_ARG, "jmin must lie in (0, 1)");
    if (!(so->beta_v_max > 0.0) || !(so->beta_v_min > 0.0) || !(so->beta_v_min <= so->beta_v_max) ||
        !std::isfinite(so->beta_v_max))
        return fail(ctx, CL_ERR_ARG, "need 0 < beta_v_min <= beta_v_max");
    if (!(so->beta_w_max >= 0.0) || !(so->beta_w_min >= 0.0) || !(so->beta_w_min <= so->beta_w_max) ||
        !std::isfinite(so->beta_w_max))
        return fail(ctx, CL_ERR_ARG, "need 0 <= beta_w_min <= beta_w_max");
    if (!(so->rel_change > 0.0 && so->rel_change < 1.0)) return fail(ctx, CL_ERR_ARG, "rel_change must lie in (0, 1)");
    if (so->search_beta_w && so->beta_w_max > 0.0 && !(so->beta_w_min > 0.0))
        return fail(ctx, CL_ERR_ARG, "the beta_w search needs beta_w_min > 0");
    return CL_OK;
}

int check_options(const cl_options *o, cl_ctx *ctx)
{
    if (!o) return fail(ctx, CL_ERR_ARG, "options pointer is NULL");
    if (o->struct_version != CL_OPTIONS_VERSION) return fail(ctx, CL_ERR_ARG, "cl_options.struct_version mismatch");
    if (o->nt < 1 || o->nt > MAX_T - 1) return fail(ctx, CL_ERR_ARG, "nt out of range [1, 64]");
    if (!(o->beta_v > 0.0) || !std::isfinite(o->beta_v)) return fail(ctx, CL_ERR_ARG, "beta_v must be > 0");
    if (!(o->beta_w >= 0.0) || !std::isfinite(o->beta_w)) return fail(ctx, CL_ERR_ARG, "beta_w must be >= 0");
    if (o->max_outer < 0 || o->max_pcg < 1) return fail(ctx, CL_ERR_ARG, "iteration limits out of range");
    if (o->interp_order != 1 && o->interp_order != 3) return fail(ctx, CL_ERR_ARG, "interp_order must be 1 or 3");
    if (o->overlap_spectral != 0 && o->overlap_spectral != 1) return fail(ctx, CL_ERR_ARG, "overlap_spectral must be 0 or 1");
    if (o->fault_flip_direction != 0 && o->fault_flip_direction != 1)
        return fail(ctx, CL_ERR_ARG, "fault_flip_direction must be 0 or 1");
    if (o->precond != CL_PRECOND_SPECTRAL && o->precond != CL_PRECOND_H0 && o->precond != CL_PRECOND_H0_2LEVEL)
        return fail(ctx, CL_ERR_ARG, "unknown preconditioner");
    if (o->precond != CL_PRECOND_SPECTRAL && (o->precond_inner < 1 || o->precond_inner > 100))
        return fail(ctx, CL_ERR_ARG, "precond_inner out of range [1, 100]");
    if (!(o->gtol >= 0.0)) return fail(ctx, CL_ERR_ARG, "gtol must be >= 0");
    for (int dt : {o->storage_state, o->storage_adjoint})
        if (dt != CL_F32 && dt != CL_BF16 && dt != CL_F16) return fail(ctx, CL_ERR_DTYPE, "unknown storage dtype");
    return CL_OK;
}

#define API_BEGIN try {
#define API_END                                                                 \
    }                                                                           \
    catch (const Fail &f_) { return f_.code; }                                  \
    catch (...) { return fail(ctx, CL_ERR_HIP, "unexpected host exception"); }

#define NEED_CTX()                                                              \
    if (!ctx) return CL_ERR_ARG

} // namespace

namespace clh {

void ctx_dims(const cl_ctx *ctx, int *n1, int *n2, int *n3)
{
    *n1 = ctx->g.n1;
    *n2 = ctx->g.n2;
    *n3 = ctx->g.n3;
}

hipStream_t ctx_stream(const cl_ctx *ctx) { return ctx->s; }

bool ctx_has_images(const cl_ctx *ctx) { return ctx->images; }

void ctx_images_f32(cl_ctx *ctx, float *m0, float *m1)
{
    launch_to_f32(ctx->dts, ctx->m0, m0, ctx->N, ctx->s);
    launch_to_f32(ctx->dts, ctx->m1, m1, ctx->N, ctx->s);
}

} // namespace clh

extern "C" {

void cl_default_options(cl_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->struct_version = CL_OPTIONS_VERSION;
    o->nt = 4;
    o->beta_v = 5e-4;
    o->beta_w = 0.0;
    o->precond = CL_PRECOND_SPECTRAL;
    o->precond_inner = 5;
    o->interp_order = 3;
    o->overlap_spectral = 0;
    o->fault_flip_direction = 0;
    o->gtol = 1e-2;
    o->max_outer = 50;
    o->max_pcg = 10;
    o->forcing = 1;
    o->eta_fixed = 0.1;
    o->storage_state = CL_F32;
    o->storage_adjoint = CL_F32;
    o->stream = nullptr;
    o->workspace_cap_bytes = 0;
}

int cl_query_workspace(int n1, int n2, int n3, const cl_options *opt, unsigned long long *bytes)
{
    if (!bytes) return CL_ERR_ARG;
    int st = check_options(opt, nullptr);
    if (st) return st;
    if (!pow2_ok(n1) || !pow2_ok(n2) || !pow2_ok(n3)) return CL_ERR_SHAPE;
    const size_t full = workspace_bytes(n1, n2, n3, *opt, false);
    const bool lean = opt->workspace_cap_bytes && full > opt->workspace_cap_bytes;
    *bytes = lean ? workspace_bytes(n1, n2, n3, *opt, true) : full;
    return CL_OK;
}

int cl_create(cl_ctx **out, int n1, int n2, int n3, const cl_options *opt)
{
    if (!out) return CL_ERR_ARG;
    *out = nullptr;
    int st = check_options(opt, nullptr);
    if (st) return st;
    if (!pow2_ok(n1) || !pow2_ok(n2) || !pow2_ok(n3)) return CL_ERR_SHAPE;
    // layout: the full one when it fits the cap (or, without a cap, the free
    // device memory), else the lean one; CL_ERR_OOM if neither fits the cap
    const size_t full = workspace_bytes(n1, n2, n3, *opt, false);
    size_t limit = opt->workspace_cap_bytes;
    if (!limit) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) limit = fr - fr / 16;
    }
    const bool lean = limit && full > limit;
    if (lean && opt->precond != CL_PRECOND_SPECTRAL) return CL_ERR_UNSUPPORTED;
    if (opt->precond == CL_PRECOND_H0_2LEVEL && (n1 < 32 || n2 < 32 || n3 < 32)) return CL_ERR_SHAPE;
    if (lean && opt->workspace_cap_bytes && workspace_bytes(n1, n2, n3, *opt, true) > opt->workspace_cap_bytes)
        return CL_ERR_OOM;
    cl_ctx *ctx = new (std::nothrow) cl_ctx();
    if (!ctx) return CL_ERR_OOM;
    ctx->lean = lean;
    ctx->S_all = !lean;
    ctx->G_levels = grad_levels(n1, n2, n3, *opt, lean);
    ctx->opt = *opt;
    ctx->s = (hipStream_t)opt->stream;
    ctx->nt = opt->nt;
    ctx->dt = (float)(1.0 / opt->nt);
    ctx->dts = opt->storage_state;
    ctx->dta = opt->storage_adjoint;
    ctx->g = make_grid(n1, n2, n3, opt->interp_order);
    const Grid &g = ctx->g;
    ctx->N = (size_t)g.N;
    ctx->hv = (TWO_PI / n1) * (TWO_PI / n2) * (TWO_PI / n3);
    const size_t N = ctx->N;
    auto alloc = [&](size_t bytes) -> void * {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) throw Fail{CL_ERR_OOM};
        ctx->allocs.push_back(p);
        return p;
    };
    try {
        const size_t es = dtype_size(ctx->dts), ea = dtype_size(ctx->dta);
        ctx->m0 = alloc(N * es);
        ctx->m1 = alloc(N * es);
        ctx->m = alloc((size_t)(ctx->nt + 1) * N * es);
        ctx->lam = alloc((size_t)(ctx->nt + 1) * N * ea);
        ctx->q[0] = alloc(N * ea);
        ctx->q[1] = alloc(N * ea);
        if (ctx->G_levels) ctx->G = (float *)alloc((size_t)ctx->G_levels * 3 * N * sizeof(float));
        ctx->S = (float *)alloc((size_t)(ctx->S_all ? ctx->nt : 1) * N * sizeof(float));
        {
            const size_t nb = std::max<size_t>(tile_box_ints(ctx->g), 8) * sizeof(int);
            ctx->box_f = (int *)alloc(nb);
            ctx->box_b = (int *)alloc(nb);
            ctx->box_t = (int *)alloc(nb);
        }
        float **vecs[] = {&ctx->v, &ctx->vtrial, &ctx->df, &ctx->db, &ctx->grad, &ctx->Av, &ctx->tmp3,
                          &ctx->px, &ctx->pr, &ctx->pz, &ctx->pp, &ctx->pHp};
        for (float **pv : vecs) *pv = (float *)alloc(3 * N * sizeof(float));
        if (opt->precond == CL_PRECOND_H0) {
            float **hv[] = {&ctx->ir, &ctx->izi, &ctx->ip, &ctx->iLp, &ctx->ih, &ctx->ilz, &ctx->zold};
            for (float **pv : hv) *pv = (float *)alloc(3 * N * sizeof(float));
        }
        if (opt->precond == CL_PRECOND_H0_2LEVEL) {
            float **hv[] = {&ctx->ir, &ctx->ilz, &ctx->zold};
            for (float **pv : hv) *pv = (float *)alloc(3 * N * sizeof(float));
            auto &c = ctx->cz;
            c.g = make_grid(n1 / 2, n2 / 2, n3 / 2, opt->interp_order);
            c.N = N / 8;
            c.hv = ctx->hv * 8.0;
            c.m0 = (float *)alloc(c.N * sizeof(float));
            float **cv[] = {&c.G0, &c.r, &c.z, &c.ir, &c.izi, &c.ip, &c.iLp, &c.ih};
            for (float **pv : cv) *pv = (float *)alloc(3 * c.N * sizeof(float));
            try {
                fft_plan_init(c.fft, n1 / 2, n2 / 2, n3 / 2, 3, alloc);
            } catch (hipError_t e) {
                ctx->err = std::string("FFT tables: ") + hipGetErrorString(e);
                throw Fail{CL_ERR_HIP};
            }
        }
        // the feet are computed outside PCG, where z is free
        ctx->fscr = ctx->pz;
        ctx->c = (float *)alloc(N * sizeof(float));
        ctx->divv = (float *)alloc(N * sizeof(float));
        ctx->nparts = reduce_blocks(3 * N);
        ctx->partials = (double *)alloc(ctx->nparts * sizeof(double));
        ctx->dscal = (double *)alloc(sizeof(double) * 4);
        ctx->nqparts = std::max(quadrature_blocks_max(ctx->g), 6 * reduce_blocks(ctx->N));
        ctx->qparts = (double *)alloc(sizeof(double) * ctx->nqparts);
        ctx->pscal = (double *)alloc(sizeof(double) * PCG_NSCAL);
        if (hipHostMalloc((void **)&ctx->hscal, sizeof(double) * PCG_NSCAL, hipHostMallocDefault) != hipSuccess)
            throw Fail{CL_ERR_OOM};
        if (opt->overlap_spectral) {
            HIPCHK(hipStreamCreateWithFlags(&ctx->s2, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming));
        }
        try {
            fft_plan_init(ctx->fft, n1, n2, n3, 3, alloc);
        } catch (hipError_t e) {
            ctx->err = std::string("FFT tables: ") + hipGetErrorString(e);
            throw Fail{CL_ERR_HIP};
        }
        // a defined initial velocity: v = 0
        HIPCHK(hipMemsetAsync(ctx->v, 0, 3 * N * sizeof(float), ctx->s));
        ctx->vel = true;
        HIPCHK(hipStreamSynchronize(ctx->s));
    } catch (const Fail &f) {
        cl_destroy(ctx);
        return f.code;
    }
    *out = ctx;
    return CL_OK;
}

int cl_layout(const cl_ctx *ctx)
{
    if (!ctx) return CL_ERR_ARG;
    return ctx->lean ? 1 : 0;
}

void cl_destroy(cl_ctx *ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->s);
    if (ctx->s2) {
        (void)hipStreamSynchronize(ctx->s2);
        (void)hipStreamDestroy(ctx->s2);
    }
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->join) (void)hipEventDestroy(ctx->join);
    for (void *p : ctx->allocs) (void)hipFree(p);
    if (ctx->hscal) (void)hipHostFree(ctx->hscal);
    for (int k = 0; k < CL_K_COUNT; ++k)
        for (auto &pr : ctx->prof.pending[k]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (hipEvent_t e : ctx->prof.pool) (void)hipEventDestroy(e);
    delete ctx;
}

int cl_set_images(cl_ctx *ctx, const void *m0, const void *m1, int dt)
{
    NEED_CTX();
    if (!m0 || !m1) return fail(ctx, CL_ERR_ARG, "NULL image pointer");
    if (dt != CL_F32) return fail(ctx, CL_ERR_DTYPE, "images must be passed as CL_F32");
    API_BEGIN
    const size_t N = ctx->N;
    if (count_nonfinite(ctx, (const float *)m0, N) > 0 || count_nonfinite(ctx, (const float *)m1, N) > 0)
        return fail(ctx, CL_ERR_NONFINITE, "image contains NaN or Inf");
    run(ctx, CL_K_VEC, [&] {
        launch_convert(ctx->dts, ctx->m0, (const float *)m0, N, ctx->s);
        launch_convert(ctx->dts, ctx->m1, (const float *)m1, N, ctx->s);
    });
    ctx->images = true;
    ctx->state = false;
    ctx->gref_valid = false;
    ctx->cz.valid = false;
    return CL_OK;
    API_END
}

int cl_set_velocity(cl_ctx *ctx, const float *v)
{
    NEED_CTX();
    if (!v) return fail(ctx, CL_ERR_ARG, "NULL velocity pointer");
    API_BEGIN
    if (count_nonfinite(ctx, v, 3 * ctx->N) > 0) return fail(ctx, CL_ERR_NONFINITE, "velocity contains NaN or Inf");
    load_velocity(ctx, v);
    return CL_OK;
    API_END
}

int cl_get_velocity(cl_ctx *ctx, float *v_out)
{
    NEED_CTX();
    if (!v_out) return fail(ctx, CL_ERR_ARG, "NULL output pointer");
    API_BEGIN
    HIPCHK(hipMemcpyAsync(v_out, ctx->v, 3 * ctx->N * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
    return CL_OK;
    API_END
}

int cl_objective(cl_ctx *ctx, double *J, double *mismatch, double *reg)
{
    NEED_CTX();
    if (!ctx->images) return fail(ctx, CL_ERR_STATE, "cl_set_images has not been called");
    API_BEGIN
    objective(ctx, J, mismatch, reg);
    return CL_OK;
    API_END
}

int cl_gradient(cl_ctx *ctx, float *g_out, double *gnorm, double *J)
{
    NEED_CTX();
    if (!ctx->images) return fail(ctx, CL_ERR_STATE, "cl_set_images has not been called");
    API_BEGIN
    const double gn = gradient(ctx, J, nullptr, nullptr);
    if (gnorm) *gnorm = gn;
    if (g_out) {
        HIPCHK(hipMemcpyAsync(g_out, reduced_grad(ctx), 3 * ctx->N * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
        HIPCHK(hipStreamSynchronize(ctx->s));
    }
    return CL_OK;
    API_END
}

int cl_hessian_matvec(cl_ctx *ctx, const float *vt, float *Hvt)
{
    NEED_CTX();
    if (!vt || !Hvt) return fail(ctx, CL_ERR_ARG, "NULL vector pointer");
    if (!ctx->images) return fail(ctx, CL_ERR_STATE, "cl_set_images has not been called");
    const size_t b = 3 * ctx->N * sizeof(float);
    if (overlap(vt, b, Hvt, b)) return fail(ctx, CL_ERR_ALIAS, "vt and Hvt overlap");
    if (((uintptr_t)vt | (uintptr_t)Hvt) & 15) return fail(ctx, CL_ERR_ARG, "vt and Hvt must be 16-byte aligned");
    API_BEGIN
    if (ctx->opt.beta_w == 0.0) {
        matvec(ctx, vt, Hvt);
    } else if (ctx->opt.overlap_spectral) {
        // reduced form H vt = beta_v A vt + K b~; beta_v A vt on the side
        // stream beside the data term's sweeps (after the feet, whose
        // computation precedes the fork), joined before K b~ takes the FFT
        // work space
        ensure_feet(ctx, true);
        ensure_sgrad(ctx);
        HIPCHK(hipEventRecord(ctx->fork, ctx->s));
        HIPCHK(hipStreamWaitEvent(ctx->s2, ctx->fork, 0));
        run_on(ctx, ctx->s2, CL_K_FFT, [&] {
            spectral_apply(ctx->fft, 0, (float)ctx->opt.beta_v, 0.f, 3, vt, ctx->tmp3, nullptr, ctx->s2);
        });
        HIPCHK(hipEventRecord(ctx->join, ctx->s2));
        matvec(ctx, vt, Hvt, nullptr, nullptr, true);
        HIPCHK(hipStreamWaitEvent(ctx->s, ctx->join, 0));
        spectral(ctx, 3, 3, Hvt, Hvt, nullptr);
        run(ctx, CL_K_VEC, [&] { launch_axpy(Hvt, Hvt, ctx->tmp3, 1.0f, 3 * ctx->N, ctx->s); });
    } else {
        // reduced form H vt = beta_v A vt + K b~, each term formed directly
        matvec(ctx, vt, Hvt, nullptr, nullptr, true);
        spectral(ctx, 3, 3, Hvt, Hvt, nullptr);
        spectral_scalar(ctx, 0, 3, vt, ctx->tmp3);
        run(ctx, CL_K_VEC, [&] { launch_axpy(Hvt, Hvt, ctx->tmp3, 1.0f, 3 * ctx->N, ctx->s); });
    }
    return CL_OK;
    API_END
}

int cl_precond_apply(cl_ctx *ctx, const float *r, float *z)
{
    NEED_CTX();
    if (!r || !z) return fail(ctx, CL_ERR_ARG, "NULL vector pointer");
    const size_t b = 3 * ctx->N * sizeof(float);
    if (overlap(r, b, z, b)) return fail(ctx, CL_ERR_ALIAS, "r and z overlap");
    if (ctx->opt.precond != CL_PRECOND_SPECTRAL && !ctx->images)
        return fail(ctx, CL_ERR_STATE, "the zero-velocity preconditioner needs the images");
    API_BEGIN
    precond(ctx, r, z);
    return CL_OK;
    API_END
}

int cl_solve(cl_ctx *ctx, cl_solve_report *rep)
{
    NEED_CTX();
    if (!ctx->images) return fail(ctx, CL_ERR_STATE, "cl_set_images has not been called");
    API_BEGIN
    return solve(ctx, nullptr, nullptr, 0, rep);
    API_END
}

int cl_solve_forced(cl_ctx *ctx, const int *forced_pcg, const double *forced_alpha, int n_outer,
                    cl_solve_report *rep)
{
    NEED_CTX();
    if (!forced_pcg || !forced_alpha || n_outer < 0) return fail(ctx, CL_ERR_ARG, "bad forced decisions");
    if (!ctx->images) return fail(ctx, CL_ERR_STATE, "cl_set_images has not been called");
    API_BEGIN
    return solve(ctx, forced_pcg, forced_alpha, n_outer, rep);
    API_END
}

int cl_get_solve_log(cl_ctx *ctx, double *rows, int max_rows, int *n_rows)
{
    NEED_CTX();
    if (n_rows) *n_rows = (int)ctx->log.size();
    if (rows)
        for (int r = 0; r < std::min(max_rows, (int)ctx->log.size()); ++r)
            for (int c = 0; c < 8; ++c) rows[8 * r + c] = ctx->log[r][c];
    return CL_OK;
}

int cl_set_regularization(cl_ctx *ctx, double beta_v, double beta_w)
{
    NEED_CTX();
    const int st = check_reg(beta_v, beta_w, ctx);
    if (st != CL_OK) return st;
    set_regularization(ctx, beta_v, beta_w);
    return CL_OK;
}

int cl_jacobian_det(cl_ctx *ctx, float *J_out, double *jmin, double *jmax)
{
    NEED_CTX();
    if (!ctx->vel) return fail(ctx, CL_ERR_STATE, "cl_set_velocity has not been called");
    API_BEGIN
    double lo = 0, hi = 0;
    jacobian(ctx, &lo, &hi, J_out);
    if (jmin) *jmin = lo;
    if (jmax) *jmax = hi;
    return CL_OK;
    API_END
}

void cl_default_search_options(cl_search_options *so)
{
    if (!so) return;
    std::memset(so, 0, sizeof(*so));
    so->jmin = 0.25;
    so->beta_v_max = 1.0;
    so->beta_v_min = 1e-5;
    so->beta_w_max = 1e-5;
    so->beta_w_min = 1e-7;
    so->rel_change = 0.1;
    so->search_beta_w = 1;
}

int cl_param_search(cl_ctx *ctx, const cl_search_options *so, cl_search_report *rep)
{
    NEED_CTX();
    const int st = check_search(so, ctx);
    if (st != CL_OK) return st;
    if (!ctx->images) return fail(ctx, CL_ERR_STATE, "cl_set_images has not been called");
    API_BEGIN
    return param_search(ctx, *so, rep);
    API_END
}

int cl_param_continuation(cl_ctx *ctx, const cl_search_options *so, double beta_v_target, double beta_w_target,
                          cl_search_report *rep)
{
    NEED_CTX();
    int st = check_search(so, ctx);
    if (st != CL_OK) return st;
    st = check_reg(beta_v_target, beta_w_target, ctx);
    if (st != CL_OK) return st;
    if (beta_w_target > so->beta_w_max) return fail(ctx, CL_ERR_ARG, "beta_w target above beta_w_max");
    if (!ctx->images) return fail(ctx, CL_ERR_STATE, "cl_set_images has not been called");
    API_BEGIN
    return param_continuation(ctx, *so, beta_v_target, beta_w_target, rep);
    API_END
}

int cl_get_search_log(cl_ctx *ctx, double *rows, int max_rows, int *n_rows)
{
    NEED_CTX();
    if (n_rows) *n_rows = (int)ctx->slog.size();
    if (rows)
        for (int r = 0; r < std::min(max_rows, (int)ctx->slog.size()); ++r)
            for (int c = 0; c < 10; ++c) rows[10 * r + c] = ctx->slog[r][c];
    return CL_OK;
}

int cl_deformed_template(cl_ctx *ctx, float *m_out)
{
    NEED_CTX();
    if (!m_out) return fail(ctx, CL_ERR_ARG, "NULL output pointer");
    if (!ctx->images) return fail(ctx, CL_ERR_STATE, "cl_set_images has not been called");
    API_BEGIN
    ensure_state(ctx);
    run(ctx, CL_K_VEC, [&] { launch_to_f32(ctx->dts, slot(ctx, ctx->m, ctx->dts, ctx->nt), m_out, ctx->N, ctx->s); });
    return CL_OK;
    API_END
}

int cl_get_field(cl_ctx *ctx, int which, int j, float *out)
{
    NEED_CTX();
    if (!out) return fail(ctx, CL_ERR_ARG, "NULL output pointer");
    if ((which <= CL_FIELD_INC_ADJOINT) && (j < 0 || j > ctx->nt)) return fail(ctx, CL_ERR_ARG, "time index out of range");
    API_BEGIN
    const size_t N = ctx->N;
    switch (which) {
    case CL_FIELD_STATE:
        run(ctx, CL_K_VEC, [&] { launch_to_f32(ctx->dts, slot(ctx, ctx->m, ctx->dts, j), out, N, ctx->s); });
        break;
    case CL_FIELD_ADJOINT:
    case CL_FIELD_INC_ADJOINT:
        run(ctx, CL_K_VEC, [&] { launch_to_f32(ctx->dta, slot(ctx, ctx->lam, ctx->dta, j), out, N, ctx->s); });
        break;
    case CL_FIELD_INC_STATE:
        if (j != ctx->nt) return fail(ctx, CL_ERR_ARG, "only mt^nt is kept");
        run(ctx, CL_K_VEC, [&] {   // mt^nt = -lam~^nt
            launch_to_f32(ctx->dta, slot(ctx, ctx->lam, ctx->dta, ctx->nt), out, N, ctx->s);
            launch_scale(out, out, -1.0f, N, ctx->s);
        });
        break;
    case CL_FIELD_FEET_F:
        run(ctx, CL_K_VEC, [&] { launch_feet_fields(ctx->g, ctx->df, out, ctx->s); });
        break;
    case CL_FIELD_FEET_B:
        run(ctx, CL_K_VEC, [&] { launch_feet_fields(ctx->g, ctx->db, out, ctx->s); });
        break;
    case CL_FIELD_ADJ_FACTOR:
        HIPCHK(hipMemcpyAsync(out, ctx->c, N * sizeof(float), hipMemcpyDeviceToDevice, ctx->s));
        break;
    default:
        return fail(ctx, CL_ERR_ARG, "unknown field");
    }
    return CL_OK;
    API_END
}

int cl_interp(cl_ctx *ctx, const float *u, const float *d, float *out)
{
    NEED_CTX();
    if (!u || !d || !out) return fail(ctx, CL_ERR_ARG, "NULL pointer");
    const size_t b = ctx->N * sizeof(float);
    if (overlap(u, b, out, b) || overlap(d, 3 * b, out, b)) return fail(ctx, CL_ERR_ALIAS, "output overlaps an input");
    API_BEGIN
    run(ctx, CL_K_SL_STATE, [&] { launch_interp_f32(ctx->g, u, d, ctx->box_t, out, ctx->s); });
    return CL_OK;
    API_END
}

} // extern "C"

// Scratch of cl_interp_noalloc: the per-tile stencil boxes (8 ints per tile
// of the tiled gather).  Each device holds its own copy until the process
// ends; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) int scratch[CL_NOALLOC_BOX_INTS];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex scratch_mu;
int *scratch_dev[NOALLOC_MAX_DEVICES] = {};

// device address of the current device's scratch (looked up once per device)
int scratch_address(int **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return CL_ERR_HIP;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CL_ERR_HIP;
        scratch_dev[dev] = (int *)p;
    }
    *out = scratch_dev[dev];
    return CL_OK;
}

} // namespace

extern "C" {

int cl_interp_noalloc(int n1, int n2, int n3, int interp_order, const float *u, const float *d, float *out,
                      void *stream)
{
    if (!u || !d || !out) return CL_ERR_ARG;
    if (interp_order != 1 && interp_order != 3) return CL_ERR_ARG;
    if (!pow2_ok(n1) || !pow2_ok(n2) || !pow2_ok(n3)) return CL_ERR_SHAPE;
    const Grid g = make_grid(n1, n2, n3, interp_order);
    if (tile_box_ints(g) > (size_t)CL_NOALLOC_BOX_INTS) return CL_ERR_OOM;
    const size_t b = (size_t)g.N * sizeof(float);
    if (overlap(u, b, out, b) || overlap(d, 3 * b, out, b)) return CL_ERR_ALIAS;
    int *boxes = nullptr;
    const int st = scratch_address(&boxes);
    if (st != CL_OK) return st;
    launch_interp_f32(g, u, d, boxes, out, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? CL_OK : CL_ERR_HIP;
}

int cl_fd_grad(cl_ctx *ctx, const float *u, float *gout)
{
    NEED_CTX();
    if (!u || !gout) return fail(ctx, CL_ERR_ARG, "NULL pointer");
    if (overlap(u, ctx->N * 4, gout, 3 * ctx->N * 4)) return fail(ctx, CL_ERR_ALIAS, "output overlaps input");
    API_BEGIN
    run(ctx, CL_K_FD, [&] { launch_fd_grad(ctx->g, u, gout, ctx->s); });
    return CL_OK;
    API_END
}

int cl_fd_div(cl_ctx *ctx, const float *v, float *out)
{
    NEED_CTX();
    if (!v || !out) return fail(ctx, CL_ERR_ARG, "NULL pointer");
    if (overlap(v, 3 * ctx->N * 4, out, ctx->N * 4)) return fail(ctx, CL_ERR_ALIAS, "output overlaps input");
    API_BEGIN
    run(ctx, CL_K_FD, [&] { launch_fd_div(ctx->g, v, out, ctx->s); });
    return CL_OK;
    API_END
}

int cl_spectral(cl_ctx *ctx, int kind, int ncomp, const float *in, float *out)
{
    NEED_CTX();
    if (!in || !out) return fail(ctx, CL_ERR_ARG, "NULL pointer");
    if (kind < 0 || kind > 3 || ncomp < 1) return fail(ctx, CL_ERR_ARG, "bad kind or ncomp");
    const size_t b = (size_t)ncomp * ctx->N * 4;
    if (overlap(in, b, out, b)) return fail(ctx, CL_ERR_ALIAS, "output overlaps input");
    API_BEGIN
    spectral(ctx, kind, ncomp, in, out, nullptr);
    return CL_OK;
    API_END
}

int cl_dot(cl_ctx *ctx, const float *a, const float *b, size_t n, double *out)
{
    NEED_CTX();
    if (!a || !b || !out) return fail(ctx, CL_ERR_ARG, "NULL pointer");
    API_BEGIN
    const int nb = std::min(ctx->nparts, reduce_blocks(n));
    run(ctx, CL_K_VEC, [&] {
        launch_dot(a, b, n, ctx->partials, nb, ctx->s);
        launch_finalize(ctx->partials, nb, ctx->hv, ctx->dscal, ctx->s);
    });
    *out = read_scalar(ctx);
    return CL_OK;
    API_END
}

int cl_copy_f32(cl_ctx *ctx, const float *src, float *dst, size_t n)
{
    NEED_CTX();
    if (!src || !dst) return fail(ctx, CL_ERR_ARG, "NULL pointer");
    if (overlap(src, n * 4, dst, n * 4)) return fail(ctx, CL_ERR_ALIAS, "copy buffers overlap");
    API_BEGIN
    run(ctx, CL_K_VEC, [&] { launch_copy_f32(src, dst, n, ctx->s); });
    return CL_OK;
    API_END
}

int cl_profile_enable(cl_ctx *ctx, unsigned mask)
{
    NEED_CTX();
    API_BEGIN
    prof_drain(ctx);
    ctx->prof.mask = mask;
    for (int k = 0; k < CL_K_COUNT; ++k) { ctx->prof.ms[k] = 0.0; ctx->prof.n[k] = 0; }
    return CL_OK;
    API_END
}

int cl_profile_query(cl_ctx *ctx, int kclass, double *ms_total, long long *launches)
{
    NEED_CTX();
    if (kclass < 0 || kclass >= CL_K_COUNT) return fail(ctx, CL_ERR_ARG, "bad kernel class");
    API_BEGIN
    prof_drain(ctx);
    if (ms_total) *ms_total = ctx->prof.ms[kclass];
    if (launches) *launches = ctx->prof.n[kclass];
    return CL_OK;
    API_END
}

const char *cl_kernel_class_name(int k)
{
    static const char *names[CL_K_COUNT] = {"feet", "sl_state", "sl_adjoint", "sl_inc", "fd", "quadrature", "fft", "vec"};
    return (k >= 0 && k < CL_K_COUNT) ? names[k] : "unknown";
}

const char *cl_status_string(int s)
{
    switch (s) {
    case CL_OK: return "ok";
    case CL_ERR_ARG: return "invalid argument";
    case CL_ERR_SHAPE: return "unsupported grid shape";
    case CL_ERR_DTYPE: return "unsupported dtype";
    case CL_ERR_OOM: return "out of device memory / workspace cap";
    case CL_ERR_HIP: return "HIP runtime error";
    case CL_ERR_NONFINITE: return "non-finite input";
    case CL_ERR_UNSUPPORTED: return "unsupported option";
    case CL_ERR_STATE: return "call order violated";
    case CL_ERR_ALIAS: return "buffers overlap";
    case CL_STATUS_MAXIT: return "iteration limit reached";
    case CL_STATUS_LINESEARCH_FAIL: return "line search failed";
    default: return "unknown status";
    }
}

const char *cl_last_error(const cl_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

} // extern "C"
