// k_stencil.hip -- 8th-order finite-difference kernels (Section 2.2 and
// Section 3, FD kernel) and the fused consumers of FD8 gradients: the
// incremental source, the trapezoid time quadrature of the gradient and
// Hessian bodies, and the adjoint final condition with its mismatch
// reduction.  One thread per node in memory order; the +-4 neighbours along
// x1/x2 are re-read from L2 by neighbouring workgroups.
#include "internal.h"

namespace clh {

namespace {

constexpr int TPB = 256;

inline dim3 grid_of(const Grid &g) { return dim3((g.N + TPB - 1) / TPB); }

template <typename T>
__device__ __forceinline__ void grad_at(const Grid &g, const T *u, int p, float out[3])
{
    int i, j, k;
    node_of(g, p, i, j, k);
    out[0] = fd8(u, p, i, g.n1, g.n2 * g.n3, g.ih1);
    out[1] = fd8(u, p, j, g.n2, g.n3, g.ih2);
    out[2] = fd8(u, p, k, g.n3, 1, g.ih3);
}

__global__ __launch_bounds__(TPB) void k_fd_grad(Grid g, const float *__restrict__ u, float *__restrict__ out)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    float gr[3];
    grad_at(g, u, p, gr);
    out[p] = gr[0];
    out[g.N + p] = gr[1];
    out[2 * (size_t)g.N + p] = gr[2];
}

__global__ __launch_bounds__(TPB) void k_fd_div(Grid g, const float *__restrict__ v, float *__restrict__ out)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    int i, j, k;
    node_of(g, p, i, j, k);
    const float d1 = fd8(v, p, i, g.n1, g.n2 * g.n3, g.ih1);
    const float d2 = fd8(v + g.N, p, j, g.n2, g.n3, g.ih2);
    const float d3 = fd8(v + 2 * (size_t)g.N, p, k, g.n3, 1, g.ih3);
    out[p] = d1 + d2 + d3;
}

template <typename Tm, typename Tq>
__global__ __launch_bounds__(TPB) void k_inc_init(Grid g, const Tm *__restrict__ m0, const float *__restrict__ vt,
                                                  float scale, Tq *__restrict__ q0)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    float gr[3];
    grad_at(g, m0, p, gr);
    const float s = -(vt[p] * gr[0] + vt[g.N + p] * gr[1] + vt[2 * (size_t)g.N + p] * gr[2]);
    stf(q0 + p, scale * s);
}

template <typename Tl, typename Tm>
__global__ __launch_bounds__(TPB) void k_quadrature(Grid g, QuadArgs qa, const float *__restrict__ add,
                                                    float *__restrict__ out)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    float b0 = 0.f, b1 = 0.f, b2 = 0.f;
    for (int t = 0; t < qa.count; ++t) {
        float gr[3];
        grad_at(g, (const Tm *)qa.m[t], p, gr);
        const float wl = qa.w[t] * ldf((const Tl *)qa.lam[t] + p);
        b0 = fmaf(wl, gr[0], b0);
        b1 = fmaf(wl, gr[1], b1);
        b2 = fmaf(wl, gr[2], b2);
    }
    if (add) {
        b0 += add[p];
        b1 += add[g.N + p];
        b2 += add[2 * (size_t)g.N + p];
    }
    out[p] = b0;
    out[g.N + p] = b1;
    out[2 * (size_t)g.N + p] = b2;
}

// lam^nt = m1 - m^nt and per-block partial sums of its square, grid-stride.
template <typename Tm, typename Tl>
__global__ __launch_bounds__(TPB) void k_residual(Grid g, const Tm *__restrict__ m1, const Tm *__restrict__ mN,
                                                  Tl *__restrict__ lam, double *__restrict__ partials)
{
    double acc = 0.0;
    for (int p = blockIdx.x * TPB + threadIdx.x; p < g.N; p += gridDim.x * TPB) {
        const float r = ldf(m1 + p) - ldf(mN + p);
        if (lam) stf(lam + p, r);
        acc += (double)r * (double)r;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

} // namespace

void launch_fd_grad(const Grid &g, const float *u, float *out3, hipStream_t s)
{
    hipLaunchKernelGGL(k_fd_grad, grid_of(g), dim3(TPB), 0, s, g, u, out3);
}

void launch_fd_div(const Grid &g, const float *v, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_fd_div, grid_of(g), dim3(TPB), 0, s, g, v, out);
}

void launch_inc_init(const Grid &g, int dt_m, const void *m0, const float *vt, float scale, int dt_q, void *q0,
                     hipStream_t s)
{
    with_dtype(dt_m, [&](auto tm) {
        using Tm = decltype(tm);
        with_dtype(dt_q, [&](auto tq) {
            using Tq = decltype(tq);
            hipLaunchKernelGGL((k_inc_init<Tm, Tq>), grid_of(g), dim3(TPB), 0, s, g, (const Tm *)m0, vt, scale,
                               (Tq *)q0);
        });
    });
}

void launch_quadrature(const Grid &g, int dt_lam, int dt_m, const QuadArgs &qa, const float *addend3, float *out3,
                       hipStream_t s)
{
    with_dtype(dt_lam, [&](auto tl) {
        using Tl = decltype(tl);
        with_dtype(dt_m, [&](auto tm) {
            using Tm = decltype(tm);
            hipLaunchKernelGGL((k_quadrature<Tl, Tm>), grid_of(g), dim3(TPB), 0, s, g, qa, addend3, out3);
        });
    });
}

void launch_residual(const Grid &g, int dt_m, const void *m1, const void *mN, int dt_lam, void *lam,
                     double *partials, int nblocks, hipStream_t s)
{
    with_dtype(dt_m, [&](auto tm) {
        using Tm = decltype(tm);
        with_dtype(dt_lam, [&](auto tl) {
            using Tl = decltype(tl);
            hipLaunchKernelGGL((k_residual<Tm, Tl>), dim3(nblocks), dim3(TPB), 0, s, g, (const Tm *)m1,
                               (const Tm *)mN, (Tl *)lam, partials);
        });
    });
}

void launch_sq_diff(const Grid &g, int dt_m, const void *a, const void *b, double *partials, int nblocks,
                    hipStream_t s)
{
    with_dtype(dt_m, [&](auto tm) {
        using Tm = decltype(tm);
        hipLaunchKernelGGL((k_residual<Tm, float>), dim3(nblocks), dim3(TPB), 0, s, g, (const Tm *)a,
                           (const Tm *)b, (float *)nullptr, partials);
    });
}

} // namespace clh
