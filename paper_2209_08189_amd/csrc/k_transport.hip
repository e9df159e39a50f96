// k_transport.hip -- semi-Lagrangian transport kernels for gfx950:
// RK2 characteristic feet and the tricubic Lagrange gather for the state,
// adjoint and incremental-state steps (Section 2.2, semi-Lagrangian scheme;
// Section 3, IP kernel, cubic Lagrange variant).
//
// One thread per output node, 256-thread workgroups walking the field in
// memory order, so a wavefront covers 64 consecutive x3 nodes and its 64
// stencil rows are contiguous runs that the vector L1/L2 caches share
// between neighbouring lanes and neighbouring workgroups.
#include "internal.h"

namespace clh {

namespace {

constexpr int TPB = 256;

// Cubic Lagrange weights of the nodes base-1..base+2 at fraction f in [0,1).
// At f = 0 they are exactly (0, 1, 0, 0).
__device__ __forceinline__ void lagrange4(float f, float w[4])
{
    const float fm1 = f - 1.0f, fm2 = f - 2.0f, fp1 = f + 1.0f;
    w[0] = -f * fm1 * fm2 * (1.0f / 6.0f);
    w[1] = fp1 * fm1 * fm2 * 0.5f;
    w[2] = -fp1 * f * fm2 * 0.5f;
    w[3] = fp1 * f * fm1 * (1.0f / 6.0f);
}

// Stencil of one foot: row offsets of the 4 x1 planes, 4 x2 rows, 4 x3
// columns (periodic wrap by masking) and the separable weights.  The
// integer part of the foot is node + floor(d), the fraction d - floor(d),
// both from the displacement alone so FP32 keeps full relative precision
// of d at any grid size.
struct Foot {
    int o1[4], o2[4], o3[4];
    float w1[4], w2[4], w3[4];
};

__device__ __forceinline__ void make_foot(const Grid &g, int i, int j, int k, float d1, float d2, float d3, Foot &F)
{
    const float f1 = floorf(d1), f2 = floorf(d2), f3 = floorf(d3);
    lagrange4(d1 - f1, F.w1);
    lagrange4(d2 - f2, F.w2);
    lagrange4(d3 - f3, F.w3);
    const int b1 = i + (int)f1 - 1, b2 = j + (int)f2 - 1, b3 = k + (int)f3 - 1;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        F.o1[a] = ((b1 + a) & (g.n1 - 1)) << (g.l2 + g.l3);
        F.o2[a] = ((b2 + a) & (g.n2 - 1)) << g.l3;
        F.o3[a] = (b3 + a) & (g.n3 - 1);
    }
}

template <typename T>
__device__ __forceinline__ float gather(const T *__restrict__ u, const Foot &F)
{
    float s = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        float sa = 0.0f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const T *row = u + (F.o1[a] + F.o2[b]);
            float t = F.w3[0] * ldf(row + F.o3[0]);
            t = fmaf(F.w3[1], ldf(row + F.o3[1]), t);
            t = fmaf(F.w3[2], ldf(row + F.o3[2]), t);
            t = fmaf(F.w3[3], ldf(row + F.o3[3]), t);
            sa = fmaf(F.w2[b], t, sa);
        }
        s = fmaf(F.w1[a], sa, s);
    }
    return s;
}

__device__ __forceinline__ void gather3(const float *__restrict__ u0, const float *__restrict__ u1,
                                        const float *__restrict__ u2, const Foot &F, float out[3])
{
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r = F.o1[a] + F.o2[b];
            float t0 = 0.f, t1 = 0.f, t2 = 0.f;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                t0 = fmaf(F.w3[c], u0[r + F.o3[c]], t0);
                t1 = fmaf(F.w3[c], u1[r + F.o3[c]], t1);
                t2 = fmaf(F.w3[c], u2[r + F.o3[c]], t2);
            }
            a0 = fmaf(F.w2[b], t0, a0);
            a1 = fmaf(F.w2[b], t1, a1);
            a2 = fmaf(F.w2[b], t2, a2);
        }
        s0 = fmaf(F.w1[a], a0, s0);
        s1 = fmaf(F.w1[a], a1, s1);
        s2 = fmaf(F.w1[a], a2, s2);
    }
    out[0] = s0; out[1] = s1; out[2] = s2;
}

// ------------------------------------------------------------- kernels

// RK2 (Heun) feet of both characteristic directions, as index-unit
// displacements:  X_f = x - dt/2 [v(x) + v(x - dt v(x))],
//                 X_b = x + dt/2 [v(x) + v(x + dt v(x))].
// If db != NULL also the adjoint factor c = 1 + dt/2 (dbar + d + dt dbar d),
// d = div_h v (precomputed), dbar = d(X_b).
__global__ __launch_bounds__(TPB) void k_feet(Grid g, float dt, const float *__restrict__ v,
                                              float *__restrict__ df, float *__restrict__ db,
                                              const float *__restrict__ divv, float *__restrict__ c)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    int i, j, k;
    node_of(g, p, i, j, k);
    const float *v0 = v, *v1 = v + g.N, *v2 = v + 2 * (size_t)g.N;
    const float a0 = v0[p], a1 = v1[p], a2 = v2[p];
    // Displacements divide by h (correctly rounded), so a velocity that is an
    // exact multiple of h/dt gives an exactly integer foot.
    const float h[3] = {g.h1, g.h2, g.h3};
    const float va[3] = {a0, a1, a2};
    Foot F;
    float vi[3];
    make_foot(g, i, j, k, (-dt * a0) / g.h1, (-dt * a1) / g.h2, (-dt * a2) / g.h3, F);
    gather3(v0, v1, v2, F, vi);
#pragma unroll
    for (int a = 0; a < 3; ++a) df[a * (size_t)g.N + p] = (-0.5f * dt * (va[a] + vi[a])) / h[a];
    if (!db) return;
    make_foot(g, i, j, k, (dt * a0) / g.h1, (dt * a1) / g.h2, (dt * a2) / g.h3, F);
    gather3(v0, v1, v2, F, vi);
    float dbv[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dbv[a] = (0.5f * dt * (va[a] + vi[a])) / h[a];
        db[a * (size_t)g.N + p] = dbv[a];
    }
    if (!c) return;
    make_foot(g, i, j, k, dbv[0], dbv[1], dbv[2], F);
    const float dbar = gather(divv, F);
    const float d = divv[p];
    c[p] = 1.0f + 0.5f * dt * (dbar + d + dt * dbar * d);
}

template <typename Tu, typename To>
__global__ __launch_bounds__(TPB) void k_sl_state(Grid g, const Tu *__restrict__ u, const float *__restrict__ d,
                                                  To *__restrict__ out)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    int i, j, k;
    node_of(g, p, i, j, k);
    Foot F;
    make_foot(g, i, j, k, d[p], d[g.N + p], d[2 * (size_t)g.N + p], F);
    stf(out + p, gather(u, F));
}

template <typename Tu, typename To>
__global__ __launch_bounds__(TPB) void k_sl_adjoint(Grid g, const Tu *__restrict__ u, const float *__restrict__ d,
                                                    const float *__restrict__ c, To *__restrict__ out)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    int i, j, k;
    node_of(g, p, i, j, k);
    Foot F;
    make_foot(g, i, j, k, d[p], d[g.N + p], d[2 * (size_t)g.N + p], F);
    stf(out + p, c[p] * gather(u, F));
}

template <typename Tq, typename Tm>
__global__ __launch_bounds__(TPB) void k_sl_inc(Grid g, const Tq *__restrict__ q, const float *__restrict__ d,
                                                const Tm *__restrict__ m, const float *__restrict__ vt,
                                                float sI, float sS, Tq *__restrict__ out)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    int i, j, k;
    node_of(g, p, i, j, k);
    Foot F;
    make_foot(g, i, j, k, d[p], d[g.N + p], d[2 * (size_t)g.N + p], F);
    const float gi = gather(q, F);
    const float g1 = fd8(m, p, i, g.n1, g.n2 * g.n3, g.ih1);
    const float g2 = fd8(m, p, j, g.n2, g.n3, g.ih2);
    const float g3 = fd8(m, p, k, g.n3, 1, g.ih3);
    const float src = -(vt[p] * g1 + vt[g.N + p] * g2 + vt[2 * (size_t)g.N + p] * g3);
    stf(out + p, sI * gi + sS * src);
}

inline dim3 grid_of(const Grid &g) { return dim3((g.N + TPB - 1) / TPB); }

} // namespace

void launch_feet(const Grid &g, float dt, const float *v, float *df, float *db, const float *divv, float *c,
                 hipStream_t s)
{
    hipLaunchKernelGGL(k_feet, grid_of(g), dim3(TPB), 0, s, g, dt, v, df, db, divv, c);
}

void launch_sl_state(const Grid &g, int dt_u, const void *u, const float *d, int dt_out, void *out, hipStream_t s)
{
    with_dtype(dt_u, [&](auto tu) {
        using Tu = decltype(tu);
        with_dtype(dt_out, [&](auto to) {
            using To = decltype(to);
            hipLaunchKernelGGL((k_sl_state<Tu, To>), grid_of(g), dim3(TPB), 0, s, g, (const Tu *)u, d, (To *)out);
        });
    });
}

void launch_sl_adjoint(const Grid &g, int dt_u, const void *u, const float *d, const float *c, int dt_out,
                       void *out, hipStream_t s)
{
    with_dtype(dt_u, [&](auto tu) {
        using Tu = decltype(tu);
        with_dtype(dt_out, [&](auto to) {
            using To = decltype(to);
            hipLaunchKernelGGL((k_sl_adjoint<Tu, To>), grid_of(g), dim3(TPB), 0, s, g, (const Tu *)u, d, c,
                               (To *)out);
        });
    });
}

void launch_sl_inc(const Grid &g, int dt_q, const void *q, const float *d, int dt_m, const void *m,
                   const float *vt, float sI, float sS, void *out, hipStream_t s)
{
    with_dtype(dt_q, [&](auto tq) {
        using Tq = decltype(tq);
        with_dtype(dt_m, [&](auto tm) {
            using Tm = decltype(tm);
            hipLaunchKernelGGL((k_sl_inc<Tq, Tm>), grid_of(g), dim3(TPB), 0, s, g, (const Tq *)q, d,
                               (const Tm *)m, vt, sI, sS, (Tq *)out);
        });
    });
}

void launch_interp_f32(const Grid &g, const float *u, const float *d, float *out, hipStream_t s)
{
    hipLaunchKernelGGL((k_sl_state<float, float>), grid_of(g), dim3(TPB), 0, s, g, u, d, out);
}

} // namespace clh
