// k_stencil.hip -- 8th-order finite-difference kernels (Section 2.2 and
// Section 3, FD kernel) and the fused consumers of FD8 gradients: the
// incremental source, the trapezoid time quadrature of the gradient and
// Hessian bodies, and the adjoint final condition with its mismatch
// reduction.  One thread per node in memory order; the +-4 neighbours along
// x1/x2 are re-read from L2 by neighbouring workgroups.
#include "internal.h"

#include <type_traits>

#include <algorithm>

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

// G^j = grad_h m^j for every stored time point j = blockIdx.y.
template <typename Tm>
__global__ __launch_bounds__(TPB) void k_state_grad(Grid g, StateGradArgs a)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    const int t = blockIdx.y;
    float gr[3];
    grad_at(g, (const Tm *)a.m[t], p, gr);
    float *G = a.G[t];
    G[p] = gr[0];
    G[g.N + p] = gr[1];
    G[2 * (size_t)g.N + p] = gr[2];
}

// incremental sources s^j = -vt . G^j for j = 0..nt, four nodes per thread:
// q0 = scale * s^0, S_j = s^j (j >= 1).  vt is read once for all times.
template <typename Tq>
__global__ __launch_bounds__(TPB) void k_inc_sources(Grid g, const float *__restrict__ G, const float *__restrict__ vt,
                                                     int nt, float scale, Tq *__restrict__ q0, float *__restrict__ S)
{
    const size_t N = g.N;
    const int p = (blockIdx.x * TPB + threadIdx.x) * 4;
    if (p >= g.N) return;
    const float4 v0 = *(const float4 *)(vt + p), v1 = *(const float4 *)(vt + N + p), v2 = *(const float4 *)(vt + 2 * N + p);
    for (int t = 0; t <= nt; ++t) {
        const float *Gt = G + 3 * N * t;
        const float4 g0 = *(const float4 *)(Gt + p), g1 = *(const float4 *)(Gt + N + p),
                     g2 = *(const float4 *)(Gt + 2 * N + p);
        float4 r;
        r.x = -(v0.x * g0.x + v1.x * g1.x + v2.x * g2.x);
        r.y = -(v0.y * g0.y + v1.y * g1.y + v2.y * g2.y);
        r.z = -(v0.z * g0.z + v1.z * g1.z + v2.z * g2.z);
        r.w = -(v0.w * g0.w + v1.w * g1.w + v2.w * g2.w);
        if (t == 0) {
            stf(q0 + p + 0, scale * r.x);
            stf(q0 + p + 1, scale * r.y);
            stf(q0 + p + 2, scale * r.z);
            stf(q0 + p + 3, scale * r.w);
        } else {
            *(float4 *)(S + N * (t - 1) + p) = r;
        }
    }
}

template <typename T> __device__ __forceinline__ float4 ld4(const T *p)
{
    return make_float4(ldf(p), ldf(p + 1), ldf(p + 2), ldf(p + 3));
}
template <> __device__ __forceinline__ float4 ld4<float>(const float *p) { return *(const float4 *)p; }

// out3 = add3 + sum_j w_j lam^j G^j, four nodes per thread (streaming).
// With dp != NULL also the per-block FP64 partial sums of dp . out3 (from
// the FP32 values stored), one per block in partials[blockIdx.x].
template <typename Tl>
__global__ __launch_bounds__(TPB) void k_quadrature(Grid g, QuadArgs qa, const float *__restrict__ add,
                                                    float *__restrict__ out, const float *__restrict__ dp,
                                                    double *__restrict__ partials)
{
    const size_t N = g.N;
    const int p = (blockIdx.x * TPB + threadIdx.x) * 4;
    double acc = 0.0;
    if (p < g.N) {
        float4 b0 = make_float4(0.f, 0.f, 0.f, 0.f), b1 = b0, b2 = b0;
        for (int t = 0; t < qa.count; ++t) {
            const float4 l = ld4((const Tl *)qa.lam[t] + p);
            const float w = qa.w[t];
            const float4 wl = make_float4(w * l.x, w * l.y, w * l.z, w * l.w);
            const float *G = qa.G[t];
            const float4 g0 = *(const float4 *)(G + p), g1 = *(const float4 *)(G + N + p),
                         g2 = *(const float4 *)(G + 2 * N + p);
            b0.x = fmaf(wl.x, g0.x, b0.x); b0.y = fmaf(wl.y, g0.y, b0.y); b0.z = fmaf(wl.z, g0.z, b0.z); b0.w = fmaf(wl.w, g0.w, b0.w);
            b1.x = fmaf(wl.x, g1.x, b1.x); b1.y = fmaf(wl.y, g1.y, b1.y); b1.z = fmaf(wl.z, g1.z, b1.z); b1.w = fmaf(wl.w, g1.w, b1.w);
            b2.x = fmaf(wl.x, g2.x, b2.x); b2.y = fmaf(wl.y, g2.y, b2.y); b2.z = fmaf(wl.z, g2.z, b2.z); b2.w = fmaf(wl.w, g2.w, b2.w);
        }
        if (add) {
            const float4 a0 = *(const float4 *)(add + p), a1 = *(const float4 *)(add + N + p),
                         a2 = *(const float4 *)(add + 2 * N + p);
            b0.x += a0.x; b0.y += a0.y; b0.z += a0.z; b0.w += a0.w;
            b1.x += a1.x; b1.y += a1.y; b1.z += a1.z; b1.w += a1.w;
            b2.x += a2.x; b2.y += a2.y; b2.z += a2.z; b2.w += a2.w;
        }
        *(float4 *)(out + p) = b0;
        *(float4 *)(out + N + p) = b1;
        *(float4 *)(out + 2 * N + p) = b2;
        if (dp) {
            const float4 d0 = *(const float4 *)(dp + p), d1 = *(const float4 *)(dp + N + p),
                         d2 = *(const float4 *)(dp + 2 * N + p);
            acc = (double)d0.x * b0.x + (double)d0.y * b0.y + (double)d0.z * b0.z + (double)d0.w * b0.w;
            acc += (double)d1.x * b1.x + (double)d1.y * b1.y + (double)d1.z * b1.z + (double)d1.w * b1.w;
            acc += (double)d2.x * b2.x + (double)d2.y * b2.y + (double)d2.z * b2.z + (double)d2.w * b2.w;
        }
    }
    if (dp) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) partials[blockIdx.x] = acc;
    }
}

// Lean layout (no stored gradients): the same quadrature with grad_h m^j
// taken by FD8 in the kernel, four consecutive x3 nodes per thread.
template <typename Tm, typename Tl>
__global__ __launch_bounds__(TPB) void k_quadrature_fd(Grid g, QuadArgs qa, const float *__restrict__ add,
                                                       float *__restrict__ out, const float *__restrict__ dp,
                                                       double *__restrict__ partials)
{
    const size_t N = g.N;
    const int p0 = (blockIdx.x * TPB + threadIdx.x) * 4;
    double acc = 0.0;
    if (p0 < g.N) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int p = p0 + u;
            float b0 = 0.f, b1 = 0.f, b2 = 0.f;
            for (int t = 0; t < qa.count; ++t) {
                const float wl = qa.w[t] * ldf((const Tl *)qa.lam[t] + p);
                float gr[3];
                grad_at(g, (const Tm *)qa.m[t], p, gr);
                b0 = fmaf(wl, gr[0], b0);
                b1 = fmaf(wl, gr[1], b1);
                b2 = fmaf(wl, gr[2], b2);
            }
            if (add) {
                b0 += add[p];
                b1 += add[N + p];
                b2 += add[2 * N + p];
            }
            out[p] = b0;
            out[N + p] = b1;
            out[2 * N + p] = b2;
            if (dp) acc += (double)dp[p] * b0 + (double)dp[N + p] * b1 + (double)dp[2 * N + p] * b2;
        }
    }
    if (dp) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) partials[blockIdx.x] = acc;
    }
}

// Lean layout: out = scale * (-vt . grad_h m), FD8 in the kernel.
template <typename Tm, typename To>
__global__ __launch_bounds__(TPB) void k_inc_source_fd(Grid g, const Tm *__restrict__ m, const float *__restrict__ vt,
                                                       float scale, To *__restrict__ out)
{
    const size_t N = g.N;
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    float gr[3];
    grad_at(g, m, p, gr);
    const float r = -(vt[p] * gr[0] + vt[N + p] * gr[1] + vt[2 * N + p] * gr[2]);
    stf(out + p, scale * r);
}

// ------------------------------------------------ FD8 by marching along x1
// Lean-layout consumers of grad_h m on grids whose +-4 planes along x1 do not
// stay in L2 (a plane of a 1024^3 grid is 4 MiB): a block owns a 64 (x3) by
// 8 (x2) tile of nodes, one per thread, and walks a chunk of planes along x1.
// Each thread keeps m(i-4 .. i+4) at its (x2, x3) position in registers and
// loads one new plane per step, so m is read from HBM once per chunk (plus 8
// halo planes); the current plane with a 4-node halo in x2 and x3 is staged
// in LDS for the other two derivatives (two buffers: one barrier per step).
// Every derivative is the same expression, in the same order, as fd8().
constexpr int MX = 64, MY = 8, MH = 4;
constexpr int MPX = MX + 2 * MH, MPY = MY + 2 * MH;    // staged plane 72 x 16
constexpr int TPB_M = MX * MY;                         // 512 threads, wave w = row w
constexpr int MAX_NL = 5;                              // time levels kept in registers

struct MarchGeom {
    int ntx, nty;   // tiles along x3 and x2
    int nch;        // chunks per tile column: chunk c covers planes [c n1 / nch, (c + 1) n1 / nch)
};

__device__ __forceinline__ float fd8_ring(const float *u, float ih)   // u[4] is the centre
{
    float s = 0.8f * (u[5] - u[3]);
    s = fmaf(-0.2f, u[6] - u[2], s);
    s = fmaf(4.0f / 105.0f, u[7] - u[1], s);
    s = fmaf(-1.0f / 280.0f, u[8] - u[0], s);
    return s * ih;
}

__device__ __forceinline__ float fd8_lds(const float *c, int st, float ih)   // c -> centre, stride st
{
    float s = 0.8f * (c[st] - c[-st]);
    s = fmaf(-0.2f, c[2 * st] - c[-2 * st], s);
    s = fmaf(4.0f / 105.0f, c[3 * st] - c[-3 * st], s);
    s = fmaf(-1.0f / 280.0f, c[4 * st] - c[-4 * st], s);
    return s * ih;
}

// MODE 0: out3 = add + sum_t w_t lam^t grad_h m^t (NL = qa.count levels),
//         optional FP64 partials of dp . out3 per block.
// MODE 1: out1 = scale * (-vt . grad_h m^0) (NL = 1).
// MODE 2: the incremental sources of every level at once, s^t = -vt .
//         grad_h m^t: out1 = scale * s^0, out3[(t - 1) N ..] = s^t, t >= 1.
template <typename Tm, typename Tl, typename To, int NL, int MODE>
__global__ __launch_bounds__(TPB_M) void k_fd_march(Grid g, MarchGeom mg, QuadArgs qa, const float *__restrict__ add,
                                                    float *__restrict__ out3, const float *__restrict__ dp,
                                                    double *__restrict__ partials, const float *__restrict__ vt,
                                                    float scale, To *__restrict__ out1)
{
    __shared__ float pl[2][NL][MPY][MPX];
    const unsigned N = (unsigned)g.N;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // XCD-aware order: each XCD takes a contiguous range of tiles, so the
    // x2 neighbours of a tile run on the same L2
    int b = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
    const int tx = b % mg.ntx;
    b /= mg.ntx;
    const int ty = b % mg.nty;
    const int c = b / mg.nty;
    const int i0 = (int)(((long)c * g.n1) / mg.nch);
    const int len = (int)(((long)(c + 1) * g.n1) / mg.nch) - i0;
    const int l23 = g.l2 + g.l3, m1 = g.n1 - 1;
    const int k = tx * MX + lane, j = ty * MY + w;
    // element offsets inside a plane (unsigned: every access below is a
    // wave-uniform field base plus a 32-bit offset)
    const unsigned col = ((unsigned)j << g.l3) + k;
    const int hr = w < MH ? w - MH : w + MH;                             // x2 halo row of this thread
    const unsigned hcol = ((unsigned)((ty * MY + hr) & (g.n2 - 1)) << g.l3) + k;
    const bool xh = lane < 2 * MH;                                       // lanes that load the x3 halo
    const int xc = lane < MH ? lane - MH : MX + lane - MH;
    const unsigned xcol = ((unsigned)j << g.l3) + ((tx * MX + xc) & (g.n3 - 1));
    auto plane = [&](int i) { return (unsigned)(i & m1) << l23; };
    const Tm *mp[NL];
#pragma unroll
    for (int t = 0; t < NL; ++t) mp[t] = (const Tm *)qa.m[t];
    const float *add1 = add ? add + N : nullptr, *add2 = add ? add + 2 * (size_t)N : nullptr;
    const float *vt1 = vt ? vt + N : nullptr, *vt2 = vt ? vt + 2 * (size_t)N : nullptr;

    // prefetched values stay at storage precision until they are used, so a
    // 16-bit load does not have to complete before the next one is issued
    float ring[NL][9];
    Tm nxt[NL], hv[NL], xv[NL];
#pragma unroll
    for (int t = 0; t < NL; ++t) {
#pragma unroll
        for (int s = 0; s < 8; ++s) ring[t][s] = tof(at(mp[t], plane(i0 - MH + s) + col));
        const unsigned base = plane(i0);
        hv[t] = at(mp[t], base + hcol);
        if (xh) xv[t] = at(mp[t], base + xcol);                     // used by the x3-halo lanes only
        nxt[t] = at(mp[t], plane(i0 + MH) + col);
    }
    // operands of a plane's epilogue (lam^t weighted and the addend, or vt),
    // requested one plane ahead like the stencil values
    // lam^t: FP32 values are weighted when they arrive; 16-bit values are kept
    // raw until the plane that uses them
    typedef typename std::conditional<sizeof(Tl) == 4, float, Tl>::type LamT;
    LamT nlam[NL];
    float ne0, ne1, ne2;
    auto epilogue_operands = [&](unsigned pp) {
        if (MODE == 0) {
#pragma unroll
            for (int t = 0; t < NL; ++t) {
                if constexpr (sizeof(Tl) == 4)
                    nlam[t] = qa.w[t] * tof(at((const Tl *)qa.lam[t], pp));
                else
                    nlam[t] = at((const Tl *)qa.lam[t], pp);
            }
            ne0 = add ? at(add, pp) : 0.f;
            ne1 = add ? at(add1, pp) : 0.f;
            ne2 = add ? at(add2, pp) : 0.f;
        } else {
            ne0 = at(vt, pp);
            ne1 = at(vt1, pp);
            ne2 = at(vt2, pp);
        }
    };
    epilogue_operands(plane(i0) + col);
    double acc = 0.0;
    for (int step = 0; step < len; ++step) {
        const int i = i0 + step;
        const int buf = step & 1;
        const unsigned p = plane(i) + col;
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            ring[t][8] = tof(nxt[t]);
            pl[buf][t][w + MH][lane + MH] = ring[t][4];
            pl[buf][t][hr + MH][lane + MH] = tof(hv[t]);
            if (xh) pl[buf][t][w + MH][xc + MH] = tof(xv[t]);
        }
        float lw[NL];
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            if constexpr (sizeof(Tl) == 4)
                lw[t] = MODE == 0 ? nlam[t] : 0.f;
            else
                lw[t] = MODE == 0 ? qa.w[t] * tof(nlam[t]) : 0.f;
        }
        const float e0 = ne0, e1 = ne1, e2 = ne2;
        __syncthreads();
        // prefetch the next plane's halo, the plane i + 5 of the ring and the
        // next plane's epilogue operands
        if (step + 1 < len) {
            const unsigned nbase = plane(i + 1);
            const unsigned rbase = plane(i + 1 + MH);
#pragma unroll
            for (int t = 0; t < NL; ++t) {
                hv[t] = at(mp[t], nbase + hcol);
                if (xh) xv[t] = at(mp[t], nbase + xcol);
                nxt[t] = at(mp[t], rbase + col);
            }
            epilogue_operands(nbase + col);
        }
        float b0 = 0.f, b1 = 0.f, b2 = 0.f;
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            const float *c = &pl[buf][t][w + MH][lane + MH];
            const float d0 = fd8_ring(ring[t], g.ih1);
            const float d1 = fd8_lds(c, MPX, g.ih2);
            const float d2 = fd8_lds(c, 1, g.ih3);
            if (MODE == 0) {
                b0 = fmaf(lw[t], d0, b0);
                b1 = fmaf(lw[t], d1, b1);
                b2 = fmaf(lw[t], d2, b2);
            } else if (MODE == 2) {
                const float sv = -(e0 * d0 + e1 * d1 + e2 * d2);
                if (t == 0) stf(&at(out1, p), scale * sv);
                else at(out3 + (size_t)(t - 1) * N, p) = sv;
            } else {
                b0 = d0;
                b1 = d1;
                b2 = d2;
            }
        }
        if (MODE == 2) {
        } else if (MODE == 0) {
            if (add) {
                b0 += e0;
                b1 += e1;
                b2 += e2;
            }
            at(out3, p) = b0;
            at(out3 + N, p) = b1;
            at(out3 + 2 * (size_t)N, p) = b2;
            if (dp)
                acc += (double)at(dp, p) * b0 + (double)at(dp + N, p) * b1 + (double)at(dp + 2 * (size_t)N, p) * b2;
        } else {
            stf(&at(out1, p), scale * -(e0 * b0 + e1 * b1 + e2 * b2));
        }
#pragma unroll
        for (int t = 0; t < NL; ++t)
#pragma unroll
            for (int s = 0; s < 8; ++s) ring[t][s] = ring[t][s + 1];
    }
    if (MODE == 0 && dp) {
        acc = block_sum(acc);
        if (threadIdx.x == 0) partials[blockIdx.x] = acc;
    }
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

void launch_state_grad(const Grid &g, int dt_m, const StateGradArgs &a, int count, hipStream_t s)
{
    with_dtype(dt_m, [&](auto tm) {
        using Tm = decltype(tm);
        hipLaunchKernelGGL((k_state_grad<Tm>), dim3((g.N + TPB - 1) / TPB, count), dim3(TPB), 0, s, g, a);
    });
}

bool sources_march(const Grid &g, int nt) { return g.n3 >= 64 && g.n2 >= 8 && nt + 1 <= 5; }

void launch_inc_sources_march(const Grid &g, int dt_m, const QuadArgs &qa, const float *vt, int nt, float scale,
                              int dt_q, void *q0, float *S, hipStream_t s);

void launch_inc_sources(const Grid &g, const float *G, const float *vt, int nt, float scale, int dt_q, void *q0,
                        float *S, hipStream_t s)
{
    with_dtype(dt_q, [&](auto tq) {
        using Tq = decltype(tq);
        hipLaunchKernelGGL((k_inc_sources<Tq>), dim3((g.N / 4 + TPB - 1) / TPB), dim3(TPB), 0, s, g, G, vt, nt, scale,
                           (Tq *)q0, S);
    });
}

void launch_quadrature(const Grid &g, int dt_lam, const QuadArgs &qa, const float *addend3, float *out3, hipStream_t s)
{
    launch_quadrature_dot(g, dt_lam, qa, addend3, out3, nullptr, nullptr, s);
}

namespace {

// The marching kernels need whole 64 x 8 tiles in (x3, x2).  Each tile
// column along x1 is cut into nch chunks, and a chunk reads 8 halo planes of
// m beside its own.  nch minimises (rounds of resident blocks) x (longest
// chunk + halo), with two resident 512-thread blocks per CU (the register
// use of five time levels): at 256^3 four chunks of 64 planes, 512 blocks
// that all run at once (12.5 % halo reads), where 16-plane chunks took 2048
// blocks in four rounds (50 % halo reads).
bool march_ok(const Grid &g) { return g.n3 >= MX && g.n2 >= MY; }

int device_cus()
{
    static const int n = [] {
        int d = 0, v = 0;
        if (hipGetDevice(&d) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, d) !=
                                                   hipSuccess)
            v = 0;
        return v > 0 ? v : 256;
    }();
    return n;
}

MarchGeom march_geom(const Grid &g)
{
    MarchGeom mg;
    mg.ntx = g.n3 / MX;
    mg.nty = g.n2 / MY;
    const long tiles = (long)mg.ntx * mg.nty, resident = 2L * device_cus();
    double best = 1e300;
    mg.nch = 1;
    for (int n = 1; n <= std::max(1, g.n1 / 8); ++n) {
        const double cost = (double)((tiles * n + resident - 1) / resident) * ((g.n1 + n - 1) / n + 2 * MH);
        if (cost < best) {
            best = cost;
            mg.nch = n;
        }
    }
    return mg;
}

int march_blocks(const Grid &g)
{
    const MarchGeom mg = march_geom(g);
    return mg.ntx * mg.nty * mg.nch;
}

template <typename Tm, typename Tl>
void launch_quad_march(const Grid &g, const QuadArgs &qa, const float *add, float *out3, const float *dp,
                       double *partials, hipStream_t s)
{
    const MarchGeom mg = march_geom(g);
    const dim3 grid(march_blocks(g));
    switch (qa.count) {
#define CLH_QM(NL)                                                                                                   \
    case NL:                                                                                                         \
        hipLaunchKernelGGL((k_fd_march<Tm, Tl, float, NL, 0>), grid, dim3(TPB_M), 0, s, g, mg, qa, add, out3, dp,    \
                           partials, (const float *)nullptr, 0.f, (float *)nullptr);                                 \
        break;
        CLH_QM(1) CLH_QM(2) CLH_QM(3) CLH_QM(4) CLH_QM(5)
#undef CLH_QM
    }
}

} // namespace

// The marching kernel reads m^j (plus halo planes) instead of the stored
// gradients (3 fields per time level), so it is used in both layouts; its
// derivatives are the stored ones bit for bit.  More than MAX_NL time
// levels are summed in groups of MAX_NL, each launch adding its group to
// the previous partial sum (the first adds the addend).
bool quadrature_marches(const Grid &g, const QuadArgs &qa) { (void)qa; return march_ok(g); }

int quadrature_blocks(const Grid &g, const QuadArgs &qa)
{
    return quadrature_marches(g, qa) ? march_blocks(g) : (int)((g.N / 4 + TPB - 1) / TPB);
}

int quadrature_blocks_max(const Grid &g)
{
    return std::max((int)((g.N / 4 + TPB - 1) / TPB), march_ok(g) ? march_blocks(g) : 0);
}

void launch_quadrature_dot(const Grid &g, int dt_lam, const QuadArgs &qa, const float *addend3, float *out3,
                           const float *dp, double *partials, hipStream_t s)
{
    with_dtype(dt_lam, [&](auto tl) {
        using Tl = decltype(tl);
        if (quadrature_marches(g, qa)) {
            with_dtype(qa.dt_m, [&](auto tm) {
                using Tm = decltype(tm);
                for (int t0 = 0; t0 < qa.count; t0 += MAX_NL) {
                    QuadArgs sub = qa;
                    sub.count = std::min(MAX_NL, qa.count - t0);
                    for (int t = 0; t < sub.count; ++t) {
                        sub.lam[t] = qa.lam[t0 + t];
                        sub.m[t] = qa.m[t0 + t];
                        sub.G[t] = qa.G[t0 + t];
                        sub.w[t] = qa.w[t0 + t];
                    }
                    const bool last = t0 + MAX_NL >= qa.count;
                    launch_quad_march<Tm, Tl>(g, sub, t0 == 0 ? addend3 : out3, out3, last ? dp : nullptr,
                                              last ? partials : nullptr, s);
                }
            });
        } else if (qa.lean) {
            with_dtype(qa.dt_m, [&](auto tm) {
                using Tm = decltype(tm);
                hipLaunchKernelGGL((k_quadrature_fd<Tm, Tl>), dim3(quadrature_blocks(g, qa)), dim3(TPB), 0, s, g, qa,
                                   addend3, out3, dp, partials);
            });
        } else {
            hipLaunchKernelGGL((k_quadrature<Tl>), dim3(quadrature_blocks(g, qa)), dim3(TPB), 0, s, g, qa, addend3,
                               out3, dp, partials);
        }
    });
}

// sources of every level from m^0 .. m^nt by the marching kernel (the
// same FD8 and products as from stored gradients, bit for bit)
void launch_inc_sources_march(const Grid &g, int dt_m, const QuadArgs &qa, const float *vt, int nt, float scale,
                              int dt_q, void *q0, float *S, hipStream_t s)
{
    with_dtype(dt_m, [&](auto tm) {
        using Tm = decltype(tm);
        with_dtype(dt_q, [&](auto tq) {
            using Tq = decltype(tq);
            const dim3 grid(march_blocks(g));
            switch (nt + 1) {
#define CLH_SM(NL)                                                                                                   \
    case NL:                                                                                                         \
        hipLaunchKernelGGL((k_fd_march<Tm, float, Tq, NL, 2>), grid, dim3(TPB_M), 0, s, g, march_geom(g), qa,        \
                           (const float *)nullptr, S, (const float *)nullptr, (double *)nullptr, vt, scale, (Tq *)q0); \
        break;
                CLH_SM(2) CLH_SM(3) CLH_SM(4) CLH_SM(5)
#undef CLH_SM
            default: break;
            }
        });
    });
}

void launch_inc_source_fd(const Grid &g, int dt_m, const void *m, const float *vt, float scale, int dt_out, void *out,
                          hipStream_t s)
{
    with_dtype(dt_m, [&](auto tm) {
        using Tm = decltype(tm);
        with_dtype(dt_out, [&](auto to) {
            using To = decltype(to);
            if (march_ok(g)) {
                QuadArgs qa{};
                qa.m[0] = m;
                qa.count = 1;
                hipLaunchKernelGGL((k_fd_march<Tm, float, To, 1, 1>), dim3(march_blocks(g)), dim3(TPB_M), 0, s, g,
                                   march_geom(g), qa, (const float *)nullptr, (float *)nullptr,
                                   (const float *)nullptr, (double *)nullptr, vt, scale, (To *)out);
            } else {
                hipLaunchKernelGGL((k_inc_source_fd<Tm, To>), dim3((g.N + TPB - 1) / TPB), dim3(TPB), 0, s, g,
                                   (const Tm *)m, vt, scale, (To *)out);
            }
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
