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
    // integer parts clamped to +-2^24 so the conversion is defined for any
    // finite input; indices are wrapped by masking below
    const float c1 = fminf(fmaxf(f1, -16777216.0f), 16777216.0f);
    const float c2 = fminf(fmaxf(f2, -16777216.0f), 16777216.0f);
    const float c3 = fminf(fmaxf(f3, -16777216.0f), 16777216.0f);
    const int b1 = i + (int)c1 - 1, b2 = j + (int)c2 - 1, b3 = k + (int)c3 - 1;
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

// ------------------------------------------------ semi-Lagrangian steps
// One SL step gathers u at the feet of every node and applies a mode-specific
// epilogue:
//   SL_STATE:  out = I[u](X)
//   SL_ADJ:    out = c * I[u](X)                    (adjoint divergence factor)
//   SL_INC:    out = sI * I[u](X) + sS * (-vt . G)  (incremental source,
//              G = grad_h m^{j+1} precomputed once per velocity)
enum { SL_STATE = 0, SL_ADJ = 1, SL_INC = 2 };

template <int MODE>
__device__ __forceinline__ float epilogue(const Grid &g, const SLParams &prm, int p, float val)
{
    if (MODE == SL_ADJ) return prm.c[p] * val;
    if (MODE == SL_INC) {
        const size_t N = g.N;
        const float src = -(prm.vt[p] * prm.G[p] + prm.vt[N + p] * prm.G[N + p] + prm.vt[2 * N + p] * prm.G[2 * N + p]);
        return prm.sI * val + prm.sS * src;
    }
    return val;
}

// Per-node version (small grids, and tiles whose feet spread too far).
template <typename Tu, typename To, int MODE>
__global__ __launch_bounds__(TPB) void k_sl_node(Grid g, const Tu *__restrict__ u, const float *__restrict__ d,
                                                 SLParams prm, To *__restrict__ out)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    int i, j, k;
    node_of(g, p, i, j, k);
    Foot F;
    make_foot(g, i, j, k, d[p], d[g.N + p], d[2 * (size_t)g.N + p], F);
    stf(out + p, epilogue<MODE>(g, prm, p, gather(u, F)));
}

// Tiled version: a workgroup owns a TZ x TY x TX tile (x1, x2, x3), finds
// the bounding box of the 4x4x4 stencils of its feet, stages that box in LDS
// and gathers from LDS.  For a smooth velocity the feet of a tile form a
// slightly deformed copy of the tile, so the box is the tile plus a thin
// shell.  The box is stored with fixed pitches (PZ, PY, PX) so that the 64
// stencil offsets of a point are compile-time LDS immediates; a tile whose
// box exceeds them gathers straight from global memory instead (same
// arithmetic, same result).  The kernel is VALU-bound, so the per-point
// instruction count is what the layout minimises.
constexpr int TX = 32, TY = 8, TZ = 8;
constexpr int PX = 40, PY = 14, PZ = 14;      // box pitches: tile + 3 + slack of 5 / 3 / 3

__device__ __forceinline__ int ifloor(float x)
{
    const float f = fminf(fmaxf(floorf(x), -16777216.0f), 16777216.0f);
    return (int)f;
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Cubic Lagrange weights at fraction f with shared factors: a = f(f-1),
// b = (f+1)(f-2) = a - 2; 10 VALU operations.  Exactly (0, 1, 0, 0) at f = 0.
__device__ __forceinline__ void lagrange4_fast(float f, float w[4])
{
    const float a = fmaf(f, f, -f);
    const float b = a - 2.0f;
    w[0] = a * fmaf(f, -1.0f / 6.0f, 1.0f / 3.0f);   // -f(f-1)(f-2)/6
    w[1] = b * fmaf(f, 0.5f, -0.5f);                 //  (f+1)(f-1)(f-2)/2
    w[2] = b * (-0.5f * f);                          // -(f+1)f(f-2)/2
    w[3] = a * fmaf(f, 1.0f / 6.0f, 1.0f / 6.0f);    //  (f+1)f(f-1)/6
}

template <typename Tu, typename To, int MODE>
__global__ __launch_bounds__(TPB, 4) void k_sl_tile(Grid g, const Tu *__restrict__ u, const float *__restrict__ d,
                                                 SLParams prm, To *__restrict__ out, int ntx, int nty, int nblk)
{
    __shared__ Tu box[PZ * PY * PX];
    __shared__ int red[TPB / 64][6];
    // Workgroups go round-robin to the 8 XCDs; give each XCD a contiguous
    // run of tiles so that neighbouring boxes meet in the same L2.
    const int b = blockIdx.x;
    const int tile = (nblk & 7) ? b : (b & 7) * (nblk >> 3) + (b >> 3);
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    const int lane = threadIdx.x & (TX - 1), row = threadIdx.x / TX;
    const int i0 = tz * TZ, j = ty * TY + row, k = tx * TX + lane;
    const int plane = g.n2 << g.l3;
    const int p0 = ((i0 << g.l2) + j) * g.n3 + k;
    const size_t N = g.N;

    float d1[TZ], d2[TZ], d3[TZ];
    int mn1 = 1 << 30, mx1 = -(1 << 30), mn2 = 1 << 30, mx2 = -(1 << 30), mn3 = 1 << 30, mx3 = -(1 << 30);
#pragma unroll
    for (int q = 0; q < TZ; ++q) {
        const int p = p0 + q * plane;
        d1[q] = d[p];
        d2[q] = d[N + p];
        d3[q] = d[2 * N + p];
        const int b1 = q + ifloor(d1[q]), b2 = ifloor(d2[q]), b3 = ifloor(d3[q]);
        mn1 = min(mn1, b1); mx1 = max(mx1, b1);
        mn2 = min(mn2, b2); mx2 = max(mx2, b2);
        mn3 = min(mn3, b3); mx3 = max(mx3, b3);
    }
    // row / lane are constant per thread: add them after the loop
    mn2 += row; mx2 += row; mn3 += lane; mx3 += lane;
    mn1 = wave_min(mn1); mx1 = wave_max(mx1);
    mn2 = wave_min(mn2); mx2 = wave_max(mx2);
    mn3 = wave_min(mn3); mx3 = wave_max(mx3);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if ((threadIdx.x & 63) == 0) {
        red[wv][0] = mn1; red[wv][1] = mx1; red[wv][2] = mn2;
        red[wv][3] = mx2; red[wv][4] = mn3; red[wv][5] = mx3;
    }
    __syncthreads();
    mn1 = red[0][0]; mx1 = red[0][1]; mn2 = red[0][2]; mx2 = red[0][3]; mn3 = red[0][4]; mx3 = red[0][5];
#pragma unroll
    for (int w = 1; w < TPB / 64; ++w) {
        mn1 = min(mn1, red[w][0]); mx1 = max(mx1, red[w][1]);
        mn2 = min(mn2, red[w][2]); mx2 = max(mx2, red[w][3]);
        mn3 = min(mn3, red[w][4]); mx3 = max(mx3, red[w][5]);
    }
    // box origin (stencil starts one node below the floor), extents
    mn1 -= 1; mn2 -= 1; mn3 -= 1;
    const int E1 = mx1 + 3 - mn1, E2 = mx2 + 3 - mn2, E3 = mx3 + 3 - mn3;
    const bool fits = E1 <= PZ && E2 <= PY && E3 <= PX;

    if (fits) {
        // Stage rows (a, bb) of the box: wave wv loads rows bb = wv, wv+4, ...
        // of two x1 planes per batch, lane c < E3 loads column c.
        const int l64 = threadIdx.x & 63;
        const int gi0 = i0 + mn1, gj0 = ty * TY + mn2;
        const int col = (tx * TX + mn3 + l64) & (g.n3 - 1);
        const bool act = l64 < E3;
        for (int a0 = 0; a0 < E1; a0 += 2) {
            Tu vals[8];
#pragma unroll
            for (int ia = 0; ia < 2; ++ia)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) {
                    const int a = a0 + ia, bb = wv + 4 * jb;
                    if (act && a < E1 && bb < E2)
                        vals[ia * 4 + jb] =
                            u[(((gi0 + a) & (g.n1 - 1)) << (g.l2 + g.l3)) + (((gj0 + bb) & (g.n2 - 1)) << g.l3) + col];
                }
#pragma unroll
            for (int ia = 0; ia < 2; ++ia)
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) {
                    const int a = a0 + ia, bb = wv + 4 * jb;
                    if (act && a < E1 && bb < E2) box[(a * PY + bb) * PX + l64] = vals[ia * 4 + jb];
                }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TZ; ++q) {
            const float f1 = floorf(d1[q]), f2 = floorf(d2[q]), f3 = floorf(d3[q]);
            float w1[4], w2[4], w3[4];
            lagrange4_fast(d1[q] - f1, w1);
            lagrange4_fast(d2[q] - f2, w2);
            lagrange4_fast(d3[q] - f3, w3);
            // same clamped integer parts as the bounding box, so the stencil
            // lies inside the box for any finite displacement
            const int s1 = q + ifloor(d1[q]) - mn1 - 1;
            const int s2 = row + ifloor(d2[q]) - mn2 - 1;
            const int s3 = lane + ifloor(d3[q]) - mn3 - 1;
            const Tu *bp = box + (s1 * PY + s2) * PX + s3;
            float s = 0.0f;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                float sa = 0.0f;
#pragma unroll
                for (int bq = 0; bq < 4; ++bq) {
                    const Tu *rp = bp + (a * PY + bq) * PX;
                    float t = w3[0] * ldf(rp);
                    t = fmaf(w3[1], ldf(rp + 1), t);
                    t = fmaf(w3[2], ldf(rp + 2), t);
                    t = fmaf(w3[3], ldf(rp + 3), t);
                    sa = fmaf(w2[bq], t, sa);
                }
                s = fmaf(w1[a], sa, s);
                __builtin_amdgcn_sched_barrier(0);
            }
            const int p = p0 + q * plane;
            stf(out + p, epilogue<MODE>(g, prm, p, s));
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        for (int q = 0; q < TZ; ++q) {
            const int p = p0 + q * plane;
            Foot F;
            make_foot(g, i0 + q, j, k, d1[q], d2[q], d3[q], F);
            stf(out + p, epilogue<MODE>(g, prm, p, gather(u, F)));
        }
    }
}

inline dim3 grid_of(const Grid &g) { return dim3((g.N + TPB - 1) / TPB); }

template <typename Tu, typename To, int MODE>
void launch_sl(const Grid &g, const Tu *u, const float *d, const SLParams &prm, To *out, hipStream_t s)
{
    if (g.n3 >= TX && g.n2 >= TY && g.n1 >= TZ) {
        const int ntx = g.n3 / TX, nty = g.n2 / TY, ntz = g.n1 / TZ;
        const int nblk = ntx * nty * ntz;
        hipLaunchKernelGGL((k_sl_tile<Tu, To, MODE>), dim3(nblk), dim3(TPB), 0, s, g, u, d, prm, out, ntx, nty, nblk);
    } else {
        hipLaunchKernelGGL((k_sl_node<Tu, To, MODE>), grid_of(g), dim3(TPB), 0, s, g, u, d, prm, out);
    }
}

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
            launch_sl<Tu, To, SL_STATE>(g, (const Tu *)u, d, SLParams{}, (To *)out, s);
        });
    });
}

void launch_sl_adjoint(const Grid &g, int dt_u, const void *u, const float *d, const float *c, int dt_out,
                       void *out, hipStream_t s)
{
    SLParams prm{};
    prm.c = c;
    with_dtype(dt_u, [&](auto tu) {
        using Tu = decltype(tu);
        with_dtype(dt_out, [&](auto to) {
            using To = decltype(to);
            launch_sl<Tu, To, SL_ADJ>(g, (const Tu *)u, d, prm, (To *)out, s);
        });
    });
}

void launch_sl_inc(const Grid &g, int dt_q, const void *q, const float *d, const float *G, const float *vt, float sI,
                   float sS, int dt_out, void *out, hipStream_t s)
{
    SLParams prm{};
    prm.G = G;
    prm.vt = vt;
    prm.sI = sI;
    prm.sS = sS;
    with_dtype(dt_q, [&](auto tq) {
        using Tq = decltype(tq);
        with_dtype(dt_out, [&](auto to) {
            using To = decltype(to);
            launch_sl<Tq, To, SL_INC>(g, (const Tq *)q, d, prm, (To *)out, s);
        });
    });
}

void launch_interp_f32(const Grid &g, const float *u, const float *d, float *out, hipStream_t s)
{
    launch_sl<float, float, SL_STATE>(g, u, d, SLParams{}, out, s);
}

} // namespace clh
