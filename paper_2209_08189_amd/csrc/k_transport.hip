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

#include <utility>

namespace clh {

namespace {

constexpr int TPB = 256;

// Twice the cubic Lagrange weights of the nodes base-1..base+2 at fraction
// f in [0,1), with the shared factors a = f(f-1), a/3 and b = (f+1)(f-2) =
// a - 2 (8 VALU operations); exactly (0, 2, 0, 0) at f = 0.  A tricubic
// value is the contraction with these weights times CUBIC_SCALE = 1/8 (a
// power of two: no rounding).  Every tricubic path (per node, tiled,
// global-memory fallback) takes these weights and the same contraction
// order, so the three agree bitwise.
constexpr float CUBIC_SCALE = 0.125f;
__device__ __forceinline__ void lagrange4_fast(float f, float w[4])
{
    const float a = fmaf(f, f, -f);
    const float b = a - 2.0f;
    const float a3 = a * (1.0f / 3.0f);
    w[0] = a3 * (2.0f - f);          // -f(f-1)(f-2)/3
    w[1] = fmaf(b, f, -b);           //  (f+1)(f-1)(f-2)
    w[2] = -b * f;                   // -(f+1)f(f-2)
    w[3] = fmaf(a3, f, a3);          //  (f+1)f(f-1)/3
}

// Fraction d - floor(d) of a displacement (v_fract_f32: one instruction,
// exact wherever the difference is representable, and below 1 where it
// would round up to 1).  Every SL path takes its fractions from here, so
// the paths agree bitwise.
__device__ __forceinline__ float frac_of(float d) { return __builtin_amdgcn_fractf(d); }

// floor(d) as an integer in one instruction, for displacements known to be
// small (the feet of a tile whose box fits, whose floors lie within the box).
__device__ __forceinline__ int floor_small(float d)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(d));
    return r;
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
    lagrange4_fast(frac_of(d1), F.w1);
    lagrange4_fast(frac_of(d2), F.w2);
    lagrange4_fast(frac_of(d3), F.w3);
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
    return s * CUBIC_SCALE;
}

// ------------------------------------------------------------- kernels

// RK2 (Heun) feet of both characteristic directions, as index-unit
// displacements:  X_f = x - dt/2 [v(x) + v(x - dt v(x))],
//                 X_b = x + dt/2 [v(x) + v(x + dt v(x))],
// and the adjoint factor c = 1 + dt/2 (dbar + d + dt dbar d), d = div_h v,
// dbar = d(X_b).  The velocity at the predictor feet and dbar are tricubic
// interpolations done by the tiled SL gather (launch_feet below); these
// kernels are the elementwise steps around them.  Displacements divide by h
// (correctly rounded), so a velocity that is an exact multiple of h/dt gives
// an exactly integer foot.

// The solver keeps its displacements interleaved per node (d1 d2 d3 of node
// p at 3p), so an SL step reads the feet of a node with one 12-byte load;
// the interpolation entry points take three separate fields from the caller.
template <bool AOS>
__device__ __forceinline__ void foot_of(const float *__restrict__ d, size_t N, size_t p, float &a1, float &a2,
                                        float &a3)
{
    if constexpr (AOS) {
        const float3 f = *reinterpret_cast<const float3 *>(d + 3 * p);
        a1 = f.x;
        a2 = f.y;
        a3 = f.z;
    } else {
        a1 = d[p];
        a2 = d[N + p];
        a3 = d[2 * N + p];
    }
}

// predictor displacement d = (a v) / h, a = -dt (X_f) or +dt (X_b), interleaved
__global__ __launch_bounds__(TPB) void k_feet_pred(Grid g, float a, const float *__restrict__ v, float *__restrict__ d)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    const size_t N = g.N;
    *reinterpret_cast<float3 *>(d + 3 * (size_t)p) =
        make_float3((a * v[p]) / g.h1, (a * v[N + p]) / g.h2, (a * v[2 * N + p]) / g.h3);
}

// corrector displacement d = (b (v + vi)) / h, b = -dt/2 (X_f) or +dt/2 (X_b),
// vi = v interpolated at the predictor feet (three fields); d interleaved
__global__ __launch_bounds__(TPB) void k_feet_corr(Grid g, float b, const float *__restrict__ v,
                                                   const float *__restrict__ vi, float *__restrict__ d)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    const size_t N = g.N;
    *reinterpret_cast<float3 *>(d + 3 * (size_t)p) =
        make_float3((b * (v[p] + vi[p])) / g.h1, (b * (v[N + p] + vi[N + p])) / g.h2,
                    (b * (v[2 * N + p] + vi[2 * N + p])) / g.h3);
}

// interleaved feet -> three fields (the feet a caller reads back)
__global__ __launch_bounds__(TPB) void k_feet_fields(Grid g, const float *__restrict__ d, float *__restrict__ out)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    const size_t N = g.N;
    foot_of<true>(d, N, p, out[p], out[N + p], out[2 * N + p]);
}

__global__ __launch_bounds__(TPB) void k_adj_factor(Grid g, float dt, const float *__restrict__ divv,
                                                    const float *__restrict__ dbar, float *__restrict__ c)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    const float d = divv[p], db = dbar[p];
    c[p] = 1.0f + 0.5f * dt * (db + d + dt * db * d);
}

// Source factor of the Jacobian determinant transport d_t J + v.grad J =
// -(div v) J over one step along the forward characteristic (Heun):
// f = 1 - dt/2 (d_f + d - dt d_f d), d_f = div v at the foot X_f (in place:
// dfoot holds d_f on entry and f on exit).
__global__ __launch_bounds__(TPB) void k_jac_factor(Grid g, float dt, const float *__restrict__ divv, float *dfoot)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    const float d = divv[p], df = dfoot[p];
    dfoot[p] = 1.0f - 0.5f * dt * (df + d - dt * df * d);
}

__global__ __launch_bounds__(TPB) void k_fill1(float *x, int n)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p < n) x[p] = 1.0f;
}

// ------------------------------------------------ semi-Lagrangian steps
// One SL step gathers u at the feet of every node and applies a mode-specific
// epilogue with one per-node operand e:
//   SL_STATE:  out = I[u](X)
//   SL_ADJ:    out = e * I[u](X)             (e = c, adjoint divergence factor)
//   SL_INC:    out = sI * I[u](X) + sS * e   (e = s^{j+1} = -vt . grad_h m^{j+1},
//                                             incremental source, precomputed)
enum { SL_STATE = 0, SL_ADJ = 1, SL_INC = 2 };

template <int MODE>
__device__ __forceinline__ float epilogue(const SLParams &prm, float e, float val)
{
    if (MODE == SL_ADJ) return e * val;
    if (MODE == SL_INC) return fmaf(prm.sI, val, prm.sS * e);
    return val;
}

// Per-node version (small grids, and tiles whose feet spread too far).
template <typename Tu, typename To, int MODE, bool AOS>
__global__ __launch_bounds__(TPB) void k_sl_node(Grid g, const Tu *__restrict__ u, const float *__restrict__ d,
                                                 SLParams prm, To *__restrict__ out)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    int i, j, k;
    node_of(g, p, i, j, k);
    const float e = MODE == SL_STATE ? 0.0f : prm.e[p];
    float a1, a2, a3;
    foot_of<AOS>(d, g.N, p, a1, a2, a3);
    Foot F;
    make_foot(g, i, j, k, a1, a2, a3, F);
    stf(out + p, epilogue<MODE>(prm, e, gather(u, F)));
}

// Trilinear interpolation (the linear interpolation option) of u at node
// (i, j, k) + d from global memory: 2 x 2 x 2 nodes from base = node +
// floor(d) with weights (1 - f, f) per axis, contracted along x3, then x2,
// then x1.  The tiled kernel takes the same operations on LDS values.
template <typename Tu>
__device__ __forceinline__ float lin_node(const Grid &g, const Tu *__restrict__ u, int i, int j, int k, float d1,
                                          float d2, float d3)
{
    const float f1 = floorf(d1), f2 = floorf(d2), f3 = floorf(d3);
    const float a1 = frac_of(d1), a2 = frac_of(d2), a3 = frac_of(d3);
    const int b1 = i + (int)fminf(fmaxf(f1, -16777216.0f), 16777216.0f);
    const int b2 = j + (int)fminf(fmaxf(f2, -16777216.0f), 16777216.0f);
    const int b3 = k + (int)fminf(fmaxf(f3, -16777216.0f), 16777216.0f);
    const int r0 = (b1 & (g.n1 - 1)) << (g.l2 + g.l3), r1 = ((b1 + 1) & (g.n1 - 1)) << (g.l2 + g.l3);
    const int c0 = (b2 & (g.n2 - 1)) << g.l3, c1 = ((b2 + 1) & (g.n2 - 1)) << g.l3;
    const int k0 = b3 & (g.n3 - 1), k1 = (b3 + 1) & (g.n3 - 1);
    const float w30 = 1.0f - a3;
    const float s00 = fmaf(a3, ldf(u + r0 + c0 + k1), w30 * ldf(u + r0 + c0 + k0));
    const float s01 = fmaf(a3, ldf(u + r0 + c1 + k1), w30 * ldf(u + r0 + c1 + k0));
    const float s10 = fmaf(a3, ldf(u + r1 + c0 + k1), w30 * ldf(u + r1 + c0 + k0));
    const float s11 = fmaf(a3, ldf(u + r1 + c1 + k1), w30 * ldf(u + r1 + c1 + k0));
    const float s0 = fmaf(a2, s01, (1.0f - a2) * s00);
    const float s1 = fmaf(a2, s11, (1.0f - a2) * s10);
    return fmaf(a1, s1, (1.0f - a1) * s0);
}

// Per-node trilinear version (grids too small for tiles): one node per
// thread; the eight values come from L2 (the feet of neighbouring threads
// are neighbours).
template <typename Tu, typename To, int MODE, bool AOS>
__global__ __launch_bounds__(TPB) void k_sl_lin(Grid g, const Tu *__restrict__ u, const float *__restrict__ d,
                                                SLParams prm, To *__restrict__ out)
{
    const int p = blockIdx.x * TPB + threadIdx.x;
    if (p >= g.N) return;
    int i, j, k;
    node_of(g, p, i, j, k);
    const float e = MODE == SL_STATE ? 0.0f : prm.e[p];
    float a1, a2, a3;
    foot_of<AOS>(d, g.N, p, a1, a2, a3);
    stf(out + p, epilogue<MODE>(prm, e, lin_node(g, u, i, j, k, a1, a2, a3)));
}

// Tiled version: tiles of TZ x TY x TX nodes (x1, x2, x3).  For a smooth
// velocity the feet of a tile form a slightly deformed copy of the tile, so
// the 4x4x4 stencils of all its feet lie in a box that is the tile plus a
// thin shell.  The box of every tile is computed once per velocity and
// direction (k_tile_boxes); an SL step stages the box in LDS and gathers
// from LDS.  The box is stored with fixed pitches (PZ, PY, PX) so that the
// 64 stencil offsets of a point are compile-time LDS immediates; a tile whose
// box exceeds them gathers straight from global memory instead (same
// arithmetic, same result).
//
// Bank layout: PX (in 32-bit words) and PY * PX are multiples of 32, so the
// LDS bank of a lane's stencil element depends only on its x3 position;
// lanes whose feet fall in different box rows or planes do not collide.
//
// Latency: the feet, the epilogue operands and the box (as direct-to-LDS
// loads: one wave-uniform box row per instruction, lane = column) are all
// requested before the first wait; several workgroups per CU overlap one
// another's memory waits with their gathers.
constexpr int TX = 32, TY = 8, TZ = 8;
// box pitches: tile + 3 + slack (x1: 2, x2: 1); 13 x 12 x 64 words = 39.9 KB,
// so four workgroups share a CU's 160 KB of LDS
constexpr int PY = 12, PZ = 13;
// x3 pitch in elements: 64 words for FP32; 16-bit boxes load element pairs
// from an even start (one-element shift) and use 64 elements (32 words).
template <typename T> constexpr int box_px() { return sizeof(T) == 4 ? 64 : 64; }

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


typedef __attribute__((address_space(3))) void lds_void;

// Thread layout of the tile kernels: with 256 * SPLIT threads, thread
// (part, row, lane) owns nodes (i0 + q0 + q, j, k), q < TZ / SPLIT, where
// q0 = part * TZ / SPLIT.
struct TileIdx {
    int tx, ty, tz, lane, row, i0, q0, j, k, p0, plane;
};
template <int SPLIT>
__device__ __forceinline__ TileIdx tile_idx(const Grid &g, int tile, int ntx, int nty)
{
    // tile counts are powers of two (as are the grid sizes)
    const int lx = __builtin_ctz(ntx), ly = __builtin_ctz(nty);
    TileIdx t;
    t.tx = tile & (ntx - 1);
    t.ty = (tile >> lx) & (nty - 1);
    t.tz = tile >> (lx + ly);
    t.lane = threadIdx.x & (TX - 1);
    t.row = (threadIdx.x & 255) / TX;
    t.i0 = t.tz * TZ;
    t.q0 = SPLIT == 1 ? 0 : (threadIdx.x >> 8) * (TZ / SPLIT);
    t.j = t.ty * TY + t.row;
    t.k = t.tx * TX + t.lane;
    t.plane = g.n2 << g.l3;
    t.p0 = (((t.i0 + t.q0) << g.l2) + t.j) * g.n3 + t.k;
    return t;
}

// Bounding box of the 4x4x4 stencils of the feet of every tile, once per
// velocity and direction: box[8 tile + 0..2] = origin relative to the tile
// origin (x1, x2, x3), box[8 tile + 3..5] = extents.  The integer parts are
// the same clamped floors that the SL kernels use, so every stencil lies
// inside its box for any finite displacement.
template <bool AOS>
__global__ __launch_bounds__(TPB) void k_tile_boxes(Grid g, const float *__restrict__ d, int ntx, int nty,
                                                    int *__restrict__ box, int lo, int span)
{
    __shared__ int red[TPB / 64][6];
    const TileIdx t = tile_idx<1>(g, blockIdx.x, ntx, nty);
    const size_t N = g.N;
    int mn1 = 1 << 30, mx1 = -(1 << 30), mn2 = 1 << 30, mx2 = -(1 << 30), mn3 = 1 << 30, mx3 = -(1 << 30);
#pragma unroll
    for (int q = 0; q < TZ; ++q) {
        const int p = t.p0 + q * t.plane;
        float a1, a2, a3;
        foot_of<AOS>(d, N, p, a1, a2, a3);
        const int b1 = q + ifloor(a1), b2 = ifloor(a2), b3 = ifloor(a3);
        mn1 = min(mn1, b1); mx1 = max(mx1, b1);
        mn2 = min(mn2, b2); mx2 = max(mx2, b2);
        mn3 = min(mn3, b3); mx3 = max(mx3, b3);
    }
    mn2 += t.row; mx2 += t.row; mn3 += t.lane; mx3 += t.lane;
    mn1 = wave_min(mn1); mx1 = wave_max(mx1);
    mn2 = wave_min(mn2); mx2 = wave_max(mx2);
    mn3 = wave_min(mn3); mx3 = wave_max(mx3);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[wv][0] = mn1; red[wv][1] = mx1; red[wv][2] = mn2;
        red[wv][3] = mx2; red[wv][4] = mn3; red[wv][5] = mx3;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 1; w < TPB / 64; ++w) {
        mn1 = min(mn1, red[w][0]); mx1 = max(mx1, red[w][1]);
        mn2 = min(mn2, red[w][2]); mx2 = max(mx2, red[w][3]);
        mn3 = min(mn3, red[w][4]); mx3 = max(mx3, red[w][5]);
    }
    // the stencil starts lo nodes below the floor and spans span nodes
    // (cubic: 1, 4; trilinear: 0, 2)
    int *o = box + 8 * blockIdx.x;
    o[0] = mn1 - lo; o[1] = mn2 - lo; o[2] = mn3 - lo;
    o[3] = mx1 - mn1 + span; o[4] = mx2 - mn2 + span; o[5] = mx3 - mn3 + span;
    o[6] = 0; o[7] = 0;
}

// Box of one tile as the SL kernels use it.
struct TileBox {
    int r1, r2, r3, E1, E2, E3, c0, sh;
    bool fits;
};
template <typename Tu>
__device__ __forceinline__ TileBox tile_box(const int *__restrict__ boxes, int tile, const TileIdx &t)
{
    constexpr int PX = box_px<Tu>();
    TileBox B;
    const int *bx = boxes + 8 * tile;
    B.r1 = bx[0]; B.r2 = bx[1]; B.r3 = bx[2];
    B.E1 = bx[3]; B.E2 = bx[4]; B.E3 = bx[5];
    // global x3 index of box column 0; 16-bit boxes start at the even index
    // at or below it and shift the stencil by the difference
    B.c0 = t.tx * TX + B.r3;
    B.sh = sizeof(Tu) == 2 ? (B.c0 & 1) : 0;
    B.fits = B.E1 <= PZ && B.E2 <= PY && B.E3 + B.sh <= PX;
    return B;
}

// SL tile kernel: 512 threads, each owning QT = 4 nodes along x1.
constexpr int SPLIT = 2, QT = TZ / SPLIT, TPB_SL = 256 * SPLIT;

// Feet and epilogue operand of the QT nodes of this thread.
template <int MODE, bool AOS>
__device__ __forceinline__ void load_feet(const Grid &g, const float *__restrict__ d, const SLParams &prm,
                                          const TileIdx &t, float (&d1)[QT], float (&d2)[QT], float (&d3)[QT],
                                          float (&e)[QT])
{
    // each field from its own wave-uniform base with a 32-bit byte offset
    // (a field has at most 2^30 nodes)
    const size_t N = g.N;
    const char *be = reinterpret_cast<const char *>(prm.e);
    const unsigned o0 = (unsigned)t.p0 * 4u, dq = (unsigned)t.plane * 4u;
    if constexpr (AOS) {
        // interleaved feet: the tile's first node is the wave-uniform base,
        // 12 bytes per node from there (under 2^32 within a tile)
        const int pt = (((t.i0 << g.l2) + t.ty * TY) << g.l3) + t.tx * TX;
        const char *bd = reinterpret_cast<const char *>(d + 3 * (size_t)pt);
        const unsigned r0 = (unsigned)(t.p0 - pt) * 12u, rq = (unsigned)t.plane * 12u;
#pragma unroll
        for (int q = 0; q < QT; ++q) {
            const float3 f = *reinterpret_cast<const float3 *>(bd + (r0 + q * rq));
            d1[q] = f.x;
            d2[q] = f.y;
            d3[q] = f.z;
        }
    } else {
        const char *b1 = reinterpret_cast<const char *>(d), *b2 = reinterpret_cast<const char *>(d + N),
                   *b3 = reinterpret_cast<const char *>(d + 2 * N);
#pragma unroll
        for (int q = 0; q < QT; ++q) {
            const unsigned o = o0 + q * dq;
            d1[q] = *reinterpret_cast<const float *>(b1 + o);
            d2[q] = *reinterpret_cast<const float *>(b2 + o);
            d3[q] = *reinterpret_cast<const float *>(b3 + o);
        }
    }
#pragma unroll
    for (int q = 0; q < QT; ++q)
        e[q] = MODE == SL_STATE ? 0.0f : *reinterpret_cast<const float *>(be + (o0 + q * dq));
}

// Direct-to-LDS staging of a box: wave wv loads box rows (a, bb) with
// bb = wv, wv + NW, ... (NW waves); lane l loads column l (FP32) or the column pair 2l,
// 2l+1 (16-bit) into LDS at row start + 4 l bytes; lanes past the row are
// switched off.  A row wider than one wave's load takes several chunks.
template <typename Tu>
__device__ __forceinline__ void stage_box(const Grid &g, const Tu *__restrict__ u, Tu *box, const TileIdx &t,
                                          const TileBox &B)
{
    constexpr int PX = box_px<Tu>();
    constexpr int EPL = sizeof(Tu) == 2 ? 2 : 1;       // elements per lane
    constexpr int NCH = (PX + 64 * EPL - 1) / (64 * EPL);
    constexpr int NW = TPB_SL / 64;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int l64 = threadIdx.x & 63;
    const int gi0 = t.i0 + B.r1, gj0 = t.ty * TY + B.r2;
    // byte offset of this lane's element(s) within a field row (periodic)
    unsigned cb[NCH];
    bool on[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const int c = 64 * EPL * ch + EPL * l64;            // box column of this lane's first element
        on[ch] = c < B.E3 + B.sh;
        cb[ch] = (unsigned)((B.c0 - B.sh + c) & (g.n3 - 1)) * (unsigned)sizeof(Tu);
    }
    for (int a = 0; a < B.E1; ++a) {
        const int ga = ((gi0 + a) & (g.n1 - 1)) << (g.l2 + g.l3);
        for (int bb = wv; bb < B.E2; bb += NW) {
            const char *row = reinterpret_cast<const char *>(u + (ga + (((gj0 + bb) & (g.n2 - 1)) << g.l3)));
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                if (on[ch])
                    __builtin_amdgcn_global_load_lds((const void *)(row + cb[ch]),
                                                     (lds_void *)(box + (a * PY + bb) * PX + 64 * EPL * ch), 4, 0,
                                                     0);
        }
    }
}

// FP32 LDS load by 32-bit LDS byte address (the 32-bit box path).
template <typename T> __device__ __forceinline__ float lds_ld(unsigned a);
template <> __device__ __forceinline__ float lds_ld<float>(unsigned a)
{
    return *reinterpret_cast<__attribute__((address_space(3))) const float *>(static_cast<uintptr_t>(a));
}
__device__ __forceinline__ unsigned lds_ld_u32(unsigned a)
{
    return *reinterpret_cast<__attribute__((address_space(3))) const unsigned *>(static_cast<uintptr_t>(a));
}
__device__ __forceinline__ void lds_st_u32(unsigned a, unsigned v)
{
    *reinterpret_cast<__attribute__((address_space(3))) unsigned *>(static_cast<uintptr_t>(a)) = v;
}

// x3 row of 4 consecutive 16-bit values held in two words (lo, hi halves),
// contracted with the weights w3 in FP32.  FP16: the conversions fold into
// mixed-precision FMAs; BF16: a value is the high half of an FP32 word.
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
template <typename T> __device__ __forceinline__ float row4(unsigned d0, unsigned d1, const float w3[4]);
template <> __device__ __forceinline__ float row4<__half>(unsigned d0, unsigned d1, const float w3[4])
{
    const h2_t a = __builtin_bit_cast(h2_t, d0), b = __builtin_bit_cast(h2_t, d1);
    float t = fmaf(w3[0], (float)a.x, 0.0f);
    t = fmaf(w3[1], (float)a.y, t);
    t = fmaf(w3[2], (float)b.x, t);
    return fmaf(w3[3], (float)b.y, t);
}
template <> __device__ __forceinline__ float row4<__hip_bfloat16>(unsigned d0, unsigned d1, const float w3[4])
{
    float t = w3[0] * __uint_as_float(d0 << 16);
    t = fmaf(w3[1], __uint_as_float(d0 & 0xffff0000u), t);
    t = fmaf(w3[2], __uint_as_float(d1 << 16), t);
    return fmaf(w3[3], __uint_as_float(d1 & 0xffff0000u), t);
}

template <typename T> __device__ __forceinline__ unsigned lds_addr(const T *p)
{
    return (unsigned)(uintptr_t)(lds_void *)(p);
}

// The two values of a trilinear stencil row at LDS byte address a: FP32
// boxes read two words; 16-bit boxes read the one aligned word of the copy
// the caller chose (lo half first).
template <typename T> __device__ __forceinline__ void row2(unsigned a, float &x0, float &x1);
template <> __device__ __forceinline__ void row2<float>(unsigned a, float &x0, float &x1)
{
    x0 = lds_ld<float>(a);
    x1 = lds_ld<float>(a + 4);
}
template <> __device__ __forceinline__ void row2<__half>(unsigned a, float &x0, float &x1)
{
    const h2_t h = __builtin_bit_cast(h2_t, lds_ld_u32(a));
    x0 = (float)h.x;
    x1 = (float)h.y;
}
template <> __device__ __forceinline__ void row2<__hip_bfloat16>(unsigned a, float &x0, float &x1)
{
    const unsigned w = lds_ld_u32(a);
    x0 = __uint_as_float(w << 16);
    x1 = __uint_as_float(w & 0xffff0000u);
}

// LDS addressing of the stencils of a thread's nodes in a staged box: the
// stencil of node q starts at box element (q0 + q + i1 + lo, row + i2 + lo,
// lane + i3 + lo) - (r1, r2, r3) (plus the 16-bit shift), i = floor(d) and
// lo = -1 (cubic) or 0 (linear).  The part that does not depend on the
// floors is formed once per thread; each node adds its floors by 24-bit
// multiply-adds (the floors of a fitting tile are small).
struct BoxAddr {
    int row0;   // byte offset of element (q0 + lo - r1, row + lo - r2, 0) from the box start
    int c3;     // x3 index (in elements) of the stencil start for a zero floor
};
template <typename Tu>
__device__ __forceinline__ BoxAddr box_addr(const Tu *box, const TileIdx &t, const TileBox &B, int lo)
{
    constexpr int PX = box_px<Tu>();
    BoxAddr A;
    A.row0 = (int)lds_addr(box) + ((t.q0 + lo - B.r1) * PY + (t.row + lo - B.r2)) * PX * (int)sizeof(Tu);
    A.c3 = t.lane + lo - B.r3 + B.sh;
    return A;
}
// Byte address of the stencil start of node q (FP32 boxes: any column;
// 16-bit boxes: the even column at or below it, in the copy in which the
// stencil's rows are whole words).
template <typename Tu>
__device__ __forceinline__ unsigned stencil_addr(const BoxAddr &A, int q, float d1, float d2, float d3)
{
    constexpr int PX = box_px<Tu>();
    constexpr int ES = sizeof(Tu);
    const int rowb = A.row0 + q * (PY * PX * ES) + __mul24(floor_small(d1), PY * PX * ES) +
                     __mul24(floor_small(d2), PX * ES);
    const int s3 = A.c3 + floor_small(d3);
    if constexpr (ES == 2)
        return (unsigned)(rowb + (s3 & ~1) * 2 + ((s3 & 1) ? PZ * PY * PX * 2 : 0));
    else
        return (unsigned)(rowb + s3 * ES);
}

// Trilinear gather of the QT nodes of this thread from a staged box (box
// origin at the lowest floor of the tile's feet), with the operations of
// lin_node.
template <typename Tu, int MODE>
__device__ __forceinline__ void compute_tile_lin(const Tu *box, const TileIdx &t, const TileBox &B,
                                                 const float (&d1)[QT], const float (&d2)[QT], const float (&d3)[QT],
                                                 const float (&e)[QT], const SLParams &prm, float (&res)[QT])
{
    constexpr int PX = box_px<Tu>();
    constexpr unsigned ES = sizeof(Tu);
    const BoxAddr A = box_addr(box, t, B, 0);
#pragma unroll
    for (int q = 0; q < QT; ++q) {
        const float a1 = frac_of(d1[q]), a2 = frac_of(d2[q]), a3 = frac_of(d3[q]);
        const unsigned bp = stencil_addr<Tu>(A, q, d1[q], d2[q], d3[q]);
        float x000, x001, x010, x011, x100, x101, x110, x111;
        row2<Tu>(bp, x000, x001);
        row2<Tu>(bp + PX * ES, x010, x011);
        row2<Tu>(bp + PY * PX * ES, x100, x101);
        row2<Tu>(bp + (PY * PX + PX) * ES, x110, x111);
        const float w30 = 1.0f - a3;
        const float s00 = fmaf(a3, x001, w30 * x000);
        const float s01 = fmaf(a3, x011, w30 * x010);
        const float s10 = fmaf(a3, x101, w30 * x100);
        const float s11 = fmaf(a3, x111, w30 * x110);
        const float s0 = fmaf(a2, s01, (1.0f - a2) * s00);
        const float s1v = fmaf(a2, s11, (1.0f - a2) * s10);
        res[q] = epilogue<MODE>(prm, e[q], fmaf(a1, s1v, (1.0f - a1) * s0));
    }
}

// Gather of the QT nodes of this thread from a staged box and the epilogue,
// into res.  ORDER 1: trilinear, 3: tricubic.
template <typename Tu, int MODE, int ORDER>
__device__ __forceinline__ void compute_tile(const Tu *box, const TileIdx &t, const TileBox &B, const float (&d1)[QT], const float (&d2)[QT],
                                             const float (&d3)[QT], const float (&e)[QT], const SLParams &prm,
                                             float (&res)[QT])
{
    constexpr int PX = box_px<Tu>();
    if constexpr (ORDER == 1) {
        compute_tile_lin<Tu, MODE>(box, t, B, d1, d2, d3, e, prm, res);
    } else if constexpr (sizeof(Tu) == 2) {
        // 16-bit box: copy A as loaded, copy B shifted by one element, so the
        // 4 values of any stencil row are two aligned words of one copy
        const BoxAddr A = box_addr(box, t, B, -1);
#pragma unroll
        for (int q = 0; q < QT; ++q) {
            float w1[4], w2[4], w3[4];
            lagrange4_fast(frac_of(d1[q]), w1);
            lagrange4_fast(frac_of(d2[q]), w2);
            lagrange4_fast(frac_of(d3[q]), w3);
            const unsigned bp = stencil_addr<Tu>(A, q, d1[q], d2[q], d3[q]);
            float s = 0.0f;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                unsigned ba = bp + a * PY * PX * 2;
                asm volatile("" : "+v"(ba));
                float sa = 0.0f;
#pragma unroll
                for (int bq = 0; bq < 4; ++bq) {
                    const unsigned rp = ba + bq * PX * 2;
                    sa = fmaf(w2[bq], row4<Tu>(lds_ld_u32(rp), lds_ld_u32(rp + 4), w3), sa);
                }
                s = fmaf(w1[a], sa, s);
                __builtin_amdgcn_sched_barrier(0);
            }
            res[q] = epilogue<MODE>(prm, e[q], s * CUBIC_SCALE);
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        const BoxAddr A = box_addr(box, t, B, -1);
#pragma unroll
        for (int q = 0; q < QT; ++q) {
            float w1[4], w2[4], w3[4];
            lagrange4_fast(frac_of(d1[q]), w1);
            lagrange4_fast(frac_of(d2[q]), w2);
            lagrange4_fast(frac_of(d3[q]), w3);
            const unsigned bp = stencil_addr<Tu>(A, q, d1[q], d2[q], d3[q]);
            float s = 0.0f;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                // one base register per x1 slice: its 16 rows are then
                // within the 8-bit word offsets of paired LDS reads
                unsigned ba = bp + a * PY * PX * (unsigned)sizeof(Tu);
                asm volatile("" : "+v"(ba));
                float sa = 0.0f;
#pragma unroll
                for (int bq = 0; bq < 4; ++bq) {
                    const unsigned rp = ba + bq * PX * (unsigned)sizeof(Tu);
                    float tt = w3[0] * lds_ld<Tu>(rp);
                    tt = fmaf(w3[1], lds_ld<Tu>(rp + sizeof(Tu)), tt);
                    tt = fmaf(w3[2], lds_ld<Tu>(rp + 2 * sizeof(Tu)), tt);
                    tt = fmaf(w3[3], lds_ld<Tu>(rp + 3 * sizeof(Tu)), tt);
                    sa = fmaf(w2[bq], tt, sa);
                }
                s = fmaf(w1[a], sa, s);
                __builtin_amdgcn_sched_barrier(0);
            }
            res[q] = epilogue<MODE>(prm, e[q], s * CUBIC_SCALE);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <typename To>
__device__ __forceinline__ void store_tile(To *__restrict__ out, const TileIdx &t, const float (&res)[QT])
{
    char *b = reinterpret_cast<char *>(out);
    const unsigned o0 = (unsigned)t.p0 * (unsigned)sizeof(To), dq = (unsigned)t.plane * (unsigned)sizeof(To);
#pragma unroll
    for (int q = 0; q < QT; ++q) stf(reinterpret_cast<To *>(b + (o0 + q * dq)), res[q]);
}

// 16-bit boxes: copy B (words after copy A) holds the elements shifted by
// one, B word j = elements 2j+1, 2j+2 of copy A, built from copy A in LDS.
template <typename Tu>
__device__ __forceinline__ void shift_copy(const Tu *box, const TileBox &B)
{
    constexpr int PX = box_px<Tu>();
    constexpr int WPR = PX / 2;                        // words per box row
    const unsigned A0 = lds_addr(box), B0 = A0 + PZ * PY * PX * 2;
    const int nw = (B.E3 + B.sh + 1) >> 1;             // words of copy A in use per row
    const int tot = B.E1 * PY * WPR;
    for (int e = threadIdx.x; e < tot; e += TPB_SL) {
        const int r = e / WPR, j = e - r * WPR;
        const int bb = r - (r / PY) * PY;
        if (bb < B.E2 && j < nw) {
            const unsigned o = (unsigned)e * 4u;
            lds_st_u32(B0 + o, __builtin_amdgcn_alignbit(lds_ld_u32(A0 + o + 4), lds_ld_u32(A0 + o), 16));
        }
    }
}

// A tile whose box exceeds the pitches: each node gathers straight from
// global memory, with the weights and contraction order of the tiled path
// (same results), one node at a time so that the path needs few registers.
template <typename Tu, typename To, int MODE, int ORDER, bool AOS>
__device__ __forceinline__ void tile_fallback(const Grid &g, const Tu *__restrict__ u, const float *__restrict__ d,
                                              const SLParams &prm, To *__restrict__ out, const TileIdx &t)
{
    const size_t N = g.N;
#pragma unroll 1
    for (int q = 0; q < QT; ++q) {
        const int p = t.p0 + q * t.plane;
        float a1, a2, a3;
        foot_of<AOS>(d, N, p, a1, a2, a3);
        const float ev = MODE == SL_STATE ? 0.0f : prm.e[p];
        float v;
        if constexpr (ORDER == 1) {
            v = lin_node(g, u, t.i0 + t.q0 + q, t.j, t.k, a1, a2, a3);
        } else {
            Foot F;
            make_foot(g, t.i0 + t.q0 + q, t.j, t.k, a1, a2, a3, F);
            v = gather(u, F);
        }
        stf(out + p, epilogue<MODE>(prm, ev, v));
    }
}

// One tile per workgroup: the feet, epilogue operands and box of the tile
// are requested together, then one wait, then the gather.  The fitting path
// needs about 50 VGPRs (the global-memory fallback runs one node at a time
// and adds none), so the 39.9 KB box sets the occupancy: four 512-thread
// workgroups per CU, whose phases (waiting for memory, gathering) overlap.
template <typename Tu, typename To, int MODE, int ORDER, bool AOS>
__global__ __launch_bounds__(TPB_SL, 8) void k_sl_tile(Grid g, const Tu *__restrict__ u, const float *__restrict__ d,
                                                  SLParams prm, To *__restrict__ out, const int *__restrict__ boxes,
                                                  int ntx, int nty, int nblk)
{
    constexpr int PX = box_px<Tu>();
    // 16-bit boxes hold two copies (and a word of padding read by the shift)
    constexpr int BOXN = sizeof(Tu) == 2 ? 2 * PZ * PY * PX + 2 : PZ * PY * PX;
    __shared__ __align__(16) Tu box[BOXN];
    // XCD-contiguous tile order (workgroups go round-robin to the 8 XCDs)
    const int b = blockIdx.x;
    const int tile = (nblk & 7) ? b : (b & 7) * (nblk >> 3) + (b >> 3);
    const TileIdx t = tile_idx<SPLIT>(g, tile, ntx, nty);
    const TileBox B = tile_box<Tu>(boxes, tile, t);
    if (!B.fits) {                 // the whole workgroup takes this branch
        tile_fallback<Tu, To, MODE, ORDER, AOS>(g, u, d, prm, out, t);
        return;
    }
    float d1[QT], d2[QT], d3[QT], e[QT], r[QT];
    load_feet<MODE, AOS>(g, d, prm, t, d1, d2, d3, e);
    __builtin_amdgcn_sched_barrier(0);
    stage_box(g, u, box, t, B);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (sizeof(Tu) == 2) {
        shift_copy(box, B);
        __syncthreads();
    }
    compute_tile<Tu, MODE, ORDER>(box, t, B, d1, d2, d3, e, prm, r);
    store_tile(out, t, r);
}

inline bool tiled(const Grid &g) { return g.n3 >= TX && g.n2 >= TY && g.n1 >= TZ; }

inline dim3 grid_of(const Grid &g) { return dim3((g.N + TPB - 1) / TPB); }

// AOS: interleaved feet (the solver's own); otherwise three fields
template <typename Tu, typename To, int MODE, bool AOS = true>
void launch_sl(const Grid &g, const Tu *u, const float *d, const SLParams &prm, To *out, const int *boxes,
               hipStream_t s)
{
    if (tiled(g)) {
        const int ntx = g.n3 / TX, nty = g.n2 / TY, ntz = g.n1 / TZ;
        const int nblk = ntx * nty * ntz;
        if (g.interp == 1)
            hipLaunchKernelGGL((k_sl_tile<Tu, To, MODE, 1, AOS>), dim3(nblk), dim3(TPB_SL), 0, s, g, u, d, prm, out,
                               boxes, ntx, nty, nblk);
        else
            hipLaunchKernelGGL((k_sl_tile<Tu, To, MODE, 3, AOS>), dim3(nblk), dim3(TPB_SL), 0, s, g, u, d, prm, out,
                               boxes, ntx, nty, nblk);
    } else if (g.interp == 1) {
        hipLaunchKernelGGL((k_sl_lin<Tu, To, MODE, AOS>), grid_of(g), dim3(TPB), 0, s, g, u, d, prm, out);
    } else {
        hipLaunchKernelGGL((k_sl_node<Tu, To, MODE, AOS>), grid_of(g), dim3(TPB), 0, s, g, u, d, prm, out);
    }
}

template <bool AOS> void tile_boxes(const Grid &g, const float *d, int *boxes, hipStream_t s)
{
    if (!tiled(g)) return;
    const int ntx = g.n3 / TX, nty = g.n2 / TY, ntz = g.n1 / TZ;
    const int lo = g.interp == 1 ? 0 : 1, span = g.interp == 1 ? 2 : 4;
    hipLaunchKernelGGL(k_tile_boxes<AOS>, dim3(ntx * nty * ntz), dim3(TPB), 0, s, g, d, ntx, nty, boxes, lo, span);
}

} // namespace

void launch_feet(const Grid &g, float dt, const float *v, float *df, float *db, const float *divv, float *c,
                 int *box_f, int *box_b, float *scratch3, hipStream_t s)
{
    const size_t N = g.N;
    // one direction: predictor, interpolate v there (one SL gather per
    // component), corrector; the tile boxes follow the displacements
    auto heun = [&](float a, float b, float *d, int *box) {
        hipLaunchKernelGGL(k_feet_pred, grid_of(g), dim3(TPB), 0, s, g, a, v, d);
        launch_tile_boxes(g, d, box, s);
        for (int k = 0; k < 3; ++k)
            launch_sl<float, float, SL_STATE>(g, v + k * N, d, SLParams{}, scratch3 + k * N, box, s);
        hipLaunchKernelGGL(k_feet_corr, grid_of(g), dim3(TPB), 0, s, g, b, v, scratch3, d);
        launch_tile_boxes(g, d, box, s);
    };
    heun(-dt, -0.5f * dt, df, box_f);
    if (!db) return;
    heun(dt, 0.5f * dt, db, box_b);
    if (!c) return;
    launch_sl<float, float, SL_STATE>(g, divv, db, SLParams{}, scratch3, box_b, s);
    hipLaunchKernelGGL(k_adj_factor, grid_of(g), dim3(TPB), 0, s, g, dt, divv, scratch3, c);
}

size_t tile_box_ints(const Grid &g) { return tiled(g) ? (size_t)8 * (g.N / (TX * TY * TZ)) : 0; }

void launch_tile_boxes(const Grid &g, const float *d, int *boxes, hipStream_t s) { tile_boxes<true>(g, d, boxes, s); }

void launch_feet_fields(const Grid &g, const float *d, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_feet_fields, grid_of(g), dim3(TPB), 0, s, g, d, out);
}

void launch_sl_state(const Grid &g, int dt_u, const void *u, const float *d, const int *boxes, int dt_out, void *out,
                     hipStream_t s)
{
    with_dtype(dt_u, [&](auto tu) {
        using Tu = decltype(tu);
        with_dtype(dt_out, [&](auto to) {
            using To = decltype(to);
            launch_sl<Tu, To, SL_STATE>(g, (const Tu *)u, d, SLParams{}, (To *)out, boxes, s);
        });
    });
}

void launch_sl_adjoint(const Grid &g, int dt_u, const void *u, const float *d, const int *boxes, const float *c,
                       int dt_out, void *out, hipStream_t s)
{
    SLParams prm{};
    prm.e = c;
    with_dtype(dt_u, [&](auto tu) {
        using Tu = decltype(tu);
        with_dtype(dt_out, [&](auto to) {
            using To = decltype(to);
            launch_sl<Tu, To, SL_ADJ>(g, (const Tu *)u, d, prm, (To *)out, boxes, s);
        });
    });
}

void launch_sl_inc(const Grid &g, int dt_q, const void *q, const float *d, const int *boxes, const float *S, float sI,
                   float sS, int dt_out, void *out, hipStream_t s)
{
    SLParams prm{};
    prm.e = S;
    prm.sI = sI;
    prm.sS = sS;
    with_dtype(dt_q, [&](auto tq) {
        using Tq = decltype(tq);
        with_dtype(dt_out, [&](auto to) {
            using To = decltype(to);
            launch_sl<Tq, To, SL_INC>(g, (const Tq *)q, d, prm, (To *)out, boxes, s);
        });
    });
}

// J = det grad y of the map y with m(1) = m0 o y: J^0 = 1, J^{j+1} =
// f . I[J^j](X_f) with the Heun source factor f; work holds 2N floats (f and
// one ping-pong half), the result goes to out (N floats).
void launch_jacobian(const Grid &g, float dt, int nt, const float *divv, const float *df, const int *box_f,
                     float *work, float *out, hipStream_t s)
{
    float *f = work, *tmp = work + (size_t)g.N;
    launch_sl<float, float, SL_STATE>(g, divv, df, SLParams{}, f, box_f, s);
    hipLaunchKernelGGL(k_jac_factor, grid_of(g), dim3(TPB), 0, s, g, dt, divv, f);
    // ping-pong so that the last step writes out
    float *a = (nt & 1) ? tmp : out, *b = (nt & 1) ? out : tmp;
    hipLaunchKernelGGL(k_fill1, grid_of(g), dim3(TPB), 0, s, a, g.N);
    SLParams prm{};
    prm.e = f;
    for (int j = 0; j < nt; ++j) {
        launch_sl<float, float, SL_ADJ>(g, a, df, prm, b, box_f, s);
        std::swap(a, b);
    }
}

// d: three fields from the caller
void launch_interp_f32(const Grid &g, const float *u, const float *d, int *boxes, float *out, hipStream_t s)
{
    tile_boxes<false>(g, d, boxes, s);
    launch_sl<float, float, SL_STATE, false>(g, u, d, SLParams{}, out, boxes, s);
}

} // namespace clh
