// internal.h -- declarations shared by the HIP translation units of
// libclairehip.so (kernels + host solver).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <cstddef>
#include <cstdint>

#include "../../include/claire_hip.h"

namespace clh {

// Periodic grid on [0, 2pi)^3 with power-of-two extents (x3 fastest).
struct Grid {
    int n1, n2, n3;
    int l1, l2, l3;       // log2 of the extents
    int N;                // n1 * n2 * n3 (<= 2^30)
    float ih1, ih2, ih3;  // 1 / h_d = n_d / (2 pi)
    float h1, h2, h3;     // h_d = 2 pi / n_d
    int interp;           // interpolation order of every SL step: 3 tricubic, 1 trilinear
};

// ------------------------------------------------------------ storage I/O
template <typename T> __device__ __forceinline__ float ldf(const T *p);
template <> __device__ __forceinline__ float ldf<float>(const float *p) { return *p; }
template <> __device__ __forceinline__ float ldf<__half>(const __half *p) { return __half2float(*p); }
template <> __device__ __forceinline__ float ldf<__hip_bfloat16>(const __hip_bfloat16 *p) { return __bfloat162float(*p); }

// value at storage precision -> FP32 (so that a load can be issued early and
// its conversion placed where the value is used)
__device__ __forceinline__ float tof(float v) { return v; }
__device__ __forceinline__ float tof(__half v) { return __half2float(v); }
__device__ __forceinline__ float tof(__hip_bfloat16 v) { return __bfloat162float(v); }

// element idx of a field at a wave-uniform base, addressed by a 32-bit byte
// offset (a field has at most 2^30 nodes, so idx * sizeof(T) < 2^32): the
// access then takes the scalar-base form with no 64-bit address arithmetic
template <typename T> __device__ __forceinline__ const T &at(const T *base, unsigned idx)
{
    return *(const T *)((const char *)base + idx * (unsigned)sizeof(T));
}
template <typename T> __device__ __forceinline__ T &at(T *base, unsigned idx)
{
    return *(T *)((char *)base + idx * (unsigned)sizeof(T));
}

template <typename T> __device__ __forceinline__ void stf(T *p, float v);
template <> __device__ __forceinline__ void stf<float>(float *p, float v) { *p = v; }
template <> __device__ __forceinline__ void stf<__half>(__half *p, float v) { *p = __float2half(v); }
template <> __device__ __forceinline__ void stf<__hip_bfloat16>(__hip_bfloat16 *p, float v) { *p = __float2bfloat16(v); }

__device__ __forceinline__ void node_of(const Grid &g, int p, int &i, int &j, int &k)
{
    k = p & (g.n3 - 1);
    j = (p >> g.l3) & (g.n2 - 1);
    i = p >> (g.l3 + g.l2);
}

// 8th-order central first derivative along one axis (stride st, coordinate
// c of extent n), times 1/h.
template <typename T>
__device__ __forceinline__ float fd8(const T *__restrict__ u, int p, int c, int n, int st, float ih)
{
    const int base = p - c * st;
    const int m = n - 1;
    float s = 0.8f * (ldf(u + base + ((c + 1) & m) * st) - ldf(u + base + ((c - 1) & m) * st));
    s = fmaf(-0.2f, ldf(u + base + ((c + 2) & m) * st) - ldf(u + base + ((c - 2) & m) * st), s);
    s = fmaf(4.0f / 105.0f, ldf(u + base + ((c + 3) & m) * st) - ldf(u + base + ((c - 3) & m) * st), s);
    s = fmaf(-1.0f / 280.0f, ldf(u + base + ((c + 4) & m) * st) - ldf(u + base + ((c - 4) & m) * st), s);
    return s * ih;
}

// Sum of v over a workgroup of blockDim.x (multiple of 64, <= 1024) threads
// in a fixed order (wavefront shuffles, then wave 0 over the wave sums);
// the result is valid in thread 0.  Every thread of the block must call it;
// the closing barrier keeps wave 0's reads of wsum ahead of the writes of a
// following call.
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double wsum[16];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wsum[w] = v;
    __syncthreads();
    if (w == 0) {
        const int nw = blockDim.x >> 6;
        v = lane < nw ? wsum[lane] : 0.0;
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    }
    __syncthreads();
    return v;
}

inline size_t dtype_size(int dt) { return dt == CL_F32 ? 4 : 2; }

// Run f(T{}) with T the C++ type of storage code dt.
template <typename F> inline void with_dtype(int dt, F &&f)
{
    switch (dt) {
    case CL_BF16: f(__hip_bfloat16{}); break;
    case CL_F16: f(__half{}); break;
    default: f(float{}); break;
    }
}

// ------------------------------------------------------------ launches
// Every launcher enqueues on `s` and returns nothing; errors surface through
// hipGetLastError in the caller.

// epilogue operands of the semi-Lagrangian step kernels
struct SLParams {
    const float *e;       // per-node operand: adjoint factor c, or incremental source s^{j+1}
    float sI, sS;
};

// transport (k_transport.hip)
// Heun feet d_f (and d_b, c when db / c are not NULL) of velocity v, with the
// tile boxes of each; scratch3: 3 FP32 fields of workspace.  The feet are
// stored interleaved (d1 d2 d3 of node p at 3p); every SL step below takes
// them in that layout, except launch_interp_f32 (three fields).
void launch_feet(const Grid &g, float dt, const float *v, float *df, float *db, const float *divv, float *c,
                 int *box_f, int *box_b, float *scratch3, hipStream_t s);
// interleaved feet d -> three fields out
void launch_feet_fields(const Grid &g, const float *d, float *out, hipStream_t s);
// Per-tile stencil bounding boxes of the feet d (8 ints per 8x8x32 tile;
// tile_box_ints() == 0 for grids too small for the tiled kernels).  Computed
// once per velocity and direction and passed to every SL step with those feet.
size_t tile_box_ints(const Grid &g);
void launch_tile_boxes(const Grid &g, const float *d, int *boxes, hipStream_t s);
void launch_sl_state(const Grid &g, int dt_u, const void *u, const float *d, const int *boxes, int dt_out, void *out,
                     hipStream_t s);
void launch_sl_adjoint(const Grid &g, int dt_u, const void *u, const float *d, const int *boxes, const float *c,
                       int dt_out, void *out, hipStream_t s);
// out = sI * I[q](x + d) + sS * S(x), S = s^{j+1} = -vt . grad_h m^{j+1} (FP32)
void launch_sl_inc(const Grid &g, int dt_q, const void *q, const float *d, const int *boxes, const float *S, float sI,
                   float sS, int dt_out, void *out, hipStream_t s);
// boxes: scratch of tile_box_ints(g) ints (filled here from d)
void launch_interp_f32(const Grid &g, const float *u, const float *d, int *boxes, float *out, hipStream_t s);
// det grad y by SL transport with the Heun source factor (forward feet and
// boxes); work: 2N floats; out: N floats
void launch_jacobian(const Grid &g, float dt, int nt, const float *divv, const float *df, const int *box_f,
                     float *work, float *out, hipStream_t s);
// min and max of n floats into out[0], out[1] (FP64), partials: 2 * nblocks
void launch_minmax(const float *a, size_t n, double *partials, int nblocks, double *out, hipStream_t s);

// stencils (k_stencil.hip)
void launch_fd_grad(const Grid &g, const float *u, float *out3, hipStream_t s);
void launch_fd_div(const Grid &g, const float *v, float *out, hipStream_t s);
constexpr int MAX_T = 65;
// G^j = grad_h m^j, j < count (FP32, 3 fields each)
struct StateGradArgs {
    const void *m[MAX_T];
    float *G[MAX_T];
};
void launch_state_grad(const Grid &g, int dt_m, const StateGradArgs &a, int count, hipStream_t s);
// lean layout: out = scale * (-vt . grad_h m), FD8 in the kernel (out stored as dt_out)
void launch_inc_source_fd(const Grid &g, int dt_m, const void *m, const float *vt, float scale, int dt_out, void *out,
                          hipStream_t s);
// incremental sources s^j = -vt . G^j (G^j = G + 3 N j): q0 = scale * s^0
// (stored as dt_q) and S + N (j - 1) = s^j for j = 1..nt (FP32)
void launch_inc_sources(const Grid &g, const float *G, const float *vt, int nt, float scale, int dt_q, void *q0,
                        float *S, hipStream_t s);
struct QuadArgs {
    const void *lam[MAX_T];
    const float *G[MAX_T];    // grad_h m^j (full layout)
    const void *m[MAX_T];     // m^j, gradients by FD8 in the kernel (lean layout)
    float w[MAX_T];
    int count;
    int lean;                 // 1: use m[] (storage dtype dt_m), 0: use G[]
    int dt_m;
};
// all-level sources by the marching FD8 kernel when sources_march(g, nt)
bool sources_march(const Grid &g, int nt);
void launch_inc_sources_march(const Grid &g, int dt_m, const QuadArgs &qa, const float *vt, int nt, float scale,
                              int dt_q, void *q0, float *S, hipStream_t s);
// out3 = addend3 (may be NULL) + sum_j w_j lam^j G^j
void launch_quadrature(const Grid &g, int dt_lam, const QuadArgs &qa, const float *addend3, float *out3, hipStream_t s);
// same, and per-block FP64 partial sums of dp . out3 in partials[0 .. quadrature_blocks(g, qa))
int quadrature_blocks(const Grid &g, const QuadArgs &qa);
// largest block count any quadrature launch on g uses (partials buffer size)
int quadrature_blocks_max(const Grid &g);
// whether the quadrature of qa on g runs the marching FD8 kernel (lean layout)
bool quadrature_marches(const Grid &g, const QuadArgs &qa);
void launch_quadrature_dot(const Grid &g, int dt_lam, const QuadArgs &qa, const float *addend3, float *out3,
                           const float *dp, double *partials, hipStream_t s);
// lam = m1 - mN (stored as dt_lam); partial sums of (m1 - mN)^2 per block
void launch_residual(const Grid &g, int dt_m, const void *m1, const void *mN, int dt_lam, void *lam,
                     double *partials, int nblocks, hipStream_t s);
void launch_sq_diff(const Grid &g, int dt_m, const void *a, const void *b, double *partials, int nblocks,
                    hipStream_t s);

// reductions and vector ops (k_reduce.hip)
int reduce_blocks(size_t n);
void launch_dot(const float *a, const float *b, size_t n, double *partials, int nblocks, hipStream_t s);
void launch_finalize(const double *partials, int nblocks, double scale, double *out, hipStream_t s);
void launch_count_nonfinite(const float *a, size_t n, double *partials, int nblocks, hipStream_t s);
// x += alpha p; r -= alpha Hp; partials of r.r
// Fused PCG: FP64 device scalars sc[PCG_*]
// (PCG_INNER: a second block with the same slots for the inner solve of the
// zero-velocity preconditioner)
enum { PCG_RR = 0, PCG_SUMR = 1, PCG_PHP = 4, PCG_RZ = 5, PCG_RZNEW = 6, PCG_ALPHA = 7, PCG_BETA = 8, PCG_NEG = 9,
       PCG_RZOLD = 10, PCG_INNER = 16, PCG_NSCAL = 32 };
// flexible beta = (rz_new - rz_old) / rz, then rz = rz_new
void launch_pcg_beta_flex(double *sc, hipStream_t s);
// p = z + beta p, q = Lz + beta q (3 n values)
void launch_pcg_direction_lz(float *p, float *q, const float *z, const float *Lz, const double *sc, size_t n,
                             hipStream_t s);
// y += sc[PCG_ALPHA] x over 3 n values
void launch_axpy_sc(float *y, const float *x, const double *sc, size_t n, hipStream_t s);
// p = z + beta p, q = r + beta q, out = q + (G . p) G (beta = sc[PCG_BETA]),
// per-block partials of p . out
void launch_h0_direction_apply(float *p, float *q, const float *z, const float *r, const float *G, float *out,
                               const double *sc, size_t n, double *partials, int nblocks, hipStream_t s);
// z += alpha p, r -= alpha H (alpha = sc[PCG_ALPHA]) over 3 n values
void launch_h0_update(float *z, float *r, const float *p, const float *H, const double *sc, size_t n, hipStream_t s);
// y_c += scale * sums[c] (3 components of n values)
void launch_add_sums3(float *y, const double *sums, double scale, size_t n, hipStream_t s);
// out = Lp + (G . p) G per node (3 components n apart), per-block partials
// of p . out in partials[0 .. nblocks)
void launch_h0_apply(const float *p, const float *Lp, const float *G, float *out, size_t n, double *partials,
                     int nblocks, hipStream_t s);
void launch_pcg_alpha(double *sc, hipStream_t s);
void launch_pcg_beta(double *sc, hipStream_t s);
// x += alpha p, r -= alpha Hp (nothing when alpha = 0); sc[PCG_RR] = rscale
// ||r||^2, sc[PCG_SUMR + c] = sum of component c; partials needs 6 nblocks
// entries
void launch_pcg_update3(float *x, float *r, const float *p, const float *Hp, double *sc, size_t n, double *partials,
                        int nblocks, double rscale, hipStream_t s);
// p = z + beta p, q = (r - mean r) + beta q (beta, means from sc)
void launch_pcg_direction(float *p, float *q, const float *z, const float *r, const double *sc, size_t n,
                          hipStream_t s);
void launch_pcg_update(float *x, float *r, const float *p, const float *Hp, float alpha, size_t n,
                       double *partials, int nblocks, hipStream_t s);
// y = a + alpha * b   (y may alias a)
void launch_axpy(float *y, const float *a, const float *b, float alpha, size_t n, hipStream_t s);
// sums_out[c] = sum of component c of a 3-field vector (device, FP64);
// partials must hold 3 * nblocks doubles
void launch_comp_sums3(const float *a, size_t n, double *partials, int nblocks, double *sums_out, hipStream_t s);
// y_c = (r_c - sums[c] / n) + beta * y_c  (3 components of n values)
void launch_mean_free_axpy(float *y, const float *r, const double *sums, float beta, size_t n, hipStream_t s);
// y = alpha * a  (y may alias a)
void launch_scale(float *y, const float *a, float alpha, size_t n, hipStream_t s);
void launch_convert(int dt_out, void *out, const float *in, size_t n, hipStream_t s);
void launch_to_f32(int dt_in, const void *in, float *out, size_t n, hipStream_t s);
void launch_copy_f32(const float *src, float *dst, size_t n, hipStream_t s);
void launch_fill_f32(float *dst, float v, size_t n, hipStream_t s);

// FFT (k_fft.hip)
// Row pitch of a half spectrum in complex values: nh = n3 / 2 + 1 rounded up
// to a multiple of 16, so that every row starts on a 128-byte boundary (the
// column passes read 16-column tiles of 128-byte row pieces).
__host__ __device__ inline int fft_row_pitch(int n3) { return (n3 / 2 + 1 + 15) & ~15; }
struct FFTPlan {
    int n1, n2, n3, nh;          // nh = n3 / 2 + 1 complex values per x3 row
    int np;                      // row pitch of the half spectrum, fft_row_pitch(n3)
    float2 *tw1, *tw2;           // exp(-2 pi i t / n_d), t < n_d
    float2 *twM;                 // exp(-2 pi i t / M), t < M = n3 / 2
    float2 *twS;                 // exp(-2 pi i k / n3), k <= M (real-FFT split)
    float2 *spec;                // complex work, ncomp_max * n1 * n2 * np
    int ncomp_max;
};
size_t fft_spec_bytes(int n1, int n2, int n3, int ncomp);
// out_c = F^-1[ mult(k) F[in_c] ] (+ add_c), c < ncomp; kind as cl_spectral.
// With beta_w != 0 and ncomp = 3, kinds 0, 1 and 3 couple the components per
// mode (regularisation Hessian L, its inverse, K); in may equal out.
void spectral_apply(const FFTPlan &P, int kind, float beta, float beta_w, int ncomp, const float *in, float *out,
                    const float *add, hipStream_t s);
// out (grid B) = spectral resampling of in (grid A): modes with |k_d| <
// min(n_a, n_b)/2 kept, others zero, scaled so band-limited fields are
// reproduced; both plans' spectra are used as work space
void spectral_resample(const FFTPlan &A, const FFTPlan &B, int ncomp, const float *in, float *out, hipStream_t s);
// host[t] = exp(-2 pi i t / n), t < count, computed in FP64
void fft_make_twiddles(float2 *host, int n, int count);

// read-only views of a registration context for the warm-start code
void ctx_dims(const cl_ctx *ctx, int *n1, int *n2, int *n3);
hipStream_t ctx_stream(const cl_ctx *ctx);
// images of the context as FP32 into m0 / m1 (device, N values each)
void ctx_images_f32(cl_ctx *ctx, float *m0, float *m1);
bool ctx_has_images(const cl_ctx *ctx);

// FFT plan owning its twiddle tables and spectrum (allocated with alloc)
template <typename Alloc> inline void fft_plan_init(FFTPlan &P, int n1, int n2, int n3, int ncomp, Alloc &&alloc)
{
    P.n1 = n1; P.n2 = n2; P.n3 = n3; P.nh = n3 / 2 + 1; P.np = fft_row_pitch(n3); P.ncomp_max = ncomp;
    P.spec = (float2 *)alloc(fft_spec_bytes(n1, n2, n3, ncomp));
    float2 **tabs[4] = {&P.tw1, &P.tw2, &P.twM, &P.twS};
    const int tn[4] = {n1, n2, n3 / 2, n3};
    const int tc[4] = {n1, n2, n3 / 2, n3 / 2 + 1};
    for (int a = 0; a < 4; ++a) {
        float2 *host = new float2[tc[a]];
        fft_make_twiddles(host, tn[a], tc[a]);
        *tabs[a] = (float2 *)alloc(tc[a] * sizeof(float2));
        const hipError_t e = hipMemcpy(*tabs[a], host, tc[a] * sizeof(float2), hipMemcpyHostToDevice);
        delete[] host;
        if (e != hipSuccess) throw e;
    }
}

} // namespace clh
