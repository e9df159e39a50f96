// k_nn.hip -- kernels of the learned warm-start network: a 3D convolutional
// encoder-decoder that predicts an initial stationary velocity from the
// image pair (restricted to a coarser grid); the registration solve stays
// the judge of its output.
//
// Activations are channels-last BF16 tensors [D][H][W][C] (C a multiple of
// 16); arithmetic is FP32.  3x3x3 convolutions run on the matrix cores as an
// implicit GEMM with v_mfma_f32_16x16x16_bf16:
//   M = 16 consecutive voxels along x, N = 16 output channels, K = 16 input
//   channels of one tap; a wavefront owns 16 voxels x all output channels
//   and loops over the 27 taps and the input-channel chunks.
// Operand layouts of the 16x16x16 MFMA (lane l, element j = 0..3):
//   A[m][k]: m = l % 16, k = 4 (l / 16) + j
//   B[k][n]: n = l % 16, k = 4 (l / 16) + j
//   D[m][n]: n = l % 16, m = 4 (l / 16) + j
// Weights are packed once per update into the exact B-fragment order, so a
// B fragment is one 8-byte load per lane.  The transpose needed by the
// backward data pass is the same convolution with flipped taps and swapped
// channel roles, i.e. the same kernel with a differently packed weight.
#include "internal.h"

namespace clh {

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int TPB = 256;

__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }
__device__ __forceinline__ unsigned short f2bf(float f)
{
    // round to nearest even (inputs are finite)
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// --- weight packing -------------------------------------------------------
// w: FP32 [27][Ci][Co].  Forward packing (flip = 0): K = Ci, N = Co,
//   out[((t * KC + kc) * NT + nt) * 64 + l][j] = w[t][kc*16 + 4(l/16) + j][nt*16 + l%16]
// Backward-data packing (flip = 1): K = Co, N = Ci, tap 26 - t,
//   out[...] = w[26 - t][nt*16 + l%16][kc*16 + 4(l/16) + j]
__global__ __launch_bounds__(TPB) void k_pack_w(const float *__restrict__ w, unsigned short *__restrict__ out, int Ci,
                                               int Co, int flip)
{
    const int K = flip ? Co : Ci, Nn = flip ? Ci : Co;
    const int KC = K / 16, NT = Nn / 16;
    const int total = 27 * K * Nn;
    const int e = blockIdx.x * TPB + threadIdx.x;
    if (e >= total) return;
    const int j = e & 3, l = (e >> 2) & 63;
    int r = e >> 8;                  // ((t * KC + kc) * NT + nt)
    const int nt = r % NT;
    r /= NT;
    const int kc = r % KC, t = r / KC;
    const int k = kc * 16 + 4 * (l >> 4) + j, n = nt * 16 + (l & 15);
    float val;
    if (!flip) val = w[((size_t)t * Ci + k) * Co + n];
    else val = w[((size_t)(26 - t) * Ci + n) * Co + k];
    out[e] = f2bf(val);
}

// --- 3x3x3 convolution (zero padding), MFMA implicit GEMM ----------------
// in: BF16 [D][H][W][Ci]; wp: packed (K = Ci); bias FP32 [Co] or NULL;
// act: 0 none, 1 LeakyReLU(slope).  out: BF16 or FP32 [D][H][W][Co].
template <int NT, typename To>
__global__ __launch_bounds__(TPB) void k_conv3(const unsigned short *__restrict__ in, const s4 *__restrict__ wp,
                                               const float *__restrict__ bias, To *__restrict__ out, int D, int H,
                                               int W, int Ci, int act, float slope)
{
    const int l = threadIdx.x & 63;
    const int wave = blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
    const int WB = (W + 15) >> 4;            // x blocks of 16 (the last may be partial)
    if (wave >= D * H * WB) return;           // whole wavefront exits together
    const int x0 = (wave % WB) << 4, y = (wave / WB) % H, z = wave / (WB * H);
    const int KC = Ci >> 4;
    const int Co = NT * 16;
    f4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
    const int xi = x0 + (l & 15), kq = 4 * (l >> 4);
    for (int t = 0; t < 27; ++t) {
        const int zz = z + t / 9 - 1, yy = y + (t / 3) % 3 - 1, xx = xi + t % 3 - 1;
        if (zz < 0 || zz >= D || yy < 0 || yy >= H) continue;   // uniform per wave
        const bool ok = xx >= 0 && xx < W;
        const unsigned short *src = in + (((size_t)zz * H + yy) * W + (ok ? xx : 0)) * Ci + kq;
        const s4 *wt = wp + (size_t)t * KC * NT * 64 + l;
        for (int kc = 0; kc < KC; ++kc) {
            s4 a = ok ? *(const s4 *)(src + kc * 16) : s4{0, 0, 0, 0};
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, wt[(kc * NT + nt) * 64], acc[nt], 0, 0, 0);
        }
    }
    const int n = l & 15;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int co = nt * 16 + n;
        const float b = bias ? bias[co] : 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int x = x0 + kq + j;
            if (x >= W) continue;
            float v = acc[nt][j] + b;
            if (act) v = v > 0.f ? v : slope * v;
            const size_t o = (((size_t)z * H + y) * W + x) * Co + co;
            if constexpr (sizeof(To) == 2) out[o] = f2bf(v);
            else out[o] = v;
        }
    }
}

// --- weight gradient: partial[chunk][t][Ci][Co] = sum over the chunk's
// voxels p of X[p + t - 1][i] dZ[p][o].  One wavefront per (chunk, tap,
// 16-input-channel tile); K = voxels, 16 consecutive x per MFMA.
template <int NT>
__global__ __launch_bounds__(64) void k_conv3_dw(const unsigned short *__restrict__ X, const unsigned short *__restrict__ dZ,
                                                 float *__restrict__ partial, int D, int H, int W, int Ci,
                                                 int rows_per_chunk)
{
    const int l = threadIdx.x;
    const int KC = Ci >> 4, Co = NT * 16;
    const int t = blockIdx.x % 27;
    const int kc = (blockIdx.x / 27) % KC;
    const int chunk = blockIdx.x / (27 * KC);
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const int WB = (W + 15) >> 4;
    const int nrows = D * H * WB;
    f4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = f4{0.f, 0.f, 0.f, 0.f};
    const int i = kc * 16 + (l & 15), kq = 4 * (l >> 4);
    const int r0 = chunk * rows_per_chunk, r1 = min(nrows, r0 + rows_per_chunk);
    for (int r = r0; r < r1; ++r) {
        const int x0 = (r % WB) << 4, y = (r / WB) % H, z = r / (WB * H);
        const int zz = z + dz, yy = y + dy;
        const bool zy_ok = zz >= 0 && zz < D && yy >= 0 && yy < H;
        s4 a;
        const unsigned short *xrow = X + (((size_t)(zy_ok ? zz : 0) * H + (zy_ok ? yy : 0)) * W) * Ci + i;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int xx = x0 + kq + j + dx;
            a[j] = (zy_ok && xx >= 0 && xx < W && x0 + kq + j < W) ? (short)xrow[(size_t)xx * Ci] : (short)0;
        }
        const unsigned short *zrow = dZ + (((size_t)z * H + y) * W + x0 + kq) * Co + (l & 15);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            s4 b;
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = x0 + kq + j < W ? (short)zrow[(size_t)j * Co + nt * 16] : (short)0;
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[nt], 0, 0, 0);
        }
    }
    float *dst = partial + ((size_t)chunk * 27 + t) * Ci * Co;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int j = 0; j < 4; ++j) dst[(size_t)(kc * 16 + kq + j) * Co + nt * 16 + (l & 15)] = acc[nt][j];
}

// out[e] = sum_c partial[c][e] (fixed order)
__global__ __launch_bounds__(TPB) void k_sum_partials(const float *__restrict__ partial, int nchunk, size_t n,
                                                      float *__restrict__ out)
{
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= n) return;
    float s = 0.f;
    for (int c = 0; c < nchunk; ++c) s += partial[(size_t)c * n + e];
    out[e] = s;
}

// gb[o] = sum_p dZ[p][o]; one workgroup per output channel, fixed order
__global__ __launch_bounds__(TPB) void k_bias_grad(const unsigned short *__restrict__ dZ, size_t P, int C,
                                                   float *__restrict__ gb)
{
    const int o = blockIdx.x;
    double s = 0.0;
    for (size_t p = threadIdx.x; p < P; p += TPB) s += bf2f(dZ[p * C + o]);
    s = block_sum(s);
    if (threadIdx.x == 0) gb[o] = (float)s;
}

// dZ = dY * (Y > 0 ? 1 : slope)   (LeakyReLU backward from the output sign)
__global__ __launch_bounds__(TPB) void k_lrelu_bwd(const unsigned short *__restrict__ dY,
                                                   const unsigned short *__restrict__ Y, float slope, size_t n,
                                                   unsigned short *__restrict__ dZ)
{
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= n) return;
    const float g = bf2f(dY[e]);
    dZ[e] = f2bf(bf2f(Y[e]) > 0.f ? g : slope * g);
}

// 2x2x2 average pooling, channels-last (D, H, W of the input)
__global__ __launch_bounds__(TPB) void k_pool2(const unsigned short *__restrict__ in, unsigned short *__restrict__ out,
                                               int D, int H, int W, int C)
{
    const int d = D / 2, h = H / 2, w = W / 2;
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= (size_t)d * h * w * C) return;
    const int c = e % C;
    size_t v = e / C;
    const int x = v % w, y = (v / w) % h, z = v / ((size_t)w * h);
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int q = 0; q < 2; ++q) s += bf2f(in[((((size_t)(2 * z + a)) * H + 2 * y + b) * W + 2 * x + q) * C + c]);
    out[e] = f2bf(0.125f * s);
}

// backward of pool2: gin[fine] (+)= gout[coarse] / 8
__global__ __launch_bounds__(TPB) void k_pool2_bwd(const unsigned short *__restrict__ gout, unsigned short *__restrict__ gin,
                                                   int D, int H, int W, int C, int accumulate)
{
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= (size_t)D * H * W * C) return;
    const int c = e % C;
    size_t v = e / C;
    const int x = v % W, y = (v / W) % H, z = v / ((size_t)W * H);
    const float g = 0.125f * bf2f(gout[((((size_t)z / 2) * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c]);
    gin[e] = f2bf(accumulate ? bf2f(gin[e]) + g : g);
}

// out[p][0:Ca] = a[p / 2], out[p][Ca:Ca+Cb] = b[p]  (D, H, W fine)
__global__ __launch_bounds__(TPB) void k_up2cat(const unsigned short *__restrict__ a, const unsigned short *__restrict__ b,
                                                unsigned short *__restrict__ out, int D, int H, int W, int Ca, int Cb)
{
    const int C = Ca + Cb;
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= (size_t)D * H * W * C) return;
    const int c = e % C;
    size_t v = e / C;
    const int x = v % W, y = (v / W) % H, z = v / ((size_t)W * H);
    if (c < Ca) out[e] = a[((((size_t)z / 2) * (H / 2) + y / 2) * (W / 2) + x / 2) * Ca + c];
    else out[e] = b[v * Cb + (c - Ca)];
}

// backward of up2cat: ga[coarse] = sum of the 8 children's first Ca
// channels; gb[fine] (+)= last Cb channels
__global__ __launch_bounds__(TPB) void k_up2cat_bwd_a(const unsigned short *__restrict__ g, unsigned short *__restrict__ ga,
                                                      int D, int H, int W, int Ca, int Cb)
{
    const int C = Ca + Cb, d = D / 2, h = H / 2, w = W / 2;
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= (size_t)d * h * w * Ca) return;
    const int c = e % Ca;
    size_t v = e / Ca;
    const int x = v % w, y = (v / w) % h, z = v / ((size_t)w * h);
    float s = 0.f;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int q = 0; q < 2; ++q) s += bf2f(g[((((size_t)(2 * z + a)) * H + 2 * y + b) * W + 2 * x + q) * C + c]);
    ga[e] = f2bf(s);
}

__global__ __launch_bounds__(TPB) void k_up2cat_bwd_b(const unsigned short *__restrict__ g, unsigned short *__restrict__ gb,
                                                      size_t P, int Ca, int Cb, int accumulate)
{
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= P * Cb) return;
    const size_t p = e / Cb;
    const int c = e % Cb;
    const float v = bf2f(g[p * (Ca + Cb) + Ca + c]);
    gb[e] = f2bf(accumulate ? bf2f(gb[e]) + v : v);
}

// head: 1x1x1 convolution Ci -> 3, FP32 output as SoA [3][P]
__global__ __launch_bounds__(TPB) void k_head(const unsigned short *__restrict__ in, const float *__restrict__ w,
                                              const float *__restrict__ b, float *__restrict__ out, size_t P, int Ci)
{
    const size_t p = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (p >= P) return;
    float s0 = b[0], s1 = b[1], s2 = b[2];
    for (int i = 0; i < Ci; ++i) {
        const float x = bf2f(in[p * Ci + i]);
        s0 = fmaf(w[i * 3 + 0], x, s0);
        s1 = fmaf(w[i * 3 + 1], x, s1);
        s2 = fmaf(w[i * 3 + 2], x, s2);
    }
    out[p] = s0;
    out[P + p] = s1;
    out[2 * P + p] = s2;
}

// head backward: gin[p][i] = sum_o w[i][o] gout[o][p]  (BF16 out)
__global__ __launch_bounds__(TPB) void k_head_bwd_x(const float *__restrict__ gout, const float *__restrict__ w,
                                                    unsigned short *__restrict__ gin, size_t P, int Ci)
{
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= P * Ci) return;
    const size_t p = e / Ci;
    const int i = e % Ci;
    const float g = w[i * 3 + 0] * gout[p] + w[i * 3 + 1] * gout[P + p] + w[i * 3 + 2] * gout[2 * P + p];
    gin[e] = f2bf(g);
}

// head weight gradient: per workgroup partial sums over voxels, then a
// second pass; out[(i * 3 + o)] for i < Ci, then 3 bias entries
__global__ __launch_bounds__(TPB) void k_head_bwd_w(const unsigned short *__restrict__ in, const float *__restrict__ gout,
                                                    size_t P, int Ci, int comp, double *__restrict__ partials)
{
    // comp = i * 3 + o for weights, Ci * 3 + o for the bias
    const int i = comp / 3, o = comp % 3;
    double s = 0.0;
    for (size_t p = (size_t)blockIdx.x * TPB + threadIdx.x; p < P; p += (size_t)gridDim.x * TPB) {
        const float x = i < Ci ? bf2f(in[p * Ci + i]) : 1.0f;
        s += (double)x * gout[o * P + p];
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// loss = 0.5 / P sum (pred - label)^2 over 3 components; grad = (pred - label) / P
__global__ __launch_bounds__(TPB) void k_mse(const float *__restrict__ pred, const float *__restrict__ label, size_t n,
                                             float inv, float *__restrict__ grad, double *__restrict__ partials)
{
    double s = 0.0;
    for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < n; e += (size_t)gridDim.x * TPB) {
        const float r = pred[e] - label[e];
        grad[e] = r * inv;
        s += (double)r * r;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Adam on FP32 master parameters
__global__ __launch_bounds__(TPB) void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2)
{
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= n) return;
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// two FP32 scalar fields [P] -> BF16 channels-last [P][16] (channels 2..15 zero)
__global__ __launch_bounds__(TPB) void k_pack_input(const float *__restrict__ a, const float *__restrict__ b,
                                                    unsigned short *__restrict__ out, size_t P)
{
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= P * 16) return;
    const size_t p = e >> 4;
    const int c = e & 15;
    out[e] = c == 0 ? f2bf(a[p]) : c == 1 ? f2bf(b[p]) : (unsigned short)0;
}

inline unsigned nblk(size_t n) { return (unsigned)((n + TPB - 1) / TPB); }

} // namespace

void nn_pack_weights(const float *w, unsigned short *out, int Ci, int Co, int flip, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_w, dim3(nblk((size_t)27 * Ci * Co)), dim3(TPB), 0, s, w, out, Ci, Co, flip);
}

template <typename To>
static void conv3_dispatch(const unsigned short *in, const void *wp, const float *bias, To *out, int D, int H, int W,
                           int Ci, int Co, int act, float slope, hipStream_t s)
{
    const int waves = D * H * ((W + 15) / 16);
    const dim3 grid((waves + 3) / 4), block(TPB);
    const s4 *w = (const s4 *)wp;
    switch (Co / 16) {
    case 1: hipLaunchKernelGGL((k_conv3<1, To>), grid, block, 0, s, in, w, bias, out, D, H, W, Ci, act, slope); break;
    case 2: hipLaunchKernelGGL((k_conv3<2, To>), grid, block, 0, s, in, w, bias, out, D, H, W, Ci, act, slope); break;
    case 3: hipLaunchKernelGGL((k_conv3<3, To>), grid, block, 0, s, in, w, bias, out, D, H, W, Ci, act, slope); break;
    case 4: hipLaunchKernelGGL((k_conv3<4, To>), grid, block, 0, s, in, w, bias, out, D, H, W, Ci, act, slope); break;
    case 6: hipLaunchKernelGGL((k_conv3<6, To>), grid, block, 0, s, in, w, bias, out, D, H, W, Ci, act, slope); break;
    case 8: hipLaunchKernelGGL((k_conv3<8, To>), grid, block, 0, s, in, w, bias, out, D, H, W, Ci, act, slope); break;
    case 12: hipLaunchKernelGGL((k_conv3<12, To>), grid, block, 0, s, in, w, bias, out, D, H, W, Ci, act, slope); break;
    default: break;
    }
}

void nn_conv3(const unsigned short *in, const void *wp, const float *bias, void *out, int out_f32, int D, int H, int W,
              int Ci, int Co, int act, float slope, hipStream_t s)
{
    if (out_f32) conv3_dispatch(in, wp, bias, (float *)out, D, H, W, Ci, Co, act, slope, s);
    else conv3_dispatch(in, wp, bias, (unsigned short *)out, D, H, W, Ci, Co, act, slope, s);
}

int nn_dw_chunks(int D, int H, int W, int *rows_per_chunk)
{
    const int nrows = D * H * ((W + 15) / 16);
    int rpc = 256;
    if (rpc > nrows) rpc = nrows;
    *rows_per_chunk = rpc;
    return (nrows + rpc - 1) / rpc;
}

void nn_conv3_dw(const unsigned short *X, const unsigned short *dZ, float *partial, float *gw, float *gb, int D, int H,
                 int W, int Ci, int Co, hipStream_t s)
{
    int rpc;
    const int nchunk = nn_dw_chunks(D, H, W, &rpc);
    const dim3 grid(nchunk * 27 * (Ci / 16)), block(64);
    switch (Co / 16) {
    case 1: hipLaunchKernelGGL((k_conv3_dw<1>), grid, block, 0, s, X, dZ, partial, D, H, W, Ci, rpc); break;
    case 2: hipLaunchKernelGGL((k_conv3_dw<2>), grid, block, 0, s, X, dZ, partial, D, H, W, Ci, rpc); break;
    case 3: hipLaunchKernelGGL((k_conv3_dw<3>), grid, block, 0, s, X, dZ, partial, D, H, W, Ci, rpc); break;
    case 4: hipLaunchKernelGGL((k_conv3_dw<4>), grid, block, 0, s, X, dZ, partial, D, H, W, Ci, rpc); break;
    case 6: hipLaunchKernelGGL((k_conv3_dw<6>), grid, block, 0, s, X, dZ, partial, D, H, W, Ci, rpc); break;
    case 8: hipLaunchKernelGGL((k_conv3_dw<8>), grid, block, 0, s, X, dZ, partial, D, H, W, Ci, rpc); break;
    case 12: hipLaunchKernelGGL((k_conv3_dw<12>), grid, block, 0, s, X, dZ, partial, D, H, W, Ci, rpc); break;
    default: break;
    }
    const size_t n = (size_t)27 * Ci * Co;
    hipLaunchKernelGGL(k_sum_partials, dim3(nblk(n)), dim3(TPB), 0, s, partial, nchunk, n, gw);
    if (gb) hipLaunchKernelGGL(k_bias_grad, dim3(Co), dim3(TPB), 0, s, dZ, (size_t)D * H * W, Co, gb);
}

void nn_lrelu_bwd(const unsigned short *dY, const unsigned short *Y, float slope, size_t n, unsigned short *dZ,
                  hipStream_t s)
{
    hipLaunchKernelGGL(k_lrelu_bwd, dim3(nblk(n)), dim3(TPB), 0, s, dY, Y, slope, n, dZ);
}

void nn_pool2(const unsigned short *in, unsigned short *out, int D, int H, int W, int C, hipStream_t s)
{
    hipLaunchKernelGGL(k_pool2, dim3(nblk((size_t)D * H * W * C / 8)), dim3(TPB), 0, s, in, out, D, H, W, C);
}

void nn_pool2_bwd(const unsigned short *gout, unsigned short *gin, int D, int H, int W, int C, int accumulate,
                  hipStream_t s)
{
    hipLaunchKernelGGL(k_pool2_bwd, dim3(nblk((size_t)D * H * W * C)), dim3(TPB), 0, s, gout, gin, D, H, W, C, accumulate);
}

void nn_up2cat(const unsigned short *a, const unsigned short *b, unsigned short *out, int D, int H, int W, int Ca,
               int Cb, hipStream_t s)
{
    hipLaunchKernelGGL(k_up2cat, dim3(nblk((size_t)D * H * W * (Ca + Cb))), dim3(TPB), 0, s, a, b, out, D, H, W, Ca, Cb);
}

void nn_up2cat_bwd(const unsigned short *g, unsigned short *ga, unsigned short *gb, int D, int H, int W, int Ca, int Cb,
                   int accumulate_b, hipStream_t s)
{
    hipLaunchKernelGGL(k_up2cat_bwd_a, dim3(nblk((size_t)D * H * W * Ca / 8)), dim3(TPB), 0, s, g, ga, D, H, W, Ca, Cb);
    hipLaunchKernelGGL(k_up2cat_bwd_b, dim3(nblk((size_t)D * H * W * Cb)), dim3(TPB), 0, s, g, gb, (size_t)D * H * W,
                       Ca, Cb, accumulate_b);
}

void nn_head(const unsigned short *in, const float *w, const float *b, float *out, size_t P, int Ci, hipStream_t s)
{
    hipLaunchKernelGGL(k_head, dim3(nblk(P)), dim3(TPB), 0, s, in, w, b, out, P, Ci);
}

void nn_head_bwd(const unsigned short *in, const float *gout, const float *w, unsigned short *gin, double *partials,
                 int nparts, double *dst_dev, size_t P, int Ci, hipStream_t s)
{
    hipLaunchKernelGGL(k_head_bwd_x, dim3(nblk(P * Ci)), dim3(TPB), 0, s, gout, w, gin, P, Ci);
    for (int comp = 0; comp < 3 * (Ci + 1); ++comp) {
        hipLaunchKernelGGL(k_head_bwd_w, dim3(nparts), dim3(TPB), 0, s, in, gout, P, Ci, comp, partials);
        launch_finalize(partials, nparts, 1.0, dst_dev + comp, s);
    }
}

void nn_mse(const float *pred, const float *label, size_t n, float inv, float *grad, double *partials, int nparts,
            hipStream_t s)
{
    hipLaunchKernelGGL(k_mse, dim3(nparts), dim3(TPB), 0, s, pred, label, n, inv, grad, partials);
}

void nn_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2, float eps, float c1,
             float c2, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(TPB), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

void nn_pack_input(const float *a, const float *b, unsigned short *out, size_t P, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_input, dim3(nblk(P * 16)), dim3(TPB), 0, s, a, b, out, P);
}

} // namespace clh
