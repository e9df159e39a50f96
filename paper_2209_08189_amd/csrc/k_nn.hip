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

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

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
// The 3x3x3 convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16:
// M = 16 voxels, N = 16 output channels, K = 32 = two taps x 16 input
// channels.  Lane l supplies row/column l % 16 of A/B and the 8 K values
// (l / 16, j): tap 2 tp + (l / 32), channel 8 ((l / 16) % 2) + j of the
// 16-channel chunk.  The same (lane, j) -> K assignment is used for both
// operands, so the product is the K sum whatever order the hardware takes
// the K values in.  27 taps are padded to 14 tap pairs with a zero tap.
// Forward packing (flip = 0): K = Ci, N = Co,
//   out[(((kc * 14 + tp) * NT + nt) * 64 + l) * 8 + j] = w[tap][kc*16 + c][nt*16 + l%16]
// Backward-data packing (flip = 1): K = Co, N = Ci, tap 26 - tap,
//   out[...] = w[26 - tap][nt*16 + l%16][kc*16 + c]
// with tap = 2 tp + l / 32, c = 8 ((l / 16) % 2) + j; zero for tap 27.
constexpr int NTP = 14;   // tap pairs

__global__ __launch_bounds__(TPB) void k_pack_w(const float *__restrict__ w, unsigned short *__restrict__ out, int Ci,
                                               int Co, int flip)
{
    const int K = flip ? Co : Ci, Nn = flip ? Ci : Co;
    const int KC = K / 16, NT = Nn / 16;
    const int total = KC * NTP * NT * 512;
    const int e = blockIdx.x * TPB + threadIdx.x;
    if (e >= total) return;
    const int j = e & 7, l = (e >> 3) & 63;
    int r = e >> 9;                  // (kc * NTP + tp) * NT + nt
    const int nt = r % NT;
    r /= NT;
    const int tp = r % NTP, kc = r / NTP;
    const int tap = 2 * tp + (l >> 5);
    const int k = kc * 16 + 8 * ((l >> 4) & 1) + j, n = nt * 16 + (l & 15);
    float val = 0.f;
    if (tap < 27) {
        if (!flip) val = w[((size_t)tap * Ci + k) * Co + n];
        else val = w[((size_t)(26 - tap) * Ci + n) * Co + k];
    }
    out[e] = f2bf(val);
}

// Workgroups are dealt to the 8 XCDs round robin; renumber them so that
// consecutive logical tiles (which share input halos) run on one XCD and
// share its L2.
__device__ __forceinline__ int xcd_tile(int b, int n) { return (n & 7) ? b : (b & 7) * (n >> 3) + (b >> 3); }

__device__ __forceinline__ bf8 as_bf8(u4 v) { return __builtin_bit_cast(bf8, v); }

// --- 3x3x3 convolution (zero padding), LDS-staged MFMA implicit GEMM -------
// in: BF16 [D][H][W][Ci]; wp: packed (K = Ci); bias FP32 [Co] or NULL;
// act: 0 none, 1 LeakyReLU(slope).  out: BF16 or FP32 [D][H][W][Co].
// A workgroup (4 wavefronts) owns a 16 (x) x 4 (y) x MT (z) output brick;
// wavefront w owns the MT x-runs at y = y0 + w and NTS of the NTT 16-channel
// output tiles (group blockIdx.y: tiles NTS blockIdx.y ...; small grids split
// the output channels over several groups to fill the CUs).  Per 16-channel input chunk the 18 x 6 x (MT + 2) input halo is
// staged in LDS once (two planes of 8 channels, so 16 lanes read 256
// contiguous bytes) and serves all 27 taps; B fragments stream from the
// packed weights (L2-resident).
template <int MT, int NTS, typename To>
__global__ __launch_bounds__(TPB) void k_conv3(const unsigned short *__restrict__ in, const u4 *__restrict__ wp,
                                               const float *__restrict__ bias, To *__restrict__ out, int D, int H,
                                               int W, int Ci, int act, float slope, int nbx, int nby, int nblk,
                                               int NTT)
{
    constexpr int XS = 18, YS = 6, ZS = MT + 2, NV = XS * YS * ZS;
    __shared__ u4 tile[2 * NV];
    int b = xcd_tile(blockIdx.x, nblk);
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby, bz = b / nby;
    const int x0 = bx * 16, y0 = by * 4, z0 = bz * MT;
    const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6;
    const int m = l & 15, half = (l >> 4) & 1, tsel = l >> 5;
    const int KC = Ci >> 4, nt0 = blockIdx.y * NTS;
    f4 acc[MT][NTS];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int nt = 0; nt < NTS; ++nt) acc[i][nt] = f4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < KC; ++kc) {
        if (kc) __syncthreads();
        for (int q = tid; q < 2 * NV; q += TPB) {
            const int hq = q & 1, v = q >> 1;
            const int xt = v % XS, r = v / XS;
            const int yt = r % YS, zt = r / YS;
            const int x = x0 - 1 + xt, y = y0 - 1 + yt, z = z0 - 1 + zt;
            u4 val = u4{0u, 0u, 0u, 0u};
            if (x >= 0 && x < W && y >= 0 && y < H && z >= 0 && z < D)
                val = *(const u4 *)(in + (((size_t)z * H + y) * W + x) * Ci + kc * 16 + hq * 8);
            tile[hq * NV + v] = val;
        }
        __syncthreads();
        const u4 *wk = wp + ((size_t)kc * NTP * NTT + nt0) * 64 + l;
        for (int tp = 0; tp < NTP; ++tp) {
            const int tap = 2 * tp + tsel;
            const int tt = tap < 27 ? tap : 13;
            const int dz = tt / 9, dy = (tt / 3) % 3, dx = tt % 3;
            const int base = half * NV + (dz * YS + wv + dy) * XS + m + dx;
            bf8 a[MT];
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                u4 raw = tile[base + i * (YS * XS)];
                if (tap >= 27) raw = u4{0u, 0u, 0u, 0u};
                a[i] = as_bf8(raw);
            }
#pragma unroll
            for (int nt = 0; nt < NTS; ++nt) {
                const bf8 bw = as_bf8(wk[(tp * NTT + nt) * 64]);
#pragma unroll
                for (int i = 0; i < MT; ++i)
                    acc[i][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bw, acc[i][nt], 0, 0, 0);
            }
        }
    }
    // D[m][n]: n = l % 16 (channel), m = 4 (l / 16) + j (voxel along x)
    const int Co = NTT * 16, n = l & 15, xq = x0 + 4 * (l >> 4), y = y0 + wv;
    if (y >= H) return;
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        const int z = z0 + i;
        if (z >= D) continue;
#pragma unroll
        for (int nt = 0; nt < NTS; ++nt) {
            const int co = (nt0 + nt) * 16 + n;
            const float bb = bias ? bias[co] : 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int x = xq + j;
                if (x >= W) continue;
                float v = acc[i][nt][j] + bb;
                if (act) v = v > 0.f ? v : slope * v;
                const size_t o = (((size_t)z * H + y) * W + x) * Co + co;
                if constexpr (sizeof(To) == 2) out[o] = f2bf(v);
                else out[o] = v;
            }
        }
    }
}

// --- weight gradient --------------------------------------------------------
// part[chunk] = (gw partial [t][Ci][Co], gb partial [Co]): sums over the
// chunk's voxels p of X[p + t - 1][i] dZ[p][o] and of dZ[p][o].  GEMM with M = 16 input channels
// (one chunk kc), N = 16 output channels, K = 32 voxels.  A workgroup owns
// one 16-channel input chunk, NG output tiles and a run of 16 x 4 x 2
// voxel tiles.  Per tile, X (with a one-voxel halo) is staged in LDS
// transposed to [channel][z][y][x] in three copies shifted by dx = -1, 0, 1,
// so each A fragment (8 consecutive x of one channel) is one aligned 16-byte
// read, and dZ is staged transposed to [channel][row][x]; the dZ fragments
// are loaded once per tile and serve every tap.  Wavefront w owns the taps
// t = w (mod 4); the bias sums use an all-ones A operand.
// K index (lane group g = l / 16, item j): row 2 s + g / 2 of the tile
// (row = 4 z + y), x = 8 (g % 2) + j, for K step s = 0..3.
template <int NG>
__global__ __launch_bounds__(TPB) void k_conv3_dw(const unsigned short *__restrict__ X,
                                                  const unsigned short *__restrict__ dZ, float *__restrict__ part,
                                                  int D, int H, int W, int Ci, int Co, int ntx, int nty, int ntiles,
                                                  int tpc, int ngrp)
{
    constexpr int XR = 4 * 6;                 // staged X rows: z in [z0-1, z0+2], y in [y0-1, y0+4]
    // channel planes padded by 16 bytes: a plane pitch of 4 (mod 8) words puts
    // the 16-byte A / B fragment reads of the 16 channel lanes on distinct
    // banks (an unpadded pitch, a multiple of 64 words, sent all 16 to the
    // same four banks)
    constexpr int XP = XR * 16 + 8, ZP = 8 * 16 + 8;   // plane pitches in 16-bit elements
    __shared__ __attribute__((aligned(16))) unsigned short xs[3][16][XP];
    __shared__ __attribute__((aligned(16))) unsigned short zs[NG * 16][ZP];
    const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6;
    const int g = l >> 4, ln = l & 15;
    const int KC = Ci >> 4;
    int bq = blockIdx.x;
    const int grp = bq % ngrp;
    bq /= ngrp;
    const int kc = bq % KC, chunk = bq / KC;
    const int co0 = grp * NG * 16;
    const int t0 = chunk * tpc, t1 = min(ntiles, t0 + tpc);
    f4 acc[7][NG], accb[NG];
#pragma unroll
    for (int i = 0; i < 7; ++i)
#pragma unroll
        for (int nt = 0; nt < NG; ++nt) acc[i][nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < NG; ++nt) accb[nt] = f4{0.f, 0.f, 0.f, 0.f};
    const bool do_bias = kc == 0 && wv == 3;
    for (int tI = t0; tI < t1; ++tI) {
        const int tx = tI % ntx, ty = (tI / ntx) % nty, tz = tI / (ntx * nty);
        const int x0 = tx * 16, y0 = ty * 4, z0 = tz * 2;
        __syncthreads();
        // X halo: 18 x 6 x 4 voxels x 16 channels, two 8-channel halves each
        for (int q = tid; q < 18 * XR * 2; q += TPB) {
            const int hq = q & 1, v = q >> 1;
            const int xt = v % 18, r = v / 18;      // r = zt * 6 + yt
            const int yt = r % 6, zt = r / 6;
            const int x = x0 - 1 + xt, y = y0 - 1 + yt, z = z0 - 1 + zt;
            u4 val = u4{0u, 0u, 0u, 0u};
            if (x >= 0 && x < W && y >= 0 && y < H && z >= 0 && z < D)
                val = *(const u4 *)(X + (((size_t)z * H + y) * W + x) * Ci + kc * 16 + hq * 8);
            const unsigned short *e = (const unsigned short *)&val;
#pragma unroll
            for (int sx = 0; sx < 3; ++sx) {
                const int xc = xt - sx;             // copy sx holds X[x0 + xc + sx - 1]
                if (xc < 0 || xc >= 16) continue;
#pragma unroll
                for (int c = 0; c < 8; ++c) xs[sx][hq * 8 + c][r * 16 + xc] = e[c];
            }
        }
        // dZ tile: 16 x 4 x 2 voxels x NG * 16 channels
        for (int q = tid; q < 128 * NG * 2; q += TPB) {
            const int hq = q % (NG * 2), v = q / (NG * 2);
            const int xt = v & 15, r = v >> 4;      // r = zl * 4 + yl
            const int x = x0 + xt, y = y0 + (r & 3), z = z0 + (r >> 2);
            u4 val = u4{0u, 0u, 0u, 0u};
            if (x < W && y < H && z < D)
                val = *(const u4 *)(dZ + (((size_t)z * H + y) * W + x) * Co + co0 + hq * 8);
            const unsigned short *e = (const unsigned short *)&val;
#pragma unroll
            for (int c = 0; c < 8; ++c) zs[hq * 8 + c][r * 16 + xt] = e[c];
        }
        __syncthreads();
        bf8 bz[NG][4];
#pragma unroll
        for (int nt = 0; nt < NG; ++nt)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                bz[nt][s] = as_bf8(*(const u4 *)&zs[nt * 16 + ln][(2 * s + (g >> 1)) * 16 + 8 * (g & 1)]);
#pragma unroll
        for (int ti = 0; ti < 7; ++ti) {
            const int t = wv + 4 * ti;
            if (t >= 27) break;
            const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int row = 2 * s + (g >> 1);               // 4 zl + yl
                const int r = ((row >> 2) + dz) * 6 + (row & 3) + dy;
                const bf8 a = as_bf8(*(const u4 *)&xs[dx][ln][r * 16 + 8 * (g & 1)]);
#pragma unroll
                for (int nt = 0; nt < NG; ++nt)
                    acc[ti][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bz[nt][s], acc[ti][nt], 0, 0, 0);
            }
        }
        if (do_bias) {
            const u4 ones4 = u4{0x3f803f80u, 0x3f803f80u, 0x3f803f80u, 0x3f803f80u};
            const bf8 ones = as_bf8(ones4);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int nt = 0; nt < NG; ++nt)
                    accb[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ones, bz[nt][s], accb[nt], 0, 0, 0);
        }
    }
    // D[m][n]: m = 4 g + j (input channel), n = ln (output channel)
#pragma unroll
    for (int ti = 0; ti < 7; ++ti) {
        const int t = wv + 4 * ti;
        if (t >= 27) break;
        float *dst = part + (size_t)chunk * (27 * Ci * Co + Co) + (size_t)t * Ci * Co;
#pragma unroll
        for (int nt = 0; nt < NG; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                dst[(size_t)(kc * 16 + 4 * g + j) * Co + co0 + nt * 16 + ln] = acc[ti][nt][j];
    }
    if (do_bias && g == 0) {
#pragma unroll
        for (int nt = 0; nt < NG; ++nt) part[(size_t)chunk * (27 * Ci * Co + Co) + 27 * Ci * Co + co0 + nt * 16 + ln] = accb[nt][0];
    }
}

// Fixed-order sum of the chunk partials: row c of partial holds nw weight
// values then nb bias values (row stride nw + nb).  A workgroup owns 64
// consecutive outputs; wave w sums the chunks c = w (mod 4) in order, then
// the four wave sums are added in order.
__global__ __launch_bounds__(TPB) void k_sum_partials(const float *__restrict__ partial, int nchunk, int nw, int nb,
                                                      float *__restrict__ gw, float *__restrict__ gb)
{
    __shared__ float red[TPB / 64][64];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + l;
    const int rs = nw + nb;
    float s = 0.f;
    if (e < rs)
        for (int c = w; c < nchunk; c += TPB / 64) s += partial[(size_t)c * rs + e];
    red[w][l] = s;
    __syncthreads();
    if (w == 0 && e < rs) {
        const float t = ((red[0][l] + red[1][l]) + red[2][l]) + red[3][l];
        if (e < nw) gw[e] = t;
        else if (gb) gb[e - nw] = t;
    }
}

// Elementwise layers on channels-last BF16 tensors work on 8-channel
// groups (one 16-byte load per tensor and thread); channel counts are
// multiples of 16, so a group never straddles two voxels.
__device__ __forceinline__ void unpack8(u4 v, float (&f)[8])
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = __uint_as_float(v[i] << 16);
        f[2 * i + 1] = __uint_as_float(v[i] & 0xffff0000u);
    }
}
__device__ __forceinline__ u4 pack8(const float (&f)[8])
{
    u4 v;
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = (unsigned)f2bf(f[2 * i]) | ((unsigned)f2bf(f[2 * i + 1]) << 16);
    return v;
}

// dZ = dY * (Y > 0 ? 1 : slope)   (LeakyReLU backward from the output sign)
__global__ __launch_bounds__(TPB) void k_lrelu_bwd(const u4 *__restrict__ dY, const u4 *__restrict__ Y, float slope,
                                                   size_t n8, u4 *__restrict__ dZ)
{
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= n8) return;
    float g[8], y[8];
    unpack8(dY[e], g);
    unpack8(Y[e], y);
#pragma unroll
    for (int i = 0; i < 8; ++i) g[i] = y[i] > 0.f ? g[i] : slope * g[i];
    dZ[e] = pack8(g);
}

// 2x2x2 average pooling, channels-last (D, H, W of the input)
__global__ __launch_bounds__(TPB) void k_pool2(const u4 *__restrict__ in, u4 *__restrict__ out, int D, int H, int W,
                                               int C)
{
    const int d = D / 2, h = H / 2, w = W / 2, C8 = C / 8;
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= (size_t)d * h * w * C8) return;
    const int c = e % C8;
    const size_t v = e / C8;
    const int x = v % w, y = (v / w) % h, z = v / ((size_t)w * h);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int q = 0; q < 2; ++q) {
                float f[8];
                unpack8(in[((((size_t)(2 * z + a)) * H + 2 * y + b) * W + 2 * x + q) * C8 + c], f);
#pragma unroll
                for (int i = 0; i < 8; ++i) s[i] += f[i];
            }
#pragma unroll
    for (int i = 0; i < 8; ++i) s[i] *= 0.125f;
    out[e] = pack8(s);
}

// backward of pool2: gin[fine] (+)= gout[coarse] / 8
__global__ __launch_bounds__(TPB) void k_pool2_bwd(const u4 *__restrict__ gout, u4 *__restrict__ gin, int D, int H,
                                                   int W, int C, int accumulate)
{
    const int C8 = C / 8;
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= (size_t)D * H * W * C8) return;
    const int c = e % C8;
    const size_t v = e / C8;
    const int x = v % W, y = (v / W) % H, z = v / ((size_t)W * H);
    float g[8];
    unpack8(gout[((((size_t)z / 2) * (H / 2) + y / 2) * (W / 2) + x / 2) * C8 + c], g);
#pragma unroll
    for (int i = 0; i < 8; ++i) g[i] *= 0.125f;
    if (accumulate) {
        float f[8];
        unpack8(gin[e], f);
#pragma unroll
        for (int i = 0; i < 8; ++i) g[i] = f[i] + g[i];
    }
    gin[e] = pack8(g);
}

// out[p][0:Ca] = a[p / 2], out[p][Ca:Ca+Cb] = b[p]  (D, H, W fine)
__global__ __launch_bounds__(TPB) void k_up2cat(const u4 *__restrict__ a, const u4 *__restrict__ b, u4 *__restrict__ out,
                                                int D, int H, int W, int Ca, int Cb)
{
    const int A8 = Ca / 8, B8 = Cb / 8, C8 = A8 + B8;
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= (size_t)D * H * W * C8) return;
    const int c = e % C8;
    const size_t v = e / C8;
    const int x = v % W, y = (v / W) % H, z = v / ((size_t)W * H);
    if (c < A8) out[e] = a[((((size_t)z / 2) * (H / 2) + y / 2) * (W / 2) + x / 2) * A8 + c];
    else out[e] = b[v * B8 + (c - A8)];
}

// backward of up2cat: ga[coarse] = sum of the 8 children's first Ca
// channels; gb[fine] (+)= last Cb channels
__global__ __launch_bounds__(TPB) void k_up2cat_bwd_a(const u4 *__restrict__ g, u4 *__restrict__ ga, int D, int H, int W,
                                                      int Ca, int Cb)
{
    const int A8 = Ca / 8, C8 = (Ca + Cb) / 8, d = D / 2, h = H / 2, w = W / 2;
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= (size_t)d * h * w * A8) return;
    const int c = e % A8;
    const size_t v = e / A8;
    const int x = v % w, y = (v / w) % h, z = v / ((size_t)w * h);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int q = 0; q < 2; ++q) {
                float f[8];
                unpack8(g[((((size_t)(2 * z + a)) * H + 2 * y + b) * W + 2 * x + q) * C8 + c], f);
#pragma unroll
                for (int i = 0; i < 8; ++i) s[i] += f[i];
            }
    ga[e] = pack8(s);
}

__global__ __launch_bounds__(TPB) void k_up2cat_bwd_b(const u4 *__restrict__ g, u4 *__restrict__ gb, size_t P, int Ca,
                                                      int Cb, int accumulate)
{
    const int A8 = Ca / 8, B8 = Cb / 8;
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= P * B8) return;
    const size_t p = e / B8;
    const int c = e % B8;
    const u4 v = g[p * (A8 + B8) + A8 + c];
    if (!accumulate) {
        gb[e] = v;
        return;
    }
    float f[8], h[8];
    unpack8(v, f);
    unpack8(gb[e], h);
#pragma unroll
    for (int i = 0; i < 8; ++i) h[i] = h[i] + f[i];
    gb[e] = pack8(h);
}

// head: 1x1x1 convolution Ci -> 3, FP32 output as SoA [3][P]
__global__ __launch_bounds__(TPB) void k_head(const unsigned short *__restrict__ in, const float *__restrict__ w,
                                              const float *__restrict__ b, float *__restrict__ out, size_t P, int Ci)
{
    const size_t p = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (p >= P) return;
    float s0 = b[0], s1 = b[1], s2 = b[2];
    const u4 *src = (const u4 *)(in + p * Ci);
    for (int i8 = 0; i8 < Ci / 8; ++i8) {
        float x[8];
        unpack8(src[i8], x);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i8 * 8 + u;
            s0 = fmaf(w[i * 3 + 0], x[u], s0);
            s1 = fmaf(w[i * 3 + 1], x[u], s1);
            s2 = fmaf(w[i * 3 + 2], x[u], s2);
        }
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

// head weight gradient: every workgroup sums, over its voxels, the 16 x 3
// products in[p][i] gout[o][p] and the 3 bias terms gout[o][p] (FP64), then
// writes them as partials[c][block], c = i * 3 + o (bias: 48 + o)
constexpr int HEAD_CI = 16, HEAD_NC = HEAD_CI * 3 + 3;

__global__ __launch_bounds__(TPB) void k_head_bwd_w(const unsigned short *__restrict__ in,
                                                    const float *__restrict__ gout, size_t P,
                                                    double *__restrict__ partials)
{
    double acc[HEAD_NC];
#pragma unroll
    for (int c = 0; c < HEAD_NC; ++c) acc[c] = 0.0;
    for (size_t p = (size_t)blockIdx.x * TPB + threadIdx.x; p < P; p += (size_t)gridDim.x * TPB) {
        const float g0 = gout[p], g1 = gout[P + p], g2 = gout[2 * P + p];
        const u4 lo = *(const u4 *)(in + p * HEAD_CI), hi = *(const u4 *)(in + p * HEAD_CI + 8);
        const unsigned short *e0 = (const unsigned short *)&lo, *e1 = (const unsigned short *)&hi;
#pragma unroll
        for (int i = 0; i < HEAD_CI; ++i) {
            const double x = bf2f(i < 8 ? e0[i] : e1[i - 8]);
            acc[i * 3 + 0] += x * g0;
            acc[i * 3 + 1] += x * g1;
            acc[i * 3 + 2] += x * g2;
        }
        acc[48] += g0;
        acc[49] += g1;
        acc[50] += g2;
    }
#pragma unroll
    for (int c = 0; c < HEAD_NC; ++c) {
        const double v = block_sum(acc[c]);
        if (threadIdx.x == 0) partials[(size_t)c * gridDim.x + blockIdx.x] = v;
    }
}

// out[c] = sum_b partials[c][b] in a fixed order, one workgroup per c
__global__ __launch_bounds__(TPB) void k_finalize_rows(const double *__restrict__ partials, int nb,
                                                       double *__restrict__ out)
{
    const double *row = partials + (size_t)blockIdx.x * nb;
    double acc = 0.0;
    for (int q = threadIdx.x; q < nb; q += TPB) acc += row[q];
    acc = block_sum(acc);
    if (threadIdx.x == 0) out[blockIdx.x] = acc;
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
                                                    u4 *__restrict__ out, size_t P)
{
    const size_t p = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (p >= P) return;
    out[2 * p] = u4{(unsigned)f2bf(a[p]) | ((unsigned)f2bf(b[p]) << 16), 0u, 0u, 0u};
    out[2 * p + 1] = u4{0u, 0u, 0u, 0u};
}

inline unsigned nblk(size_t n) { return (unsigned)((n + TPB - 1) / TPB); }

} // namespace

size_t nn_packed_weight_elems(int Ci, int Co) { return (size_t)NTP * 2 * Ci * Co; }

void nn_pack_weights(const float *w, unsigned short *out, int Ci, int Co, int flip, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_w, dim3(nblk(nn_packed_weight_elems(Ci, Co))), dim3(TPB), 0, s, w, out, Ci, Co, flip);
}

// NTS of the NT output tiles per workgroup, NT / NTS workgroup groups
template <int MT, int NTS, typename To>
static void conv3_launch(const unsigned short *in, const void *wp, const float *bias, To *out, int D, int H, int W,
                         int Ci, int NT, int act, float slope, hipStream_t s)
{
    const int nbx = (W + 15) / 16, nby = (H + 3) / 4, nbz = (D + MT - 1) / MT;
    const int nb = nbx * nby * nbz;
    hipLaunchKernelGGL((k_conv3<MT, NTS, To>), dim3(nb, NT / NTS), dim3(TPB), 0, s, in, (const u4 *)wp, bias, out, D,
                       H, W, Ci, act, slope, nbx, nby, nb, NT);
}

// all NT tiles per workgroup when the bricks alone give 512 workgroups (two
// per CU); otherwise the output channels are split over groups of 2 or 1
// tiles (the input halo of a brick is then staged once per group)
template <int MT, int NT, typename To>
static void conv3_split(const unsigned short *in, const void *wp, const float *bias, To *out, int D, int H, int W,
                        int Ci, int act, float slope, hipStream_t s)
{
    const int nb = ((W + 15) / 16) * ((H + 3) / 4) * ((D + MT - 1) / MT);
    if constexpr (MT == 1 && NT == 12) {
        // one output row per wavefront uses each streamed B fragment once;
        // two rows of 6 tiles in two groups use it twice for the same
        // accumulator count
        if (nb >= 512) {
            conv3_launch<2, 6, To>(in, wp, bias, out, D, H, W, Ci, NT, act, slope, s);
            return;
        }
    }
    if (nb >= 512 || NT == 1) {
        conv3_launch<MT, NT, To>(in, wp, bias, out, D, H, W, Ci, NT, act, slope, s);
        return;
    }
    if constexpr (NT % 2 == 0) {
        if (nb * (NT / 2) >= 512) {
            conv3_launch<MT, 2, To>(in, wp, bias, out, D, H, W, Ci, NT, act, slope, s);
            return;
        }
    }
    conv3_launch<MT, 1, To>(in, wp, bias, out, D, H, W, Ci, NT, act, slope, s);
}

// output rows per wavefront (MT) chosen so that MT * NT accumulator tiles stay near 16
template <typename To>
static void conv3_dispatch(const unsigned short *in, const void *wp, const float *bias, To *out, int D, int H, int W,
                           int Ci, int Co, int act, float slope, hipStream_t s)
{
    switch (Co / 16) {
    case 1: conv3_split<8, 1, To>(in, wp, bias, out, D, H, W, Ci, act, slope, s); break;
    case 2: conv3_split<8, 2, To>(in, wp, bias, out, D, H, W, Ci, act, slope, s); break;
    case 3: conv3_split<4, 3, To>(in, wp, bias, out, D, H, W, Ci, act, slope, s); break;
    case 4: conv3_split<4, 4, To>(in, wp, bias, out, D, H, W, Ci, act, slope, s); break;
    case 6: conv3_split<2, 6, To>(in, wp, bias, out, D, H, W, Ci, act, slope, s); break;
    case 8: conv3_split<2, 8, To>(in, wp, bias, out, D, H, W, Ci, act, slope, s); break;
    case 12: conv3_split<1, 12, To>(in, wp, bias, out, D, H, W, Ci, act, slope, s); break;
    default: break;
    }
}

void nn_conv3(const unsigned short *in, const void *wp, const float *bias, void *out, int out_f32, int D, int H, int W,
              int Ci, int Co, int act, float slope, hipStream_t s)
{
    if (out_f32) conv3_dispatch(in, wp, bias, (float *)out, D, H, W, Ci, Co, act, slope, s);
    else conv3_dispatch(in, wp, bias, (unsigned short *)out, D, H, W, Ci, Co, act, slope, s);
}

// weight-gradient work split: NG output tiles per workgroup, ngrp groups,
// voxel tiles of 16 x 4 x 2 dealt in runs of tpc to nchunk chunks so that
// about 1024 workgroups are in flight
struct DwPlan {
    int ng, ngrp, ntx, nty, ntiles, tpc, nchunk;
};

static DwPlan dw_plan(int D, int H, int W, int Ci, int Co)
{
    DwPlan p{};
    const int nt = Co / 16;
    p.ng = nt % 4 == 0 ? 4 : nt % 3 == 0 ? 3 : nt;
    p.ngrp = nt / p.ng;
    p.ntx = (W + 15) / 16;
    p.nty = (H + 3) / 4;
    p.ntiles = p.ntx * p.nty * ((D + 1) / 2);
    // one resident wave of workgroups: three per CU (one for NG = 4, whose
    // accumulators take the whole register file)
    const int per = (Ci / 16) * p.ngrp;
    const int resident = (p.ng == 4 ? 1 : 3) * 256;
    int want = (resident + per - 1) / per;
    if (want > p.ntiles) want = p.ntiles;
    if (want < 1) want = 1;
    p.tpc = (p.ntiles + want - 1) / want;
    p.nchunk = (p.ntiles + p.tpc - 1) / p.tpc;
    return p;
}

size_t nn_dw_workspace_floats(int D, int H, int W, int Ci, int Co)
{
    const DwPlan p = dw_plan(D, H, W, Ci, Co);
    return (size_t)p.nchunk * (27 * (size_t)Ci * Co + Co);
}

void nn_conv3_dw(const unsigned short *X, const unsigned short *dZ, float *partial, float *gw, float *gb, int D, int H,
                 int W, int Ci, int Co, hipStream_t s)
{
    const DwPlan p = dw_plan(D, H, W, Ci, Co);
    const dim3 grid(p.nchunk * (Ci / 16) * p.ngrp), block(TPB);
    switch (p.ng) {
    case 1: hipLaunchKernelGGL((k_conv3_dw<1>), grid, block, 0, s, X, dZ, partial, D, H, W, Ci, Co, p.ntx, p.nty, p.ntiles, p.tpc, p.ngrp); break;
    case 2: hipLaunchKernelGGL((k_conv3_dw<2>), grid, block, 0, s, X, dZ, partial, D, H, W, Ci, Co, p.ntx, p.nty, p.ntiles, p.tpc, p.ngrp); break;
    case 3: hipLaunchKernelGGL((k_conv3_dw<3>), grid, block, 0, s, X, dZ, partial, D, H, W, Ci, Co, p.ntx, p.nty, p.ntiles, p.tpc, p.ngrp); break;
    case 4: hipLaunchKernelGGL((k_conv3_dw<4>), grid, block, 0, s, X, dZ, partial, D, H, W, Ci, Co, p.ntx, p.nty, p.ntiles, p.tpc, p.ngrp); break;
    default: break;
    }
    const int nw = 27 * Ci * Co;
    hipLaunchKernelGGL(k_sum_partials, dim3((nw + Co + 63) / 64), dim3(TPB), 0, s, partial, p.nchunk, nw, Co, gw, gb);
}

void nn_lrelu_bwd(const unsigned short *dY, const unsigned short *Y, float slope, size_t n, unsigned short *dZ,
                  hipStream_t s)
{
    hipLaunchKernelGGL(k_lrelu_bwd, dim3(nblk(n / 8)), dim3(TPB), 0, s, (const u4 *)dY, (const u4 *)Y, slope, n / 8,
                       (u4 *)dZ);
}

void nn_pool2(const unsigned short *in, unsigned short *out, int D, int H, int W, int C, hipStream_t s)
{
    hipLaunchKernelGGL(k_pool2, dim3(nblk((size_t)D * H * W * C / 64)), dim3(TPB), 0, s, (const u4 *)in, (u4 *)out, D,
                       H, W, C);
}

void nn_pool2_bwd(const unsigned short *gout, unsigned short *gin, int D, int H, int W, int C, int accumulate,
                  hipStream_t s)
{
    hipLaunchKernelGGL(k_pool2_bwd, dim3(nblk((size_t)D * H * W * C / 8)), dim3(TPB), 0, s, (const u4 *)gout, (u4 *)gin,
                       D, H, W, C, accumulate);
}

void nn_up2cat(const unsigned short *a, const unsigned short *b, unsigned short *out, int D, int H, int W, int Ca,
               int Cb, hipStream_t s)
{
    hipLaunchKernelGGL(k_up2cat, dim3(nblk((size_t)D * H * W * (Ca + Cb) / 8)), dim3(TPB), 0, s, (const u4 *)a,
                       (const u4 *)b, (u4 *)out, D, H, W, Ca, Cb);
}

void nn_up2cat_bwd(const unsigned short *g, unsigned short *ga, unsigned short *gb, int D, int H, int W, int Ca, int Cb,
                   int accumulate_b, hipStream_t s)
{
    hipLaunchKernelGGL(k_up2cat_bwd_a, dim3(nblk((size_t)D * H * W * Ca / 64)), dim3(TPB), 0, s, (const u4 *)g, (u4 *)ga,
                       D, H, W, Ca, Cb);
    hipLaunchKernelGGL(k_up2cat_bwd_b, dim3(nblk((size_t)D * H * W * Cb / 8)), dim3(TPB), 0, s, (const u4 *)g, (u4 *)gb,
                       (size_t)D * H * W,
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
    // partials holds HEAD_NC rows of nparts values
    hipLaunchKernelGGL(k_head_bwd_w, dim3(nparts), dim3(TPB), 0, s, in, gout, P, partials);
    hipLaunchKernelGGL(k_finalize_rows, dim3(HEAD_NC), dim3(TPB), 0, s, partials, nparts, dst_dev);
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
    hipLaunchKernelGGL(k_pack_input, dim3(nblk(P)), dim3(TPB), 0, s, a, b, (u4 *)out, P);
}

} // namespace clh
