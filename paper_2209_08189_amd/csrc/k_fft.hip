// k_fft.hip -- 3D real FFT spectral operators for gfx950 (Section 2.2: a
// spectral operator costs two FFTs and one Hadamard product; Section 3 uses
// a vendor 3D FFT on one GPU, here it is written from scratch).
//
// Layout: real fields [n1][n2][n3]; half spectrum [n1][n2][nh], nh = n3/2+1.
// One spectral apply is five LDS-staged passes, each a single read and a
// single write of the field:
//   x3 R2C    rows of n3 reals packed as n3/2 complex, radix-2 DIF in LDS,
//             split into the half spectrum of the real row;
//   x2 C2C    columns of a fixed-x1 plane, DIF, natural-order store;
//   x1 fused  columns along x1: DIF forward (bit-reversed order in LDS),
//             Hadamard multiply by the symbol, DIT inverse (natural order)
//             -- no permutation pass is needed in between;
//   x2 C2C    inverse;
//   x3 C2R    Hermitian merge, inverse, unpack to reals, optional fused add.
// Twiddles e^{-2 pi i t / n} come from tables computed on the host in FP64
// and are staged in LDS; data tiles use at most 32 KB of LDS.
#include "internal.h"

#include <cmath>

namespace clh {

namespace {

constexpr int TPB = 256;
constexpr int LDS_C = 4096;   // complex values per data tile

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

__device__ __forceinline__ int brev(int q, int logL) { return logL ? (int)(__brev((unsigned)q) >> (32 - logL)) : 0; }

// In-place radix-2 FFT of nl lines of length L = 2^logL in LDS; element
// (line l, index q) at buf[l * ls + q * es].  tw[t * tws] = e^{-2 pi i t/L}.
// DIF: natural order in, bit-reversed out.  DIT: bit-reversed in, natural
// out.  inv conjugates the twiddles.  line_fast maps consecutive threads to
// consecutive lines (column tiles) instead of consecutive butterflies.
template <bool DIF>
__device__ void lds_fft(float2 *buf, int logL, int lognl, int ls, int es, const float2 *tw, int tws, bool inv,
                        bool line_fast)
{
    const int L = 1 << logL;
    const int nb = (1 << lognl) * (L >> 1);
    const int nlm = (1 << lognl) - 1, hm = (L >> 1) - 1;
    for (int s = 0; s < logL; ++s) {
        const int loghalf = DIF ? (logL - 1 - s) : s;
        const int half = 1 << loghalf;
        const int tstep = (L >> (loghalf + 1)) * tws;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            int l, t;
            if (line_fast) { l = b & nlm; t = b >> lognl; }
            else { t = b & hm; l = b >> (logL - 1); }
            const int grp = t >> loghalf, pos = t & (half - 1);
            const int ia = (grp << (loghalf + 1)) + pos, ib = ia + half;
            float2 w = tw[pos * tstep];
            if (inv) w.y = -w.y;
            float2 *pa = buf + l * ls + ia * es, *pb = buf + l * ls + ib * es;
            const float2 x = *pa, y = *pb;
            if (DIF) {
                *pa = cadd(x, y);
                *pb = cmul(csub(x, y), w);
            } else {
                const float2 t2 = cmul(y, w);
                *pa = cadd(x, t2);
                *pb = csub(x, t2);
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void load_tw(float2 *dst, const float2 *__restrict__ src, int n)
{
    for (int t = threadIdx.x; t < n; t += blockDim.x) dst[t] = src[t];
}

// --- x3 forward: real rows -> half spectrum.  R rows per workgroup.
__global__ __launch_bounds__(TPB) void k_fft_x3_r2c(const float *__restrict__ in, float2 *__restrict__ spec,
                                                    const float2 *__restrict__ tw3, int n3, int logM, int logR,
                                                    int nrows, size_t in_cstride, size_t spec_cstride)
{
    extern __shared__ float2 sm[];
    const int M = 1 << logM, R = 1 << logR, nh = M + 1;
    float2 *tw = sm;                  // M entries: e^{-2 pi i t / n3}
    float2 *buf = sm + M;             // R * M
    const int comp = blockIdx.y;
    const float2 *src = (const float2 *)(in + comp * in_cstride);
    float2 *dst = spec + comp * spec_cstride;
    const int row0 = blockIdx.x * R;
    load_tw(tw, tw3, M);
    for (int e = threadIdx.x; e < R * M; e += blockDim.x) {
        const int r = e >> logM, q = e & (M - 1);
        buf[e] = row0 + r < nrows ? src[(size_t)(row0 + r) * M + q] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    lds_fft<true>(buf, logM, logR, M, 1, tw, 2, false, false);
    // split: X[k] = E[k] + w^k O[k], E = (Z[k] + conj Z[M-k]) / 2, O = -i (Z[k] - conj Z[M-k]) / 2
    for (int e = threadIdx.x; e < R * nh; e += blockDim.x) {
        const int r = e / nh, k = e - r * nh;
        if (row0 + r >= nrows) continue;
        const float2 *z = buf + r * M;
        const float2 zk = z[brev(k & (M - 1), logM)];
        const float2 zc = cconj(z[brev((M - k) & (M - 1), logM)]);
        const float2 E = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
        const float2 O = make_float2(0.5f * (zk.y - zc.y), -0.5f * (zk.x - zc.x));
        const float2 w = k < M ? tw[k] : make_float2(-1.f, 0.f);
        dst[(size_t)(row0 + r) * nh + k] = cadd(E, cmul(w, O));
    }
}

// --- x3 inverse: half spectrum -> real rows (unnormalised), optional add.
__global__ __launch_bounds__(TPB) void k_fft_x3_c2r(const float2 *__restrict__ spec, float *__restrict__ out,
                                                    const float *__restrict__ add, const float2 *__restrict__ tw3,
                                                    int n3, int logM, int logR, int nrows, size_t out_cstride,
                                                    size_t spec_cstride)
{
    extern __shared__ float2 sm[];
    const int M = 1 << logM, R = 1 << logR, nh = M + 1;
    float2 *tw = sm;
    float2 *buf = sm + M;
    const int comp = blockIdx.y;
    const float2 *src = spec + comp * spec_cstride;
    float2 *dst = (float2 *)(out + comp * out_cstride);
    const float2 *ad = add ? (const float2 *)(add + comp * out_cstride) : nullptr;
    const int row0 = blockIdx.x * R;
    load_tw(tw, tw3, M);
    __syncthreads();
    // Z[k] = (X[k] + conj X[M-k]) + i e^{+2 pi i k / n3} (X[k] - conj X[M-k]),  k < M
    for (int e = threadIdx.x; e < R * M; e += blockDim.x) {
        const int r = e >> logM, k = e & (M - 1);
        float2 Z = make_float2(0.f, 0.f);
        if (row0 + r < nrows) {
            const float2 *X = src + (size_t)(row0 + r) * nh;
            const float2 a = X[k], b = cconj(X[M - k]);
            const float2 sum = cadd(a, b), dif = csub(a, b);
            const float2 wd = cmul(cconj(tw[k]), dif);
            Z = make_float2(sum.x - wd.y, sum.y + wd.x);
        }
        buf[e] = Z;
    }
    __syncthreads();
    lds_fft<true>(buf, logM, logR, M, 1, tw, 2, true, false);
    for (int e = threadIdx.x; e < R * M; e += blockDim.x) {
        const int r = e >> logM, n = e & (M - 1);
        if (row0 + r >= nrows) continue;
        float2 z = buf[r * M + brev(n, logM)];
        const size_t o = (size_t)(row0 + r) * M + n;
        if (ad) {
            const float2 a = ad[o];
            z.x += a.x;
            z.y += a.y;
        }
        dst[o] = z;
    }
}

// --- x2 C2C in place on the half spectrum: plane i1 = blockIdx.y, columns
// [c0, c0 + C) of the nh per row.  Natural-order result.
__global__ __launch_bounds__(TPB) void k_fft_x2(float2 *__restrict__ spec, const float2 *__restrict__ tw2, int n2,
                                                int logn2, int nh, int logC, bool inv, size_t spec_cstride)
{
    extern __shared__ float2 sm[];
    const int C = 1 << logC, half = n2 >> 1;
    float2 *tw = sm;
    float2 *buf = sm + half;
    const int comp = blockIdx.z, i1 = blockIdx.y, c0 = blockIdx.x * C;
    const int cw = min(C, nh - c0);
    float2 *plane = spec + comp * spec_cstride + (size_t)i1 * n2 * nh;
    load_tw(tw, tw2, half);
    for (int e = threadIdx.x; e < n2 * C; e += blockDim.x) {
        const int q = e >> logC, l = e & (C - 1);
        buf[e] = l < cw ? plane[(size_t)q * nh + c0 + l] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    lds_fft<true>(buf, logn2, logC, 1, C, tw, 1, inv, true);
    for (int e = threadIdx.x; e < n2 * C; e += blockDim.x) {
        const int q = e >> logC, l = e & (C - 1);
        if (l < cw) plane[(size_t)q * nh + c0 + l] = buf[(brev(q, logn2) << logC) + l];
    }
}

// --- x1 fused: forward DIF along x1, symbol multiply, inverse DIT.
// plane i2 = blockIdx.y, columns [c0, c0 + C).
__global__ __launch_bounds__(TPB) void k_fft_x1_mult(float2 *__restrict__ spec, const float2 *__restrict__ tw1,
                                                     int n1, int logn1, int n2, int nh, int logC, int kind,
                                                     float beta, float scale, size_t spec_cstride)
{
    extern __shared__ float2 sm[];
    const int C = 1 << logC, half = n1 >> 1;
    float2 *tw = sm;
    float2 *buf = sm + half;
    const int comp = blockIdx.z, i2 = blockIdx.y, c0 = blockIdx.x * C;
    const int cw = min(C, nh - c0);
    float2 *base = spec + comp * spec_cstride + (size_t)i2 * nh;
    const size_t rs = (size_t)n2 * nh;
    load_tw(tw, tw1, half);
    for (int e = threadIdx.x; e < n1 * C; e += blockDim.x) {
        const int q = e >> logC, l = e & (C - 1);
        buf[e] = l < cw ? base[(size_t)q * rs + c0 + l] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    lds_fft<true>(buf, logn1, logC, 1, C, tw, 1, false, true);
    const float k2 = (float)(i2 < (n2 >> 1) ? i2 : i2 - n2);
    for (int e = threadIdx.x; e < n1 * C; e += blockDim.x) {
        const int r = e >> logC, l = e & (C - 1);
        const int q = brev(r, logn1);      // frequency index held at LDS row r
        const float k1 = (float)(q < half ? q : q - n1);
        const float k3 = (float)(c0 + l);
        const float ksq = k1 * k1 + k2 * k2 + k3 * k3;
        float sym;
        if (kind == 0) sym = beta * ksq;
        else if (kind == 1) sym = 1.0f / (beta * fmaxf(ksq, 1.0f));
        else sym = 1.0f;
        sym *= scale;
        buf[e].x *= sym;
        buf[e].y *= sym;
    }
    __syncthreads();
    lds_fft<false>(buf, logn1, logC, 1, C, tw, 1, true, true);
    for (int e = threadIdx.x; e < n1 * C; e += blockDim.x) {
        const int q = e >> logC, l = e & (C - 1);
        if (l < cw) base[(size_t)q * rs + c0 + l] = buf[e];
    }
}

int ilog2(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

} // namespace

size_t fft_spec_bytes(int n1, int n2, int n3, int ncomp)
{
    return (size_t)ncomp * n1 * n2 * (n3 / 2 + 1) * sizeof(float2);
}

void fft_make_twiddles(float2 *host, int n)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int t = 0; t < n / 2; ++t) {
        const double a = -two_pi * t / n;
        host[t] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
}

void spectral_apply(const FFTPlan &P, int kind, float beta, int ncomp, const float *in, float *out,
                    const float *add, hipStream_t s)
{
    const int n1 = P.n1, n2 = P.n2, n3 = P.n3, nh = P.nh;
    const int M = n3 / 2, logM = ilog2(M);
    const size_t N = (size_t)n1 * n2 * n3;
    const size_t spec_cs = (size_t)n1 * n2 * nh;
    const float scale = (float)(1.0 / (double)N);
    const int nrows = n1 * n2;
    int logR = ilog2(LDS_C) - logM;
    if (logR < 0) logR = 0;
    if ((1 << logR) > nrows) logR = ilog2(nrows);
    const int R = 1 << logR;
    for (int c0 = 0; c0 < ncomp; c0 += P.ncomp_max) {
        const int nc = ncomp - c0 < P.ncomp_max ? ncomp - c0 : P.ncomp_max;
        const float *inc = in + c0 * N;
        float *outc = out + c0 * N;
        const float *addc = add ? add + c0 * N : nullptr;
        const size_t lds3 = (size_t)(M + R * M) * sizeof(float2);
        hipLaunchKernelGGL(k_fft_x3_r2c, dim3(nrows / R, nc), dim3(TPB), lds3, s, inc, P.spec, P.tw3, n3, logM,
                           logR, nrows, N, spec_cs);
        // x2 forward
        int logC2 = ilog2(LDS_C) - ilog2(n2);
        if (logC2 > 5) logC2 = 5;
        const int C2 = 1 << logC2;
        const size_t lds2 = (size_t)(n2 / 2 + n2 * C2) * sizeof(float2);
        hipLaunchKernelGGL(k_fft_x2, dim3((nh + C2 - 1) / C2, n1, nc), dim3(TPB), lds2, s, P.spec, P.tw2, n2,
                           ilog2(n2), nh, logC2, false, spec_cs);
        // x1 forward, multiply, inverse
        int logC1 = ilog2(LDS_C) - ilog2(n1);
        if (logC1 > 5) logC1 = 5;
        const int C1 = 1 << logC1;
        const size_t lds1 = (size_t)(n1 / 2 + n1 * C1) * sizeof(float2);
        hipLaunchKernelGGL(k_fft_x1_mult, dim3((nh + C1 - 1) / C1, n2, nc), dim3(TPB), lds1, s, P.spec, P.tw1,
                           n1, ilog2(n1), n2, nh, logC1, kind, beta, scale, spec_cs);
        // x2 inverse
        hipLaunchKernelGGL(k_fft_x2, dim3((nh + C2 - 1) / C2, n1, nc), dim3(TPB), lds2, s, P.spec, P.tw2, n2,
                           ilog2(n2), nh, logC2, true, spec_cs);
        hipLaunchKernelGGL(k_fft_x3_c2r, dim3(nrows / R, nc), dim3(TPB), lds3, s, P.spec, outc, addc, P.tw3, n3,
                           logM, logR, nrows, N, spec_cs);
    }
}

} // namespace clh
