// k_fft.hip -- 3D real FFT spectral operators for gfx950 (Section 2.2: a
// spectral operator costs two FFTs and one Hadamard product; Section 3 uses
// a vendor 3D FFT on one GPU, here it is written from scratch).
//
// Layout: real fields [n1][n2][n3]; half spectrum [n1][n2][np]: nh = n3/2+1
// values per row at a row pitch np of nh rounded up to 16 (128-byte rows).
// One spectral apply is five passes, each a single read and a single write
// of the field:
//   x3 R2C    rows of n3 reals packed as M = n3/2 complex, complex FFT of
//             length M, split into the half spectrum of the real row;
//   x2 C2C    columns of a fixed-x1 plane;
//   x1 fused  columns along x1: forward FFT, Hadamard multiply by the
//             symbol, inverse FFT, all in one LDS tile;
//   x2 C2C    inverse;
//   x3 C2R    Hermitian merge, inverse FFT of length M, unpack to reals,
//             optional fused add.
// Lines of 128 ... 1024 points take register-resident passes (below); the
// generic passes for shorter lines work on LDS tiles: a workgroup owns a
// tile of nl lines x L points (nl L = 4096 complex, 32 KB), coalesced
// batched loads into LDS, then Stockham stages of radix 16 (and one of
// radix 2/4/8 for the remainder) with every group's R values in registers,
// twiddles from FP64-computed tables staged in LDS, and a coalesced store.  The LDS tile is stored as [q][l] with pitch nl + 1 so
// that both row-wise and column-wise accesses are conflict-free.
#include "internal.h"

#include <cmath>

namespace clh {

namespace {

constexpr int TPB = 256;
constexpr int TILE = 4096;   // complex values per LDS tile
constexpr int EPT = TILE / TPB;

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// cos / sin of 2 pi k / 16, k = 0..7 (folded at compile time)
__device__ __forceinline__ constexpr float c16(int k)
{
    return k == 0 ? 1.0f : k == 1 ? 0.92387953251128674f : k == 2 ? 0.70710678118654752f
         : k == 3 ? 0.38268343236508977f : k == 4 ? 0.0f : k == 5 ? -0.38268343236508977f
         : k == 6 ? -0.70710678118654752f : -0.92387953251128674f;
}
__device__ __forceinline__ constexpr float s16(int k)
{
    return k == 0 ? 0.0f : k == 1 ? 0.38268343236508977f : k == 2 ? 0.70710678118654752f
         : k == 3 ? 0.92387953251128674f : k == 4 ? 1.0f : k == 5 ? 0.92387953251128674f
         : k == 6 ? 0.70710678118654752f : 0.38268343236508977f;
}

template <int R> __device__ constexpr int brev_c(int i)
{
    int r = 0;
    for (int b = 1; b < R; b <<= 1) {
        r <<= 1;
        if (i & b) r |= 1;
    }
    return r;
}

// y * e^{-+2 pi i k / 16}; k is a compile-time constant after unrolling
template <bool INV> __device__ __forceinline__ float2 rot16(float2 y, int k)
{
    if (k == 0) return y;
    if (k == 4) return INV ? make_float2(-y.y, y.x) : make_float2(y.y, -y.x);
    const float c = c16(k), s = INV ? s16(k) : -s16(k);
    return make_float2(y.x * c - y.y * s, y.x * s + y.y * c);
}

// In-register DFT of length R (2, 4, 8, 16), natural order in and out:
// radix-2 DIT after a compile-time bit-reversal (register renaming only).
template <int R, bool INV> __device__ __forceinline__ void dft_reg(float2 *v)
{
    float2 a[R];
#pragma unroll
    for (int i = 0; i < R; ++i) a[i] = v[brev_c<R>(i)];
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
        for (int s = 0; s < R; s += len) {
#pragma unroll
            for (int k = 0; k < len / 2; ++k) {
                const float2 x = a[s + k];
                const float2 y = rot16<INV>(a[s + k + len / 2], k * (16 / len));
                a[s + k] = cadd(x, y);
                a[s + k + len / 2] = csub(x, y);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = a[i];
}

// One Stockham radix-R stage in place on the LDS tile (element (l, q) at
// q * P + l), for nl = 2^lognl lines of length L = 2^logL; Ns = 2^logNs is
// the product of the radices of the earlier stages.  tw[t] = e^{-2 pi i t / L}
// (t < L).  Every thread reads all its groups, the workgroup synchronises,
// then the results are written back, so the stage is safe in place.
template <int R, bool INV, int NT>
__device__ __forceinline__ void stage(float2 *lds, int P, int lognl, int logL, int logNs, const float2 *tw)
{
    constexpr int LOGR = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
    constexpr int G = EPT / R;          // groups per thread (the tile holds EPT values per thread)
    const int nl = 1 << lognl, L = 1 << logL, Ns = 1 << logNs;
    const int ngroups = nl << (logL - LOGR);
    const int LR = L >> LOGR;
    float2 v[G][R];
#pragma unroll
    for (int gq = 0; gq < G; ++gq) {
        const int gi = gq * NT + threadIdx.x;
        if (gi < ngroups) {
            const int l = gi & (nl - 1), j = gi >> lognl;
#pragma unroll
            for (int r = 0; r < R; ++r) v[gq][r] = lds[(j + r * LR) * P + l];
        }
    }
    __syncthreads();
#pragma unroll
    for (int gq = 0; gq < G; ++gq) {
        const int gi = gq * NT + threadIdx.x;
        if (gi < ngroups) {
            const int l = gi & (nl - 1), j = gi >> lognl;
            const int jm = j & (Ns - 1);
            if (logNs > 0) {
                const int tsh = logL - logNs - LOGR;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw[(r * jm) << tsh];
                    if (INV) w.y = -w.y;
                    v[gq][r] = cmul(v[gq][r], w);
                }
            }
            dft_reg<R, INV>(v[gq]);
            const int base = ((j >> logNs) << (logNs + LOGR)) + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[(base + r * Ns) * P + l] = v[gq][r];
        }
    }
    __syncthreads();
}

// Full FFT of the tile's lines: radix-16 stages, then one radix-2/4/8 stage.
// NT threads per workgroup, EPT values per thread.
template <bool INV, int NT = TPB> __device__ void fft_lines(float2 *lds, int P, int lognl, int logL, const float2 *tw)
{
    int logNs = 0;
    while (logL - logNs >= 4) {
        stage<16, INV, NT>(lds, P, lognl, logL, logNs, tw);
        logNs += 4;
    }
    const int rem = logL - logNs;
    if (rem == 3) stage<8, INV, NT>(lds, P, lognl, logL, logNs, tw);
    else if (rem == 2) stage<4, INV, NT>(lds, P, lognl, logL, logNs, tw);
    else if (rem == 1) stage<2, INV, NT>(lds, P, lognl, logL, logNs, tw);
}

template <int NT = TPB> __device__ __forceinline__ void load_table(float2 *dst, const float2 *__restrict__ src, int n)
{
    for (int t = threadIdx.x; t < n; t += NT) dst[t] = src[t];
}

// --- x3 forward: real rows -> half spectrum.  nl = 2^lognl rows per tile.
__global__ __launch_bounds__(TPB) void k_fft_x3_r2c(const float *__restrict__ in, float2 *__restrict__ spec,
                                                    const float2 *__restrict__ twM, const float2 *__restrict__ tw3,
                                                    int logM, int lognl, int nrows, size_t in_cs, size_t spec_cs,
                                                    int np)
{
    extern __shared__ float2 sm[];
    const int M = 1 << logM, nl = 1 << lognl, P = nl + 1, nh = M + 1;
    float2 *twm = sm;                 // M: e^{-2 pi i t / M}
    float2 *tws = sm + M;             // M + 1: e^{-2 pi i k / n3}, k <= M
    float2 *lds = tws + M + 1;        // M * P
    const int comp = blockIdx.y;
    const float2 *src = (const float2 *)(in + comp * in_cs);
    float2 *dst = spec + comp * spec_cs;
    const int row0 = blockIdx.x * nl;
    load_table(twm, twM, M);
    load_table(tws, tw3, M + 1);
    const int tot = nl << logM;
    float2 buf[EPT];
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
        const int e = it * TPB + threadIdx.x;
        if (e < tot) buf[it] = src[(size_t)row0 * M + e];
    }
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
        const int e = it * TPB + threadIdx.x;
        if (e < tot) lds[(e & (M - 1)) * P + (e >> logM)] = buf[it];
    }
    __syncthreads();
    fft_lines<false>(lds, P, lognl, logM, twm);
    // X[k] = E[k] + w^k O[k], E = (Z[k] + conj Z[M-k]) / 2, O = -i (Z[k] - conj Z[M-k]) / 2
    const int totk = nl * nh;
    for (int e = threadIdx.x; e < totk; e += TPB) {
        const int r = e / nh, k = e - r * nh;
        const float2 zk = lds[(k & (M - 1)) * P + r];
        const float2 zc = cconj(lds[((M - k) & (M - 1)) * P + r]);
        const float2 E = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
        const float2 O = make_float2(0.5f * (zk.y - zc.y), -0.5f * (zk.x - zc.x));
        dst[(size_t)(row0 + r) * np + k] = cadd(E, cmul(tws[k], O));
    }
}

// --- x3 inverse: half spectrum -> real rows (unnormalised), optional add.
__global__ __launch_bounds__(TPB) void k_fft_x3_c2r(const float2 *__restrict__ spec, float *__restrict__ out,
                                                    const float *__restrict__ add, const float2 *__restrict__ twM,
                                                    const float2 *__restrict__ tw3, int logM, int lognl, int nrows,
                                                    size_t out_cs, size_t spec_cs, int np)
{
    extern __shared__ float2 sm[];
    const int M = 1 << logM, nl = 1 << lognl, P = nl + 1, nh = M + 1;
    float2 *twm = sm;
    float2 *tws = sm + M;
    float2 *lds = tws + M + 1;
    const int comp = blockIdx.y;
    const float2 *src = spec + comp * spec_cs;
    float2 *dst = (float2 *)(out + comp * out_cs);
    const float2 *ad = add ? (const float2 *)(add + comp * out_cs) : nullptr;
    const int row0 = blockIdx.x * nl;
    load_table(twm, twM, M);
    load_table(tws, tw3, M + 1);
    // stage the half-spectrum rows (nh values each) at lds[k * P + r], k <= M
    // (row M of the tile doubles as the Nyquist slot; the tile has M + 1 rows).
    // nl * nh = TILE + nl <= TILE + TILE / 8 values (M >= 8), i.e. at most
    // EPT + 2 per thread.
    const int totk = nl * nh;
    {
        constexpr int NB = EPT + EPT / 8;
        float2 buf[NB];
#pragma unroll
        for (int it = 0; it < NB; ++it) {
            const int e = it * TPB + threadIdx.x;
            if (e < totk) {
                const int r = e / nh, k = e - r * nh;
                buf[it] = src[(size_t)(row0 + r) * np + k];
            }
        }
#pragma unroll
        for (int it = 0; it < NB; ++it) {
            const int e = it * TPB + threadIdx.x;
            if (e < totk) {
                const int r = e / nh, k = e - r * nh;
                lds[k * P + r] = buf[it];
            }
        }
    }
    __syncthreads();
    // Z[k] = (X[k] + conj X[M-k]) + i e^{+2 pi i k / n3} (X[k] - conj X[M-k]),  k < M
    float2 z[EPT];
    const int tot = nl << logM;
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
        const int e = it * TPB + threadIdx.x;
        if (e < tot) {
            const int r = e & (nl - 1), k = e >> lognl;
            const float2 a = lds[k * P + r], b = cconj(lds[(M - k) * P + r]);
            const float2 sum = cadd(a, b), dif = csub(a, b);
            const float2 wd = cmul(cconj(tws[k]), dif);
            z[it] = make_float2(sum.x - wd.y, sum.y + wd.x);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
        const int e = it * TPB + threadIdx.x;
        if (e < tot) lds[(e >> lognl) * P + (e & (nl - 1))] = z[it];
    }
    __syncthreads();
    fft_lines<true>(lds, P, lognl, logM, twm);
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
        const int e = it * TPB + threadIdx.x;
        if (e < tot) {
            const int r = e >> logM, n = e & (M - 1);
            float2 v = lds[n * P + r];
            const size_t o = (size_t)row0 * M + e;
            if (ad) {
                const float2 a = ad[o];
                v.x += a.x;
                v.y += a.y;
            }
            dst[o] = v;
        }
    }
}

// --- column tile load/store for the x2 and x1 passes: element (l, q) of
// the tile is base[q * rs + l], l < cw valid columns; NT threads.  A thread
// keeps its column l and steps through the rows q0, q0 + NT / C, ...: the
// row part of an address is wave-uniform (a scalar base), the thread's part a
// 32-bit byte offset (below 1/16 of one component's half spectrum).
template <int NT>
__device__ __forceinline__ void load_cols(float2 *lds, const float2 *__restrict__ base, size_t rs, int logC, int logL,
                                          int cw, int P)
{
    const int C = 1 << logC, L = 1 << logL;
    const int l = threadIdx.x & (C - 1), q0 = threadIdx.x >> logC, QS = NT >> logC;
    const unsigned off = (unsigned)(((size_t)q0 * rs + l) * sizeof(float2));
    float2 buf[EPT];
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
        const char *row = (const char *)(base + (size_t)it * QS * rs);
        if (q0 + it * QS < L) buf[it] = l < cw ? *(const float2 *)(row + off) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int it = 0; it < EPT; ++it)
        if (q0 + it * QS < L) lds[(q0 + it * QS) * P + l] = buf[it];
    __syncthreads();
}

template <int NT>
__device__ __forceinline__ void store_cols(const float2 *lds, float2 *__restrict__ base, size_t rs, int logC, int logL,
                                           int cw, int P)
{
    const int C = 1 << logC, L = 1 << logL;
    const int l = threadIdx.x & (C - 1), q0 = threadIdx.x >> logC, QS = NT >> logC;
    const unsigned off = (unsigned)(((size_t)q0 * rs + l) * sizeof(float2));
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
        char *row = (char *)(base + (size_t)it * QS * rs);
        if (q0 + it * QS < L && l < cw) *(float2 *)(row + off) = lds[(q0 + it * QS) * P + l];
    }
}

// --- x2 C2C in place on the half spectrum: plane i1 = blockIdx.y, columns
// [c0, c0 + C) of the nh per row; NT threads hold the tile of NT EPT values.
template <bool INV, int NT>
__global__ __launch_bounds__(NT) void k_fft_x2(float2 *__restrict__ spec, const float2 *__restrict__ tw2, int logn2,
                                                int n2, int nh, int np, int logC, size_t spec_cs)
{
    extern __shared__ float2 sm[];
    const int C = 1 << logC, P = C + 1;
    float2 *tw = sm;
    float2 *lds = sm + n2;
    const int comp = blockIdx.z, i1 = blockIdx.y, c0 = blockIdx.x * C;
    const int cw = min(C, nh - c0);
    float2 *base = spec + comp * spec_cs + (size_t)i1 * n2 * np + c0;
    load_table<NT>(tw, tw2, n2);
    load_cols<NT>(lds, base, np, logC, logn2, cw, P);
    fft_lines<INV, NT>(lds, P, logC, logn2, tw);
    store_cols<NT>(lds, base, np, logC, logn2, cw, P);
}

// --- x1 fused: forward FFT along x1, symbol multiply, inverse FFT.
// plane i2 = blockIdx.y, columns [c0, c0 + C).
// mode 0: forward, multiply, inverse; 1: forward only; 2: inverse only
template <int NT>
__global__ __launch_bounds__(NT) void k_fft_x1_mult(float2 *__restrict__ spec, const float2 *__restrict__ tw1,
                                                     int logn1, int n1, int n2, int nh, int np, int logC, int kind,
                                                     float beta, float scale, size_t spec_cs, int mode)
{
    extern __shared__ float2 sm[];
    const int C = 1 << logC, P = C + 1;
    float2 *tw = sm;
    float2 *lds = sm + n1;
    const int comp = blockIdx.z, i2 = blockIdx.y, c0 = blockIdx.x * C;
    const int cw = min(C, nh - c0);
    float2 *base = spec + comp * spec_cs + (size_t)i2 * np + c0;
    const size_t rs = (size_t)n2 * np;
    load_table<NT>(tw, tw1, n1);
    load_cols<NT>(lds, base, rs, logC, logn1, cw, P);
    if (mode == 2) {
        fft_lines<true, NT>(lds, P, logC, logn1, tw);
        store_cols<NT>(lds, base, rs, logC, logn1, cw, P);
        return;
    }
    fft_lines<false, NT>(lds, P, logC, logn1, tw);
    if (mode == 1) {
        store_cols<NT>(lds, base, rs, logC, logn1, cw, P);
        return;
    }
    const float k2 = (float)(i2 < (n2 >> 1) ? i2 : i2 - n2);
    const int tot = C << logn1;
    for (int e = threadIdx.x; e < tot; e += NT) {
        const int l = e & (C - 1), q = e >> logC;
        const float k1 = (float)(q < (n1 >> 1) ? q : q - n1);
        const float k3 = (float)(c0 + l);
        const float ksq = k1 * k1 + k2 * k2 + k3 * k3;
        float sym;
        if (kind == 0) sym = beta * ksq;
        else if (kind == 1) sym = 1.0f / (beta * fmaxf(ksq, 1.0f));
        else sym = 1.0f;
        sym *= scale;
        float2 &x = lds[q * P + l];
        x.x *= sym;
        x.y *= sym;
    }
    __syncthreads();
    fft_lines<true, NT>(lds, P, logC, logn1, tw);
    store_cols<NT>(lds, base, rs, logC, logn1, cw, P);
}

// --- register-resident column passes for lines of L = 16 R2 points (R2 =
// 8 or 16, i.e. L = 128 or 256; 512 and 1024 below) in tiles of C = 256 / R2
// columns.  With
// n = R2 a + b and k = c + 16 d,
//   X[c + 16 d] = sum_b W_R2^{bd} W_L^{bc} sum_a x[R2 a + b] W_16^{ac},
// so each thread holds 16 (or 2 x R2) values in registers: the length-16
// DFTs over a run on the "b" layout (thread = column l, residue b), the
// length-R2 DFTs over b on the "c" layout (thread = column l, c), and one
// LDS exchange [c][b][l] (pitch 272 complex per c: row reads and writes of a
// half-wavefront hit distinct banks) connects them.  The inverse runs the
// same steps backwards.  A tile therefore crosses LDS twice per transform
// (Stockham stages in LDS cross it four times plus the staging).
// MODE 0: forward, symbol multiply (x1 pass), inverse; 1: forward only;
// 2: inverse only.  Element (row q, column l) of the tile is base[q rs + l].
constexpr int CSC = 272;   // LDS pitch per c (R2 C + 16 complex)

template <int R2>
__device__ __forceinline__ void cols_load_b(float2 (&v)[16], const float2 *__restrict__ base, size_t rs, int l, int b,
                                            bool ok)
{
#pragma unroll
    for (int a = 0; a < 16; ++a) v[a] = ok ? base[(size_t)(R2 * a + b) * rs + l] : make_float2(0.f, 0.f);
}

template <int R2, int MODE>
__global__ __launch_bounds__(TPB) void k_fft_cols(float2 *__restrict__ spec, const float2 *__restrict__ twL,
                                                  int nh, size_t plane_stride, size_t rs, size_t spec_cs, int kind,
                                                  float beta, float scale, int n1, int n2)
{
    constexpr int L = 16 * R2, C = 256 / R2, P2 = C / 16;   // P2: (l, c) pairs per thread
    __shared__ float2 tw[L];
    __shared__ float2 ex[16 * CSC];
    const int comp = blockIdx.z, pl = blockIdx.y, c0 = blockIdx.x * C;
    const int cw = min(C, nh - c0);
    float2 *base = spec + comp * spec_cs + pl * plane_stride + c0;
    for (int t = threadIdx.x; t < L; t += TPB) tw[t] = twL[t];
    const int l = threadIdx.x % C, r = threadIdx.x / C;     // r: b (b layout) or the first c (c layout)
    const bool ok = l < cw;
    float2 v[16];
    if (MODE != 2) {
        // forward: b layout, DFT-16 over a, twiddle W_L^{bc}, exchange
        cols_load_b<R2>(v, base, rs, l, r, ok);
        __syncthreads();                                      // twiddle table
        dft_reg<16, false>(v);
#pragma unroll
        for (int c = 1; c < 16; ++c) v[c] = cmul(v[c], tw[r * c]);
#pragma unroll
        for (int c = 0; c < 16; ++c) ex[c * CSC + r * C + l] = v[c];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < P2; ++u) {
            const int c = r + (256 / C) * u;
            float2 w[R2];
#pragma unroll
            for (int b = 0; b < R2; ++b) w[b] = ex[c * CSC + b * C + l];
            dft_reg<R2, false>(w);                            // w[d] = X[c + 16 d]
#pragma unroll
            for (int d = 0; d < R2; ++d) v[u * R2 + d] = w[d];
        }
        if (MODE == 1) {
#pragma unroll
            for (int u = 0; u < P2; ++u) {
                const int c = r + (256 / C) * u;
#pragma unroll
                for (int d = 0; d < R2; ++d)
                    if (ok) base[(size_t)(c + 16 * d) * rs + l] = v[u * R2 + d];
            }
            return;
        }
        // symbol of the x1 pass: k1 = c + 16 d, k2 = plane, k3 = c0 + l
        const float k2 = (float)(pl < (n2 >> 1) ? pl : pl - n2);
        const float k3 = (float)(c0 + l);
#pragma unroll
        for (int u = 0; u < P2; ++u) {
            const int c = r + (256 / C) * u;
#pragma unroll
            for (int d = 0; d < R2; ++d) {
                const int q = c + 16 * d;
                const float k1 = (float)(q < (n1 >> 1) ? q : q - n1);
                const float ksq = k1 * k1 + k2 * k2 + k3 * k3;
                float sym;
                if (kind == 0) sym = beta * ksq;
                else if (kind == 1) sym = 1.0f / (beta * fmaxf(ksq, 1.0f));
                else sym = 1.0f;
                sym *= scale;
                v[u * R2 + d].x *= sym;
                v[u * R2 + d].y *= sym;
            }
        }
        __syncthreads();                                      // exchange buffer free again
    } else {
        // inverse only: c layout loads X[c + 16 d]
#pragma unroll
        for (int u = 0; u < P2; ++u) {
            const int c = r + (256 / C) * u;
#pragma unroll
            for (int d = 0; d < R2; ++d)
                v[u * R2 + d] = ok ? base[(size_t)(c + 16 * d) * rs + l] : make_float2(0.f, 0.f);
        }
        __syncthreads();                                      // twiddle table
    }
    // inverse: c layout, DFT-R2 over d, twiddle W_L^{-bc}, exchange, DFT-16 over c
#pragma unroll
    for (int u = 0; u < P2; ++u) {
        const int c = r + (256 / C) * u;
        float2 w[R2];
#pragma unroll
        for (int d = 0; d < R2; ++d) w[d] = v[u * R2 + d];
        dft_reg<R2, true>(w);                                 // w[b] = sum_d X[c + 16 d] W_R2^{-bd}
#pragma unroll
        for (int b = 0; b < R2; ++b) ex[c * CSC + b * C + l] = b ? cmul(w[b], cconj(tw[b * c])) : w[b];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = ex[c * CSC + r * C + l];
    dft_reg<16, true>(v);                                     // v[a] = x[r + R2 a]
    if (ok) {
#pragma unroll
        for (int a = 0; a < 16; ++a) base[(size_t)(R2 * a + r) * rs + l] = v[a];
    }
}

// --- register-resident column passes for lines of L = 256 E points (E = 2
// or 4: 512 or 1024 points) in tiles of C = 32 / E columns, 512 threads.
// The split n = R2 a + b, k = c + 16 d (R2 = 16 E) of k_fft_cols leaves a
// length-R2 DFT over b for every (column, c); it is split again as
// b = E beta + eps, d = d' + 16 m:
//   X[c + 16 d' + 256 m] = sum_eps W_E^{eps m} W_R2^{eps d'} Z_eps[d'],
//   Z_eps[d'] = sum_beta y_c[E beta + eps] W_16^{beta d'},
// so a thread holds 16 values in both layouts: the E lanes eps of a
// (column, c) pair are neighbours, each runs one length-16 DFT, and the
// length-E DFT over eps runs across them (radix-2 lane exchanges; with E = 4
// lane eps ends with m = the bit reverse of eps).  The inverse applies the
// same steps backwards with conjugate twiddles.  Tiles of 16 (512 points) or
// 8 columns (1024 points) keep row pieces of 128 or 64 bytes and 66 KB of
// exchange buffer, so that two workgroups fit a CU.
constexpr int NTX = 512;

// length-E DFT over the lanes eps S, in place on 16 values (eps = (lane / S)
// mod E: the partners of a lane are lane ^ S and lane ^ 2S)
template <int E, bool INV, int S = 1> __device__ __forceinline__ void cross_dft(float2 (&v)[16], int eps)
{
    auto bfly = [&](int bit) {        // lane bit 0: own + partner; bit 1: partner - own
        const bool hi = (eps & bit) != 0;
        const int mask = bit * S;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float px = __shfl_xor(v[i].x, mask), py = __shfl_xor(v[i].y, mask);
            v[i] = hi ? make_float2(px - v[i].x, py - v[i].y) : make_float2(v[i].x + px, v[i].y + py);
        }
    };
    if (E == 2) {
        bfly(1);
        return;
    }
    bfly(INV ? 1 : 2);
    if (eps == 3) {                   // W_4^{+-1}
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = INV ? make_float2(-v[i].y, v[i].x) : make_float2(v[i].y, -v[i].x);
    }
    bfly(INV ? 2 : 1);
}

template <int E, int MODE>
__global__ __launch_bounds__(NTX, 4) void k_fft_colsx(float2 *__restrict__ spec, const float2 *__restrict__ twL,
                                                      int nh, size_t plane_stride, size_t rs, size_t spec_cs, int kind,
                                                      float beta, float scale, int n1, int n2)
{
    constexpr int R2 = 16 * E, L = 16 * R2, C = NTX / R2, LOGC = C == 16 ? 4 : 3, LOGE = E == 2 ? 1 : 2;
    constexpr int CS = R2 * C + 16;   // exchange pitch per c
    __shared__ float2 tw[L];
    __shared__ float2 ex[16 * CS];
    const int comp = blockIdx.z, pl = blockIdx.y, c0 = blockIdx.x * C;
    const int cw = min(C, nh - c0);
    float2 *base = spec + comp * spec_cs + pl * plane_stride + c0;
    for (int t = threadIdx.x; t < L; t += NTX) tw[t] = twL[t];
    // b layout: thread (column lb, b); c layout: thread (eps, column lc, c), eps fastest
    const int lb = threadIdx.x & (C - 1), b = threadIdx.x >> LOGC;
    const int eps = threadIdx.x & (E - 1), lc = (threadIdx.x >> LOGE) & (C - 1), c = threadIdx.x >> (LOGE + LOGC);
    const int m = E == 4 ? ((eps & 1) << 1 | eps >> 1) : eps;
    const bool okb = lb < cw, okc = lc < cw;
    float2 v[16];
    if (MODE != 2) {
        cols_load_b<R2>(v, base, rs, lb, b, okb);            // v[a] = x[R2 a + b]
        __syncthreads();                                      // twiddle table
        dft_reg<16, false>(v);
#pragma unroll
        for (int k = 1; k < 16; ++k) v[k] = cmul(v[k], tw[b * k]);
#pragma unroll
        for (int k = 0; k < 16; ++k) ex[k * CS + b * C + lb] = v[k];
        __syncthreads();
#pragma unroll
        for (int bt = 0; bt < 16; ++bt) v[bt] = ex[c * CS + (E * bt + eps) * C + lc];
        dft_reg<16, false>(v);                                // Z_eps[d']
#pragma unroll
        for (int k = 1; k < 16; ++k)
            if (eps) v[k] = cmul(v[k], tw[16 * eps * k]);
        cross_dft<E, false>(v, eps);                          // v[d'] = X[c + 16 d' + 256 m]
        if (MODE == 1) {
            if (okc) {
#pragma unroll
                for (int k = 0; k < 16; ++k) base[(size_t)(c + 16 * k + 256 * m) * rs + lc] = v[k];
            }
            return;
        }
        // symbol of the x1 pass: k1 = c + 16 d' + 256 m, k2 = plane, k3 = c0 + lc
        const float k2 = (float)(pl < (n2 >> 1) ? pl : pl - n2);
        const float k3 = (float)(c0 + lc);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int q = c + 16 * k + 256 * m;
            const float k1 = (float)(q < (n1 >> 1) ? q : q - n1);
            const float ksq = k1 * k1 + k2 * k2 + k3 * k3;
            float sym;
            if (kind == 0) sym = beta * ksq;
            else if (kind == 1) sym = 1.0f / (beta * fmaxf(ksq, 1.0f));
            else sym = 1.0f;
            sym *= scale;
            v[k].x *= sym;
            v[k].y *= sym;
        }
        __syncthreads();                                      // exchange buffer free again
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k)
            v[k] = okc ? base[(size_t)(c + 16 * k + 256 * m) * rs + lc] : make_float2(0.f, 0.f);
        __syncthreads();                                      // twiddle table
    }
    // inverse: lanes, twiddle W_R2^{-eps d'}, DFT-16 over d', exchange,
    // twiddle W_L^{-b c}, DFT-16 over c
    cross_dft<E, true>(v, eps);
#pragma unroll
    for (int k = 1; k < 16; ++k)
        if (eps) v[k] = cmul(v[k], cconj(tw[16 * eps * k]));
    dft_reg<16, true>(v);                                     // v[beta] = y_c[E beta + eps]
#pragma unroll
    for (int bt = 0; bt < 16; ++bt) ex[c * CS + (E * bt + eps) * C + lc] = v[bt];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = ex[k * CS + b * C + lb];
#pragma unroll
    for (int k = 1; k < 16; ++k) v[k] = cmul(v[k], cconj(tw[b * k]));
    dft_reg<16, true>(v);                                     // v[a] = x[R2 a + b]
    if (okb) {
#pragma unroll
        for (int a = 0; a < 16; ++a) base[(size_t)(R2 * a + b) * rs + lb] = v[a];
    }
}

// --- register-resident x3 passes for rows of M = 16 R2 complex values (M =
// 64 ... 512, i.e. n3 = 128 ... 1024), NR = 256 / R2 rows per tile.  With
// input index n = c + 16 d and output index k = b + R2 a (M = 16 R2),
//   X[b + R2 a] = sum_c W_16^{ac} W_M^{bc} sum_d x[c + 16 d] W_R2^{bd}
// (conjugate twiddles for the inverse): the length-R2 DFTs over d run on the
// "c" layout (thread = row, c; 16 / R2 pairs per thread; R2 = 32 below),
// the length-16 DFTs over c on the "b" layout (thread = row, b), joined by one LDS exchange
// [row][c][b] (row pitch 17 R2 + 16 complex).  Loads on the c layout read
// 16 consecutive complex values per row per instruction.
// Rows of M = 512 complex values (n3 = 1024, R2 = 32, NR = 8 rows per tile)
// split the length-32 DFTs over d once more, d = 2 delta + eps, b = b' + 16 m:
//   Y_c[b' + 16 m] = sum_eps (-1)^{eps m} W_32^{eps b'}
//                    sum_delta x[c + 16 (2 delta + eps)] W_16^{delta b'},
// so the c layout holds (row, c, eps) with eps = bit 4 of the lane, every
// thread runs one length-16 DFT, and the length-2 DFT over eps is a lane
// exchange (lane ^ 16).
template <int R2> constexpr int rows_pitch() { return 17 * R2 + 16; }

// Lane i of each 16-lane row receives x of lane 16 - i of the same row
// (DPP row mirror, i -> 15 - i, then a shift by one lane); lane 0 receives 0.
__device__ __forceinline__ float row_reflect16(float x)
{
    const int m = __builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xf, 0xf, false);   // row_mirror
    return __int_as_float(__builtin_amdgcn_update_dpp(0, m, 0x111, 0xf, 0xf, false));         // row_shr:1
}

template <int R2, bool INV>
__device__ __forceinline__ void rows_cb(float2 (&v)[16], float2 *ex, const float2 *tw)
{
    constexpr int PP = 16 / R2, RS = rows_pitch<R2>();
    const int c = threadIdx.x & 15, r0 = threadIdx.x >> 4;
#pragma unroll
    for (int u = 0; u < PP; ++u) {
        const int row = r0 + 16 * u;
        float2 w[R2];
#pragma unroll
        for (int d = 0; d < R2; ++d) w[d] = v[u * R2 + d];
        dft_reg<R2, INV>(w);
#pragma unroll
        for (int b = 0; b < R2; ++b) {
            float2 t = w[b];
            if (b) t = cmul(t, INV ? cconj(tw[b * c]) : tw[b * c]);
            ex[row * RS + c * (R2 + 1) + b] = t;
        }
    }
    __syncthreads();
    const int b = threadIdx.x % R2, row = threadIdx.x / R2;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) v[cc] = ex[row * RS + cc * (R2 + 1) + b];
    dft_reg<16, INV>(v);                                      // v[a] = X[b + R2 a]
}

// rows_cb for R2 = 32: v[delta] = x[c + 16 (2 delta + eps)] on the c layout
// (c = lane bits 0-3, eps = bit 4, row = thread / 32) in, v[a] = X[b + 32 a]
// on the b layout out
template <bool INV> __device__ __forceinline__ void rows_cbx(float2 (&v)[16], float2 *ex, const float2 *tw)
{
    constexpr int R2 = 32, RS = rows_pitch<32>();
    const int c = threadIdx.x & 15, eps = (threadIdx.x >> 4) & 1, row = threadIdx.x >> 5;
    dft_reg<16, INV>(v);                                      // v[b'] = sum_delta ... W_16^{delta b'}
    if (eps) {
#pragma unroll
        for (int k = 1; k < 16; ++k) v[k] = cmul(v[k], INV ? cconj(tw[16 * k]) : tw[16 * k]);   // W_32^{b'}
    }
    cross_dft<2, INV, 16>(v, eps);                            // v[b'] = Y_c[b' + 16 eps]
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int b = k + 16 * eps;
        float2 t = v[k];
        if (b * c) t = cmul(t, INV ? cconj(tw[b * c]) : tw[b * c]);
        ex[row * RS + c * (R2 + 1) + b] = t;
    }
    __syncthreads();
    const int bb = threadIdx.x % R2, rb = threadIdx.x / R2;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) v[cc] = ex[rb * RS + cc * (R2 + 1) + bb];
    dft_reg<16, INV>(v);                                      // v[a] = X[b + R2 a]
}

// x3 forward: real rows -> half spectrum
template <int R2>
__global__ __launch_bounds__(TPB) void k_fft_rows_r2c(const float *__restrict__ in, float2 *__restrict__ spec,
                                                      const float2 *__restrict__ twM, const float2 *__restrict__ tw3,
                                                      size_t in_cs, size_t spec_cs)
{
    constexpr int M = 16 * R2, NR = 256 / R2, PP = 16 / R2, NP = M + 16;   // NP: spectrum row pitch
    __shared__ float2 twm[M], tws[M + 1];
    __shared__ float2 ex[NR * rows_pitch<R2>()];
    const int comp = blockIdx.y;
    const size_t row0 = (size_t)blockIdx.x * NR;
    const float2 *src = (const float2 *)(in + comp * in_cs) + row0 * M;
    float2 *dst = spec + comp * spec_cs + row0 * NP;
    for (int t = threadIdx.x; t < M; t += TPB) twm[t] = twM[t];
    for (int t = threadIdx.x; t <= M; t += TPB) tws[t] = tw3[t];
    const int c = threadIdx.x & 15, r0 = threadIdx.x >> 4;
    float2 v[16];
    if constexpr (R2 == 32) {
        const int eps = r0 & 1, rw = r0 >> 1;
#pragma unroll
        for (int dl = 0; dl < 16; ++dl) v[dl] = src[(size_t)rw * M + c + 16 * eps + 32 * dl];
        __syncthreads();                                      // twiddle tables
        rows_cbx<false>(v, ex, twm);
    } else {
#pragma unroll
        for (int u = 0; u < PP; ++u)
#pragma unroll
            for (int d = 0; d < R2; ++d) v[u * R2 + d] = src[(size_t)(r0 + 16 * u) * M + c + 16 * d];
        __syncthreads();                                      // twiddle tables
        rows_cb<R2, false>(v, ex, twm);
    }
    // X[k] = E + W_n3^k O with E = (Z[k] + conj Z[M-k]) / 2, O = -i (Z[k] -
    // conj Z[M-k]) / 2; Z[M-k] of k = b + R2 a is v[15 - a] of the lane with
    // b' = R2 - b (b > 0) or this lane's v[(16 - a) mod 16] (b = 0)
    const int b = threadIdx.x % R2, row = threadIdx.x / R2;
    const int lane = threadIdx.x & 63, partner = lane - b + ((R2 - b) & (R2 - 1));
    float2 *drow = dst + (size_t)row * NP;
#pragma unroll
    for (int a = 0; a < 16; ++a) {
        float2 zc;
        zc.x = __shfl(v[15 - a].x, partner, 64);
        zc.y = __shfl(v[15 - a].y, partner, 64);
        if (b == 0) zc = v[(16 - a) & 15];
        zc = cconj(zc);
        const float2 zk = v[a];
        const int k = b + R2 * a;
        const float2 E = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
        const float2 O = make_float2(0.5f * (zk.y - zc.y), -0.5f * (zk.x - zc.x));
        drow[k] = cadd(E, cmul(tws[k], O));
    }
    if (b == 0) {
        // k = M: Z[M mod M] = Z[0]
        const float2 zk = v[0], zc = cconj(v[0]);
        const float2 E = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
        const float2 O = make_float2(0.5f * (zk.y - zc.y), -0.5f * (zk.x - zc.x));
        drow[M] = cadd(E, cmul(tws[M], O));
    }
}

// x3 inverse: half spectrum -> real rows (unnormalised), optional add
template <int R2>
__global__ __launch_bounds__(TPB) void k_fft_rows_c2r(const float2 *__restrict__ spec, float *__restrict__ out,
                                                      const float *__restrict__ add, const float2 *__restrict__ twM,
                                                      const float2 *__restrict__ tw3, size_t out_cs, size_t spec_cs)
{
    constexpr int M = 16 * R2, NR = 256 / R2, PP = 16 / R2, NP = M + 16;   // NP: spectrum row pitch
    __shared__ float2 twm[M], tws[M + 1];
    __shared__ float2 ex[NR * rows_pitch<R2>()];
    const int comp = blockIdx.y;
    const size_t row0 = (size_t)blockIdx.x * NR;
    const float2 *src = spec + comp * spec_cs + row0 * NP;
    float2 *dst = (float2 *)(out + comp * out_cs) + row0 * M;
    const float2 *ad = add ? (const float2 *)(add + comp * out_cs) + row0 * M : nullptr;
    for (int t = threadIdx.x; t < M; t += TPB) twm[t] = twM[t];
    for (int t = threadIdx.x; t <= M; t += TPB) tws[t] = tw3[t];
    const int c = threadIdx.x & 15, r0 = threadIdx.x >> 4;
    float2 v[16];
    if constexpr (R2 == 32) {
        // X[k] and X[M - k] for k = c + 16 (2 delta + eps), both read from
        // the row (k = 0 pairs with the Nyquist value X[M])
        const int eps = r0 & 1, rw = r0 >> 1;
        const float2 *srow = src + (size_t)rw * NP;
        float2 xa[16], xb[16];
#pragma unroll
        for (int dl = 0; dl < 16; ++dl) {
            const int k = c + 16 * eps + 32 * dl;
            xa[dl] = srow[k];
            xb[dl] = srow[M - k];
        }
        __syncthreads();                                      // twiddle tables
#pragma unroll
        for (int dl = 0; dl < 16; ++dl) {
            const int k = c + 16 * eps + 32 * dl;
            const float2 a = xa[dl], bb = cconj(xb[dl]);
            const float2 sum = cadd(a, bb), dif = csub(a, bb);
            const float2 wd = cmul(cconj(tws[k]), dif);
            v[dl] = make_float2(sum.x - wd.y, sum.y + wd.x);
        }
        rows_cbx<true>(v, ex, twm);
    } else {
        float2 xa[16], xb[16], nyq[PP];
#pragma unroll
        for (int u = 0; u < PP; ++u) {
            const float2 *srow = src + (size_t)(r0 + 16 * u) * NP;
#pragma unroll
            for (int d = 0; d < R2; ++d) xa[u * R2 + d] = srow[c + 16 * d];
            nyq[u] = c == 0 ? srow[M] : make_float2(0.f, 0.f);
        }
        // X[M - k] for k = c + 16 d: for c > 0 it is X[(16 - c) + 16 (R2 - 1 - d)],
        // held by lane 16 - c of the same 16-lane row (a row reflection by DPP);
        // for c = 0 it is this lane's X[16 (R2 - d)], or the Nyquist value at d = 0
#pragma unroll
        for (int u = 0; u < PP; ++u)
#pragma unroll
            for (int d = 0; d < R2; ++d) {
                const float2 o = xa[u * R2 + R2 - 1 - d];
                const float2 m = make_float2(row_reflect16(o.x), row_reflect16(o.y));
                xb[u * R2 + d] = c ? m : (d ? xa[u * R2 + R2 - d] : nyq[u]);
            }
        __syncthreads();                                      // twiddle tables
        // Z[k] = (X[k] + conj X[M-k]) + i e^{+2 pi i k / n3} (X[k] - conj X[M-k])
#pragma unroll
        for (int u = 0; u < PP; ++u)
#pragma unroll
            for (int d = 0; d < R2; ++d) {
                const int k = c + 16 * d;
                const float2 a = xa[u * R2 + d], bb = cconj(xb[u * R2 + d]);
                const float2 sum = cadd(a, bb), dif = csub(a, bb);
                const float2 wd = cmul(cconj(tws[k]), dif);
                v[u * R2 + d] = make_float2(sum.x - wd.y, sum.y + wd.x);
            }
        rows_cb<R2, true>(v, ex, twm);
    }
    const int b = threadIdx.x % R2, row = threadIdx.x / R2;
#pragma unroll
    for (int a = 0; a < 16; ++a) {
        const size_t o = (size_t)row * M + b + R2 * a;
        float2 val = v[a];
        if (ad) {
            const float2 t = ad[o];
            val.x += t.x;
            val.y += t.y;
        }
        dst[o] = val;
    }
}

// Copy the half-spectrum modes with |k_d| < min(na_d, nb_d)/2 from grid a
// to grid b (the coarse Nyquist planes are dropped), zero elsewhere.
__global__ __launch_bounds__(TPB) void k_mode_copy(const float2 *__restrict__ sa, float2 *__restrict__ sb, int a1, int a2,
                                                   int a3, int b1, int b2, int b3, int ncomp)
{
    const int bh = b3 / 2 + 1, ap = fft_row_pitch(a3), bp = fft_row_pitch(b3);
    const size_t nb = (size_t)b1 * b2 * bh;
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e >= nb * ncomp) return;
    const int comp = (int)(e / nb);
    const size_t r = e - comp * nb;
    const int q3 = (int)(r % bh), q2 = (int)((r / bh) % b2), q1 = (int)(r / ((size_t)bh * b2));
    const int k1 = q1 < b1 / 2 ? q1 : q1 - b1, k2 = q2 < b2 / 2 ? q2 : q2 - b2, k3 = q3;
    const int c1 = min(a1, b1), c2 = min(a2, b2), c3 = min(a3, b3);
    float2 v = make_float2(0.f, 0.f);
    if (2 * abs(k1) < c1 && 2 * abs(k2) < c2 && 2 * k3 < c3) {
        const int p1 = k1 < 0 ? k1 + a1 : k1, p2 = k2 < 0 ? k2 + a2 : k2;
        v = sa[(size_t)comp * a1 * a2 * ap + ((size_t)p1 * a2 + p2) * ap + k3];
    }
    sb[(size_t)comp * b1 * b2 * bp + ((size_t)q1 * b2 + q2) * bp + q3] = v;
}

// Per-mode 3x3 operators of the near-incompressible regularisation on the
// half spectrum of a vector field (three components spec_cs apart), scaled
// by 1/N.  With a = beta_v |k|^2, c = beta_w (1 + |k|^2) and kappa the
// derivative wavenumber (k_d, 0 at the Nyquist index):
//   kind 0: L = a I + c kappa kappa^T (Hessian of the regularisation)
//   kind 1: L^-1 = (I - c/(a + c |kappa|^2) kappa kappa^T) / a, 1/beta_v at k = 0
//   kind 3: K = beta_v A L^-1 = I - c/(a + c |kappa|^2) kappa kappa^T, I at k = 0
// (Sherman-Morrison on the rank-one term).
__global__ __launch_bounds__(TPB) void k_spec_mult3(float2 *__restrict__ spec, int n1, int n2, int nh, int np,
                                                    int kind, float beta_v, float beta_w, float scale, size_t spec_cs)
{
    const size_t m = (size_t)blockIdx.x * TPB + threadIdx.x;   // mode index over the n1 n2 nh modes
    if (m >= (size_t)n1 * n2 * nh) return;
    const int q3 = (int)(m % nh);
    const int q2 = (int)((m / nh) % n2);
    const int q1 = (int)(m / ((size_t)nh * n2));
    const size_t e = ((size_t)q1 * n2 + q2) * np + q3;
    const float k1 = (float)(q1 < (n1 >> 1) ? q1 : q1 - n1);
    const float k2 = (float)(q2 < (n2 >> 1) ? q2 : q2 - n2);
    const float k3 = (float)q3;
    const float c1 = q1 == (n1 >> 1) ? 0.f : k1, c2 = q2 == (n2 >> 1) ? 0.f : k2, c3 = q3 == nh - 1 ? 0.f : k3;
    const float ksq = k1 * k1 + k2 * k2 + k3 * k3;
    const float a = beta_v * ksq, c = beta_w * (1.0f + ksq);
    float2 x0 = spec[e], x1 = spec[spec_cs + e], x2 = spec[2 * spec_cs + e];
    const float pr = c1 * x0.x + c2 * x1.x + c3 * x2.x;   // kappa . x
    const float pi = c1 * x0.y + c2 * x1.y + c3 * x2.y;
    float d, f;   // y = d x + f kappa (kappa . x)
    if (kind == 0) {
        d = a;
        f = c;
    } else if (ksq == 0.f) {
        d = kind == 1 ? 1.0f / beta_v : 1.0f;
        f = 0.f;
    } else {
        const float r = c / (a + c * (c1 * c1 + c2 * c2 + c3 * c3));
        d = kind == 1 ? 1.0f / a : 1.0f;
        f = -r * d;
    }
    d *= scale;
    f *= scale;
    x0 = make_float2(fmaf(f * c1, pr, d * x0.x), fmaf(f * c1, pi, d * x0.y));
    x1 = make_float2(fmaf(f * c2, pr, d * x1.x), fmaf(f * c2, pi, d * x1.y));
    x2 = make_float2(fmaf(f * c3, pr, d * x2.x), fmaf(f * c3, pi, d * x2.y));
    spec[e] = x0;
    spec[spec_cs + e] = x1;
    spec[2 * spec_cs + e] = x2;
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
    return (size_t)ncomp * n1 * n2 * fft_row_pitch(n3) * sizeof(float2);
}

void fft_make_twiddles(float2 *host, int n, int count)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int t = 0; t < count; ++t) {
        const double a = -two_pi * t / n;
        host[t] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
}

namespace {
struct PassGeom;
void coupled3(const FFTPlan &P, int kind, float beta_v, float beta_w, const float *in, float *out, hipStream_t s);
} // namespace

namespace {

bool cols_ok(int L) { return L == 128 || L == 256 || L == 512 || L == 1024; }

// columns per tile of the register-resident column passes
int cols_width(int L) { return L <= 256 ? 4096 / L : 8192 / L; }

template <int MODE>
void launch_cols(int L, dim3 grid, float2 *spec, const float2 *tw, int nh, size_t plane_stride, size_t rs,
                 size_t spec_cs, int kind, float beta, float scale, int n1, int n2, hipStream_t s)
{
    if (L == 1024)
        hipLaunchKernelGGL((k_fft_colsx<4, MODE>), grid, dim3(NTX), 0, s, spec, tw, nh, plane_stride, rs, spec_cs, kind,
                           beta, scale, n1, n2);
    else if (L == 512)
        hipLaunchKernelGGL((k_fft_colsx<2, MODE>), grid, dim3(NTX), 0, s, spec, tw, nh, plane_stride, rs, spec_cs, kind,
                           beta, scale, n1, n2);
    else if (L == 256)
        hipLaunchKernelGGL((k_fft_cols<16, MODE>), grid, dim3(TPB), 0, s, spec, tw, nh, plane_stride, rs, spec_cs, kind,
                           beta, scale, n1, n2);
    else
        hipLaunchKernelGGL((k_fft_cols<8, MODE>), grid, dim3(TPB), 0, s, spec, tw, nh, plane_stride, rs, spec_cs, kind,
                           beta, scale, n1, n2);
}

bool rows_ok(int n3) { return n3 == 128 || n3 == 256 || n3 == 512 || n3 == 1024; }

// register-resident row kernel for rows of n3 reals (R2 = n3 / 32, NR = 256 / R2 rows per tile)
template <int R2>
void launch_rows_r2c(const FFTPlan &P, const float *in, int nc, size_t N, size_t spec_cs, hipStream_t s)
{
    hipLaunchKernelGGL((k_fft_rows_r2c<R2>), dim3(P.n1 * P.n2 / (256 / R2), nc), dim3(TPB), 0, s, in, P.spec, P.twM,
                       P.twS, N, spec_cs);
}

template <int R2>
void launch_rows_c2r(const FFTPlan &P, float *out, const float *add, int nc, size_t N, size_t spec_cs, hipStream_t s)
{
    hipLaunchKernelGGL((k_fft_rows_c2r<R2>), dim3(P.n1 * P.n2 / (256 / R2), nc), dim3(TPB), 0, s, P.spec, out, add,
                       P.twM, P.twS, N, spec_cs);
}

// x3 forward pass (real rows -> half spectrum), nc components
void pass_r2c(const FFTPlan &P, const float *in, int nc, int logM, int lognl3, size_t lds3, size_t spec_cs,
              hipStream_t s)
{
    const size_t N = (size_t)P.n1 * P.n2 * P.n3;
    const int nrows = P.n1 * P.n2;
    if (rows_ok(P.n3) && nrows % (256 / (P.n3 / 32)) == 0) {
        if (P.n3 == 1024) launch_rows_r2c<32>(P, in, nc, N, spec_cs, s);
        else if (P.n3 == 512) launch_rows_r2c<16>(P, in, nc, N, spec_cs, s);
        else if (P.n3 == 256) launch_rows_r2c<8>(P, in, nc, N, spec_cs, s);
        else launch_rows_r2c<4>(P, in, nc, N, spec_cs, s);
        return;
    }
    hipLaunchKernelGGL(k_fft_x3_r2c, dim3(nrows >> lognl3, nc), dim3(TPB), lds3, s, in, P.spec, P.twM, P.twS, logM,
                       lognl3, nrows, N, spec_cs, P.np);
}

// x3 inverse pass (half spectrum -> real rows, optional add), nc components
void pass_c2r(const FFTPlan &P, float *out, const float *add, int nc, int logM, int lognl3, size_t lds3,
              size_t spec_cs, hipStream_t s)
{
    const size_t N = (size_t)P.n1 * P.n2 * P.n3;
    const int nrows = P.n1 * P.n2;
    if (rows_ok(P.n3) && nrows % (256 / (P.n3 / 32)) == 0) {
        if (P.n3 == 1024) launch_rows_c2r<32>(P, out, add, nc, N, spec_cs, s);
        else if (P.n3 == 512) launch_rows_c2r<16>(P, out, add, nc, N, spec_cs, s);
        else if (P.n3 == 256) launch_rows_c2r<8>(P, out, add, nc, N, spec_cs, s);
        else launch_rows_c2r<4>(P, out, add, nc, N, spec_cs, s);
        return;
    }
    hipLaunchKernelGGL(k_fft_x3_c2r, dim3(nrows >> lognl3, nc), dim3(TPB), lds3, s, P.spec, out, add, P.twM, P.twS,
                       logM, lognl3, nrows, N, spec_cs, P.np);
}

// Stockham column passes (lines of 16 ... 64 points; 128 ... 1024 take the
// register-resident passes): a 256-thread tile of 4096 values holds C =
// 4096 / L columns (at most 32).
struct ColGeom {
    int logC;
    size_t lds;   // twiddle table + tile at pitch C + 1
};

ColGeom col_geom(int L)
{
    ColGeom c;
    const int logT = ilog2(TPB * EPT);
    c.logC = logT - ilog2(L) > 5 ? 5 : logT - ilog2(L);
    c.lds = (size_t)(L + (size_t)L * ((1 << c.logC) + 1)) * sizeof(float2);
    return c;
}


// x2 pass over every x1 plane (forward or inverse), nc components
void pass_x2(const FFTPlan &P, bool inv, int nc, size_t spec_cs, hipStream_t s)
{
    if (cols_ok(P.n2)) {
        const int C = cols_width(P.n2);
        const dim3 grid((P.nh + C - 1) / C, P.n1, nc);
        if (inv) launch_cols<2>(P.n2, grid, P.spec, P.tw2, P.nh, (size_t)P.n2 * P.np, P.np, spec_cs, 2, 0.f, 1.f, P.n1, P.n2, s);
        else launch_cols<1>(P.n2, grid, P.spec, P.tw2, P.nh, (size_t)P.n2 * P.np, P.np, spec_cs, 2, 0.f, 1.f, P.n1, P.n2, s);
        return;
    }
    const ColGeom cg = col_geom(P.n2);
    const int C2 = 1 << cg.logC;
    const dim3 grid((P.nh + C2 - 1) / C2, P.n1, nc);
    if (inv)
        hipLaunchKernelGGL((k_fft_x2<true, TPB>), grid, dim3(TPB), cg.lds, s, P.spec, P.tw2, ilog2(P.n2), P.n2, P.nh,
                           P.np, cg.logC, spec_cs);
    else
        hipLaunchKernelGGL((k_fft_x2<false, TPB>), grid, dim3(TPB), cg.lds, s, P.spec, P.tw2, ilog2(P.n2), P.n2, P.nh,
                           P.np, cg.logC, spec_cs);
}

// x1 pass over every x2 plane: mode 0 forward, symbol, inverse; 1 forward; 2 inverse
void pass_x1(const FFTPlan &P, int mode, int kind, float beta, float scale, int nc, size_t spec_cs, hipStream_t s)
{
    if (cols_ok(P.n1)) {
        const int C = cols_width(P.n1);
        const dim3 grid((P.nh + C - 1) / C, P.n2, nc);
        const size_t rs = (size_t)P.n2 * P.np;
        if (mode == 0) launch_cols<0>(P.n1, grid, P.spec, P.tw1, P.nh, P.np, rs, spec_cs, kind, beta, scale, P.n1, P.n2, s);
        else if (mode == 1) launch_cols<1>(P.n1, grid, P.spec, P.tw1, P.nh, P.np, rs, spec_cs, kind, beta, scale, P.n1, P.n2, s);
        else launch_cols<2>(P.n1, grid, P.spec, P.tw1, P.nh, P.np, rs, spec_cs, kind, beta, scale, P.n1, P.n2, s);
        return;
    }
    const ColGeom cg = col_geom(P.n1);
    const int C1 = 1 << cg.logC;
    const dim3 grid((P.nh + C1 - 1) / C1, P.n2, nc);
    hipLaunchKernelGGL((k_fft_x1_mult<TPB>), grid, dim3(TPB), cg.lds, s, P.spec, P.tw1, ilog2(P.n1), P.n1, P.n2, P.nh,
                       P.np, cg.logC, kind, beta, scale, spec_cs, mode);
}

} // namespace

void spectral_apply(const FFTPlan &P, int kind, float beta, float beta_w, int ncomp, const float *in, float *out,
                    const float *add, hipStream_t s)
{
    if (beta_w != 0.f && ncomp == 3 && kind != 2) {
        // the three components are coupled per mode: forward transforms,
        // one 3x3 pass over the half spectrum, inverse transforms
        coupled3(P, kind, beta, beta_w, in, out, s);
        if (add) launch_axpy(out, out, add, 1.0f, 3 * (size_t)P.n1 * P.n2 * P.n3, s);
        return;
    }
    if (kind == 3) kind = 2;   // K = I without the divergence term
    const int n1 = P.n1, n2 = P.n2, n3 = P.n3;
    const int M = n3 / 2, logM = ilog2(M);
    const size_t N = (size_t)n1 * n2 * n3;
    const size_t spec_cs = (size_t)n1 * n2 * P.np;
    const float scale = (float)(1.0 / (double)N);
    const int nrows = n1 * n2;
    const int logT = ilog2(TILE);
    // x3: nl rows of M per tile
    int lognl3 = logT - logM;            // M >= 8, so nl <= TILE / 8
    if ((1 << lognl3) > nrows) lognl3 = ilog2(nrows);
    const size_t lds3 = (size_t)(M + M + 1 + ((size_t)M + 1) * ((1 << lognl3) + 1)) * sizeof(float2);
    for (int c0 = 0; c0 < ncomp; c0 += P.ncomp_max) {
        const int nc = ncomp - c0 < P.ncomp_max ? ncomp - c0 : P.ncomp_max;
        const float *inc = in + c0 * N;
        float *outc = out + c0 * N;
        const float *addc = add ? add + c0 * N : nullptr;
        pass_r2c(P, inc, nc, logM, lognl3, lds3, spec_cs, s);
        pass_x2(P, false, nc, spec_cs, s);
        pass_x1(P, 0, kind, beta, scale, nc, spec_cs, s);
        pass_x2(P, true, nc, spec_cs, s);
        pass_c2r(P, outc, addc, nc, logM, lognl3, lds3, spec_cs, s);
    }
}

namespace {

struct PassGeom {
    int logM, lognl3, nrows;
    size_t lds3, N, spec_cs;
};

PassGeom geom(const FFTPlan &P)
{
    PassGeom G;
    const int logT = ilog2(TILE);
    G.logM = ilog2(P.n3 / 2);
    G.nrows = P.n1 * P.n2;
    G.lognl3 = logT - G.logM;
    if ((1 << G.lognl3) > G.nrows) G.lognl3 = ilog2(G.nrows);
    const int M = P.n3 / 2;
    G.lds3 = (size_t)(M + M + 1 + ((size_t)M + 1) * ((1 << G.lognl3) + 1)) * sizeof(float2);
    G.N = (size_t)P.n1 * P.n2 * P.n3;
    G.spec_cs = (size_t)P.n1 * P.n2 * P.np;
    return G;
}

void forward3(const FFTPlan &P, const PassGeom &G, int nc, const float *in, hipStream_t s)
{
    pass_r2c(P, in, nc, G.logM, G.lognl3, G.lds3, G.spec_cs, s);
    pass_x2(P, false, nc, G.spec_cs, s);
    pass_x1(P, 1, 2, 0.f, 1.f, nc, G.spec_cs, s);
}

void inverse3(const FFTPlan &P, const PassGeom &G, int nc, float *out, hipStream_t s)
{
    pass_x1(P, 2, 2, 0.f, 1.f, nc, G.spec_cs, s);
    pass_x2(P, true, nc, G.spec_cs, s);
    pass_c2r(P, out, nullptr, nc, G.logM, G.lognl3, G.lds3, G.spec_cs, s);
}

void coupled3(const FFTPlan &P, int kind, float beta_v, float beta_w, const float *in, float *out, hipStream_t s)
{
    // every plan of the library holds three components of spectrum
    const PassGeom G = geom(P);
    forward3(P, G, 3, in, s);
    const size_t modes = (size_t)P.n1 * P.n2 * P.nh;
    hipLaunchKernelGGL(k_spec_mult3, dim3((unsigned)((modes + TPB - 1) / TPB)), dim3(TPB), 0, s, P.spec, P.n1, P.n2,
                       P.nh, P.np, kind, beta_v, beta_w, (float)(1.0 / (double)G.N), G.spec_cs);
    inverse3(P, G, 3, out, s);
}

__global__ __launch_bounds__(TPB) void k_scale_f(float *x, float a, size_t n)
{
    const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (e < n) x[e] *= a;
}

} // namespace

void spectral_resample(const FFTPlan &A, const FFTPlan &B, int ncomp, const float *in, float *out, hipStream_t s)
{
    const PassGeom GA = geom(A), GB = geom(B);
    for (int c0 = 0; c0 < ncomp; c0 += min(A.ncomp_max, B.ncomp_max)) {
        const int nc = min(ncomp - c0, min(A.ncomp_max, B.ncomp_max));
        forward3(A, GA, nc, in + c0 * GA.N, s);
        const size_t nb = (size_t)B.n1 * B.n2 * B.nh * nc;
        hipLaunchKernelGGL(k_mode_copy, dim3((unsigned)((nb + TPB - 1) / TPB)), dim3(TPB), 0, s, A.spec, B.spec, A.n1,
                           A.n2, A.n3, B.n1, B.n2, B.n3, nc);
        inverse3(B, GB, nc, out + c0 * GB.N, s);
        const size_t n = GB.N * nc;
        hipLaunchKernelGGL(k_scale_f, dim3((unsigned)((n + TPB - 1) / TPB)), dim3(TPB), 0, s, out + c0 * GB.N,
                           (float)(1.0 / (double)GA.N), n);
    }
}

} // namespace clh
