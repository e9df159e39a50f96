// k_reduce.hip -- FP64 reductions (Krylov dot products, norms) and the
// streaming vector updates of PCG.  Reductions are two-stage and
// deterministic: a fixed number of workgroups accumulate FP64 partial sums
// in grid-stride order and one workgroup adds the partials in index order.
#include "internal.h"

namespace clh {

namespace {

constexpr int TPB = 256;

__global__ __launch_bounds__(TPB) void k_dot(const float *__restrict__ a, const float *__restrict__ b, size_t n,
                                             double *__restrict__ partials)
{
    double acc = 0.0;
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t p = (size_t)blockIdx.x * TPB + threadIdx.x; p < n; p += stride)
        acc += (double)a[p] * (double)b[p];
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

__global__ __launch_bounds__(TPB) void k_count_nonfinite(const float *__restrict__ a, size_t n,
                                                         double *__restrict__ partials)
{
    double acc = 0.0;
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t p = (size_t)blockIdx.x * TPB + threadIdx.x; p < n; p += stride)
        acc += isfinite(a[p]) ? 0.0 : 1.0;
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

__global__ __launch_bounds__(TPB) void k_finalize(const double *__restrict__ partials, int nb, double scale,
                                                  double *__restrict__ out)
{
    // each thread sums a contiguous slice in order, then the slices in order
    const int per = (nb + TPB - 1) / TPB;
    double acc = 0.0;
    for (int q = threadIdx.x * per; q < min(nb, (int)(threadIdx.x + 1) * per); ++q) acc += partials[q];
    __shared__ double s[TPB];
    s[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < TPB; ++q) t += s[q];
        out[0] = scale * t;
    }
}

// per-block min and max (a non-finite value turns both into NaN)
__global__ __launch_bounds__(TPB) void k_minmax(const float *__restrict__ a, size_t n, double *__restrict__ partials)
{
    float lo = INFINITY, hi = -INFINITY;
    bool bad = false;
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t p = (size_t)blockIdx.x * TPB + threadIdx.x; p < n; p += stride) {
        const float x = a[p];
        bad |= !isfinite(x);
        lo = fminf(lo, x);
        hi = fmaxf(hi, x);
    }
    if (bad) lo = hi = NAN;
    __shared__ float slo[TPB], shi[TPB];
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    if (threadIdx.x == 0) {
        float l = slo[0], h = shi[0];
        for (int q = 1; q < TPB; ++q) {
            const float lq = slo[q], hq = shi[q];
            l = (isnan(l) || isnan(lq)) ? NAN : fminf(l, lq);
            h = (isnan(h) || isnan(hq)) ? NAN : fmaxf(h, hq);
        }
        partials[2 * blockIdx.x] = l;
        partials[2 * blockIdx.x + 1] = h;
    }
}

__global__ __launch_bounds__(TPB) void k_minmax_final(const double *__restrict__ partials, int nb,
                                                      double *__restrict__ out)
{
    if (threadIdx.x != 0) return;
    double l = partials[0], h = partials[1];
    for (int q = 1; q < nb; ++q) {
        const double lq = partials[2 * q], hq = partials[2 * q + 1];
        l = (isnan(l) || isnan(lq)) ? NAN : fmin(l, lq);
        h = (isnan(h) || isnan(hq)) ? NAN : fmax(h, hq);
    }
    out[0] = l;
    out[1] = h;
}

__global__ __launch_bounds__(TPB) void k_pcg_update(float *__restrict__ x, float *__restrict__ r,
                                                    const float *__restrict__ p, const float *__restrict__ Hp,
                                                    float alpha, size_t n, double *__restrict__ partials)
{
    double acc = 0.0;
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t q = (size_t)blockIdx.x * TPB + threadIdx.x; q < n; q += stride) {
        x[q] = fmaf(alpha, p[q], x[q]);
        const float rq = fmaf(-alpha, Hp[q], r[q]);
        r[q] = rq;
        acc += (double)rq * (double)rq;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

__global__ __launch_bounds__(TPB) void k_axpy(float *y, const float *a, const float *b, float alpha,
                                              size_t n)
{
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t q = (size_t)blockIdx.x * TPB + threadIdx.x; q < n; q += stride) y[q] = fmaf(alpha, b[q], a[q]);
}

__global__ __launch_bounds__(TPB) void k_scale(float *__restrict__ y, const float *__restrict__ a, float alpha,
                                               size_t n)
{
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t q = (size_t)blockIdx.x * TPB + threadIdx.x; q < n; q += stride) y[q] = alpha * a[q];
}

// per-component sums of a 3-field vector: partials[c * nb + block]
__global__ __launch_bounds__(TPB) void k_comp_sums(const float *__restrict__ a, size_t n, double *__restrict__ partials)
{
    const int c = blockIdx.y;
    const float *x = a + c * n;
    double acc = 0.0;
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t p = (size_t)blockIdx.x * TPB + threadIdx.x; p < n; p += stride) acc += (double)x[p];
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[c * gridDim.x + blockIdx.x] = acc;
}

// y_c = (r_c - sum_c / n) + beta * y_c  for the 3 components (sums on device)
__global__ __launch_bounds__(TPB) void k_mean_free_axpy(float *y, const float *__restrict__ r,
                                                        const double *__restrict__ sums, float beta, size_t n)
{
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t q = (size_t)blockIdx.x * TPB + threadIdx.x; q < 3 * n; q += stride) {
        const int c = (int)(q / n);
        const float mean = (float)(sums[c] / (double)n);
        y[q] = (r[q] - mean) + beta * y[q];
    }
}

// Fused PCG kernels.  Device scalars (FP64) in sc[]: see the PCG_* slots in
// internal.h.

// alpha = rz / pHp; a non-positive curvature sets the flag and alpha = 0, so
// the update that follows leaves x and r unchanged
__global__ void k_pcg_alpha(double *sc)
{
    const double pHp = sc[PCG_PHP], rz = sc[PCG_RZ];
    const bool ok = pHp > 0.0;
    sc[PCG_ALPHA] = ok ? rz / pHp : 0.0;
    sc[PCG_NEG] = ok ? 0.0 : 1.0;
}

// beta = rz_new / rz, then rz = rz_new
__global__ void k_pcg_beta(double *sc)
{
    sc[PCG_BETA] = sc[PCG_RZNEW] / sc[PCG_RZ];
    sc[PCG_RZ] = sc[PCG_RZNEW];
}

// x += alpha p, r -= alpha Hp on component c = blockIdx.y; per-block partial
// sums of r^2 (partials[c nb + b]) and of r (partials[(3 + c) nb + b])
__global__ __launch_bounds__(TPB) void k_pcg_update3(float *__restrict__ x, float *__restrict__ r,
                                                     const float *__restrict__ p, const float *__restrict__ Hp,
                                                     const double *__restrict__ sc, size_t n,
                                                     double *__restrict__ partials)
{
    const int c = blockIdx.y, nb = gridDim.x;
    const float alpha = (float)sc[PCG_ALPHA];
    const size_t off = c * n;
    double a2 = 0.0, a1 = 0.0;
    const size_t stride = (size_t)nb * TPB;
    for (size_t q = (size_t)blockIdx.x * TPB + threadIdx.x; q < n; q += stride) {
        float rq = r[off + q];
        if (alpha != 0.0f) {          // alpha = 0: curvature exit, x and r stay as they are
            x[off + q] = fmaf(alpha, p[off + q], x[off + q]);
            rq = fmaf(-alpha, Hp[off + q], rq);
            r[off + q] = rq;
        }
        a2 += (double)rq * (double)rq;
        a1 += (double)rq;
    }
    a2 = block_sum(a2);
    if (threadIdx.x == 0) partials[c * nb + blockIdx.x] = a2;
    a1 = block_sum(a1);
    if (threadIdx.x == 0) partials[(3 + c) * nb + blockIdx.x] = a1;
}

__global__ void k_pcg_beta_flex(double *sc)
{
    sc[PCG_BETA] = (sc[PCG_RZNEW] - sc[PCG_RZOLD]) / sc[PCG_RZ];
    sc[PCG_RZ] = sc[PCG_RZNEW];
}

__global__ __launch_bounds__(TPB) void k_pcg_direction_lz(float *__restrict__ p, float *__restrict__ q,
                                                          const float *__restrict__ z, const float *__restrict__ Lz,
                                                          const double *__restrict__ sc, size_t n3)
{
    const float beta = (float)sc[PCG_BETA];
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < n3; e += stride) {
        p[e] = fmaf(beta, p[e], z[e]);
        q[e] = Lz[e] + beta * q[e];
    }
}

__global__ __launch_bounds__(TPB) void k_axpy_sc(float *__restrict__ y, const float *__restrict__ x,
                                                 const double *__restrict__ sc, size_t n3)
{
    const float alpha = (float)sc[PCG_ALPHA];
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < n3; e += stride) y[e] = fmaf(alpha, x[e], y[e]);
}

// y_c += scale * sums[c] on the 3 components of n values
__global__ __launch_bounds__(TPB) void k_add_sums3(float *__restrict__ y, const double *__restrict__ sums, double scale,
                                                   size_t n)
{
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < 3 * n; e += stride)
        y[e] += (float)(scale * sums[e / n]);
}

// Zero-velocity Hessian: out = Lp + (G . p) G, and p . out per block
__global__ __launch_bounds__(TPB) void k_h0_apply(const float *__restrict__ p, const float *__restrict__ Lp,
                                                  const float *__restrict__ G, float *__restrict__ out, size_t n,
                                                  double *__restrict__ partials)
{
    double acc = 0.0;
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t q = (size_t)blockIdx.x * TPB + threadIdx.x; q < n; q += stride) {
        const float g0 = G[q], g1 = G[n + q], g2 = G[2 * n + q];
        const float p0 = p[q], p1 = p[n + q], p2 = p[2 * n + q];
        const float gp = g0 * p0 + g1 * p1 + g2 * p2;
        const float o0 = fmaf(gp, g0, Lp[q]), o1 = fmaf(gp, g1, Lp[n + q]), o2 = fmaf(gp, g2, Lp[2 * n + q]);
        out[q] = o0;
        out[n + q] = o1;
        out[2 * n + q] = o2;
        acc += (double)p0 * o0 + (double)p1 * o1 + (double)p2 * o2;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// Inner step of the zero-velocity preconditioner, direction and operator in
// one pass: p = z + beta p, q = r + beta q (q = L_0 p), out = q + (G . p) G,
// per-block partials of p . out
__global__ __launch_bounds__(TPB) void k_h0_direction_apply(float *__restrict__ p, float *__restrict__ q,
                                                            const float *__restrict__ z, const float *__restrict__ r,
                                                            const float *__restrict__ G, float *__restrict__ out,
                                                            const double *__restrict__ sc, size_t n,
                                                            double *__restrict__ partials)
{
    const float beta = (float)sc[PCG_BETA];
    double acc = 0.0;
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < n; e += stride) {
        const float p0 = fmaf(beta, p[e], z[e]), p1 = fmaf(beta, p[n + e], z[n + e]),
                    p2 = fmaf(beta, p[2 * n + e], z[2 * n + e]);
        const float q0 = r[e] + beta * q[e], q1 = r[n + e] + beta * q[n + e], q2 = r[2 * n + e] + beta * q[2 * n + e];
        p[e] = p0;
        p[n + e] = p1;
        p[2 * n + e] = p2;
        q[e] = q0;
        q[n + e] = q1;
        q[2 * n + e] = q2;
        const float g0 = G[e], g1 = G[n + e], g2 = G[2 * n + e];
        const float gp = g0 * p0 + g1 * p1 + g2 * p2;
        const float o0 = fmaf(gp, g0, q0), o1 = fmaf(gp, g1, q1), o2 = fmaf(gp, g2, q2);
        out[e] = o0;
        out[n + e] = o1;
        out[2 * n + e] = o2;
        acc += (double)p0 * o0 + (double)p1 * o1 + (double)p2 * o2;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// z += alpha p, r -= alpha H over 3 n values (alpha = sc[PCG_ALPHA]; no
// reductions)
__global__ __launch_bounds__(TPB) void k_h0_update(float *__restrict__ z, float *__restrict__ r,
                                                   const float *__restrict__ p, const float *__restrict__ H,
                                                   const double *__restrict__ sc, size_t n3)
{
    const float alpha = (float)sc[PCG_ALPHA];
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < n3; e += stride) {
        z[e] = fmaf(alpha, p[e], z[e]);
        r[e] = fmaf(-alpha, H[e], r[e]);
    }
}

// p = z + beta p and q = (r - mean r) + beta q on every component (q is
// beta A p carried by recurrence; means from the component sums in sc)
__global__ __launch_bounds__(TPB) void k_pcg_direction(float *__restrict__ p, float *__restrict__ q,
                                                       const float *__restrict__ z, const float *__restrict__ r,
                                                       const double *__restrict__ sc, size_t n)
{
    const float beta = (float)sc[PCG_BETA];
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < 3 * n; e += stride) {
        const int c = (int)(e / n);
        const float mean = (float)(sc[PCG_SUMR + c] / (double)n);
        p[e] = fmaf(beta, p[e], z[e]);
        q[e] = (r[e] - mean) + beta * q[e];
    }
}

template <typename To>
__global__ __launch_bounds__(TPB) void k_convert(To *__restrict__ out, const float *__restrict__ in, size_t n)
{
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t q = (size_t)blockIdx.x * TPB + threadIdx.x; q < n; q += stride) stf(out + q, in[q]);
}

template <typename Ti>
__global__ __launch_bounds__(TPB) void k_to_f32(const Ti *__restrict__ in, float *__restrict__ out, size_t n)
{
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t q = (size_t)blockIdx.x * TPB + threadIdx.x; q < n; q += stride) out[q] = ldf(in + q);
}

// Streaming copy, 16 bytes per lane per iteration when aligned.
__global__ __launch_bounds__(TPB) void k_copy4(const float4 *__restrict__ src, float4 *__restrict__ dst, size_t n4)
{
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t q = (size_t)blockIdx.x * TPB + threadIdx.x; q < n4; q += stride) dst[q] = src[q];
}

__global__ __launch_bounds__(TPB) void k_copy1(const float *__restrict__ src, float *__restrict__ dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t q = (size_t)blockIdx.x * TPB + threadIdx.x; q < n; q += stride) dst[q] = src[q];
}

__global__ __launch_bounds__(TPB) void k_fill(float *__restrict__ dst, float v, size_t n)
{
    const size_t stride = (size_t)gridDim.x * TPB;
    for (size_t q = (size_t)blockIdx.x * TPB + threadIdx.x; q < n; q += stride) dst[q] = v;
}

inline dim3 stream_grid(size_t n)
{
    size_t b = (n + TPB - 1) / TPB;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

} // namespace

int reduce_blocks(size_t n)
{
    size_t b = (n + TPB * 4 - 1) / (TPB * 4);
    if (b > 2048) b = 2048;
    if (b < 1) b = 1;
    return (int)b;
}

void launch_dot(const float *a, const float *b, size_t n, double *partials, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot, dim3(nblocks), dim3(TPB), 0, s, a, b, n, partials);
}

void launch_count_nonfinite(const float *a, size_t n, double *partials, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_nonfinite, dim3(nblocks), dim3(TPB), 0, s, a, n, partials);
}

void launch_minmax(const float *a, size_t n, double *partials, int nblocks, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_minmax, dim3(nblocks), dim3(TPB), 0, s, a, n, partials);
    hipLaunchKernelGGL(k_minmax_final, dim3(1), dim3(TPB), 0, s, partials, nblocks, out);
}

void launch_finalize(const double *partials, int nblocks, double scale, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(TPB), 0, s, partials, nblocks, scale, out);
}

void launch_pcg_update(float *x, float *r, const float *p, const float *Hp, float alpha, size_t n,
                       double *partials, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_update, dim3(nblocks), dim3(TPB), 0, s, x, r, p, Hp, alpha, n, partials);
}

void launch_axpy(float *y, const float *a, const float *b, float alpha, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy, stream_grid(n), dim3(TPB), 0, s, y, a, b, alpha, n);
}

void launch_scale(float *y, const float *a, float alpha, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale, stream_grid(n), dim3(TPB), 0, s, y, a, alpha, n);
}

void launch_comp_sums3(const float *a, size_t n, double *partials, int nblocks, double *sums_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_comp_sums, dim3(nblocks, 3), dim3(TPB), 0, s, a, n, partials);
    for (int c = 0; c < 3; ++c) launch_finalize(partials + c * nblocks, nblocks, 1.0, sums_out + c, s);
}

void launch_mean_free_axpy(float *y, const float *r, const double *sums, float beta, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_mean_free_axpy, stream_grid(3 * n), dim3(TPB), 0, s, y, r, sums, beta, n);
}

void launch_pcg_alpha(double *sc, hipStream_t s) { hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(1), 0, s, sc); }

void launch_pcg_beta(double *sc, hipStream_t s) { hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(1), 0, s, sc); }

void launch_pcg_update3(float *x, float *r, const float *p, const float *Hp, double *sc, size_t n, double *partials,
                        int nblocks, double rscale, hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_update3, dim3(nblocks, 3), dim3(TPB), 0, s, x, r, p, Hp, sc, n, partials);
    // ||r||^2 over the three components in order, then the component sums
    launch_finalize(partials, 3 * nblocks, rscale, sc + PCG_RR, s);
    for (int c = 0; c < 3; ++c) launch_finalize(partials + (3 + c) * nblocks, nblocks, 1.0, sc + PCG_SUMR + c, s);
}

void launch_pcg_beta_flex(double *sc, hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_beta_flex, dim3(1), dim3(1), 0, s, sc);
}

void launch_pcg_direction_lz(float *p, float *q, const float *z, const float *Lz, const double *sc, size_t n,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_direction_lz, stream_grid(3 * n), dim3(TPB), 0, s, p, q, z, Lz, sc, 3 * n);
}

void launch_axpy_sc(float *y, const float *x, const double *sc, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy_sc, stream_grid(3 * n), dim3(TPB), 0, s, y, x, sc, 3 * n);
}

void launch_add_sums3(float *y, const double *sums, double scale, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_sums3, stream_grid(3 * n), dim3(TPB), 0, s, y, sums, scale, n);
}

void launch_h0_direction_apply(float *p, float *q, const float *z, const float *r, const float *G, float *out,
                               const double *sc, size_t n, double *partials, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_h0_direction_apply, dim3(nblocks), dim3(TPB), 0, s, p, q, z, r, G, out, sc, n, partials);
}

void launch_h0_update(float *z, float *r, const float *p, const float *H, const double *sc, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_h0_update, stream_grid(3 * n), dim3(TPB), 0, s, z, r, p, H, sc, 3 * n);
}

void launch_h0_apply(const float *p, const float *Lp, const float *G, float *out, size_t n, double *partials,
                     int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_h0_apply, dim3(nblocks), dim3(TPB), 0, s, p, Lp, G, out, n, partials);
}

void launch_pcg_direction(float *p, float *q, const float *z, const float *r, const double *sc, size_t n,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_direction, stream_grid(3 * n), dim3(TPB), 0, s, p, q, z, r, sc, n);
}

void launch_convert(int dt_out, void *out, const float *in, size_t n, hipStream_t s)
{
    with_dtype(dt_out, [&](auto to) {
        using To = decltype(to);
        hipLaunchKernelGGL((k_convert<To>), stream_grid(n), dim3(TPB), 0, s, (To *)out, in, n);
    });
}

void launch_to_f32(int dt_in, const void *in, float *out, size_t n, hipStream_t s)
{
    with_dtype(dt_in, [&](auto ti) {
        using Ti = decltype(ti);
        hipLaunchKernelGGL((k_to_f32<Ti>), stream_grid(n), dim3(TPB), 0, s, (const Ti *)in, out, n);
    });
}

void launch_copy_f32(const float *src, float *dst, size_t n, hipStream_t s)
{
    if (((uintptr_t)src % 16) == 0 && ((uintptr_t)dst % 16) == 0 && n % 4 == 0)
        hipLaunchKernelGGL(k_copy4, stream_grid(n / 4), dim3(TPB), 0, s, (const float4 *)src, (float4 *)dst, n / 4);
    else
        hipLaunchKernelGGL(k_copy1, stream_grid(n), dim3(TPB), 0, s, src, dst, n);
}

void launch_fill_f32(float *dst, float v, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, stream_grid(n), dim3(TPB), 0, s, dst, v, n);
}

} // namespace clh
