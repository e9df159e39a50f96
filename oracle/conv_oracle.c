/*
 * conv_oracle.c -- plain FP64 CPU reference of the layers of the learned
 * warm-start network (3D convolutional encoder-decoder that predicts an
 * initial velocity from the image pair; the registration method itself is
 * the judge of its output).
 *
 * TEST INFRASTRUCTURE ONLY.  Shares no code with the HIP implementation.
 *
 * Tensors are channels-last: x[z][y][x][c], D x H x W voxels, C channels.
 * Every operation is the definition written out as nested loops.
 *   conv3:     out[p][o] = b[o] + sum_{t in 3x3x3} sum_i w[t][i][o] in[p + t - 1][i]
 *              (zero padding outside the volume; t = (tz*3 + ty)*3 + tx)
 *   conv3_t:   the exact transpose (adjoint) of conv3 without bias:
 *              gin[q][i] = sum_t sum_o w[t][i][o] gout[q - t + 1][o]
 *   conv3_dw:  gw[t][i][o] = sum_p in[p + t - 1][i] gout[p][o];  gb[o] = sum_p gout[p][o]
 *   lrelu:     y = x > 0 ? x : s x
 *   pool2:     2x2x2 average
 *   up2cat:    out[p][0:Ca] = a[p / 2][:], out[p][Ca:Ca+Cb] = b[p][:]
 *   head:      out[p][o] = hb[o] + sum_i hw[i][o] in[p][i]
 */
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static long vidx(int D, int H, int W, int z, int y, int x) { (void)D; return ((long)z * H + y) * W + x; }

void cnv_conv3(int D, int H, int W, int Ci, int Co, const double *in, const double *w, const double *b, double *out)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double *o = out + vidx(D, H, W, z, y, x) * Co;
                for (int c = 0; c < Co; ++c) o[c] = b ? b[c] : 0.0;
                for (int tz = 0; tz < 3; ++tz)
                    for (int ty = 0; ty < 3; ++ty)
                        for (int tx = 0; tx < 3; ++tx) {
                            const int zz = z + tz - 1, yy = y + ty - 1, xx = x + tx - 1;
                            if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                            const double *src = in + vidx(D, H, W, zz, yy, xx) * Ci;
                            const double *wt = w + (long)((tz * 3 + ty) * 3 + tx) * Ci * Co;
                            for (int i = 0; i < Ci; ++i)
                                for (int c = 0; c < Co; ++c) o[c] += wt[(long)i * Co + c] * src[i];
                        }
            }
}

void cnv_conv3_t(int D, int H, int W, int Ci, int Co, const double *gout, const double *w, double *gin)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double *g = gin + vidx(D, H, W, z, y, x) * Ci;
                for (int i = 0; i < Ci; ++i) g[i] = 0.0;
                for (int tz = 0; tz < 3; ++tz)
                    for (int ty = 0; ty < 3; ++ty)
                        for (int tx = 0; tx < 3; ++tx) {
                            /* output point p with p + t - 1 = q */
                            const int zz = z - tz + 1, yy = y - ty + 1, xx = x - tx + 1;
                            if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                            const double *go = gout + vidx(D, H, W, zz, yy, xx) * Co;
                            const double *wt = w + (long)((tz * 3 + ty) * 3 + tx) * Ci * Co;
                            for (int i = 0; i < Ci; ++i) {
                                double s = 0.0;
                                for (int c = 0; c < Co; ++c) s += wt[(long)i * Co + c] * go[c];
                                g[i] += s;
                            }
                        }
            }
}

void cnv_conv3_dw(int D, int H, int W, int Ci, int Co, const double *in, const double *gout, double *gw, double *gb)
{
    memset(gw, 0, sizeof(double) * 27 * Ci * Co);
    if (gb) memset(gb, 0, sizeof(double) * Co);
    for (int t = 0; t < 27; ++t) {
        const int tz = t / 9, ty = (t / 3) % 3, tx = t % 3;
        double *wt = gw + (long)t * Ci * Co;
        for (int z = 0; z < D; ++z)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    const int zz = z + tz - 1, yy = y + ty - 1, xx = x + tx - 1;
                    if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                    const double *src = in + vidx(D, H, W, zz, yy, xx) * Ci;
                    const double *go = gout + vidx(D, H, W, z, y, x) * Co;
                    for (int i = 0; i < Ci; ++i)
                        for (int c = 0; c < Co; ++c) wt[(long)i * Co + c] += src[i] * go[c];
                }
    }
    if (gb)
        for (long p = 0; p < (long)D * H * W; ++p)
            for (int c = 0; c < Co; ++c) gb[c] += gout[p * Co + c];
}

void cnv_lrelu(long n, const double *x, double s, double *y)
{
    for (long q = 0; q < n; ++q) y[q] = x[q] > 0.0 ? x[q] : s * x[q];
}

void cnv_pool2(int D, int H, int W, int C, const double *in, double *out)
{
    const int d = D / 2, h = H / 2, w = W / 2;
    for (int z = 0; z < d; ++z)
        for (int y = 0; y < h; ++y)
            for (int x = 0; x < w; ++x)
                for (int c = 0; c < C; ++c) {
                    double s = 0.0;
                    for (int a = 0; a < 2; ++a)
                        for (int b2 = 0; b2 < 2; ++b2)
                            for (int e = 0; e < 2; ++e)
                                s += in[vidx(D, H, W, 2 * z + a, 2 * y + b2, 2 * x + e) * C + c];
                    out[vidx(d, h, w, z, y, x) * C + c] = s / 8.0;
                }
}

/* a: coarse (D/2, H/2, W/2, Ca); b: fine (D, H, W, Cb); out: fine, Ca + Cb */
void cnv_up2cat(int D, int H, int W, int Ca, int Cb, const double *a, const double *b, double *out)
{
    const int C = Ca + Cb;
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double *o = out + vidx(D, H, W, z, y, x) * C;
                const double *s = a + vidx(D / 2, H / 2, W / 2, z / 2, y / 2, x / 2) * Ca;
                for (int c = 0; c < Ca; ++c) o[c] = s[c];
                const double *t = b + vidx(D, H, W, z, y, x) * Cb;
                for (int c = 0; c < Cb; ++c) o[Ca + c] = t[c];
            }
}

void cnv_head(long n, int Ci, int Co, const double *in, const double *w, const double *b, double *out)
{
    for (long p = 0; p < n; ++p)
        for (int o = 0; o < Co; ++o) {
            double s = b ? b[o] : 0.0;
            for (int i = 0; i < Ci; ++i) s += w[(long)i * Co + o] * in[p * Ci + i];
            out[p * Co + o] = s;
        }
}
