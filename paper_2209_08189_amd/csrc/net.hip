// net.hip -- host orchestration of the learned warm-start network and its
// C ABI (cl_net_* and the cl_nn_* layer entry points).
//
// Network (input: template and reference at n^3, output: velocity at n^3):
//   encoder  L1 (n^3, 16 ch)   conv(2->16) conv(16->16)       pool
//            L2 (n/2, 32 ch)   conv(16->32) conv(32->32)      pool
//            L3 (n/4, 64 ch)   conv(32->64) conv(64->64)      pool
//            L4 (n/8, 128 ch)  conv(64->128) conv(128->128)
//   decoder  L3: up(L4) ++ enc L3 -> conv(192->64) conv(64->64)
//            L2: up(L3) ++ enc L2 -> conv(96->32) conv(32->32)
//            L1: up(L2) ++ enc L1 -> conv(48->16) conv(16->16)
//   head     1x1x1 conv 16 -> 3, FP32
// every 3x3x3 conv is followed by LeakyReLU; the two input channels are
// carried in a 16-channel tensor (channels 2..15 zero).  Loss: mean squared
// error on the velocity; optimiser: Adam on FP32 master weights, BF16
// weight copies packed for the matrix cores after every update.
#include "internal.h"

#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

namespace clh {
void nn_pack_weights(const float *w, unsigned short *out, int Ci, int Co, int flip, hipStream_t s);
void nn_conv3(const unsigned short *in, const void *wp, const float *bias, void *out, int out_f32, int D, int H, int W,
              int Ci, int Co, int act, float slope, hipStream_t s);
size_t nn_packed_weight_elems(int Ci, int Co);
size_t nn_dw_workspace_floats(int D, int H, int W, int Ci, int Co);
void nn_conv3_dw(const unsigned short *X, const unsigned short *dZ, float *partial, float *gw, float *gb, int D, int H,
                 int W, int Ci, int Co, hipStream_t s);
void nn_lrelu_bwd(const unsigned short *dY, const unsigned short *Y, float slope, size_t n, unsigned short *dZ,
                  hipStream_t s);
void nn_pool2(const unsigned short *in, unsigned short *out, int D, int H, int W, int C, hipStream_t s);
void nn_pool2_bwd(const unsigned short *gout, unsigned short *gin, int D, int H, int W, int C, int accumulate,
                  hipStream_t s);
void nn_up2cat(const unsigned short *a, const unsigned short *b, unsigned short *out, int D, int H, int W, int Ca,
               int Cb, hipStream_t s);
void nn_up2cat_bwd(const unsigned short *g, unsigned short *ga, unsigned short *gb, int D, int H, int W, int Ca, int Cb,
                   int accumulate_b, hipStream_t s);
void nn_head(const unsigned short *in, const float *w, const float *b, float *out, size_t P, int Ci, hipStream_t s);
void nn_head_bwd(const unsigned short *in, const float *gout, const float *w, unsigned short *gin, double *partials,
                 int nparts, double *dst_dev, size_t P, int Ci, hipStream_t s);
void nn_mse(const float *pred, const float *label, size_t n, float inv, float *grad, double *partials, int nparts,
            hipStream_t s);
void nn_adam(float *p, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2, float eps, float c1,
             float c2, hipStream_t s);
void nn_pack_input(const float *a, const float *b, unsigned short *out, size_t P, hipStream_t s);
} // namespace clh

using namespace clh;

namespace {

__global__ void k_d2f_add(const double *src, float *dst, int n, int accumulate)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = accumulate ? dst[e] + (float)src[e] : (float)src[e];
}

__global__ void k_axpy_f(float *y, const float *x, float a, size_t n)
{
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) y[e] += a * x[e];
}

struct ConvL {
    int Ci, Co, lvl;     // channels, resolution level (0 = n^3)
    size_t wo, bo;       // offsets of weight and bias in the parameter vector
    unsigned short *wpf, *wpb;   // packed forward / transposed weights (BF16)
};

struct Act {
    unsigned short *p = nullptr;
    int lvl = 0, C = 0;
};

} // namespace

struct cl_resampler {
    FFTPlan A{}, B{};
    hipStream_t s = nullptr;
    std::vector<void *> allocs;
};

struct cl_net {
    cl_net_options opt{};
    hipStream_t s = nullptr;
    int n = 128;
    int dims[4];
    std::vector<void *> allocs;
    std::vector<ConvL> conv;
    size_t nparam = 0, head_w = 0, head_b = 0;
    float *param = nullptr, *grad = nullptr, *gacc = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    float *partial = nullptr;   // weight-gradient partial sums
    double *dpart = nullptr, *dscal = nullptr, *hscal = nullptr, *dhead = nullptr;
    int nparts = 512;
    long step = 0;
    // activations (forward) and their gradients
    Act x0, a1, e1, p1, a2, e2, p2, a3, e3, p3, a4, e4, c3, b3, d3, c2, b2, d2, c1, b1, d1;
    Act g_a, g_b, g_c, dz;     // per-level scratch (max channels at each level is handled by sizing to level 0)
    Act ge1, ge2, ge3, ge4, gd2, gd3, gd1;
    float *vout = nullptr, *gv = nullptr;
    // warm-start work space for one registration grid (created on first use)
    cl_resampler *down = nullptr, *up = nullptr;
    int full[3] = {0, 0, 0};
    float *in0 = nullptr, *in1 = nullptr, *full_buf = nullptr;
    std::string err;
};

namespace {

struct NFail {
    int code;
};

#define NCHK(expr)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            net->err = std::string(#expr) + ": " + hipGetErrorString(e_);                \
            throw NFail{CL_ERR_HIP};                                                      \
        }                                                                                 \
    } while (0)

size_t vox(const cl_net *net, int lvl) { size_t d = net->dims[lvl]; return d * d * d; }

void *nalloc(cl_net *net, size_t bytes)
{
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) throw NFail{CL_ERR_OOM};
    net->allocs.push_back(p);
    return p;
}

Act act(cl_net *net, int lvl, int C)
{
    Act a;
    a.lvl = lvl;
    a.C = C;
    a.p = (unsigned short *)nalloc(net, vox(net, lvl) * C * 2);
    return a;
}

void conv_fwd(cl_net *net, const ConvL &c, const Act &in, const Act &out)
{
    const int d = net->dims[c.lvl];
    nn_conv3(in.p, c.wpf, net->param + c.bo, out.p, 0, d, d, d, c.Ci, c.Co, 1, net->opt.slope, net->s);
}

// backward of out = lrelu(conv(in)): given gout (w.r.t. out), accumulate the
// weight gradient into net->grad and write gin (w.r.t. in) unless gin is NULL
void conv_bwd(cl_net *net, const ConvL &c, const Act &in, const Act &out, const Act &gout, const Act *gin)
{
    const int d = net->dims[c.lvl];
    const size_t n = vox(net, c.lvl) * c.Co;
    nn_lrelu_bwd(gout.p, out.p, net->opt.slope, n, net->dz.p, net->s);
    nn_conv3_dw(in.p, net->dz.p, net->partial, net->grad + c.wo, net->grad + c.bo, d, d, d, c.Ci, c.Co, net->s);
    if (gin) nn_conv3(net->dz.p, c.wpb, nullptr, gin->p, 0, d, d, d, c.Co, c.Ci, 0, 0.f, net->s);
}

void pack_all(cl_net *net)
{
    for (const ConvL &c : net->conv) {
        nn_pack_weights(net->param + c.wo, c.wpf, c.Ci, c.Co, 0, net->s);
        nn_pack_weights(net->param + c.wo, c.wpb, c.Ci, c.Co, 1, net->s);
    }
}

void forward(cl_net *net, const float *m0, const float *m1)
{
    hipStream_t s = net->s;
    auto &C = net->conv;
    const int *dm = net->dims;
    nn_pack_input(m0, m1, net->x0.p, vox(net, 0), s);
    conv_fwd(net, C[0], net->x0, net->a1);
    conv_fwd(net, C[1], net->a1, net->e1);
    nn_pool2(net->e1.p, net->p1.p, dm[0], dm[0], dm[0], 16, s);
    conv_fwd(net, C[2], net->p1, net->a2);
    conv_fwd(net, C[3], net->a2, net->e2);
    nn_pool2(net->e2.p, net->p2.p, dm[1], dm[1], dm[1], 32, s);
    conv_fwd(net, C[4], net->p2, net->a3);
    conv_fwd(net, C[5], net->a3, net->e3);
    nn_pool2(net->e3.p, net->p3.p, dm[2], dm[2], dm[2], 64, s);
    conv_fwd(net, C[6], net->p3, net->a4);
    conv_fwd(net, C[7], net->a4, net->e4);
    nn_up2cat(net->e4.p, net->e3.p, net->c3.p, dm[2], dm[2], dm[2], 128, 64, s);
    conv_fwd(net, C[8], net->c3, net->b3);
    conv_fwd(net, C[9], net->b3, net->d3);
    nn_up2cat(net->d3.p, net->e2.p, net->c2.p, dm[1], dm[1], dm[1], 64, 32, s);
    conv_fwd(net, C[10], net->c2, net->b2);
    conv_fwd(net, C[11], net->b2, net->d2);
    nn_up2cat(net->d2.p, net->e1.p, net->c1.p, dm[0], dm[0], dm[0], 32, 16, s);
    conv_fwd(net, C[12], net->c1, net->b1);
    conv_fwd(net, C[13], net->b1, net->d1);
    nn_head(net->d1.p, net->param + net->head_w, net->param + net->head_b, net->vout, vox(net, 0), 16, s);
    NCHK(hipGetLastError());
}

// gradient of the loss w.r.t. every parameter into net->grad (overwritten);
// net->gv must hold dLoss/dv
void backward(cl_net *net)
{
    hipStream_t s = net->s;
    auto &C = net->conv;
    const int *dm = net->dims;
    nn_head_bwd(net->d1.p, net->gv, net->param + net->head_w, net->gd1.p, net->dpart, net->nparts, net->dhead,
                vox(net, 0), 16, s);
    hipLaunchKernelGGL(k_d2f_add, dim3(1), dim3(64), 0, s, net->dhead, net->grad + net->head_w, 51, 0);
    // decoder L1
    Act gb1{net->g_a.p, 0, 16}, gc1{net->g_b.p, 0, 48};
    conv_bwd(net, C[13], net->b1, net->d1, net->gd1, &gb1);
    conv_bwd(net, C[12], net->c1, net->b1, gb1, &gc1);
    Act gd2{net->gd2.p, 1, 32};
    nn_up2cat_bwd(gc1.p, gd2.p, net->ge1.p, dm[0], dm[0], dm[0], 32, 16, 0, s);
    // decoder L2
    Act gb2{net->g_a.p, 1, 32}, gc2{net->g_b.p, 1, 96};
    conv_bwd(net, C[11], net->b2, net->d2, gd2, &gb2);
    conv_bwd(net, C[10], net->c2, net->b2, gb2, &gc2);
    Act gd3{net->gd3.p, 2, 64};
    nn_up2cat_bwd(gc2.p, gd3.p, net->ge2.p, dm[1], dm[1], dm[1], 64, 32, 0, s);
    // decoder L3
    Act gb3{net->g_a.p, 2, 64}, gc3{net->g_b.p, 2, 192};
    conv_bwd(net, C[9], net->b3, net->d3, gd3, &gb3);
    conv_bwd(net, C[8], net->c3, net->b3, gb3, &gc3);
    nn_up2cat_bwd(gc3.p, net->ge4.p, net->ge3.p, dm[2], dm[2], dm[2], 128, 64, 0, s);
    // bottleneck
    Act ga4{net->g_a.p, 3, 128}, gp3{net->g_c.p, 3, 64};
    conv_bwd(net, C[7], net->a4, net->e4, net->ge4, &ga4);
    conv_bwd(net, C[6], net->p3, net->a4, ga4, &gp3);
    nn_pool2_bwd(gp3.p, net->ge3.p, dm[2], dm[2], dm[2], 64, 1, s);
    // encoder L3
    Act ga3{net->g_a.p, 2, 64}, gp2{net->g_c.p, 2, 32};
    conv_bwd(net, C[5], net->a3, net->e3, net->ge3, &ga3);
    conv_bwd(net, C[4], net->p2, net->a3, ga3, &gp2);
    nn_pool2_bwd(gp2.p, net->ge2.p, dm[1], dm[1], dm[1], 32, 1, s);
    // encoder L2
    Act ga2{net->g_a.p, 1, 32}, gp1{net->g_c.p, 1, 16};
    conv_bwd(net, C[3], net->a2, net->e2, net->ge2, &ga2);
    conv_bwd(net, C[2], net->p1, net->a2, ga2, &gp1);
    nn_pool2_bwd(gp1.p, net->ge1.p, dm[0], dm[0], dm[0], 16, 1, s);
    // encoder L1
    Act ga1{net->g_a.p, 0, 16};
    conv_bwd(net, C[1], net->a1, net->e1, net->ge1, &ga1);
    conv_bwd(net, C[0], net->x0, net->a1, ga1, nullptr);
    NCHK(hipGetLastError());
}

double loss_and_grad(cl_net *net, const float *label)
{
    const size_t n = 3 * vox(net, 0);
    nn_mse(net->vout, label, n, (float)(1.0 / (double)n), net->gv, net->dpart, net->nparts, net->s);
    launch_finalize(net->dpart, net->nparts, 0.5 / (double)n, net->dscal, net->s);
    NCHK(hipMemcpyAsync(net->hscal, net->dscal, sizeof(double), hipMemcpyDeviceToHost, net->s));
    NCHK(hipStreamSynchronize(net->s));
    return *net->hscal;
}

void init_params(cl_net *net)
{
    // He-style uniform initialisation from a seeded generator, biases 0;
    // the head starts at zero so an untrained network predicts v = 0.
    std::vector<float> h(net->nparam, 0.0f);
    std::mt19937_64 rng(net->opt.seed);
    for (const ConvL &c : net->conv) {
        const float a = std::sqrt(6.0f / (27.0f * c.Ci));
        std::uniform_real_distribution<float> U(-a, a);
        for (size_t e = 0; e < (size_t)27 * c.Ci * c.Co; ++e) h[c.wo + e] = U(rng);
    }
    NCHK(hipMemcpy(net->param, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
    NCHK(hipMemset(net->adam_m, 0, h.size() * sizeof(float)));
    NCHK(hipMemset(net->adam_v, 0, h.size() * sizeof(float)));
}

// output-channel tile counts the convolution kernels are instantiated for
bool tile_count_ok(int nt) { return nt == 1 || nt == 2 || nt == 3 || nt == 4 || nt == 6 || nt == 8 || nt == 12; }

} // namespace

extern "C" {

void cl_net_default_options(cl_net_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->struct_version = CL_NET_OPTIONS_VERSION;
    o->in_n = 128;
    o->base_channels = 16;
    o->slope = 0.2f;
    o->lr = 1e-3f;
    o->beta1 = 0.9f;
    o->beta2 = 0.999f;
    o->eps = 1e-8f;
    o->seed = 1;
    o->stream = nullptr;
}

int cl_net_create(cl_net **out, const cl_net_options *opt)
{
    if (!out || !opt) return CL_ERR_ARG;
    *out = nullptr;
    if (opt->struct_version != CL_NET_OPTIONS_VERSION) return CL_ERR_ARG;
    if (opt->base_channels != 16) return CL_ERR_UNSUPPORTED;
    const int n = opt->in_n;
    if (n < 32 || n > 256 || (n & (n - 1))) return CL_ERR_SHAPE;
    cl_net *net = new (std::nothrow) cl_net();
    if (!net) return CL_ERR_OOM;
    net->opt = *opt;
    net->s = (hipStream_t)opt->stream;
    net->n = n;
    for (int l = 0; l < 4; ++l) net->dims[l] = n >> l;
    try {
        const int ch[14][3] = {{16, 16, 0}, {16, 16, 0}, {16, 32, 1}, {32, 32, 1}, {32, 64, 2}, {64, 64, 2},
                               {64, 128, 3}, {128, 128, 3}, {192, 64, 2}, {64, 64, 2}, {96, 32, 1}, {32, 32, 1},
                               {48, 16, 0}, {16, 16, 0}};
        size_t off = 0, maxpart = 0;
        for (auto &c : ch) {
            ConvL L{};
            L.Ci = c[0]; L.Co = c[1]; L.lvl = c[2];
            L.wo = off; off += (size_t)27 * L.Ci * L.Co;
            L.bo = off; off += L.Co;
            net->conv.push_back(L);
            const int d = net->dims[L.lvl];
            const size_t part = nn_dw_workspace_floats(d, d, d, L.Ci, L.Co);
            if (part > maxpart) maxpart = part;
        }
        net->head_w = off; off += 16 * 3;
        net->head_b = off; off += 3;
        net->nparam = off;
        float **vecs[] = {&net->param, &net->grad, &net->gacc, &net->adam_m, &net->adam_v};
        for (float **v : vecs) *v = (float *)nalloc(net, off * sizeof(float));
        net->partial = (float *)nalloc(net, maxpart * sizeof(float));
        for (ConvL &L : net->conv) {
            L.wpf = (unsigned short *)nalloc(net, nn_packed_weight_elems(L.Ci, L.Co) * 2);
            L.wpb = (unsigned short *)nalloc(net, nn_packed_weight_elems(L.Ci, L.Co) * 2);
        }
        // FP64 partial sums: the loss uses one row, the head's weight gradient 51 rows
        net->dpart = (double *)nalloc(net, (size_t)51 * net->nparts * sizeof(double));
        net->dscal = (double *)nalloc(net, 4 * sizeof(double));
        net->dhead = (double *)nalloc(net, 64 * sizeof(double));
        if (hipHostMalloc((void **)&net->hscal, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess)
            throw NFail{CL_ERR_OOM};
        net->x0 = act(net, 0, 16); net->a1 = act(net, 0, 16); net->e1 = act(net, 0, 16);
        net->p1 = act(net, 1, 16); net->a2 = act(net, 1, 32); net->e2 = act(net, 1, 32);
        net->p2 = act(net, 2, 32); net->a3 = act(net, 2, 64); net->e3 = act(net, 2, 64);
        net->p3 = act(net, 3, 64); net->a4 = act(net, 3, 128); net->e4 = act(net, 3, 128);
        net->c3 = act(net, 2, 192); net->b3 = act(net, 2, 64); net->d3 = act(net, 2, 64);
        net->c2 = act(net, 1, 96); net->b2 = act(net, 1, 32); net->d2 = act(net, 1, 32);
        net->c1 = act(net, 0, 48); net->b1 = act(net, 0, 16); net->d1 = act(net, 0, 16);
        // gradient scratch: sized for the largest use at level 0 (48 channels)
        net->g_a = act(net, 0, 16); net->g_b = act(net, 0, 48); net->g_c = act(net, 1, 32);
        net->dz = act(net, 0, 48);
        net->ge1 = act(net, 0, 16); net->ge2 = act(net, 1, 32); net->ge3 = act(net, 2, 64); net->ge4 = act(net, 3, 128);
        net->gd1 = act(net, 0, 16); net->gd2 = act(net, 1, 32); net->gd3 = act(net, 2, 64);
        net->vout = (float *)nalloc(net, 3 * vox(net, 0) * sizeof(float));
        net->gv = (float *)nalloc(net, 3 * vox(net, 0) * sizeof(float));
        init_params(net);
        pack_all(net);
        NCHK(hipStreamSynchronize(net->s));
    } catch (const NFail &f) {
        cl_net_destroy(net);
        return f.code;
    }
    *out = net;
    return CL_OK;
}

void cl_net_destroy(cl_net *net)
{
    if (!net) return;
    (void)hipStreamSynchronize(net->s);
    cl_resampler_destroy(net->down);
    cl_resampler_destroy(net->up);
    for (void *p : net->allocs) (void)hipFree(p);
    if (net->hscal) (void)hipHostFree(net->hscal);
    delete net;
}

int cl_net_num_params(cl_net *net, size_t *n)
{
    if (!net || !n) return CL_ERR_ARG;
    *n = net->nparam;
    return CL_OK;
}

int cl_net_get_params(cl_net *net, float *dst)
{
    if (!net || !dst) return CL_ERR_ARG;
    try {
        NCHK(hipMemcpyAsync(dst, net->param, net->nparam * sizeof(float), hipMemcpyDeviceToDevice, net->s));
    } catch (const NFail &f) { return f.code; }
    return CL_OK;
}

int cl_net_set_params(cl_net *net, const float *src)
{
    if (!net || !src) return CL_ERR_ARG;
    try {
        NCHK(hipMemcpyAsync(net->param, src, net->nparam * sizeof(float), hipMemcpyDeviceToDevice, net->s));
        pack_all(net);
        NCHK(hipGetLastError());
    } catch (const NFail &f) { return f.code; }
    return CL_OK;
}

int cl_net_forward(cl_net *net, const float *m0, const float *m1, float *v_out)
{
    if (!net || !m0 || !m1 || !v_out) return CL_ERR_ARG;
    try {
        forward(net, m0, m1);
        NCHK(hipMemcpyAsync(v_out, net->vout, 3 * vox(net, 0) * sizeof(float), hipMemcpyDeviceToDevice, net->s));
    } catch (const NFail &f) { return f.code; }
    return CL_OK;
}

int cl_net_loss_grad(cl_net *net, const float *m0, const float *m1, const float *v_label, float *grad_out,
                     double *loss)
{
    if (!net || !m0 || !m1 || !v_label) return CL_ERR_ARG;
    try {
        forward(net, m0, m1);
        const double L = loss_and_grad(net, v_label);
        backward(net);
        if (grad_out)
            NCHK(hipMemcpyAsync(grad_out, net->grad, net->nparam * sizeof(float), hipMemcpyDeviceToDevice, net->s));
        NCHK(hipStreamSynchronize(net->s));
        if (loss) *loss = L;
    } catch (const NFail &f) { return f.code; }
    return CL_OK;
}

int cl_net_train_step(cl_net *net, const float *m0, const float *m1, const float *v_label, int batch, double *loss)
{
    if (!net || !m0 || !m1 || !v_label || batch < 1) return CL_ERR_ARG;
    try {
        const size_t P = vox(net, 0);
        double Ls = 0.0;
        NCHK(hipMemsetAsync(net->gacc, 0, net->nparam * sizeof(float), net->s));
        for (int b = 0; b < batch; ++b) {
            forward(net, m0 + (size_t)b * P, m1 + (size_t)b * P);
            Ls += loss_and_grad(net, v_label + (size_t)b * 3 * P);
            backward(net);
            hipLaunchKernelGGL(k_axpy_f, dim3((unsigned)((net->nparam + 255) / 256)), dim3(256), 0, net->s, net->gacc,
                               net->grad, 1.0f / batch, net->nparam);
        }
        ++net->step;
        const float c1 = 1.0f - std::pow(net->opt.beta1, (float)net->step);
        const float c2 = 1.0f - std::pow(net->opt.beta2, (float)net->step);
        nn_adam(net->param, net->gacc, net->adam_m, net->adam_v, net->nparam, net->opt.lr, net->opt.beta1,
                net->opt.beta2, net->opt.eps, c1, c2, net->s);
        pack_all(net);
        NCHK(hipGetLastError());
        NCHK(hipStreamSynchronize(net->s));
        if (loss) *loss = Ls / batch;
    } catch (const NFail &f) { return f.code; }
    return CL_OK;
}

const char *cl_net_last_error(const cl_net *net) { return net ? net->err.c_str() : "no network"; }

int cl_resampler_create(cl_resampler **out, int a1, int a2, int a3, int b1, int b2, int b3, void *stream)
{
    if (!out) return CL_ERR_ARG;
    *out = nullptr;
    const int d[6] = {a1, a2, a3, b1, b2, b3};
    for (int v : d)
        if (v < 16 || v > 1024 || (v & (v - 1))) return CL_ERR_SHAPE;
    cl_resampler *r = new (std::nothrow) cl_resampler();
    if (!r) return CL_ERR_OOM;
    r->s = (hipStream_t)stream;
    auto alloc = [&](size_t bytes) -> void * {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) throw NFail{CL_ERR_OOM};
        r->allocs.push_back(p);
        return p;
    };
    try {
        fft_plan_init(r->A, a1, a2, a3, 3, alloc);
        fft_plan_init(r->B, b1, b2, b3, 3, alloc);
    } catch (const NFail &f) {
        cl_resampler_destroy(r);
        return f.code;
    } catch (hipError_t) {
        cl_resampler_destroy(r);
        return CL_ERR_HIP;
    }
    *out = r;
    return CL_OK;
}

void cl_resampler_destroy(cl_resampler *r)
{
    if (!r) return;
    (void)hipStreamSynchronize(r->s);
    for (void *p : r->allocs) (void)hipFree(p);
    delete r;
}

int cl_resample(cl_resampler *r, const float *in, float *out, int ncomp)
{
    if (!r || !in || !out || ncomp < 1) return CL_ERR_ARG;
    spectral_resample(r->A, r->B, ncomp, in, out, r->s);
    return hipGetLastError() == hipSuccess ? CL_OK : CL_ERR_HIP;
}

int cl_warm_start(cl_ctx *ctx, cl_net *net, int *used, double *J_pred, double *J_zero)
{
    if (!ctx || !net) return CL_ERR_ARG;
    if (!ctx_has_images(ctx)) return CL_ERR_STATE;
    if (ctx_stream(ctx) != net->s) return CL_ERR_ARG;
    int n1, n2, n3;
    ctx_dims(ctx, &n1, &n2, &n3);
    const size_t N = (size_t)n1 * n2 * n3;
    const int n = net->n;
    try {
        if (net->full[0] != n1 || net->full[1] != n2 || net->full[2] != n3) {
            cl_resampler_destroy(net->down);
            cl_resampler_destroy(net->up);
            net->down = net->up = nullptr;
            int st = cl_resampler_create(&net->down, n1, n2, n3, n, n, n, net->s);
            if (st) return st;
            st = cl_resampler_create(&net->up, n, n, n, n1, n2, n3, net->s);
            if (st) return st;
            if (!net->in0) {
                net->in0 = (float *)nalloc(net, vox(net, 0) * sizeof(float));
                net->in1 = (float *)nalloc(net, vox(net, 0) * sizeof(float));
            }
            net->full_buf = (float *)nalloc(net, 3 * N * sizeof(float));
            net->full[0] = n1; net->full[1] = n2; net->full[2] = n3;
        }
        // J(0) first: the objective at the zero velocity
        NCHK(hipMemsetAsync(net->full_buf, 0, 3 * N * sizeof(float), net->s));
    } catch (const NFail &f) {
        return f.code;
    }
    double Jp = 0, J0 = 0;
    int st = cl_set_velocity(ctx, net->full_buf);
    if (st) return st;
    if ((st = cl_objective(ctx, &J0, nullptr, nullptr))) return st;
    try {
        // images -> FP32 (components 0 and 1 of the work buffer) -> network grid
        ctx_images_f32(ctx, net->full_buf, net->full_buf + N);
        spectral_resample(net->down->A, net->down->B, 1, net->full_buf, net->in0, net->s);
        spectral_resample(net->down->A, net->down->B, 1, net->full_buf + N, net->in1, net->s);
        forward(net, net->in0, net->in1);
        spectral_resample(net->up->A, net->up->B, 3, net->vout, net->full_buf, net->s);
        NCHK(hipGetLastError());
    } catch (const NFail &f) {
        return f.code;
    }
    st = cl_set_velocity(ctx, net->full_buf);
    if (st == CL_ERR_NONFINITE) {
        // a diverged network (NaN or Inf in its prediction) is judged like
        // any other prediction and discarded: the context keeps v = 0, whose
        // state is the one just evaluated
        if (used) *used = 0;
        if (J_pred) *J_pred = HUGE_VAL;
        if (J_zero) *J_zero = J0;
        return CL_OK;
    }
    if (st) return st;
    if ((st = cl_objective(ctx, &Jp, nullptr, nullptr))) return st;
    const bool keep = Jp < J0;
    if (!keep) {
        if (hipMemsetAsync(net->full_buf, 0, 3 * N * sizeof(float), net->s) != hipSuccess) return CL_ERR_HIP;
        if ((st = cl_set_velocity(ctx, net->full_buf))) return st;
    }
    if (used) *used = keep ? 1 : 0;
    if (J_pred) *J_pred = Jp;
    if (J_zero) *J_zero = J0;
    return CL_OK;
}

// ---- single layers (parity tests) ----------------------------------------

int cl_nn_conv3(const void *in, const float *w, const float *b, void *out, int out_f32, int D, int H, int W, int Ci,
                int Co, int act, float slope, int transpose, void *wpack, void *stream)
{
    if (!in || !w || !out || !wpack) return CL_ERR_ARG;
    if (Ci < 16 || Co < 16 || Ci % 16 || Co % 16 || W < 1 || D < 1 || H < 1) return CL_ERR_SHAPE;
    const int Kout = transpose ? Ci : Co, Kin = transpose ? Co : Ci;
    if (!tile_count_ok(Kout / 16)) return CL_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    nn_pack_weights(w, (unsigned short *)wpack, Ci, Co, transpose, s);
    nn_conv3((const unsigned short *)in, wpack, transpose ? nullptr : b, out, out_f32, D, H, W, Kin, Kout, act, slope, s);
    return hipGetLastError() == hipSuccess ? CL_OK : CL_ERR_HIP;
}

int cl_nn_conv3_dw_workspace(int D, int H, int W, int Ci, int Co, size_t *bytes)
{
    if (!bytes || W < 1) return CL_ERR_ARG;
    if (Ci < 16 || Co < 16 || Ci % 16 || Co % 16 || D < 1 || H < 1) return CL_ERR_SHAPE;
    *bytes = nn_dw_workspace_floats(D, H, W, Ci, Co) * sizeof(float);
    return CL_OK;
}

int cl_nn_conv3_dw(const void *x, const void *dz, float *gw, float *gb, void *workspace, int D, int H, int W, int Ci,
                   int Co, void *stream)
{
    if (!x || !dz || !gw || !workspace) return CL_ERR_ARG;
    if (Ci < 16 || Co < 16 || Ci % 16 || Co % 16 || W < 1 || D < 1 || H < 1) return CL_ERR_SHAPE;
    if (!tile_count_ok(Co / 16)) return CL_ERR_UNSUPPORTED;
    nn_conv3_dw((const unsigned short *)x, (const unsigned short *)dz, (float *)workspace, gw, gb, D, H, W, Ci, Co,
                (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? CL_OK : CL_ERR_HIP;
}

} // extern "C"
