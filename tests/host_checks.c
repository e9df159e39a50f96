/* Host-side checks of the C ABI that need no GPU: option validation,
 * workspace queries, argument errors, status strings, and clean failure of
 * the creation calls when no device can be used.  Built with
 * AddressSanitizer (host code only) and run by tests/test_host_asan.py;
 * exits non-zero on the first failed expectation count. */
#include "claire_hip.h"

#include <stdio.h>
#include <string.h>

static int fails = 0;
#define EXPECT(c)                                                                   \
    do {                                                                            \
        if (!(c)) {                                                                 \
            fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);          \
            ++fails;                                                                \
        }                                                                           \
    } while (0)

static int query(const cl_options *o, int n1, int n2, int n3)
{
    unsigned long long b = 0;
    return cl_query_workspace(n1, n2, n3, o, &b);
}

int main(void)
{
    cl_options o;
    cl_default_options(&o);
    EXPECT(o.struct_version == CL_OPTIONS_VERSION && o.nt == 4 && o.max_pcg == 10 && o.fault_flip_direction == 0);

    unsigned long long full = 0, lean = 0, f16 = 0;
    EXPECT(cl_query_workspace(256, 256, 256, &o, &full) == CL_OK && full > 0);
    cl_options c = o;
    c.workspace_cap_bytes = full - 1;                   /* below the full layout: lean */
    EXPECT(cl_query_workspace(256, 256, 256, &c, &lean) == CL_OK && lean < full);
    c = o;
    c.storage_state = CL_F16;
    c.storage_adjoint = CL_BF16;
    EXPECT(cl_query_workspace(256, 256, 256, &c, &f16) == CL_OK && f16 < full);
    EXPECT(cl_query_workspace(1024, 1024, 1024, &o, &full) == CL_OK);
    EXPECT(cl_query_workspace(256, 256, 256, &o, NULL) == CL_ERR_ARG);
    EXPECT(cl_query_workspace(256, 256, 256, NULL, &full) == CL_ERR_ARG);

    /* shapes: powers of two in [16, 1024] */
    EXPECT(query(&o, 24, 32, 32) == CL_ERR_SHAPE);
    EXPECT(query(&o, 8, 32, 32) == CL_ERR_SHAPE);
    EXPECT(query(&o, 32, 32, 2048) == CL_ERR_SHAPE);
    EXPECT(query(&o, 16, 1024, 64) == CL_OK);

    /* every option field is validated */
    c = o; c.struct_version = 1; EXPECT(query(&c, 32, 32, 32) == CL_ERR_ARG);
    c = o; c.nt = 0; EXPECT(query(&c, 32, 32, 32) == CL_ERR_ARG);
    c = o; c.beta_v = 0.0; EXPECT(query(&c, 32, 32, 32) == CL_ERR_ARG);
    c = o; c.beta_w = -1.0; EXPECT(query(&c, 32, 32, 32) == CL_ERR_ARG);
    c = o; c.max_pcg = 0; EXPECT(query(&c, 32, 32, 32) == CL_ERR_ARG);
    c = o; c.max_outer = -1; EXPECT(query(&c, 32, 32, 32) == CL_ERR_ARG);
    c = o; c.interp_order = 2; EXPECT(query(&c, 32, 32, 32) == CL_ERR_ARG);
    c = o; c.overlap_spectral = 3; EXPECT(query(&c, 32, 32, 32) == CL_ERR_ARG);
    c = o; c.fault_flip_direction = 2; EXPECT(query(&c, 32, 32, 32) == CL_ERR_ARG);
    c = o; c.precond = 7; EXPECT(query(&c, 32, 32, 32) == CL_ERR_ARG);
    c = o; c.precond = CL_PRECOND_H0; c.precond_inner = 0; EXPECT(query(&c, 32, 32, 32) == CL_ERR_ARG);
    c = o; c.gtol = -1.0; EXPECT(query(&c, 32, 32, 32) == CL_ERR_ARG);
    c = o; c.storage_state = 9; EXPECT(query(&c, 32, 32, 32) == CL_ERR_DTYPE);

    /* creation: argument errors before any device call, and a clean failure
     * (no leak, no crash) where no device can be used */
    cl_ctx *ctx = (cl_ctx *)&o;
    EXPECT(cl_create(&ctx, 24, 32, 32, &o) == CL_ERR_SHAPE && ctx == NULL);
    EXPECT(cl_create(NULL, 32, 32, 32, &o) == CL_ERR_ARG);
    c = o; c.nt = 0;
    EXPECT(cl_create(&ctx, 32, 32, 32, &c) == CL_ERR_ARG && ctx == NULL);
    c = o; c.workspace_cap_bytes = 1024;
    EXPECT(cl_create(&ctx, 32, 32, 32, &c) == CL_ERR_OOM && ctx == NULL);
    int st = cl_create(&ctx, 32, 32, 32, &o);
    if (st == CL_OK) cl_destroy(ctx);
    else EXPECT(st < 0 && ctx == NULL);

    /* NULL contexts are rejected by every entry point */
    float f = 0.f;
    double d = 0.0;
    EXPECT(cl_layout(NULL) < 0);
    cl_destroy(NULL);
    EXPECT(cl_set_images(NULL, &f, &f, CL_F32) == CL_ERR_ARG);
    EXPECT(cl_set_velocity(NULL, &f) == CL_ERR_ARG);
    EXPECT(cl_get_velocity(NULL, &f) == CL_ERR_ARG);
    EXPECT(cl_objective(NULL, &d, &d, &d) == CL_ERR_ARG);
    EXPECT(cl_gradient(NULL, &f, &d, &d) == CL_ERR_ARG);
    EXPECT(cl_hessian_matvec(NULL, &f, &f) == CL_ERR_ARG);
    EXPECT(cl_precond_apply(NULL, &f, &f) == CL_ERR_ARG);
    EXPECT(cl_solve(NULL, NULL) == CL_ERR_ARG);
    EXPECT(cl_deformed_template(NULL, &f) == CL_ERR_ARG);
    EXPECT(cl_jacobian_det(NULL, &f, &d, &d) == CL_ERR_ARG);
    EXPECT(cl_set_regularization(NULL, 1.0, 0.0) == CL_ERR_ARG);
    EXPECT(strlen(cl_last_error(NULL)) > 0);

    /* status and class names */
    for (int s = -9; s <= 3; ++s) EXPECT(cl_status_string(s) != NULL && strlen(cl_status_string(s)) > 0);
    EXPECT(cl_status_string(-99) != NULL);
    for (int k = 0; k < CL_K_COUNT; ++k) EXPECT(cl_kernel_class_name(k) != NULL);

    /* search and network options, layer workspace sizes */
    cl_search_options so;
    cl_default_search_options(&so);
    EXPECT(so.jmin > 0.0 && so.jmin < 1.0 && so.beta_v_max > so.beta_v_min);
    cl_net_options no;
    cl_net_default_options(&no);
    EXPECT(no.struct_version == CL_NET_OPTIONS_VERSION && no.in_n == 128 && no.base_channels == 16);
    size_t wb = 0;
    /* 3 x 3 x 6 = 54 voxel tiles of 16 x 4 x 2, one per chunk: 27 Ci Co weight
     * and Co bias partial sums each */
    EXPECT(cl_nn_conv3_dw_workspace(12, 12, 40, 16, 32, &wb) == CL_OK && wb == (size_t)54 * (27 * 16 * 32 + 32) * 4);
    EXPECT(cl_nn_conv3_dw_workspace(12, 12, 40, 8, 32, &wb) == CL_ERR_SHAPE);
    EXPECT(cl_nn_conv3_dw_workspace(12, 12, 40, 16, 32, NULL) == CL_ERR_ARG);
    cl_net *net = NULL;
    no.struct_version = 0;
    EXPECT(cl_net_create(&net, &no) == CL_ERR_ARG && net == NULL);
    cl_net_destroy(NULL);

    printf("host checks: %d failure(s)\n", fails);
    return fails ? 1 : 0;
}
