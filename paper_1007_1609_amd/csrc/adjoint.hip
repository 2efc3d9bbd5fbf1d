// Reverse-mode derivative of the batched recursion (placeholder until the
// checkpointed adjoint kernels land).
#include "common.hpp"

using namespace cbdg;

extern "C" int cbdg_backward_workspace_size(const cbdg_op *op, int32_t tile, int32_t N,
                                            int32_t ckpt_stride, size_t *bytes)
{
    clear_error();
    (void)op; (void)tile; (void)N; (void)ckpt_stride; (void)bytes;
    return fail(CBDG_EUNSUPPORTED, "backward_workspace_size: not implemented yet");
}

extern "C" int cbdg_chebyshev_moments_backward(const cbdg_op *op, const int32_t *start_sites,
                                               int64_t n_start, int32_t N, int32_t tile,
                                               int32_t ckpt_stride, const double *dmu_ee,
                                               const double *dmu_he, void *workspace,
                                               size_t workspace_bytes, double *grad_eps,
                                               double *grad_delta, void *stream)
{
    clear_error();
    (void)op; (void)start_sites; (void)n_start; (void)N; (void)tile; (void)ckpt_stride;
    (void)dmu_ee; (void)dmu_he; (void)workspace; (void)workspace_bytes; (void)grad_eps;
    (void)grad_delta; (void)stream;
    return fail(CBDG_EUNSUPPORTED, "chebyshev_moments_backward: not implemented yet");
}
