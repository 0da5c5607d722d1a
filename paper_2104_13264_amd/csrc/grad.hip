// Derivative of ln Z~ with frozen truncation isometries (placeholder until the
// adjoint kernels land).
#include "common.hpp"

int tn_grad_device(tn_ctx *ctx, double *, double *, double *) {
    return tn_fail(ctx, TN_EINVAL, "tn_grad is not available in this build");
}
