// placeholder replaced below
#include "common.h"
extern "C" bdg_status bdg_eigs_grad(bdg_ctx* c, int k, const double* omega, const void* UV_dev, double* dV_dev,
                                    double* dbeta_n, double* dbeta_s) {
    if (!c) return BDG_EINVAL;
    return ctx_fail(c, BDG_ESTATE, "bdg_eigs_grad: not built");
}
