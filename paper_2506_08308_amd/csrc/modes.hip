// Perturbed densities of normal modes (Section 4.2, Applications): for an eigenpair
// (omega_l; u^l, v^l) of the BdG problem around the ground state Phi and an amplitude eps,
//   n_j^l(x, t) = | phi_j(x) + eps (u_j^l(x) e^{-i omega_l t} + conj(v_j^l(x)) e^{i omega_l t}) |^2,
// j = 1, 0, -1.  One pass over the modes: every thread owns one (mode, component, point),
// reads u and v once and writes the densities at all requested times (HBM-bound: 32 B read
// per point and mode plus 8 B written per time).
#include "common.h"

#include <cmath>
#include <vector>

namespace {

// cs[2 (l nt + s)] = cos(omega_l t_s), cs[2 (l nt + s) + 1] = sin(omega_l t_s)
__global__ void __launch_bounds__(256) k_perturbed_density(long long npts, int nmodes, int nt,
                                                           const double* __restrict__ phi,
                                                           const double2* __restrict__ phic,
                                                           const double2* __restrict__ uv,
                                                           const double* __restrict__ cs, double eps,
                                                           double* __restrict__ out) {
    const long long total = (long long)nmodes * 3 * npts;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long p = e % npts;
        const int j = (int)((e / npts) % 3);
        const int l = (int)(e / (3 * npts));
        const double2 u = uv[((long long)l * 6 + j) * npts + p];
        const double2 v = uv[((long long)l * 6 + 3 + j) * npts + p];
        // real ground state (phi) or complex one (phic)
        const double2 ph = phic ? phic[(long long)j * npts + p] : double2{phi[(long long)j * npts + p], 0.0};
        for (int s = 0; s < nt; ++s) {
            const double c = cs[2 * ((long long)l * nt + s)];
            const double sn = cs[2 * ((long long)l * nt + s) + 1];
            // u e^{-i w t} + conj(v) e^{i w t}
            const double re = (u.x + v.x) * c + (u.y + v.y) * sn;
            const double im = (u.y - v.y) * c + (v.x - u.x) * sn;
            const double a = ph.x + eps * re, b = ph.y + eps * im;
            out[(((long long)l * nt + s) * 3 + j) * npts + p] = a * a + b * b;
        }
    }
}

}  // namespace

extern "C" bdg_status bdg_perturbed_density(bdg_ctx* c, int nmodes, const double* omega, const void* UV_dev,
                                            double eps, int nt, const double* t, void* out_dev) {
    if (!c) return BDG_EINVAL;
    if (nmodes < 0 || nt < 0) return ctx_fail(c, BDG_EINVAL, "bdg_perturbed_density: negative count");
    if (!std::isfinite(eps)) return ctx_fail(c, BDG_EINVAL, "bdg_perturbed_density: eps not finite");
    if (!c->has_gs) return ctx_fail(c, BDG_ESTATE, "bdg_perturbed_density: no ground state set");
    if (nmodes == 0 || nt == 0) return BDG_OK;
    if (!omega || !UV_dev || !t || !out_dev) return ctx_fail(c, BDG_EINVAL, "bdg_perturbed_density: null pointer");
    std::vector<double> cs(2 * (size_t)nmodes * nt);
    for (int l = 0; l < nmodes; ++l) {
        if (!std::isfinite(omega[l])) return ctx_fail(c, BDG_EINVAL, "bdg_perturbed_density: omega not finite");
        for (int s = 0; s < nt; ++s) {
            if (!std::isfinite(t[s])) return ctx_fail(c, BDG_EINVAL, "bdg_perturbed_density: t not finite");
            const double a = omega[l] * t[s];
            cs[2 * ((size_t)l * nt + s)] = std::cos(a);
            cs[2 * ((size_t)l * nt + s) + 1] = std::sin(a);
        }
    }
    void* dcs = nullptr;
    BDG_TRY(ctx_scratch(c, 6, cs.size() * sizeof(double), &dcs));
    BDG_HIP(c, hipMemcpyAsync(dcs, cs.data(), cs.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    const long long total = (long long)nmodes * 3 * c->npts;
    const unsigned nblk = (unsigned)std::min<long long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_perturbed_density, dim3(nblk), dim3(256), 0, c->stream, c->npts, nmodes, nt,
                       (const double*)c->phi, c->complex_gs ? (const double2*)c->phic : nullptr,
                       (const double2*)UV_dev, (const double*)dcs, eps, (double*)out_dev);
    BDG_HIP(c, hipGetLastError());
    // the host table must outlive the copy
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    return BDG_OK;
}
