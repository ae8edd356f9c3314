// Postprocessing of normal modes (Section 4.2, Applications).
//
// Perturbed densities: for an eigenpair (omega_l; u^l, v^l) of the BdG problem around the
// ground state Phi and an amplitude eps,
//   n_j^l(x, t) = | phi_j(x) + eps (u_j^l(x) e^{-i omega_l t} + conj(v_j^l(x)) e^{i omega_l t}) |^2,
// j = 1, 0, -1.  One pass over the modes: every thread owns one (mode, component, point),
// reads u and v once and writes the densities at all requested times (HBM-bound: 32 B read
// per point and mode plus 8 B written per time).
//
// Amplitude summaries (the 3-D example's isosurfaces of u_j^l and v_j^l, reduced to numbers):
// per mode and field w of (u_1, u_0, u_-1, v_1, v_0, v_-1) the norm h^d sum |w|^2, max |w|,
// the second moments h^d sum x_a^2 |w|^2 / norm and the reflection parities
// Re h^d sum w(x) conj(w(R_a x)) / norm.  One pass: workgroups own a slice of one field's
// points, read w and its mirror images (the mirror of a row is the same row read backwards,
// so those reads hit cached lines), reduce in a fixed order, and a second launch combines
// the slices in order (deterministic).
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

constexpr int AMP_SLICES = 64;      // workgroups per field
constexpr int AMP_N = 8;            // entries per field (bdg.h)

// part[(field * AMP_SLICES + slice) * AMP_N + q]: q = 0 sum |w|^2, 1 max |w|^2, 2..4 sum x_a^2 |w|^2,
// 5..7 sum Re w conj(w(R_a x)) over the slice (without h^d)
__global__ void __launch_bounds__(256) k_mode_amp_part(long long npts, int nx, int ny, int nz, int dim, double x0,
                                                       double y0, double z0, double hx, double hy, double hz,
                                                       const double2* __restrict__ uv, double* __restrict__ part) {
    const int field = blockIdx.y;
    const double2* w = uv + (long long)field * npts;
    const long long per = (npts + AMP_SLICES - 1) / AMP_SLICES;
    const long long p0 = (long long)blockIdx.x * per;
    const long long p1 = p0 + per < npts ? p0 + per : npts;
    double acc[AMP_N] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (long long p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
        const int ix = (int)(p % nx);
        const int iy = (int)((p / nx) % ny);
        const int iz = (int)(p / ((long long)nx * ny));
        const double2 a = w[p];
        const double m2 = a.x * a.x + a.y * a.y;
        acc[0] += m2;
        acc[1] = fmax(acc[1], m2);
        const double x = x0 + ix * hx, y = y0 + iy * hy, z = z0 + iz * hz;
        acc[2] += x * x * m2;
        // reflected points: index m -> (N - m) mod N along one axis
        const int rx = ix == 0 ? 0 : nx - ix;
        const double2 bx = w[p - ix + rx];
        acc[5] += a.x * bx.x + a.y * bx.y;
        if (dim >= 2) {
            acc[3] += y * y * m2;
            const int ry = iy == 0 ? 0 : ny - iy;
            const double2 by = w[p + (long long)(ry - iy) * nx];
            acc[6] += a.x * by.x + a.y * by.y;
        }
        if (dim >= 3) {
            acc[4] += z * z * m2;
            const int rz = iz == 0 ? 0 : nz - iz;
            const double2 bz = w[p + (long long)(rz - iz) * nx * ny];
            acc[7] += a.x * bz.x + a.y * bz.y;
        }
    }
    __shared__ double red[AMP_N][4];
    for (int q = 0; q < AMP_N; ++q) {
        double v = acc[q];
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_down(v, off);
            v = q == 1 ? fmax(v, o) : v + o;
        }
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < AMP_N) {
        const int q = threadIdx.x;
        double v = red[q][0];
        for (int i = 1; i < (int)(blockDim.x / 64); ++i) v = q == 1 ? fmax(v, red[q][i]) : v + red[q][i];
        part[((long long)field * AMP_SLICES + blockIdx.x) * AMP_N + q] = v;
    }
}

// out[field * AMP_N + q]: the slices combined in order, scaled by h^d and normalized
__global__ void k_mode_amp_final(int nfields, double hd, const double* __restrict__ part, double* __restrict__ out) {
    const int field = blockIdx.x * blockDim.x + threadIdx.x;
    if (field >= nfields) return;
    double s[AMP_N] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = 0; b < AMP_SLICES; ++b)
        for (int q = 0; q < AMP_N; ++q) {
            const double v = part[((long long)field * AMP_SLICES + b) * AMP_N + q];
            s[q] = q == 1 ? fmax(s[q], v) : s[q] + v;
        }
    const double N = hd * s[0];
    out[field * AMP_N + 0] = N;
    out[field * AMP_N + 1] = sqrt(s[1]);
    for (int q = 2; q < AMP_N; ++q) out[field * AMP_N + q] = N > 0 ? hd * s[q] / N : 0.0;
}

}  // namespace

extern "C" bdg_status bdg_mode_amplitudes(bdg_ctx* c, int nmodes, const void* UV_dev, double* out) {
    if (!c) return BDG_EINVAL;
    if (nmodes < 0) return ctx_fail(c, BDG_EINVAL, "bdg_mode_amplitudes: negative count");
    if (nmodes == 0) return BDG_OK;
    if (!UV_dev || !out) return ctx_fail(c, BDG_EINVAL, "bdg_mode_amplitudes: null pointer");
    const int nfields = 6 * nmodes;
    if (nfields > 65535) return ctx_fail(c, BDG_EINVAL, "bdg_mode_amplitudes: at most 10922 modes per call");
    void* ws = nullptr;
    BDG_TRY(ctx_scratch(c, 6, ((size_t)nfields * AMP_SLICES + (size_t)nfields) * AMP_N * sizeof(double), &ws));
    double* part = (double*)ws;
    double* res = part + (size_t)nfields * AMP_SLICES * AMP_N;
    hipLaunchKernelGGL(k_mode_amp_part, dim3(AMP_SLICES, (unsigned)nfields), dim3(256), 0, c->stream, c->npts,
                       c->n[0], c->n[1], c->n[2], c->dim, -c->L[0], -c->L[1], -c->L[2], c->h[0], c->h[1], c->h[2],
                       (const double2*)UV_dev, part);
    BDG_HIP(c, hipGetLastError());
    hipLaunchKernelGGL(k_mode_amp_final, dim3((unsigned)((nfields + 63) / 64)), dim3(64), 0, c->stream, nfields, c->hd,
                       (const double*)part, res);
    BDG_HIP(c, hipGetLastError());
    BDG_HIP(c, hipMemcpyAsync(out, res, (size_t)nfields * AMP_N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    return BDG_OK;
}

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
