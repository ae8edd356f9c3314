// Ground state of the spin-1 condensate on the device (Section 1: eqs. groundDef, NLEP):
// preconditioned normalized gradient flow with least-squares multipliers.
//   r   = H(Phi) Phi - mu Phi - lambda S_z Phi,   (mu, lambda) minimizing ||r||
//   Phi <- Phi - tau F^-1 (|k|^2/2 + alpha)^-1 F r
//   Phi_j <- sigma_j Phi_j with sigma solving: mass, magnetization, sigma_1 sigma_-1 = sigma_0^2
// H(Phi) Phi is the right-hand side of eq. (GPE) for a real spinor.  Its fixed point
// satisfies eq. (NLEP) with Lambda = diag(mu + lambda, mu, mu - lambda).
#include "common.h"

#include <cmath>
#include <vector>

namespace {

constexpr int GB = 256;
constexpr int GBLK = 1024;

template <int NQ> __device__ void block_reduce_store(double (&v)[NQ], double* part) {
    __shared__ double red[NQ][GB / 64];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = v[q];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = s;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        double a = 0;
        for (int w = 0; w < GB / 64; ++w) a += red[threadIdx.x][w];
        part[threadIdx.x * gridDim.x + blockIdx.x] = a;
    }
}

__global__ void k_final_sum(int nq, int nblk, const double* __restrict__ part, double scale, double* out) {
    const int q = threadIdx.x;
    if (q >= nq) return;
    double a = 0;
    const double* pq = part + (long long)q * nblk;
    // eight loads in flight, summed in block order (the same rounding as one at a time)
    int b = 0;
    for (; b + 8 <= nblk; b += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = pq[b + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) a += v[u];
    }
    for (; b < nblk; ++b) a += pq[b];
    out[q] = a * scale;
}

// Gaussian start exp(-|x|^2/2) times the spin weights
__global__ void k_gs_init(long long npts, int nx, int ny, int dim, double Lx, double Ly, double Lz, double hx, double hy,
                          double hz, double w1, double w0, double wm, double* phi) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
        const int ix = (int)(p % nx);
        const int iy = (int)((p / nx) % ny);
        const int iz = (int)(p / ((long long)nx * ny));
        double r2 = 0;
        const double x = -Lx + ix * hx;
        r2 += x * x;
        if (dim > 1) { const double y = -Ly + iy * hy; r2 += y * y; }
        if (dim > 2) { const double z = -Lz + iz * hz; r2 += z * z; }
        const double g = exp(-0.5 * r2);
        phi[p] = w1 * g;
        phi[npts + p] = w0 * g;
        phi[2 * npts + p] = wm * g;
    }
}

__global__ void k_real_to_cplx(long long n, const double* __restrict__ a, double2* __restrict__ z) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        z[i] = cmk<double2>(a[i], 0.0);
}

// H(Phi) Phi (eq. GPE, real spinor) from the kinetic part tphi
__global__ void k_gs_rhs(long long npts, const double* __restrict__ phi, const double* __restrict__ V,
                         const double2* __restrict__ tphi, double bn, double bs, double* __restrict__ hphi) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
        const double a = phi[p], b = phi[npts + p], d = phi[2 * npts + p];
        const double rho = a * a + b * b + d * d, rz = a * a - d * d;
        const double v = V[p];
        hphi[p] = tphi[p].x + (v + bn * rho + bs * (b * b + rz)) * a + bs * b * b * d;
        hphi[npts + p] = tphi[npts + p].x + (v + bn * rho + bs * (a * a + d * d)) * b + 2.0 * bs * d * b * a;
        hphi[2 * npts + p] = tphi[2 * npts + p].x + (v + bn * rho + bs * (b * b - rz)) * d + bs * a * b * b;
    }
}

// sums: <Phi,Phi>, <Phi,SzPhi>, <SzPhi,SzPhi>, <Phi,HPhi>, <SzPhi,HPhi>
__global__ void __launch_bounds__(GB) k_gs_dots(long long npts, const double* __restrict__ phi,
                                                const double* __restrict__ hphi, double* part) {
    double v[5] = {0, 0, 0, 0, 0};
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
        const double a = phi[p], b = phi[npts + p], d = phi[2 * npts + p];
        const double ha = hphi[p], hb = hphi[npts + p], hd = hphi[2 * npts + p];
        v[0] += a * a + b * b + d * d;
        v[1] += a * a - d * d;
        v[2] += a * a + d * d;
        v[3] += a * ha + b * hb + d * hd;
        v[4] += a * ha - d * hd;
    }
    block_reduce_store<5>(v, part);
}

// r = HPhi - mu Phi - lam SzPhi (into complex buffer), sum |r|^2
__global__ void __launch_bounds__(GB) k_gs_resid(long long npts, const double* __restrict__ phi,
                                                 const double* __restrict__ hphi, double mu, double lam,
                                                 double2* __restrict__ r, double* part) {
    double v[1] = {0};
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
        const double sz[3] = {1.0, 0.0, -1.0};
        for (int c = 0; c < 3; ++c) {
            const long long q = c * npts + p;
            const double rv = hphi[q] - mu * phi[q] - lam * sz[c] * phi[q];
            r[q] = cmk<double2>(rv, 0.0);
            v[0] += rv * rv;
        }
    }
    block_reduce_store<1>(v, part);
}

// Phi <- Phi - tau Re(Pr); component masses
__global__ void __launch_bounds__(GB) k_gs_step(long long npts, double* __restrict__ phi, const double2* __restrict__ pr,
                                                double tau, double* part) {
    double v[3] = {0, 0, 0};
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
        for (int c = 0; c < 3; ++c) {
            const long long q = c * npts + p;
            const double x = phi[q] - tau * pr[q].x;
            phi[q] = x;
            v[c] += x * x;
        }
    }
    block_reduce_store<3>(v, part);
}

__global__ void k_gs_scale(long long npts, double* __restrict__ phi, double s1, double s0, double sm) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
        phi[p] *= s1;
        phi[npts + p] *= s0;
        phi[2 * npts + p] *= sm;
    }
}

__global__ void __launch_bounds__(GB) k_vmax(long long n, const double* __restrict__ V, double* part) {
    __shared__ double red[GB / 64];
    double m = -1e300;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        m = fmax(m, V[i]);
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = red[0];
        for (int w = 1; w < GB / 64; ++w) a = fmax(a, red[w]);
        part[blockIdx.x] = a;
    }
}

// normalization factors: s = (1 - M^2) / (a0 + sqrt(a0^2 M^2 + 4 a1 am (1 - M^2)))
bool norm_factors(double a1, double a0, double am, double M, double* s1, double* s0, double* sm) {
    const double s = (1.0 - M * M) / (a0 + std::sqrt(a0 * a0 * M * M + 4.0 * a1 * am * (1.0 - M * M)));
    const double q1 = (1.0 - s * a0 + M) / (2.0 * a1), qm = (1.0 - s * a0 - M) / (2.0 * am);
    if (!(q1 > 0) || !(qm > 0) || !(s >= 0)) return false;
    *s1 = std::sqrt(q1);
    *sm = std::sqrt(qm);
    *s0 = std::sqrt(s);
    return true;
}

}  // namespace

extern "C" bdg_status bdg_ground_state(bdg_ctx* c, const double* phi0_dev, double tol, int max_iter, double* phi_dev,
                                       double mu_out[3], double* residual, int* iters) {
    if (!c) return BDG_EINVAL;
    if (!(tol > 0) || max_iter < 1 || !phi_dev || !mu_out)
        return ctx_fail(c, BDG_EINVAL, "bdg_ground_state: bad arguments");
    const long long npts = c->npts;
    const bdg_problem& pr = c->prob;
    const double M = pr.magnetization, mass = pr.mass;
    double* phi = c->phi;
    double* hphi = nullptr;
    double2* z = nullptr;
    double2* tz = nullptr;
    double* part = nullptr;
    double* sums = nullptr;
    BDG_TRY(ctx_alloc(c, (void**)&hphi, 3 * npts * sizeof(double)));
    BDG_TRY(ctx_alloc(c, (void**)&z, 3 * npts * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&tz, 3 * npts * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&part, 8 * GBLK * sizeof(double)));
    BDG_TRY(ctx_alloc(c, (void**)&sums, 8 * sizeof(double)));
    const int nblk = (int)std::min<long long>(GBLK, (npts + GB - 1) / GB);
    auto finish = [&](bdg_status s) {
        ctx_free(c, hphi);
        ctx_free(c, z);
        ctx_free(c, tz);
        ctx_free(c, part);
        ctx_free(c, sums);
        return s;
    };
    auto reduce = [&](int nq, double* host) -> bdg_status {
        hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(64), 0, c->stream, nq, nblk, (const double*)part, c->hd, sums);
        BDG_HIP(c, hipMemcpyAsync(host, sums, nq * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        BDG_HIP(c, hipStreamSynchronize(c->stream));
        return BDG_OK;
    };
    c->has_gs = false;
    // start
    if (phi0_dev) {
        if (hipMemcpyAsync(phi, phi0_dev, 3 * npts * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
            return finish(hip_check(c, hipGetLastError(), "copy phi0"));
    } else {
        double w1, w0, wm;
        if (pr.beta_s < 0) { w1 = (1 + M) / 2; w0 = std::sqrt((1 - M * M) / 2); wm = (1 - M) / 2; }
        else { w1 = std::sqrt((1 + M) / 2); w0 = 0.0; wm = std::sqrt((1 - M) / 2); }
        hipLaunchKernelGGL(k_gs_init, dim3(nblk), dim3(GB), 0, c->stream, npts, c->n[0], c->n[1], c->dim, c->L[0],
                           c->L[1], c->L[2], c->h[0], c->h[1], c->h[2], w1, w0, wm, phi);
    }
    // alpha = max V + 1
    hipLaunchKernelGGL(k_vmax, dim3(nblk), dim3(GB), 0, c->stream, npts, (const double*)c->V, part);
    std::vector<double> vm(nblk);
    if (hipMemcpyAsync(vm.data(), part, nblk * sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return finish(hip_check(c, hipGetLastError(), "vmax"));
    double vmax = -1e300;
    for (double v : vm) vmax = std::max(vmax, v);
    const double alpha = vmax + 1.0, tau = 1.0;
    // initial normalization
    auto normalize = [&]() -> bdg_status {
        hipLaunchKernelGGL(k_gs_step, dim3(nblk), dim3(GB), 0, c->stream, npts, phi, (const double2*)z, 0.0, part);
        double a[3];
        BDG_TRY(reduce(3, a));
        double s1, s0, sm;
        if (!norm_factors(a[0] / mass, a[1] / mass, a[2] / mass, M, &s1, &s0, &sm))
            return ctx_fail(c, BDG_EBREAKDOWN, "ground state: normalization has no solution");
        hipLaunchKernelGGL(k_gs_scale, dim3(nblk), dim3(GB), 0, c->stream, npts, phi, s1, s0, sm);
        return hip_check(c, hipGetLastError(), "k_gs_scale");
    };
    {
        // k_gs_step with tau = 0 only measures the masses (z is not read when tau = 0)
        if (hipMemsetAsync(z, 0, 3 * npts * sizeof(double2), c->stream) != hipSuccess)
            return finish(BDG_EDEVICE);
        bdg_status s = normalize();
        if (s != BDG_OK) return finish(s);
    }
    double res = INFINITY, mu = 0, lam = 0;
    int it = 0;
    bdg_status st = BDG_ENOCONV;
    for (it = 1; it <= max_iter; ++it) {
        hipLaunchKernelGGL(k_real_to_cplx, dim3(nblk), dim3(GB), 0, c->stream, 3 * npts, (const double*)phi, z);
        bdg_status s = launch_fourier<double>(c, 3, 3, 3 * npts, z, tz, 0, 0.0, nullptr);
        if (s != BDG_OK) return finish(s);
        hipLaunchKernelGGL(k_gs_rhs, dim3(nblk), dim3(GB), 0, c->stream, npts, (const double*)phi,
                           (const double*)c->V, (const double2*)tz, pr.beta_n, pr.beta_s, hphi);
        hipLaunchKernelGGL(k_gs_dots, dim3(nblk), dim3(GB), 0, c->stream, npts, (const double*)phi,
                           (const double*)hphi, part);
        double d[5];
        if ((s = reduce(5, d)) != BDG_OK) return finish(s);
        // least squares [[d0, d1], [d1, d2]] [mu; lam] = [d3; d4]
        const double det = d[0] * d[2] - d[1] * d[1];
        if (std::fabs(det) > 1e-14 * d[0] * d[2]) {
            mu = (d[3] * d[2] - d[1] * d[4]) / det;
            lam = (d[0] * d[4] - d[1] * d[3]) / det;
        } else {
            mu = d[3] / d[0];
            lam = 0.0;
        }
        hipLaunchKernelGGL(k_gs_resid, dim3(nblk), dim3(GB), 0, c->stream, npts, (const double*)phi,
                           (const double*)hphi, mu, lam, z, part);
        double r2;
        if ((s = reduce(1, &r2)) != BDG_OK) return finish(s);
        res = std::sqrt(std::max(r2, 0.0) / mass);
        if (!(res == res)) return finish(ctx_fail(c, BDG_EBREAKDOWN, "ground state: non-finite residual"));
        if (res <= tol) { st = BDG_OK; break; }
        if ((s = launch_fourier<double>(c, 3, 3, 3 * npts, z, tz, 1, alpha, nullptr)) != BDG_OK) return finish(s);
        hipLaunchKernelGGL(k_gs_step, dim3(nblk), dim3(GB), 0, c->stream, npts, phi, (const double2*)tz, tau, part);
        double a[3];
        if ((s = reduce(3, a)) != BDG_OK) return finish(s);
        double s1, s0, sm;
        if (!norm_factors(a[0] / mass, a[1] / mass, a[2] / mass, M, &s1, &s0, &sm))
            return finish(ctx_fail(c, BDG_EBREAKDOWN, "ground state: normalization has no solution"));
        hipLaunchKernelGGL(k_gs_scale, dim3(nblk), dim3(GB), 0, c->stream, npts, phi, s1, s0, sm);
    }
    c->mu[0] = mu + lam;
    c->mu[1] = mu;
    c->mu[2] = mu - lam;
    for (int j = 0; j < 3; ++j) mu_out[j] = c->mu[j];
    if (residual) *residual = res;
    if (iters) *iters = std::min(it, max_iter);
    bdg_status s = build_coefficients(c);
    if (s != BDG_OK) return finish(s);
    if (phi_dev != phi &&
        hipMemcpyAsync(phi_dev, phi, 3 * npts * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return finish(hip_check(c, hipGetLastError(), "copy phi"));
    if (hipStreamSynchronize(c->stream) != hipSuccess) return finish(hip_check(c, hipGetLastError(), "sync"));
    c->has_gs = true;
    c->complex_gs = false;
    if (st != BDG_OK) return finish(ctx_fail(c, BDG_ENOCONV, "ground state: iteration limit reached"));
    return finish(BDG_OK);
}
