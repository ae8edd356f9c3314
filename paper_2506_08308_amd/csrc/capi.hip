// C ABI: context life cycle, argument validation, tables, coefficient fields and the
// standalone operator application (bdg_create, bdg_destroy, bdg_last_error,
// bdg_set_ground_state, bdg_apply, bdg_stats).
#include "common.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

// ------------------------------------------------------------------------------------
// context helpers
// ------------------------------------------------------------------------------------
bdg_status ctx_fail(bdg_ctx* c, bdg_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

bdg_status hip_check(bdg_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return BDG_OK;
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return ctx_fail(c, e == hipErrorOutOfMemory ? BDG_ENOMEM : BDG_EDEVICE, m);
}

// a piece of the caller-provided workspace (context arena mode)
static bdg_status arena_take(bdg_ctx* c, void** p, size_t bytes) {
    const size_t at = (c->arena.used + 255) & ~(size_t)255;
    if (bytes > c->arena.size || at > c->arena.size - bytes) {
        char buf[160];
        snprintf(buf, sizeof buf, "workspace of %zu more bytes exceeds the static scratch of %zu bytes", bytes,
                 c->arena.size);
        return ctx_fail(c, BDG_EINVAL, buf);
    }
    *p = c->arena.base + at;
    c->arena.used = at + bytes;
    return BDG_OK;
}

static bool in_arena(const bdg_ctx* c, const void* p) {
    const char* q = (const char*)p;
    return c->arena.base && q >= c->arena.base && q < c->arena.base + c->arena.size;
}

bdg_status ctx_alloc(bdg_ctx* c, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    if (c->arena.base) return arena_take(c, p, bytes);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        char buf[128];
        snprintf(buf, sizeof buf, "device allocation of %zu bytes failed", bytes);
        return ctx_fail(c, BDG_ENOMEM, buf);
    }
    c->owned.push_back(*p);
    return BDG_OK;
}

void ctx_free(bdg_ctx* c, void* p) {
    if (!p || in_arena(c, p)) return;
    for (size_t i = 0; i < c->owned.size(); ++i)
        if (c->owned[i] == p) {
            c->owned.erase(c->owned.begin() + i);
            break;
        }
    (void)hipFree(p);
}

bdg_status ctx_scratch(bdg_ctx* c, int slot, size_t bytes, void** out) {
    if (c->arena.base) return arena_take(c, out, bytes == 0 ? 16 : bytes);
    DevBuf& b = c->scratch[slot];
    if (b.bytes < bytes) {
        if (b.p) {
            // the stream may still read the old buffer
            BDG_HIP(c, hipStreamSynchronize(c->stream));
            ctx_free(c, b.p);
        }
        b.p = nullptr;
        b.bytes = 0;
        size_t want = bytes + bytes / 4;
        BDG_TRY(ctx_alloc(c, &b.p, want));
        b.bytes = want;
    }
    *out = b.p;
    return BDG_OK;
}

namespace {

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

__global__ void k_check_finite(long long n, const double* __restrict__ v, int* flag) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        if (!isfinite(v[i])) *flag = 1;
}

// Pointwise parts of H_+ and H_- for a real ground state (symmetric 3x3, entries 00 01 02 11 12 22).
// With s_x = sqrt2 phi_0 (phi_1 + phi_-1), s_z = phi_1^2 - phi_-1^2 (s_y = 0 for real Phi),
// S_x Phi = (phi_0, phi_1 + phi_-1, phi_0)/sqrt2, S_z Phi = (phi_1, 0, -phi_-1) and
// K Phi = -i S_y Phi = (-phi_0, phi_1 - phi_-1, phi_0)/sqrt2:
//   H_+ = V - Lambda + beta_n (rho I + 2 Phi Phi^T)
//         + beta_s (S.s + 2 (S_x Phi)(S_x Phi)^T + 2 (S_z Phi)(S_z Phi)^T),
//   H_- = V - Lambda + beta_n rho I + beta_s (S.s + 2 (K Phi)(K Phi)^T).
// Also the pointwise factor of the eigensolver's preconditioner,
//   D = sqrt(ps / (ps + max(V - mu_0, 0))).
__global__ void k_coef(long long npts, const double* __restrict__ V, const double* __restrict__ phi, double mu1,
                       double mu0, double mum, double bn, double bs, double* __restrict__ c64,
                       float* __restrict__ c32, double ps, double* __restrict__ w64, float* __restrict__ w32) {
    const double r2 = 0.70710678118654752440;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts;
         p += (long long)gridDim.x * blockDim.x) {
        const double a = phi[p], b = phi[npts + p], d = phi[2 * npts + p];
        const double rho = a * a + b * b + d * d;
        const double sx = 1.4142135623730950488 * b * (a + d), sz = a * a - d * d;
        const double x0 = r2 * b, x1 = r2 * (a + d), x2 = r2 * b;      // S_x Phi
        const double k0 = -r2 * b, k1 = r2 * (a - d), k2 = r2 * b;     // K Phi
        const double vp = V[p];
        const double ss01 = sx * r2;                                    // (S.s)_01 = (S.s)_12
        double P[6], M[6];
        // H_+
        P[0] = vp - mu1 + bn * (rho + 2 * a * a) + bs * (sz + 2 * x0 * x0 + 2 * a * a);
        P[1] = bn * 2 * a * b + bs * (ss01 + 2 * x0 * x1);
        P[2] = bn * 2 * a * d + bs * (2 * x0 * x2 - 2 * a * d);
        P[3] = vp - mu0 + bn * (rho + 2 * b * b) + bs * (2 * x1 * x1);
        P[4] = bn * 2 * b * d + bs * (ss01 + 2 * x1 * x2);
        P[5] = vp - mum + bn * (rho + 2 * d * d) + bs * (-sz + 2 * x2 * x2 + 2 * d * d);
        // H_-
        M[0] = vp - mu1 + bn * rho + bs * (sz + 2 * k0 * k0);
        M[1] = bs * (ss01 + 2 * k0 * k1);
        M[2] = bs * (2 * k0 * k2);
        M[3] = vp - mu0 + bn * rho + bs * (2 * k1 * k1);
        M[4] = bs * (ss01 + 2 * k1 * k2);
        M[5] = vp - mum + bn * rho + bs * (-sz + 2 * k2 * k2);
        for (int s = 0; s < 6; ++s) {
            c64[s * npts + p] = P[s];
            c64[(6 + s) * npts + p] = M[s];
            c32[s * npts + p] = (float)P[s];
            c32[(6 + s) * npts + p] = (float)M[s];
        }
        const double u = vp - mu0 > 0.0 ? vp - mu0 : 0.0;
        const double dw = sqrt(ps / (ps + u));
        w64[p] = dw;
        w32[p] = (float)dw;
    }
}

// Complex ground state: A = (V - Lambda) I + beta_n (rho I + Phi Phi^H)
// + beta_s (S.s + sum_j (S_j Phi)(S_j Phi)^H) and B = beta_n Phi Phi^T + beta_s sum_j (S_j Phi)(S_j Phi)^T
// (eqs. def_A, def_B with s = Phi^H S Phi), stored as the 21 fields described in common.h.
__device__ __forceinline__ double2 cm(double2 a, double2 b) { return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ double2 cj(double2 a) { return double2{a.x, -a.y}; }

__global__ void k_coef_complex(long long npts, const double* __restrict__ V, const double2* __restrict__ phi,
                               double mu1, double mu0, double mum, double bn, double bs, double* __restrict__ cc,
                               double ps, double* __restrict__ w64, float* __restrict__ w32) {
    const double r2 = 0.70710678118654752440;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts;
         p += (long long)gridDim.x * blockDim.x) {
        const double2 f[3] = {phi[p], phi[npts + p], phi[2 * npts + p]};
        // S_j Phi, j = x, y, z (S_y = i/sqrt2 [[0, -1, 0], [1, 0, -1], [0, 1, 0]])
        double2 v[3][3];
        v[0][0] = double2{r2 * f[1].x, r2 * f[1].y};
        v[0][1] = double2{r2 * (f[0].x + f[2].x), r2 * (f[0].y + f[2].y)};
        v[0][2] = v[0][0];
        v[1][0] = double2{r2 * f[1].y, -r2 * f[1].x};                           // -i b / sqrt2
        v[1][1] = double2{-r2 * (f[0].y - f[2].y), r2 * (f[0].x - f[2].x)};     // i (a - d) / sqrt2
        v[1][2] = double2{-r2 * f[1].y, r2 * f[1].x};                           // i b / sqrt2
        v[2][0] = f[0];
        v[2][1] = double2{0, 0};
        v[2][2] = double2{-f[2].x, -f[2].y};
        double s[3], rho = 0;
        for (int c = 0; c < 3; ++c) rho += f[c].x * f[c].x + f[c].y * f[c].y;
        for (int j = 0; j < 3; ++j) {
            double acc = 0;
            for (int c = 0; c < 3; ++c) acc += f[c].x * v[j][c].x + f[c].y * v[j][c].y;   // Re conj(f) . v
            s[j] = acc;
        }
        const double2 sm = double2{r2 * s[0], -r2 * s[1]};     // (s_x - i s_y) / sqrt2: (S.s)_01 = (S.s)_12
        double2 A[3][3], B[3][3];
        const double lam[3] = {mu1, mu0, mum};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double2 x = cm(f[a], cj(f[b]));
                double2 y = cm(f[a], f[b]);
                double2 av = double2{bn * x.x, bn * x.y}, bv = double2{bn * y.x, bn * y.y};
                for (int j = 0; j < 3; ++j) {
                    const double2 xa = cm(v[j][a], cj(v[j][b])), ya = cm(v[j][a], v[j][b]);
                    av.x += bs * xa.x; av.y += bs * xa.y;
                    bv.x += bs * ya.x; bv.y += bs * ya.y;
                }
                A[a][b] = av;
                B[a][b] = bv;
            }
        for (int a = 0; a < 3; ++a) A[a][a].x += V[p] - lam[a] + bn * rho;
        A[0][0].x += bs * s[2];
        A[2][2].x -= bs * s[2];
        A[0][1].x += bs * sm.x; A[0][1].y += bs * sm.y;
        A[1][2].x += bs * sm.x; A[1][2].y += bs * sm.y;
        double* o = cc + p;
        o[0] = A[0][0].x; o[npts] = A[1][1].x; o[2 * npts] = A[2][2].x;
        o[3 * npts] = A[0][1].x; o[4 * npts] = A[0][1].y;
        o[5 * npts] = A[0][2].x; o[6 * npts] = A[0][2].y;
        o[7 * npts] = A[1][2].x; o[8 * npts] = A[1][2].y;
        const int bi[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
        for (int e = 0; e < 6; ++e) {
            o[(9 + 2 * e) * npts] = B[bi[e][0]][bi[e][1]].x;
            o[(10 + 2 * e) * npts] = B[bi[e][0]][bi[e][1]].y;
        }
        const double u = V[p] - mu0 > 0.0 ? V[p] - mu0 : 0.0;
        const double dw = sqrt(ps / (ps + u));
        w64[p] = dw;
        w32[p] = (float)dw;
    }
}

}  // namespace

bdg_status build_coefficients(bdg_ctx* c) {
    const bdg_problem& pr = c->prob;
    const long long n = c->npts;
    int blocks = (int)std::min<long long>(4096, (n + 255) / 256);
    c->pshift = std::max(0.5 * c->mu[1], 0.5);
    hipLaunchKernelGGL(k_coef, dim3(blocks), dim3(256), 0, c->stream, n, c->V, c->phi, c->mu[0], c->mu[1],
                       c->mu[2], pr.beta_n, pr.beta_s, c->coef64, c->coef32, c->pshift, c->pw64, c->pw32);
    return hip_check(c, hipGetLastError(), "k_coef");
}

extern "C" {

bdg_status bdg_create(const bdg_problem* pr, const double* V_dev, void* hip_stream, bdg_ctx** out) {
    if (!out) return BDG_EINVAL;
    *out = nullptr;
    if (!pr || !V_dev) return BDG_EINVAL;
    if (pr->dim < 1 || pr->dim > 3) return BDG_EINVAL;
    for (int a = 0; a < pr->dim; ++a) {
        if (!is_pow2(pr->n[a]) || pr->n[a] < 8 || pr->n[a] > 1024) return BDG_EINVAL;
        if (!(pr->L[a] > 0) || !std::isfinite(pr->L[a])) return BDG_EINVAL;
    }
    if (!std::isfinite(pr->beta_n) || !std::isfinite(pr->beta_s)) return BDG_EINVAL;
    if (!(pr->mass > 0) || !std::isfinite(pr->mass)) return BDG_EINVAL;
    if (!(pr->magnetization > -1.0 && pr->magnetization < 1.0)) return BDG_EINVAL;
    if (pr->precision != BDG_FP64 && pr->precision != BDG_FP32_APPLY) return BDG_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return BDG_EDEVICE;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return BDG_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return BDG_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return BDG_EDEVICE;

    bdg_ctx* c = new bdg_ctx();
    c->prob = *pr;
    c->stream = (hipStream_t)hip_stream;
    c->device = dev;
    c->ncu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (const char* e = std::getenv("BDG_APPLY_CHUNK_MB")) c->apply_chunk_bytes = (size_t)std::atoll(e) << 20;
    if (const char* e = std::getenv("BDG_APPLY_PLANES")) c->apply_planes = e[0] != '0';
    if (const char* e = std::getenv("BDG_APPLY_PLANES64")) c->apply_planes64 = e[0] != '0';
    if (const char* e = std::getenv("BDG_GRAM_WIDE")) c->gram_wide = e[0] != '0';
    if (const char* e = std::getenv("BDG_GRAM_W8")) c->gram_w8 = std::atoi(e);
    if (const char* e = std::getenv("BDG_JACOBI_SPLIT")) c->jacobi_split = std::max(1, std::min(8, std::atoi(e)));
    if (const char* e = std::getenv("BDG_DEEP_LOADS")) c->deep_loads = e[0] != '0';
    c->dim = pr->dim;
    c->npts = 1;
    c->hd = 1.0;
    for (int a = 0; a < 3; ++a) {
        c->n[a] = a < pr->dim ? pr->n[a] : 1;
        c->L[a] = a < pr->dim ? pr->L[a] : 1.0;
        c->h[a] = a < pr->dim ? 2.0 * pr->L[a] / pr->n[a] : 1.0;
        c->npts *= c->n[a];
        if (a < pr->dim) c->hd *= c->h[a];
    }
    auto fail = [&](bdg_status s) {
        bdg_destroy(c);
        return s;
    };
    const long long n = c->npts;
    if (ctx_alloc(c, (void**)&c->V, n * sizeof(double)) != BDG_OK) return fail(BDG_ENOMEM);
    if (ctx_alloc(c, (void**)&c->phi, 3 * n * sizeof(double)) != BDG_OK) return fail(BDG_ENOMEM);
    if (ctx_alloc(c, (void**)&c->coef64, 12 * n * sizeof(double)) != BDG_OK) return fail(BDG_ENOMEM);
    if (ctx_alloc(c, (void**)&c->coef32, 12 * n * sizeof(float)) != BDG_OK) return fail(BDG_ENOMEM);
    if (ctx_alloc(c, (void**)&c->pw64, n * sizeof(double)) != BDG_OK) return fail(BDG_ENOMEM);
    if (ctx_alloc(c, (void**)&c->pw32, n * sizeof(float)) != BDG_OK) return fail(BDG_ENOMEM);
    if (hipMemcpyAsync(c->V, V_dev, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return fail(BDG_EDEVICE);
    // finiteness of V
    int* flag = nullptr;
    if (ctx_alloc(c, (void**)&flag, sizeof(int)) != BDG_OK) return fail(BDG_ENOMEM);
    int hflag = 0;
    if (hipMemsetAsync(flag, 0, sizeof(int), c->stream) != hipSuccess) return fail(BDG_EDEVICE);
    hipLaunchKernelGGL(k_check_finite, dim3(256), dim3(256), 0, c->stream, n, (const double*)c->V, flag);
    if (hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return fail(BDG_EDEVICE);
    ctx_free(c, flag);
    if (hflag) return fail(BDG_EINVAL);
    // twiddle and kinetic-symbol tables (host float64 libm, rounded for float32)
    for (int a = 0; a < 3; ++a) {
        const int N = c->n[a];
        std::vector<double2> tw(N);
        std::vector<float2> tw32(N);
        std::vector<double> sym(N);
        std::vector<float> sym32(N);
        for (int m = 0; m < N; ++m) {
            const double ang = -2.0 * M_PI * (double)m / (double)N;
            tw[m].x = std::cos(ang);
            tw[m].y = std::sin(ang);
            tw32[m].x = (float)tw[m].x;
            tw32[m].y = (float)tw[m].y;
            const int k = (m < N / 2) ? m : m - N;        // FFT order, Nyquist stored as -N/2
            const double mu = (a < c->dim) ? M_PI * (double)k / c->L[a] : 0.0;
            sym[m] = 0.5 * mu * mu;
            sym32[m] = (float)sym[m];
        }
        if (ctx_alloc(c, (void**)&c->tw64[a], N * sizeof(double2)) != BDG_OK ||
            ctx_alloc(c, (void**)&c->tw32[a], N * sizeof(float2)) != BDG_OK ||
            ctx_alloc(c, (void**)&c->sym64[a], N * sizeof(double)) != BDG_OK ||
            ctx_alloc(c, (void**)&c->sym32[a], N * sizeof(float)) != BDG_OK)
            return fail(BDG_ENOMEM);
        if (hipMemcpy(c->tw64[a], tw.data(), N * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->tw32[a], tw32.data(), N * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->sym64[a], sym.data(), N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->sym32[a], sym32.data(), N * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
            return fail(BDG_EDEVICE);
    }
    *out = c;
    return BDG_OK;
}

void bdg_destroy(bdg_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (void* p : c->owned) (void)hipFree(p);
    c->owned.clear();
    delete c;
}

const char* bdg_last_error(const bdg_ctx* c) {
    if (!c) return "null context";
    return c->err.c_str();
}

bdg_status bdg_set_ground_state(bdg_ctx* c, const double* phi_dev, const double mu[3]) {
    if (!c) return BDG_EINVAL;
    if (!phi_dev || !mu) return ctx_fail(c, BDG_EINVAL, "bdg_set_ground_state: null argument");
    for (int j = 0; j < 3; ++j)
        if (!std::isfinite(mu[j])) return ctx_fail(c, BDG_EINVAL, "bdg_set_ground_state: non-finite mu");
    if (phi_dev != c->phi)
        BDG_HIP(c, hipMemcpyAsync(c->phi, phi_dev, 3 * c->npts * sizeof(double), hipMemcpyDeviceToDevice,
                                  c->stream));
    for (int j = 0; j < 3; ++j) c->mu[j] = mu[j];
    BDG_TRY(build_coefficients(c));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    c->has_gs = true;
    c->complex_gs = false;
    return BDG_OK;
}

bdg_status bdg_set_ground_state_complex(bdg_ctx* c, const void* phi_dev, const double mu[3]) {
    if (!c) return BDG_EINVAL;
    if (!phi_dev || !mu) return ctx_fail(c, BDG_EINVAL, "bdg_set_ground_state_complex: null argument");
    if (c->prob.precision != BDG_FP64)
        return ctx_fail(c, BDG_EINVAL, "bdg_set_ground_state_complex: needs a BDG_FP64 context");
    for (int j = 0; j < 3; ++j)
        if (!std::isfinite(mu[j])) return ctx_fail(c, BDG_EINVAL, "bdg_set_ground_state_complex: non-finite mu");
    const long long n = c->npts;
    if (!c->phic) BDG_TRY(ctx_alloc(c, (void**)&c->phic, 3 * n * sizeof(double2)));
    if (!c->ccoef) BDG_TRY(ctx_alloc(c, (void**)&c->ccoef, 21 * n * sizeof(double)));
    if (phi_dev != c->phic)
        BDG_HIP(c, hipMemcpyAsync(c->phic, phi_dev, 3 * n * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
    for (int j = 0; j < 3; ++j) c->mu[j] = mu[j];
    c->pshift = std::max(0.5 * c->mu[1], 0.5);
    const int blocks = (int)std::min<long long>(4096, (n + 255) / 256);
    const bdg_problem& pr = c->prob;
    hipLaunchKernelGGL(k_coef_complex, dim3(blocks), dim3(256), 0, c->stream, n, c->V, (const double2*)c->phic,
                       c->mu[0], c->mu[1], c->mu[2], pr.beta_n, pr.beta_s, c->ccoef, c->pshift, c->pw64, c->pw32);
    BDG_TRY(hip_check(c, hipGetLastError(), "k_coef_complex"));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    c->has_gs = true;
    c->complex_gs = true;
    return BDG_OK;
}

bdg_status bdg_apply(bdg_ctx* c, int form, int transpose, int nvec, const void* X, void* Y) {
    if (!c) return BDG_EINVAL;
    if (form != BDG_FORM_FG && form != BDG_FORM_UV) return ctx_fail(c, BDG_EINVAL, "bdg_apply: bad form");
    if (transpose != 0 && transpose != 1) return ctx_fail(c, BDG_EINVAL, "bdg_apply: bad transpose flag");
    if (nvec < 0) return ctx_fail(c, BDG_EINVAL, "bdg_apply: nvec < 0");
    if (nvec == 0) return BDG_OK;
    if (!X || !Y) return ctx_fail(c, BDG_EINVAL, "bdg_apply: null pointer");
    if (!c->has_gs) return ctx_fail(c, BDG_ESTATE, "bdg_apply: no ground state set");
    if (c->complex_gs && (form != BDG_FORM_UV || transpose != 0))
        return ctx_fail(c, BDG_EINVAL, "bdg_apply: a complex ground state takes the (u, v) form, no transpose");
    const bool f32 = c->prob.precision == BDG_FP32_APPLY;
    const size_t bytes = (size_t)nvec * 6 * c->npts * (f32 ? sizeof(float2) : sizeof(double2));
    const char* xa = (const char*)X;
    const char* ya = (const char*)Y;
    if (xa < ya + bytes && ya < xa + bytes) return ctx_fail(c, BDG_EINVAL, "bdg_apply: X and Y overlap");
    const long long vs = 6 * c->npts;
    if (f32) {
        BlockRef<const float2> xr{(const float2*)X, (const float2*)X + 3 * c->npts, vs};
        BlockRef<float2> yr{(float2*)Y, (float2*)Y + 3 * c->npts, vs};
        return launch_apply<float>(c, form, transpose, nvec, xr, yr);
    }
    BlockRef<const double2> xr{(const double2*)X, (const double2*)X + 3 * c->npts, vs};
    BlockRef<double2> yr{(double2*)Y, (double2*)Y + 3 * c->npts, vs};
    if (c->complex_gs) return launch_apply_complex(c, 0, nvec, xr, yr);
    return launch_apply<double>(c, form, transpose, nvec, xr, yr);
}

bdg_status bdg_stats(const bdg_ctx* c, double* out, int n_out) {
    if (!c || !out || n_out < 0) return BDG_EINVAL;
    for (int i = 0; i < n_out && i < 10; ++i) out[i] = c->stats[i];
    return BDG_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------
// kernel-level entry points for parity tests (include/bdg_testing.h)
// ------------------------------------------------------------------------------------
#include "../../include/bdg_testing.h"

extern "C" {

bdg_status bdg_test_gram(bdg_ctx* c, long long K, int m1, int m2, const void* A, long long lda, const void* B,
                         long long ldb, double alpha, void* C, int ldc, int hermitian) {
    if (!c || !A || !B || !C || K < 1 || m1 < 1 || m2 < 1 || ldc < m1) return ctx_fail(c, BDG_EINVAL, "bad args");
    if (hermitian && m1 != m2) return ctx_fail(c, BDG_EINVAL, "hermitian needs m1 == m2");
    BDG_TRY(gram<double2, double2>(c, K, m1, m2, (const double2*)A, lda, (const double2*)B, ldb, alpha,
                                   (double2*)C, ldc, hermitian));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    return BDG_OK;
}

bdg_status bdg_test_update(bdg_ctx* c, long long K, int m, const void* S, long long lds, const void* Cm, int ldcm,
                           int nb, double beta, void* Y, long long ldy) {
    if (!c || !S || !Cm || !Y || K < 1 || m < 1 || nb < 1 || ldcm < m) return ctx_fail(c, BDG_EINVAL, "bad args");
    Seg s{S, m};
    BDG_TRY(update(c, K, &s, 1, lds, (const double2*)Cm, ldcm, nb, beta, (double2*)Y, ldy));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    return BDG_OK;
}

bdg_status bdg_test_gram_pair(bdg_ctx* c, long long K, int m1, int m2, const void* A, long long lda, const void* B,
                              long long ldb, double alpha, void* C, int ldc, int symmetric) {
    if (!c || !A || !B || !C || K < 1 || m1 < 1 || m2 < 1 || ldc < 2 * m1) return ctx_fail(c, BDG_EINVAL, "bad args");
    if (symmetric && m1 != m2) return ctx_fail(c, BDG_EINVAL, "symmetric needs m1 == m2");
    Seg a{A, m1}, b{B, m2};
    BDG_TRY(gram_seg_pair(c, K, &a, 1, lda, &b, 1, ldb, alpha, (double2*)C, ldc, symmetric));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    return BDG_OK;
}

bdg_status bdg_test_precond_mixed(bdg_ctx* c, int nvec, void* X32, void* Y64) {
    if (!c || !X32 || !Y64 || nvec < 1) return ctx_fail(c, BDG_EINVAL, "bad args");
    const long long np = c->npts;
    BlockRef<float2> x{(float2*)X32, (float2*)X32 + 3 * np, 6 * np};
    BlockRef<double2> y{(double2*)Y64, (double2*)Y64 + 3 * np, 6 * np};
    BDG_TRY(launch_precond_mixed(c, nvec, x, y));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    return BDG_OK;
}

bdg_status bdg_test_update_pair(bdg_ctx* c, long long K, int m, const void* S, long long lds, const void* Cm, int ldcm,
                                int nb, double beta, void* Y, long long ldy) {
    if (!c || !S || !Cm || !Y || K < 1 || m < 1 || nb < 2 || (nb & 1) || ldcm < 2 * m)
        return ctx_fail(c, BDG_EINVAL, "bad args");
    Seg s{S, m};
    BDG_TRY(update_pair(c, K, &s, 1, lds, (const double2*)Cm, ldcm, 0, nb, beta, (const double2*)Y, ldy, (double2*)Y,
                        ldy));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    return BDG_OK;
}

bdg_status bdg_test_update_pair_fused(bdg_ctx* c, long long K, int m, int mF, const void* S, long long lds,
                                      const void* Cm, int ldcm, int nb, void* Yp, void* Yf, long long ldy) {
    if (!c || !S || !Cm || !Yp || !Yf || K < 1 || m < 1 || nb < 2 || (nb & 1) || nb > 96 || mF < 0 || mF > m ||
        mF % 8 != 0 || ldcm < 2 * m || ldy < K)
        return ctx_fail(c, BDG_EINVAL, "bad args");
    Seg s{S, m};
    BDG_TRY(update_pair_fused(c, K, &s, 1, lds, (const double2*)Cm, ldcm, nb, mF, (double2*)Yp, ldy, (double2*)Yf,
                              ldy));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    return BDG_OK;
}

bdg_status bdg_test_svd(bdg_ctx* c, int rows, int m, void* G, int ldg, void* V, int ldv, void* s) {
    if (!c || !G || !V || !s || m < 1 || m > 512 || rows < 1 || ldg < rows || ldv < m)
        return ctx_fail(c, BDG_EINVAL, "bad args");
    BDG_TRY(small_svd(c, rows, m, (double2*)G, ldg, (double2*)V, ldv, (double*)s));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    return BDG_OK;
}

bdg_status bdg_test_svd_real(bdg_ctx* c, int rows, int m, void* G, int ldg, void* V, int ldv, void* s) {
    if (!c || !G || !V || !s || m < 1 || m > 512 || rows < 1 || ldg < rows || ldv < m)
        return ctx_fail(c, BDG_EINVAL, "bad args");
    BDG_TRY(small_svd(c, rows, m, (double2*)G, ldg, (double2*)V, ldv, (double*)s, 1e-13, true));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    return BDG_OK;
}

bdg_status bdg_test_cholesky(bdg_ctx* c, int m, void* A, int lda) {
    if (!c || !A || m < 1 || m > 512 || lda < m) return ctx_fail(c, BDG_EINVAL, "bad args");
    int* info = nullptr;
    BDG_TRY(ctx_alloc(c, (void**)&info, sizeof(int)));
    bdg_status st = small_cholesky(c, m, (double2*)A, lda, info);
    int h = 0;
    if (st == BDG_OK) {
        if (hipMemcpy(&h, info, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) st = BDG_EDEVICE;
    }
    ctx_free(c, info);
    if (st != BDG_OK) return st;
    return h ? ctx_fail(c, BDG_EBREAKDOWN, "not positive definite") : BDG_OK;
}

bdg_status bdg_test_pchol(bdg_ctx* c, int m, void* A, int lda, double rtol, void* R, int* rank) {
    if (!c || !A || !R || !rank || m < 1 || m > 512 || lda < m) return ctx_fail(c, BDG_EINVAL, "bad args");
    int* d = nullptr;
    BDG_TRY(ctx_alloc(c, (void**)&d, sizeof(int)));
    bdg_status st = small_pchol_orth(c, m, (double2*)A, lda, rtol, (double2*)R, d);
    if (st == BDG_OK && hipMemcpy(rank, d, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) st = BDG_EDEVICE;
    ctx_free(c, d);
    return st;
}

bdg_status bdg_test_plu(bdg_ctx* c, int p, int q, void* B, int ldb, double tol, void* Cf, void* Cg, int* rank) {
    if (!c || !B || !Cf || !Cg || !rank || p < 1 || q < 1 || p > 512 || q > 512 || ldb < p)
        return ctx_fail(c, BDG_EINVAL, "bad args");
    int* d = nullptr;
    BDG_TRY(ctx_alloc(c, (void**)&d, sizeof(int)));
    bdg_status st = small_plu_biorth(c, p, q, (double2*)B, ldb, tol, (double2*)Cf, (double2*)Cg, d);
    if (st == BDG_OK && hipMemcpy(rank, d, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) st = BDG_EDEVICE;
    ctx_free(c, d);
    return st;
}

}  // extern "C"
