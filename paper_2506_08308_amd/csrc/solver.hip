// Structure-preserving block subspace iteration for the linear-response form of the BdG
// problem (Section 3.2):  [[0, H_-], [H_+, 0]] [f; g] = omega [f; g].
//
// The paper solves it with its bi-orthogonal structure-preserving (BOSP) iteration and
// names its ingredients (bi-orthogonal Gram-Schmidt, use of the generalized nullspace of
// Section 2.3, LAPACK for the projected problem) without printing its steps.  This
// implementation is a locally optimal block iteration of the Bai-Li family:
//   basis      S_f = [F, W_f, P_f], S_g = [G, W_g, P_g] and their images H_+ S_f, H_- S_g;
//   residual   R = H_+ F - G diag(w) (f-direction), H_- G - F diag(w) (g-direction);
//   correction W = D (|k|^2/2 + sigma)^-1 D R (kinetic-potential preconditioner, D^2 =
//              sigma / (sigma + max(V - mu_0, 0)), sigma = max(mu_0 / 2, 1/2)) for the active
//              columns only (res above max(tol, 100 eps ||H|| / |w|), the float64 floor
//              of the relative residual; converged columns are soft-locked), projected off
//              the generalized nullspace (f orthogonal to ns(H_-), g orthogonal to
//              ns(H_+) + Jordan partners);
//   projection each basis is made orthonormal on its own by a pivoted Cholesky of its
//              diagonally scaled Gram matrix (rank-revealing: S R_f, S R_g), the pairing
//              matrix B = R_g^H S_g^H S_f R_f of the two orthonormal bases is
//              bi-orthogonalized by an LU with complete pivoting (the modified Gram-Schmidt
//              bi-orthogonalization in factored form: C_f = R_f P_c^T [U11^-1; 0],
//              C_g = R_g P_r^T [L11^-H; 0], C_g^H B_r C_f = I), and the
//              projected problem K b = w a, M a = w b (M = C_f^H S_f^H H_+ S_f C_f,
//              K = C_g^H S_g^H H_- S_g C_g) is solved through the Cholesky factors
//              M = L_M L_M^H, K = L_K L_K^H and the SVD L_K^H L_M = U_G diag(w) V_G^H:
//              a = L_K u, b = L_M v;
//   update     P <- [W, P] a_{W,P} (and images), then F <- F a_F + P, G likewise with b;
//              W and P keep their raw scale, their unit-column scaling enters the Gram
//              matrices and the coefficient rows.  With float64 images, H P is recomputed
//              from P before each projection (the recurrence image of the short step P
//              loses relative accuracy by the inverse convergence factor per iteration).
// For a real ground state H_+ and H_- are real, so the eigenvectors can be taken real and the
// iteration runs on real vectors, two to a complex column (paired form: real part and
// imaginary part).  The FFT apply and the preconditioner act on both halves of a complex
// column at once; Gram matrices and updates treat the halves as separate real columns, so a
// block of b real vectors costs the MFMA work of b / 2 complex ones in both (a complex Gram of
// m columns needs 4 m^2 real products per row, the real Gram of m columns m^2).
// Gram matrices and updates run on the FP64 matrix cores; the projected problems on the
// device in FP64; the host only reads back residual norms and small singular values.
#include "common.h"

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

namespace {

// BDG_DEBUG=1 prints per-iteration diagnostics of the subspace iteration to stderr
bool debug_on() {
    static int v = -1;
    if (v < 0) {
        const char* e = std::getenv("BDG_DEBUG");
        v = (e && e[0] && e[0] != '0') ? 1 : 0;
    }
    return v == 1;
}

// the basis update: one pass in both phases (2, the default); BDG_UPDATE_FUSE=1 keeps the
// two launches in the float32 phase, 0 everywhere
int update_fuse_mode() {
    static const int v = [] {
        const char* e = std::getenv("BDG_UPDATE_FUSE");
        return e ? std::atoi(e) : 2;
    }();
    return v;
}

// runs a callable when the scope ends (workspace release on every return path)
template <typename Fn> struct Defer {
    Fn fn;
    ~Defer() { fn(); }
};
template <typename Fn> Defer<Fn> defer(Fn fn) { return Defer<Fn>{fn}; }

// A(p, q) = A(q, p) for r0 <= p < m, q = blockIdx.y < r0: the first r0 rows of a symmetric
// m x m matrix (ld lda) copied into its first r0 columns below them
__global__ void k_small_mirror_rows(int m, int r0, double2* A, int lda) {
    const int p = r0 + blockIdx.x * blockDim.x + threadIdx.x, q = blockIdx.y;
    if (p >= m) return;
    A[(long long)q * lda + p] = A[(long long)p * lda + q];
}

// Y(:, t) = X(:, idx[t]) for t < gridDim.y; X and Y must not overlap
__global__ void k_cols_gather(long long K, const double2* __restrict__ X, long long ldx, const int* __restrict__ idx,
                              double2* __restrict__ Y, long long ldy) {
    const int t = blockIdx.y;
    const long long j = idx[t];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (long long)gridDim.x * blockDim.x)
        Y[t * ldy + i] = X[j * ldx + i];
}

__global__ void k_cols_scale(long long K, int ncols, double2* __restrict__ X, long long ldx, const double* __restrict__ s,
                             int inv_sqrt) {
    const int j = blockIdx.y;
    double f = s[j];
    if (inv_sqrt) f = f > 0 ? 1.0 / sqrt(f) : 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (long long)gridDim.x * blockDim.x) {
        double2 a = X[j * ldx + i];
        X[j * ldx + i] = cmk<double2>(a.x * f, a.y * f);
    }
}

// Y += alpha X (complex alpha), single column
__global__ void k_axpy(long long K, double2 alpha, const double2* __restrict__ X, double2* __restrict__ Y) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (long long)gridDim.x * blockDim.x) {
        double2 x = X[i], y = Y[i];
        Y[i] = cmk<double2>(y.x + alpha.x * x.x - alpha.y * x.y, y.y + alpha.x * x.y + alpha.y * x.x);
    }
}

// P = Z + beta P
__global__ void k_xpby(long long K, const double2* __restrict__ Z, double2 beta, double2* __restrict__ P) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (long long)gridDim.x * blockDim.x) {
        double2 z = Z[i], p = P[i];
        P[i] = cmk<double2>(z.x + beta.x * p.x - beta.y * p.y, z.y + beta.x * p.y + beta.y * p.x);
    }
}

// generators of the nullspaces (Section 2.3): Phi, S_z Phi, S_x Phi, K Phi (K = -i S_y), complex
__global__ void k_candidates(long long npts, const double* __restrict__ phi, double2* __restrict__ out) {
    const double r2 = 0.70710678118654752440;
    const long long nh = 3 * npts;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
        const double a = phi[p], b = phi[npts + p], d = phi[2 * npts + p];
        const double v[4][3] = {{a, b, d}, {a, 0.0, -d}, {r2 * b, r2 * (a + d), r2 * b}, {-r2 * b, r2 * (a - d), r2 * b}};
        for (int c = 0; c < 4; ++c)
            for (int s = 0; s < 3; ++s) out[c * nh + s * npts + p] = cmk<double2>(v[c][s], 0.0);
    }
}

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

// complex standard normal (re + i im)/sqrt2 from a counter-based generator (Box-Muller)
__global__ void k_randn(long long n, unsigned long long seed, double2* __restrict__ out) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        unsigned long long a = splitmix64(seed * 0x632BE59BD9B4E019ULL + 2 * (unsigned long long)i);
        unsigned long long b = splitmix64(seed * 0x632BE59BD9B4E019ULL + 2 * (unsigned long long)i + 1);
        const double u1 = ((a >> 11) + 1) * (1.0 / 9007199254740993.0);
        const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);
        const double r = sqrt(-2.0 * log(u1));
        double s, co;
        sincos(2.0 * M_PI * u2, &s, &co);
        out[i] = cmk<double2>(r * co * 0.70710678118654752440, r * s * 0.70710678118654752440);
    }
}

// small matrices: A(:, j) *= s_j^pw (s_j <= 0 -> 0)
__global__ void k_small_colpow(int rows, int cols, double2* A, int lda, const double* __restrict__ s, double pw) {
    const int j = blockIdx.x;
    if (j >= cols) return;
    const double sj = s[j];
    const double f = sj > 0 ? pow(sj, pw) : 0.0;
    for (int i = threadIdx.x; i < rows; i += blockDim.x) {
        double2 a = A[(long long)j * lda + i];
        A[(long long)j * lda + i] = cmk<double2>(a.x * f, a.y * f);
    }
}

// out(:, t) = A(:, idx[t]) * scale[t]
__global__ void k_small_gather(int rows, int nsel, const double2* __restrict__ A, int lda, const int* __restrict__ idx,
                               const double* __restrict__ scale, double2* __restrict__ out, int ldo) {
    const int t = blockIdx.x;
    if (t >= nsel) return;
    const int j = idx[t];
    const double f = scale[t];
    for (int i = threadIdx.x; i < rows; i += blockDim.x) {
        double2 a = A[(long long)j * lda + i];
        out[(long long)t * ldo + i] = cmk<double2>(a.x * f, a.y * f);
    }
}

__global__ void k_small_herm(int m, double2* A, int lda) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= m || j >= m || i > j) return;
    double2 a = A[(long long)j * lda + i], b = A[(long long)i * lda + j];
    const double2 h = cmk<double2>(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    A[(long long)j * lda + i] = h;
    A[(long long)i * lda + j] = cmk<double2>(h.x, -h.y);
}

__global__ void k_small_copy(int rows, int cols, const double2* __restrict__ A, int lda, double2* __restrict__ B, int ldb) {
    const int j = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += gridDim.x * blockDim.x)
        B[(long long)j * ldb + i] = A[(long long)j * lda + i];
}

// A(:, j) = 0 for j0 <= j < cols
__global__ void k_small_zero_cols(int rows, int j0, double2* A, int lda) {
    const int j = j0 + blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += gridDim.x * blockDim.x)
        A[(long long)j * lda + i] = double2{0.0, 0.0};
}

// ---------------------------------------------------------------------------------------
// Paired real form (real ground states): the operator is real, so the iteration runs on real
// trial vectors, two to a complex column (real column 2 J = real part of complex column J,
// 2 J + 1 = its imaginary part).  The FFT apply acts on both at once (H (a + i b) = H a + i H b
// for real H); the Gram matrices and updates take the parts as separate real columns.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double pget(const double2* X, long long ld, int j, long long i) {
    const double2 v = X[(long long)(j >> 1) * ld + i];
    return (j & 1) ? v.y : v.x;
}

// 1 / sqrt(sq) (0 for sq <= 0): the unit-column factor from a squared norm
__device__ __forceinline__ double unit_scale(double sq) { return sq > 0.0 ? 1.0 / sqrt(sq) : 0.0; }

// complex output column T of Z holds real columns 2 T, 2 T + 1:
// Z_r(t) = (X_r(j) - w[j] Y_r(j)) / sqrt(sq[j]) with j = idx[t], t < 2 gridDim.y; sq holds the
// squared norms of those differences, so every output column has unit norm.  Two real vectors
// share one complex FFT downstream, whose rounding is relative to the larger of the pair: a
// column kept at its raw (possibly tiny) scale would take the rounding of its partner.
__global__ void k_pair_axmy_idx(long long K, const double2* __restrict__ X, const double2* __restrict__ Y, long long ld,
                                const double* __restrict__ w, const int* __restrict__ idx,
                                const double* __restrict__ sq, double2* __restrict__ Z, long long ldz) {
    const int T = blockIdx.y;
    const int j0 = idx[2 * T], j1 = idx[2 * T + 1];
    const double s0 = w[j0], s1 = w[j1];
    const double c0 = unit_scale(sq[j0]), c1 = unit_scale(sq[j1]);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (long long)gridDim.x * blockDim.x)
        Z[T * ldz + i] = cmk<double2>(c0 * (pget(X, ld, j0, i) - s0 * pget(Y, ld, j0, i)),
                                      c1 * (pget(X, ld, j1, i) - s1 * pget(Y, ld, j1, i)));
}

// the same in float32 output (the mixed form's correction block)
__global__ void k_pair_axmy_idx32(long long K, const double2* __restrict__ X, const double2* __restrict__ Y,
                                  long long ld, const double* __restrict__ w, const int* __restrict__ idx,
                                  const double* __restrict__ sq, float2* __restrict__ Z, long long ldz) {
    const int T = blockIdx.y;
    const int j0 = idx[2 * T], j1 = idx[2 * T + 1];
    const double s0 = w[j0], s1 = w[j1];
    const double c0 = unit_scale(sq[j0]), c1 = unit_scale(sq[j1]);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (long long)gridDim.x * blockDim.x)
        Z[T * ldz + i] = cmk<float2>((float)(c0 * (pget(X, ld, j0, i) - s0 * pget(Y, ld, j0, i))),
                                     (float)(c1 * (pget(X, ld, j1, i) - s1 * pget(Y, ld, j1, i))));
}

// X_r(t) *= 1 / sqrt(sq[t]) for the 2 gridDim.y real columns of gridDim.y complex columns
__global__ void k_pair_unit_cols(long long K, double2* __restrict__ X, long long ld, const double* __restrict__ sq) {
    const int T = blockIdx.y;
    const double c0 = unit_scale(sq[2 * T]), c1 = unit_scale(sq[2 * T + 1]);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (long long)gridDim.x * blockDim.x) {
        const double2 v = X[T * ld + i];
        X[T * ld + i] = cmk<double2>(c0 * v.x, c1 * v.y);
    }
}

// k_pair_unit_cols followed by the float32 copy in one pass: X scaled in place, Y = float(X)
__global__ void k_pair_unit_to32(long long K, double2* __restrict__ X, long long ld, const double* __restrict__ sq,
                                 float2* __restrict__ Y, long long ldy) {
    const int T = blockIdx.y;
    const double c0 = unit_scale(sq[2 * T]), c1 = unit_scale(sq[2 * T + 1]);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (long long)gridDim.x * blockDim.x) {
        const double2 v = X[T * ld + i];
        const double2 u = cmk<double2>(c0 * v.x, c1 * v.y);
        X[T * ld + i] = u;
        Y[T * ldy + i] = cmk<float2>((float)u.x, (float)u.y);
    }
}

// Y_r(t) = X_r(idx[t]) for t < 2 gridDim.y; X and Y must not overlap
__global__ void k_pair_gather(long long K, const double2* __restrict__ X, long long ldx, const int* __restrict__ idx,
                              double2* __restrict__ Y, long long ldy) {
    const int T = blockIdx.y;
    const int j0 = idx[2 * T], j1 = idx[2 * T + 1];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (long long)gridDim.x * blockDim.x)
        Y[T * ldy + i] = cmk<double2>(pget(X, ldx, j0, i), pget(X, ldx, j1, i));
}

// real start columns from a complex start block in (f, g) form (vector j at X0 + 2 j nh):
// real column j = real part plus imaginary part of vector j, for j < nvec
__global__ void k_pair_start(long long nh, int nvec, const double2* __restrict__ X0, double2* __restrict__ F,
                             double2* __restrict__ G) {
    const int T = blockIdx.y;
    const int j0 = 2 * T, j1 = 2 * T + 1;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nh; i += (long long)gridDim.x * blockDim.x) {
        double2 f = F[T * nh + i], g = G[T * nh + i];
        if (j0 < nvec) {
            const double2 a = X0[(long long)j0 * 2 * nh + i], b = X0[(long long)j0 * 2 * nh + nh + i];
            f.x = a.x + a.y;
            g.x = b.x + b.y;
        }
        if (j1 < nvec) {
            const double2 a = X0[(long long)j1 * 2 * nh + i], b = X0[(long long)j1 * 2 * nh + nh + i];
            f.y = a.x + a.y;
            g.y = b.x + b.y;
        }
        F[T * nh + i] = f;
        G[T * nh + i] = g;
    }
}

// (u, v) = scale_j (f_j + g_j, f_j - g_j) for the real columns j < ncols, written as complex
// vectors with zero imaginary parts
__global__ void k_pair_make_uv(long long nh, int ncols, const double2* __restrict__ F, const double2* __restrict__ G,
                               const double* __restrict__ scale, double2* __restrict__ UV) {
    const int j = blockIdx.y;
    const double s = scale[j];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nh; i += (long long)gridDim.x * blockDim.x) {
        const double f = pget(F, nh, j, i), g = pget(G, nh, j, i);
        UV[j * 2 * nh + i] = cmk<double2>(s * (f + g), 0.0);
        UV[j * 2 * nh + nh + i] = cmk<double2>(s * (f - g), 0.0);
    }
}

dim3 grid_cols(long long K, int ncols) {
    long long bx = (K + 255) / 256;
    if (bx > 1024) bx = 1024;
    return dim3((unsigned)bx, (unsigned)ncols);
}

// ---------------------------------------------------------------------------------------
// Host-side helpers
// ---------------------------------------------------------------------------------------
// max over grid points of the row sums |H_+(x)|, |H_-(x)| of the pointwise 3x3 blocks (12
// fields: the symmetric 00, 01, 02, 11, 12, 22 entries of H_+ then of H_-); one partial per block
__global__ void __launch_bounds__(256) k_coef_bound(long long npts, const double* __restrict__ coef,
                                                    double* __restrict__ part) {
    __shared__ double red[4];
    double mx = 0;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double* S = coef + (long long)6 * h * npts + p;
            const double a00 = fabs(S[0]), a01 = fabs(S[npts]), a02 = fabs(S[2 * npts]);
            const double a11 = fabs(S[3 * npts]), a12 = fabs(S[4 * npts]), a22 = fabs(S[5 * npts]);
            mx = fmax(mx, fmax(a00 + a01 + a02, fmax(a01 + a11 + a12, a02 + a12 + a22)));
        }
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

struct Small {
    int cap = 0;                 // max dimension
    double2* buf[14] = {};
    double* s[4] = {};
    int* info = nullptr;
    int* idx = nullptr;
    double* dscale = nullptr;
};

bdg_status small_alloc(bdg_ctx* c, Small& w, int cap) {
    w.cap = cap;
    for (int i = 0; i < 14; ++i) BDG_TRY(ctx_alloc(c, (void**)&w.buf[i], (size_t)cap * cap * sizeof(double2)));
    for (int i = 0; i < 4; ++i) BDG_TRY(ctx_alloc(c, (void**)&w.s[i], (size_t)cap * sizeof(double)));
    BDG_TRY(ctx_alloc(c, (void**)&w.info, 4 * sizeof(int)));
    BDG_TRY(ctx_alloc(c, (void**)&w.idx, (size_t)cap * sizeof(int)));
    BDG_TRY(ctx_alloc(c, (void**)&w.dscale, 2 * (size_t)cap * sizeof(double)));
    return BDG_OK;
}
void small_free(bdg_ctx* c, Small& w) {
    for (int i = 0; i < 14; ++i) ctx_free(c, w.buf[i]);
    for (int i = 0; i < 4; ++i) ctx_free(c, w.s[i]);
    ctx_free(c, w.info);
    ctx_free(c, w.idx);
    ctx_free(c, w.dscale);
    w = Small{};
}

const double2 ONE = {1.0, 0.0}, ZERO = {0.0, 0.0};

bdg_status d2h(bdg_ctx* c, void* dst, const void* src, size_t bytes) {
    BDG_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    return BDG_OK;
}
bdg_status h2d(bdg_ctx* c, void* dst, const void* src, size_t bytes) {
    BDG_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    return BDG_OK;
}

bdg_status small_copy(bdg_ctx* c, int rows, int cols, const double2* A, int lda, double2* B, int ldb) {
    if (rows <= 0 || cols <= 0) return BDG_OK;
    hipLaunchKernelGGL(k_small_copy, dim3((unsigned)((rows + 255) / 256), (unsigned)cols), dim3(256), 0, c->stream,
                       rows, cols, A, lda, B, ldb);
    return hip_check(c, hipGetLastError(), "k_small_copy");
}

bdg_status small_colpow(bdg_ctx* c, int rows, int cols, double2* A, int lda, const double* s, double pw) {
    if (rows <= 0 || cols <= 0) return BDG_OK;
    hipLaunchKernelGGL(k_small_colpow, dim3((unsigned)cols), dim3(256), 0, c->stream, rows, cols, A, lda, s, pw);
    return hip_check(c, hipGetLastError(), "k_small_colpow");
}

// Projected problem (see file header).  Inputs m x m (ld m): Gf, Gg, Br, Mr, Kr.  Outputs
// acoef, bcoef (m x nb, ld m) and omega (host, ascending).  Returns BDG_EBREAKDOWN when the
// usable rank is below nb or a projected matrix is not numerically positive definite.
bdg_status rr_once(bdg_ctx* c, Small& w, int m, int nb, const double2* Gf, const double2* Gg,
                         const double2* Br, const double2* Mr, const double2* Kr, double2* acoef, double2* bcoef,
                         std::vector<double>& omega, double rtol, double eps) {
    double2* T = w.buf[5];
    double2* Rf = w.buf[6];
    double2* Rg = w.buf[7];
    double2* B = w.buf[8];
    double2* V3 = w.buf[9];
    double2* Cf = w.buf[10];
    double2* Cg = w.buf[11];
    double2* X1 = w.buf[12];
    double2* X2 = w.buf[13];
    // orthonormal bases of the two spaces (pivoted Cholesky of the scaled Gram matrices)
    BDG_TRY(small_copy(c, m, m, Gf, m, T, m));
    BDG_TRY(small_copy(c, m, m, Gg, m, B, m));
    BDG_TRY(small_pchol_orth2(c, m, T, B, m, rtol, Rf, Rg, w.info + 2, w.info + 3));
    int rk[2];
    BDG_TRY(d2h(c, rk, w.info + 2, 2 * sizeof(int)));
    const int rf = rk[0], rg = rk[1];
    if (rf < nb || rg < nb) return ctx_fail(c, BDG_EBREAKDOWN, "basis rank below block size");
    // pairing matrix of the orthonormal bases B = Rg^H Br Rf (rg x rf), bi-orthogonalized by
    // LU with complete pivoting: Cg'^H B Cf' = I_r
    BDG_TRY(small_gemm(c, 0, 0, m, rf, m, ONE, Br, m, Rf, m, ZERO, T, m));
    BDG_TRY(small_gemm(c, 1, 0, rg, rf, m, ONE, Rg, m, T, m, ZERO, B, m));
    BDG_TRY(small_plu_biorth(c, rg, rf, B, m, eps, X1, X2, w.info + 2));
    int r = 0;
    BDG_TRY(d2h(c, &r, w.info + 2, sizeof(int)));
    if (r < nb) return ctx_fail(c, BDG_EBREAKDOWN, "bi-orthogonal rank below block size");
    // Cf = Rf Cf' (m x r), Cg = Rg Cg' (m x r)
    BDG_TRY(small_gemm(c, 0, 0, m, r, rf, ONE, Rf, m, X1, rf, ZERO, Cf, m));
    BDG_TRY(small_gemm(c, 0, 0, m, r, rg, ONE, Rg, m, X2, rg, ZERO, Cg, m));
    // Mt = Cf^H Mr Cf -> X1 ; Kt = Cg^H Kr Cg -> X2
    BDG_TRY(small_gemm(c, 0, 0, m, r, m, ONE, Mr, m, Cf, m, ZERO, T, m));
    BDG_TRY(small_gemm(c, 1, 0, r, r, m, ONE, Cf, m, T, m, ZERO, X1, m));
    BDG_TRY(small_gemm(c, 0, 0, m, r, m, ONE, Kr, m, Cg, m, ZERO, T, m));
    BDG_TRY(small_gemm(c, 1, 0, r, r, m, ONE, Cg, m, T, m, ZERO, X2, m));
    hipLaunchKernelGGL(k_small_herm, dim3((unsigned)((r + 127) / 128), (unsigned)r), dim3(128), 0, c->stream, r, X1, m);
    hipLaunchKernelGGL(k_small_herm, dim3((unsigned)((r + 127) / 128), (unsigned)r), dim3(128), 0, c->stream, r, X2, m);
    BDG_TRY(small_cholesky2(c, r, X1, X2, m, w.info, w.info + 1));
    // G = L_K^H L_M -> B ; SVD -> V3, s[3]
    BDG_TRY(small_gemm(c, 1, 0, r, r, r, ONE, X2, m, X1, m, ZERO, B, m));
    BDG_TRY(small_svd(c, r, r, B, m, V3, m, w.s[3], 1e-13, true));
    int info[2];
    std::vector<double> s4(r);
    BDG_TRY(d2h(c, info, w.info, 2 * sizeof(int)));
    if (debug_on())
        fprintf(stderr, "[bdg rr] m=%d rf=%d rg=%d r=%d chol=(%d,%d) rtol=%.1e eps=%.1e\n", m, rf, rg, r, info[0],
                info[1], rtol, eps);
    if (info[0] || info[1]) return ctx_fail(c, BDG_EBREAKDOWN, "projected matrix not positive definite");
    BDG_TRY(d2h(c, s4.data(), w.s[3], r * sizeof(double)));
    // the nb smallest singular values, ascending
    std::vector<int> idx(nb);
    std::vector<double> scl(2 * nb);
    omega.assign(nb, 0.0);
    for (int t = 0; t < nb; ++t) {
        const int j = r - 1 - t;
        idx[t] = j;
        const double om = s4[j];
        if (!(om > 0)) return ctx_fail(c, BDG_EBREAKDOWN, "zero projected frequency");
        omega[t] = om;
        scl[t] = 1.0 / (om * std::sqrt(4.0 * om));      // u = G col / sigma, times 1/sqrt(4 w)
        scl[nb + t] = 1.0 / std::sqrt(4.0 * om);
    }
    BDG_TRY(h2d(c, w.idx, idx.data(), nb * sizeof(int)));
    BDG_TRY(h2d(c, w.dscale, scl.data(), 2 * nb * sizeof(double)));
    // A1 = Cf L_K (m x r) -> T ; a = A1 Gsel
    BDG_TRY(small_gemm(c, 0, 0, m, r, r, ONE, Cf, m, X2, m, ZERO, T, m));
    hipLaunchKernelGGL(k_small_gather, dim3((unsigned)nb), dim3(256), 0, c->stream, r, nb, (const double2*)B, m,
                       (const int*)w.idx, (const double*)w.dscale, Rf, m);
    BDG_TRY(small_gemm(c, 0, 0, m, nb, r, ONE, T, m, Rf, m, ZERO, acoef, m));
    // B1 = Cg L_M -> T ; b = B1 Vsel
    BDG_TRY(small_gemm(c, 0, 0, m, r, r, ONE, Cg, m, X1, m, ZERO, T, m));
    hipLaunchKernelGGL(k_small_gather, dim3((unsigned)nb), dim3(256), 0, c->stream, r, nb, (const double2*)V3, m,
                       (const int*)w.idx, (const double*)(w.dscale + nb), Rg, m);
    BDG_TRY(small_gemm(c, 0, 0, m, nb, r, ONE, T, m, Rg, m, ZERO, bcoef, m));
    return hip_check(c, hipGetLastError(), "rayleigh_ritz");
}

// rr_once with escalating cut-offs: rounding in the projected matrices can make them
// indefinite along nearly dependent directions; dropping those directions (larger rtol,
// eps) restores definiteness without changing the spanned space's useful part.
bdg_status rayleigh_ritz(bdg_ctx* c, Small& w, int m, int nb, const double2* Gf, const double2* Gg,
                         const double2* Br, const double2* Mr, const double2* Kr, double2* acoef, double2* bcoef,
                         std::vector<double>& omega, double rtol, double eps) {
    bdg_status st = BDG_OK;
    for (int attempt = 0; attempt < 4; ++attempt) {
        st = rr_once(c, w, m, nb, Gf, Gg, Br, Mr, Kr, acoef, bcoef, omega, rtol, eps);
        if (st != BDG_EBREAKDOWN) return st;
        rtol *= 100.0;
        eps *= 100.0;
    }
    return st;
}

// ---------------------------------------------------------------------------------------
// Block storage of the iteration: four arrays (S_f, S_g, H_+ S_f, H_- S_g) of four slots of
// nb columns (nh complex each); three slots hold F, W, P and one is free for the update.
// ---------------------------------------------------------------------------------------
struct Basis {
    long long nh = 0;
    int nb = 0;
    double2* arr[4] = {};
    int slotF = 0, slotW = 1, slotP = -1, slotFree = 2, slotFree2 = 3;
    double2* col(int a, int slot) const { return arr[a] + (long long)slot * nb * nh; }
};
enum { SF = 0, SG = 1, HSF = 2, HSG = 3 };

// images of a block: [H_- g; H_+ f] for columns f (arr SF slot) and g (arr SG slot)
bdg_status apply64(bdg_ctx* c, int ncols, const double2* f, const double2* g, long long nh, double2* Hf,
                   double2* Hg) {
    BlockRef<const double2> X{f, g, nh};
    BlockRef<double2> Y{Hg, Hf, nh};
    return launch_apply<double>(c, BDG_FORM_FG, 0, ncols, X, Y);
}

// X (nh x ncols) -= Q (Q^H X h^d) with Q orthonormal (nh x q)
bdg_status project_out(bdg_ctx* c, Small& w, long long nh, const double2* Q, int q, double2* X, int ncols) {
    if (q == 0 || ncols == 0) return BDG_OK;
    double2* Cq = w.buf[4];
    BDG_TRY(gram<double2, double2>(c, nh, q, ncols, Q, nh, X, nh, -c->hd, Cq, q, 0));
    Seg s{Q, q};
    return update(c, nh, &s, 1, nh, Cq, q, ncols, 1.0, X, nh);
}

// orthonormal basis (nh x r) of the columns of X (nh x p) into Out; rank by rtol on the Gram
bdg_status orthonormalize(bdg_ctx* c, Small& w, long long nh, const double2* X, int p, double2* Out, double rtol,
                          int* r_out) {
    *r_out = 0;
    if (p == 0) return BDG_OK;
    BDG_TRY(gram<double2, double2>(c, nh, p, p, X, nh, X, nh, c->hd, w.buf[0], p, 1));
    int r = 0;
    BDG_TRY(small_pchol_orth(c, p, w.buf[0], p, rtol, w.buf[2], w.info + 2));
    BDG_TRY(d2h(c, &r, w.info + 2, sizeof(int)));
    Seg s{X, p};
    BDG_TRY(update(c, nh, &s, 1, nh, w.buf[2], p, r, 0.0, Out, nh));
    *r_out = r;
    return BDG_OK;
}

double host_dot_re(bdg_ctx* c, Small& w, long long nh, const double2* a, const double2* b, bdg_status* st) {
    double2 v{0, 0};
    *st = gram<double2, double2>(c, nh, 1, 1, a, nh, b, nh, c->hd, w.buf[3], 1, 0);
    if (*st == BDG_OK) *st = d2h(c, &v, w.buf[3], sizeof(double2));
    return v.x;
}

// Projected preconditioned CG for H_+ x = b on span(Np)^perp (Jordan partners).
bdg_status pcg_hplus(bdg_ctx* c, Small& w, long long nh, const double2* Np, int np, const double2* b, double2* x,
                     double2* ws, double tol, int max_iter) {
    double2* r = ws;
    double2* z = ws + nh;
    double2* p = ws + 2 * nh;
    double2* Ap = ws + 3 * nh;
    double2* tmp = ws + 4 * nh;
    const dim3 g1 = grid_cols(nh, 1);
    BDG_HIP(c, hipMemsetAsync(x, 0, nh * sizeof(double2), c->stream));
    BDG_HIP(c, hipMemcpyAsync(r, b, nh * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
    BDG_TRY(project_out(c, w, nh, Np, np, r, 1));
    BDG_TRY(launch_precond<double>(c, 3, 3, nh, r, z));
    BDG_TRY(project_out(c, w, nh, Np, np, z, 1));
    BDG_HIP(c, hipMemcpyAsync(p, z, nh * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
    bdg_status st;
    double rz = host_dot_re(c, w, nh, z, r, &st);
    BDG_TRY(st);
    const double bnorm = std::sqrt(std::max(0.0, host_dot_re(c, w, nh, r, r, &st)));
    BDG_TRY(st);
    if (bnorm == 0) return BDG_OK;
    for (int it = 0; it < max_iter; ++it) {
        BDG_TRY(apply64(c, 1, p, p, nh, Ap, tmp));
        BDG_TRY(project_out(c, w, nh, Np, np, Ap, 1));
        const double pAp = host_dot_re(c, w, nh, Ap, p, &st);
        BDG_TRY(st);
        if (!(pAp > 0)) return ctx_fail(c, BDG_EBREAKDOWN, "Jordan-partner solve: H_+ not positive");
        const double alpha = rz / pAp;
        hipLaunchKernelGGL(k_axpy, g1, dim3(256), 0, c->stream, nh, cmk<double2>(alpha, 0.0), (const double2*)p, x);
        hipLaunchKernelGGL(k_axpy, g1, dim3(256), 0, c->stream, nh, cmk<double2>(-alpha, 0.0), (const double2*)Ap, r);
        const double rn = std::sqrt(std::max(0.0, host_dot_re(c, w, nh, r, r, &st)));
        BDG_TRY(st);
        if (rn <= tol * bnorm) {
            if (debug_on()) fprintf(stderr, "[bdg pcg] converged in %d iterations (%.2e)\n", it + 1, rn / bnorm);
            return BDG_OK;
        }
        BDG_TRY(launch_precond<double>(c, 3, 3, nh, r, z));
        BDG_TRY(project_out(c, w, nh, Np, np, z, 1));
        const double rz_new = host_dot_re(c, w, nh, z, r, &st);
        BDG_TRY(st);
        hipLaunchKernelGGL(k_xpby, g1, dim3(256), 0, c->stream, nh, (const double2*)z, cmk<double2>(rz_new / rz, 0.0), p);
        rz = rz_new;
    }
    return ctx_fail(c, BDG_ENOCONV, "Jordan-partner solve did not converge");
}

struct Deflation {
    double2* Nm = nullptr;   // nh x pm, orthonormal basis of ns(H_-) (f-space deflation)
    int pm = 0;
    double2* Qg = nullptr;   // nh x pg, ns(H_+) + Jordan partners (g-space deflation)
    int pg = 0;
};

bdg_status build_deflation(bdg_ctx* c, Small& w, Deflation& d, double null_tol) {
    const long long npts = c->npts, nh = 3 * npts;
    double2* cand = nullptr;
    double2* img = nullptr;
    double2* ws = nullptr;
    BDG_TRY(ctx_alloc(c, (void**)&cand, 4 * nh * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&img, 8 * nh * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&ws, 5 * nh * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&d.Nm, 3 * nh * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&d.Qg, 4 * nh * sizeof(double2)));
    hipLaunchKernelGGL(k_candidates, dim3(1024), dim3(256), 0, c->stream, npts, (const double*)c->phi, cand);
    BDG_HIP(c, hipGetLastError());
    // images: [H_- c; H_+ c] for each candidate c (taken as both f and g)
    double2* Hm = img;
    double2* Hp = img + 4 * nh;
    BDG_TRY(apply64(c, 4, cand, cand, nh, Hp, Hm));
    double nc[4], nm[4], np_[4];
    BDG_TRY(colnorm2(c, nh, 4, cand, nh, w.s[0]));
    BDG_TRY(colnorm2(c, nh, 4, Hm, nh, w.s[1]));
    BDG_TRY(colnorm2(c, nh, 4, Hp, nh, w.s[2]));
    BDG_TRY(d2h(c, nc, w.s[0], 4 * sizeof(double)));
    BDG_TRY(d2h(c, nm, w.s[1], 4 * sizeof(double)));
    BDG_TRY(d2h(c, np_, w.s[2], 4 * sizeof(double)));
    const double cmax = std::max(std::max(nc[0], nc[1]), std::max(nc[2], nc[3]));
    double2* keep = ws;            // up to 3 columns (reuses PCG space before the solves)
    int km = 0;
    for (int j = 0; j < 3; ++j)
        if (nc[j] > 1e-24 * cmax && std::sqrt(nm[j]) <= null_tol * std::sqrt(nc[j])) {
            BDG_HIP(c, hipMemcpyAsync(keep + km * nh, cand + j * nh, nh * sizeof(double2), hipMemcpyDeviceToDevice,
                                      c->stream));
            ++km;
        }
    BDG_TRY(orthonormalize(c, w, nh, keep, km, d.Nm, 1e-10, &d.pm));
    // ns(H_+) candidate: K Phi
    double2* Np = img;             // reuse
    int pp = 0;
    if (nc[3] > 1e-20 * cmax && std::sqrt(np_[3]) <= null_tol * std::sqrt(nc[3])) {
        BDG_TRY(orthonormalize(c, w, nh, cand + 3 * nh, 1, Np, 1e-10, &pp));
    }
    // sources of the Jordan partners: part of N_- orthogonal to N_+.  A column that keeps less
    // than 1e-4 of its norm after the projection lies in N_+ up to the ground state's own
    // error (at M = 0 in the ferromagnetic phase K Phi = -S_z Phi): it has no partner, and
    // rescaling its remainder would deflate that error pattern, a smooth low-mode direction
    double2* src = img + nh;       // up to 3 columns
    BDG_HIP(c, hipMemcpyAsync(keep, d.Nm, d.pm * nh * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
    double n0[3] = {0, 0, 0}, n1[3] = {0, 0, 0};
    BDG_TRY(colnorm2(c, nh, d.pm, keep, nh, w.s[0]));
    BDG_TRY(d2h(c, n0, w.s[0], d.pm * sizeof(double)));
    BDG_TRY(project_out(c, w, nh, Np, pp, keep, d.pm));
    BDG_TRY(colnorm2(c, nh, d.pm, keep, nh, w.s[0]));
    BDG_TRY(d2h(c, n1, w.s[0], d.pm * sizeof(double)));
    int nsrc = 0;
    for (int j = 0; j < d.pm; ++j) {
        if (!(n1[j] >= 1e-8 * n0[j])) continue;
        if (nsrc != j)
            BDG_HIP(c, hipMemcpyAsync(keep + nsrc * nh, keep + j * nh, nh * sizeof(double2), hipMemcpyDeviceToDevice,
                                      c->stream));
        ++nsrc;
    }
    int ps = 0;
    BDG_TRY(orthonormalize(c, w, nh, keep, nsrc, src, 1e-8, &ps));
    // partners into the columns after N_+
    double2* qcols = cand;         // [N_+, partners], up to 4 columns
    if (pp) BDG_HIP(c, hipMemcpyAsync(qcols, Np, nh * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
    for (int j = 0; j < ps; ++j)
        BDG_TRY(pcg_hplus(c, w, nh, Np, pp, src + j * nh, qcols + (pp + j) * nh, ws, 1e-13, 5000));
    BDG_TRY(orthonormalize(c, w, nh, qcols, pp + ps, d.Qg, 1e-10, &d.pg));
    if (debug_on()) {
        fprintf(stderr, "[bdg deflation] |c|^2=(%.3e %.3e %.3e %.3e) |H_- c|^2=(%.3e %.3e %.3e %.3e) |H_+ c|^2=(%.3e %.3e %.3e %.3e)\n",
                nc[0], nc[1], nc[2], nc[3], nm[0], nm[1], nm[2], nm[3], np_[0], np_[1], np_[2], np_[3]);
        fprintf(stderr, "[bdg deflation] N_- dim %d, N_+ dim %d, partners %d, Q_g dim %d\n", d.pm, pp, ps, d.pg);
    }
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    ctx_free(c, cand);
    ctx_free(c, img);
    ctx_free(c, ws);
    return BDG_OK;
}

}  // namespace

// =====================================================================================
// bdg_biortho, bdg_biortho_noalloc
// =====================================================================================
namespace {

// Factors of the bi-orthogonalization: B = h^d G^H F = U diag(s) V^H, C_f = V s^-1/2 into
// w.buf[1], C_g = U s^-1/2 into w.buf[2] (nvec x nvec, ld nvec; columns with
// s_j <= 1e-12 s_1 dropped and set to zero).  s_host: nvec values; *rank: the columns kept.
// Workspace from ctx_alloc / ctx_scratch (the context's own memory, or its arena).
bdg_status biortho_factors(bdg_ctx* c, Small& w, int nvec, const double2* F, const double2* G, double* s_host,
                           int* rank) {
    const long long nh = 3 * c->npts;
    BDG_TRY(small_alloc(c, w, nvec));
    double2* B = w.buf[0];
    double2* V = w.buf[1];
    double2* Cg = w.buf[2];
    BDG_TRY(gram<double2, double2>(c, nh, nvec, nvec, G, nh, F, nh, c->hd, B, nvec, 0));
    BDG_TRY(small_svd(c, nvec, nvec, B, nvec, V, nvec, w.s[0]));
    BDG_TRY(d2h(c, s_host, w.s[0], nvec * sizeof(double)));
    int r = 0;
    while (r < nvec && s_host[r] > 1e-12 * s_host[0] && s_host[r] > 0) ++r;
    // C_f = V s^-1/2 ; C_g = (U s) s^-3/2 ; dropped columns -> 0
    BDG_TRY(small_colpow(c, nvec, nvec, V, nvec, w.s[0], -0.5));
    BDG_TRY(small_copy(c, nvec, nvec, B, nvec, Cg, nvec));
    BDG_TRY(small_colpow(c, nvec, nvec, Cg, nvec, w.s[0], -1.5));
    if (r < nvec) {
        hipLaunchKernelGGL(k_small_zero_cols, dim3((unsigned)((nvec + 255) / 256), (unsigned)(nvec - r)), dim3(256),
                           0, c->stream, nvec, r, V, nvec);
        hipLaunchKernelGGL(k_small_zero_cols, dim3((unsigned)((nvec + 255) / 256), (unsigned)(nvec - r)), dim3(256),
                           0, c->stream, nvec, r, Cg, nvec);
        BDG_HIP(c, hipGetLastError());
    }
    *rank = r;
    return BDG_OK;
}

bool overlaps(const void* a, const void* b, size_t bytes) {
    const char* p = (const char*)a;
    const char* q = (const char*)b;
    return p < q + bytes && q < p + bytes;
}

}  // namespace

extern "C" bdg_status bdg_biortho(bdg_ctx* c, int nvec, void* F_dev, void* G_dev, double* sigma, int* rank) {
    if (!c) return BDG_EINVAL;
    if (nvec <= 0 || nvec > 512 || !F_dev || !G_dev) return ctx_fail(c, BDG_EINVAL, "bdg_biortho: bad arguments");
    const long long nh = 3 * c->npts;
    const size_t bytes = (size_t)nvec * nh * sizeof(double2);
    double2* F = (double2*)F_dev;
    double2* G = (double2*)G_dev;
    Small w;
    double2* tmp = nullptr;
    auto release = defer([&] {
        ctx_free(c, tmp);
        small_free(c, w);
    });
    std::vector<double> s(nvec);
    int r = 0;
    BDG_TRY(biortho_factors(c, w, nvec, F, G, s.data(), &r));
    BDG_TRY(ctx_alloc(c, (void**)&tmp, bytes));
    Seg sf{F, nvec}, sg{G, nvec};
    BDG_TRY(update(c, nh, &sf, 1, nh, w.buf[1], nvec, nvec, 0.0, tmp, nh));
    BDG_HIP(c, hipMemcpyAsync(F, tmp, bytes, hipMemcpyDeviceToDevice, c->stream));
    BDG_TRY(update(c, nh, &sg, 1, nh, w.buf[2], nvec, nvec, 0.0, tmp, nh));
    BDG_HIP(c, hipMemcpyAsync(G, tmp, bytes, hipMemcpyDeviceToDevice, c->stream));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    if (sigma) std::memcpy(sigma, s.data(), nvec * sizeof(double));
    if (rank) *rank = r;
    return BDG_OK;
}

// The allocation-free variant's workspace: one static array per device, reached through the
// address hipGetSymbolAddress gives for it on that device (the array's name is a host-side
// stand-in and is never passed to a kernel).  Every call on a device uses that device's
// array, so calls that overlap on one device race.  Its size: the split-K partials of the
// Gram matrix (at most NOALLOC_GRAM_BYTES) and the small matrices of the SVD.
namespace {
constexpr size_t NOALLOC_GRAM_BYTES = 40ull << 20;
static_assert(NOALLOC_GRAM_BYTES < BDG_NOALLOC_SCRATCH_BYTES, "Gram share inside the scratch");
}  // namespace
static __device__ __align__(256) unsigned char scratch[BDG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of `scratch` on the context's device (looked up once per device)
bdg_status noalloc_scratch(bdg_ctx* c, void** out) {
    if (c->device < 0 || c->device >= NOALLOC_MAX_DEVICES)
        return ctx_fail(c, BDG_EDEVICE, "bdg_biortho_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[c->device]) {
        int cur = -1;
        BDG_HIP(c, hipGetDevice(&cur));
        if (cur != c->device) BDG_HIP(c, hipSetDevice(c->device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != c->device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) return hip_check(c, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                    "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[c->device] = p;
    }
    *out = g_scratch_ptr[c->device];
    return BDG_OK;
}
}  // namespace

extern "C" bdg_status bdg_biortho_noalloc(bdg_ctx* c, int nvec, const void* F_dev, const void* G_dev, void* Fout_dev,
                                          void* Gout_dev, double* sigma, int* rank) {
    if (!c) return BDG_EINVAL;
    if (nvec <= 0 || nvec > BDG_NOALLOC_MAX_VEC || !F_dev || !G_dev || !Fout_dev || !Gout_dev) {
        char buf[160];
        snprintf(buf, sizeof buf, "bdg_biortho_noalloc: need 1 <= nvec <= %d (the static scratch bound) and four "
                 "buffers, got nvec = %d", BDG_NOALLOC_MAX_VEC, nvec);
        return ctx_fail(c, BDG_EINVAL, buf);
    }
    const size_t bytes = (size_t)nvec * 3 * c->npts * sizeof(double2);
    const void* ins[2] = {F_dev, G_dev};
    const void* outs[2] = {Fout_dev, Gout_dev};
    if (overlaps(Fout_dev, Gout_dev, bytes))
        return ctx_fail(c, BDG_EINVAL, "bdg_biortho_noalloc: the two outputs overlap");
    for (const void* o : outs)
        for (const void* i : ins)
            if (overlaps(o, i, bytes)) return ctx_fail(c, BDG_EINVAL, "bdg_biortho_noalloc: an output overlaps an input");
    void* base = nullptr;
    BDG_TRY(noalloc_scratch(c, &base));
    // every piece of workspace below comes from the static array (arena mode of the context)
    c->arena = bdg_ctx::Arena{(char*)base, BDG_NOALLOC_SCRATCH_BYTES, 0, NOALLOC_GRAM_BYTES};
    Small w;
    auto leave = defer([&] {
        small_free(c, w);
        c->arena = bdg_ctx::Arena{};
    });
    const long long nh = 3 * c->npts;
    double s[BDG_NOALLOC_MAX_VEC];
    int r = 0;
    BDG_TRY(biortho_factors(c, w, nvec, (const double2*)F_dev, (const double2*)G_dev, s, &r));
    Seg sf{F_dev, nvec}, sg{G_dev, nvec};
    BDG_TRY(update(c, nh, &sf, 1, nh, w.buf[1], nvec, nvec, 0.0, (double2*)Fout_dev, nh));
    BDG_TRY(update(c, nh, &sg, 1, nh, w.buf[2], nvec, nvec, 0.0, (double2*)Gout_dev, nh));
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    if (sigma) std::memcpy(sigma, s, nvec * sizeof(double));
    if (rank) *rank = r;
    return BDG_OK;
}

// =====================================================================================
// bdg_eigs
// =====================================================================================
namespace {

struct EigsOpts {
    double rtol = 1e-12;        // pivoted-Cholesky cut-off (Schur complement of the scaled Gram)
    double eps = 1e-10;         // LU pivot cut-off of the pairing matrix
    double null_tol = 1e-6;     // nullspace candidate test
    int refresh_every = 25;     // float64 re-projection and image refresh period (iterations)
    int refresh_every32 = 10;   // the same while W and P are applied in float32: F's recurrence
                                // images then gather float32 rounding in proportion to the steps
                                // taken since the last refresh
    int stall_iters = 10;       // mixed form: switch to float64 applies after this many
                                // iterations without halving the residual, or at once when
                                // it grows past rise_factor times its best value
    double rise_factor = 4.0;
    double rtol32 = 1e-10;      // cut-offs while images carry float32 rounding
    double eps32 = 1e-8;
    double floor_c = 100.0;     // a column also counts as converged once its residual reaches
                                // floor_c * eps ||H|| / |omega|, the float64 rounding floor of
                                // the relative residual (a smaller tol is not attainable there)
};

// upper bound of ||H||: largest kinetic symbol plus the largest pointwise row sum of H_+-
bdg_status operator_bound(bdg_ctx* c, double* out) {
    double kin = 0;
    for (int a = 0; a < c->dim; ++a) {
        const double kmax = M_PI * c->n[a] / (2.0 * c->L[a]);
        kin += 0.5 * kmax * kmax;
    }
    constexpr int NB = 256;
    double* part = nullptr;
    BDG_TRY(ctx_alloc(c, (void**)&part, NB * sizeof(double)));
    hipLaunchKernelGGL(k_coef_bound, dim3(NB), dim3(256), 0, c->stream, c->npts, (const double*)c->coef64, part);
    bdg_status st = hip_check(c, hipGetLastError(), "k_coef_bound");
    double hp[NB];
    if (st == BDG_OK) st = d2h(c, hp, part, NB * sizeof(double));
    ctx_free(c, part);
    if (st != BDG_OK) return st;
    double mx = 0;
    for (int i = 0; i < NB; ++i) mx = std::max(mx, hp[i]);
    *out = kin + mx;
    return BDG_OK;
}

bdg_status eigs_impl(bdg_ctx* c, int k, int nb_req, double tol, int max_iter, const void* X0_dev,
                     unsigned long long seed, double* omega_out, void* UV_dev, double* res_out, int* iters_out) {
    const EigsOpts opt;
    const long long npts = c->npts, nh = 3 * npts;
    const bool mixed = c->prob.precision == BDG_FP32_APPLY;
    // real trial vectors in the paired form: nb real columns (the block rounded up to even)
    // in nbc complex columns
    const int nb = nb_req + (nb_req & 1);
    const int nbc = nb / 2;
    const int m = 3 * nb;
    auto t_start = std::chrono::steady_clock::now();
    for (double& s : c->stats) s = 0;
    // ------------------------------------------------------------------ allocation
    Small w;
    Basis S;
    float2* w32 = nullptr;
    float2* y32 = nullptr;
    double2* acoef = nullptr;
    double2* bcoef = nullptr;
    double* dvec = nullptr;
    int* d_act = nullptr;
    double* d_scl = nullptr;
    Deflation D;
    // every exit path releases the workspace
    auto release = defer([&] {
        small_free(c, w);
        for (int a = 0; a < 4; ++a) ctx_free(c, S.arr[a]);
        ctx_free(c, w32);
        ctx_free(c, y32);
        ctx_free(c, acoef);
        ctx_free(c, bcoef);
        ctx_free(c, dvec);
        ctx_free(c, d_act);
        ctx_free(c, d_scl);
        ctx_free(c, D.Nm);
        ctx_free(c, D.Qg);
    });
    BDG_TRY(small_alloc(c, w, std::max(m, 8)));
    S.nh = nh;
    S.nb = nbc;
    for (int a = 0; a < 4; ++a) BDG_TRY(ctx_alloc(c, (void**)&S.arr[a], 4 * (size_t)nbc * nh * sizeof(double2)));
    if (mixed) {
        // float32 staging of [W, P] (f halves, then g halves) and of their images
        BDG_TRY(ctx_alloc(c, (void**)&w32, 4 * (size_t)nbc * nh * sizeof(float2)));
        BDG_TRY(ctx_alloc(c, (void**)&y32, 4 * (size_t)nbc * nh * sizeof(float2)));
    }
    BDG_TRY(ctx_alloc(c, (void**)&acoef, (size_t)m * nb * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&bcoef, (size_t)m * nb * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&dvec, 8 * (size_t)nb * sizeof(double)));
    BDG_TRY(ctx_alloc(c, (void**)&d_act, (size_t)nb * sizeof(int)));
    BDG_TRY(ctx_alloc(c, (void**)&d_scl, 2 * (size_t)m * sizeof(double)));
    double* d_sf = d_scl;          // squared column norms of S_f = [F, W_f, P_f] (W, P part)
    double* d_sg = d_scl + m;      // and of S_g
    double* d_om = dvec;
    double* d_n = dvec + nb;      // 4 nb norms
    // ------------------------------------------------------------------ deflation
    BDG_TRY(build_deflation(c, w, D, opt.null_tol));
    double hbound = 0;
    BDG_TRY(operator_bound(c, &hbound));
    auto t_setup = std::chrono::steady_clock::now();
    c->stats[6] = std::chrono::duration<double, std::milli>(t_setup - t_start).count();
    // ------------------------------------------------------------------ start block
    S.slotF = 0; S.slotW = 1; S.slotP = -1; S.slotFree = 2; S.slotFree2 = 3;
    double2* F = S.col(SF, S.slotF);
    double2* G = S.col(SG, S.slotF);
    // real start vectors: normals from `seed` (each complex normal gives two), then, with a start
    // block, real column j = Re + Im of its vector j (a generic real direction of the vector's
    // span; the operator is real, so its eigenvectors may be taken real)
    hipLaunchKernelGGL(k_randn, dim3(2048), dim3(256), 0, c->stream, (long long)nbc * nh, seed, F);
    hipLaunchKernelGGL(k_randn, dim3(2048), dim3(256), 0, c->stream, (long long)nbc * nh, seed ^ 0x5851F42D4C957F2DULL, G);
    if (X0_dev)
        hipLaunchKernelGGL(k_pair_start, grid_cols(nh, nbc), dim3(256), 0, c->stream, nh, nb_req,
                           (const double2*)X0_dev, F, G);
    BDG_HIP(c, hipGetLastError());
    BDG_TRY(project_out(c, w, nh, D.Nm, D.pm, F, nbc));
    BDG_TRY(project_out(c, w, nh, D.Qg, D.pg, G, nbc));
    double napply64 = 0, napply32 = 0;
    BDG_TRY(apply64(c, nbc, F, G, nh, S.col(HSF, S.slotF), S.col(HSG, S.slotF)));
    napply64 += nb;
    double2* Gf = w.buf[0];
    double2* Gg = w.buf[1];
    double2* Br = w.buf[2];
    double2* Mr = w.buf[3];
    double2* Kr = w.buf[4];
    std::vector<double> om;
    // per-column target: tol, or the rounding floor of the relative residual when that is larger
    auto target = [&](int j) { return std::max(tol, opt.floor_c * DBL_EPSILON * hbound / std::fabs(om[j])); };
    // Gram matrices of S_f = [F, W_f, P_f], S_g = [G, W_g, P_g] and their images.  With
    // cross_from_f the first block row of the projected operators is taken as (H F)^T S
    // instead of F^T (H S): the images of W and P then enter only the [W, P] x [W, P] block.
    // (Used while W and P are applied in float32: their images carry eps32 ||H|| whatever
    // the residual, and in the F x [W, P] blocks that error would couple the converged
    // directions to the corrections and stall the residual near eps32 ||H|| / omega; the
    // images of F follow by recurrence and carry an error that falls with the step.)
    auto grams = [&](const Seg* sf, const Seg* sg, const Seg* hf, const Seg* hg, int ns, int ldc,
                     bool cross_from_f) -> bdg_status {
        BDG_TRY(gram_seg_pair(c, nh, sf, ns, nh, sf, ns, nh, c->hd, Gf, ldc, 1));
        BDG_TRY(gram_seg_pair(c, nh, sg, ns, nh, sg, ns, nh, c->hd, Gg, ldc, 1));
        BDG_TRY(gram_seg_pair(c, nh, sg, ns, nh, sf, ns, nh, c->hd, Br, ldc, 0));
        if (!cross_from_f) {
            BDG_TRY(gram_seg_pair(c, nh, sf, ns, nh, hf, ns, nh, c->hd, Mr, ldc, 1));
            BDG_TRY(gram_seg_pair(c, nh, sg, ns, nh, hg, ns, nh, c->hd, Kr, ldc, 1));
            return BDG_OK;
        }
        const int r0 = 2 * sf[0].ncols;       // real columns of F
        const size_t d = (size_t)r0 * ldc + r0;
        BDG_TRY(gram_seg_pair(c, nh, hf, 1, nh, sf, ns, nh, c->hd, Mr, ldc, 0));
        BDG_TRY(gram_seg_pair(c, nh, sf + 1, ns - 1, nh, hf + 1, ns - 1, nh, c->hd, Mr + d, ldc, 1));
        BDG_TRY(gram_seg_pair(c, nh, hg, 1, nh, sg, ns, nh, c->hd, Kr, ldc, 0));
        BDG_TRY(gram_seg_pair(c, nh, sg + 1, ns - 1, nh, hg + 1, ns - 1, nh, c->hd, Kr + d, ldc, 1));
        const dim3 gm((unsigned)((ldc - r0 + 127) / 128), (unsigned)r0);
        hipLaunchKernelGGL(k_small_mirror_rows, gm, dim3(128), 0, c->stream, ldc, r0, Mr, ldc);
        hipLaunchKernelGGL(k_small_mirror_rows, gm, dim3(128), 0, c->stream, ldc, r0, Kr, ldc);
        return hip_check(c, hipGetLastError(), "k_small_mirror_rows");
    };
    // re-deflate F, G (and P) and recompute their images with float64 applies; with_p = false
    // leaves P alone (its images are recomputed from P in the same iteration anyway)
    auto refresh = [&](double2* F_, double2* G_, double2* HF_, double2* HG_, bool with_p = true) -> bdg_status {
        BDG_TRY(project_out(c, w, nh, D.Nm, D.pm, F_, nbc));
        BDG_TRY(project_out(c, w, nh, D.Qg, D.pg, G_, nbc));
        BDG_TRY(apply64(c, nbc, F_, G_, nh, HF_, HG_));
        napply64 += nb;
        if (with_p && S.slotP >= 0) {
            double2* Pf = S.col(SF, S.slotP);
            double2* Pg = S.col(SG, S.slotP);
            BDG_TRY(project_out(c, w, nh, D.Nm, D.pm, Pf, nbc));
            BDG_TRY(project_out(c, w, nh, D.Qg, D.pg, Pg, nbc));
            BDG_TRY(apply64(c, nbc, Pf, Pg, nh, S.col(HSF, S.slotP), S.col(HSG, S.slotP)));
            napply64 += nb;
        }
        return BDG_OK;
    };
    {
        Seg sf{F, nbc}, sg{G, nbc}, hf{S.col(HSF, S.slotF), nbc}, hg{S.col(HSG, S.slotF), nbc};
        BDG_TRY(grams(&sf, &sg, &hf, &hg, 1, nb, false));
        BDG_TRY(rayleigh_ritz(c, w, nb, nb, Gf, Gg, Br, Mr, Kr, acoef, bcoef, om, opt.rtol, opt.eps));
        const int s_new = S.slotW;
        for (int a = 0; a < 4; ++a) {
            Seg src{S.col(a, S.slotF), nbc};
            BDG_TRY(update_pair(c, nh, &src, 1, nh, (a == SF || a == HSF) ? acoef : bcoef, nb, 0, nb, 0.0,
                                S.col(a, s_new), nh, S.col(a, s_new), nh));
        }
        S.slotW = S.slotF;
        S.slotF = s_new;
    }
    int it = 0;
    int last_refresh = 0, recoveries = 0, best_it = 0;
    double best_r = 1e300;
    bool switch64 = false;
    bool armed = false;
    bool converged = false;
    bool refreshed = false;
    int certifications = 0;
    bool force64 = false;
    std::vector<double> res(nb, 1.0), hn(4 * nb);
    bdg_status final_status = BDG_ENOCONV;
    // phase times from events on the stream (no host synchronization of their own): marks
    // 0..5 bound correction, apply, Gram, projected problem and update of one iteration; they
    // are read after the next host synchronization.  BDG_PHASE_SYNC=1 adds a stream
    // synchronization after every phase (host-side view of the same split).
    // Two sets alternate, so an iteration records into one while the other waits to be read.
    double t_phase[5] = {0, 0, 0, 0, 0};
    hipEvent_t ev[2][6] = {};
    for (auto& set : ev)
        for (auto& e : set) BDG_HIP(c, hipEventCreate(&e));
    auto ev_free = defer([&] {
        for (auto& set : ev)
            for (auto& e : set)
                if (e) (void)hipEventDestroy(e);
    });
    int ev_cur = 0, ev_pending = -1;
    auto mark = [&](int i) -> bdg_status {
        BDG_HIP(c, hipEventRecord(ev[ev_cur][i], c->stream));
        if (i == 5) {
            ev_pending = ev_cur;
            ev_cur ^= 1;
        }
        return BDG_OK;
    };
    auto collect = [&]() -> bdg_status {
        if (ev_pending < 0) return BDG_OK;
        for (int i = 0; i < 5; ++i) {
            float ms = 0;
            BDG_HIP(c, hipEventElapsedTime(&ms, ev[ev_pending][i], ev[ev_pending][i + 1]));
            t_phase[i] += ms;
        }
        ev_pending = -1;
        return BDG_OK;
    };
    const bool phase_sync = [] {
        const char* v = std::getenv("BDG_PHASE_SYNC");
        return v && v[0] == '1';
    }();
    auto sync_if = [&]() -> bdg_status {
        if (phase_sync) BDG_HIP(c, hipStreamSynchronize(c->stream));
        return BDG_OK;
    };
    std::vector<int> act;
    for (it = 1; it <= max_iter; ++it) {
        F = S.col(SF, S.slotF);
        G = S.col(SG, S.slotF);
        double2* HF = S.col(HSF, S.slotF);
        double2* HG = S.col(HSG, S.slotF);
        double2* Wf = S.col(SF, S.slotW);
        double2* Wg = S.col(SG, S.slotW);
        // residual norms of every column in one pass over F, G and their images
        BDG_TRY(mark(0));
        BDG_TRY(h2d(c, d_om, om.data(), nb * sizeof(double)));
        BDG_TRY(resnorm2_pair(c, nh, nbc, HF, G, HG, F, nh, d_om, d_n));
        BDG_TRY(d2h(c, hn.data(), d_n, 4 * nb * sizeof(double)));
        BDG_TRY(collect());
        double rmax = 0;
        bool all_k = true;
        act.clear();
        for (int j = 0; j < nb; ++j) {
            res[j] = std::sqrt(hn[j] + hn[nb + j]) / (std::fabs(om[j]) * std::sqrt(hn[2 * nb + j] + hn[3 * nb + j]));
            const bool done = res[j] <= target(j);
            if (j < k) { rmax = std::max(rmax, res[j]); all_k = all_k && done; }
            if (!done) act.push_back(j);      // soft locking: converged columns get no correction
        }
        if (act.size() & 1) {
            // corrections go two to a complex column: add the converged column with the largest
            // residual (nb is even, so one exists)
            int jb = -1;
            for (int j = 0; j < nb; ++j)
                if (std::find(act.begin(), act.end(), j) == act.end() && (jb < 0 || res[j] > res[jb])) jb = j;
            act.push_back(jb);
        }
        const int nact = (int)act.size();
        const int nactc = nact / 2;
        if (!(rmax == rmax)) return ctx_fail(c, BDG_EBREAKDOWN, "non-finite residual");
        if (debug_on())
            fprintf(stderr, "[bdg it %d] omega0=%.12f omega_k=%.12f res_max(k)=%.3e res0=%.3e active=%d\n", it, om[0],
                    om[k - 1], rmax, res[0], nact);
        // mixed form: W and P are applied in float32 (their images carry relative rounding
        // eps32 in every iteration) and F's images follow by recurrence, refreshed in float64
        // every refresh_every32 iterations, so the rounding they gather is proportional to
        // the steps taken since and falls with the residual.  Should the residual still stop
        // falling (10 iterations without halving) or rise 4x above its best, float64 applies
        // finish the solve.
        if (mixed && !force64) {
            // both detectors are armed once the start-up transient is over (residual < 0.1)
            if (!armed && rmax < 0.1) { armed = true; best_r = rmax; best_it = it; }
            if (armed) {
                if (rmax < best_r * 0.5) { best_r = rmax; best_it = it; }
                if (it - best_it > opt.stall_iters || rmax > opt.rise_factor * best_r) {
                    switch64 = true;
                    if (debug_on()) {
                        fprintf(stderr, "[bdg it %d] float64 applies from here: residual %.3e, best %.3e at it %d\n",
                                it, rmax, best_r, best_it);
                        for (int j = 0; j < k; ++j)
                            if (res[j] > 4.0 * best_r)
                                fprintf(stderr, "[bdg it %d]   column %d omega %.12f residual %.3e\n", it, j, om[j],
                                        res[j]);
                    }
                }
            }
        }
        const bool phase32 = mixed && !force64;
        const bool want_refresh =
            switch64 || (it - last_refresh >= (phase32 ? opt.refresh_every32 : opt.refresh_every));
        if (want_refresh) {
            // re-project the basis off the generalized nullspace and recompute its images in
            // float64 (bounds the drift of the recurrence-updated images; in the mixed form
            // it also removes the float32 rounding the images carry)
            BDG_TRY(refresh(F, G, HF, HG, !(phase32 && !switch64)));
            if (switch64) { force64 = true; refreshed = true; switch64 = false; }
            last_refresh = it;
            --it;
            continue;
        }
        if (all_k || nact == 0) {
            // certify with a float64 apply of the current block
            double2* CF = S.col(HSF, S.slotFree);
            double2* CG = S.col(HSG, S.slotFree);
            BDG_TRY(apply64(c, nbc, F, G, nh, CF, CG));
            napply64 += nb;
            BDG_TRY(resnorm2_pair(c, nh, nbc, CF, G, CG, F, nh, d_om, d_n));
            BDG_TRY(d2h(c, hn.data(), d_n, 4 * nb * sizeof(double)));
            bool certified = true;
            for (int j = 0; j < nb; ++j) {
                res[j] = std::sqrt(hn[j] + hn[nb + j]) / (std::fabs(om[j]) * std::sqrt(hn[2 * nb + j] + hn[3 * nb + j]));
                if (j < k) certified = certified && res[j] <= target(j);
            }
            if (certified) {
                converged = true;
                break;
            }
            // images drifted: refresh and continue (float64 corrections from now on)
            BDG_TRY(refresh(F, G, HF, HG));
            last_refresh = it;
            force64 = true;
            if (++certifications > 4) break;
            --it;
            continue;
        }
        // residual directions of the active columns: f-direction H_+ f - w g, g-direction
        // H_- g - w f, then the preconditioner (its precision only affects the rate; the
        // mixed form writes the residuals in float32 and gets float64 back from the
        // preconditioner's last pass)
        BDG_TRY(h2d(c, d_act, act.data(), nact * sizeof(int)));
        // residual directions scaled to unit columns (their squared norms are in d_n: q = 0
        // for H_+ f - w g, q = 1 for H_- g - w f)
        if (mixed) {
            hipLaunchKernelGGL(k_pair_axmy_idx32, grid_cols(nh, nactc), dim3(256), 0, c->stream, nh,
                               (const double2*)HF, (const double2*)G, nh, (const double*)d_om, (const int*)d_act,
                               (const double*)d_n, w32, nh);
            hipLaunchKernelGGL(k_pair_axmy_idx32, grid_cols(nh, nactc), dim3(256), 0, c->stream, nh,
                               (const double2*)HG, (const double2*)F, nh, (const double*)d_om, (const int*)d_act,
                               (const double*)(d_n + nb), w32 + (size_t)nactc * nh, nh);
            BDG_HIP(c, hipGetLastError());
            BlockRef<float2> x32{w32, w32 + (size_t)nactc * nh, nh};
            BlockRef<double2> y64{Wf, Wg, nh};
            BDG_TRY(launch_precond_mixed(c, nactc, x32, y64));
        } else {
            hipLaunchKernelGGL(k_pair_axmy_idx, grid_cols(nh, nactc), dim3(256), 0, c->stream, nh, (const double2*)HF,
                               (const double2*)G, nh, (const double*)d_om, (const int*)d_act, (const double*)d_n, Wf,
                               nh);
            hipLaunchKernelGGL(k_pair_axmy_idx, grid_cols(nh, nactc), dim3(256), 0, c->stream, nh, (const double2*)HG,
                               (const double2*)F, nh, (const double*)d_om, (const int*)d_act,
                               (const double*)(d_n + nb), Wg, nh);
            BDG_HIP(c, hipGetLastError());
            BDG_TRY(launch_precond<double>(c, 3 * nactc, 3, nh, Wf, Wf));
            BDG_TRY(launch_precond<double>(c, 3 * nactc, 3, nh, Wg, Wg));
        }
        BDG_TRY(project_out(c, w, nh, D.Nm, D.pm, Wf, nactc));
        BDG_TRY(project_out(c, w, nh, D.Qg, D.pg, Wg, nactc));
        // W and P are scaled to unit columns in memory before they are applied: two real
        // vectors share a complex FFT, whose rounding is relative to the larger of the pair
        // (see k_pair_axmy_idx); the Gram matrices are then those of unit columns.  With
        // float32 images the scaling rides in the float32 copy made for the apply
        const bool w32img = mixed && !force64;
        BDG_TRY(colnorm2_pair(c, nh, nactc, Wf, nh, d_sf + nb));
        BDG_TRY(colnorm2_pair(c, nh, nactc, Wg, nh, d_sg + nb));
        if (!w32img) {
            hipLaunchKernelGGL(k_pair_unit_cols, grid_cols(nh, nactc), dim3(256), 0, c->stream, nh, Wf, nh,
                               (const double*)(d_sf + nb));
            hipLaunchKernelGGL(k_pair_unit_cols, grid_cols(nh, nactc), dim3(256), 0, c->stream, nh, Wg, nh,
                               (const double*)(d_sg + nb));
        }
        // P of the active columns only: gather them (and their images) into the free slot
        if (S.slotP >= 0 && nact < nb) {
            for (int a = 0; a < 4; ++a)
                hipLaunchKernelGGL(k_pair_gather, grid_cols(nh, nactc), dim3(256), 0, c->stream, nh,
                                   (const double2*)S.col(a, S.slotP), nh, (const int*)d_act, S.col(a, S.slotFree),
                                   nh);
            BDG_HIP(c, hipGetLastError());
            std::swap(S.slotP, S.slotFree);
        }
        const int np = S.slotP >= 0 ? nact : 0;
        if (np) {
            BDG_TRY(colnorm2_pair(c, nh, np / 2, S.col(SF, S.slotP), nh, d_sf + nb + nact));
            BDG_TRY(colnorm2_pair(c, nh, np / 2, S.col(SG, S.slotP), nh, d_sg + nb + nact));
            if (!w32img) {
                hipLaunchKernelGGL(k_pair_unit_cols, grid_cols(nh, np / 2), dim3(256), 0, c->stream, nh,
                                   S.col(SF, S.slotP), nh, (const double*)(d_sf + nb + nact));
                hipLaunchKernelGGL(k_pair_unit_cols, grid_cols(nh, np / 2), dim3(256), 0, c->stream, nh,
                                   S.col(SG, S.slotP), nh, (const double*)(d_sg + nb + nact));
            }
        }
        BDG_HIP(c, hipGetLastError());
        BDG_TRY(sync_if());
        BDG_TRY(mark(1));
        double2* HWf = S.col(HSF, S.slotW);
        double2* HWg = S.col(HSG, S.slotW);
        if (w32img) {
            // W and P (when present) in one float32 launch: f halves [W_f, P_f], g halves
            // [W_g, P_g]; P's images are recomputed from P as in the float64 form below
            const int nv = S.slotP >= 0 ? 2 * nactc : nactc;
            float2* f32 = w32;
            float2* g32 = w32 + (size_t)nv * nh;
            double2* src_f[2] = {Wf, S.slotP >= 0 ? S.col(SF, S.slotP) : nullptr};
            double2* src_g[2] = {Wg, S.slotP >= 0 ? S.col(SG, S.slotP) : nullptr};
            const double* sq_f[2] = {d_sf + nb, d_sf + nb + nact};
            const double* sq_g[2] = {d_sg + nb, d_sg + nb + nact};
            double2* dst_hf[2] = {HWf, S.slotP >= 0 ? S.col(HSF, S.slotP) : nullptr};
            double2* dst_hg[2] = {HWg, S.slotP >= 0 ? S.col(HSG, S.slotP) : nullptr};
            const int nparts = S.slotP >= 0 ? 2 : 1;
            for (int q = 0; q < nparts; ++q) {
                hipLaunchKernelGGL(k_pair_unit_to32, grid_cols(nh, nactc), dim3(256), 0, c->stream, nh, src_f[q], nh,
                                   sq_f[q], f32 + (size_t)q * nactc * nh, nh);
                hipLaunchKernelGGL(k_pair_unit_to32, grid_cols(nh, nactc), dim3(256), 0, c->stream, nh, src_g[q], nh,
                                   sq_g[q], g32 + (size_t)q * nactc * nh, nh);
            }
            BDG_HIP(c, hipGetLastError());
            // one float32 apply per part, its images written in float64 by the last pass
            // (lo: H_- g, hi: H_+ f; the float32 work block is y32)
            for (int q = 0; q < nparts; ++q) {
                BlockRef<const float2> X{f32 + (size_t)q * nactc * nh, g32 + (size_t)q * nactc * nh, nh};
                BlockRef<float2> Yw{y32 + (size_t)q * nactc * nh, y32 + (size_t)(nv + q * nactc) * nh, nh};
                BlockRef<double2> Y64{dst_hg[q], dst_hf[q], nh};
                BDG_TRY(launch_apply_fg_to64(c, nactc, X, Yw, Y64));
            }
            napply32 += 2 * nv;
        } else {
            BDG_TRY(apply64(c, nactc, Wf, Wg, nh, HWf, HWg));
            napply64 += nact;
        }
        // P's images are recomputed from P (in float32 above, in float64 here): the recurrence
        // [H W, H P] a carries the cancellation in P = [W, P] a (a short step built from unit
        // columns) into the images, whose relative error then grows by the convergence factor
        // per iteration
        if (S.slotP >= 0 && !(mixed && !force64)) {
            BDG_TRY(apply64(c, nactc, S.col(SF, S.slotP), S.col(SG, S.slotP), nh, S.col(HSF, S.slotP),
                            S.col(HSG, S.slotP)));
            napply64 += nact;
        }
        BDG_TRY(sync_if());
        BDG_TRY(mark(2));
        // Gram matrices of [F, W, P] (W and P: active columns)
        const int ns = np > 0 ? 3 : 2;
        const int mc = nb + nact + np;
        const int npc = np / 2;
        Seg sf[3] = {{F, nbc}, {Wf, nactc}, {npc ? S.col(SF, S.slotP) : nullptr, npc}};
        Seg sg[3] = {{G, nbc}, {Wg, nactc}, {npc ? S.col(SG, S.slotP) : nullptr, npc}};
        Seg hf[3] = {{HF, nbc}, {HWf, nactc}, {npc ? S.col(HSF, S.slotP) : nullptr, npc}};
        Seg hg[3] = {{HG, nbc}, {HWg, nactc}, {npc ? S.col(HSG, S.slotP) : nullptr, npc}};
        BDG_TRY(grams(sf, sg, hf, hg, ns, mc, w32img));
        BDG_TRY(sync_if());
        BDG_TRY(mark(3));
        const bool f32img = mixed && !refreshed && !force64;
        std::vector<double> om_prev = om;
        bdg_status rst = rayleigh_ritz(c, w, mc, nb, Gf, Gg, Br, Mr, Kr, acoef, bcoef, om,
                                       f32img ? opt.rtol32 : opt.rtol, f32img ? opt.eps32 : opt.eps);
        if (rst == BDG_EBREAKDOWN && recoveries < 8) {
            // projected problem lost definiteness: refresh the basis, drop P, and redo the step
            ++recoveries;
            om = om_prev;
            BDG_TRY(refresh(F, G, HF, HG));
            last_refresh = it;
            S.slotFree2 = S.slotP;     // P is discarded
            S.slotP = -1;
            force64 = force64 || mixed;
            continue;
        }
        if (rst != BDG_OK) { final_status = rst; break; }
        BDG_TRY(mark(4));
        // updates: P_new = [W, P] a[nb:] into the free slot and F_new = F a[:nb] + P_new into
        // W's slot.  Blocks of up to 96 real columns take one fused launch per array, which
        // reads F, W and P once and writes both (F_new over W's rows is row-local); otherwise
        // two launches, P_new first, so that no output overlaps an input.  The two forms
        // differ in rounding order only; the float32 phase's trajectory is sensitive to such
        // differences (on an earlier state of this solver the one-pass form made it end at
        // iteration 41 instead of 80; on the current one it does not)
        const int dst_P = S.slotFree, dst_F = S.slotW;
        const int fmode = update_fuse_mode();
        const bool fuse = nb <= 96 && nbc % 8 == 0 && ((!w32img && fmode >= 1) || fmode == 2);
        for (int a = 0; a < 4; ++a) {
            const Seg* seg = (a == SF) ? sf : (a == SG) ? sg : (a == HSF) ? hf : hg;
            const double2* coef = (a == SF || a == HSF) ? acoef : bcoef;
            if (fuse) {
                BDG_TRY(update_pair_fused(c, nh, seg, ns, nh, coef, mc, nb, nbc, S.col(a, dst_P), nh, S.col(a, dst_F),
                                          nh));
            } else {
                BDG_TRY(update_pair(c, nh, seg + 1, ns - 1, nh, coef, mc, nb, nb, 0.0, S.col(a, dst_P), nh,
                                    S.col(a, dst_P), nh));
                BDG_TRY(update_pair(c, nh, seg, 1, nh, coef, mc, 0, nb, 1.0, S.col(a, dst_P), nh, S.col(a, dst_F),
                                    nh));
            }
        }
        // rotate slot roles
        const int oldF = S.slotF, oldP = S.slotP;
        S.slotF = dst_F;
        S.slotP = dst_P;
        S.slotW = oldF;
        S.slotFree = (oldP >= 0) ? oldP : S.slotFree2;
        S.slotFree2 = -1;
        BDG_TRY(sync_if());
        BDG_TRY(mark(5));
    }
    if (converged) final_status = BDG_OK;
    F = S.col(SF, S.slotF);
    G = S.col(SG, S.slotF);
    // outputs
    const int kk = std::min(k, (int)om.size());
    if (omega_out) for (int j = 0; j < kk; ++j) omega_out[j] = om[j];
    if (res_out) for (int j = 0; j < kk; ++j) res_out[j] = res[j];
    if (iters_out) *iters_out = std::min(it, max_iter);
    if (UV_dev) {
        // exact <f, g> = 1/4 through one real scale per column
        const int kkc = (kk + 1) / 2;
        BDG_TRY(dot_pair(c, nh, kkc, F, G, nh, d_n));
        std::vector<double> fg(2 * kkc);
        BDG_TRY(d2h(c, fg.data(), d_n, fg.size() * sizeof(double)));
        std::vector<double> scl(kk);
        for (int j = 0; j < kk; ++j) {
            const double v = c->hd * fg[j];
            scl[j] = v > 0 ? 1.0 / std::sqrt(4.0 * v) : 0.0;
        }
        BDG_TRY(h2d(c, d_n, scl.data(), kk * sizeof(double)));
        hipLaunchKernelGGL(k_pair_make_uv, grid_cols(nh, kk), dim3(256), 0, c->stream, nh, kk, (const double2*)F,
                           (const double2*)G, (const double*)d_n, (double2*)UV_dev);
        BDG_HIP(c, hipGetLastError());
    }
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    BDG_TRY(collect());
    c->stats[0] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    c->stats[1] = t_phase[1];
    c->stats[2] = t_phase[0];
    c->stats[3] = t_phase[2];
    c->stats[4] = t_phase[3];
    c->stats[5] = t_phase[4];
    c->stats[7] = std::min(it, max_iter);
    c->stats[8] = napply64;
    c->stats[9] = napply32;
    if (final_status == BDG_ENOCONV) return ctx_fail(c, BDG_ENOCONV, "bdg_eigs: iteration limit reached");
    return final_status;
}

}  // namespace

// =====================================================================================
// Complex ground states: the general BdG form (Section 2.1) as a Hermitian pencil
//
// For a complex Phi the coefficients A (Hermitian) and B (symmetric) are complex, the (f, g)
// reduction to two real symmetric operators does not apply, and H = [[T + A, B],
// [-conj B, -(T + conj A)]] is handled through K = sigma_3 H = [[T + A, B], [conj B, T + conj A]],
// Hermitian positive semidefinite at a stable ground state:  H x = w x  <=>  sigma_3 x = (1/w) K x.
// The k smallest positive w are the k largest eigenvalues theta = 1/w of the pencil
// (sigma_3, K), found by a locally optimal block iteration on S = [X, W, P]:
//   Rayleigh-Ritz  pivoted Cholesky of the scaled Gram S^H K S gives S R with R^H S^H K S R = I;
//                  the Hermitian R^H (S^H sigma_3 S) R (shifted to be positive semidefinite) is
//                  diagonalized by the one-sided Jacobi SVD; the nb largest theta are kept;
//   correction     W = T (K x - w sigma_3 x) with the kinetic-potential preconditioner T on
//                  both halves, for the active columns (soft locking as in the real path);
//   deflation      the zero modes z_G = (-i G Phi, conj(-i G Phi)), G in {1, S_z, S_x, S_y},
//                  that K annihilates, and Jordan partners y with K y = sigma_3 z for the
//                  sigma_3-isotropic part of that nullspace; every search direction is made
//                  sigma_3-orthogonal to D = [Z, Y] (x - D (D^H s3 D)^-1 D^H s3 x), which every
//                  eigenvector with w != 0 is;
//   images         K P is recomputed from P every iteration; K X by the recurrence, refreshed
//                  every 25 iterations and before the float64 certification.
// =====================================================================================
namespace {

// zero-mode candidates (-i G Phi, conj(-i G Phi)) for G = 1, S_z, S_x, S_y: 4 (u, v) columns
__global__ void k_candidates_c(long long npts, const double2* __restrict__ phi, double2* __restrict__ out) {
    const double r2 = 0.70710678118654752440;
    const long long nh2 = 6 * npts;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
        const double2 a = phi[p], b = phi[npts + p], d = phi[2 * npts + p];
        double2 g[4][3];
        g[0][0] = a; g[0][1] = b; g[0][2] = d;
        g[1][0] = a; g[1][1] = cmk<double2>(0, 0); g[1][2] = cmk<double2>(-d.x, -d.y);
        g[2][0] = cmk<double2>(r2 * b.x, r2 * b.y);
        g[2][1] = cmk<double2>(r2 * (a.x + d.x), r2 * (a.y + d.y));
        g[2][2] = g[2][0];
        g[3][0] = cmk<double2>(r2 * b.y, -r2 * b.x);                       // -i b / sqrt2
        g[3][1] = cmk<double2>(-r2 * (a.y - d.y), r2 * (a.x - d.x));       // i (a - d) / sqrt2
        g[3][2] = cmk<double2>(-r2 * b.y, r2 * b.x);                       // i b / sqrt2
        for (int c = 0; c < 4; ++c)
            for (int s = 0; s < 3; ++s) {
                const double2 z = g[c][s];
                out[c * nh2 + s * npts + p] = cmk<double2>(z.y, -z.x);          // -i z
                out[c * nh2 + 3 * npts + s * npts + p] = cmk<double2>(z.y, z.x); // conj(-i z)
            }
    }
}

// W(:, t) = K X(:, idx[t]) - w[idx[t]] sigma_3 X(:, idx[t]) (rows >= half get the minus sign of sigma_3)
__global__ void k_pencil_res(long long K, long long half, const double2* __restrict__ KX, const double2* __restrict__ X,
                             long long ld, const double* __restrict__ om, const int* __restrict__ idx,
                             double2* __restrict__ W, long long ldw) {
    const int t = blockIdx.y;
    const long long j = idx[t];
    const double w = om[j];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (long long)gridDim.x * blockDim.x) {
        const double2 kx = KX[j * ld + i], x = X[j * ld + i];
        const double s = i < half ? w : -w;
        W[t * ldw + i] = cmk<double2>(kx.x - s * x.x, kx.y - s * x.y);
    }
}

// A -= B (m x m)
__global__ void k_small_sub(int m, double2* A, int lda, const double2* __restrict__ B, int ldb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= m) return;
    const double2 b = B[(long long)j * ldb + i];
    double2& a = A[(long long)j * lda + i];
    a.x -= b.x;
    a.y -= b.y;
}

// A += s I
__global__ void k_small_shift(int m, double2* A, int lda, double s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) A[(long long)i * lda + i].x += s;
}

// largest pointwise row sum of |[[A, B], [conj B, conj A]]| over the 21 complex-state fields
__global__ void __launch_bounds__(256) k_ccoef_bound(long long npts, const double* __restrict__ cc,
                                                     double* __restrict__ part) {
    __shared__ double red[4];
    double mx = 0;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
        double f[21];
        for (int s = 0; s < 21; ++s) f[s] = cc[s * npts + p];
        const double a01 = hypot(f[3], f[4]), a02 = hypot(f[5], f[6]), a12 = hypot(f[7], f[8]);
        const double b00 = hypot(f[9], f[10]), b01 = hypot(f[11], f[12]), b02 = hypot(f[13], f[14]);
        const double b11 = hypot(f[15], f[16]), b12 = hypot(f[17], f[18]), b22 = hypot(f[19], f[20]);
        const double r0 = fabs(f[0]) + a01 + a02 + b00 + b01 + b02;
        const double r1 = a01 + fabs(f[1]) + a12 + b01 + b11 + b12;
        const double r2 = a02 + a12 + fabs(f[2]) + b02 + b12 + b22;
        mx = fmax(mx, fmax(r0, fmax(r1, r2)));
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

bdg_status applyK(bdg_ctx* c, int ncols, const double2* X, long long nh2, double2* Y) {
    BlockRef<const double2> xr{X, X + nh2 / 2, nh2};
    BlockRef<double2> yr{Y, Y + nh2 / 2, nh2};
    return launch_apply_complex(c, 1, ncols, xr, yr);
}

// small dense helpers on the host (deflation only, q <= 8)
bool host_inverse(int q, std::vector<std::complex<double>>& A) {    // column-major, in place
    std::vector<std::complex<double>> I(q * q, 0.0);
    for (int i = 0; i < q; ++i) I[i * q + i] = 1.0;
    for (int col = 0; col < q; ++col) {
        int piv = col;
        for (int r = col + 1; r < q; ++r)
            if (std::abs(A[col * q + r]) > std::abs(A[col * q + piv])) piv = r;
        if (std::abs(A[col * q + piv]) == 0.0) return false;
        for (int j = 0; j < q; ++j) {
            std::swap(A[j * q + col], A[j * q + piv]);
            std::swap(I[j * q + col], I[j * q + piv]);
        }
        const std::complex<double> d = A[col * q + col];
        for (int j = 0; j < q; ++j) { A[j * q + col] /= d; I[j * q + col] /= d; }
        for (int r = 0; r < q; ++r) {
            if (r == col) continue;
            const std::complex<double> f = A[col * q + r];
            if (f == 0.0) continue;
            for (int j = 0; j < q; ++j) { A[j * q + r] -= f * A[j * q + col]; I[j * q + r] -= f * I[j * q + col]; }
        }
    }
    A = I;
    return true;
}

// Hermitian eigen-decomposition (q <= 8) through the real symmetric matrix
// [[Re A, -Im A], [Im A, Re A]] and cyclic Jacobi rotations; every eigenvalue appears twice
// there, with eigenvectors (x; y) and (-y; x) of the same complex vector x + i y.  Returns
// the 2q real eigenvalues and the complex vectors x + i y (column-major, q x 2q).
void host_heig(int q, const std::vector<std::complex<double>>& A, std::vector<double>& e,
               std::vector<std::complex<double>>& V) {
    const int n = 2 * q;
    std::vector<double> M(n * n), U(n * n, 0.0);
    for (int j = 0; j < q; ++j)
        for (int i = 0; i < q; ++i) {
            const std::complex<double> a = A[j * q + i];
            M[j * n + i] = a.real();
            M[(j + q) * n + (i + q)] = a.real();
            M[(j + q) * n + i] = -a.imag();
            M[j * n + (i + q)] = a.imag();
        }
    for (int i = 0; i < n; ++i) U[i * n + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0, tot = 0;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) { tot += M[j * n + i] * M[j * n + i]; if (i != j) off += M[j * n + i] * M[j * n + i]; }
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < n; ++p)
            for (int r = p + 1; r < n; ++r) {
                const double apr = M[r * n + p];
                if (std::fabs(apr) < 1e-300) continue;
                const double th = (M[r * n + r] - M[p * n + p]) / (2 * apr);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
                const double cs = 1 / std::sqrt(t * t + 1), sn = t * cs;
                // M <- J^T M J with J = I except J_pp = J_rr = cs, J_pr = sn, J_rp = -sn
                for (int k = 0; k < n; ++k) {              // columns p, r
                    const double a = M[p * n + k], b = M[r * n + k];
                    M[p * n + k] = cs * a - sn * b;
                    M[r * n + k] = sn * a + cs * b;
                }
                for (int k = 0; k < n; ++k) {              // rows p, r
                    const double a = M[k * n + p], b = M[k * n + r];
                    M[k * n + p] = cs * a - sn * b;
                    M[k * n + r] = sn * a + cs * b;
                }
                for (int k = 0; k < n; ++k) {
                    const double a = U[p * n + k], b = U[r * n + k];
                    U[p * n + k] = cs * a - sn * b;
                    U[r * n + k] = sn * a + cs * b;
                }
            }
    }
    e.resize(n);
    V.assign(q * n, 0.0);
    for (int j = 0; j < n; ++j) {
        e[j] = M[j * n + j];
        for (int i = 0; i < q; ++i) V[j * q + i] = {U[j * n + i], U[j * n + i + q]};
    }
}

struct PencilDefl {
    double2* D = nullptr;      // nh2 x q: [Z, partners]
    int q = 0;
    double2* Finv = nullptr;   // q x q: (D^H sigma_3 D)^-1
    int pz = 0;                // zero modes, partners = q - pz
};

// C (q x n) = h^d (Y_u^H X_u - Y_v^H X_v): sigma_3 Gram of two column blocks
bdg_status gram_sigma(bdg_ctx* c, Small& w, long long npts, const double2* Y, int q, const double2* X, int n,
                      double2* C, int ldc, int herm) {
    const long long nh2 = 6 * npts, hf = 3 * npts;
    BDG_TRY(gram<double2, double2>(c, hf, q, n, Y, nh2, X, nh2, c->hd, C, ldc, herm));
    double2* T = w.buf[13];
    BDG_TRY(gram<double2, double2>(c, hf, q, n, Y + hf, nh2, X + hf, nh2, c->hd, T, ldc, herm));
    hipLaunchKernelGGL(k_small_sub, dim3((unsigned)((q + 127) / 128), (unsigned)n), dim3(128), 0, c->stream, q, C, ldc,
                       (const double2*)T, ldc);
    return hip_check(c, hipGetLastError(), "k_small_sub");
}

// X -= D (D^H s3 D)^-1 D^H s3 X for ncols columns
bdg_status project_sigma(bdg_ctx* c, Small& w, long long npts, const PencilDefl& d, double2* X, int ncols) {
    if (d.q == 0 || ncols == 0) return BDG_OK;
    const long long nh2 = 6 * npts;
    double2* C = w.buf[11];
    double2* C2 = w.buf[12];
    BDG_TRY(gram_sigma(c, w, npts, d.D, d.q, X, ncols, C, d.q, 0));
    const double2 MONE = {-1.0, 0.0}, Z0 = {0.0, 0.0};
    BDG_TRY(small_gemm(c, 0, 0, d.q, ncols, d.q, MONE, d.Finv, d.q, C, d.q, Z0, C2, d.q));
    Seg s{d.D, d.q};
    return update_add(c, nh2, &s, 1, nh2, C2, d.q, ncols, 1.0, X, nh2, X, nh2);
}

bdg_status pcg_k(bdg_ctx* c, Small& w, long long nh2, const double2* Z, int pz, const double2* b, double2* x,
                 double2* ws, double tol, int max_iter) {
    double2* r = ws;
    double2* z = ws + nh2;
    double2* p = ws + 2 * nh2;
    double2* Ap = ws + 3 * nh2;
    const dim3 g1 = grid_cols(nh2, 1);
    BDG_HIP(c, hipMemsetAsync(x, 0, nh2 * sizeof(double2), c->stream));
    BDG_HIP(c, hipMemcpyAsync(r, b, nh2 * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
    BDG_TRY(project_out(c, w, nh2, Z, pz, r, 1));
    BDG_TRY(launch_precond<double>(c, 6, 6, nh2, r, z));
    BDG_TRY(project_out(c, w, nh2, Z, pz, z, 1));
    BDG_HIP(c, hipMemcpyAsync(p, z, nh2 * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
    bdg_status st;
    double rz = host_dot_re(c, w, nh2, z, r, &st);
    BDG_TRY(st);
    const double bnorm = std::sqrt(std::max(0.0, host_dot_re(c, w, nh2, r, r, &st)));
    BDG_TRY(st);
    if (bnorm == 0) return BDG_OK;
    for (int it = 0; it < max_iter; ++it) {
        BDG_TRY(applyK(c, 1, p, nh2, Ap));
        BDG_TRY(project_out(c, w, nh2, Z, pz, Ap, 1));
        const double pAp = host_dot_re(c, w, nh2, Ap, p, &st);
        BDG_TRY(st);
        if (!(pAp > 0)) return ctx_fail(c, BDG_EBREAKDOWN, "Jordan-partner solve: K not positive");
        const double alpha = rz / pAp;
        hipLaunchKernelGGL(k_axpy, g1, dim3(256), 0, c->stream, nh2, cmk<double2>(alpha, 0.0), (const double2*)p, x);
        hipLaunchKernelGGL(k_axpy, g1, dim3(256), 0, c->stream, nh2, cmk<double2>(-alpha, 0.0), (const double2*)Ap, r);
        const double rn = std::sqrt(std::max(0.0, host_dot_re(c, w, nh2, r, r, &st)));
        BDG_TRY(st);
        if (rn <= tol * bnorm) return BDG_OK;
        BDG_TRY(launch_precond<double>(c, 6, 6, nh2, r, z));
        BDG_TRY(project_out(c, w, nh2, Z, pz, z, 1));
        const double rz_new = host_dot_re(c, w, nh2, z, r, &st);
        BDG_TRY(st);
        hipLaunchKernelGGL(k_xpby, g1, dim3(256), 0, c->stream, nh2, (const double2*)z, cmk<double2>(rz_new / rz, 0.0), p);
        rz = rz_new;
    }
    return ctx_fail(c, BDG_ENOCONV, "Jordan-partner solve did not converge");
}

bdg_status build_pencil_deflation(bdg_ctx* c, Small& w, PencilDefl& d, double null_tol) {
    const long long npts = c->npts, nh2 = 6 * npts;
    double2* cand = nullptr;
    double2* img = nullptr;
    double2* ws = nullptr;
    auto release = defer([&] { ctx_free(c, cand); ctx_free(c, img); ctx_free(c, ws); });
    BDG_TRY(ctx_alloc(c, (void**)&cand, 4 * nh2 * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&img, 4 * nh2 * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&ws, 4 * nh2 * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&d.D, 8 * nh2 * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&d.Finv, 64 * sizeof(double2)));
    hipLaunchKernelGGL(k_candidates_c, dim3(1024), dim3(256), 0, c->stream, npts, (const double2*)c->phic, cand);
    BDG_HIP(c, hipGetLastError());
    BDG_TRY(applyK(c, 4, cand, nh2, img));
    double nc[4], nk[4];
    BDG_TRY(colnorm2(c, nh2, 4, cand, nh2, w.s[0]));
    BDG_TRY(colnorm2(c, nh2, 4, img, nh2, w.s[1]));
    BDG_TRY(d2h(c, nc, w.s[0], 4 * sizeof(double)));
    BDG_TRY(d2h(c, nk, w.s[1], 4 * sizeof(double)));
    const double cmax = std::max(std::max(nc[0], nc[1]), std::max(nc[2], nc[3]));
    int kz = 0;
    for (int j = 0; j < 4; ++j)
        if (nc[j] > 1e-24 * cmax && std::sqrt(nk[j]) <= null_tol * std::sqrt(nc[j])) {
            if (kz != j)
                BDG_HIP(c, hipMemcpyAsync(cand + kz * nh2, cand + j * nh2, nh2 * sizeof(double2), hipMemcpyDeviceToDevice,
                                          c->stream));
            ++kz;
        }
    BDG_TRY(orthonormalize(c, w, nh2, cand, kz, d.D, 1e-10, &d.pz));
    // sigma_3-isotropic part of the nullspace: eigenvectors of E = Z^H s3 Z with |e| small
    int ps = 0;
    if (d.pz > 0) {
        const int pz = d.pz;
        double2* E = w.buf[10];
        BDG_TRY(gram_sigma(c, w, npts, d.D, pz, d.D, pz, E, pz, 0));
        std::vector<double2> eh(pz * pz);
        BDG_TRY(d2h(c, eh.data(), E, eh.size() * sizeof(double2)));
        std::vector<std::complex<double>> Ec(pz * pz), Vc;
        for (int i = 0; i < pz * pz; ++i) Ec[i] = {eh[i].x, eh[i].y};
        for (int j = 0; j < pz; ++j)
            for (int i = 0; i < j; ++i) {
                const std::complex<double> h = 0.5 * (Ec[j * pz + i] + std::conj(Ec[i * pz + j]));
                Ec[j * pz + i] = h;
                Ec[i * pz + j] = std::conj(h);
            }
        std::vector<double> ev;
        host_heig(pz, Ec, ev, Vc);
        // isotropic eigenvectors (|e| small), each complex vector kept once (Gram-Schmidt)
        std::vector<std::vector<std::complex<double>>> iso;
        for (int i = 0; i < 2 * pz; ++i) {
            if (std::fabs(ev[i]) > 1e-6) continue;
            std::vector<std::complex<double>> v(Vc.begin() + i * pz, Vc.begin() + (i + 1) * pz);
            for (const auto& u : iso) {
                std::complex<double> dot = 0;
                for (int r = 0; r < pz; ++r) dot += std::conj(u[r]) * v[r];
                for (int r = 0; r < pz; ++r) v[r] -= dot * u[r];
            }
            double nv = 0;
            for (int r = 0; r < pz; ++r) nv += std::norm(v[r]);
            if (nv < 0.25) continue;
            for (int r = 0; r < pz; ++r) v[r] /= std::sqrt(nv);
            iso.push_back(v);
        }
        std::vector<double2> src;
        for (const auto& v : iso)
            for (int r = 0; r < pz; ++r) src.push_back(double2{v[r].real(), v[r].imag()});
        ps = (int)iso.size();
        if (ps > 0) {
            // sources sigma_3 Z v: combine, then negate the v half
            double2* Cv = w.buf[9];
            BDG_TRY(h2d(c, Cv, src.data(), src.size() * sizeof(double2)));
            Seg sz{d.D, pz};
            BDG_TRY(update(c, nh2, &sz, 1, nh2, Cv, pz, ps, 0.0, img, nh2));
            const double mone = -1.0;
            BDG_TRY(h2d(c, w.s[2], &mone, sizeof(double)));
            for (int j = 0; j < ps; ++j)
                hipLaunchKernelGGL(k_cols_scale, grid_cols(3 * npts, 1), dim3(256), 0, c->stream, 3 * npts, 1,
                                   img + j * nh2 + 3 * npts, nh2, (const double*)w.s[2], 0);
            BDG_HIP(c, hipGetLastError());
            for (int j = 0; j < ps; ++j)
                BDG_TRY(pcg_k(c, w, nh2, d.D, pz, img + j * nh2, d.D + (pz + j) * nh2, ws, 1e-13, 5000));
        }
    }
    d.q = d.pz + ps;
    if (d.q > 0) {
        double2* Fm = w.buf[10];
        BDG_TRY(gram_sigma(c, w, npts, d.D, d.q, d.D, d.q, Fm, d.q, 0));
        std::vector<double2> fh(d.q * d.q);
        BDG_TRY(d2h(c, fh.data(), Fm, fh.size() * sizeof(double2)));
        std::vector<std::complex<double>> Fc(d.q * d.q);
        for (int i = 0; i < d.q * d.q; ++i) Fc[i] = {fh[i].x, fh[i].y};
        if (!host_inverse(d.q, Fc)) return ctx_fail(c, BDG_EBREAKDOWN, "deflation: singular sigma_3 Gram");
        for (int i = 0; i < d.q * d.q; ++i) fh[i] = double2{Fc[i].real(), Fc[i].imag()};
        BDG_TRY(h2d(c, d.Finv, fh.data(), fh.size() * sizeof(double2)));
    }
    if (debug_on()) fprintf(stderr, "[bdg pencil deflation] zero modes %d, partners %d\n", d.pz, ps);
    return BDG_OK;
}

bdg_status eigs_pencil_impl(bdg_ctx* c, int k, int nb, double tol, int max_iter, const void* X0_dev,
                            unsigned long long seed, double* omega_out, void* UV_dev, double* res_out, int* iters_out) {
    const long long npts = c->npts, nh2 = 6 * npts, half = 3 * npts;
    const int m = 3 * nb;
    auto t_start = std::chrono::steady_clock::now();
    for (double& s : c->stats) s = 0;
    Small w;
    double2* arr[2] = {nullptr, nullptr};    // S, K S: 4 slots of nb columns each
    double2* acoef = nullptr;
    double* dvec = nullptr;
    int* d_act = nullptr;
    PencilDefl D;
    auto release = defer([&] {
        small_free(c, w);
        ctx_free(c, arr[0]);
        ctx_free(c, arr[1]);
        ctx_free(c, acoef);
        ctx_free(c, dvec);
        ctx_free(c, d_act);
        ctx_free(c, D.D);
        ctx_free(c, D.Finv);
    });
    BDG_TRY(small_alloc(c, w, std::max(m, 8)));
    for (int a = 0; a < 2; ++a) BDG_TRY(ctx_alloc(c, (void**)&arr[a], 4 * (size_t)nb * nh2 * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&acoef, (size_t)m * nb * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&dvec, 8 * (size_t)nb * sizeof(double)));
    BDG_TRY(ctx_alloc(c, (void**)&d_act, (size_t)nb * sizeof(int)));
    auto col = [&](int a, int slot) { return arr[a] + (long long)slot * nb * nh2; };
    double* d_om = dvec;
    double* d_n = dvec + nb;         // 2 nb norms
    // Per-column target max(tol, floor_c eps ||H|| / |w|) as in the real path; after
    // stall_limit iterations without halving the largest residual the iteration stops with
    // BDG_ENOCONV and the last iterate.
    const double null_tol = 1e-6, rtol = 1e-12, floor_c = 100.0;
    const int stall_limit = 100;
    double best_r = 1e300;
    int best_it = 0;
    BDG_TRY(build_pencil_deflation(c, w, D, null_tol));
    // ||H|| bound for the rounding floor of the relative residual
    double hbound = 0;
    {
        double kin = 0;
        for (int a = 0; a < c->dim; ++a) {
            const double kmax = M_PI * c->n[a] / (2.0 * c->L[a]);
            kin += 0.5 * kmax * kmax;
        }
        double* part = w.s[3];
        const int NBK = std::min(256, std::max(w.cap, 8));
        hipLaunchKernelGGL(k_ccoef_bound, dim3(NBK), dim3(256), 0, c->stream, npts, (const double*)c->ccoef, part);
        BDG_TRY(hip_check(c, hipGetLastError(), "k_ccoef_bound"));
        std::vector<double> hp(NBK);
        BDG_TRY(d2h(c, hp.data(), part, NBK * sizeof(double)));
        double mx = 0;
        for (double v : hp) mx = std::max(mx, v);
        hbound = kin + mx;
    }
    c->stats[6] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    int slotX = 0, slotW = 1, slotP = -1, slotFree = 2, slotFree2 = 3;
    double2* X = col(0, slotX);
    if (X0_dev) {
        BDG_HIP(c, hipMemcpyAsync(X, X0_dev, (size_t)nb * nh2 * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
    } else {
        hipLaunchKernelGGL(k_randn, dim3(2048), dim3(256), 0, c->stream, (long long)nb * nh2, seed, X);
        BDG_HIP(c, hipGetLastError());
    }
    BDG_TRY(project_sigma(c, w, npts, D, X, nb));
    BDG_TRY(applyK(c, nb, X, nh2, col(1, slotX)));
    std::vector<double> om(nb, 1.0), res(nb, 1.0), hn(2 * nb);
    auto target = [&](int j) { return std::max(tol, floor_c * DBL_EPSILON * hbound / std::fabs(om[j])); };
    double2* Gk = w.buf[0];
    double2* Gs = w.buf[1];
    double2* R = w.buf[2];
    double2* T = w.buf[3];
    double2* Mm = w.buf[4];
    double2* Vv = w.buf[5];
    const double2 ONE_ = {1.0, 0.0}, ZERO_ = {0.0, 0.0};
    // Rayleigh-Ritz on segments; writes the nb coefficient columns to acoef (ld mc) and om
    auto rr = [&](const Seg* ss, const Seg* ks, int ns, int mc) -> bdg_status {
        BDG_TRY(gram_seg(c, nh2, ss, ns, nh2, ks, ns, nh2, c->hd, Gk, mc, 1));
        BDG_TRY(gram_seg(c, half, ss, ns, nh2, ss, ns, nh2, c->hd, Gs, mc, 1));
        Seg sv[3];
        for (int i = 0; i < ns; ++i) sv[i] = Seg{ss[i].p ? (const void*)((const double2*)ss[i].p + half) : nullptr, ss[i].ncols};
        BDG_TRY(gram_seg(c, half, sv, ns, nh2, sv, ns, nh2, c->hd, T, mc, 1));
        hipLaunchKernelGGL(k_small_sub, dim3((unsigned)((mc + 127) / 128), (unsigned)mc), dim3(128), 0, c->stream, mc, Gs,
                           mc, (const double2*)T, mc);
        BDG_HIP(c, hipGetLastError());
        BDG_TRY(small_pchol_orth(c, mc, Gk, mc, rtol, R, w.info + 2));
        int r = 0;
        BDG_TRY(d2h(c, &r, w.info + 2, sizeof(int)));
        if (r < nb) return ctx_fail(c, BDG_EBREAKDOWN, "bdg_eigs: basis rank below block size");
        BDG_TRY(small_gemm(c, 0, 0, mc, r, mc, ONE_, Gs, mc, R, mc, ZERO_, T, mc));
        BDG_TRY(small_gemm(c, 1, 0, r, r, mc, ONE_, R, mc, T, mc, ZERO_, Mm, mc));
        hipLaunchKernelGGL(k_small_herm, dim3((unsigned)((r + 127) / 128), (unsigned)r), dim3(128), 0, c->stream, r, Mm, mc);
        BDG_TRY(colnorm2(c, r, r, Mm, mc, w.s[0]));
        std::vector<double> cn(r);
        BDG_TRY(d2h(c, cn.data(), w.s[0], r * sizeof(double)));
        double fro = 0;
        for (double v : cn) fro += v;
        const double shift = std::sqrt(fro) * (1.0 + 1e-12) + 1e-300;
        hipLaunchKernelGGL(k_small_shift, dim3((unsigned)((r + 127) / 128)), dim3(128), 0, c->stream, r, Mm, mc, shift);
        BDG_HIP(c, hipGetLastError());
        // the shifted matrix's eigenvectors must resolve gaps of 1/w against a shift of order
        // max 1/w: converge the rotations to the rounding level
        BDG_TRY(small_svd(c, r, r, Mm, mc, Vv, mc, w.s[1], 1e-15));
        std::vector<double> sv_(r);
        BDG_TRY(d2h(c, sv_.data(), w.s[1], r * sizeof(double)));
        for (int j = 0; j < nb; ++j) {
            const double th = sv_[j] - shift;
            om[j] = th > 0 ? 1.0 / th : 1.0 / std::max(std::fabs(th), 1e-300);
        }
        BDG_TRY(small_gemm(c, 0, 0, mc, nb, r, ONE_, R, mc, Vv, mc, ZERO_, acoef, mc));
        return BDG_OK;
    };
    {
        Seg sx{X, nb}, kx{col(1, slotX), nb};
        BDG_TRY(rr(&sx, &kx, 1, nb));
        for (int a = 0; a < 2; ++a) {
            Seg src{col(a, slotX), nb};
            BDG_TRY(update(c, nh2, &src, 1, nh2, acoef, nb, nb, 0.0, col(a, slotW), nh2));
        }
        std::swap(slotX, slotW);
    }
    int it = 0, last_refresh = 0, certifications = 0;
    bool converged = false;
    bdg_status final_status = BDG_ENOCONV;
    std::vector<int> act, all(nb);
    for (int j = 0; j < nb; ++j) all[j] = j;
    for (it = 1; it <= max_iter; ++it) {
        X = col(0, slotX);
        double2* KX = col(1, slotX);
        double2* Wx = col(0, slotW);
        double2* Wk = col(1, slotW);
        if (it - last_refresh >= 25) {
            BDG_TRY(project_sigma(c, w, npts, D, X, nb));
            BDG_TRY(applyK(c, nb, X, nh2, KX));
            last_refresh = it;
        }
        // residual K x - w s3 x of every column (into the W slot), its norm and |x|
        BDG_TRY(h2d(c, d_om, om.data(), nb * sizeof(double)));
        BDG_TRY(h2d(c, d_act, all.data(), nb * sizeof(int)));
        hipLaunchKernelGGL(k_pencil_res, grid_cols(nh2, nb), dim3(256), 0, c->stream, nh2, half, (const double2*)KX,
                           (const double2*)X, nh2, (const double*)d_om, (const int*)d_act, Wx, nh2);
        BDG_HIP(c, hipGetLastError());
        BDG_TRY(colnorm2(c, nh2, nb, Wx, nh2, d_n));
        BDG_TRY(colnorm2(c, nh2, nb, X, nh2, d_n + nb));
        BDG_TRY(d2h(c, hn.data(), d_n, 2 * nb * sizeof(double)));
        act.clear();
        bool all_k = true;
        double rmax = 0;
        for (int j = 0; j < nb; ++j) {
            res[j] = std::sqrt(hn[j]) / (std::fabs(om[j]) * std::sqrt(hn[nb + j]));
            const bool done = res[j] <= target(j);
            if (j < k) { all_k = all_k && done; rmax = std::max(rmax, res[j]); }
            if (!done) act.push_back(j);
        }
        if (!(rmax == rmax)) return ctx_fail(c, BDG_EBREAKDOWN, "non-finite residual");
        if (rmax < 0.5 * best_r) { best_r = rmax; best_it = it; }
        if (it - best_it > stall_limit) break;
        if (debug_on())
            fprintf(stderr, "[bdg pencil it %d] omega0=%.12f omega_k=%.12f res_max(k)=%.3e active=%d\n", it, om[0],
                    om[k - 1], rmax, (int)act.size());
        if (all_k || act.empty()) {
            // certify with an explicit apply
            BDG_TRY(applyK(c, nb, X, nh2, KX));
            last_refresh = it;
            hipLaunchKernelGGL(k_pencil_res, grid_cols(nh2, nb), dim3(256), 0, c->stream, nh2, half, (const double2*)KX,
                               (const double2*)X, nh2, (const double*)d_om, (const int*)d_act, Wx, nh2);
            BDG_TRY(colnorm2(c, nh2, nb, Wx, nh2, d_n));
            BDG_TRY(d2h(c, hn.data(), d_n, nb * sizeof(double)));
            bool ok = true;
            for (int j = 0; j < nb; ++j) {
                res[j] = std::sqrt(hn[j]) / (std::fabs(om[j]) * std::sqrt(hn[nb + j]));
                if (j < k) ok = ok && res[j] <= target(j);
            }
            if (ok) { converged = true; break; }
            if (++certifications > 4) break;
            --it;
            continue;
        }
        const int nact = (int)act.size();
        // active residuals into the free slot, preconditioned, made s3-orthogonal to D
        BDG_TRY(h2d(c, d_act, act.data(), nact * sizeof(int)));
        double2* Wa = col(0, slotFree);
        hipLaunchKernelGGL(k_cols_gather, grid_cols(nh2, nact), dim3(256), 0, c->stream, nh2, (const double2*)Wx, nh2,
                           (const int*)d_act, Wa, nh2);
        BDG_HIP(c, hipGetLastError());
        BDG_TRY(launch_precond<double>(c, 6 * nact, 6, nh2, Wa, Wa));
        BDG_TRY(project_sigma(c, w, npts, D, Wa, nact));
        std::swap(slotW, slotFree);
        Wx = col(0, slotW);
        Wk = col(1, slotW);
        BDG_TRY(applyK(c, nact, Wx, nh2, Wk));
        // remove X from W in the K inner product (X^H K X = I for the Ritz basis), twice: with
        // a preconditioner close to K^-1 a correction is mostly X plus a small new part, which
        // the rank cut of the K Gram would otherwise discard as the residual shrinks
        for (int pass = 0; pass < 2; ++pass) {
            double2* Cx = w.buf[6];
            BDG_TRY(gram<double2, double2>(c, nh2, nb, nact, KX, nh2, Wx, nh2, -c->hd, Cx, nb, 0));
            Seg sx{X, nb}, skx{KX, nb};
            BDG_TRY(update_add(c, nh2, &sx, 1, nh2, Cx, nb, nact, 1.0, Wx, nh2, Wx, nh2));
            BDG_TRY(update_add(c, nh2, &skx, 1, nh2, Cx, nb, nact, 1.0, Wk, nh2, Wk, nh2));
        }
        // unit columns: the corrections shrink with the residual, and beside the Ritz columns
        // (K norm about w) a column of K norm about res sqrt(w / shift) falls under the K
        // Gram's relative cut of 1e-20 on the squared norms once res nears 1e-9
        BDG_TRY(colnorm2(c, nh2, nact, Wx, nh2, w.dscale));
        hipLaunchKernelGGL(k_cols_scale, grid_cols(nh2, nact), dim3(256), 0, c->stream, nh2, nact, Wx, nh2,
                           (const double*)w.dscale, 1);
        hipLaunchKernelGGL(k_cols_scale, grid_cols(nh2, nact), dim3(256), 0, c->stream, nh2, nact, Wk, nh2,
                           (const double*)w.dscale, 1);
        BDG_HIP(c, hipGetLastError());
        // P of the active columns, unit columns, with explicit images
        int np = 0;
        if (slotP >= 0) {
            np = nact;
            if (nact < nb) {
                hipLaunchKernelGGL(k_cols_gather, grid_cols(nh2, nact), dim3(256), 0, c->stream, nh2,
                                   (const double2*)col(0, slotP), nh2, (const int*)d_act, col(0, slotFree), nh2);
                BDG_HIP(c, hipGetLastError());
                std::swap(slotP, slotFree);
            }
            BDG_TRY(colnorm2(c, nh2, np, col(0, slotP), nh2, w.dscale));
            hipLaunchKernelGGL(k_cols_scale, grid_cols(nh2, np), dim3(256), 0, c->stream, nh2, np, col(0, slotP), nh2,
                               (const double*)w.dscale, 1);
            BDG_HIP(c, hipGetLastError());
            BDG_TRY(applyK(c, np, col(0, slotP), nh2, col(1, slotP)));
        }
        const int ns = np ? 3 : 2;
        const int mc = nb + nact + np;
        Seg ss[3] = {{X, nb}, {Wx, nact}, {np ? col(0, slotP) : nullptr, np}};
        Seg ks[3] = {{KX, nb}, {Wk, nact}, {np ? col(1, slotP) : nullptr, np}};
        bdg_status rst = rr(ss, ks, ns, mc);
        if (rst != BDG_OK) { final_status = rst; break; }
        // P_new = [W, P] a[nb:] into the free slot, X_new = X a[:nb] + P_new into W's slot
        const int dst_P = slotFree, dst_X = slotW;
        for (int a = 0; a < 2; ++a) {
            const Seg* seg = a == 0 ? ss : ks;
            BDG_TRY(update(c, nh2, seg + 1, ns - 1, nh2, acoef + nb, mc, nb, 0.0, col(a, dst_P), nh2));
        }
        for (int a = 0; a < 2; ++a) {
            const Seg* seg = a == 0 ? ss : ks;
            BDG_TRY(update_add(c, nh2, seg, 1, nh2, acoef, mc, nb, 1.0, col(a, dst_P), nh2, col(a, dst_X), nh2));
        }
        const int oldX = slotX, oldP = slotP;
        slotX = dst_X;
        slotP = dst_P;
        slotW = oldX;
        slotFree = oldP >= 0 ? oldP : slotFree2;
        slotFree2 = -1;
        if (slotFree < 0) slotFree = 6 - slotX - slotP - slotW;   // the one slot left of 0..3
    }
    if (converged) final_status = BDG_OK;
    X = col(0, slotX);
    const int kk = std::min(k, nb);
    if (omega_out) for (int j = 0; j < kk; ++j) omega_out[j] = om[j];
    if (res_out) for (int j = 0; j < kk; ++j) res_out[j] = res[j];
    if (iters_out) *iters_out = std::min(it, max_iter);
    if (UV_dev) {
        // int |u|^2 - |v|^2 = 1 per column
        BDG_TRY(colnorm2(c, half, kk, X, nh2, w.s[0]));
        BDG_TRY(colnorm2(c, half, kk, X + half, nh2, w.s[1]));
        std::vector<double> nu(kk), nv(kk), scl(kk);
        BDG_TRY(d2h(c, nu.data(), w.s[0], kk * sizeof(double)));
        BDG_TRY(d2h(c, nv.data(), w.s[1], kk * sizeof(double)));
        for (int j = 0; j < kk; ++j) {
            const double q = c->hd * (nu[j] - nv[j]);
            scl[j] = q > 0 ? 1.0 / std::sqrt(q) : 0.0;
        }
        BDG_TRY(h2d(c, w.s[2], scl.data(), kk * sizeof(double)));
        BDG_HIP(c, hipMemcpyAsync(UV_dev, X, (size_t)kk * nh2 * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
        hipLaunchKernelGGL(k_cols_scale, grid_cols(nh2, kk), dim3(256), 0, c->stream, nh2, kk, (double2*)UV_dev, nh2,
                           (const double*)w.s[2], 0);
        BDG_HIP(c, hipGetLastError());
    }
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    c->stats[0] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    c->stats[7] = std::min(it, max_iter);
    if (final_status == BDG_ENOCONV) return ctx_fail(c, BDG_ENOCONV, "bdg_eigs: iteration limit reached");
    return final_status;
}

}  // namespace

extern "C" bdg_status bdg_eigs(bdg_ctx* c, int k, int block, double tol, int max_iter, const void* X0_dev,
                               unsigned long long seed, double* omega, void* UV_dev, double* residual, int* iters) {
    if (!c) return BDG_EINVAL;
    // each half (f or g) lives in 3 npts dimensions minus at most 4 deflated directions
    if (k < 1 || block < k || block > 160 || (long long)block > 3 * c->npts - 4)
        return ctx_fail(c, BDG_EINVAL, "bdg_eigs: need 1 <= k <= block <= min(160, 3 npts - 4)");
    if (!(tol > 0) || max_iter < 1) return ctx_fail(c, BDG_EINVAL, "bdg_eigs: bad tol or max_iter");
    if (!omega) return ctx_fail(c, BDG_EINVAL, "bdg_eigs: omega is null");
    if (!c->has_gs) return ctx_fail(c, BDG_ESTATE, "bdg_eigs: no ground state set");
    if (c->complex_gs) return eigs_pencil_impl(c, k, block, tol, max_iter, X0_dev, seed, omega, UV_dev, residual, iters);
    return eigs_impl(c, k, block, tol, max_iter, X0_dev, seed, omega, UV_dev, residual, iters);
}

// =====================================================================================
// bdg_eigs_grad: eigenvalue gradients (Hellmann-Feynman form plus the ground-state
// sensitivity through the linearized Euler-Lagrange problem of Section 1)
//
// With the left eigenvector (g, f) of [[0, H_-], [H_+, 0]] (the matrix J H = diag(H_+, H_-)
// is Hermitian), d omega = (<dH_+ f, f> + <dH_- g, g>) / (2 Re <f, g>).  H_+- depend on a
// parameter theta explicitly (V, beta_n, beta_s) and through Phi and Lambda = mu + lambda S_z.
// The real-direction linearization of H(Phi) Phi - Lambda Phi is H_+, so the ground-state
// sensitivity solves the bordered system
//   H_+ dPhi - dmu Phi - dlambda S_z Phi = -d_theta(H Phi),  <Phi, dPhi> = <S_z Phi, dPhi> = 0.
// The implicit part of d omega is <q, dPhi> + a_mu dmu + a_lambda dlambda with
//   q = s grad_Phi (f^H C_+(Phi) f + g^H C_-(Phi) g),  a_mu = -s (|f|^2 + |g|^2),
//   a_lambda = -s (<S_z f, f> + <S_z g, g>),  s = 1 / (2 Re <f, g>),
// and the adjoint y (H_+ y + e_1 Phi + e_2 S_z Phi = q, <Phi, y> = -a_mu,
// <S_z Phi, y> = -a_lambda) turns it into -<y, d_theta(H Phi)>:
//   d omega / d V(x) / h^d = s sum_c (|f_c|^2 + |g_c|^2)(x) - sum_c y_c(x) Phi_c(x),
//   d omega / d beta_n = s (<(rho + 2 Phi Phi^T) f, f> + <rho g, g>) - <y, rho Phi>,
//   d omega / d beta_s = s (<(S.s + 2 x x^T + 2 z z^T) f, f> + <(S.s + 2 k k^T) g, g>) - <y, (S.s) Phi>
// with x = S_x Phi, z = S_z Phi, k = K Phi.
// =====================================================================================
namespace {

constexpr int RB2 = 256;

template <int NQ> __device__ void reduce_store(double (&v)[NQ], double* part) {
    __shared__ double red[NQ][RB2 / 64];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = v[q];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = s;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        double a = 0;
        for (int w = 0; w < RB2 / 64; ++w) a += red[threadIdx.x][w];
        part[threadIdx.x * gridDim.x + blockIdx.x] = a;
    }
}

__global__ void k_sum_parts(int nq, int nblk, const double* __restrict__ part, double scale, double* out) {
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

// per point: densities, q field (unscaled), and the sums
//   0: Re<f,g>, 1: <(rho+2PP^T)f,f> + <rho g,g>, 2: beta_s explicit form, 3: |f|^2+|g|^2,
//   4: <S_z f,f> + <S_z g,g>
__global__ void __launch_bounds__(RB2) k_grad_fields(long long npts, const double* __restrict__ phi,
                                                     const double2* __restrict__ uv, double bn, double bs,
                                                     double* __restrict__ dens, double2* __restrict__ qout,
                                                     double* part) {
    const double r2 = 0.70710678118654752440;
    double acc[5] = {0, 0, 0, 0, 0};
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
        const double P[3] = {phi[p], phi[npts + p], phi[2 * npts + p]};
        double2 F[3], G[3];
        for (int c = 0; c < 3; ++c) {
            const double2 u = uv[c * npts + p], v = uv[(3 + c) * npts + p];
            F[c] = cmk<double2>(0.5 * (u.x + v.x), 0.5 * (u.y + v.y));
            G[c] = cmk<double2>(0.5 * (u.x - v.x), 0.5 * (u.y - v.y));
        }
        const double rho = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
        const double sx = 1.4142135623730950488 * P[1] * (P[0] + P[2]), sz = P[0] * P[0] - P[2] * P[2];
        // real symmetric matrices applied to complex vectors
        auto Sx = [&](const double2* a, double2* o) {
            o[0] = cmk<double2>(r2 * a[1].x, r2 * a[1].y);
            o[1] = cmk<double2>(r2 * (a[0].x + a[2].x), r2 * (a[0].y + a[2].y));
            o[2] = cmk<double2>(r2 * a[1].x, r2 * a[1].y);
        };
        auto Sz = [&](const double2* a, double2* o) { o[0] = a[0]; o[1] = cmk<double2>(0, 0); o[2] = cmk<double2>(-a[2].x, -a[2].y); };
        auto Kt = [&](const double2* a, double2* o) {   // K^T a, K = [[0,-1,0],[1,0,-1],[0,1,0]]/sqrt2
            o[0] = cmk<double2>(r2 * a[1].x, r2 * a[1].y);
            o[1] = cmk<double2>(r2 * (-a[0].x + a[2].x), r2 * (-a[0].y + a[2].y));
            o[2] = cmk<double2>(-r2 * a[1].x, -r2 * a[1].y);
        };
        auto dotr = [&](const double* a, const double2* b) {   // a^T b (a real)
            return cmk<double2>(a[0] * b[0].x + a[1] * b[1].x + a[2] * b[2].x, a[0] * b[0].y + a[1] * b[1].y + a[2] * b[2].y);
        };
        auto herm = [&](const double2* a, const double2* b) {   // a^H b, real part
            return a[0].x * b[0].x + a[0].y * b[0].y + a[1].x * b[1].x + a[1].y * b[1].y + a[2].x * b[2].x + a[2].y * b[2].y;
        };
        double2 SxF[3], SzF[3], SxG[3], SzG[3], KtG[3];
        Sx(F, SxF); Sz(F, SzF); Sx(G, SxG); Sz(G, SzG); Kt(G, KtG);
        const double nF = herm(F, F), nG = herm(G, G);
        const double2 pF = dotr(P, F), pxF = dotr(P, SxF), pzF = dotr(P, SzF), pkG = dotr(P, KtG);
        const double fSxf = herm(F, SxF), fSzf = herm(F, SzF), gSxg = herm(G, SxG), gSzg = herm(G, SzG);
        const double a2F = pF.x * pF.x + pF.y * pF.y, ax2 = pxF.x * pxF.x + pxF.y * pxF.y;
        const double az2 = pzF.x * pzF.x + pzF.y * pzF.y, ak2 = pkG.x * pkG.x + pkG.y * pkG.y;
        acc[0] += F[0].x * G[0].x + F[0].y * G[0].y + F[1].x * G[1].x + F[1].y * G[1].y + F[2].x * G[2].x + F[2].y * G[2].y;
        acc[1] += rho * nF + 2.0 * a2F + rho * nG;
        acc[2] += sx * fSxf + sz * fSzf + 2.0 * ax2 + 2.0 * az2 + sx * gSxg + sz * gSzg + 2.0 * ak2;
        acc[3] += nF + nG;
        acc[4] += fSzf + gSzg;
        dens[p] = nF + nG;
        // grad_Phi of F^H C_+ F + G^H C_- G (real 3-vector), Re(conj(s) v) = s.x v.x + s.y v.y
        const double SxP[3] = {r2 * P[1], r2 * (P[0] + P[2]), r2 * P[1]};
        const double SzP[3] = {P[0], 0.0, -P[2]};
        for (int c = 0; c < 3; ++c) {
            double gq = bn * (2.0 * P[c] * nF + 4.0 * (pF.x * F[c].x + pF.y * F[c].y))
                      + bs * (2.0 * fSxf * SxP[c] + 2.0 * fSzf * SzP[c] + 4.0 * (pxF.x * SxF[c].x + pxF.y * SxF[c].y)
                              + 4.0 * (pzF.x * SzF[c].x + pzF.y * SzF[c].y))
                      + bn * 2.0 * P[c] * nG
                      + bs * (2.0 * gSxg * SxP[c] + 2.0 * gSzg * SzP[c] + 4.0 * (pkG.x * KtG[c].x + pkG.y * KtG[c].y));
            qout[c * npts + p] = cmk<double2>(gq, 0.0);
        }
    }
    reduce_store<5>(acc, part);
}

// sums <y, rho Phi>, <y, (S.s) Phi> (y real part) and the V gradient
__global__ void __launch_bounds__(RB2) k_grad_final(long long npts, const double* __restrict__ phi,
                                                    const double2* __restrict__ y, const double* __restrict__ dens,
                                                    double s, double* __restrict__ dV, double* part) {
    const double r2 = 0.70710678118654752440;
    double acc[2] = {0, 0};
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
        const double a = phi[p], b = phi[npts + p], d = phi[2 * npts + p];
        const double ya = y[p].x, yb = y[npts + p].x, yd = y[2 * npts + p].x;
        const double rho = a * a + b * b + d * d;
        const double sx = 1.4142135623730950488 * b * (a + d), sz = a * a - d * d;
        // (S.s) Phi = sx S_x Phi + sz S_z Phi
        const double sp0 = sx * r2 * b + sz * a, sp1 = sx * r2 * (a + d), sp2 = sx * r2 * b - sz * d;
        acc[0] += rho * (ya * a + yb * b + yd * d);
        acc[1] += ya * sp0 + yb * sp1 + yd * sp2;
        dV[p] = s * dens[p] - (ya * a + yb * b + yd * d);
    }
    reduce_store<2>(acc, part);
}

__global__ void k_axpy_real_cols(long long n, double a1, const double* __restrict__ x1, double a2,
                                 const double* __restrict__ x2, double2* __restrict__ out) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        out[i] = cmk<double2>(a1 * x1[i] + a2 * x2[i], 0.0);
}

__global__ void k_szphi(long long npts, const double* __restrict__ phi, double* __restrict__ out) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
        out[p] = phi[p];
        out[npts + p] = 0.0;
        out[2 * npts + p] = -phi[2 * npts + p];
    }
}

__global__ void k_scale_add(long long n, double s, const double2* __restrict__ x, double2* __restrict__ y) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const double2 a = x[i], b = y[i];
        y[i] = cmk<double2>(b.x + s * a.x, b.y + s * a.y);
    }
}

__global__ void k_mean_rows(long long npts, int j0, int cnt, double* __restrict__ dV) {
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < npts; p += (long long)gridDim.x * blockDim.x) {
        double a = 0;
        for (int j = 0; j < cnt; ++j) a += dV[(long long)(j0 + j) * npts + p];
        a /= cnt;
        for (int j = 0; j < cnt; ++j) dV[(long long)(j0 + j) * npts + p] = a;
    }
}

}  // namespace

extern "C" bdg_status bdg_eigs_grad(bdg_ctx* c, int k, const double* omega, const void* UV_dev, double* dV_dev,
                                    double* dbeta_n, double* dbeta_s) {
    if (!c) return BDG_EINVAL;
    if (k < 1 || !omega || !UV_dev || !dV_dev || !dbeta_n || !dbeta_s)
        return ctx_fail(c, BDG_EINVAL, "bdg_eigs_grad: bad arguments");
    if (!c->has_gs) return ctx_fail(c, BDG_ESTATE, "bdg_eigs_grad: no ground state set");
    if (c->complex_gs) return ctx_fail(c, BDG_EINVAL, "bdg_eigs_grad: real ground states only");
    const long long npts = c->npts, nh = 3 * npts;
    const bdg_problem& pr = c->prob;
    Small w;
    double2* Q = nullptr;      // orthonormal basis of span{Phi, S_z Phi} (complex, 2 columns)
    double* szphi = nullptr;
    double* dens = nullptr;
    double2* qv = nullptr;     // q, then the right-hand side
    double2* y = nullptr;
    double2* yc = nullptr;
    double2* ws = nullptr;
    double* part = nullptr;
    double* sums = nullptr;
    // every exit path releases the workspace
    auto release = defer([&] {
        small_free(c, w);
        for (void* p : {(void*)Q, (void*)szphi, (void*)dens, (void*)qv, (void*)y, (void*)yc, (void*)ws, (void*)part,
                        (void*)sums})
            ctx_free(c, p);
    });
    BDG_TRY(small_alloc(c, w, 8));
    const int nblk = (int)std::min<long long>(1024, (npts + RB2 - 1) / RB2);
    BDG_TRY(ctx_alloc(c, (void**)&Q, 2 * nh * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&szphi, nh * sizeof(double)));
    BDG_TRY(ctx_alloc(c, (void**)&dens, npts * sizeof(double)));
    BDG_TRY(ctx_alloc(c, (void**)&qv, nh * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&y, nh * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&yc, 2 * nh * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&ws, 5 * nh * sizeof(double2)));
    BDG_TRY(ctx_alloc(c, (void**)&part, 8 * (size_t)nblk * sizeof(double)));
    BDG_TRY(ctx_alloc(c, (void**)&sums, 8 * sizeof(double)));
    auto reduce = [&](int nq, double* host, double scale) -> bdg_status {
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, c->stream, nq, nblk, (const double*)part, scale, sums);
        return d2h(c, host, sums, nq * sizeof(double));
    };
    // tangent-space basis: Phi and S_z Phi (orthonormalized; S_z Phi may vanish)
    hipLaunchKernelGGL(k_szphi, dim3(nblk), dim3(RB2), 0, c->stream, npts, (const double*)c->phi, szphi);
    hipLaunchKernelGGL(k_axpy_real_cols, dim3(nblk), dim3(RB2), 0, c->stream, nh, 1.0, (const double*)c->phi, 0.0,
                       (const double*)c->phi, yc);
    hipLaunchKernelGGL(k_axpy_real_cols, dim3(nblk), dim3(RB2), 0, c->stream, nh, 1.0, (const double*)szphi, 0.0,
                       (const double*)szphi, yc + nh);
    int nq = 0;
    BDG_TRY(orthonormalize(c, w, nh, yc, 2, Q, 1e-12, &nq));
    // Gram of the raw constraint vectors (for the component of y along them)
    double g11, g12, g22;
    {
        bdg_status st;
        g11 = host_dot_re(c, w, nh, yc, yc, &st); BDG_TRY(st);
        g12 = host_dot_re(c, w, nh, yc, yc + nh, &st); BDG_TRY(st);
        g22 = host_dot_re(c, w, nh, yc + nh, yc + nh, &st); BDG_TRY(st);
    }
    std::vector<double> gbn(k), gbs(k);
    for (int j = 0; j < k; ++j) {
        const double2* uv = (const double2*)UV_dev + (size_t)j * 2 * nh;
        hipLaunchKernelGGL(k_grad_fields, dim3(nblk), dim3(RB2), 0, c->stream, npts, (const double*)c->phi, uv,
                           pr.beta_n, pr.beta_s, dens, qv, part);
        double sm[5];
        BDG_TRY(reduce(5, sm, c->hd));
        if (!(sm[0] > 0)) return ctx_fail(c, BDG_EINVAL, "bdg_eigs_grad: <f, g> <= 0 (not a positive excitation)");
        const double s = 1.0 / (2.0 * sm[0]);
        const double a_mu = -s * sm[3], a_lam = -s * sm[4];
        // y_c = c1 Phi + c2 S_z Phi with <Phi, y_c> = -a_mu, <S_z Phi, y_c> = -a_lam
        double c1 = 0, c2 = 0;
        const double det = g11 * g22 - g12 * g12;
        if (det > 1e-14 * g11 * g22) {
            c1 = (-a_mu * g22 + a_lam * g12) / det;
            c2 = (-a_lam * g11 + a_mu * g12) / det;
        } else {
            c1 = -a_mu / g11;
        }
        // rhs = s q - H_+ y_c, solve H_+ t = rhs on the tangent space, y = y_c + t
        hipLaunchKernelGGL(k_axpy_real_cols, dim3(nblk), dim3(RB2), 0, c->stream, nh, c1, (const double*)c->phi, c2,
                           (const double*)szphi, y);
        BDG_TRY(apply64(c, 1, y, y, nh, ws, ws + nh));          // ws = H_+ y_c
        // qv <- s qv - H_+ y_c
        {
            double sv = s;
            BDG_TRY(h2d(c, sums, &sv, sizeof(double)));
            hipLaunchKernelGGL(k_cols_scale, grid_cols(nh, 1), dim3(256), 0, c->stream, nh, 1, qv, nh,
                               (const double*)sums, 0);
        }
        hipLaunchKernelGGL(k_scale_add, dim3(nblk), dim3(RB2), 0, c->stream, nh, -1.0, (const double2*)ws, qv);
        double2* t = yc;   // reuse
        BDG_TRY(pcg_hplus(c, w, nh, Q, nq, qv, t, ws, 1e-12, 20000));
        hipLaunchKernelGGL(k_scale_add, dim3(nblk), dim3(RB2), 0, c->stream, nh, 1.0, (const double2*)t, y);
        double* dVj = dV_dev + (size_t)j * npts;
        hipLaunchKernelGGL(k_grad_final, dim3(nblk), dim3(RB2), 0, c->stream, npts, (const double*)c->phi,
                           (const double2*)y, (const double*)dens, s, dVj, part);
        double fin[2];
        BDG_TRY(reduce(2, fin, c->hd));
        gbn[j] = s * sm[1] - fin[0];
        gbs[j] = s * sm[2] - fin[1];
        // restore yc columns (reused as PCG output) for the next eigenpair
        hipLaunchKernelGGL(k_axpy_real_cols, dim3(nblk), dim3(RB2), 0, c->stream, nh, 1.0, (const double*)c->phi, 0.0,
                           (const double*)c->phi, yc);
        hipLaunchKernelGGL(k_axpy_real_cols, dim3(nblk), dim3(RB2), 0, c->stream, nh, 1.0, (const double*)szphi, 0.0,
                           (const double*)szphi, yc + nh);
    }
    // cluster means (|omega_i - omega_j| <= 1e-8 omega)
    int j0 = 0;
    while (j0 < k) {
        int j1 = j0 + 1;
        while (j1 < k && std::fabs(omega[j1] - omega[j0]) <= 1e-8 * std::fabs(omega[j0])) ++j1;
        const int cnt = j1 - j0;
        double mbn = 0, mbs = 0;
        for (int j = j0; j < j1; ++j) { mbn += gbn[j]; mbs += gbs[j]; }
        for (int j = j0; j < j1; ++j) { dbeta_n[j] = mbn / cnt; dbeta_s[j] = mbs / cnt; }
        if (cnt > 1)
            hipLaunchKernelGGL(k_mean_rows, dim3(nblk), dim3(RB2), 0, c->stream, npts, j0, cnt, dV_dev);
        j0 = j1;
    }
    BDG_HIP(c, hipStreamSynchronize(c->stream));
    return BDG_OK;
}
