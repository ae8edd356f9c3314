// Internal declarations shared by the library's HIP sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bdg.h"

// ------------------------------------------------------------------------------------
// Complex helpers (interleaved re, im in HIP vector types)
// ------------------------------------------------------------------------------------
template <typename R> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };

template <typename V> __host__ __device__ __forceinline__ V cmk(decltype(V::x) a, decltype(V::x) b) {
    V r; r.x = a; r.y = b; return r;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return cmk<V>(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return cmk<V>(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    return cmk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b) {
    return cmk<V>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename V> __device__ __forceinline__ V cscale(V a, decltype(V::x) s) { return cmk<V>(a.x * s, a.y * s); }

// ------------------------------------------------------------------------------------
// Context
// ------------------------------------------------------------------------------------
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct bdg_ctx {
    bdg_problem prob{};
    hipStream_t stream = nullptr;
    int device = 0;
    int ncu = 256;                // compute units of the device
    int dim = 1;
    int n[3] = {1, 1, 1};
    double L[3] = {1, 1, 1};
    double h[3] = {1, 1, 1};
    double hd = 1.0;              // h_x h_y h_z (weight of the discrete inner product)
    long long npts = 1;           // grid points
    // device tables
    double* V = nullptr;          // npts
    double* phi = nullptr;        // 3 npts (ground state)
    double mu[3] = {0, 0, 0};
    bool has_gs = false;
    // complex ground state (general BdG form [[A, B], [-conj B, -conj A]]): the spinor and
    // 21 real fields per point, A's real diagonal (3), A's upper entries 01, 02, 12 (re, im),
    // then B's symmetric entries 00, 01, 02, 11, 12, 22 (re, im); V - mu folded into A
    bool complex_gs = false;
    double2* phic = nullptr;      // 3 npts
    double* ccoef = nullptr;      // 21 npts
    double* coef64 = nullptr;     // 12 npts: H_+ (6 sym entries) then H_- (6), V - mu folded in
    float* coef32 = nullptr;      // same, rounded
    // kinetic-potential preconditioner D (|k|^2/2 + pshift)^-1 D of the eigensolver:
    // pshift = max(mu_0 / 2, 1/2), D = sqrt(pshift / (pshift + max(V - mu_0, 0)))
    double pshift = 20.0;
    double* pw64 = nullptr;       // D, npts
    float* pw32 = nullptr;
    double2* tw64[3] = {nullptr, nullptr, nullptr};   // exp(-2 pi i m / N_a), m < N_a
    float2* tw32[3] = {nullptr, nullptr, nullptr};
    double* sym64[3] = {nullptr, nullptr, nullptr};   // mu_m^2 / 2 per axis, FFT order
    float* sym32[3] = {nullptr, nullptr, nullptr};
    // the operator runs its passes over chunks of vectors whose fields (6 per vector) fit in
    // this many bytes, so the intermediate passes re-read data still held in the last-level
    // cache (0: one chunk, all vectors)
    size_t apply_chunk_bytes = 0;
    // complex64 (f, g) operator on 128 x 128 x nz grids by xy-plane passes in LDS (three
    // passes over HBM instead of five)
    bool apply_planes = true;
    bool apply_planes64 = true;   // ... and the complex128 form (two half-planes per plane)
    // symmetric paired Grams of 65..128 complex columns by one workgroup per K-split
    bool gram_wide = true;
    int gram_w8 = 2;              // ... in blocks of 8 complex columns (2: operands loaded straight to
                                  // LDS, 1: staged through registers, 0: off)
    int jacobi_split = 8;         // workgroups per column-block pair in a real Jacobi round
    // deeper staging of the loads (the same bits as the plain forms) in the split-K
    // reductions of the Grams, Grams of at most 16 x 16 and updates of at most 8 columns
    // into at most 48
    bool deep_loads = true;
    // scratch owned by the context (grown on demand)
    DevBuf scratch[9];
    // caller-provided workspace: while `base` is set, ctx_alloc and ctx_scratch hand out
    // 256-byte aligned pieces of it in order (nothing is allocated, ctx_free of a piece does
    // nothing) and the Gram launches keep their split-K partials within `gram_bytes`
    struct Arena {
        char* base = nullptr;
        size_t size = 0;
        size_t used = 0;
        size_t gram_bytes = 0;
    } arena;
    std::string err;
    double stats[10] = {0};
    std::vector<void*> owned;     // every hipMalloc of the context, freed in destroy
};

// status helpers
bdg_status ctx_fail(bdg_ctx* c, bdg_status s, const std::string& msg);
bdg_status hip_check(bdg_ctx* c, hipError_t e, const char* what);
#define BDG_HIP(ctx, ...)                                               \
    do {                                                                \
        hipError_t e_ = (__VA_ARGS__);                                  \
        if (e_ != hipSuccess) return hip_check((ctx), e_, #__VA_ARGS__); \
    } while (0)
#define BDG_TRY(...)                                                    \
    do {                                                                \
        bdg_status s_ = (__VA_ARGS__);                                  \
        if (s_ != BDG_OK) return s_;                                    \
    } while (0)

bdg_status ctx_alloc(bdg_ctx* c, void** p, size_t bytes);
void ctx_free(bdg_ctx* c, void* p);
// scratch slot i with at least `bytes` (contents undefined)
bdg_status ctx_scratch(bdg_ctx* c, int slot, size_t bytes, void** out);

// ------------------------------------------------------------------------------------
// Operator kernels (fft_apply.hip)
// ------------------------------------------------------------------------------------
// Where the six fields (f_1, f_0, f_-1, g_1, g_0, g_-1) of vector j live:
// half 0 (f or u) at lo + j * vstride + c * npts, half 1 (g or v) at hi + j * vstride + c * npts.
template <typename V> struct BlockRef {
    V* lo;
    V* hi;
    long long vstride;
};

// Y = H X for nvec vectors; form BDG_FORM_FG or BDG_FORM_UV; transpose selects the adjoint.
template <typename R>
bdg_status launch_apply(bdg_ctx* c, int form, int transpose, int nvec,
                        BlockRef<const typename cplx_of<R>::type> X, BlockRef<typename cplx_of<R>::type> Y);

// Y = T X with the eigensolver's preconditioner T = D (|k|^2/2 + pshift)^-1 D (context
// fields, set with the ground state) on `nfields` complex grid fields;
// field f at base + (f / fpv) * vstride + (f % fpv) * npts.  X and Y may alias.
template <typename R>
bdg_status launch_precond(bdg_ctx* c, int nfields, int fpv, long long vstride,
                          const typename cplx_of<R>::type* X, typename cplx_of<R>::type* Y);

// Mixed form of launch_precond on nvec (f, g) pairs: float32 passes in place on X32 (lo: the
// f halves, hi: the g halves, vector stride vstride), the last pass writes float64 into Y64.
bdg_status launch_precond_mixed(bdg_ctx* c, int nvec, BlockRef<float2> X32, BlockRef<double2> Y64);
// the (f, g) operator in float32 on X, its result widened to float64 into Y64 (Ywork: float32
// work block of X's shape, overwritten)
bdg_status launch_apply_fg_to64(bdg_ctx* c, int nvec, BlockRef<const float2> X, BlockRef<float2> Ywork,
                                BlockRef<double2> Y64);
// complex ground state, (u, v) vectors in float64: kform = 0 gives Y = H X with
// H = [[T + A, B], [-conj B, -(T + conj A)]]; kform = 1 gives Y = sigma_3 H X, i.e. the
// Hermitian positive semidefinite K = [[T + A, B], [conj B, T + conj A]]
bdg_status launch_apply_complex(bdg_ctx* c, int kform, int nvec, BlockRef<const double2> X, BlockRef<double2> Y);

// Y = D F^-1 m(k) F D X with m = |k|^2/2 (precond = 0) or (|k|^2/2 + shift)^-1
// (precond = 1); D = wgt (npts real, pointwise) or 1 when wgt is null.
template <typename R>
bdg_status launch_fourier(bdg_ctx* c, int nfields, int fpv, long long vstride,
                          const typename cplx_of<R>::type* X, typename cplx_of<R>::type* Y, int precond, double shift,
                          const R* wgt);

// Plain forward/inverse (unnormalized) d-dimensional FFT of nfields fields (tests, ground state).
template <typename R>
bdg_status launch_fft(bdg_ctx* c, int nfields, const typename cplx_of<R>::type* X,
                      typename cplx_of<R>::type* Y, int inverse);

// coefficient fields of H_+ and H_- from the ground state (capi)
bdg_status build_coefficients(bdg_ctx* c);

// ------------------------------------------------------------------------------------
// Dense kernels (dense.hip)
// ------------------------------------------------------------------------------------
// C (m1 x m2, column-major, ldc) = alpha * A^H B, A: K x m1 complex (column stride lda,
// elements in TA), B: K x m2 (ldb, TB).  hermitian != 0: A == B and only needed once
// (C is completed from its upper triangle).  Deterministic split-K reduction.
struct Seg {
    const void* p;
    int ncols;
};
// Gram with column segments (logical column order = segment order), same column stride.
bdg_status gram_seg(bdg_ctx* c, long long K, const Seg* sa, int na, long long lda, const Seg* sb, int nb_,
                    long long ldb, double alpha, double2* C, int ldc, int hermitian);
template <typename TA, typename TB>
bdg_status gram(bdg_ctx* c, long long K, int m1, int m2, const TA* A, long long lda,
                const TB* B, long long ldb, double alpha, double2* C, int ldc, int hermitian);

// Y (K x nb) = S (K x m) Cm (m x nb) + beta * Y.  S columns: segments (ptr, ncols) with
// column stride lds each; Cm device m x nb column-major (ldcm); Y column stride ldy.
bdg_status update(bdg_ctx* c, long long K, const Seg* segs, int nseg, long long lds,
                  const double2* Cm, int ldcm, int nb, double beta, double2* Y, long long ldy);
// Y = S Cm + beta Z (Z may equal Y; Y must not overlap S when nb > 80).
bdg_status update_add(bdg_ctx* c, long long K, const Seg* segs, int nseg, long long lds, const double2* Cm,
                      int ldcm, int nb, double beta, const double2* Z, long long ldz, double2* Y, long long ldy);

// Paired real form (real ground states): each complex column holds two real columns, its real
// part (real column 2 J) and its imaginary part (2 J + 1).  Segments count complex columns.
// C (2 m1 x 2 m2 real entries in complex storage, imaginary parts 0, ldc) = alpha Ar^T Br;
// hermitian != 0: A == B or Ar^T Br symmetric by structure (upper tiles, mirrored).
bdg_status gram_seg_pair(bdg_ctx* c, long long K, const Seg* sa, int na, long long lda, const Seg* sb, int nbs,
                         long long ldb, double alpha, double2* C, int ldc, int hermitian);
// Y (nbr real columns) = S (segments, 2 mp real columns) Cr[r0 :, :] (real parts of the complex-stored
// 2 mp x nbr coefficient matrix Cr, ld ldcr, from row r0) + beta Z; nbr even; Y must not overlap S
bdg_status update_pair(bdg_ctx* c, long long K, const Seg* segs, int nseg, long long lds, const double2* Cr, int ldcr,
                       int r0, int nbr, double beta, const double2* Z, long long ldz, double2* Y, long long ldy);
// Y_p (nbr real columns) = S[mF:] Cr[2 mF :, :] and Y_f = S[:mF] Cr[: 2 mF, :] + Y_p in one pass
// (S: segments of mp complex columns, the first mF of them F; Cr as in update_pair from row 0).
// nbr even and <= 96, mF a multiple of 8.  Y_f may alias the rows of an input (row-local).
bdg_status update_pair_fused(bdg_ctx* c, long long K, const Seg* segs, int nseg, long long lds, const double2* Cr,
                             int ldcr, int nbr, int mF, double2* Yp, long long ldyp, double2* Yf, long long ldyf);
// squared norms of the 2 ncols real columns of ncols complex columns
bdg_status colnorm2_pair(bdg_ctx* c, long long K, int ncols, const double2* X, long long ldx, double* out_dev);
// residual norms of the 2 ncols real columns (omega per real column, om_dev[2 ncols]):
// out_dev[q * 2 ncols + j] holds |HF_j - om_j G_j|^2 (q = 0), |HG_j - om_j F_j|^2 (1), |F_j|^2 (2),
// |G_j|^2 (3)
bdg_status resnorm2_pair(bdg_ctx* c, long long K, int ncols, const double2* HF, const double2* G, const double2* HG,
                         const double2* F, long long ld, const double* om_dev, double* out_dev);
// out_dev[j] = F_j . G_j over the 2 ncols real columns
bdg_status dot_pair(bdg_ctx* c, long long K, int ncols, const double2* F, const double2* G, long long ld,
                    double* out_dev);

// small dense FP64 complex matrices on the device (column-major)
bdg_status small_gemm(bdg_ctx* c, int transA, int transB, int m, int n, int k, double2 alpha,
                      const double2* A, int lda, const double2* B, int ldb, double2 beta,
                      double2* C, int ldc);
// in-place lower Cholesky (upper part zeroed); *info_dev = 0 ok, j+1 if the j-th pivot fails
bdg_status small_cholesky(bdg_ctx* c, int m, double2* A, int lda, int* info_dev);
// two independent factorizations of one size in one launch (one workgroup each)
bdg_status small_cholesky2(bdg_ctx* c, int m, double2* A0, double2* A1, int lda, int* info0_dev, int* info1_dev);
// one-sided Jacobi SVD: G (rows x m) -> G V = U diag(s); G overwritten by U diag(s) (columns),
// V (m x m) receives V, s (m, device) the column norms; columns sorted by descending s.
// conv: a sweep without rotations of cosine above conv ends the iteration.  real: G has zero
// imaginary parts (real rotations, V real)
bdg_status small_svd(bdg_ctx* c, int rows, int m, double2* G, int ldg, double2* V, int ldv, double* s,
                     double conv = 1e-13, bool real = false);

// pivoted Cholesky of a Gram matrix A (m x m, destroyed; diagonally scaled inside):
// R (m x m, ld m) gets r columns with R^H A R = I; *rank_dev = r (Schur diagonal cut rtol)
bdg_status small_pchol_orth(bdg_ctx* c, int m, double2* A, int lda, double rtol, double2* R, int* rank_dev);
// two independent problems of one size in one launch (one workgroup each)
bdg_status small_pchol_orth2(bdg_ctx* c, int m, double2* A0, double2* A1, int lda, double rtol, double2* R0,
                             double2* R1, int* rank0_dev, int* rank1_dev);
// LU with complete pivoting of B (p x q, destroyed): Cf (q x r, ld q), Cg (p x r, ld p) with
// Cg^H B Cf = I_r; *rank_dev = r (pivot cut tol)
bdg_status small_plu_biorth(bdg_ctx* c, int p, int q, double2* B, int ldb, double tol, double2* Cf, double2* Cg,
                            int* rank_dev);

// column norms squared (deterministic), etc.
bdg_status colnorm2(bdg_ctx* c, long long K, int ncols, const double2* X, long long ldx,
                    double* out_dev);

