/*
 * bdg_testing.h - kernel-level entry points of the library, exported for parity tests of
 * the dense building blocks of the subspace iteration (Section 3.2: Gram matrices of the
 * bi-orthogonal Gram-Schmidt and Rayleigh-Ritz steps, basis updates, projected problems).
 * Same conventions as bdg.h: device pointers, column-major complex128 (interleaved re, im),
 * synchronous on the context stream, bdg_status return codes.  They need a context only
 * for its stream and scratch memory (no ground state).
 */
#ifndef BDG_TESTING_H
#define BDG_TESTING_H

#include "bdg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C (m1 x m2, ldc) = alpha * A^H B with A: K x m1 (column stride lda), B: K x m2 (ldb), on
 * the FP64 matrix cores with a deterministic split-K reduction.  hermitian = 1 declares
 * A^H B Hermitian (A == B, or B = M A with M Hermitian): needs m1 == m2, computes the upper
 * tiles and fills C's lower triangle from them. */
bdg_status bdg_test_gram(bdg_ctx* ctx, long long K, int m1, int m2, const void* A, long long lda,
                         const void* B, long long ldb, double alpha, void* C, int ldc, int hermitian);

/* Y (K x nb, ldy) = S (K x m, lds) * Cm (m x nb, ldcm) + beta * Y on the FP64 matrix cores. */
bdg_status bdg_test_update(bdg_ctx* ctx, long long K, int m, const void* S, long long lds,
                           const void* Cm, int ldcm, int nb, double beta, void* Y, long long ldy);

/* Paired real form (two real columns per complex column: real part 2 j, imaginary part
 * 2 j + 1).  C (2 m1 x 2 m2 real entries stored as complex with zero imaginary parts, ldc >= 2 m1)
 * = alpha * Ar^T Br for A: K x m1 complex columns (lda), B: K x m2 (ldb).  symmetric = 1
 * declares Ar^T Br symmetric (needs m1 == m2): upper tiles, mirrored. */
bdg_status bdg_test_gram_pair(bdg_ctx* ctx, long long K, int m1, int m2, const void* A, long long lda,
                              const void* B, long long ldb, double alpha, void* C, int ldc, int symmetric);

/* The kinetic-potential preconditioner D (|k|^2/2 + sigma)^-1 D (Section 2.3) as the mixed
 * solve applies it: X32 (nvec complex64 vectors of six fields, npts points each, contiguous)
 * in float32, the result widened into Y64 (complex128, the same layout).  X32 is used as
 * work space and overwritten.  Needs the ground state (bdg_set_ground_state or
 * bdg_ground_state), which fixes D and sigma.  BDG_ESTATE without it. */
bdg_status bdg_test_precond_mixed(bdg_ctx* ctx, int nvec, void* X32, void* Y64);

/* Paired real form: Y (nb real columns = nb / 2 complex columns, ldy) = S (2 m real columns =
 * m complex columns, lds) * Cm (2 m x nb real coefficients stored as complex, only the real
 * parts are read, ldcm >= 2 m) + beta * Y; nb even. */
bdg_status bdg_test_update_pair(bdg_ctx* ctx, long long K, int m, const void* S, long long lds, const void* Cm,
                                int ldcm, int nb, double beta, void* Y, long long ldy);

/* One-sided Jacobi SVD of G (rows x m, ldg), m <= 512: G is replaced by U diag(s) with
 * columns ordered by descending s; V (m x m, ldv) receives V; s (device, m). */
/* One-pass form of the paired update the eigensolver uses for blocks of up to 96 real columns:
 * S (K x m complex columns, lds; the first mF of them F, mF a multiple of 8), Cm as in
 * bdg_test_update_pair (2 m x nb real coefficients in complex storage, ldcm >= 2 m):
 * Yp = S[:, mF:] Cm[2 mF:, :] and Yf = S[:, :mF] Cm[:2 mF, :] + Yp (nb even, <= 96 real
 * columns, both K x nb / 2 complex, ld ldy). */
bdg_status bdg_test_update_pair_fused(bdg_ctx* ctx, long long K, int m, int mF, const void* S, long long lds,
                                      const void* Cm, int ldcm, int nb, void* Yp, void* Yf, long long ldy);
bdg_status bdg_test_svd(bdg_ctx* ctx, int rows, int m, void* G, int ldg, void* V, int ldv, void* s);
/* The same for a real G held in complex storage (imaginary parts zero; the projected
 * matrices of the paired real form): real rotations, V real. */
bdg_status bdg_test_svd_real(bdg_ctx* ctx, int rows, int m, void* G, int ldg, void* V, int ldv, void* s);

/* In-place lower Cholesky A = L L^H of an m x m Hermitian matrix (upper triangle zeroed);
 * returns BDG_EBREAKDOWN when a pivot is not positive. */
bdg_status bdg_test_cholesky(bdg_ctx* ctx, int m, void* A, int lda);

/* Pivoted Cholesky orthonormalization of a Hermitian PSD Gram matrix A (m x m, destroyed):
 * R (m x m, ldr = m) receives r columns with R^H A R = I; *rank (host) = r.  Columns are
 * scaled to unit diagonal first; the factorization stops when the largest remaining Schur
 * diagonal is <= rtol. */
bdg_status bdg_test_pchol(bdg_ctx* ctx, int m, void* A, int lda, double rtol, void* R, int* rank);

/* LU with complete pivoting of B (p x q, destroyed), stopping at |pivot| <= tol:
 * Cf (q x r, ld q) and Cg (p x r, ld p) with Cg^H B Cf = I_r; *rank (host) = r. */
bdg_status bdg_test_plu(bdg_ctx* ctx, int p, int q, void* B, int ldb, double tol, void* Cf, void* Cg, int* rank);

#ifdef __cplusplus
}
#endif
#endif /* BDG_TESTING_H */
