// Rank-revealing factorizations of the projected (m <= 512) matrices of the subspace
// iteration, one workgroup each, FP64 complex, column-major:
//   pivoted Cholesky of a Gram matrix -> R with (S R)^H (S R) = I on the numerical range of S;
//   LU with complete pivoting of the pairing matrix B = S_g^H S_f -> C_f, C_g with
//   C_g^H B C_f = I (the bi-orthogonal Gram-Schmidt of Section 3.2 in factored form:
//   the modified Gram-Schmidt bi-orthogonalization is an LU factorization of B).
#include "common.h"

#include <algorithm>

namespace {

__device__ __forceinline__ double2 mk(double x, double y) { double2 r; r.x = x; r.y = y; return r; }
__device__ __forceinline__ double2 cm(double2 a, double2 b) { return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ double2 cmc(double2 a, double2 b) {   // a * conj(b)
    return mk(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return mk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// block-wide argmax of (v, idx); ties resolved to the smaller index (deterministic)
__device__ void block_argmax(double v, int idx, double* sv, int* si, double* out_v, int* out_i) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_down(v, off);
        const int oi = __shfl_down(idx, off);
        if (lane + off < 64 && (ov > v || (ov == v && oi < idx))) { v = ov; idx = oi; }
    }
    if (lane == 0) { sv[wv] = v; si[wv] = idx; }
    __syncthreads();
    if (t == 0) {
        double bv = sv[0];
        int bi = si[0];
        for (int w = 1; w < (int)((blockDim.x + 63) / 64); ++w)
            if (sv[w] > bv || (sv[w] == bv && si[w] < bi)) { bv = sv[w]; bi = si[w]; }
        *out_v = bv;
        *out_i = bi;
    }
    __syncthreads();
}

// T (r x r, ld r) = Lt^-1 for the lower-triangular Lt given by the accessor (unit: diagonal 1).
template <typename Acc>
__device__ void lower_inverse(int r, Acc L, bool unit, double2* T) {
    const int t = threadIdx.x, nt = blockDim.x;
    for (long long e = t; e < (long long)r * r; e += nt) {
        const int i = (int)(e % r), c = (int)(e / r);
        T[(long long)c * r + i] = mk(i == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    for (int k = 0; k < r; ++k) {
        if (!unit) {
            const double2 d = L(k, k);
            for (int c = t; c <= k; c += nt) T[(long long)c * r + k] = cdiv(T[(long long)c * r + k], d);
            __syncthreads();
        }
        const long long rows = r - k - 1, cols = k + 1, nu = rows * cols;
        for (long long e0 = t; e0 < nu; e0 += 4 * nt) {
            double2 yv[4], pv[4];
            long long ix[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long long e = e0 + (long long)u * nt;
                ix[u] = -1;
                if (e < nu) {
                    const int i = k + 1 + (int)(e % rows), c = (int)(e / rows);
                    ix[u] = (long long)c * r + i;
                    pv[u] = cm(L(i, k), T[(long long)c * r + k]);
                    yv[u] = T[ix[u]];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (ix[u] >= 0) T[ix[u]] = mk(yv[u].x - pv[u].x, yv[u].y - pv[u].y);
        }
        __syncthreads();
    }
}

// Pivoted Cholesky of the diagonally scaled Gram matrix A (m x m, destroyed).  Stops when the
// largest remaining diagonal (Schur complement) is <= rtol.  R (m x m, ld m) receives
// D^-1/2 P [L11^-H; 0] in its first r columns; *rank = r.  Workgroup b solves problem b of
// the launch (two independent problems of one size, such as the f- and g-bases, share it).
struct PcholProb {
    double2* A;
    double2* Lb;     // m x m workspace
    double2* T;      // m x m workspace
    double2* R;
    int* rank;
};

__global__ void __launch_bounds__(1024) k_pchol_orth(int m, int lda, double rtol, PcholProb p0, PcholProb p1) {
    const PcholProb& pb = blockIdx.x ? p1 : p0;
    double2* A = pb.A;
    double2* Lb = pb.Lb;
    double2* T = pb.T;
    double2* R = pb.R;
    int* rank = pb.rank;
    __shared__ int perm[512];
    __shared__ double d[512];
    __shared__ double dinv[512];
    __shared__ double sv[16];
    __shared__ int si[16];
    __shared__ double bestv;
    __shared__ int besti;
    const int t = threadIdx.x, nt = blockDim.x;
    if (t == 0) {
        double mx = 0;
        for (int i = 0; i < m; ++i) mx = fmax(mx, A[(long long)i * lda + i].x);
        bestv = mx;
    }
    __syncthreads();
    const double dmax = bestv;
    for (int i = t; i < m; i += nt) {
        const double a = A[(long long)i * lda + i].x;
        dinv[i] = (a > 1e-20 * dmax && a > 0) ? 1.0 / sqrt(a) : 0.0;
        perm[i] = i;
    }
    __syncthreads();
    for (long long e = t; e < (long long)m * m; e += nt) {
        const int i = (int)(e % m), j = (int)(e / m);
        const double f = dinv[i] * dinv[j];
        double2 a = A[(long long)j * lda + i];
        A[(long long)j * lda + i] = mk(a.x * f, a.y * f);
    }
    __syncthreads();
    for (int i = t; i < m; i += nt) d[i] = A[(long long)i * lda + i].x;
    __syncthreads();
    int r = m;
    for (int j = 0; j < m; ++j) {
        double v = -1.0;
        int idx = m;
        for (int i = j + t; i < m; i += nt) {
            const double dv = d[perm[i]];
            if (dv > v || (dv == v && i < idx)) { v = dv; idx = i; }
        }
        block_argmax(v, idx, sv, si, &bestv, &besti);
        if (!(bestv > rtol)) { r = j; break; }
        if (t == 0) {
            const int tmp = perm[j]; perm[j] = perm[besti]; perm[besti] = tmp;
        }
        __syncthreads();
        const int pj = perm[j];
        const double piv = sqrt(bestv);
        // column j of L (stored by original row index): L[pi][j] = A[pi][pj] / piv; A keeps
        // its lower triangle in the original index order (row >= column), which the symmetric
        // pivot swaps leave intact, so an entry above it is read as the mirror's conjugate
        for (int i = j + t; i < m; i += nt) {
            const int pi = perm[i];
            double2 a;
            if (pi >= pj) {
                a = A[(long long)pj * lda + pi];
            } else {
                const double2 u = A[(long long)pi * lda + pj];
                a = mk(u.x, -u.y);
            }
            Lb[(long long)j * m + pi] = (i == j) ? mk(piv, 0.0) : mk(a.x / piv, a.y / piv);
        }
        __syncthreads();
        // Schur complement update on the remaining rows/columns, lower triangle (original
        // index order) only; four updates in flight
        const long long rem = m - j - 1;
        for (long long e0 = t; e0 < rem * rem; e0 += 4 * nt) {
            double2 av[4], pv[4];
            long long ix[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long long e = e0 + (long long)u * nt;
                ix[u] = -1;
                const int pi = e < rem * rem ? perm[j + 1 + (int)(e % rem)] : 0;
                const int pl = e < rem * rem ? perm[j + 1 + (int)(e / rem)] : 1;
                if (e < rem * rem && pi >= pl) {
                    ix[u] = (long long)pl * lda + pi;
                    pv[u] = cmc(Lb[(long long)j * m + pi], Lb[(long long)j * m + pl]);
                    av[u] = A[ix[u]];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (ix[u] >= 0) A[ix[u]] = mk(av[u].x - pv[u].x, av[u].y - pv[u].y);
        }
        for (int i = j + 1 + t; i < m; i += nt) {
            const double2 li = Lb[(long long)j * m + perm[i]];
            d[perm[i]] -= li.x * li.x + li.y * li.y;
        }
        __syncthreads();
    }
    // T = L11^-1 (in the pivoted order)
    auto Lacc = [&](int i, int k) -> double2 { return Lb[(long long)k * m + perm[i]]; };
    lower_inverse(r, Lacc, false, T);
    // R[perm[i]][c] = dinv[perm[i]] conj(T[c][i]) for i < r; other rows zero
    for (long long e = t; e < (long long)m * m; e += nt) {
        const int i = (int)(e % m), c = (int)(e / m);
        double2 v = mk(0.0, 0.0);
        if (i < r && c < r && c >= i) {
            const double2 x = T[(long long)i * r + c];
            const double f = dinv[perm[i]];
            v = mk(f * x.x, -f * x.y);
        }
        if (i < m) R[(long long)c * m + perm[i]] = v;
    }
    if (t == 0) *rank = r;
}

// LU with complete pivoting of B (p x q, destroyed): P_r B P_c^T = L U, stopping when the largest
// remaining |entry| <= tol.  Cf (q x r, ld q) = P_c^T [U11^-1; 0], Cg (p x r, ld p) =
// P_r^T [L11^-H; 0], so Cg^H B Cf = I_r.
__global__ void __launch_bounds__(1024) k_plu_biorth(int p, int q, double2* B, int ldb, double tol, double2* T,
                                                     double2* Cf, double2* Cg, int* rank) {
    __shared__ int pr[512];
    __shared__ int pc[512];
    __shared__ double sv[16];
    __shared__ int si[16];
    __shared__ double bestv;
    __shared__ int besti;
    const int t = threadIdx.x, nt = blockDim.x;
    for (int i = t; i < p; i += nt) pr[i] = i;
    for (int i = t; i < q; i += nt) pc[i] = i;
    __syncthreads();
    const int mn = p < q ? p : q;
    int r = mn;
    {
        // first pivot: the largest entry of B; later pivots come out of the Schur updates
        double v = -1.0;
        int idx = 0x7fffffff;
        for (long long e = t; e < (long long)p * q; e += nt) {
            const int i = (int)(e % p), l = (int)(e / p);
            const double2 b = B[(long long)l * ldb + i];
            const double a = b.x * b.x + b.y * b.y;
            const int code = i * 512 + l;
            if (a > v || (a == v && code < idx)) { v = a; idx = code; }
        }
        block_argmax(v, idx, sv, si, &bestv, &besti);
    }
    for (int j = 0; j < mn; ++j) {
        const long long rp = p - j, rq = q - j;
        if (!(bestv > tol * tol)) { r = j; break; }
        if (t == 0) {
            const int i = besti / 512, l = besti % 512;
            int tmp = pr[j]; pr[j] = pr[i]; pr[i] = tmp;
            tmp = pc[j]; pc[j] = pc[l]; pc[l] = tmp;
        }
        __syncthreads();
        const double2 piv = B[(long long)pc[j] * ldb + pr[j]];
        for (int i = j + 1 + t; i < p; i += nt) {
            double2& b = B[(long long)pc[j] * ldb + pr[i]];
            b = cdiv(b, piv);
        }
        __syncthreads();
        // Schur update of the trailing block; the largest updated entry is the next pivot
        const long long nu = (rp - 1) * (rq - 1);
        double v = -1.0;
        int idx = 0x7fffffff;
        for (long long e0 = t; e0 < nu; e0 += 4 * nt) {
            double2 bv[4], pv[4];
            long long ix[4];
            int code[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long long e = e0 + (long long)u * nt;
                ix[u] = -1;
                if (e < nu) {
                    const int i = j + 1 + (int)(e % (rp - 1)), l = j + 1 + (int)(e / (rp - 1));
                    ix[u] = (long long)pc[l] * ldb + pr[i];
                    code[u] = i * 512 + l;
                    pv[u] = cm(B[(long long)pc[j] * ldb + pr[i]], B[(long long)pc[l] * ldb + pr[j]]);
                    bv[u] = B[ix[u]];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (ix[u] >= 0) {
                    const double2 nb = mk(bv[u].x - pv[u].x, bv[u].y - pv[u].y);
                    B[ix[u]] = nb;
                    const double a = nb.x * nb.x + nb.y * nb.y;
                    if (a > v || (a == v && code[u] < idx)) { v = a; idx = code[u]; }
                }
        }
        // (block_argmax synchronizes the workgroup before and after)
        block_argmax(v, idx, sv, si, &bestv, &besti);
    }
    // T = L11^-1 (unit lower); Cg[pr[i]][c] = conj(T[c][i])
    auto Lacc = [&](int i, int k) -> double2 { return B[(long long)pc[k] * ldb + pr[i]]; };
    lower_inverse(r, Lacc, true, T);
    for (long long e = t; e < (long long)p * r; e += nt) {
        const int i = (int)(e % p), c = (int)(e / p);
        double2 v = mk(0.0, 0.0);
        if (i < r && c >= i) {
            const double2 x = T[(long long)i * r + c];
            v = mk(x.x, -x.y);
        }
        Cg[(long long)c * p + pr[i]] = v;
    }
    __syncthreads();
    // U11^-1 = (W^-1)^H with W = U11^H lower: W(i, k) = conj(U(k, i))
    auto Wacc = [&](int i, int k) -> double2 {
        const double2 u = B[(long long)pc[i] * ldb + pr[k]];
        return mk(u.x, -u.y);
    };
    lower_inverse(r, Wacc, false, T);
    // Cf[pc[i]][c] = (U11^-1)[i][c] = conj(T[c][i])
    for (long long e = t; e < (long long)q * r; e += nt) {
        const int i = (int)(e % q), c = (int)(e / q);
        double2 v = mk(0.0, 0.0);
        if (i < r && c >= i) {
            const double2 x = T[(long long)i * r + c];
            v = mk(x.x, -x.y);
        }
        Cf[(long long)c * q + pc[i]] = v;
    }
    if (t == 0) *rank = r;
}

}  // namespace

bdg_status small_pchol_orth(bdg_ctx* c, int m, double2* A, int lda, double rtol, double2* R, int* rank_dev) {
    if (m > 512) return ctx_fail(c, BDG_EINVAL, "small_pchol_orth: m > 512");
    void* ws = nullptr;
    BDG_TRY(ctx_scratch(c, 4, 2 * (size_t)m * m * sizeof(double2), &ws));
    const PcholProb p{A, (double2*)ws, (double2*)ws + (size_t)m * m, R, rank_dev};
    hipLaunchKernelGGL(k_pchol_orth, dim3(1), dim3(1024), 0, c->stream, m, lda, rtol, p, p);
    return hip_check(c, hipGetLastError(), "k_pchol_orth");
}

bdg_status small_pchol_orth2(bdg_ctx* c, int m, double2* A0, double2* A1, int lda, double rtol, double2* R0,
                             double2* R1, int* rank0_dev, int* rank1_dev) {
    if (m > 512) return ctx_fail(c, BDG_EINVAL, "small_pchol_orth: m > 512");
    void* ws = nullptr;
    BDG_TRY(ctx_scratch(c, 4, 4 * (size_t)m * m * sizeof(double2), &ws));
    double2* w = (double2*)ws;
    const size_t mm = (size_t)m * m;
    const PcholProb p0{A0, w, w + mm, R0, rank0_dev};
    const PcholProb p1{A1, w + 2 * mm, w + 3 * mm, R1, rank1_dev};
    hipLaunchKernelGGL(k_pchol_orth, dim3(2), dim3(1024), 0, c->stream, m, lda, rtol, p0, p1);
    return hip_check(c, hipGetLastError(), "k_pchol_orth");
}

bdg_status small_plu_biorth(bdg_ctx* c, int p, int q, double2* B, int ldb, double tol, double2* Cf, double2* Cg,
                            int* rank_dev) {
    if (p > 512 || q > 512) return ctx_fail(c, BDG_EINVAL, "small_plu_biorth: size > 512");
    void* ws = nullptr;
    const int mn = std::min(p, q);
    BDG_TRY(ctx_scratch(c, 5, (size_t)mn * mn * sizeof(double2) + 64, &ws));
    hipLaunchKernelGGL(k_plu_biorth, dim3(1), dim3(1024), 0, c->stream, p, q, B, ldb, tol, (double2*)ws, Cf, Cg,
                       rank_dev);
    return hip_check(c, hipGetLastError(), "k_plu_biorth");
}
