// The projected (m <= 512) problems of the subspace iteration, FP64, column-major, one
// workgroup per matrix unless stated: a small GEMM, Cholesky, the block one-sided Jacobi SVD
// of L_K^T L_M (one launch per round of column-block pairs), and two rank-revealing
// factorizations:
//   pivoted Cholesky of a Gram matrix -> R with (S R)^H (S R) = I on the numerical range of S;
//   LU with complete pivoting of the pairing matrix B = S_g^H S_f -> C_f, C_g with
//   C_g^H B C_f = I (the bi-orthogonal Gram-Schmidt of Section 3.2 in factored form:
//   the modified Gram-Schmidt bi-orthogonalization is an LU factorization of B).
#include "common.h"

#include <algorithm>
#include <cmath>

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

// Trailing updates of the factorizations below run in passes of 256 rows: lane l of wave w
// owns the rows r0 + l + 64 s (s < TR) of the pass and the wave the columns c0 + w + 16 n,
// TC columns at a time so that their loads are in flight together.  The values of the pivot
// column that a lane's rows need are loaded once per pass.
constexpr int TR = 4, TC = 2;
// element i of a column whose base is wave-uniform: a scalar base plus a 32-bit row offset
__device__ __forceinline__ double2* col_at(double2* col, int i) {
    return reinterpret_cast<double2*>(reinterpret_cast<char*>(col) + (unsigned)i * 16u);
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// T (r x r, ld r) = Lt^-1 for the lower-triangular Lt given by the accessor (unit: diagonal 1).
template <typename Acc>
__device__ void lower_inverse(int r, Acc L, bool unit, double2* T) {
    const int t = threadIdx.x, nt = blockDim.x;
    const int wv = uniform(t >> 6), ln = t & 63, nw = nt >> 6;
    for (int c = wv; c < r; c += nw)
        for (int i = ln; i < r; i += 64) T[(long long)c * r + i] = mk(i == c ? 1.0 : 0.0, 0.0);
    __syncthreads();
    for (int k = 0; k < r; ++k) {
        if (!unit) {
            const double2 d = L(k, k);
            for (int c = t; c <= k; c += nt) T[(long long)c * r + k] = cdiv(T[(long long)c * r + k], d);
            __syncthreads();
        }
        // rows i > k of the columns c <= k: T[c][i] -= L(i, k) T[c][k]
        for (int r0 = k + 1; r0 < r; r0 += 64 * TR) {
            double2 lik[TR];
#pragma unroll
            for (int s = 0; s < TR; ++s) {
                const int i = r0 + ln + 64 * s;
                lik[s] = i < r ? L(i, k) : mk(0.0, 0.0);
            }
            for (int c0 = wv; c0 <= k; c0 += TC * nw) {
                double2 tck[TC], yv[TC][TR];
#pragma unroll
                for (int u = 0; u < TC; ++u) {
                    const int c = c0 + u * nw;
                    if (c <= k) {
                        double2* col = T + (long long)c * r;
                        tck[u] = col[k];
#pragma unroll
                        for (int s = 0; s < TR; ++s) {
                            const int i = r0 + ln + 64 * s;
                            if (i < r) yv[u][s] = *col_at(col, i);
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < TC; ++u) {
                    const int c = c0 + u * nw;
                    if (c <= k) {
                        double2* col = T + (long long)c * r;
#pragma unroll
                        for (int s = 0; s < TR; ++s) {
                            const int i = r0 + ln + 64 * s;
                            if (i < r) {
                                const double2 pv = cm(lik[s], tck[u]);
                                *col_at(col, i) = mk(yv[u][s].x - pv.x, yv[u][s].y - pv.y);
                            }
                        }
                    }
                }
            }
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
        // index order) only
        {
            const int wv = uniform(t >> 6), ln = t & 63, nw = nt >> 6;
            double2* lcol = Lb + (long long)j * m;
            for (int r0 = j + 1; r0 < m; r0 += 64 * TR) {
                int pir[TR];
                double2 lr[TR];
#pragma unroll
                for (int s = 0; s < TR; ++s) {
                    const int i = r0 + ln + 64 * s;
                    pir[s] = i < m ? perm[i] : -1;
                    lr[s] = i < m ? *col_at(lcol, pir[s]) : mk(0.0, 0.0);
                }
                for (int l0 = j + 1 + wv; l0 < m; l0 += TC * nw) {
                    int pl[TC];
                    double2 ll[TC], av[TC][TR];
#pragma unroll
                    for (int u = 0; u < TC; ++u) {
                        const int l = l0 + u * nw;
                        pl[u] = l < m ? uniform(perm[l]) : 0x7fffffff;
                        if (l < m) {
                            double2* acol = A + (long long)pl[u] * lda;
                            ll[u] = lcol[pl[u]];
#pragma unroll
                            for (int s = 0; s < TR; ++s)
                                if (pir[s] >= pl[u]) av[u][s] = *col_at(acol, pir[s]);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < TC; ++u) {
                        double2* acol = A + (long long)(pl[u] < m ? pl[u] : 0) * lda;
#pragma unroll
                        for (int s = 0; s < TR; ++s)
                            if (pir[s] >= pl[u]) {
                                const double2 pv = cmc(lr[s], ll[u]);
                                *col_at(acol, pir[s]) = mk(av[u][s].x - pv.x, av[u][s].y - pv.y);
                            }
                    }
                }
            }
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
        double v = -1.0;
        int idx = 0x7fffffff;
        {
            const int wv = uniform(t >> 6), ln = t & 63, nw = nt >> 6;
            constexpr int TL = 1;    // one column at a time: the pivot search needs the registers
            double2* bcj = B + (long long)uniform(pc[j]) * ldb;
            const int rj = uniform(pr[j]);
            for (int r0 = j + 1; r0 < p; r0 += 64 * TR) {
                int rowi[TR];
                double2 lv[TR];
#pragma unroll
                for (int s = 0; s < TR; ++s) {
                    const int i = r0 + ln + 64 * s;
                    rowi[s] = i < p ? pr[i] : -1;
                    lv[s] = i < p ? *col_at(bcj, rowi[s]) : mk(0.0, 0.0);
                }
                for (int l0 = j + 1 + wv; l0 < q; l0 += TL * nw) {
                    double2* bcl[TL];
                    double2 uv[TL], bv[TL][TR];
#pragma unroll
                    for (int u = 0; u < TL; ++u) {
                        const int l = l0 + u * nw;
                        bcl[u] = B + (long long)(l < q ? uniform(pc[l]) : 0) * ldb;
                        if (l < q) {
                            uv[u] = bcl[u][rj];
#pragma unroll
                            for (int s = 0; s < TR; ++s)
                                if (rowi[s] >= 0) bv[u][s] = *col_at(bcl[u], rowi[s]);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < TL; ++u) {
                        const int l = l0 + u * nw;
                        if (l < q) {
#pragma unroll
                            for (int s = 0; s < TR; ++s)
                                if (rowi[s] >= 0) {
                                    const double2 pv = cm(lv[s], uv[u]);
                                    const double2 nb = mk(bv[u][s].x - pv.x, bv[u][s].y - pv.y);
                                    *col_at(bcl[u], rowi[s]) = nb;
                                    const double a = nb.x * nb.x + nb.y * nb.y;
                                    const int code = (r0 + ln + 64 * s) * 512 + l;
                                    if (a > v || (a == v && code < idx)) { v = a; idx = code; }
                                }
                        }
                    }
                }
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

typedef double d4 __attribute__((ext_vector_type(4)));
// v_mfma_f64_16x16x4f64: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator
// register r of lane l holds D[4 r + l / 16][l % 16]
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ----------------------------------------------------------------------------------------
// Small dense kernels (m <= 512), column-major complex FP64.
// ----------------------------------------------------------------------------------------
__device__ __forceinline__ double2 mkc(double x, double y) { double2 r; r.x = x; r.y = y; return r; }
__device__ __forceinline__ double2 conjd(double2 a) { return mkc(a.x, -a.y); }

__global__ void k_small_gemm(int tA, int tB, int m, int n, int k, double2 alpha, const double2* __restrict__ A,
                             int lda, const double2* __restrict__ B, int ldb, double2 beta, double2* C, int ldc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= m || j >= n) return;
    double sx = 0, sy = 0;
    for (int l = 0; l < k; ++l) {
        double2 a = tA ? conjd(A[(long long)i * lda + l]) : A[(long long)l * lda + i];
        double2 b = tB ? conjd(B[(long long)l * ldb + j]) : B[(long long)j * ldb + l];
        sx += a.x * b.x - a.y * b.y;
        sy += a.x * b.y + a.y * b.x;
    }
    double2 s = mkc(alpha.x * sx - alpha.y * sy, alpha.x * sy + alpha.y * sx);
    double2* dst = C + (long long)j * ldc + i;
    if (beta.x != 0.0 || beta.y != 0.0) {
        double2 o = *dst;
        s.x += beta.x * o.x - beta.y * o.y;
        s.y += beta.x * o.y + beta.y * o.x;
    }
    *dst = s;
}

// Right-looking Cholesky A = L L^H in one workgroup; lower triangle kept, upper zeroed.
// Workgroup b factors problem b of the launch (two independent matrices of one size).
__global__ void __launch_bounds__(1024) k_small_cholesky(int m, int lda, double2* A0, int* info0, double2* A1,
                                                         int* info1) {
    double2* A = blockIdx.x ? A1 : A0;
    int* info = blockIdx.x ? info1 : info0;
    __shared__ double piv;
    __shared__ int bad;
    const int t = threadIdx.x, nt = blockDim.x;
    if (t == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        if (t == 0) {
            double d = A[(long long)j * lda + j].x;
            if (!(d > 0.0) || !isfinite(d)) { bad = j + 1; piv = 1.0; }
            else piv = sqrt(d);
        }
        __syncthreads();
        if (bad) break;
        const double inv = 1.0 / piv;
        for (int i = j + t; i < m; i += nt) {
            double2 v = A[(long long)j * lda + i];
            A[(long long)j * lda + i] = (i == j) ? mkc(piv, 0.0) : mkc(v.x * inv, v.y * inv);
        }
        __syncthreads();
        // trailing update: A[i][l] -= L[i][j] conj(L[l][j]) for j < l <= i
        {
            const int wv = uniform(t >> 6), ln = t & 63, nw = nt >> 6;
            double2* ajc = A + (long long)j * lda;
            for (int r0 = j + 1; r0 < m; r0 += 64 * TR) {
                double2 li[TR];
#pragma unroll
                for (int s = 0; s < TR; ++s) {
                    const int i = r0 + ln + 64 * s;
                    li[s] = i < m ? *col_at(ajc, i) : mkc(0.0, 0.0);
                }
                for (int l0 = j + 1 + wv; l0 < m; l0 += TC * nw) {
                    double2 ll[TC], o[TC][TR];
#pragma unroll
                    for (int u = 0; u < TC; ++u) {
                        const int l = l0 + u * nw;
                        if (l < m) {
                            ll[u] = ajc[l];
#pragma unroll
                            for (int s = 0; s < TR; ++s) {
                                const int i = r0 + ln + 64 * s;
                                if (i < m && l <= i) o[u][s] = *col_at(A + (long long)l * lda, i);
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < TC; ++u) {
                        const int l = l0 + u * nw;
#pragma unroll
                        for (int s = 0; s < TR; ++s) {
                            const int i = r0 + ln + 64 * s;
                            if (l < m && i < m && l <= i) {
                                o[u][s].x -= li[s].x * ll[u].x + li[s].y * ll[u].y;
                                o[u][s].y -= li[s].y * ll[u].x - li[s].x * ll[u].y;
                                *col_at(A + (long long)l * lda, i) = o[u][s];
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    __syncthreads();
    // zero the strict upper triangle
    for (int l = t >> 6; l < m; l += nt >> 6)
        for (int i = t & 63; i < l; i += 64) A[(long long)l * lda + i] = mkc(0.0, 0.0);
    if (t == 0) *info = bad;
}

// One-sided Jacobi SVD by column blocks (round-robin ordering of blocks, complex rotations).
// A launch processes one round: workgroup b takes a pair of blocks of W columns and runs one
// sweep over all pairs of its 2W columns (k_bjacobi_round_g).  Rotations of columns whose
// squared norm is below negl (1e-30 ||G||_F^2) are skipped: such columns are numerically zero.
__global__ void k_identity_frob(int rows, int m, const double2* __restrict__ G, int ldg, double2* V, int ldv,
                                double* frob2, int* counter) {
    __shared__ double red[16];
    double fs = 0;
    for (long long e = threadIdx.x; e < (long long)m * m; e += blockDim.x) {
        const int i = (int)(e % m), l = (int)(e / m);
        V[(long long)l * ldv + i] = mkc(i == l ? 1.0 : 0.0, 0.0);
    }
    for (long long e = threadIdx.x; e < (long long)rows * m; e += blockDim.x) {
        const double2 g = G[(e / rows) * ldg + e % rows];
        fs += g.x * g.x + g.y * g.y;
    }
    for (int off = 32; off > 0; off >>= 1) fs += __shfl_down(fs, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = fs;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0;
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) a += red[w];
        *frob2 = a;
        *counter = 0;
    }
}

__global__ void k_zero_int(int* p) { *p = 0; }

// One round of the block one-sided Jacobi: the workgroup stages its 2W columns of G, forms their
// Gram matrix A = C^H C, runs the sweep over all pairs of its 2W columns on A alone
// (A <- R^H A R per disjoint pair, two LDS phases per step) while accumulating the unitary
// J = prod R, and applies J once to the 2W columns of G and V.  The rotations are those of
// the column form (they are computed from the same inner products); the per-step work is two
// LDS entries per thread instead of a pass over all rows.
template <int W>
__global__ void __launch_bounds__(256) k_bjacobi_round_g(int rows, int m, double2* G, int ldg, double2* V, int ldv,
                                                         int nblk, int rnd, const double* __restrict__ frob2,
                                                         int* rotations, double conv) {
    constexpr int N2 = 2 * W, PA = N2 + 1;
    extern __shared__ double2 sm[];
    __shared__ double prm[W][4];
    __shared__ int pact[W];
    __shared__ int rot_any;
    const int t = threadIdx.x, nt = blockDim.x;
    auto player = [&](int s) { return s == 0 ? 0 : ((s - 1 + rnd) % (nblk - 1)) + 1; };
    const int P = player(blockIdx.x), Q = player(nblk - 1 - blockIdx.x);
    const int c0[2] = {P * W, Q * W};
    int nc[2];
    for (int h = 0; h < 2; ++h) {
        const int lim = m - c0[h];
        nc[h] = lim <= 0 ? 0 : (lim < W ? lim : W);
    }
    auto valid = [&](int k) { return (k % W) < nc[k / W]; };
    auto colidx = [&](int k) { return c0[k / W] + (k % W); };
    const int pg = rows | 1;
    double2* lg = sm;                          // N2 columns of G, pitch pg
    double2* A = lg + (size_t)N2 * pg;         // N2 x N2, pitch PA
    double2* J = A + N2 * PA;                  // N2 x N2, pitch PA
    if (t == 0) rot_any = 0;
    {
        // 256 / N2 threads per column, 8 loads in flight per thread (the round is latency-bound)
        constexpr int TPC = 256 / N2, U = 8;
        const int kc = t / TPC, lane = t % TPC;
        const bool vk = valid(kc);
        const double2* src = G + (long long)(vk ? colidx(kc) : 0) * ldg;
        for (int i0 = lane; i0 < rows; i0 += U * TPC) {
            double2 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * TPC;
                v[u] = (vk && i < rows) ? src[i] : mkc(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * TPC;
                if (i < rows) lg[kc * pg + i] = v[u];
            }
        }
    }
    __syncthreads();
    for (int e = t; e < N2 * N2; e += nt) {
        const int r = e % N2, c = e / N2;
        if (r <= c) {
            double sx = 0, sy = 0;
            for (int i = 0; i < rows; ++i) {
                const double2 a = lg[r * pg + i], b = lg[c * pg + i];
                sx += a.x * b.x + a.y * b.y;
                sy += a.x * b.y - a.y * b.x;
            }
            A[c * PA + r] = mkc(sx, sy);            // conj(c_r) . c_c
            if (r != c) A[r * PA + c] = mkc(sx, -sy);
        }
        J[c * PA + r] = mkc(r == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    const double negl = 1e-30 * (*frob2);
    const double tol = 1e-15;
    const int tpp = nt / W;
    const int pair = t / tpp, sub = t % tpp;
    for (int r2 = 0; r2 < N2 - 1; ++r2) {
        auto pl = [&](int s) { return s == 0 ? 0 : ((s - 1 + r2) % (N2 - 1)) + 1; };
        int p = pl(pair), q = pl(N2 - 1 - pair);
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        if (sub == 0 && pair < W) {
            int act = 0;
            if (valid(p) && valid(q)) {
                const double al = A[p * PA + p].x, be = A[q * PA + q].x;
                const double2 gm = A[q * PA + p];
                const double g = sqrt(gm.x * gm.x + gm.y * gm.y);
                if (g > tol * sqrt(al * be) && g > 0.0 && al > negl && be > negl) {
                    if (g > conv * sqrt(al * be)) rot_any = 1;
                    const double zeta = (be - al) / (2.0 * g);
                    const double tt = fabs(zeta) > 1e100 ? 0.5 / zeta
                                                         : (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + tt * tt);
                    prm[pair][0] = cs;
                    prm[pair][1] = cs * tt;
                    prm[pair][2] = gm.x / g;     // e = conj(gamma) / |gamma|
                    prm[pair][3] = -gm.y / g;
                    act = 1;
                }
            }
            pact[pair] = act;
        }
        __syncthreads();
        const bool act = pair < W && pact[pair];
        double cs = 0, sn = 0, ex = 0, ey = 0;
        if (act) { cs = prm[pair][0]; sn = prm[pair][1]; ex = prm[pair][2]; ey = prm[pair][3]; }
        if (act) {
            // columns p, q of A and J: [a, b] <- [cs a - sn e b, sn a + cs e b]
            for (int i = sub; i < N2; i += tpp) {
                double2 a = A[p * PA + i], b = A[q * PA + i];
                double2 eb = mkc(ex * b.x - ey * b.y, ex * b.y + ey * b.x);
                A[p * PA + i] = mkc(cs * a.x - sn * eb.x, cs * a.y - sn * eb.y);
                A[q * PA + i] = mkc(sn * a.x + cs * eb.x, sn * a.y + cs * eb.y);
                a = J[p * PA + i];
                b = J[q * PA + i];
                eb = mkc(ex * b.x - ey * b.y, ex * b.y + ey * b.x);
                J[p * PA + i] = mkc(cs * a.x - sn * eb.x, cs * a.y - sn * eb.y);
                J[q * PA + i] = mkc(sn * a.x + cs * eb.x, sn * a.y + cs * eb.y);
            }
        }
        __syncthreads();
        if (act) {
            // rows p, q of A: [a; b] <- [cs a - sn conj(e) b; sn a + cs conj(e) b]
            for (int j = sub; j < N2; j += tpp) {
                const double2 a = A[j * PA + p], b = A[j * PA + q];
                const double2 eb = mkc(ex * b.x + ey * b.y, ex * b.y - ey * b.x);
                A[j * PA + p] = mkc(cs * a.x - sn * eb.x, cs * a.y - sn * eb.y);
                A[j * PA + q] = mkc(sn * a.x + cs * eb.x, sn * a.y + cs * eb.y);
            }
        }
        __syncthreads();
    }
    // [G; V] columns <- [G; V] columns J (row-local: each thread owns whole rows)
    for (int i = t; i < rows + m; i += nt) {
        const bool isg = i < rows;
        const int ii = isg ? i : i - rows;
        double2 x[N2];
#pragma unroll
        for (int k = 0; k < N2; ++k)
            x[k] = isg ? lg[k * pg + ii] : (valid(k) ? V[(long long)colidx(k) * ldv + ii] : mkc(0.0, 0.0));
#pragma unroll
        for (int c = 0; c < N2; ++c) {
            if (!valid(c)) continue;
            double sx = 0, sy = 0;
#pragma unroll
            for (int k = 0; k < N2; ++k) {
                const double2 jj = J[c * PA + k];
                sx += x[k].x * jj.x - x[k].y * jj.y;
                sy += x[k].x * jj.y + x[k].y * jj.x;
            }
            if (isg) G[(long long)colidx(c) * ldg + ii] = mkc(sx, sy);
            else V[(long long)colidx(c) * ldv + ii] = mkc(sx, sy);
        }
    }
    if (t == 0 && rot_any) atomicAdd(rotations, 1);
}

// The same round for real matrices held in complex storage (imaginary parts zero, as in the
// paired real form): real rotations (the phase e reduces to the sign of the off-diagonal
// entry), staging of the real parts only (half the LDS), a quarter of the flops.  Staging
// and the V rows keep several loads in flight per thread: the round is latency-bound.
// gridDim.y workgroups share a pair: each stages the pair and computes the same rotation
// (same inputs, same operations), and applies it to every gridDim.y-th block of 16 rows.
// With more than one, the round reads Gin, Vin and writes Gout, Vout (other buffers), so
// that no workgroup stages rows another one has already rotated; with one they may alias.
template <int W>
__global__ void __launch_bounds__(256) k_bjacobi_round_r(int rows, int m, const double2* Gin, int ldg,
                                                         const double2* Vin, int ldv, double2* Gout, double2* Vout,
                                                         int nblk, int rnd, const double* __restrict__ frob2,
                                                         int* rotations, double conv) {
    constexpr int N2 = 2 * W, PA = N2 + 1, TPC = 256 / N2, U = 8;
    static_assert(256 % N2 == 0, "columns divide the workgroup");
    extern __shared__ double smr[];
    __shared__ int rot_any;
    const int t = threadIdx.x;
    auto player = [&](int s) { return s == 0 ? 0 : ((s - 1 + rnd) % (nblk - 1)) + 1; };
    const int P = player(blockIdx.x), Q = player(nblk - 1 - blockIdx.x);
    const int c0[2] = {P * W, Q * W};
    int nc[2];
    for (int h = 0; h < 2; ++h) {
        const int lim = m - c0[h];
        nc[h] = lim <= 0 ? 0 : (lim < W ? lim : W);
    }
    auto valid = [&](int k) { return (k % W) < nc[k / W]; };
    auto colidx = [&](int k) { return c0[k / W] + (k % W); };
    const int pg = rows | 1;
    double* lg = smr;                          // N2 columns of G, pitch pg
    double* A = lg + (size_t)N2 * pg;          // N2 x N2, pitch PA
    double* J = A + N2 * PA;                   // N2 x N2, pitch PA
    if (t == 0) rot_any = 0;
    {
        // TPC threads per column, U loads in flight per thread
        const int kc = t / TPC, lane = t % TPC;
        const bool vk = valid(kc);
        const double2* src = Gin + (long long)(vk ? colidx(kc) : 0) * ldg;
        for (int i0 = lane; i0 < rows; i0 += U * TPC) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * TPC;
                v[u] = (vk && i < rows) ? src[i].x : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * TPC;
                if (i < rows) lg[kc * pg + i] = v[u];
            }
        }
    }
    __syncthreads();
    for (int e = t; e < N2 * N2; e += 256) {
        const int r = e % N2, c = e / N2;
        if (r <= c) {
            const double* a = lg + r * pg;
            const double* b = lg + c * pg;
            double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
            int i = 0;
            for (; i + 4 <= rows; i += 4) {
                s0 += a[i] * b[i];
                s1 += a[i + 1] * b[i + 1];
                s2 += a[i + 2] * b[i + 2];
                s3 += a[i + 3] * b[i + 3];
            }
            for (; i < rows; ++i) s0 += a[i] * b[i];
            const double sx = (s0 + s1) + (s2 + s3);
            A[c * PA + r] = sx;
            A[r * PA + c] = sx;
        }
        J[c * PA + r] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    const double negl = 1e-30 * (*frob2);
    const double tol = 1e-15;
    constexpr int tpp = 256 / W;
    const int pair = t / tpp, sub = t % tpp;
    for (int r2 = 0; r2 < N2 - 1; ++r2) {
        auto pl = [&](int s) { return s == 0 ? 0 : ((s - 1 + r2) % (N2 - 1)) + 1; };
        int p = pl(pair), q = pl(N2 - 1 - pair);
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        // every thread of the pair computes the rotation itself (same inputs, same result), so
        // no barrier separates the parameters from the updates
        bool act = false;
        double cs = 0, sn = 0, ex = 0;
        if (valid(p) && valid(q)) {
            const double al = A[p * PA + p], be = A[q * PA + q];
            const double gm = A[q * PA + p];
            const double g = fabs(gm);
            const double sab = sqrt(al * be);
            if (g > tol * sab && g > 0.0 && al > negl && be > negl) {
                if (g > conv * sab && sub == 0) rot_any = 1;
                const double zeta = (be - al) / (2.0 * g);
                const double tt = fabs(zeta) > 1e100 ? 0.5 / zeta
                                                     : (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                cs = 1.0 / sqrt(1.0 + tt * tt);
                sn = cs * tt;
                ex = gm >= 0.0 ? 1.0 : -1.0;    // e = sign(gamma)
                act = true;
            }
        }
        if (act) {
            // columns p, q of A and J: [a, b] <- [cs a - sn e b, sn a + cs e b]
            for (int i = sub; i < N2; i += tpp) {
                double a = A[p * PA + i], b = ex * A[q * PA + i];
                A[p * PA + i] = cs * a - sn * b;
                A[q * PA + i] = sn * a + cs * b;
                a = J[p * PA + i];
                b = ex * J[q * PA + i];
                J[p * PA + i] = cs * a - sn * b;
                J[q * PA + i] = sn * a + cs * b;
            }
        }
        __syncthreads();
        if (act) {
            // rows p, q of A
            for (int j = sub; j < N2; j += tpp) {
                const double a = A[j * PA + p], b = ex * A[j * PA + q];
                A[j * PA + p] = cs * a - sn * b;
                A[j * PA + q] = sn * a + cs * b;
            }
        }
        __syncthreads();
    }
    // [G; V] columns <- [G; V] columns J on the FP64 matrix cores: the rows + m rows in blocks
    // of 16 (G rows from LDS, V rows from memory), D = X J over N2 / 4 steps of four columns
    // of X; register r of lane l holds D[4 r + l / 16][l % 16], a lane's A operand is
    // X[l % 16][l / 16] and its B operand J[l / 16][l % 16] of the step
    {
        const int wave = t >> 6, lane = t & 63;
        const int li = lane & 15, lk = lane >> 4;
        const int nrb = (rows + m + 15) / 16;
        for (int rb = wave + 4 * (int)blockIdx.y; rb < nrb; rb += 4 * (int)gridDim.y) {
            const int row = 16 * rb + li;                  // this lane's A row
            const bool rg = row < rows;
            const bool rv = !rg && row < rows + m;
            d4 acc[N2 / 16 > 0 ? N2 / 16 : 1];
#pragma unroll
            for (int cb = 0; cb < (N2 + 15) / 16; ++cb) acc[cb] = d4{0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < N2 / 4; ++kc) {
                const int kk = 4 * kc + lk;
                const double a = rg ? lg[kk * pg + row]
                                    : ((rv && valid(kk)) ? Vin[(long long)colidx(kk) * ldv + (row - rows)].x : 0.0);
#pragma unroll
                for (int cb = 0; cb < (N2 + 15) / 16; ++cb) {
                    const int cc = 16 * cb + li;
                    const double b = cc < N2 ? J[cc * PA + kk] : 0.0;
                    acc[cb] = mfma(a, b, acc[cb]);
                }
            }
#pragma unroll
            for (int cb = 0; cb < (N2 + 15) / 16; ++cb) {
                const int cc = 16 * cb + li;
                if (cc >= N2 || !valid(cc)) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int orow = 16 * rb + 4 * r + lk;
                    if (orow < rows) Gout[(long long)colidx(cc) * ldg + orow] = mkc(acc[cb][r], 0.0);
                    else if (orow < rows + m)
                        Vout[(long long)colidx(cc) * ldv + (orow - rows)] = mkc(acc[cb][r], 0.0);
                }
            }
        }
    }
    if (t == 0 && rot_any && blockIdx.y == 0) atomicAdd(rotations, 1);
}

// column norms of G (rows x m) into s; permutation to descending order (stable), applied to
// G and V through the copies Gs, Vs.
__global__ void __launch_bounds__(1024) k_small_sort(int rows, int m, double2* G, int ldg, double2* V, int ldv,
                                                    double* s, double2* Gs, double2* Vs) {
    __shared__ double nrm[512];
    __shared__ int perm[512];
    const int t = threadIdx.x;
    for (int j = t; j < m; j += blockDim.x) {
        double a = 0;
        for (int i = 0; i < rows; ++i) {
            double2 v = G[(long long)j * ldg + i];
            a += v.x * v.x + v.y * v.y;
        }
        nrm[j] = sqrt(a);
    }
    __syncthreads();
    for (int j = t; j < m; j += blockDim.x) {
        int rank = 0;
        for (int i = 0; i < m; ++i)
            if (nrm[i] > nrm[j] || (nrm[i] == nrm[j] && i < j)) ++rank;
        perm[rank] = j;
    }
    __syncthreads();
    for (long long e = t; e < (long long)rows * m; e += blockDim.x) {
        const int i = (int)(e % rows), l = (int)(e / rows);
        Gs[e] = G[(long long)l * ldg + i];
    }
    for (long long e = t; e < (long long)m * m; e += blockDim.x) {
        const int i = (int)(e % m), l = (int)(e / m);
        Vs[e] = V[(long long)l * ldv + i];
    }
    __syncthreads();
    for (long long e = t; e < (long long)rows * m; e += blockDim.x) {
        const int i = (int)(e % rows), l = (int)(e / rows);
        G[(long long)l * ldg + i] = Gs[(long long)perm[l] * rows + i];
    }
    for (long long e = t; e < (long long)m * m; e += blockDim.x) {
        const int i = (int)(e % m), l = (int)(e / m);
        V[(long long)l * ldv + i] = Vs[(long long)perm[l] * m + i];
    }
    for (int j = t; j < m; j += blockDim.x) s[j] = nrm[perm[j]];
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

bdg_status small_gemm(bdg_ctx* c, int transA, int transB, int m, int n, int k, double2 alpha, const double2* A,
                      int lda, const double2* B, int ldb, double2 beta, double2* C, int ldc) {
    if (m <= 0 || n <= 0) return BDG_OK;
    dim3 grid((unsigned)((m + 127) / 128), (unsigned)n);
    hipLaunchKernelGGL(k_small_gemm, grid, dim3(128), 0, c->stream, transA, transB, m, n, k, alpha, A, lda, B, ldb,
                       beta, C, ldc);
    return hip_check(c, hipGetLastError(), "k_small_gemm");
}

bdg_status small_cholesky(bdg_ctx* c, int m, double2* A, int lda, int* info_dev) {
    if (m > 512) return ctx_fail(c, BDG_EINVAL, "small_cholesky: m > 512");
    hipLaunchKernelGGL(k_small_cholesky, dim3(1), dim3(1024), 0, c->stream, m, lda, A, info_dev, A, info_dev);
    return hip_check(c, hipGetLastError(), "k_small_cholesky");
}

bdg_status small_cholesky2(bdg_ctx* c, int m, double2* A0, double2* A1, int lda, int* info0_dev, int* info1_dev) {
    if (m > 512) return ctx_fail(c, BDG_EINVAL, "small_cholesky: m > 512");
    hipLaunchKernelGGL(k_small_cholesky, dim3(2), dim3(1024), 0, c->stream, m, lda, A0, info0_dev, A1, info1_dev);
    return hip_check(c, hipGetLastError(), "k_small_cholesky");
}

bdg_status small_svd(bdg_ctx* c, int rows, int m, double2* G, int ldg, double2* V, int ldv, double* s, double conv,
                     bool real) {
    if (m <= 0) return BDG_OK;
    if (m > 512 || rows > 512) return ctx_fail(c, BDG_EINVAL, "small_svd: size out of range");
    static int lds_limit = 0;
    if (lds_limit == 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess || v <= 0)
            v = 64 * 1024;
        lds_limit = v;
    }
    // block width W: the 2W staged columns of G and the two 2W x 2W matrices (Gram and the
    // accumulated rotation) must fit in the workgroup's LDS
    const size_t esz = real ? sizeof(double) : sizeof(double2);
    auto lds_need = [&](int w) {
        return ((size_t)2 * w * (size_t)(rows | 1) + (size_t)2 * (2 * w) * (2 * w + 1)) * esz + 1024;
    };
    // W = 8 measured fastest on the 2-D and 3-D solves and on 80..240-column real matrices
    // (a round's time grows with W^2, the number of rounds falls with W); 16 and 4 are kept
    // for the LDS fallback
    int w = 8;
    while (w > 4 && lds_need(w) > (size_t)lds_limit) w >>= 1;
    if (lds_need(w) > (size_t)lds_limit)
        return ctx_fail(c, BDG_EINVAL, "small_svd: matrix too large for the LDS-staged Jacobi");
    int nblk = (m + w - 1) / w;
    if (nblk < 2) nblk = 2;
    if (nblk & 1) ++nblk;
    void* aux = nullptr;
    BDG_TRY(ctx_scratch(c, 3, 64, &aux));
    double* frob2 = (double*)aux;
    int* counter = (int*)((char*)aux + 16);
    hipLaunchKernelGGL(k_identity_frob, dim3(1), dim3(1024), 0, c->stream, rows, m, (const double2*)G, ldg, V, ldv,
                       frob2, counter);
    BDG_HIP(c, hipGetLastError());
    const size_t lds = lds_need(w) - 1024;
    const void* kern = real ? (w == 16 ? (const void*)k_bjacobi_round_r<16>
                               : w == 8 ? (const void*)k_bjacobi_round_r<8> : (const void*)k_bjacobi_round_r<4>)
                            : (w == 16 ? (const void*)k_bjacobi_round_g<16>
                               : w == 8 ? (const void*)k_bjacobi_round_g<8> : (const void*)k_bjacobi_round_g<4>);
    BDG_HIP(c, hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    // real rounds: nsplit workgroups per pair (the rotation computed by each, the rows shared
    // out); with nsplit > 1 the rounds alternate between (G, V) and a second copy
    int nsplit = 1;
    double2* Gb[2] = {G, G};
    double2* Vb[2] = {V, V};
    if (real && !c->arena.base && c->jacobi_split > 1) {
        nsplit = c->jacobi_split;
        void* pp = nullptr;
        BDG_TRY(ctx_scratch(c, 8, ((size_t)ldg * m + (size_t)ldv * m) * sizeof(double2), &pp));
        Gb[1] = (double2*)pp;
        Vb[1] = Gb[1] + (size_t)ldg * m;
    }
    int cur = 0;
#define BDG_ROUND(KN, WV)                                                                                         \
    hipLaunchKernelGGL(KN<WV>, dim3(nblk / 2), dim3(256), lds, c->stream, rows, m, G, ldg, V, ldv, nblk, rnd,   \
                       (const double*)frob2, counter, conv)
#define BDG_ROUND_R(WV)                                                                                           \
    hipLaunchKernelGGL(k_bjacobi_round_r<WV>, dim3(nblk / 2, nsplit), dim3(256), lds, c->stream, rows, m,       \
                       (const double2*)Gb[cur], ldg, (const double2*)Vb[cur], ldv,                              \
                       Gb[nsplit > 1 ? cur ^ 1 : cur], Vb[nsplit > 1 ? cur ^ 1 : cur], nblk, rnd,              \
                       (const double*)frob2, counter, conv)
    for (int sweep = 0; sweep < 40; ++sweep) {
        hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, c->stream, counter);
        for (int rnd = 0; rnd < nblk - 1; ++rnd) {
            if (real) {
                if (w == 16) BDG_ROUND_R(16);
                else if (w == 8) BDG_ROUND_R(8);
                else BDG_ROUND_R(4);
                if (nsplit > 1) cur ^= 1;
            } else {
                if (w == 16) BDG_ROUND(k_bjacobi_round_g, 16);
                else if (w == 8) BDG_ROUND(k_bjacobi_round_g, 8);
                else BDG_ROUND(k_bjacobi_round_g, 4);
            }
        }
        BDG_HIP(c, hipGetLastError());
        int h = 0;
        BDG_HIP(c, hipMemcpyAsync(&h, counter, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        BDG_HIP(c, hipStreamSynchronize(c->stream));
        if (h == 0) break;
    }
#undef BDG_ROUND
#undef BDG_ROUND_R
    if (cur == 1) {
        BDG_HIP(c, hipMemcpy2DAsync(G, (size_t)ldg * sizeof(double2), Gb[1], (size_t)ldg * sizeof(double2),
                                    (size_t)rows * sizeof(double2), (size_t)m, hipMemcpyDeviceToDevice, c->stream));
        BDG_HIP(c, hipMemcpy2DAsync(V, (size_t)ldv * sizeof(double2), Vb[1], (size_t)ldv * sizeof(double2),
                                    (size_t)m * sizeof(double2), (size_t)m, hipMemcpyDeviceToDevice, c->stream));
    }
    void* ws = nullptr;
    BDG_TRY(ctx_scratch(c, 1, ((size_t)rows * m + (size_t)m * m) * sizeof(double2), &ws));
    hipLaunchKernelGGL(k_small_sort, dim3(1), dim3(1024), 0, c->stream, rows, m, G, ldg, V, ldv, s, (double2*)ws,
                       (double2*)ws + (size_t)rows * m);
    return hip_check(c, hipGetLastError(), "k_small_sort");
}
