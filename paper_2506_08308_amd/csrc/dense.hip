// Tall-skinny linear algebra of the subspace iteration on gfx950 (Section 3.2): the Gram
// matrices X^H Y of the bi-orthogonal Gram-Schmidt and Rayleigh-Ritz steps and the basis
// updates S C run on the FP64 matrix cores (v_mfma_f64_16x16x4f64), with the column norms
// and dot products of the block.  The projected m x m problems are in smalldense.hip.
// Complex numbers are interleaved (re, im) doubles.
//
// MFMA operand layout (16x16x4 f64, wave64; checked on the device): lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator register r of lane l holds D[4 r + l / 16][l % 16].
#include "common.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ----------------------------------------------------------------------------------------
// Gram: part[s] = A^H B over the K-range of split s.  Three forms, picked per launch: the
// thin one when m1 <= 16, else the cheaper tiling by a cost model measured on the device.
//  * k_gram: tiles of 64 x 64, 4 waves of 32 x 32.  The real form uses the interleaved
//    doubles as 2K real rows: Re C = a^T b,  Im C = a^T b'  with b'[2k] = Im B[k],
//    b'[2k+1] = -Re B[k].  Each wave reuses every fragment in two or four MFMAs.
//  * k_gram80: tiles of 80 x 80 (5 x 5 blocks of 16), 10 waves; no padding for m1, m2 that
//    are multiples of 80 (the solver's blocks), where the 64-tiling pads 80 to 128.
//  * k_gram_thin: m1 <= 16, one block row.
// ----------------------------------------------------------------------------------------
struct SegList {
    const double2* p[4];
    int start[5];
    int nseg;
};

// Column col of a segment list, the segment picked by selects over the (uniform) segment
// table: a per-lane index into the argument block would compile to vector loads, and waiting
// on them also waits on the prefetch loads already in flight.
__device__ __forceinline__ const double2* seg_col(const SegList& sl, int col, long long ld) {
    const double2* p = sl.p[0];
    int s0 = 0;
#pragma unroll
    for (int g = 1; g < 4; ++g)
        if (g < sl.nseg && col >= sl.start[g]) {
            p = sl.p[g];
            s0 = sl.start[g];
        }
    return p + (long long)(col - s0) * ld;
}

constexpr int GT = 64;          // output tile edge
constexpr int GKC = 16;         // complex rows per LDS chunk (32 real rows)
constexpr int GKR = 2 * GKC;
// LDS pitch of a staged column in doubles.  A fragment read has lane l at column l % 16 and
// real row l / 16; with a pitch of 2 mod 32 each half-wave's 32 doubles fall on 64 distinct
// 4-byte banks (a pitch of 33 put two lanes on each bank pair: 40 % of the LDS cycles were
// bank conflicts), and an even pitch keeps the complex pairs 16-byte aligned for b128 stores.
constexpr int GPAD = GKR + 2;

// Work item -> (split, tile).  Workgroups are dispatched to the 8 XCDs round-robin by linear
// id, so item w = (id % 8) * per_xcd + id / 8 gives every XCD a contiguous run of items: all
// tiles of one K-split then run on the same XCD at about the same time and share its L2,
// and each panel row is fetched from HBM about once.  Hermitian Grams enumerate the upper
// tiles only.
__device__ __forceinline__ bool gram_item(long long L, long long per_xcd, long long total, int ntiles, int tn,
                                          int herm, long long* split, int* ti, int* tj) {
    const long long w = (L & 7) * per_xcd + (L >> 3);
    if (w >= total) return false;
    *split = w / ntiles;
    int tile = (int)(w % ntiles);
    if (!herm) {
        *ti = tile / tn;
        *tj = tile % tn;
        return true;
    }
    int r = 0;
    while (tile >= tn - r) {
        tile -= tn - r;
        ++r;
    }
    *ti = r;
    *tj = r + tile;
    return true;
}

__global__ void __launch_bounds__(256) k_gram(long long K, int m1, int m2, SegList A, long long lda, SegList B,
                                              long long ldb, long long kper, int tn, int herm, int same,
                                              int ntiles, long long total, long long per_xcd,
                                              double2* __restrict__ part) {
    __shared__ __align__(16) double la[GT * GPAD];
    __shared__ __align__(16) double lb[GT * GPAD];
    long long split;
    int ti, tj;
    if (!gram_item(blockIdx.x, per_xcd, total, ntiles, tn, herm, &split, &ti, &tj)) return;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double2* out = part + split * m1 * m2;
    // diagonal tiles of a Gram of one block with itself (A == B) read one panel
    const bool diag = same && ti == tj;
    const double* lbr = diag ? la : lb;
    const int p0 = ti * GT, q0 = tj * GT;
    const long long k0 = split * kper;
    long long k1 = k0 + kper;
    if (k1 > K) k1 = K;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;   // wave sub-tile
    // the strictly lower sub-tile of a Hermitian diagonal tile is the mirror of the upper one
    // (filled by the reduction): its wave only helps stage the panels
    const bool idle = herm && ti == tj && wr > wc;
    d4 accr[2][2], acci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) { accr[a][b] = d4{0, 0, 0, 0}; acci[a][b] = d4{0, 0, 0, 0}; }
    // loader mapping: 256 threads, 16 lanes per column chunk, 16 columns per pass, 4 passes
    const int lk = t & 15, lc = t >> 4;
    const double2* acol[4];
    const double2* bcol[4];
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
        const int col = lc + 16 * pass;
        acol[pass] = (p0 + col < m1) ? seg_col(A, p0 + col, lda) : nullptr;
        bcol[pass] = (!diag && q0 + col < m2) ? seg_col(B, q0 + col, ldb) : nullptr;
    }
    // the next chunk is held in registers while the current one is multiplied
    double2 ra[4], rb[4];
    auto gload = [&](long long kc) {
        const long long kk = kc + lk;
#pragma unroll
        for (int pass = 0; pass < 4; ++pass) {
            ra[pass] = (kk < k1 && acol[pass]) ? acol[pass][kk] : double2{0, 0};
            rb[pass] = (kk < k1 && bcol[pass]) ? bcol[pass][kk] : double2{0, 0};
        }
    };
    gload(k0);
    for (long long kc = k0; kc < k1; kc += GKC) {
        __syncthreads();
#pragma unroll
        for (int pass = 0; pass < 4; ++pass) {
            const int col = lc + 16 * pass;
            *reinterpret_cast<double2*>(&la[col * GPAD + 2 * lk]) = ra[pass];
            if (!diag) *reinterpret_cast<double2*>(&lb[col * GPAD + 2 * lk]) = rb[pass];
        }
        __syncthreads();
        if (kc + GKC < k1) gload(kc + GKC);
        if (idle) continue;
        // raised issue priority while this wave streams MFMAs (the other resident waves are
        // loading or staging): measured 2-3 % on the Gram shapes of the solve
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < GKR; ks += 4) {
            const int kr = ks + (lane >> 4);        // real row of this lane
            const int ci = lane & 15;
            double av[2], bv[2], bpv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = la[(wr + 16 * a + ci) * GPAD + kr];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int row = (wc + 16 * b + ci) * GPAD;
                bv[b] = lbr[row + kr];
                // b'[2k] = Im B[k], b'[2k+1] = -Re B[k]
                bpv[b] = (kr & 1) ? -lbr[row + kr - 1] : lbr[row + kr + 1];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    accr[a][b] = mfma(av[a], bv[b], accr[a][b]);
                    acci[a][b] = mfma(av[a], bpv[b], acci[a][b]);
                }
        }
        __builtin_amdgcn_s_setprio(0);
    }
    if (idle) return;
    // write the partial tile: register r of lane l holds D[4 r + l / 16][l % 16]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = p0 + wr + 16 * a + 4 * r + (lane >> 4);
                const int q = q0 + wc + 16 * b + (lane & 15);
                if (p < m1 && q < m2) {
                    double2 v;
                    v.x = accr[a][b][r];
                    v.y = acci[a][b][r];
                    out[(long long)q * m1 + p] = v;
                }
            }
}

// Paired real form: every complex column holds two real columns (real part, imaginary part),
// and part[s] receives the real Gram R = Ar^T Br of the 2 m1 and 2 m2 real columns
// (R[2p + u][2q + v] = sum_k A_u[k, p] B_v[k, q], u, v = 0 for the real, 1 for the imaginary
// parts), column-major with leading dimension 2 m1.  Same tiles, staging and work order as
// k_gram (tiles of 64 x 64 complex columns, i.e. 128 x 128 real entries); the MFMAs run over
// complex rows with the two parts as separate operands, so a tile takes as many MFMAs as a
// complex tile while covering four real entries per pair of complex columns.
__global__ void __launch_bounds__(256) k_gram_pair(long long K, int m1, int m2, SegList A, long long lda, SegList B,
                                                   long long ldb, long long kper, int tn, int herm, int same,
                                                   int ntiles, long long total, long long per_xcd,
                                                   double* __restrict__ part) {
    __shared__ __align__(16) double la[GT * GPAD];
    __shared__ __align__(16) double lb[GT * GPAD];
    long long split;
    int ti, tj;
    if (!gram_item(blockIdx.x, per_xcd, total, ntiles, tn, herm, &split, &ti, &tj)) return;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const long long ldr = 2LL * m1;
    double* out = part + split * ldr * (2LL * m2);
    const bool diag = same && ti == tj;
    const double* lbr = diag ? la : lb;
    const int p0 = ti * GT, q0 = tj * GT;
    const long long k0 = split * kper;
    long long k1 = k0 + kper;
    if (k1 > K) k1 = K;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const bool idle = herm && ti == tj && wr > wc;
    // acc[a][b][2 u + v]: real part u of A's block a against part v of B's block b
    d4 acc[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[a][b][q] = d4{0, 0, 0, 0};
    const int lk = t & 15, lc = t >> 4;
    const double2* acol[4];
    const double2* bcol[4];
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
        const int col = lc + 16 * pass;
        acol[pass] = (p0 + col < m1) ? seg_col(A, p0 + col, lda) : nullptr;
        bcol[pass] = (!diag && q0 + col < m2) ? seg_col(B, q0 + col, ldb) : nullptr;
    }
    double2 ra[4], rb[4];
    auto gload = [&](long long kc) {
        const long long kk = kc + lk;
#pragma unroll
        for (int pass = 0; pass < 4; ++pass) {
            ra[pass] = (kk < k1 && acol[pass]) ? acol[pass][kk] : double2{0, 0};
            rb[pass] = (kk < k1 && bcol[pass]) ? bcol[pass][kk] : double2{0, 0};
        }
    };
    gload(k0);
    for (long long kc = k0; kc < k1; kc += GKC) {
        __syncthreads();
#pragma unroll
        for (int pass = 0; pass < 4; ++pass) {
            const int col = lc + 16 * pass;
            *reinterpret_cast<double2*>(&la[col * GPAD + 2 * lk]) = ra[pass];
            if (!diag) *reinterpret_cast<double2*>(&lb[col * GPAD + 2 * lk]) = rb[pass];
        }
        __syncthreads();
        if (kc + GKC < k1) gload(kc + GKC);
        if (idle) continue;
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < GKC; ks += 4) {
            const int kr = 2 * (ks + (lane >> 4));  // first double of this lane's complex row
            const int ci = lane & 15;
            double2 av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = *reinterpret_cast<const double2*>(&la[(wr + 16 * a + ci) * GPAD + kr]);
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = *reinterpret_cast<const double2*>(&lbr[(wc + 16 * b + ci) * GPAD + kr]);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc[a][b][0] = mfma(av[a].x, bv[b].x, acc[a][b][0]);
                    acc[a][b][1] = mfma(av[a].x, bv[b].y, acc[a][b][1]);
                    acc[a][b][2] = mfma(av[a].y, bv[b].x, acc[a][b][2]);
                    acc[a][b][3] = mfma(av[a].y, bv[b].y, acc[a][b][3]);
                }
        }
        __builtin_amdgcn_s_setprio(0);
    }
    if (idle) return;
    // register r of lane l holds D[4 r + l / 16][l % 16]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = p0 + wr + 16 * a + 4 * r + (lane >> 4);
                const int q = q0 + wc + 16 * b + (lane & 15);
                if (p < m1 && q < m2) {
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int v = 0; v < 2; ++v) out[(2LL * q + v) * ldr + 2 * p + u] = acc[a][b][2 * u + v][r];
                }
            }
}

// Whole-matrix form of the paired Gram: one workgroup of 8 waves holds every block pair of
// its K-split (blocks of 16 complex columns; symmetric: the upper pairs bi <= bj), so each
// input row is staged once per split instead of once per tile row and column.  Taken for
// symmetric Grams of 65..128 complex columns (the Rayleigh-Ritz Grams: 36 pairs) and for
// general ones of at most 40 pairs within 128 x 128 (the F rows of the projected operators,
// 3 x 8 pairs).  Wave w takes a contiguous run of the pairs (at most WB = 5), four
// accumulators (u, v) per pair.
constexpr int WGM = 128;        // columns staged per operand
constexpr int WB = 5;           // block pairs per wave
__global__ void __launch_bounds__(512) k_gram_pair_wide(long long K, int m1, int m2, int herm, SegList A,
                                                        long long lda, SegList B, long long ldb, long long kper,
                                                        int same, double* __restrict__ part) {
    __shared__ __align__(16) double la[WGM * GPAD];
    __shared__ __align__(16) double lb[WGM * GPAD];
    const long long split = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const long long ldr = 2LL * m1;
    double* out = part + split * ldr * (2LL * m2);
    const double* lbr = same ? la : lb;
    const long long k0 = split * kper;
    long long k1 = k0 + kper;
    if (k1 > K) k1 = K;
    // this wave's block pairs in row order, dealt out in runs
    const int nb1 = (m1 + 15) / 16, nb2 = (m2 + 15) / 16;
    const int npairs = herm ? nb1 * (nb1 + 1) / 2 : nb1 * nb2;
    const int base = npairs / 8, extra = npairs % 8;
    const int first = wave * base + (wave < extra ? wave : extra);
    const int cnt = base + (wave < extra ? 1 : 0);
    int bi[WB], bj[WB];
#pragma unroll
    for (int j = 0; j < WB; ++j) {
        int e = first + j;
        if (herm) {
            int r = 0;
            while (r < nb1 && e >= nb1 - r) {
                e -= nb1 - r;
                ++r;
            }
            bi[j] = r;
            bj[j] = r + e;
        } else {
            bi[j] = e / nb2;
            bj[j] = e % nb2;
        }
    }
    d4 acc[WB][4];
#pragma unroll
    for (int j = 0; j < WB; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[j][q] = d4{0, 0, 0, 0};
    // staging: thread t loads complex row lk of columns lc + 32 pass (pass < 4)
    const int lk = t & 15, lc = t >> 4;
    const double2* acol[4];
    const double2* bcol[4];
#pragma unroll
    for (int pass = 0; pass < 4; ++pass) {
        const int col = lc + 32 * pass;
        acol[pass] = col < m1 ? seg_col(A, col, lda) : nullptr;
        bcol[pass] = (!same && col < m2) ? seg_col(B, col, ldb) : nullptr;
    }
    double2 ra[4], rb[4];
    auto gload = [&](long long kc) {
        const long long kk = kc + lk;
#pragma unroll
        for (int pass = 0; pass < 4; ++pass) {
            ra[pass] = (kk < k1 && acol[pass]) ? acol[pass][kk] : double2{0, 0};
            rb[pass] = (kk < k1 && bcol[pass]) ? bcol[pass][kk] : double2{0, 0};
        }
    };
    gload(k0);
    for (long long kc = k0; kc < k1; kc += GKC) {
        __syncthreads();
#pragma unroll
        for (int pass = 0; pass < 4; ++pass) {
            const int col = lc + 32 * pass;
            *reinterpret_cast<double2*>(&la[col * GPAD + 2 * lk]) = ra[pass];
            if (!same) *reinterpret_cast<double2*>(&lb[col * GPAD + 2 * lk]) = rb[pass];
        }
        __syncthreads();
        if (kc + GKC < k1) gload(kc + GKC);
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < GKC; ks += 4) {
            const int kr = 2 * (ks + (lane >> 4));
            const int ci = lane & 15;
#pragma unroll
            for (int j = 0; j < WB; ++j) {
                if (j >= cnt) break;
                const double2 av = *reinterpret_cast<const double2*>(&la[(16 * bi[j] + ci) * GPAD + kr]);
                const double2 bv = *reinterpret_cast<const double2*>(&lbr[(16 * bj[j] + ci) * GPAD + kr]);
                acc[j][0] = mfma(av.x, bv.x, acc[j][0]);
                acc[j][1] = mfma(av.x, bv.y, acc[j][1]);
                acc[j][2] = mfma(av.y, bv.x, acc[j][2]);
                acc[j][3] = mfma(av.y, bv.y, acc[j][3]);
            }
        }
        __builtin_amdgcn_s_setprio(0);
    }
    // register r of lane l holds D[4 r + l / 16][l % 16]
#pragma unroll
    for (int j = 0; j < WB; ++j) {
        if (j >= cnt) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = 16 * bi[j] + 4 * r + (lane >> 4);
            const int q = 16 * bj[j] + (lane & 15);
            if (p < m1 && q < m2) {
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int v = 0; v < 2; ++v) out[(2LL * q + v) * ldr + 2 * p + u] = acc[j][2 * u + v][r];
            }
        }
    }
}

// Whole-matrix paired Gram with blocks of 8 complex columns (16 real): one 16 x 16 MFMA tile
// per block pair, so 120 complex columns need no padding and a diagonal tile wastes only its
// lower half (the 16-column blocks padded 120 to 128 and computed full 32 x 32 diagonal
// blocks: 22 % of their MFMAs).  A lane's A operand is one part of one complex column: real
// row r of block bi is part r % 2 of complex column 8 bi + r / 2.  One workgroup of 16 waves
// per K-split holds all tiles (symmetric: bi <= bj), at most W8T per wave.
constexpr int W8T = 9;
__global__ void __launch_bounds__(1024) k_gram_pair_w8(long long K, int m1, int m2, int herm, SegList A, long long lda,
                                                      SegList B, long long ldb, long long kper, int same,
                                                      double* __restrict__ part) {
    __shared__ __align__(16) double la[WGM * GPAD];
    __shared__ __align__(16) double lb[WGM * GPAD];
    const long long split = blockIdx.x;
    // the wave index (and all tile indices derived from it) is uniform: scalar registers
    const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const long long ldr = 2LL * m1;
    double* out = part + split * ldr * (2LL * m2);
    const double* lbr = same ? la : lb;
    const long long k0 = split * kper;
    long long k1 = k0 + kper;
    if (k1 > K) k1 = K;
    const int nb1 = (m1 + 7) / 8, nb2 = (m2 + 7) / 8;
    const int ntile = herm ? nb1 * (nb1 + 1) / 2 : nb1 * nb2;
    const int base = ntile / 16, extra = ntile % 16;
    const int first = wave * base + (wave < extra ? wave : extra);
    const int cnt = base + (wave < extra ? 1 : 0);
    int bi[W8T], bj[W8T];
#pragma unroll
    for (int j = 0; j < W8T; ++j) {
        int e = first + j;
        if (herm) {
            int r = 0;
            while (r < nb1 && e >= nb1 - r) {
                e -= nb1 - r;
                ++r;
            }
            bi[j] = r;
            bj[j] = r + e;
        } else {
            bi[j] = e / nb2;
            bj[j] = e % nb2;
        }
    }
    d4 acc[W8T];
#pragma unroll
    for (int j = 0; j < W8T; ++j) acc[j] = d4{0, 0, 0, 0};
    // staging: thread t loads complex row lk of columns lc + 64 pass (pass < 2) of A and B
    const int lk = t & 15, lc = t >> 4;
    const double2* acol[2];
    const double2* bcol[2];
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
        const int col = lc + 64 * pass;
        acol[pass] = col < m1 ? seg_col(A, col, lda) : nullptr;
        bcol[pass] = (!same && col < m2) ? seg_col(B, col, ldb) : nullptr;
    }
    double2 ra[2], rb[2];
    auto gload = [&](long long kc) {
        const long long kk = kc + lk;
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            ra[pass] = (kk < k1 && acol[pass]) ? acol[pass][kk] : double2{0, 0};
            rb[pass] = (kk < k1 && bcol[pass]) ? bcol[pass][kk] : double2{0, 0};
        }
    };
    // this lane's operand offsets within a block: column (lane % 16) / 2, part lane % 2,
    // complex row lane / 16 of the four of a step
    const int ci = (lane & 15) >> 1, cu = lane & 1, kq = lane >> 4;
    gload(k0);
    for (long long kc = k0; kc < k1; kc += GKC) {
        __syncthreads();
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            const int col = lc + 64 * pass;
            *reinterpret_cast<double2*>(&la[col * GPAD + 2 * lk]) = ra[pass];
            if (!same) *reinterpret_cast<double2*>(&lb[col * GPAD + 2 * lk]) = rb[pass];
        }
        __syncthreads();
        if (kc + GKC < k1) gload(kc + GKC);
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < GKC; ks += 4) {
            const int kr = 2 * (ks + kq) + cu;
#pragma unroll
            for (int j = 0; j < W8T; ++j) {
                if (j < cnt) {            // wave-uniform
                    const double av = la[(8 * bi[j] + ci) * GPAD + kr];
                    const double bv = lbr[(8 * bj[j] + ci) * GPAD + kr];
                    acc[j] = mfma(av, bv, acc[j]);
                }
            }
        }
        __builtin_amdgcn_s_setprio(0);
    }
    // register r of lane l holds D[4 r + l / 16][l % 16]: real row 16 bi + 4 r + l / 16,
    // real column 16 bj + l % 16
#pragma unroll
    for (int j = 0; j < W8T; ++j) {
        if (j >= cnt) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = 16 * bi[j] + 4 * r + (lane >> 4);
            const int q = 16 * bj[j] + (lane & 15);
            if (p < 2 * m1 && q < 2 * m2) out[(long long)q * ldr + p] = acc[j][r];
        }
    }
}

// The same Gram with the operands loaded straight into LDS (global_load_lds_dwordx4: lane l
// of a wave's load writes 16 bytes at the instruction's LDS base + 16 l).  A load fills one
// block of 8 complex columns x 8 complex rows, lane l taking column l % 8 and row l / 8, so
// a block holds row r of its columns at slots 8 r .. 8 r + 7.  An MFMA step reads, for lane l,
// real row l / 16 (complex row kq, part l % 2) of column (l % 16) / 2: in a block that is
// double 16 kq + l % 16, so a wave reads 512 contiguous bytes.  Chunks of 16 complex rows
// alternate between two buffers: one barrier per chunk, the loads of the next chunk in
// flight while this one is multiplied, and no staging registers.  Rows past the end of the
// split are loaded from its last row and zeroed by the lane that loaded them.
constexpr int W8B = 16;                      // column blocks per operand (128 complex columns)
constexpr int W8BUF = 2 * W8B * 128;         // doubles per operand and buffer (32 KiB)
__global__ void __launch_bounds__(1024) k_gram_pair_w8d(long long K, int m1, int m2, int herm, SegList A,
                                                       long long lda, SegList B, long long ldb, long long kper,
                                                       int same, double* __restrict__ part) {
    // [operand][buffer][column block][row half][64 complex]
    __shared__ __align__(16) double lds[2 * 2 * W8BUF];
    const long long split = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const long long ldr = 2LL * m1;
    double* out = part + split * ldr * (2LL * m2);
    const long long k0 = split * kper;
    long long k1 = k0 + kper;
    if (k1 > K) k1 = K;
    const int nb1 = (m1 + 7) / 8, nb2 = (m2 + 7) / 8;
    const int ntile = herm ? nb1 * (nb1 + 1) / 2 : nb1 * nb2;
    const int base = ntile / 16, extra = ntile % 16;
    const int first = wave * base + (wave < extra ? wave : extra);
    const int cnt = base + (wave < extra ? 1 : 0);
    // this lane's read addresses (bytes) of each tile's A and B blocks, row half 0, buffer 0
    unsigned ra[W8T], rb[W8T];
#pragma unroll
    for (int j = 0; j < W8T; ++j) {
        int e = first + j;
        int bi, bj;
        if (herm) {
            int r = 0;
            while (r < nb1 && e >= nb1 - r) {
                e -= nb1 - r;
                ++r;
            }
            bi = r;
            bj = r + e;
        } else {
            bi = e / nb2;
            bj = e % nb2;
        }
        ra[j] = (unsigned)(((2 * bi) * 128 + lane) * 8);
        rb[j] = (unsigned)(((same ? 0 : 2 * W8BUF) + (2 * bj) * 128 + lane) * 8);
    }
    d4 acc[W8T];
#pragma unroll
    for (int j = 0; j < W8T; ++j) acc[j] = d4{0, 0, 0, 0};
    // the blocks this wave loads each chunk: q = wave + 16 i; A blocks first (2 per column
    // block), then B's.  Column pointers are fixed; padding columns repeat the last column
    // (they only reach outputs that are not stored)
    const int nqa = 2 * nb1, nq = nqa + (same ? 0 : 2 * nb2);
    const double2* colp[4];
    unsigned ldsq[4];                 // LDS byte offset of block q, buffer 0
    int rowoff[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = wave + 16 * i;
        colp[i] = nullptr;
        ldsq[i] = 0;
        rowoff[i] = 0;
        if (q < nq) {
            const bool isa = q < nqa;
            const int qq = isa ? q : q - nqa;
            const int cb = qq >> 1, rh = qq & 1;
            const int mm = isa ? m1 : m2;
            int col = 8 * cb + (lane & 7);
            if (col >= mm) col = mm - 1;
            colp[i] = isa ? seg_col(A, col, lda) : seg_col(B, col, ldb);
            ldsq[i] = (unsigned)(((isa ? 0 : 2 * W8BUF) + (2 * cb + rh) * 128) * 8);
            rowoff[i] = 8 * rh + (lane >> 3);
        }
    }
    char* lbase = reinterpret_cast<char*>(lds);
    auto issue = [&](long long kc, int buf) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (wave + 16 * i < nq) {            // wave-uniform
                long long row = kc + rowoff[i];
                if (row >= k1) row = k1 - 1;
                __builtin_amdgcn_global_load_lds(
                    (const void*)(colp[i] + row),
                    (__attribute__((address_space(3))) void*)(lbase + ldsq[i] + buf * (W8BUF * 8)), 16, 0, 0);
            }
        }
    };
    // rows of a partial chunk past k1: zero the slots this lane loaded (after its loads landed)
    auto zero_tail = [&](long long kc, int buf) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (wave + 16 * i < nq && kc + rowoff[i] >= k1)
                *reinterpret_cast<double2*>(lbase + ldsq[i] + buf * (W8BUF * 8) + 16 * lane) = double2{0, 0};
    };
    auto step = [&](long long kc, auto bufc) {
        constexpr int BUF = decltype(bufc)::value;
        __builtin_amdgcn_s_waitcnt(0x3F70);      // vmcnt(0): this wave's loads of the chunk landed
        if (kc + GKC > k1) zero_tail(kc, BUF);
        __syncthreads();                         // every wave's loads landed; the other buffer is free
        if (kc + GKC < k1) issue(kc + GKC, BUF ^ 1);
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < GKC; ks += 4) {
            // row half ks / 8 (blocks 1 KiB apart), rows ks % 8 .. + 3 (128 bytes each)
            const unsigned off = BUF * (W8BUF * 8) + (ks >> 3) * 1024 + (ks & 7) * 128;
#pragma unroll
            for (int j = 0; j < W8T; ++j) {
                if (j < cnt) {            // wave-uniform
                    const double av = *reinterpret_cast<const double*>(lbase + ra[j] + off);
                    const double bv = *reinterpret_cast<const double*>(lbase + rb[j] + off);
                    acc[j] = mfma(av, bv, acc[j]);
                }
            }
        }
        __builtin_amdgcn_s_setprio(0);
    };
    if (k0 < k1) issue(k0, 0);
    for (long long kc = k0; kc < k1; kc += 2 * GKC) {
        step(kc, std::integral_constant<int, 0>{});
        if (kc + GKC >= k1) break;
        step(kc + GKC, std::integral_constant<int, 1>{});
    }
    // register r of lane l holds D[4 r + l / 16][l % 16]: real row 16 bi + 4 r + l / 16,
    // real column 16 bj + l % 16 (bi, bj recovered from the read addresses)
#pragma unroll
    for (int j = 0; j < W8T; ++j) {
        if (j >= cnt) continue;
        const int bi = (int)((ra[j] / 8 - lane) / 256);
        const int bj = (int)(((rb[j] / 8 - lane) - (same ? 0 : 2 * W8BUF)) / 256);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = 16 * bi + 4 * r + (lane >> 4);
            const int q = 16 * bj + (lane & 15);
            if (p < 2 * m1 && q < 2 * m2) out[(long long)q * ldr + p] = acc[j][r];
        }
    }
}

// C (m1 x m2 real entries in complex storage, imaginary parts 0) = alpha * sum over the splits
// of the real partials, in split order.  herm: only the entries on or above the diagonal
// 16 x 16 blocks are read (in their own column order, so a wave's reads are contiguous) and
// each is written to C and to its mirror; the paired kernels compute at least those blocks.
__global__ void k_gram_reduce_real(int m1, int m2, int nsplit, const double* __restrict__ part, double alpha,
                                   double2* __restrict__ C, int ldc, int herm) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)m1 * m2) return;
    const int p = (int)(idx % m1), q = (int)(idx / m1);
    if (herm && (p / 16) > (q / 16)) return;
    const long long plane = (long long)m1 * m2, off = (long long)q * m1 + p;
    double sx = 0;
    int s = 0;
    for (; s + 8 <= nsplit; s += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(s + u) * plane + off];
#pragma unroll
        for (int u = 0; u < 8; ++u) sx += v[u];
    }
    for (; s < nsplit; ++s) sx += part[s * plane + off];
    C[(long long)q * ldc + p] = double2{alpha * sx, 0.0};
    if (herm && (p / 16) < (q / 16)) C[(long long)p * ldc + q] = double2{alpha * sx, 0.0};
}

// Tiles of Q x Q blocks of 16 x 16 (k_gram80: Q = 5) on 2 Q waves.  Wave w computes the real
// (w even) or imaginary (w odd) part of its blocks with one A fragment per block row:
//   Re C = a^T b,  Im C = a'^T b  with a'[2k] = -Im A[k], a'[2k+1] = Re A[k],
// so it holds one accumulator per block.  Off-diagonal tiles give the pair w / 2 block row
// w / 2, all Q blocks.  A diagonal tile of a Hermitian Gram computes its Q (Q + 1) / 2 upper
// blocks only, numbered row by row and dealt out ND to a pair ((Q + 1) / 2 each for odd Q).
template <int Q>
struct GramShape {
    static constexpr int T = 16 * Q;
    static constexpr int NT = 128 * Q;
    static constexpr int NUP = Q * (Q + 1) / 2;
    static constexpr int ND = (NUP + Q - 1) / Q;
};

// One tile over the rows [k0, k1).
template <int Q, int NB, bool TRI>
__device__ __forceinline__ void gram_tile(double* la, double* lb, bool one_panel, long long k0, long long k1,
                                          int p0, int q0, int m1, int m2, const SegList& A, long long lda,
                                          const SegList& B, long long ldb, double2* __restrict__ out) {
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int pair = wave >> 1, part = wave & 1;
    int bi[NB], bj[NB];
    bool live[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        if (TRI) {
            int e = pair * NB + k;
            live[k] = e < GramShape<Q>::NUP;
            if (!live[k]) e = 0;
            int r = 0;
            while (e >= Q - r) {
                e -= Q - r;
                ++r;
            }
            bi[k] = r;
            bj[k] = r + e;
        } else {
            live[k] = true;
            bi[k] = pair;
            bj[k] = k;
        }
    }
    const double* lbr = one_panel ? la : lb;
    d4 acc[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) acc[k] = d4{0, 0, 0, 0};
    // loader mapping: 16 lanes per column chunk, 8 Q columns per pass, 2 passes
    const int lk = t & 15, lc = t >> 4;
    // the next chunk is held in registers while the current one is multiplied
    double2 ra[2], rb[2];
    auto gload = [&](long long kc) {
        const long long kk = kc + lk;
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            const int col = lc + 8 * Q * pass;
            ra[pass] = (kk < k1 && p0 + col < m1) ? seg_col(A, p0 + col, lda)[kk] : double2{0, 0};
            rb[pass] = (kk < k1 && !one_panel && q0 + col < m2) ? seg_col(B, q0 + col, ldb)[kk]
                                                                 : double2{0, 0};
        }
    };
    // real rows ks + lane / 16 with ks a multiple of 4: the parity is fixed per lane.  The
    // real part takes a = A[kr]; the imaginary part a' = (-Im, Re) of the complex pair:
    //   Re C = a^T b,  Im C = a'^T b.
    const bool odd = (lane >> 4) & 1;
    const bool hi = odd != (part == 1);          // take the second double of the pair
    const bool neg = part == 1 && !odd;
    gload(k0);
    for (long long kc = k0; kc < k1; kc += GKC) {
        __syncthreads();
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            const int col = lc + 8 * Q * pass;
            *reinterpret_cast<double2*>(&la[col * GPAD + 2 * lk]) = ra[pass];
            if (!one_panel) *reinterpret_cast<double2*>(&lb[col * GPAD + 2 * lk]) = rb[pass];
        }
        __syncthreads();
        if (kc + GKC < k1) gload(kc + GKC);
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < GKR; ks += 4) {
            const int kr = ks + (lane >> 4);        // real row of this lane
            const int kp = ks + ((lane >> 4) & 2);  // its complex pair (ks is a multiple of 4)
            const int ci = lane & 15;
            auto frag = [&](int blk) {
                const double2 pa = *reinterpret_cast<const double2*>(&la[(16 * blk + ci) * GPAD + kp]);
                const double v = hi ? pa.y : pa.x;
                return neg ? -v : v;
            };
            const double a0 = TRI ? 0.0 : frag(pair);
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const double a = TRI ? frag(bi[k]) : a0;
                acc[k] = mfma(a, lbr[(16 * bj[k] + ci) * GPAD + kr], acc[k]);
            }
        }
        __builtin_amdgcn_s_setprio(0);
    }
    // write the partial blocks: register r of lane l holds D[4 r + l / 16][l % 16]
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        if (!live[k]) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = p0 + 16 * bi[k] + 4 * r + (lane >> 4);
            const int q = q0 + 16 * bj[k] + (lane & 15);
            if (p < m1 && q < m2) reinterpret_cast<double*>(&out[(long long)q * m1 + p])[part] = acc[k][r];
        }
    }
}

// Four waves per SIMD (<= 128 registers): one workgroup of 10 waves per CU
__global__ void __launch_bounds__(640) __attribute__((amdgpu_waves_per_eu(4)))
k_gram80(long long K, int m1, int m2, SegList A, long long lda, SegList B, long long ldb, long long kper, int tn,
         int herm, int same, int ntiles, long long total, long long per_xcd, double2* __restrict__ part) {
    constexpr int Q = 5;
    constexpr int T = GramShape<Q>::T;
    __shared__ __align__(16) double la[T * GPAD];
    __shared__ __align__(16) double lb[T * GPAD];
    long long split;
    int ti, tj;
    if (!gram_item(blockIdx.x, per_xcd, total, ntiles, tn, herm, &split, &ti, &tj)) return;
    double2* out = part + split * m1 * m2;
    const long long k0 = split * kper;
    long long k1 = k0 + kper;
    if (k1 > K) k1 = K;
    // a diagonal tile of a Gram of one block with itself (A == B) reads one panel; a diagonal
    // tile of a Hermitian Gram computes its upper blocks only (the reduction mirrors the rest)
    const bool one_panel = same && ti == tj;
    if (herm && ti == tj)
        gram_tile<Q, GramShape<Q>::ND, true>(la, lb, one_panel, k0, k1, ti * T, tj * T, m1, m2, A, lda, B, ldb,
                                             out);
    else
        gram_tile<Q, Q, false>(la, lb, one_panel, k0, k1, ti * T, tj * T, m1, m2, A, lda, B, ldb, out);
}

// Thin Gram (m1 <= 16, e.g. projections onto a few deflation vectors and single dot
// products): one 16-row block of C.  A workgroup of 4 waves covers 64 columns of B over one
// K-split, wave w the block column w, with the real and imaginary parts from a and a' as in
// k_gram80.  Waves whose columns lie beyond m2 only help stage the panels.  The 64-tiling
// would execute at least four times the matrix-core work here.
__global__ void __launch_bounds__(256) k_gram_thin(long long K, int m1, int m2, SegList A, long long lda,
                                                   SegList B, long long ldb, long long kper, int ncg,
                                                   long long total, long long per_xcd,
                                                   double2* __restrict__ part) {
    __shared__ __align__(16) double la[16 * GPAD];
    __shared__ __align__(16) double lb[64 * GPAD];
    const long long L = blockIdx.x;
    const long long w = (L & 7) * per_xcd + (L >> 3);
    if (w >= total) return;
    const long long split = w / ncg;
    const int q0 = (int)(w % ncg) * 64;
    double2* out = part + split * m1 * m2;
    const long long k0 = split * kper;
    long long k1 = k0 + kper;
    if (k1 > K) k1 = K;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const bool idle = q0 + 16 * wave >= m2;
    // loader: 16 lanes per column chunk; A: 16 columns, B: 4 passes of 16 columns
    const int lk = t & 15, lc = t >> 4;
    double2 ra, rb[4];
    auto gload = [&](long long kc) {
        const long long kk = kc + lk;
        ra = (kk < k1 && lc < m1) ? seg_col(A, lc, lda)[kk] : double2{0, 0};
#pragma unroll
        for (int pass = 0; pass < 4; ++pass) {
            const int col = q0 + lc + 16 * pass;
            rb[pass] = (kk < k1 && col < m2) ? seg_col(B, col, ldb)[kk] : double2{0, 0};
        }
    };
    const bool odd = (lane >> 4) & 1;
    d4 accr = d4{0, 0, 0, 0}, acci = d4{0, 0, 0, 0};
    gload(k0);
    for (long long kc = k0; kc < k1; kc += GKC) {
        __syncthreads();
        *reinterpret_cast<double2*>(&la[lc * GPAD + 2 * lk]) = ra;
#pragma unroll
        for (int pass = 0; pass < 4; ++pass)
            *reinterpret_cast<double2*>(&lb[(lc + 16 * pass) * GPAD + 2 * lk]) = rb[pass];
        __syncthreads();
        if (kc + GKC < k1) gload(kc + GKC);
        if (idle) continue;
#pragma unroll
        for (int ks = 0; ks < GKR; ks += 4) {
            const int kr = ks + (lane >> 4);
            const int kp = ks + ((lane >> 4) & 2);
            const int ci = lane & 15;
            const double2 pa = *reinterpret_cast<const double2*>(&la[ci * GPAD + kp]);
            // a = A[kr]; a' = (-Im, Re) of the complex pair
            const double a = odd ? pa.y : pa.x;
            const double ap = odd ? pa.x : -pa.y;
            const double b = lb[(16 * wave + ci) * GPAD + kr];
            accr = mfma(a, b, accr);
            acci = mfma(ap, b, acci);
        }
    }
    if (idle) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int p = 4 * r + (lane >> 4);
        const int q = q0 + 16 * wave + (lane & 15);
        if (p < m1 && q < m2) {
            double2 v;
            v.x = accr[r];
            v.y = acci[r];
            out[(long long)q * m1 + p] = v;
        }
    }
}

// Thin Gram of at most 16 x 16 (dot products, projections onto one or two vectors) with deep
// staging.  k_gram_thin moves one 16-row chunk per pair of barriers; with m1 + m2 of two
// columns that is 512 bytes per workgroup in flight, a tenth of the bandwidth of the chip,
// and its one computing wave puts the matrix-core work of a CU on one SIMD.  Here a
// workgroup takes four K-splits, wave v the accumulator chain of split 4 w + v, and stages ds
// chunks of all four at once, the loads of the next ds chunks in flight while the waves
// execute the matrix-core steps of the current ones.  Split boundaries, chunk order, the
// operands of every MFMA and the accumulator chain are those of k_gram_thin (the zero padding
// of columns and rows included), so the partials are the same bits.  LDS: 4 splits x ds
// chunks x (m1 + m2) columns x GPAD doubles, A's columns first; a stage is THIN_TI items (one
// row of one column) per thread, two groups of 256 per split, rows fastest.
constexpr int THIN_TI = 8;

__global__ void __launch_bounds__(256) k_gram_thin_deep(long long K, int m1, int m2, SegList A, long long lda,
                                                        SegList B, long long ldb, long long kper, int ds,
                                                        long long nsplit, long long total, long long per_xcd,
                                                        double2* __restrict__ part) {
    extern __shared__ __align__(16) double lds_thin[];
    const long long L = blockIdx.x;
    const long long w = (L & 7) * per_xcd + (L >> 3);
    if (w >= total) return;
    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nc = m1 + m2;
    const int srows = ds * GKC;                 // rows per stage and split
    const int items = srows * nc;               // items per stage and split (<= 512)
    const int region = ds * nc * GPAD;          // doubles per split in LDS
    // the four splits' row ranges (an empty one past the last split)
    auto krange = [&](int v, long long* a, long long* e) {
        const long long sp = 4 * w + v;
        *a = sp < nsplit ? sp * kper : K;
        *e = sp < nsplit ? min(*a + kper, K) : K;
    };
    double2 rv[THIN_TI];
    auto gload = [&](long long off) {
#pragma unroll
        for (int u = 0; u < THIN_TI; ++u) {
            const int v = u >> 1;
            const int i = (u & 1) * 256 + t;
            const int col = i / srows, r = i - col * srows;
            long long a, e;
            krange(v, &a, &e);
            const long long kk = a + off + r;
            rv[u] = double2{0, 0};
            if (i < items && kk < e)
                rv[u] = col < m1 ? seg_col(A, col, lda)[kk] : seg_col(B, col - m1, ldb)[kk];
        }
    };
    const bool odd = (lane >> 4) & 1;
    const int ci = lane & 15;
    long long ka, ke;
    krange(wave, &ka, &ke);
    d4 accr = d4{0, 0, 0, 0}, acci = d4{0, 0, 0, 0};
    gload(0);
    for (long long off = 0; off < kper; off += srows) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < THIN_TI; ++u) {
            const int v = u >> 1;
            const int i = (u & 1) * 256 + t;
            if (i < items) {
                const int col = i / srows, r = i - col * srows;
                const int j = r / GKC, lk = r - j * GKC;
                *reinterpret_cast<double2*>(&lds_thin[v * region + (j * nc + col) * GPAD + 2 * lk]) = rv[u];
            }
        }
        __syncthreads();
        if (off + srows < kper) gload(off + srows);
        for (int j = 0; j < ds && ka + off + (long long)j * GKC < ke; ++j) {
            const double* la = lds_thin + wave * region + (j * nc) * GPAD;
            const double* lb = la + m1 * GPAD;
#pragma unroll
            for (int ks = 0; ks < GKR; ks += 4) {
                const int kr = ks + (lane >> 4);
                const int kp = ks + ((lane >> 4) & 2);
                const double2 pa = ci < m1 ? *reinterpret_cast<const double2*>(&la[ci * GPAD + kp]) : double2{0, 0};
                const double a = odd ? pa.y : pa.x;
                const double ap = odd ? pa.x : -pa.y;
                const double b = ci < m2 ? lb[ci * GPAD + kr] : 0.0;
                accr = mfma(a, b, accr);
                acci = mfma(ap, b, acci);
            }
        }
    }
    const long long sp = 4 * w + wave;
    if (sp >= nsplit) return;
    double2* out = part + sp * m1 * m2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int p = 4 * r + (lane >> 4);
        if (p < m1 && ci < m2) {
            double2 v;
            v.x = accr[r];
            v.y = acci[r];
            out[(long long)ci * m1 + p] = v;
        }
    }
}

// C = alpha * sum_s part[s] (fixed order); Hermitian: fill the lower triangle from the upper.
__global__ void k_gram_reduce(int m1, int m2, int nsplit, const double2* __restrict__ part, double alpha,
                              double2* __restrict__ C, int ldc, int herm) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)m1 * m2) return;
    int p = (int)(idx % m1), q = (int)(idx / m1);
    // Hermitian: both tilings compute every 16 x 16 block on and above the diagonal (k_gram
    // also the 32 x 32 diagonal sub-tiles whole); everything below is mirrored
    const bool mirror = herm && (p / 16) > (q / 16);
    const int ps = mirror ? q : p, qs = mirror ? p : q;
    double sx = 0, sy = 0;
    const long long plane = (long long)m1 * m2, off = (long long)qs * m1 + ps;
    // eight loads in flight, summed in split order (the same rounding as one at a time)
    int s = 0;
    for (; s + 8 <= nsplit; s += 8) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(s + u) * plane + off];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            sx += v[u].x;
            sy += v[u].y;
        }
    }
    for (; s < nsplit; ++s) {
        const double2 v = part[s * plane + off];
        sx += v.x;
        sy += v.y;
    }
    double2 o;
    o.x = alpha * sx;
    o.y = mirror ? -alpha * sy : alpha * sy;
    C[(long long)q * ldc + p] = o;
}

// The split-K reductions above give each entry one thread, which walks the splits with eight
// loads in flight: with few entries (a dot product, a projection onto two vectors) that is
// a few kilobytes in flight for the whole chip, and a reduction of 2500 splits takes 100 us.
// The staged form: a workgroup per G consecutive entries (G a power of two, G <= 64) stages
// the partials of RED_BYTES / (G sizeof(T)) splits at a time in LDS, every thread loading one
// entry's values at a stride of 256 / G splits, and thread e < G then adds up its entry's
// staged values in split order: the additions of the one-thread form in the same order, so
// the same bits.  The loads of the next splits are in flight while the sums run.
constexpr int RED_BYTES = 32768;

template <typename T>
__device__ __forceinline__ void red_add(T& a, const T& v) {
    if constexpr (std::is_same<T, double>::value) a += v;
    else { a.x += v.x; a.y += v.y; }
}

// sums over the splits of entry e0 + (t & (G - 1)) into *acc (threads t < G); off: offset of
// the thread's entry in a split's plane, live: whether it takes part
template <typename T>
__device__ __forceinline__ void staged_sum(int nsplit, const T* __restrict__ part, long long plane, long long off,
                                           bool live, int G, T* acc) {
    extern __shared__ __align__(16) unsigned char red_raw[];
    T* lred = reinterpret_cast<T*>(red_raw);
    constexpr int NI = RED_BYTES / (int)sizeof(T) / 256;      // staged values per thread
    const int t = threadIdx.x;
    const int sc = RED_BYTES / (int)sizeof(T) / G;          // splits per stage
    const int s_t = t / G, s_step = 256 / G;
    T rv[NI];
    auto gload = [&](int s0) {
#pragma unroll
        for (int u = 0; u < NI; ++u) {
            const int sp = s0 + s_t + u * s_step;
            rv[u] = T{};
            if (live && sp < nsplit) rv[u] = part[(long long)sp * plane + off];
        }
    };
    T a{};
    gload(0);
    for (int s0 = 0; s0 < nsplit; s0 += sc) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NI; ++u) lred[t + 256 * u] = rv[u];
        __syncthreads();
        if (s0 + sc < nsplit) gload(s0 + sc);
        if (t < G) {
            const int cnt = min(sc, nsplit - s0);
#pragma unroll 8
            for (int j = 0; j < cnt; ++j) red_add(a, lred[j * G + t]);
        }
    }
    *acc = a;
}

__global__ void __launch_bounds__(256) k_gram_reduce_st(int m1, int m2, int nsplit, const double2* __restrict__ part,
                                                        double alpha, double2* __restrict__ C, int ldc, int herm,
                                                        int G) {
    const long long tot = (long long)m1 * m2;
    const long long idx = (long long)blockIdx.x * G + (threadIdx.x & (G - 1));
    const bool live = idx < tot;
    int p = 0, q = 0;
    bool mirror = false;
    long long off = 0;
    if (live) {
        p = (int)(idx % m1);
        q = (int)(idx / m1);
        mirror = herm && (p / 16) > (q / 16);
        off = (long long)(mirror ? p : q) * m1 + (mirror ? q : p);
    }
    double2 sum;
    staged_sum<double2>(nsplit, part, tot, off, live, G, &sum);
    if ((int)threadIdx.x >= G || !live) return;
    double2 o;
    o.x = alpha * sum.x;
    o.y = mirror ? -alpha * sum.y : alpha * sum.y;
    C[(long long)q * ldc + p] = o;
}

__global__ void __launch_bounds__(256) k_gram_reduce_real_st(int m1, int m2, int nsplit,
                                                             const double* __restrict__ part, double alpha,
                                                             double2* __restrict__ C, int ldc, int herm, int G) {
    const long long tot = (long long)m1 * m2;
    const long long idx = (long long)blockIdx.x * G + (threadIdx.x & (G - 1));
    int p = 0, q = 0;
    bool live = idx < tot;
    if (live) {
        p = (int)(idx % m1);
        q = (int)(idx / m1);
        live = !(herm && (p / 16) > (q / 16));
    }
    double sum;
    staged_sum<double>(nsplit, part, tot, (long long)q * m1 + p, live, G, &sum);
    if ((int)threadIdx.x >= G || !live) return;
    C[(long long)q * ldc + p] = double2{alpha * sum, 0.0};
    if (herm && (p / 16) < (q / 16)) C[(long long)p * ldc + q] = double2{alpha * sum, 0.0};
}

// ----------------------------------------------------------------------------------------
// Update: Y (K x nb) = S (K x m) Cm (m x nb) + beta Z.  Each wave: 16 RA rows x 16 CB
// columns.
//   Re Y = Re S Re C - Im S Im C,  Im Y = Re S Im C + Im S Re C.
// Z may be Y (each element is read before it is written by the same lane); Y must not
// overlap S unless one workgroup covers all nb columns (grid.y == 1).
// Three waves per SIMD (<= 168 registers, 80 of them accumulators at CB = 5) with chunks of
// 8 columns: measured 14 % faster than two waves with 16-column chunks, whose staging
// registers do not fit three waves.
// ----------------------------------------------------------------------------------------
// PAIR: the paired real form (every complex column of S and Y holds two real columns, real
// part then imaginary part).  Cm then holds, for complex column l of S and j of Y, the real
// 2 x 2 coefficient block as two double2 at Cm[j ldcm + 2 l] = (c00, c01) and
// Cm[j ldcm + 2 l + 1] = (c10, c11) with c_uv the coefficient of real column 2 l + u of S in
// real column 2 j + v of Y; Y.x += S.x c00 + S.y c10, Y.y += S.x c01 + S.y c11.
// FUSE (paired form): the first mF columns of S are F, the rest [W, P]; the kernel writes
// Y2 = [W, P] C[mF:] (P_new) and Y = F C[:mF] + Y2 (F_new) in one pass with one set of
// accumulators: it visits the [W, P] chunks first, stores Y2 from the accumulators, and goes
// on with the F chunks.  Y may alias an input of the same rows: a workgroup reads all its
// input rows before it writes its output rows, and owns all output columns of its rows.
// ZPRE (plain form, one chunk of S, beta != 0, CB <= 3): the workgroup loads its Z
// elements first, so that their latency overlaps the loads and MFMAs of S C instead of
// following them (the projections of a block onto a few vectors, X -= Q (Q^H X)).  The same
// bits.
template <int CB, int RA, bool PAIR, bool FUSE = false, bool ZPRE = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_update(long long K, SegList segs, long long lds, int m,
                                                const double2* __restrict__ Cm, int ldcm, int nb, double beta,
                                                const double2* Z, long long ldz, double2* Y, long long ldy,
                                                int mF, double2* Y2, long long ldy2) {
    // a workgroup owns RW = 64 RA rows (each wave 16 RA rows) and 16 CB columns; LDS chunks of
    // UL columns of S and UL rows of Cm (2 UL for the paired form), the next chunk held in
    // registers while the MFMAs of the current one run
    constexpr int UL = 8;
    constexpr int NC = 16 * CB;
    constexpr int RW = 64 * RA;
    constexpr int SP = RW + 1;                       // row pitch of the S chunk (double2)
    constexpr int CR = PAIR ? 2 * UL : UL;           // staged coefficient rows per chunk
    __shared__ double2 lsS[UL * SP];
    __shared__ double2 lsC[CR * NC];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const long long R0 = (long long)blockIdx.x * RW;
    const int j0 = blockIdx.y * NC;
    const int ri = lane & 15, kq = lane >> 4;
    const int wr = wave * 16 * RA;
    d4 accr[RA][CB], acci[RA][CB];
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b) { accr[a][b] = d4{0, 0, 0, 0}; acci[a][b] = d4{0, 0, 0, 0}; }
    // chunk order: FUSE visits [mF, m) first (nwp chunks), then [0, mF); the plain form [0, m)
    const int nwp = FUSE ? (m - mF + UL - 1) / UL : 0;
    const int nchunk = FUSE ? nwp + mF / UL : (m + UL - 1) / UL;
    auto chunk_start = [&](int it) { return FUSE ? (it < nwp ? mF + it * UL : (it - nwp) * UL) : it * UL; };
    auto chunk_end = [&](int it) { return FUSE ? (it < nwp ? m : mF) : m; };
    constexpr int SPASS = UL * RW / 256;
    constexpr int CPASS = (CR * NC + 255) / 256;
    double2 rs[SPASS], rc[CPASS];
    auto gload = [&](int l0, int lend) {
#pragma unroll
        for (int u = 0; u < SPASS; ++u) {
            const int idx = u * 256 + t;
            const int l = l0 + idx / RW, row = idx % RW;
            rs[u] = double2{0, 0};
            if (l < lend && R0 + row < K) rs[u] = seg_col(segs, l, lds)[R0 + row];
        }
#pragma unroll
        for (int u = 0; u < CPASS; ++u) {
            const int idx = u * 256 + t;
            const int l = idx % CR, j = idx / CR;
            rc[u] = double2{0, 0};
            const int lc = PAIR ? l0 + l / 2 : l0 + l;
            const int row = PAIR ? 2 * l0 + l : l0 + l;
            if (idx < CR * NC && lc < lend && j0 + j < nb) rc[u] = Cm[(long long)(j0 + j) * ldcm + row];
        }
    };
    double2 zp[ZPRE ? RA : 1][ZPRE ? CB : 1][4];
    if constexpr (ZPRE) {
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const int j = j0 + 16 * b + (lane & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const long long row = R0 + wr + 16 * a + 4 * r + (lane >> 4);
                    zp[a][b][r] = (j < nb && row < K) ? Z[(long long)j * ldz + row] : double2{0, 0};
                }
            }
    }
    // accumulators -> Yo (plus beta Z in the plain form)
    auto store = [&](double2* Yo, long long ldo, bool with_z) {
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const int j = j0 + 16 * b + (lane & 15);
                if (j >= nb) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const long long row = R0 + wr + 16 * a + 4 * r + (lane >> 4);
                    if (row >= K) continue;
                    double2 v;
                    v.x = accr[a][b][r];
                    v.y = acci[a][b][r];
                    if (with_z && beta != 0.0) {
                        double2 o;
                        if constexpr (ZPRE) o = zp[a][b][r];
                        else o = Z[(long long)j * ldz + row];
                        v.x += beta * o.x;
                        v.y += beta * o.y;
                    }
                    Yo[(long long)j * ldo + row] = v;
                }
            }
    };
    if (FUSE && nwp == 0) store(Y2, ldy2, false);    // no [W, P] part: P_new = 0
    if (nchunk > 0) gload(chunk_start(0), chunk_end(0));
    for (int it = 0; it < nchunk; ++it) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < SPASS; ++u) {
            const int idx = u * 256 + t;
            lsS[(idx / RW) * SP + idx % RW] = rs[u];
        }
#pragma unroll
        for (int u = 0; u < CPASS; ++u) {
            const int idx = u * 256 + t;
            if (idx < CR * NC) lsC[(idx % CR) * NC + idx / CR] = rc[u];
        }
        __syncthreads();
        if (it + 1 < nchunk) gload(chunk_start(it + 1), chunk_end(it + 1));
#pragma unroll
        for (int ks = 0; ks < UL; ks += 4) {
            const int l = ks + kq;
            double2 sv[RA];
#pragma unroll
            for (int a = 0; a < RA; ++a) sv[a] = lsS[l * SP + wr + 16 * a + ri];
            double2 cv[CB], cw[CB];
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                if (PAIR) {
                    cv[b] = lsC[(2 * l) * NC + 16 * b + ri];        // (c00, c01)
                    cw[b] = lsC[(2 * l + 1) * NC + 16 * b + ri];    // (c10, c11)
                } else {
                    cv[b] = lsC[l * NC + 16 * b + ri];
                    cw[b] = double2{-cv[b].y, cv[b].x};              // complex: (c10, c11) = (-Im, Re)
                }
            }
            // the four real products in rounds over all tiles, so that two MFMAs into one
            // accumulator are 2 RA CB MFMAs apart
#pragma unroll
            for (int a = 0; a < RA; ++a)
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    accr[a][b] = mfma(sv[a].x, cv[b].x, accr[a][b]);
                    acci[a][b] = mfma(sv[a].x, cv[b].y, acci[a][b]);
                }
#pragma unroll
            for (int a = 0; a < RA; ++a)
#pragma unroll
                for (int b = 0; b < CB; ++b) {
                    accr[a][b] = mfma(sv[a].y, cw[b].x, accr[a][b]);
                    acci[a][b] = mfma(sv[a].y, cw[b].y, acci[a][b]);
                }
        }
        if (FUSE && it == nwp - 1) store(Y2, ldy2, false);   // P_new; F's chunks follow
    }
    store(Y, ldy, !FUSE);
}

// Update of at most 8 columns of S into at most 16 columns of Y (projections onto one or two
// vectors, dot-product sized work): one chunk of S, one column tile.  k_update spends a
// workgroup of 256 threads on 64 rows, and with one column that is 3 KB of traffic per
// workgroup, bound by the workgroup launch rate.  Here each wave walks UPD_UB row blocks of
// 16 at a time (all loads first) with the coefficients in registers, and executes for every
// block the MFMAs of k_update<1, 1, false> in the same order on the same operands (the zero
// padding of columns and rows included), so Y is the same bits.  Y may alias Z, or S within
// the same rows (a wave reads all its rows before it writes them).
constexpr int UPD_UB = 4;

__global__ void __launch_bounds__(256) k_update_thin(long long K, SegList segs, long long lds, int m,
                                                     const double2* __restrict__ Cm, int ldcm, int nb, double beta,
                                                     const double2* Z, long long ldz, double2* Y, long long ldy) {
    const int lane = threadIdx.x & 63;
    const int ri = lane & 15, kq = lane >> 4;
    // MFMA step s takes columns l = 4 s + kq of S and rows l of C, C(l, ri) on lane (ri, kq)
    double2 cv[2], cw[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int l = 4 * s + kq;
        cv[s] = (l < m && ri < nb) ? Cm[(long long)ri * ldcm + l] : double2{0, 0};
        cw[s] = double2{-cv[s].y, cv[s].x};
    }
    const double2* scol[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) scol[s] = 4 * s + kq < m ? seg_col(segs, 4 * s + kq, lds) : nullptr;
    const long long nrb = (K + 15) / 16;
    const long long nw = (long long)gridDim.x * 4;
    for (long long rb0 = ((long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * UPD_UB; rb0 < nrb; rb0 += nw * UPD_UB) {
        double2 sv[UPD_UB][2];
#pragma unroll
        for (int u = 0; u < UPD_UB; ++u) {
            const long long row = (rb0 + u) * 16 + ri;
#pragma unroll
            for (int s = 0; s < 2; ++s) sv[u][s] = (scol[s] && row < K) ? scol[s][row] : double2{0, 0};
        }
        double2 zv[UPD_UB][4];
#pragma unroll
        for (int u = 0; u < UPD_UB; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long row = (rb0 + u) * 16 + 4 * r + kq;
                zv[u][r] = (beta != 0.0 && ri < nb && row < K) ? Z[(long long)ri * ldz + row] : double2{0, 0};
            }
#pragma unroll
        for (int u = 0; u < UPD_UB; ++u) {
            d4 accr = d4{0, 0, 0, 0}, acci = d4{0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                accr = mfma(sv[u][s].x, cv[s].x, accr);
                acci = mfma(sv[u][s].x, cv[s].y, acci);
                accr = mfma(sv[u][s].y, cw[s].x, accr);
                acci = mfma(sv[u][s].y, cw[s].y, acci);
            }
            if (ri >= nb) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long row = (rb0 + u) * 16 + 4 * r + kq;
                if (row >= K) continue;
                double2 v;
                v.x = accr[r];
                v.y = acci[r];
                if (beta != 0.0) {
                    const double2 o = zv[u][r];
                    v.x += beta * o.x;
                    v.y += beta * o.y;
                }
                Y[(long long)ri * ldy + row] = v;
            }
        }
    }
}

// ----------------------------------------------------------------------------------------
// Column reductions (two-stage, fixed order)
// ----------------------------------------------------------------------------------------
constexpr int RB = 256;
__global__ void __launch_bounds__(RB) k_colnorm2_part(long long K, const double2* __restrict__ X, long long ldx,
                                                      long long kper, double* __restrict__ part) {
    __shared__ double red[RB / 64];
    const int col = blockIdx.y, chunk = blockIdx.x;
    const long long k0 = chunk * kper;
    long long k1 = k0 + kper;
    if (k1 > K) k1 = K;
    const double2* x = X + (long long)col * ldx;
    double s = 0;
    for (long long k = k0 + threadIdx.x; k < k1; k += RB) {
        double2 v = x[k];
        s += v.x * v.x + v.y * v.y;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0;
        for (int w = 0; w < RB / 64; ++w) a += red[w];
        part[(long long)col * gridDim.x + chunk] = a;
    }
}

// Paired real form: column reductions over the real columns 2 J + u (u = 0 real part, 1
// imaginary part) of complex column J.
// part[(2 J + u) * nchunk + chunk] = sum over the chunk of X_u[k, J]^2
__global__ void __launch_bounds__(RB) k_colnorm2_pair_part(long long K, const double2* __restrict__ X, long long ldx,
                                                           long long kper, double* __restrict__ part) {
    __shared__ double red[2][RB / 64];
    const int col = blockIdx.y, chunk = blockIdx.x;
    const long long k0 = chunk * kper;
    long long k1 = k0 + kper;
    if (k1 > K) k1 = K;
    const double2* x = X + (long long)col * ldx;
    double s0 = 0, s1 = 0;
    for (long long k = k0 + threadIdx.x; k < k1; k += RB) {
        const double2 v = x[k];
        s0 += v.x * v.x;
        s1 += v.y * v.y;
    }
    for (int off = 32; off > 0; off >>= 1) {
        s0 += __shfl_down(s0, off);
        s1 += __shfl_down(s1, off);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s0;
        red[1][threadIdx.x >> 6] = s1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double a = 0;
        for (int w = 0; w < RB / 64; ++w) a += red[threadIdx.x][w];
        part[(2LL * col + threadIdx.x) * gridDim.x + chunk] = a;
    }
}

// Residual norms of the real columns j = 2 J + u (omega_j = om[j]): partial sums of
// |HF_j - w G_j|^2, |HG_j - w F_j|^2, |F_j|^2, |G_j|^2 into part[((q * 2 ncols) + j) * nchunk + chunk]
// (ncols complex columns).  Dot products f_j . g_j with q = 4 when dots != 0 (5 sums).
__global__ void __launch_bounds__(RB) k_resnorm2_pair_part(long long K, const double2* __restrict__ HF,
                                                           const double2* __restrict__ G,
                                                           const double2* __restrict__ HG,
                                                           const double2* __restrict__ F, long long ld,
                                                           const double* __restrict__ om, long long kper,
                                                           double* __restrict__ part) {
    __shared__ double red[8][RB / 64];
    const int col = blockIdx.y, chunk = blockIdx.x, nr = 2 * gridDim.y;
    const long long k0 = chunk * kper;
    long long k1 = k0 + kper;
    if (k1 > K) k1 = K;
    const long long off = (long long)col * ld;
    const double w0 = om[2 * col], w1 = om[2 * col + 1];
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (long long k = k0 + threadIdx.x; k < k1; k += RB) {
        const double2 hf = HF[off + k], g = G[off + k], hg = HG[off + k], f = F[off + k];
        const double a0 = hf.x - w0 * g.x, a1 = hf.y - w1 * g.y;
        const double b0 = hg.x - w0 * f.x, b1 = hg.y - w1 * f.y;
        s[0] += a0 * a0;
        s[1] += a1 * a1;
        s[2] += b0 * b0;
        s[3] += b1 * b1;
        s[4] += f.x * f.x;
        s[5] += f.y * f.y;
        s[6] += g.x * g.x;
        s[7] += g.y * g.y;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        double v = s[q];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        const int q = threadIdx.x >> 1, u = threadIdx.x & 1;
        double a = 0;
        for (int wv = 0; wv < RB / 64; ++wv) a += red[threadIdx.x][wv];
        part[((long long)q * nr + 2 * col + u) * gridDim.x + chunk] = a;
    }
}

// Dot products of the real columns: part[(2 J + u) * nchunk + chunk] = sum F_u[k, J] G_u[k, J]
__global__ void __launch_bounds__(RB) k_dot_pair_part(long long K, const double2* __restrict__ F,
                                                      const double2* __restrict__ G, long long ld, long long kper,
                                                      double* __restrict__ part) {
    __shared__ double red[2][RB / 64];
    const int col = blockIdx.y, chunk = blockIdx.x;
    const long long k0 = chunk * kper;
    long long k1 = k0 + kper;
    if (k1 > K) k1 = K;
    const long long off = (long long)col * ld;
    double s0 = 0, s1 = 0;
    for (long long k = k0 + threadIdx.x; k < k1; k += RB) {
        const double2 f = F[off + k], g = G[off + k];
        s0 += f.x * g.x;
        s1 += f.y * g.y;
    }
    for (int o = 32; o > 0; o >>= 1) {
        s0 += __shfl_down(s0, o);
        s1 += __shfl_down(s1, o);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s0;
        red[1][threadIdx.x >> 6] = s1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double a = 0;
        for (int w = 0; w < RB / 64; ++w) a += red[threadIdx.x][w];
        part[(2LL * col + threadIdx.x) * gridDim.x + chunk] = a;
    }
}

// Paired coefficient blocks: for complex columns l < mp of S and j < nbp of Y,
// Cp[j ldp + 2 l] = (Cr[2 l, 2 j], Cr[2 l, 2 j + 1]), Cp[j ldp + 2 l + 1] = (Cr[2 l + 1, 2 j], Cr[2 l + 1, 2 j + 1])
// with Cr[i, jj] = real part of C[jj ldc + r0 + i]; ldp = 2 mp
__global__ void k_pack_pair_coef(int mp, int nbp, const double2* __restrict__ C, int ldc, int r0,
                                 double2* __restrict__ Cp) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (l >= mp || j >= nbp) return;
    const double2* c0 = C + (long long)(2 * j) * ldc + r0 + 2 * l;
    const double2* c1 = C + (long long)(2 * j + 1) * ldc + r0 + 2 * l;
    Cp[(long long)j * 2 * mp + 2 * l] = double2{c0[0].x, c1[0].x};
    Cp[(long long)j * 2 * mp + 2 * l + 1] = double2{c0[1].x, c1[1].x};
}

__global__ void k_colnorm2_final(int ncols, int nchunk, const double* __restrict__ part, double* out) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncols) return;
    double a = 0;
    const double* pc = part + (long long)col * nchunk;
    // eight loads in flight, summed in chunk order (the same rounding as one at a time)
    int c = 0;
    for (; c + 8 <= nchunk; c += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = pc[c + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) a += v[u];
    }
    for (; c < nchunk; ++c) a += pc[c];
    out[col] = a;
}

}  // namespace

// ======================================================================================
// host wrappers
// ======================================================================================
static bool make_seglist(const Seg* segs, int nseg, SegList* sl, int* m) {
    if (nseg < 1 || nseg > 4) return false;
    *sl = SegList{};
    int tot = 0;
    for (int i = 0; i < nseg; ++i) {
        sl->p[i] = (const double2*)segs[i].p;
        sl->start[i] = tot;
        tot += segs[i].ncols;
    }
    sl->start[nseg] = tot;
    sl->nseg = nseg;
    *m = tot;
    return true;
}

// K-splits of a Gram launch: about 2048 workgroups, rounded to whole rounds of the
// workgroups resident on the device at once (slots), so that the last round is not left
// partly empty; at least 512 rows per split; at most max_split splits (0: no cap).
// Returns the rows per split (a multiple of GKC).
// C = alpha * (sum over the nsplit partials in ws), by the staged or the one-thread form (the
// same bits); complex partials of the complex Grams, real ones of the paired Grams
static int reduce_group(long long tot) {
    int G = 1;
    while (G < 64 && 2LL * G * 128 <= tot) G *= 2;
    return G;
}

static bdg_status gram_reduce(bdg_ctx* c, int m1, int m2, long long nsplit, const void* ws, double alpha,
                              double2* C, int ldc, int herm) {
    const long long tot = (long long)m1 * m2;
    if (c->deep_loads) {
        const int G = reduce_group(tot);
        hipLaunchKernelGGL(k_gram_reduce_st, dim3((unsigned)((tot + G - 1) / G)), dim3(256), RED_BYTES, c->stream,
                           m1, m2, (int)nsplit, (const double2*)ws, alpha, C, ldc, herm, G);
    } else {
        hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, m1, m2,
                           (int)nsplit, (const double2*)ws, alpha, C, ldc, herm);
    }
    return hip_check(c, hipGetLastError(), "k_gram_reduce");
}

static bdg_status gram_reduce_real(bdg_ctx* c, int r1, int r2, long long nsplit, const void* ws, double alpha,
                                   double2* C, int ldc, int herm) {
    const long long tot = (long long)r1 * r2;
    if (c->deep_loads) {
        const int G = reduce_group(tot);
        hipLaunchKernelGGL(k_gram_reduce_real_st, dim3((unsigned)((tot + G - 1) / G)), dim3(256), RED_BYTES,
                           c->stream, r1, r2, (int)nsplit, (const double*)ws, alpha, C, ldc, herm, G);
    } else {
        hipLaunchKernelGGL(k_gram_reduce_real, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, r1, r2,
                           (int)nsplit, (const double*)ws, alpha, C, ldc, herm);
    }
    return hip_check(c, hipGetLastError(), "k_gram_reduce_real");
}

static long long gram_rows_per_split(long long K, long long items, long long slots, long long* nsplit,
                                     long long max_split) {
    const long long rounds = std::max<long long>(1, (2048 + slots / 2) / slots);
    long long ns = std::max<long long>(1, std::min<long long>((K + 511) / 512, rounds * slots / items));
    if (max_split > 0) ns = std::min(ns, max_split);
    long long kper = (K + ns - 1) / ns;
    kper = ((kper + GKC - 1) / GKC) * GKC;
    *nsplit = std::max<long long>(1, (K + kper - 1) / kper);
    return kper;
}

bdg_status gram_seg(bdg_ctx* c, long long K, const Seg* sa, int na, long long lda, const Seg* sb, int nbs,
                    long long ldb, double alpha, double2* C, int ldc, int hermitian) {
    SegList A, B;
    int m1 = 0, m2 = 0;
    if (!make_seglist(sa, na, &A, &m1) || !make_seglist(sb, nbs, &B, &m2))
        return ctx_fail(c, BDG_EINVAL, "gram: 1..4 segments");
    if (m1 <= 0 || m2 <= 0) return BDG_OK;
    if (hermitian && m1 != m2) return ctx_fail(c, BDG_EINVAL, "gram: Hermitian form needs m1 == m2");
    // in arena mode the split-K partials (nsplit m1 m2 complex values) stay within the
    // arena's Gram share
    const long long max_split =
        c->arena.base ? std::max<long long>(1, (long long)(c->arena.gram_bytes / ((size_t)m1 * m2 * sizeof(double2))))
                      : 0;
    // Tiling by measured cost (MI355X, 6.3 M rows): a 64-tile takes 0.204 ms per 16 x 16 block
    // it executes, an 80-tile 0.264 ms (the Hermitian diagonal tiles of either about as long
    // as a full tile), so 80-tiles win where they remove padding: m = 80 against 128, 80 x 240
    // against 128 x 256.
    auto tiles = [&](int edge) -> long long {
        const long long a = (m1 + edge - 1) / edge, b = (m2 + edge - 1) / edge;
        return hermitian ? b * (b + 1) / 2 : a * b;
    };
    if (m1 <= 16) {
        // thin form: every entry is computed, so the Hermitian flag only asks for the mirror
        // (no entry of a 16 x 16 block lies below its diagonal block)
        const int ncg = (m2 + 63) / 64;
        long long nsplit = 1;
        // five resident workgroups per CU (five waves per SIMD)
        const long long kper = gram_rows_per_split(K, ncg, 5LL * c->ncu, &nsplit, max_split);
        void* ws = nullptr;
        BDG_TRY(ctx_scratch(c, 0, (size_t)nsplit * m1 * m2 * sizeof(double2), &ws));
        const long long total = nsplit * ncg;
        const long long per_xcd = (total + 7) / 8;
        if (c->deep_loads && m2 <= 16) {
            // the same partials from deeper staging (ncg == 1): four splits per workgroup, ds
            // chunks per stage, at most 512 items per split and stage
            const int ds = THIN_TI * 64 / (GKC * (m1 + m2));
            const long long wgs = (nsplit + 3) / 4;
            const long long pxd = (wgs + 7) / 8;
            const size_t lds = (size_t)4 * ds * (m1 + m2) * GPAD * sizeof(double);
            hipLaunchKernelGGL(k_gram_thin_deep, dim3((unsigned)(8 * pxd)), dim3(256), lds, c->stream, K, m1, m2,
                               A, lda, B, ldb, kper, ds, nsplit, wgs, pxd, (double2*)ws);
        } else {
            hipLaunchKernelGGL(k_gram_thin, dim3((unsigned)(8 * per_xcd)), dim3(256), 0, c->stream, K, m1, m2, A,
                               lda, B, ldb, kper, ncg, total, per_xcd, (double2*)ws);
        }
        BDG_HIP(c, hipGetLastError());
        return gram_reduce(c, m1, m2, nsplit, ws, alpha, C, ldc, hermitian ? 1 : 0);
    }
    const bool t80 = 25 * 264 * tiles(80) < 16 * 204 * tiles(64);
    const int edge = t80 ? 80 : GT;
    const int tm = (m1 + edge - 1) / edge, tn = (m2 + edge - 1) / edge;
    const int ntiles = hermitian ? tn * (tn + 1) / 2 : tm * tn;
    long long nsplit = 1;
    // resident workgroups per CU: k_gram three (three waves per SIMD), k_gram80 one
    const long long kper = gram_rows_per_split(K, ntiles, (t80 ? 1LL : 3LL) * c->ncu, &nsplit, max_split);
    void* ws = nullptr;
    BDG_TRY(ctx_scratch(c, 0, (size_t)nsplit * m1 * m2 * sizeof(double2), &ws));
    // A == B (same segments, same stride): the diagonal tiles need one panel
    bool same = hermitian && na == nbs && lda == ldb;
    for (int i = 0; same && i < na; ++i) same = sa[i].p == sb[i].p && sa[i].ncols == sb[i].ncols;
    const long long total = nsplit * ntiles;
    const long long per_xcd = (total + 7) / 8;
    const int h = hermitian ? 1 : 0, sm = same ? 1 : 0;
    if (t80)
        hipLaunchKernelGGL(k_gram80, dim3((unsigned)(8 * per_xcd)), dim3(640), 0, c->stream, K, m1, m2, A, lda, B,
                           ldb, kper, tn, h, sm, ntiles, total, per_xcd, (double2*)ws);
    else
        hipLaunchKernelGGL(k_gram, dim3((unsigned)(8 * per_xcd)), dim3(256), 0, c->stream, K, m1, m2, A, lda, B,
                           ldb, kper, tn, h, sm, ntiles, total, per_xcd, (double2*)ws);
    BDG_HIP(c, hipGetLastError());
    return gram_reduce(c, m1, m2, nsplit, ws, alpha, C, ldc, h);
}

template <>
bdg_status gram<double2, double2>(bdg_ctx* c, long long K, int m1, int m2, const double2* A, long long lda,
                                  const double2* B, long long ldb, double alpha, double2* C, int ldc,
                                  int hermitian) {
    Seg a{A, m1}, b{B, m2};
    return gram_seg(c, K, &a, 1, lda, &b, 1, ldb, alpha, C, ldc, hermitian);
}

bdg_status update(bdg_ctx* c, long long K, const Seg* segs, int nseg, long long lds, const double2* Cm, int ldcm,
                  int nb, double beta, double2* Y, long long ldy) {
    return update_add(c, K, segs, nseg, lds, Cm, ldcm, nb, beta, Y, ldy, Y, ldy);
}

bdg_status update_add(bdg_ctx* c, long long K, const Seg* segs, int nseg, long long lds, const double2* Cm,
                      int ldcm, int nb, double beta, const double2* Z, long long ldz, double2* Y, long long ldy) {
    if (nb <= 0 || K <= 0) return BDG_OK;
    SegList sl;
    int m = 0;
    if (!make_seglist(segs, nseg, &sl, &m)) return ctx_fail(c, BDG_EINVAL, "update: 1..4 segments");
    if (c->deep_loads && m <= 8 && nb <= 16) {
        // the same bits from a row loop per wave (see k_update_thin)
        const long long nrb = (K + 15) / 16;
        const long long wg = std::max<long long>(1, std::min<long long>((nrb + 4 * UPD_UB - 1) / (4 * UPD_UB),
                                                                        4LL * c->ncu));
        hipLaunchKernelGGL(k_update_thin, dim3((unsigned)wg), dim3(256), 0, c->stream, K, sl, lds, m, Cm, ldcm, nb,
                           beta, Z, ldz, Y, ldy);
        return hip_check(c, hipGetLastError(), "k_update_thin");
    }
    const int cb = std::min(5, (nb + 15) / 16);
    const int ctiles = (nb + 16 * cb - 1) / (16 * cb);
    // 16 rows per wave (RA = 1): 10 accumulator tiles per wave leave room for two waves per
    // SIMD, measured 25 % faster on the 3-D solve than 32 rows per wave
    constexpr int RA = 1;
    dim3 grid((unsigned)((K + 64 * RA - 1) / (64 * RA)), (unsigned)ctiles);
    // one chunk of S and a Z term over at most 48 columns: Z loaded first (k_update's ZPRE;
    // measured 7 % faster on 2 into 40 columns, and twice as slow at 80 columns, where the
    // prefetched Z no longer fits three waves)
    const bool zpre = c->deep_loads && m <= 8 && beta != 0.0;
#define BDG_UPD(CBV) \
    hipLaunchKernelGGL((k_update<CBV, RA, false>), grid, dim3(256), 0, c->stream, K, sl, lds, m, Cm, ldcm, nb, beta, Z, ldz, Y, ldy, \
                       0, (double2*)nullptr, 0LL)
#define BDG_UPDZ(CBV) \
    if (zpre) \
        hipLaunchKernelGGL((k_update<CBV, RA, false, false, true>), grid, dim3(256), 0, c->stream, K, sl, lds, m, Cm, \
                           ldcm, nb, beta, Z, ldz, Y, ldy, 0, (double2*)nullptr, 0LL); \
    else \
        BDG_UPD(CBV)
    switch (cb) {
        case 1: BDG_UPDZ(1); break;
        case 2: BDG_UPDZ(2); break;
        case 3: BDG_UPDZ(3); break;
        case 4: BDG_UPD(4); break;
        default: BDG_UPD(5); break;
    }
#undef BDG_UPDZ
#undef BDG_UPD
    return hip_check(c, hipGetLastError(), "k_update");
}

bdg_status gram_seg_pair(bdg_ctx* c, long long K, const Seg* sa, int na, long long lda, const Seg* sb, int nbs,
                         long long ldb, double alpha, double2* C, int ldc, int hermitian) {
    SegList A, B;
    int m1 = 0, m2 = 0;
    if (!make_seglist(sa, na, &A, &m1) || !make_seglist(sb, nbs, &B, &m2))
        return ctx_fail(c, BDG_EINVAL, "gram: 1..4 segments");
    if (m1 <= 0 || m2 <= 0) return BDG_OK;
    if (hermitian && m1 != m2) return ctx_fail(c, BDG_EINVAL, "gram: symmetric form needs m1 == m2");
    const long long r1 = 2LL * m1, r2 = 2LL * m2;
    const long long max_split =
        c->arena.base ? std::max<long long>(1, (long long)(c->arena.gram_bytes / ((size_t)r1 * r2 * sizeof(double))))
                      : 0;
    bool same = hermitian && na == nbs && lda == ldb;
    for (int i = 0; same && i < na; ++i) same = sa[i].p == sb[i].p && sa[i].ncols == sb[i].ncols;
    const int nb1 = (m1 + 15) / 16, nb2 = (m2 + 15) / 16;
    const bool wide = c->gram_wide && m1 <= WGM && m2 <= WGM &&
                      (hermitian ? m1 > GT : (m1 > 16 && nb1 * nb2 <= 8 * WB && nb1 * nb2 > 4));
    const int t1 = (m1 + 7) / 8, t2 = (m2 + 7) / 8;
    const bool w8 = wide && c->gram_w8 && (hermitian ? t1 * (t1 + 1) / 2 : t1 * t2) <= 16 * W8T;
    if (wide) {
        // one workgroup per split covers the whole matrix: about two workgroups per CU
        long long nsplit = 1;
        const long long kper = gram_rows_per_split(K, 1, 2LL * c->ncu, &nsplit, max_split);
        void* ws = nullptr;
        BDG_TRY(ctx_scratch(c, 0, (size_t)nsplit * r1 * r2 * sizeof(double), &ws));
        // the same tiles and summation order either way: 2 loads straight to LDS, 1 stages
        // through registers
        if (w8 && c->gram_w8 == 2)
            hipLaunchKernelGGL(k_gram_pair_w8d, dim3((unsigned)nsplit), dim3(1024), 0, c->stream, K, m1, m2,
                               hermitian ? 1 : 0, A, lda, B, ldb, kper, same ? 1 : 0, (double*)ws);
        else if (w8)
            hipLaunchKernelGGL(k_gram_pair_w8, dim3((unsigned)nsplit), dim3(1024), 0, c->stream, K, m1, m2,
                               hermitian ? 1 : 0, A, lda, B, ldb, kper, same ? 1 : 0, (double*)ws);
        else
            hipLaunchKernelGGL(k_gram_pair_wide, dim3((unsigned)nsplit), dim3(512), 0, c->stream, K, m1, m2,
                               hermitian ? 1 : 0, A, lda, B, ldb, kper, same ? 1 : 0, (double*)ws);
        BDG_HIP(c, hipGetLastError());
        return gram_reduce_real(c, (int)r1, (int)r2, nsplit, ws, alpha, C, ldc, hermitian ? 1 : 0);
    }
    const int tm = (m1 + GT - 1) / GT, tn = (m2 + GT - 1) / GT;
    const int ntiles = hermitian ? tn * (tn + 1) / 2 : tm * tn;
    long long nsplit = 1;
    const long long kper = gram_rows_per_split(K, ntiles, 3LL * c->ncu, &nsplit, max_split);
    void* ws = nullptr;
    BDG_TRY(ctx_scratch(c, 0, (size_t)nsplit * r1 * r2 * sizeof(double), &ws));
    const long long total = nsplit * ntiles;
    const long long per_xcd = (total + 7) / 8;
    const int h = hermitian ? 1 : 0, sm = same ? 1 : 0;
    hipLaunchKernelGGL(k_gram_pair, dim3((unsigned)(8 * per_xcd)), dim3(256), 0, c->stream, K, m1, m2, A, lda, B, ldb,
                       kper, tn, h, sm, ntiles, total, per_xcd, (double*)ws);
    BDG_HIP(c, hipGetLastError());
    return gram_reduce_real(c, (int)r1, (int)r2, nsplit, ws, alpha, C, ldc, h);
}

bdg_status update_pair(bdg_ctx* c, long long K, const Seg* segs, int nseg, long long lds, const double2* Cr, int ldcr,
                       int r0, int nbr, double beta, const double2* Z, long long ldz, double2* Y, long long ldy) {
    if (nbr <= 0 || K <= 0) return BDG_OK;
    if (nbr & 1) return ctx_fail(c, BDG_EINVAL, "update_pair: odd real column count");
    SegList sl;
    int mp = 0;
    if (!make_seglist(segs, nseg, &sl, &mp)) return ctx_fail(c, BDG_EINVAL, "update: 1..4 segments");
    const int nbp = nbr / 2;
    void* ws = nullptr;
    BDG_TRY(ctx_scratch(c, 7, (size_t)2 * mp * nbp * sizeof(double2), &ws));
    double2* Cp = (double2*)ws;
    hipLaunchKernelGGL(k_pack_pair_coef, dim3((unsigned)((mp + 127) / 128), (unsigned)nbp), dim3(128), 0, c->stream,
                       mp, nbp, Cr, ldcr, r0, Cp);
    BDG_HIP(c, hipGetLastError());
    const int cb = std::min(5, (nbp + 15) / 16);
    const int ctiles = (nbp + 16 * cb - 1) / (16 * cb);
    constexpr int RA = 1;
    dim3 grid((unsigned)((K + 64 * RA - 1) / (64 * RA)), (unsigned)ctiles);
#define BDG_UPDP(CBV) \
    hipLaunchKernelGGL((k_update<CBV, RA, true>), grid, dim3(256), 0, c->stream, K, sl, lds, mp, (const double2*)Cp, \
                       2 * mp, nbp, beta, Z, ldz, Y, ldy, 0, (double2*)nullptr, 0LL)
    switch (cb) {
        case 1: BDG_UPDP(1); break;
        case 2: BDG_UPDP(2); break;
        case 3: BDG_UPDP(3); break;
        case 4: BDG_UPDP(4); break;
        default: BDG_UPDP(5); break;
    }
#undef BDG_UPDP
    return hip_check(c, hipGetLastError(), "k_update_pair");
}

bdg_status update_pair_fused(bdg_ctx* c, long long K, const Seg* segs, int nseg, long long lds, const double2* Cr,
                             int ldcr, int nbr, int mF, double2* Yp, long long ldyp, double2* Yf, long long ldyf) {
    if (nbr <= 0 || K <= 0) return BDG_OK;
    if ((nbr & 1) || nbr > 96 || mF % 8 != 0) return ctx_fail(c, BDG_EINVAL, "update_pair_fused: unsupported shape");
    SegList sl;
    int mp = 0;
    if (!make_seglist(segs, nseg, &sl, &mp)) return ctx_fail(c, BDG_EINVAL, "update: 1..4 segments");
    if (mF < 0 || mF > mp) return ctx_fail(c, BDG_EINVAL, "update_pair_fused: F columns out of range");
    const int nbp = nbr / 2;
    void* ws = nullptr;
    BDG_TRY(ctx_scratch(c, 7, (size_t)2 * mp * nbp * sizeof(double2), &ws));
    double2* Cp = (double2*)ws;
    hipLaunchKernelGGL(k_pack_pair_coef, dim3((unsigned)((mp + 127) / 128), (unsigned)nbp), dim3(128), 0, c->stream,
                       mp, nbp, Cr, ldcr, 0, Cp);
    BDG_HIP(c, hipGetLastError());
    // one column tile (CB <= 3 covers nbp <= 48): a workgroup owns all output columns of its rows
    const int cb = (nbp + 15) / 16;
    constexpr int RA = 1;
    dim3 grid((unsigned)((K + 64 * RA - 1) / (64 * RA)), 1);
#define BDG_UPDF(CBV)                                                                                              \
    hipLaunchKernelGGL((k_update<CBV, RA, true, true>), grid, dim3(256), 0, c->stream, K, sl, lds, mp,             \
                       (const double2*)Cp, 2 * mp, nbp, 0.0, (const double2*)nullptr, 0LL, Yf, ldyf, mF, Yp, ldyp)
    switch (cb) {
        case 1: BDG_UPDF(1); break;
        case 2: BDG_UPDF(2); break;
        default: BDG_UPDF(3); break;
    }
#undef BDG_UPDF
    return hip_check(c, hipGetLastError(), "k_update_pair_fused");
}

bdg_status colnorm2_pair(bdg_ctx* c, long long K, int ncols, const double2* X, long long ldx, double* out_dev) {
    if (ncols <= 0) return BDG_OK;
    int nchunk = (int)std::min<long long>(256, (K + 8191) / 8192);
    if (nchunk < 1) nchunk = 1;
    const long long kper = (K + nchunk - 1) / nchunk;
    void* ws = nullptr;
    BDG_TRY(ctx_scratch(c, 2, (size_t)2 * ncols * nchunk * sizeof(double), &ws));
    hipLaunchKernelGGL(k_colnorm2_pair_part, dim3((unsigned)nchunk, (unsigned)ncols), dim3(RB), 0, c->stream, K, X,
                       ldx, kper, (double*)ws);
    BDG_HIP(c, hipGetLastError());
    hipLaunchKernelGGL(k_colnorm2_final, dim3((unsigned)((2 * ncols + 127) / 128)), dim3(128), 0, c->stream,
                       2 * ncols, nchunk, (const double*)ws, out_dev);
    return hip_check(c, hipGetLastError(), "k_colnorm2_pair");
}

bdg_status resnorm2_pair(bdg_ctx* c, long long K, int ncols, const double2* HF, const double2* G, const double2* HG,
                         const double2* F, long long ld, const double* om_dev, double* out_dev) {
    if (ncols <= 0) return BDG_OK;
    int nchunk = (int)std::min<long long>(128, (K + 8191) / 8192);
    if (nchunk < 1) nchunk = 1;
    const long long kper = (K + nchunk - 1) / nchunk;
    void* ws = nullptr;
    BDG_TRY(ctx_scratch(c, 2, (size_t)8 * ncols * nchunk * sizeof(double), &ws));
    hipLaunchKernelGGL(k_resnorm2_pair_part, dim3((unsigned)nchunk, (unsigned)ncols), dim3(RB), 0, c->stream, K, HF,
                       G, HG, F, ld, om_dev, kper, (double*)ws);
    BDG_HIP(c, hipGetLastError());
    hipLaunchKernelGGL(k_colnorm2_final, dim3((unsigned)((8 * ncols + 127) / 128)), dim3(128), 0, c->stream,
                       8 * ncols, nchunk, (const double*)ws, out_dev);
    return hip_check(c, hipGetLastError(), "k_resnorm2_pair");
}

bdg_status dot_pair(bdg_ctx* c, long long K, int ncols, const double2* F, const double2* G, long long ld,
                    double* out_dev) {
    if (ncols <= 0) return BDG_OK;
    int nchunk = (int)std::min<long long>(256, (K + 8191) / 8192);
    if (nchunk < 1) nchunk = 1;
    const long long kper = (K + nchunk - 1) / nchunk;
    void* ws = nullptr;
    BDG_TRY(ctx_scratch(c, 2, (size_t)2 * ncols * nchunk * sizeof(double), &ws));
    hipLaunchKernelGGL(k_dot_pair_part, dim3((unsigned)nchunk, (unsigned)ncols), dim3(RB), 0, c->stream, K, F, G, ld,
                       kper, (double*)ws);
    BDG_HIP(c, hipGetLastError());
    hipLaunchKernelGGL(k_colnorm2_final, dim3((unsigned)((2 * ncols + 127) / 128)), dim3(128), 0, c->stream,
                       2 * ncols, nchunk, (const double*)ws, out_dev);
    return hip_check(c, hipGetLastError(), "k_dot_pair");
}

bdg_status colnorm2(bdg_ctx* c, long long K, int ncols, const double2* X, long long ldx, double* out_dev) {
    if (ncols <= 0) return BDG_OK;
    int nchunk = (int)std::min<long long>(256, (K + 8191) / 8192);
    if (nchunk < 1) nchunk = 1;
    const long long kper = (K + nchunk - 1) / nchunk;
    void* ws = nullptr;
    BDG_TRY(ctx_scratch(c, 2, (size_t)ncols * nchunk * sizeof(double), &ws));
    hipLaunchKernelGGL(k_colnorm2_part, dim3((unsigned)nchunk, (unsigned)ncols), dim3(RB), 0, c->stream, K, X, ldx,
                       kper, (double*)ws);
    BDG_HIP(c, hipGetLastError());
    hipLaunchKernelGGL(k_colnorm2_final, dim3((unsigned)((ncols + 127) / 128)), dim3(128), 0, c->stream, ncols,
                       nchunk, (const double*)ws, out_dev);
    return hip_check(c, hipGetLastError(), "k_colnorm2");
}
