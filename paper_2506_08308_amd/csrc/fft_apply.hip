// Matrix-free BdG operator on gfx950: LDS-staged Stockham FFTs along each grid axis, the
// kinetic multiplier |k|^2/2 (Section 3.1, eq. laplace_approx), and the pointwise 3x3
// coupling of H_+ = A + B, H_- = A - B in physical space (eqs. def_bfA, def_bfB; the
// matrix-vector product of Section 3.2).
//
// One pass over HBM per axis and direction; the last axis fuses forward FFT, multiplier
// and inverse FFT in LDS/registers, and the final x pass fuses the inverse FFT with the
// coupling:  3-D: x-fwd | y-fwd | z-fwd*k2*z-inv | y-inv | x-inv+couple,
//            2-D: x-fwd | y-fwd*k2*y-inv | x-inv+couple,   1-D: one fused pass.
// The output block Y doubles as the spectral workspace, so the operator needs no scratch.
//
// FFT engine: each thread owns four elements x[i + r N/4] (r = 0..3) of one line; radix-4
// Stockham passes (and one radix-2 pass when log2 N is odd) exchange through LDS.  After
// the last forward pass the thread again owns X[i + r N/4] in natural order, which is
// exactly the input pattern of the inverse transform, so the fused multiplier costs no
// extra exchange.  Twiddles exp(-2 pi i m/N) come from host-built float64 tables.
#include "common.h"

#include <type_traits>

namespace {

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

template <typename V> struct FieldAddr {
    V* lo;              // fields 0..2 of each vector (f or u half)
    V* hi;              // fields 3..5 (g or v half)
    long long vstride;  // distance between vectors
    int fpv;            // fields per vector: 6 (both halves) or 3 (one half, at lo)
    long long npts;
    __device__ __forceinline__ V* field(long long f) const {
        long long vec = f / fpv;
        int c = (int)(f % fpv);
        V* base = (c < 3) ? lo : hi;
        return base + vec * vstride + (long long)(c % 3) * npts;
    }
};

template <typename V, bool INV> __device__ __forceinline__ V mul_tw(V a, V w) {
    return INV ? cmulc(a, w) : cmul(a, w);
}

// 4-point DFT in registers (forward: W_4 = -i; inverse: +i), natural order output.
template <typename V, bool INV> __device__ __forceinline__ void dft4(V v[4]) {
    V t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    V t2 = cadd(v[1], v[3]), d = csub(v[1], v[3]);
    V t3 = INV ? cmk<V>(-d.y, d.x) : cmk<V>(d.y, -d.x);
    v[0] = cadd(t0, t2);
    v[1] = cadd(t1, t3);
    v[2] = csub(t0, t2);
    v[3] = csub(t1, t3);
}

// Workgroup barrier that orders LDS accesses only: the wave waits for its own LDS operations
// (lgkmcnt 0) and meets the others; global loads still in flight stay in flight (a full
// __syncthreads waits for them too), which lets a workgroup prefetch its next input while it
// transforms the current one in LDS.
__device__ __forceinline__ void lds_barrier() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0xC07F);      // vmcnt, expcnt at their maxima, lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Ordering of the LDS exchanges of line_fft.  SYNC_BLOCK: __syncthreads.  SYNC_WAVE: every
// line lies within one wave (its N/4 threads are consecutive and N/4 <= 64); a wave's LDS
// operations are executed in issue order, so waiting for its own (lgkmcnt 0) suffices and
// no workgroup barrier is taken.
enum { SYNC_BLOCK = 0, SYNC_WAVE = 2 };
template <int SYNC> __device__ __forceinline__ void fft_sync() {
    if constexpr (SYNC == SYNC_BLOCK) {
        __syncthreads();
    } else {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0xC07F);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
}
// wave-local exchanges for contiguous lines of up to 256 points
template <int N> constexpr int contiguous_sync() { return N / 4 <= 64 ? SYNC_WAVE : SYNC_BLOCK; }

// In-line FFT of length N.  On entry v[r] = x[i + r N/4]; on exit v[r] = X[i + r N/4].
// lds(e) = lds[lb + e * ls] is this line's exchange buffer.  With SYNC_BLOCK every thread of
// the block must call it (barriers), including threads whose line is out of range.  tw holds
// the N TWS twiddles of a transform TWS times longer (read at stride TWS).
template <typename V, int N, bool INV, int SYNC = SYNC_BLOCK, int TWS = 1>
__device__ __forceinline__ void line_fft(V v[4], int i, V* __restrict__ lds, int lb, int ls,
                                         const V* __restrict__ tw) {
    constexpr int Q = N / 4;
    constexpr int LG = ilog2c(N);
    constexpr int NP4 = LG / 2;
    constexpr bool R2 = (LG & 1) != 0;
#pragma unroll
    for (int s = 0; s < NP4; ++s) {
        const int p = 1 << (2 * s);
        const int k = i & (p - 1);
        if (s > 0) {
            const int step = N / (4 * p);
#pragma unroll
            for (int r = 1; r < 4; ++r) v[r] = mul_tw<V, INV>(v[r], tw[r * k * step * TWS]);
        }
        dft4<V, INV>(v);
        const bool last = (s == NP4 - 1) && !R2;
        if (!last) {
            const int j = ((i - k) << 2) + k;
            fft_sync<SYNC>();
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[lb + (j + r * p) * ls] = v[r];
            fft_sync<SYNC>();
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = lds[lb + (i + r * Q) * ls];
        }
    }
    if (R2) {
        // final radix-2 pass (span N/2): butterflies i and i + N/4
        v[2] = mul_tw<V, INV>(v[2], tw[i * TWS]);
        v[3] = mul_tw<V, INV>(v[3], tw[(i + Q) * TWS]);
        V a0 = cadd(v[0], v[2]), a2 = csub(v[0], v[2]);
        V a1 = cadd(v[1], v[3]), a3 = csub(v[1], v[3]);
        v[0] = a0; v[1] = a1; v[2] = a2; v[3] = a3;
    }
}

struct MultSpec {
    const double* s[3];   // |mu|^2/2 tables per axis (FFT order)
    double scale;         // 1 / npts
    double shift;         // preconditioner shift
    int precond;          // 0: kinetic, 1: (k2 + shift)^-1
};

template <typename R>
__device__ __forceinline__ R multiplier(const MultSpec& m, int mx, int my, int mz) {
    double k2 = m.s[0][mx] + m.s[1][my] + m.s[2][mz];
    double v = m.precond ? m.scale / (k2 + m.shift) : m.scale * k2;
    return (R)v;
}

// ----------------------------------------------------------------------------------------
// x pass: contiguous lines.  MODE 0: plain FFT (direction INV); MODE 1: fused forward,
// multiplier, inverse (the x axis is the only axis: 1-D preconditioner / plain fused use).
// ----------------------------------------------------------------------------------------
// wgt (optional, npts real): pointwise factor applied before a forward transform and after
// an inverse one (the D of a symmetric preconditioner D T D).
template <typename V, int N, bool INV, int MODE, typename VO = V>
__global__ void __launch_bounds__(256) k_xpass(FieldAddr<const V> in, FieldAddr<VO> out,
                                               long long nfields, long long lines_per_field,
                                               const V* __restrict__ tw, MultSpec ms, int ny,
                                               const decltype(V::x)* __restrict__ wgt) {
    using R = decltype(V::x);
    using RO = decltype(VO::x);
    constexpr int Q = N / 4;
    constexpr int LPW = (1024 / N) > 0 ? (1024 / N) : 1;
    __shared__ V lds[LPW * N];
    const int t = threadIdx.x;
    const int ln = t / Q, i = t % Q;
    const long long gl = (long long)blockIdx.x * LPW + ln;
    const bool valid = gl < nfields * lines_per_field;
    const long long f = valid ? gl / lines_per_field : 0;
    const long long l = valid ? gl % lines_per_field : 0;
    const V* src = in.field(f) + l * N;
    VO* dst = out.field(f) + l * N;
    V v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = valid ? src[i + r * Q] : cmk<V>(0, 0);
    R wv[4] = {1, 1, 1, 1};
    if (wgt != nullptr && valid) {
#pragma unroll
        for (int r = 0; r < 4; ++r) wv[r] = wgt[l * N + i + r * Q];
    }
    const bool wfwd = wgt != nullptr && (MODE == 1 || !INV);
    const bool winv = wgt != nullptr && (MODE == 1 || INV);
    if (wfwd) {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = cscale(v[r], wv[r]);
    }
    constexpr int SY = contiguous_sync<N>();
    if (MODE == 0) {
        line_fft<V, N, INV, SY>(v, i, lds, ln * N, 1, tw);
    } else {
        line_fft<V, N, false, SY>(v, i, lds, ln * N, 1, tw);
        const int my = (int)(l % ny), mz = (int)(l / ny);
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = cscale(v[r], multiplier<R>(ms, i + r * Q, my, mz));
        line_fft<V, N, true, SY>(v, i, lds, ln * N, 1, tw);
    }
    if (winv) {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = cscale(v[r], wv[r]);
    }
    if (valid) {
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[i + r * Q] = cmk<VO>((RO)v[r].x, (RO)v[r].y);
    }
}

// ----------------------------------------------------------------------------------------
// Strided pass along axis y (axis=1) or z (axis=2), tiles of TX adjacent x columns.
// MODE 0: plain FFT; MODE 1: fused forward * multiplier * inverse (last axis).
// ----------------------------------------------------------------------------------------
// TX adjacent x columns per tile (16: 32 complex64 columns measured slower on the fused z pass)
template <typename V, int N> struct StridedCfg {
    static constexpr int TXA = 2048 / N;
    static constexpr int TX = TXA < 16 ? (TXA < 1 ? 1 : TXA) : 16;
    static constexpr int THREADS = TX * (N / 4);
};

template <typename V, int N, bool INV, int MODE>
__global__ void __launch_bounds__(512) k_strided(FieldAddr<V> io, long long nfields, int nx, int ny,
                                                 int axis, int tx, const V* __restrict__ tw, MultSpec ms) {
    using R = decltype(V::x);
    constexpr int Q = N / 4;
    constexpr int TXM = StridedCfg<V, N>::TX;
    __shared__ V lds[TXM * N];
    const int t = threadIdx.x;               // blockDim.x == tx * N/4 (tx <= TXM)
    const int c = t % tx, i = t / tx;
    const int tiles = nx / tx;
    // block -> (field, outer, tile)
    const long long b = blockIdx.x;
    const int tile = (int)(b % tiles);
    const long long rest = b / tiles;
    const int outer_n = (axis == 1) ? (int)(io.npts / ((long long)nx * ny)) : ny;   // z planes or y rows
    const int outer = (int)(rest % outer_n);
    const long long f = rest / outer_n;
    const long long stride = (axis == 1) ? nx : (long long)nx * ny;
    const long long outer_stride = (axis == 1) ? (long long)nx * ny : nx;
    V* base = io.field(f) + outer * outer_stride + tile * tx + c;
    V v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = base[(i + r * Q) * stride];
    if (MODE == 0) {
        line_fft<V, N, INV>(v, i, lds, c, tx, tw);
    } else {
        line_fft<V, N, false>(v, i, lds, c, tx, tw);
        const int mx = tile * tx + c;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = i + r * Q;
            const R m = (axis == 2) ? multiplier<R>(ms, mx, outer, e) : multiplier<R>(ms, mx, e, 0);
            v[r] = cscale(v[r], m);
        }
        line_fft<V, N, true>(v, i, lds, c, tx, tw);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) base[(i + r * Q) * stride] = v[r];
}

// ----------------------------------------------------------------------------------------
// Final x pass: inverse FFT of the six kinetic fields of QL lines of one vector, then the
// pointwise coupling with the input fields.  FULL: the lines are loaded from X and
// transformed forward, multiplied and inverted here (1-D grids).
// FORM 1 (f, g):  y_f = T g + H_- g,  y_g = T f + H_+ f   (transpose swaps H_+ and H_-)
// FORM 2 / 3 (u, v), complex ground state (float64 only; 21 coefficient fields):
//                 y_u = T u + A u + B v,  y_v = -+(T v + conj(B) u + conj(A) v)  (3: the K form)
// FORM 0 (u, v):  y_u = T u + A u + B v,  y_v = -(T v + B u + A v)  with A = (H_+ + H_-)/2,
//                 B = (H_+ - H_-)/2 (transpose flips the sign of the B terms)
// ----------------------------------------------------------------------------------------
template <int N> struct CoupleCfg {
    static constexpr int QL = (256 / N) > 0 ? (256 / N) : 1;
    // fields per thread: a 1024-point line needs 256 threads per field, so six fields take
    // two rounds of 768 threads (the workgroup limit is 1024)
    static constexpr int FH = (6 * QL * (N / 4) > 1024) ? 2 : 1;
    static constexpr int THREADS = 6 * QL * (N / 4) / FH;
};

// NVB vectors per workgroup, one after the other through the same LDS: the coefficient
// fields of the workgroup's points are read once for all of them.
template <typename V, int N, int FORM, int TRANS, bool FULL, int NVB>
__global__ void __launch_bounds__(1024) k_couple(FieldAddr<const V> xin, FieldAddr<V> yout,
                                                 long long lines_per_field, long long nlinegroups, long long nvec,
                                                 const V* __restrict__ tw, MultSpec ms, int ny,
                                                 const decltype(V::x)* __restrict__ coef) {
    using R = decltype(V::x);
    constexpr int Q = N / 4;
    constexpr int QL = CoupleCfg<N>::QL;
    constexpr int FH = CoupleCfg<N>::FH;
    constexpr int NT = CoupleCfg<N>::THREADS;
    constexpr int PPT = (QL * N + NT - 1) / NT;       // grid points per thread
    constexpr int NC = FORM >= 2 ? 21 : 12;          // coefficient fields
    // one line per thread group (FH = 1): contiguous lines, wave-local exchanges up to N = 256
    constexpr int SYC = FH == 1 ? contiguous_sync<N>() : SYNC_BLOCK;
    __shared__ V lds[6 * QL * N];
    const int t = threadIdx.x;
    const int fld0 = t / (QL * Q);            // fields fld0 + h * (6 / FH), h < FH
    const int q = (t / Q) % QL;
    const int i = t % Q;
    const long long b = blockIdx.x;
    const long long vg = b / nlinegroups;
    const long long l0 = (b % nlinegroups) * QL;
    const long long l = l0 + q;
    const bool valid = l < lines_per_field;
    const long long npts = xin.npts;
    // coefficients of this thread's grid points
    R cf[PPT][NC];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int pt = t + k * NT;
        const int qq = pt / N, e = pt % N;
        const bool ok = pt < QL * N && l0 + qq < lines_per_field;
        const long long p = (l0 + qq) * N + e;
#pragma unroll
        for (int s2 = 0; s2 < NC; ++s2) cf[k][s2] = ok ? coef[s2 * npts + p] : (R)0;
    }
    for (int vi = 0; vi < NVB; ++vi) {
        const long long vec = vg * NVB + vi;
        if (vec >= nvec) break;                      // uniform over the workgroup
        if (vi > 0) __syncthreads();                 // the previous vector's LDS reads are done
        V v[FH][4];
#pragma unroll
        for (int h = 0; h < FH; ++h) {
            const int fld = fld0 + h * (6 / FH);
            if (FULL) {
                const V* src = xin.field(vec * 6 + fld) + l * N;
#pragma unroll
                for (int r = 0; r < 4; ++r) v[h][r] = valid ? src[i + r * Q] : cmk<V>(0, 0);
                line_fft<V, N, false, SYC>(v[h], i, lds, (fld * QL + q) * N, 1, tw);
                const int my = (int)(l % ny), mz = (int)(l / ny);
#pragma unroll
                for (int r = 0; r < 4; ++r) v[h][r] = cscale(v[h][r], multiplier<R>(ms, i + r * Q, my, mz));
            } else {
                const V* src = yout.field(vec * 6 + fld) + l * N;
#pragma unroll
                for (int r = 0; r < 4; ++r) v[h][r] = valid ? src[i + r * Q] : cmk<V>(0, 0);
            }
            line_fft<V, N, true, SYC>(v[h], i, lds, (fld * QL + q) * N, 1, tw);
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < FH; ++h) {
            const int fld = fld0 + h * (6 / FH);
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[(fld * QL + q) * N + i + r * Q] = v[h][r];
        }
        __syncthreads();
        // coupling: one grid point per thread iteration
        const V* x0 = xin.field(vec * 6 + 0);
        const V* x3 = xin.field(vec * 6 + 3);
        V* y0 = yout.field(vec * 6 + 0);
        V* y3 = yout.field(vec * 6 + 3);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int pt = t + k * NT;
            if (pt >= QL * N) continue;
            const int qq = pt / N, e = pt % N;
            const long long ll = l0 + qq;
            if (ll >= lines_per_field) continue;
            const long long p = ll * N + e;
            const R* C = cf[k];
            V xa[3], xb[3], ta[3], tb[3];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                xa[cc] = x0[cc * npts + p];
                xb[cc] = x3[cc * npts + p];
                ta[cc] = lds[(cc * QL + qq) * N + e];
                tb[cc] = lds[((cc + 3) * QL + qq) * N + e];
            }
            V ya[3], yb[3];
            if constexpr (FORM >= 2) {
                // complex ground state: A Hermitian (real diagonal, upper 01, 02, 12), B symmetric
                const R* ad = C;
                const R* ao = C + 3;
                const R* bb = C + 9;
                auto aent = [&](int a, int c2) -> V {
                    if (a == c2) return cmk<V>(ad[a], 0);
                    const int lo = a < c2 ? a : c2, hi = a < c2 ? c2 : a;
                    const int e2 = lo == 0 ? hi - 1 : 2;                 // 01 -> 0, 02 -> 1, 12 -> 2
                    const V up = cmk<V>(ao[2 * e2], ao[2 * e2 + 1]);
                    return a < c2 ? up : cmk<V>(up.x, -up.y);
                };
                auto bent = [&](int a, int c2) -> V {
                    const int lo = a < c2 ? a : c2, hi = a < c2 ? c2 : a;
                    const int e2 = lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
                    return cmk<V>(bb[2 * e2], bb[2 * e2 + 1]);
                };
                const R sv = FORM == 2 ? (R)-1 : (R)1;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    V su = ta[a], sw = tb[a];
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc) {
                        const V A_ = aent(a, cc), B_ = bent(a, cc);
                        // u row: A u + B v;  v row: conj(B) u + conj(A) v
                        su = cadd(su, cadd(cmul(A_, xa[cc]), cmul(B_, xb[cc])));
                        sw = cadd(sw, cadd(cmul(cmk<V>(B_.x, -B_.y), xa[cc]), cmul(cmk<V>(A_.x, -A_.y), xb[cc])));
                    }
                    ya[a] = su;
                    yb[a] = cmk<V>(sv * sw.x, sv * sw.y);
                }
            } else {
                const R* P = C;
                const R* M = C + 6;
                // symmetric 3x3 from 6 entries (00, 01, 02, 11, 12, 22)
                auto sym = [](const R* S, int a, int c2) -> R {
                    const int lo = a < c2 ? a : c2, hi = a < c2 ? c2 : a;
                    const int idx = lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
                    return S[idx];
                };
                if (FORM == 1) {
                    const R* Pa = TRANS ? M : P;   // operator acting on f (output half 1)
                    const R* Pb = TRANS ? P : M;   // operator acting on g (output half 0)
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        V s0 = tb[a], s1 = ta[a];
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) {
                            const R mb = sym(Pb, a, cc), ma = sym(Pa, a, cc);
                            s0 = cmk<V>(s0.x + mb * xb[cc].x, s0.y + mb * xb[cc].y);
                            s1 = cmk<V>(s1.x + ma * xa[cc].x, s1.y + ma * xa[cc].y);
                        }
                        ya[a] = s0;
                        yb[a] = s1;
                    }
                } else {
                    const R sB = TRANS ? (R)-1 : (R)1;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        V su = ta[a], sv = tb[a];
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) {
                            const R pa = sym(P, a, cc), mm = sym(M, a, cc);
                            const R A_ = (R)0.5 * (pa + mm), B_ = (R)0.5 * (pa - mm) * sB;
                            su = cmk<V>(su.x + A_ * xa[cc].x + B_ * xb[cc].x, su.y + A_ * xa[cc].y + B_ * xb[cc].y);
                            sv = cmk<V>(sv.x + B_ * xa[cc].x + A_ * xb[cc].x, sv.y + B_ * xa[cc].y + A_ * xb[cc].y);
                        }
                        ya[a] = su;
                        yb[a] = cmk<V>(-sv.x, -sv.y);
                    }
                }
            }
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                y0[cc * npts + p] = ya[cc];
                y3[cc * npts + p] = yb[cc];
            }
        }
    }
}

// ----------------------------------------------------------------------------------------
// xy-plane passes (complex64, nx = ny = 128, 3-D): one workgroup holds a whole 128 x 128
// plane in LDS (row pitch 129 keeps the column accesses of the y transform free of bank
// conflicts), so the x and y transforms share one pass over HBM.  With the z pass between
// them the (f, g) operator takes three passes instead of five:
//   plane-fwd:  Y[sigma(s)] = F_xy X[s]  (sigma swaps the f and g halves, see below)
//   z pass:     Y <- F_z^-1 k2 F_z Y     (k_strided, MODE 1)
//   plane-inv:  Y[o] = F_xy^-1 Y[o] + sum_c C_o(a, c) X[h(o), c]
// Output field o (half 0: y_f = T g + H_- g, half 1: y_g = T f + H_+ f) needs the kinetic
// image of the field of the other half with the same component, so the forward pass stores
// it at o's position and the inverse pass reads and writes one position only.
// The kernels are persistent (one workgroup per CU: the plane takes 129 KiB of LDS) and keep
// the next plane's 16 loads per thread in flight while the current plane is transformed
// (LDS-only barriers in between).
// ----------------------------------------------------------------------------------------
constexpr int PLN = 128, PLP = 129;
constexpr size_t PLANE_LDS = (size_t)PLN * PLP * sizeof(float2);

// rows (MODE 0: x transform) or columns (MODE 1: y transform) of the LDS plane, 32 lines per
// round (a line on 32 consecutive lanes of one wave: wave-local exchanges), four rounds, one
// workgroup barrier at the end
template <bool INV, int MODE>
__device__ __forceinline__ void plane_lines(float2* pl, const float2* __restrict__ tw) {
    constexpr int Q = PLN / 4;
    const int t = threadIdx.x;
    const int ln = t / Q, i = t % Q;
#pragma unroll 1
    for (int rnd = 0; rnd < 4; ++rnd) {
        const int line = rnd * 32 + ln;
        const int lb = MODE == 0 ? line * PLP : line;
        const int ls = MODE == 0 ? 1 : PLP;
        float2 v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = pl[lb + (i + r * Q) * ls];
        line_fft<float2, PLN, INV, SYNC_WAVE>(v, i, pl, lb, ls, tw);
        fft_sync<SYNC_WAVE>();   // the exchange buffer of the line is the line itself
#pragma unroll
        for (int r = 0; r < 4; ++r) pl[lb + (i + r * Q) * ls] = v[r];
    }
    lds_barrier();
}

__device__ __forceinline__ void plane_load(float2 (&v)[16], const float2* __restrict__ src) {
    const int t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = src[t + 1024 * j];
}

__device__ __forceinline__ void plane_to_lds(float2* pl, const float2 (&v)[16]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int e = t + 1024 * j;
        pl[(e >> 7) * PLP + (e & 127)] = v[j];
    }
}

// forward: task w = (field f, plane z), f-major; Y[sigma(f)] plane z = F_xy X[f] plane z.
// PREC (the preconditioner's first pass): Y[f] plane z = F_xy (w X[f]) plane z with the
// pointwise weight w, no half swap (the transforms of the x and y passes it replaces)
template <bool PREC = false>
__global__ void __launch_bounds__(1024) k_plane_fwd(FieldAddr<const float2> in, FieldAddr<float2> out,
                                                   long long nfields, int nz, const float2* __restrict__ twx,
                                                   const float2* __restrict__ twy,
                                                   const float* __restrict__ wgt = nullptr) {
    extern __shared__ float2 pl[];
    const long long ntask = nfields * nz;
    long long w = blockIdx.x;
    if (w >= ntask) return;
    const int t = threadIdx.x;
    float2 v[16];
    plane_load(v, in.field(w / nz) + (w % nz) * (long long)(PLN * PLN));
    for (; w < ntask; w += gridDim.x) {
        if constexpr (PREC) {
            const float* wz = wgt + (w % nz) * (long long)(PLN * PLN);
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = cscale(v[j], wz[t + 1024 * j]);
        }
        plane_to_lds(pl, v);
        lds_barrier();
        const long long wn = w + gridDim.x;
        if (wn < ntask) plane_load(v, in.field(wn / nz) + (wn % nz) * (long long)(PLN * PLN));
        plane_lines<false, 0>(pl, twx);
        plane_lines<false, 1>(pl, twy);
        const long long f = w / nz;
        const long long vec = f / 6;
        const int s = (int)(f % 6);
        const int so = PREC ? s : (s < 3 ? s + 3 : s - 3);
        float2* dst = out.field(vec * 6 + so) + (w % nz) * (long long)(PLN * PLN);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int e = t + 1024 * j;
            dst[e] = pl[(e >> 7) * PLP + (e & 127)];
        }
        lds_barrier();       // the plane is read out of LDS before the next one is staged
    }
}

// the preconditioner's last pass: task w = (field f, plane z); Y64[f] plane z =
// w F_xy^-1 X[f] plane z (y then x inverse, the pointwise weight, widened to float64), the
// transforms of the y and x inverse passes it replaces.  Persistent, the next plane's loads
// in flight as in k_plane_fwd.
__global__ void __launch_bounds__(1024) k_plane_inv_w(FieldAddr<const float2> in, FieldAddr<double2> out,
                                                     long long nfields, int nz, const float2* __restrict__ twx,
                                                     const float2* __restrict__ twy,
                                                     const float* __restrict__ wgt) {
    extern __shared__ float2 pl[];
    const long long ntask = nfields * nz;
    long long w = blockIdx.x;
    if (w >= ntask) return;
    const int t = threadIdx.x;
    float2 v[16];
    plane_load(v, in.field(w / nz) + (w % nz) * (long long)(PLN * PLN));
    for (; w < ntask; w += gridDim.x) {
        plane_to_lds(pl, v);
        lds_barrier();
        const long long wn = w + gridDim.x;
        if (wn < ntask) plane_load(v, in.field(wn / nz) + (wn % nz) * (long long)(PLN * PLN));
        plane_lines<true, 1>(pl, twy);
        plane_lines<true, 0>(pl, twx);
        const long long poff = (w % nz) * (long long)(PLN * PLN);
        double2* dst = out.field(w / nz) + poff;
        const float* wz = wgt + poff;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int e = t + 1024 * j;
            const float2 y = cscale(pl[(e >> 7) * PLP + (e & 127)], wz[e]);
            dst[e] = cmk<double2>(y.x, y.y);
        }
        lds_barrier();       // the plane is read out of LDS before the next one is staged
    }
}

// inverse + coupling.  Task (g, a): group g = (plane z, vector, half h), h fastest and z
// slowest, component a.  Workgroup b runs on XCD b % 8; each XCD takes a contiguous run of
// groups and deals their tasks to its workgroups in order, so the three components of a
// group (which read the same three input planes and coefficient rows) and the groups of one
// plane (which read the same coefficient planes) run at about the same time on one XCD and
// share its L2.  The result goes to yout, which is yio itself (float2) or the float64
// images (double2: the float32 result widened, in place of a separate conversion pass).
template <int TRANS, typename VO = float2>
__global__ void __launch_bounds__(1024) k_plane_inv_couple(FieldAddr<const float2> xin, FieldAddr<float2> yio,
                                                           FieldAddr<VO> yout, long long nvec, int nz,
                                                           const float2* __restrict__ twx,
                                                           const float2* __restrict__ twy,
                                                           const float* __restrict__ coef) {
    extern __shared__ float2 pl[];
    const long long ngroups = nvec * 2 * nz;
    const int nxcd = 8, xcd = blockIdx.x % nxcd;
    const int nslot = (gridDim.x - xcd + nxcd - 1) / nxcd;   // workgroups on this XCD
    const int slot = blockIdx.x / nxcd;
    const long long g0 = ngroups * xcd / nxcd, g1 = ngroups * (xcd + 1) / nxcd;
    const long long ntask = 3 * (g1 - g0);
    long long u = slot;
    if (u >= ntask) return;
    const int t = threadIdx.x;
    const long long npts = xin.npts;
    struct Task {
        int a, h;
        long long z, vec;
    };
    auto task_of = [&](long long uu) {
        const long long g = g0 + uu / 3;
        Task k;
        k.a = (int)(uu % 3);
        k.h = (int)(g % 2);
        k.vec = (g / 2) % nvec;
        k.z = g / (2 * nvec);
        return k;
    };
    auto plane_of = [&](const Task& k) -> float2* {
        return yio.field(k.vec * 6 + 3 * k.h + k.a) + k.z * (long long)(PLN * PLN);
    };
    auto sidx = [](int r, int c2) {
        const int lo = r < c2 ? r : c2, hi = r < c2 ? c2 : r;
        return lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
    };
    float2 v[16];
    plane_load(v, plane_of(task_of(u)));
    for (; u < ntask; u += nslot) {
        plane_to_lds(pl, v);
        lds_barrier();
        if (u + nslot < ntask) plane_load(v, plane_of(task_of(u + nslot)));
        plane_lines<true, 1>(pl, twy);
        plane_lines<true, 0>(pl, twx);
        const Task k = task_of(u);
        const int a = k.a, h = k.h;
        const long long poff = k.z * (long long)(PLN * PLN);
        VO* io = yout.field(k.vec * 6 + 3 * k.h + k.a) + poff;
        // output half 0 (y_f): H_- acting on g (input half 1); half 1 (y_g): H_+ on f (half 0);
        // the transpose exchanges H_+ and H_-
        const int hin = 1 - h;
        const bool plus = (h == 1) != (TRANS != 0);
        const float* cb = coef + (plus ? 0 : 6) * npts + poff;
        const float* c0 = cb + sidx(a, 0) * npts;
        const float* c1 = cb + sidx(a, 1) * npts;
        const float* c2 = cb + sidx(a, 2) * npts;
        const float2* x0 = xin.field(k.vec * 6 + 3 * hin + 0) + poff;
        const float2* x1 = xin.field(k.vec * 6 + 3 * hin + 1) + poff;
        const float2* x2 = xin.field(k.vec * 6 + 3 * hin + 2) + poff;
#pragma unroll 4
        for (int j = 0; j < 16; ++j) {
            const int e = t + 1024 * j;
            const float2 kk = pl[(e >> 7) * PLP + (e & 127)];
            const float m0 = c0[e], m1 = c1[e], m2 = c2[e];
            const float2 u0 = x0[e], u1 = x1[e], u2 = x2[e];
            float2 y;
            y.x = kk.x + m0 * u0.x + m1 * u1.x + m2 * u2.x;
            y.y = kk.y + m0 * u0.y + m1 * u1.y + m2 * u2.y;
            io[e] = cmk<VO>(y.x, y.y);
        }
        lds_barrier();
    }
}

// ----------------------------------------------------------------------------------------
// xy-plane passes in complex128 (nx = ny = 128, 3-D).  A complex128 plane (256 KiB) does not
// fit the LDS, so the y transform is split by decimation in frequency into two half-planes
// of 64 rows (128 KiB each, transformed in LDS one after the other):
//   P0[r] = A[r] + A[r + 64],  P1[r] = (A[r] - A[r + 64]) w^r   (r < 64, w = e^(-2 pi i/128)),
// whose 64-point y transforms are the rows 2m and 2m + 1 of the 128-point one.  The kernels
// run 512 threads (the half-plane transforms need about 90 registers, and P1 or the even
// half's result waits in registers meanwhile); a thread holds column t % 128, rows
// t / 128 + 4 j (j < 32) of a plane, so rows r and r + 64 are both its own.  The inverse pass inverts the even and the odd spectrum rows as half-planes and
// combines them in registers, y[r] = E[r] + w^-r O[r], y[r + 64] = E[r] - w^-r O[r], before
// the coupling.  Fields, tasks and the half swap are those of the complex64 kernels.
// ----------------------------------------------------------------------------------------
constexpr int PLH = PLN / 2;
constexpr size_t HALF64_LDS = (size_t)PLH * PLP * sizeof(double2);

// MODE 0: the 64 rows (128-point x transforms, 32 lanes per line); MODE 1: the 128 columns
// (64-point y transforms, 16 lanes per line, the 128-point table at stride 2).  Lines lie on
// consecutive lanes of one wave; one workgroup barrier at the end.
constexpr int P64T = 512;                         // threads of the complex128 plane kernels
// compiler barrier: bounds how far the unrolled loops below hoist their loads (all of them
// in flight at once would not fit the registers)
__device__ __forceinline__ void hoist_fence() { asm volatile("" ::: "memory"); }
template <bool INV, int MODE>
__device__ __forceinline__ void half_lines(double2* pl, const double2* __restrict__ tw) {
    constexpr int NL = MODE == 0 ? PLN : PLH;
    constexpr int Q = NL / 4;
    constexpr int NLINES = MODE == 0 ? PLH : PLN;
    constexpr int LPR = P64T / Q;
    const int t = threadIdx.x;
    const int ln = t / Q, i = t % Q;
#pragma unroll 1
    for (int rnd = 0; rnd < NLINES / LPR; ++rnd) {
        const int line = rnd * LPR + ln;
        const int lb = MODE == 0 ? line * PLP : line;
        const int ls = MODE == 0 ? 1 : PLP;
        // the twiddle loads stay in this round (hoisted out of the kernel's loops, the float64
        // twiddles of every stage would stay live in registers)
        const double2* twr = tw;
        asm volatile("" : "+s"(twr));
        double2 v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = pl[lb + (i + r * Q) * ls];
        line_fft<double2, NL, INV, SYNC_WAVE, (MODE == 0 ? 1 : 2)>(v, i, pl, lb, ls, twr);
        fft_sync<SYNC_WAVE>();
#pragma unroll
        for (int r = 0; r < 4; ++r) pl[lb + (i + r * Q) * ls] = v[r];
    }
    lds_barrier();
}

// forward: workgroup w = (field f, plane z); Y[sigma(f)] plane z = F_xy X[f] plane z.  One
// plane per workgroup (a persistent loop would keep the unrolled loops' address arithmetic
// live across planes, more than the registers hold)
__global__ void __launch_bounds__(P64T) k_plane_fwd64(FieldAddr<const double2> in, FieldAddr<double2> out,
                                                     long long nfields, int nz, const double2* __restrict__ twx,
                                                     const double2* __restrict__ twy) {
    extern __shared__ double2 ph[];
    const long long ntask = nfields * nz;
    const long long w = blockIdx.x;
    if (w >= ntask) return;
    const int t = threadIdx.x;
    const int r0 = t >> 7, c = t & 127;
    {
        const double2* src = in.field(w / nz) + (w % nz) * (long long)(PLN * PLN);
        const long long f = w / nz;
        const long long vec = f / 6;
        const int s = (int)(f % 6);
        const int so = s < 3 ? s + 3 : s - 3;
        double2* dst = out.field(vec * 6 + so) + (w % nz) * (long long)(PLN * PLN);
        double2 p1[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int r = r0 + 4 * j;
            const double2 a = src[r * PLN + c], b = src[(r + PLH) * PLN + c];
            ph[r * PLP + c] = cadd(a, b);
            p1[j] = mul_tw<double2, false>(csub(a, b), twy[r]);
            if ((j & 3) == 3) hoist_fence();
        }
        lds_barrier();
        half_lines<false, 0>(ph, twx);
        half_lines<false, 1>(ph, twy);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int e = t + P64T * j;        // half-plane row e / 128 -> plane row 2 (e / 128)
            dst[(2 * (e >> 7)) * PLN + (e & 127)] = ph[(e >> 7) * PLP + (e & 127)];
            if ((j & 3) == 3) hoist_fence();
        }
        lds_barrier();
#pragma unroll
        for (int j = 0; j < 16; ++j) ph[(r0 + 4 * j) * PLP + c] = p1[j];
        lds_barrier();
        half_lines<false, 0>(ph, twx);
        half_lines<false, 1>(ph, twy);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int e = t + P64T * j;
            dst[(2 * (e >> 7) + 1) * PLN + (e & 127)] = ph[(e >> 7) * PLP + (e & 127)];
            if ((j & 3) == 3) hoist_fence();
        }
        lds_barrier();
    }
}

// inverse + coupling in complex128, tasks as in k_plane_inv_couple (in place on Y), one task per
// workgroup: the grid has a workgroup per task, dealt to the XCDs as there
template <int TRANS>
__global__ void __launch_bounds__(P64T) k_plane_inv_couple64(FieldAddr<const double2> xin, FieldAddr<double2> yio,
                                                             long long nvec, int nz,
                                                             const double2* __restrict__ twx,
                                                             const double2* __restrict__ twy,
                                                             const double* __restrict__ coef) {
    extern __shared__ double2 ph[];
    const long long ngroups = nvec * 2 * nz;
    const int nxcd = 8, xcd = blockIdx.x % nxcd;
    const int nslot = (gridDim.x - xcd + nxcd - 1) / nxcd;
    const int slot = blockIdx.x / nxcd;
    const long long g0 = ngroups * xcd / nxcd, g1 = ngroups * (xcd + 1) / nxcd;
    const long long ntask = 3 * (g1 - g0);
    long long u = slot;
    if (u >= ntask) return;
    const int t = threadIdx.x;
    const int r0 = t >> 7, c = t & 127;
    const long long npts = xin.npts;
    auto sidx = [](int r, int c2) {
        const int lo = r < c2 ? r : c2, hi = r < c2 ? c2 : r;
        return lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
    };
    // spectrum rows 2m + half of the plane -> LDS half-plane, inverse y then x, this thread's
    // rows r0 + 8 j back into registers
    auto inv_half = [&](const double2* io, int half, double2 (&res)[16]) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int e = t + P64T * j;
            ph[(e >> 7) * PLP + (e & 127)] = io[(2 * (e >> 7) + half) * PLN + (e & 127)];
            if ((j & 7) == 7) hoist_fence();
        }
        lds_barrier();
        half_lines<true, 1>(ph, twy);
        half_lines<true, 0>(ph, twx);
#pragma unroll
        for (int j = 0; j < 16; ++j) res[j] = ph[(r0 + 4 * j) * PLP + c];
        lds_barrier();
    };
    {
        const long long g = g0 + u / 3;
        const int a = (int)(u % 3);
        const int h = (int)(g % 2);
        const long long vec = (g / 2) % nvec;
        const long long z = g / (2 * nvec);
        const long long poff = z * (long long)(PLN * PLN);
        double2* io = yio.field(vec * 6 + 3 * h + a) + poff;
        double2 ev[16], od[16];
        inv_half(io, 0, ev);
        inv_half(io, 1, od);
        const int hin = 1 - h;
        const bool plus = (h == 1) != (TRANS != 0);
        const double* cb = coef + (plus ? 0 : 6) * npts + poff;
        const double* c0 = cb + sidx(a, 0) * npts;
        const double* c1 = cb + sidx(a, 1) * npts;
        const double* c2 = cb + sidx(a, 2) * npts;
        const double2* x0 = xin.field(vec * 6 + 3 * hin + 0) + poff;
        const double2* x1 = xin.field(vec * 6 + 3 * hin + 1) + poff;
        const double2* x2 = xin.field(vec * 6 + 3 * hin + 2) + poff;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            if (j & 1) hoist_fence();
            const double2 o = mul_tw<double2, true>(od[j], twy[r0 + 4 * j]);
            const double2 kk2[2] = {cadd(ev[j], o), csub(ev[j], o)};
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int e = (r0 + 4 * j + PLH * q) * PLN + c;     // row r0 + 4 j + 64 q
                const double2 kk = kk2[q];
                const double m0 = c0[e], m1 = c1[e], m2 = c2[e];
                const double2 u0 = x0[e], u1 = x1[e], u2 = x2[e];
                double2 y;
                y.x = kk.x + m0 * u0.x + m1 * u1.x + m2 * u2.x;
                y.y = kk.y + m0 * u0.y + m1 * u1.y + m2 * u2.y;
                io[e] = y;
            }
        }
    }
}

template <typename V> FieldAddr<V> fa_block(V* lo, V* hi, long long vstride, long long npts) {
    FieldAddr<V> a; a.lo = lo; a.hi = hi; a.vstride = vstride; a.fpv = 6; a.npts = npts; return a;
}
template <typename V> FieldAddr<V> fa_fields(V* base, int fpv, long long vstride, long long npts) {
    FieldAddr<V> a; a.lo = base; a.hi = base + 3 * npts; a.vstride = vstride; a.fpv = fpv; a.npts = npts; return a;
}

template <typename R> const typename cplx_of<R>::type* tw_of(bdg_ctx* c, int axis);
template <> const double2* tw_of<double>(bdg_ctx* c, int axis) { return c->tw64[axis]; }
template <> const float2* tw_of<float>(bdg_ctx* c, int axis) { return c->tw32[axis]; }
template <typename R> const R* coef_of(bdg_ctx* c);
template <> const double* coef_of<double>(bdg_ctx* c) { return c->coef64; }
template <> const float* coef_of<float>(bdg_ctx* c) { return c->coef32; }

MultSpec make_ms(bdg_ctx* c, int precond, double shift) {
    MultSpec m;
    for (int a = 0; a < 3; ++a) m.s[a] = c->sym64[a];
    m.scale = 1.0 / (double)c->npts;
    m.shift = shift;
    m.precond = precond;
    return m;
}

// --------------------------- dispatch over N ---------------------------------------------
#define BDG_DISPATCH_N(NVAL, ...)                                        \
    switch (NVAL) {                                                      \
        case 8: { constexpr int NN = 8; __VA_ARGS__; } break;            \
        case 16: { constexpr int NN = 16; __VA_ARGS__; } break;          \
        case 32: { constexpr int NN = 32; __VA_ARGS__; } break;          \
        case 64: { constexpr int NN = 64; __VA_ARGS__; } break;          \
        case 128: { constexpr int NN = 128; __VA_ARGS__; } break;        \
        case 256: { constexpr int NN = 256; __VA_ARGS__; } break;        \
        case 512: { constexpr int NN = 512; __VA_ARGS__; } break;        \
        case 1024: { constexpr int NN = 1024; __VA_ARGS__; } break;      \
        default: return ctx_fail(c, BDG_EINVAL, "unsupported axis length"); \
    }

template <typename V, bool INV, int MODE, typename VO = V>
bdg_status run_xpass(bdg_ctx* c, FieldAddr<const V> in, FieldAddr<VO> out, long long nfields, MultSpec ms,
                     const decltype(V::x)* wgt = nullptr) {
    const int N = c->n[0];
    const long long lpf = c->npts / N;
    BDG_DISPATCH_N(N, {
        constexpr int LPW = (1024 / NN) > 0 ? (1024 / NN) : 1;
        const long long nl = nfields * lpf;
        dim3 grid((unsigned)((nl + LPW - 1) / LPW));
        hipLaunchKernelGGL((k_xpass<V, NN, INV, MODE, VO>), grid, dim3(LPW * (NN / 4)), 0, c->stream,
                           in, out, nfields, lpf, (const V*)tw_of<decltype(V::x)>(c, 0), ms, c->n[1], wgt);
    });
    return hip_check(c, hipGetLastError(), "k_xpass");
}

template <typename V, bool INV, int MODE>
bdg_status run_strided(bdg_ctx* c, FieldAddr<V> io, long long nfields, int axis, MultSpec ms) {
    const int N = c->n[axis];
    const int nx = c->n[0], ny = c->n[1];
    BDG_DISPATCH_N(N, {
        constexpr int TXM = StridedCfg<V, NN>::TX;
        const int tx = nx < TXM ? nx : TXM;
        const long long outer = (axis == 1) ? (long long)c->n[2] : (long long)ny;
        dim3 grid((unsigned)(nfields * outer * (nx / tx)));
        hipLaunchKernelGGL((k_strided<V, NN, INV, MODE>), grid, dim3(tx * (NN / 4)), 0, c->stream,
                           io, nfields, nx, ny, axis, tx, (const V*)tw_of<decltype(V::x)>(c, axis), ms);
    });
    return hip_check(c, hipGetLastError(), "k_strided");
}

template <typename V, int FORM, int TRANS, bool FULL>
bdg_status run_couple(bdg_ctx* c, FieldAddr<const V> xin, FieldAddr<V> yout, long long nvec, MultSpec ms) {
    using R = decltype(V::x);
    const int N = c->n[0];
    const long long lpf = c->npts / N;
    // four vectors per workgroup (the coefficients are read once for them) when that still
    // leaves a few thousand workgroups
    constexpr int NVB = FULL ? 1 : 4;
    BDG_DISPATCH_N(N, {
        constexpr int QL = CoupleCfg<NN>::QL;
        const long long ngroups = (lpf + QL - 1) / QL;
        const bool wide = ngroups * ((nvec + NVB - 1) / NVB) >= 4096;
        const int nvb = wide ? NVB : 1;
        dim3 grid((unsigned)(((nvec + nvb - 1) / nvb) * ngroups));
        if (wide)
            hipLaunchKernelGGL((k_couple<V, NN, FORM, TRANS, FULL, NVB>), grid, dim3(CoupleCfg<NN>::THREADS), 0,
                               c->stream, xin, yout, lpf, ngroups, nvec, (const V*)tw_of<R>(c, 0), ms, c->n[1],
                               FORM >= 2 ? (const R*)c->ccoef : coef_of<R>(c));
        else
            hipLaunchKernelGGL((k_couple<V, NN, FORM, TRANS, FULL, 1>), grid, dim3(CoupleCfg<NN>::THREADS), 0,
                               c->stream, xin, yout, lpf, ngroups, nvec, (const V*)tw_of<R>(c, 0), ms, c->n[1],
                               FORM >= 2 ? (const R*)c->ccoef : coef_of<R>(c));
    });
    return hip_check(c, hipGetLastError(), "k_couple");
}

template <typename V, int FORM, int TRANS>
bdg_status apply_chunk(bdg_ctx* c, int nvec, FieldAddr<const V> X, FieldAddr<V> Y);

template <typename V, int FORM, int TRANS>
bdg_status apply_impl(bdg_ctx* c, int nvec, FieldAddr<const V> X, FieldAddr<V> Y) {
    int chunk = nvec;
    if (c->apply_chunk_bytes > 0) {
        const size_t per_vec = 6 * (size_t)c->npts * sizeof(V);
        chunk = (int)std::max<size_t>(1, c->apply_chunk_bytes / per_vec);
    }
    for (int v0 = 0; v0 < nvec; v0 += chunk) {
        const int nv = std::min(chunk, nvec - v0);
        FieldAddr<const V> Xc = X;
        FieldAddr<V> Yc = Y;
        Xc.lo += v0 * X.vstride;
        Xc.hi += v0 * X.vstride;
        Yc.lo += v0 * Y.vstride;
        Yc.hi += v0 * Y.vstride;
        BDG_TRY((apply_chunk<V, FORM, TRANS>(c, nv, Xc, Yc)));
    }
    return BDG_OK;
}

// the three-pass (f, g) operator of complex64 128 x 128 x nz grids (see k_plane_fwd); Y is
// the work block of the first two passes, Yout receives the result (Y itself, or float64)
template <int TRANS, typename VO = float2>
bdg_status apply_planes(bdg_ctx* c, int nvec, FieldAddr<const float2> X, FieldAddr<float2> Y, FieldAddr<VO> Yout,
                        MultSpec ms) {
    static bool lds_set = false;
    if (!lds_set) {
        BDG_HIP(c, hipFuncSetAttribute((const void*)k_plane_fwd<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)PLANE_LDS));
        BDG_HIP(c, hipFuncSetAttribute((const void*)k_plane_inv_couple<0>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)PLANE_LDS));
        BDG_HIP(c, hipFuncSetAttribute((const void*)k_plane_inv_couple<1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)PLANE_LDS));
        BDG_HIP(c, hipFuncSetAttribute((const void*)k_plane_inv_couple<0, double2>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)PLANE_LDS));
        lds_set = true;
    }
    const long long nf = 6LL * nvec;
    const int nz = c->n[2];
    const long long ntask = nf * nz;
    const unsigned grid = (unsigned)std::min<long long>(ntask, c->ncu);
    hipLaunchKernelGGL(k_plane_fwd<false>, dim3(grid), dim3(1024), PLANE_LDS, c->stream, X, Y, nf, nz,
                       (const float2*)c->tw32[0], (const float2*)c->tw32[1], (const float*)nullptr);
    BDG_TRY(hip_check(c, hipGetLastError(), "k_plane_fwd"));
    BDG_TRY((run_strided<float2, false, 1>(c, Y, nf, 2, ms)));
    const unsigned grid_inv = (unsigned)std::max<long long>(8, std::min<long long>(ntask, c->ncu));
    hipLaunchKernelGGL((k_plane_inv_couple<TRANS, VO>), dim3(grid_inv), dim3(1024), PLANE_LDS, c->stream, X, Y,
                       Yout, (long long)nvec, nz, (const float2*)c->tw32[0], (const float2*)c->tw32[1],
                       (const float*)c->coef32);
    return hip_check(c, hipGetLastError(), "k_plane_inv_couple");
}

// the three-pass (f, g) operator of complex128 128 x 128 x nz grids (see k_plane_fwd64)
template <int TRANS>
bdg_status apply_planes64(bdg_ctx* c, int nvec, FieldAddr<const double2> X, FieldAddr<double2> Y, MultSpec ms) {
    static bool lds_set = false;
    if (!lds_set) {
        BDG_HIP(c, hipFuncSetAttribute((const void*)k_plane_fwd64, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)HALF64_LDS));
        BDG_HIP(c, hipFuncSetAttribute((const void*)k_plane_inv_couple64<0>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)HALF64_LDS));
        BDG_HIP(c, hipFuncSetAttribute((const void*)k_plane_inv_couple64<1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)HALF64_LDS));
        lds_set = true;
    }
    const long long nf = 6LL * nvec;
    const int nz = c->n[2];
    const long long ntask = nf * nz;
    hipLaunchKernelGGL(k_plane_fwd64, dim3((unsigned)ntask), dim3(P64T), HALF64_LDS, c->stream, X, Y, nf, nz,
                       (const double2*)c->tw64[0], (const double2*)c->tw64[1]);
    BDG_TRY(hip_check(c, hipGetLastError(), "k_plane_fwd64"));
    BDG_TRY((run_strided<double2, false, 1>(c, Y, nf, 2, ms)));
    // one workgroup per task: each XCD's share of the 2 nvec nz groups, three tasks each, plus
    // a workgroup of slack per XCD for the rounding of the shares
    const unsigned grid_inv = (unsigned)(8 * (3 * ((2 * (long long)nvec * nz + 7) / 8) + 3));
    hipLaunchKernelGGL(k_plane_inv_couple64<TRANS>, dim3(grid_inv), dim3(P64T), HALF64_LDS, c->stream, X, Y,
                       (long long)nvec, nz, (const double2*)c->tw64[0], (const double2*)c->tw64[1],
                       (const double*)c->coef64);
    return hip_check(c, hipGetLastError(), "k_plane_inv_couple64");
}

template <typename V, int FORM, int TRANS>
bdg_status apply_chunk(bdg_ctx* c, int nvec, FieldAddr<const V> X, FieldAddr<V> Y) {
    MultSpec ms = make_ms(c, 0, 0.0);
    const long long nf = 6LL * nvec;
    if constexpr (std::is_same<V, float2>::value && FORM == 1) {
        if (c->apply_planes && c->dim == 3 && c->n[0] == PLN && c->n[1] == PLN)
            return apply_planes<TRANS>(c, nvec, X, Y, Y, ms);
    }
    if constexpr (std::is_same<V, double2>::value && FORM == 1) {
        if (c->apply_planes64 && c->dim == 3 && c->n[0] == PLN && c->n[1] == PLN)
            return apply_planes64<TRANS>(c, nvec, X, Y, ms);
    }
    if (c->dim == 1) return run_couple<V, FORM, TRANS, true>(c, X, Y, nvec, ms);
    BDG_TRY((run_xpass<V, false, 0>(c, X, Y, nf, ms)));
    if (c->dim == 2) {
        BDG_TRY((run_strided<V, false, 1>(c, Y, nf, 1, ms)));
    } else {
        BDG_TRY((run_strided<V, false, 0>(c, Y, nf, 1, ms)));
        BDG_TRY((run_strided<V, false, 1>(c, Y, nf, 2, ms)));
        BDG_TRY((run_strided<V, true, 0>(c, Y, nf, 1, ms)));
    }
    return run_couple<V, FORM, TRANS, false>(c, X, Y, nvec, ms);
}

// float32 images widened to float64 (one vector, its 6 fields, per gridDim.y)
__global__ void k_fields_to64(long long npts3, FieldAddr<const float2> y, FieldAddr<double2> out) {
    const long long vec = blockIdx.y / 2;
    const int half = blockIdx.y % 2;
    const float2* src = y.field(vec * 6 + 3 * half);
    double2* dst = out.field(vec * 6 + 3 * half);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < npts3; i += (long long)gridDim.x * blockDim.x)
        dst[i] = cmk<double2>(src[i].x, src[i].y);
}

}  // namespace

template <typename R>
bdg_status launch_apply(bdg_ctx* c, int form, int transpose, int nvec,
                        BlockRef<const typename cplx_of<R>::type> X, BlockRef<typename cplx_of<R>::type> Y) {
    using V = typename cplx_of<R>::type;
    if (nvec <= 0) return BDG_OK;
    FieldAddr<const V> xa = fa_block<const V>(X.lo, X.hi, X.vstride, c->npts);
    FieldAddr<V> ya = fa_block<V>(Y.lo, Y.hi, Y.vstride, c->npts);
    if (form == BDG_FORM_FG) {
        return transpose ? apply_impl<V, 1, 1>(c, nvec, xa, ya) : apply_impl<V, 1, 0>(c, nvec, xa, ya);
    }
    return transpose ? apply_impl<V, 0, 1>(c, nvec, xa, ya) : apply_impl<V, 0, 0>(c, nvec, xa, ya);
}

bdg_status launch_apply_fg_to64(bdg_ctx* c, int nvec, BlockRef<const float2> X, BlockRef<float2> Ywork,
                                BlockRef<double2> Y64) {
    if (nvec <= 0) return BDG_OK;
    FieldAddr<const float2> xa = fa_block<const float2>(X.lo, X.hi, X.vstride, c->npts);
    FieldAddr<float2> wa = fa_block<float2>(Ywork.lo, Ywork.hi, Ywork.vstride, c->npts);
    FieldAddr<double2> ya = fa_block<double2>(Y64.lo, Y64.hi, Y64.vstride, c->npts);
    if (c->apply_chunk_bytes == 0 && c->apply_planes && c->dim == 3 && c->n[0] == PLN && c->n[1] == PLN)
        return apply_planes<0, double2>(c, nvec, xa, wa, ya, make_ms(c, 0, 0.0));
    BDG_TRY((apply_impl<float2, 1, 0>(c, nvec, xa, wa)));
    const long long npts3 = 3 * c->npts;
    long long bx = (npts3 + 255) / 256;
    if (bx > 1024) bx = 1024;
    FieldAddr<const float2> wc = fa_block<const float2>(Ywork.lo, Ywork.hi, Ywork.vstride, c->npts);
    hipLaunchKernelGGL(k_fields_to64, dim3((unsigned)bx, (unsigned)(2 * nvec)), dim3(256), 0, c->stream, npts3, wc,
                       ya);
    return hip_check(c, hipGetLastError(), "k_fields_to64");
}

bdg_status launch_apply_complex(bdg_ctx* c, int kform, int nvec, BlockRef<const double2> X, BlockRef<double2> Y) {
    if (nvec <= 0) return BDG_OK;
    if (!c->complex_gs || !c->ccoef) return ctx_fail(c, BDG_ESTATE, "complex apply needs a complex ground state");
    FieldAddr<const double2> xa = fa_block<const double2>(X.lo, X.hi, X.vstride, c->npts);
    FieldAddr<double2> ya = fa_block<double2>(Y.lo, Y.hi, Y.vstride, c->npts);
    return kform ? apply_impl<double2, 3, 0>(c, nvec, xa, ya) : apply_impl<double2, 2, 0>(c, nvec, xa, ya);
}

template <typename R>
bdg_status launch_fourier(bdg_ctx* c, int nfields, int fpv, long long vstride,
                          const typename cplx_of<R>::type* X, typename cplx_of<R>::type* Y, int precond, double shift,
                          const R* wgt) {
    using V = typename cplx_of<R>::type;
    if (nfields <= 0) return BDG_OK;
    MultSpec ms = make_ms(c, precond, shift);
    FieldAddr<const V> xa = fa_fields<const V>(X, fpv, vstride, c->npts);
    FieldAddr<V> ya = fa_fields<V>(Y, fpv, vstride, c->npts);
    if (c->dim == 1) return run_xpass<V, false, 1>(c, xa, ya, nfields, ms, wgt);
    BDG_TRY((run_xpass<V, false, 0>(c, xa, ya, nfields, ms, wgt)));
    if (c->dim == 2) {
        BDG_TRY((run_strided<V, false, 1>(c, ya, nfields, 1, ms)));
    } else {
        BDG_TRY((run_strided<V, false, 0>(c, ya, nfields, 1, ms)));
        BDG_TRY((run_strided<V, false, 1>(c, ya, nfields, 2, ms)));
        BDG_TRY((run_strided<V, true, 0>(c, ya, nfields, 1, ms)));
    }
    FieldAddr<const V> yc = fa_fields<const V>(Y, fpv, vstride, c->npts);
    return run_xpass<V, true, 0>(c, yc, ya, nfields, ms, wgt);
}

template <typename R>
bdg_status launch_fft(bdg_ctx* c, int nfields, const typename cplx_of<R>::type* X,
                      typename cplx_of<R>::type* Y, int inverse) {
    using V = typename cplx_of<R>::type;
    if (nfields <= 0) return BDG_OK;
    MultSpec ms = make_ms(c, 0, 0.0);
    const long long vs = c->npts;
    FieldAddr<const V> xa = fa_fields<const V>(X, 1, vs, c->npts);
    FieldAddr<V> ya = fa_fields<V>(Y, 1, vs, c->npts);
    if (inverse) {
        BDG_TRY((run_xpass<V, true, 0>(c, xa, ya, nfields, ms)));
        for (int a = 1; a < c->dim; ++a) BDG_TRY((run_strided<V, true, 0>(c, ya, nfields, a, ms)));
    } else {
        BDG_TRY((run_xpass<V, false, 0>(c, xa, ya, nfields, ms)));
        for (int a = 1; a < c->dim; ++a) BDG_TRY((run_strided<V, false, 0>(c, ya, nfields, a, ms)));
    }
    return BDG_OK;
}

template bdg_status launch_apply<double>(bdg_ctx*, int, int, int, BlockRef<const double2>, BlockRef<double2>);
template bdg_status launch_apply<float>(bdg_ctx*, int, int, int, BlockRef<const float2>, BlockRef<float2>);
template <typename R> const R* pw_of(bdg_ctx* c);
template <> const double* pw_of<double>(bdg_ctx* c) { return c->pw64; }
template <> const float* pw_of<float>(bdg_ctx* c) { return c->pw32; }

template <typename R>
bdg_status launch_precond(bdg_ctx* c, int nfields, int fpv, long long vstride,
                          const typename cplx_of<R>::type* X, typename cplx_of<R>::type* Y) {
    if (!c->has_gs) return ctx_fail(c, BDG_ESTATE, "preconditioner needs the ground state");
    return launch_fourier<R>(c, nfields, fpv, vstride, X, Y, 1, c->pshift, pw_of<R>(c));
}

bdg_status launch_precond_mixed(bdg_ctx* c, int nvec, BlockRef<float2> X32, BlockRef<double2> Y64) {
    if (nvec <= 0) return BDG_OK;
    if (!c->has_gs) return ctx_fail(c, BDG_ESTATE, "preconditioner needs the ground state");
    MultSpec ms = make_ms(c, 1, c->pshift);
    const long long nf = 6LL * nvec;
    FieldAddr<float2> xa = fa_block<float2>(X32.lo, X32.hi, X32.vstride, c->npts);
    FieldAddr<const float2> xc = fa_block<const float2>(X32.lo, X32.hi, X32.vstride, c->npts);
    FieldAddr<double2> ya = fa_block<double2>(Y64.lo, Y64.hi, Y64.vstride, c->npts);
    const float* wgt = c->pw32;
    if (c->apply_planes && c->dim == 3 && c->n[0] == PLN && c->n[1] == PLN) {
        // three passes: weighted xy forward in LDS, z with the multiplier, xy inverse weighted
        // and widened (the x and y passes below, fused by planes; the weight's products round
        // before the transforms here, where the x pass may contract them into its first
        // butterflies)
        static bool lds_set = false;
        if (!lds_set) {
            BDG_HIP(c, hipFuncSetAttribute((const void*)k_plane_fwd<true>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)PLANE_LDS));
            BDG_HIP(c, hipFuncSetAttribute((const void*)k_plane_inv_w, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)PLANE_LDS));
            lds_set = true;
        }
        const int nz = c->n[2];
        const unsigned grid = (unsigned)std::min<long long>(nf * nz, c->ncu);
        hipLaunchKernelGGL(k_plane_fwd<true>, dim3(grid), dim3(1024), PLANE_LDS, c->stream, xc, xa, nf, nz,
                           (const float2*)c->tw32[0], (const float2*)c->tw32[1], wgt);
        BDG_TRY(hip_check(c, hipGetLastError(), "k_plane_fwd"));
        BDG_TRY((run_strided<float2, false, 1>(c, xa, nf, 2, ms)));
        hipLaunchKernelGGL(k_plane_inv_w, dim3(grid), dim3(1024), PLANE_LDS, c->stream, xc, ya, nf, nz,
                           (const float2*)c->tw32[0], (const float2*)c->tw32[1], wgt);
        return hip_check(c, hipGetLastError(), "k_plane_inv_w");
    }
    if (c->dim == 1) return run_xpass<float2, false, 1, double2>(c, xc, ya, nf, ms, wgt);
    BDG_TRY((run_xpass<float2, false, 0>(c, xc, xa, nf, ms, wgt)));
    if (c->dim == 2) {
        BDG_TRY((run_strided<float2, false, 1>(c, xa, nf, 1, ms)));
    } else {
        BDG_TRY((run_strided<float2, false, 0>(c, xa, nf, 1, ms)));
        BDG_TRY((run_strided<float2, false, 1>(c, xa, nf, 2, ms)));
        BDG_TRY((run_strided<float2, true, 0>(c, xa, nf, 1, ms)));
    }
    return run_xpass<float2, true, 0, double2>(c, xc, ya, nf, ms, wgt);
}

template bdg_status launch_fourier<double>(bdg_ctx*, int, int, long long, const double2*, double2*, int, double,
                                           const double*);
template bdg_status launch_fourier<float>(bdg_ctx*, int, int, long long, const float2*, float2*, int, double,
                                          const float*);
template bdg_status launch_precond<double>(bdg_ctx*, int, int, long long, const double2*, double2*);
template bdg_status launch_precond<float>(bdg_ctx*, int, int, long long, const float2*, float2*);
template bdg_status launch_fft<double>(bdg_ctx*, int, const double2*, double2*, int);
template bdg_status launch_fft<float>(bdg_ctx*, int, const float2*, float2*, int);
