// Local SCS: assembly, Cholesky factorisation and solves of
//   B~_K alpha~_K = d_K                         (Sec. III.B, local polarisability system)
//   B~_K,ij = delta_ij / abar_i + T_SR,K,ij     (i, j in K1)
//   d_K,i   = I - sum_{j in K2} T_SR,K,ij abar_j
//   T_SR,K,ij = f_inner f_SR (1 - f(r, S)) (-T g + h)     (Sec. II.B and III.B)
// and the adjoint of the isotropic polarisabilities alpha~_iso = Tr(X_i)/3.
//
// One workgroup per (atom, frequency).  B~_K is symmetric positive definite on
// the workloads (measured: diagonally scaled condition numbers below 12), so it
// is factorised by a left-looking blocked Cholesky in its own slot of device
// memory; the factor is kept for the adjoint solve.  A non-positive pivot is a
// breakdown reported to the host.  Kernels: k_pairlist (pair lists of an atom),
// k_scs_dvec (d and the rows of d^T), k_scs_factor (assembly of B~,
// factorisation, first solve and the mixed path's refinement), k_scs_solve (the
// adjoint solve), k_scs_adjoint (pair gradients).
//
// Precision: the kernels are templated on the matrix type R.  R = double is the
// plain FP64 path.  R = float is the mixed path: pair tensors, the matrix and
// its factor in FP32 (MFMA f32), the forward solve refined in FP64 against the
// matrix rebuilt from its FP32 pair coefficients, solutions and all sums in FP64.
#include <type_traits>

#include "lmbd_internal.h"

namespace lmbd {

constexpr int NB = 16;      // block size of the factorisation

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));


// MFMA 16x16x4 in the matrix type.  Lane layouts measured on gfx950: A[i][k] <- lane
// i + 16k and B[k][j] <- lane j + 16k for both types; the accumulator holds D[i][j] in
// lane j + 16 (i % 4), register i / 4 for f64, and in lane j + 16 (i / 4), register
// i % 4 for f32.  acc_row(g, q) is the row held by lane group g = lane / 16 in register q.
template <typename R> struct Mfma;
template <> struct Mfma<double> {
    typedef d4_t acc;
    static __device__ inline acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int acc_row(int g, int q) { return g + 4 * q; }
};
template <> struct Mfma<float> {
    typedef f4_t acc;
    static __device__ inline acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int acc_row(int g, int q) { return 4 * g + q; }
};

// T_SR,K for one pair as A rhat rhat^T + B I, with radial derivatives.
template <typename P>
struct SrPair {
    P A, B, dA, dB;
};

template <typename P>
__device__ inline SrPair<P> sr_pair(P r, P ir, P s_ij, P S, P damp_d, P rc, P rb, P wmul, P dwmul) {
    P A, B, dA, dB;
    sr_core<P>(r, ir, s_ij, A, B, dA, dB);
    P dfdr, dfdS, dcut;
    const P f = fermi<P>(r, S, damp_d, dfdr, dfdS);
    const P fc = cutoff_poly<P>(r, rc, rb, dcut);
    const P w = wmul * fc * (P(1) - f);
    const P dw = dwmul * fc * (P(1) - f) + wmul * dcut * (P(1) - f) - wmul * fc * dfdr;
    return SrPair<P>{w * A, w * B, dw * A + w * dA, dw * B + w * dB};
}

__device__ inline void tri_decode(int t, int& i, int& j) {
    // a single-precision estimate of the row, corrected in integers
    int a = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((a + 1) * (a + 2) / 2 <= t) ++a;
    while (a * (a + 1) / 2 > t) --a;
    i = a;
    j = t - a * (a + 1) / 2;
}

__device__ inline void inner_buffer(double r, double rin, double& fin, double& dfin) {
    fin = 1.0;
    dfin = 0.0;
    if (r < rin) {
        const double x = r / rin;
        fin = 3.0 * x * x - 2.0 * x * x * x;
        dfin = (6.0 * x - 6.0 * x * x) / rin;
    }
}

// ---------------------------------------------------------------------------
// Storage: the N x N matrix is row-major, lower triangle (A[row * ld + col],
// col <= row), ld a multiple of 4 so that a 16-column row segment is four
// aligned 4-vectors.  After the factorisation the strict upper part of each
// 16x16 diagonal block holds the strict lower part of that block's inverse
// Z = L_bb^{-1}, transposed (Z[r][q], r > q, at (q, r)); the diagonal of Z is
// 1 / L[r][r].
//
// Left-looking blocked Cholesky by one workgroup, 32-column panels P (two 16-column
// tiles, h = 0, 1), in units of two 16-row tiles from the panel's diagonal down:
//  (1) update  A[c0:N+3, c0:c0+32] -= L[c0:N+3, 0:c0] L[c0:c0+32, 0:c0]^T  on MFMA
//      16x16x4, 16 k at a time from aligned 4-vector loads, a ring of chunks in
//      flight per wavefront.  The tiles of a unit stay in registers, held
//      transposed (M = A^T: the accumulator layout in which a tile's four
//      registers are directly the right-hand operands of the four k-steps of
//      the next 16 x 16 x 16 product).  Units are handed out from a counter in
//      LDS; with fewer units than wavefronts their k range is split and the
//      parts meet in LDS; in long panels the k range of unit 0 is split over
//      all wavefronts first;
//  (2) unit 0 (the diagonal tiles), by one wavefront at raised priority:
//      factorise the first diagonal tile and invert it (Z1 = L11^{-1}), L21 =
//      A21 Z1^T, A22 -= L21 L21^T, factorise and invert the second (Z2), all
//      into the matrix and Z1, L21, Z2 into LDS, then raise a flag in LDS;
//  (3) any other unit, once the flag is up: X1 = A1 Z1^T, A2 -= X1 L21^T,
//      X2 = A2 Z2^T on its own registers, written to the matrix.
// One barrier per panel (two with split units).  The three extra rows (d^T) are
// ordinary rows of the last row tiles, so the factorisation leaves y = L^{-1} d
// in them.  Which wavefront takes the diagonal rotates over the workgroups, so
// that the chains of the workgroups sharing a compute unit spread over its SIMDs.
// LDS: a few tiles and the split parts, so several factorisations share a
// compute unit and hide each other's memory latency.
// ---------------------------------------------------------------------------
constexpr int kSlotLd = 17;   // row stride of a 16x16 tile in LDS (padding against bank conflicts)
#ifndef LMBD_FACTOR_RING
#define LMBD_FACTOR_RING 2
#endif
constexpr int kRing = LMBD_FACTOR_RING;   // chunks of the panel update in flight per wavefront

// value of x in lane `lane` (a wavefront-uniform constant) for every lane
__device__ __forceinline__ double bcast(double x, int lane) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ float bcast(float x, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

// 1/sqrt(x): the hardware estimate and one Newton step (error a few ulp)
__device__ __forceinline__ double rsqrt_refined(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return y * fma(-0.5 * x * y, y, 1.5);
}
__device__ __forceinline__ float rsqrt_refined(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    return y * fmaf(-0.5f * x * y, y, 1.5f);
}

template <typename R> struct Vec4T;
template <> struct Vec4T<double> { typedef d4_t type; };
template <> struct Vec4T<float> { typedef f4_t type; };

template <typename R>
__device__ inline typename Vec4T<R>::type load4(const R* p) {
    return *reinterpret_cast<const typename Vec4T<R>::type*>(p);
}

constexpr int kMaxParts = 3;          // stored k-split parts of a panel: at most wavefronts - 1
constexpr int kSpinMax = 1 << 22;     // polls of the diagonal flag before a wavefront gives up

// Diagonal block by one wavefront: the 16 x 16 tile in Lt (row-major, rows < jb) is
// factorised with lane l < 16 holding row l of the tile and lane 16 + l column l of
// Z = L^{-1}.  Step c scales entry c of every lane by 1 / L_cc and reads L[s][c] (s > c)
// from lane s; the same update x[s] -= L[s][c] x[c], one instruction for both halves,
// is the right-looking update of the later rows of the tile and the forward
// substitution of every column of Z in the order of c.  L goes to the matrix at
// (c0, c0), Z to Zs (row-major) and its strict lower part, transposed, to the block's
// strict upper part in the matrix.  Rows from jb on are those of the identity.  good
// turns false on a pivot that is not positive.
template <typename R>
__device__ __forceinline__ void diag_block(R* __restrict__ Lt, int jb, R* __restrict__ A, int ld, int c0,
                                           R* __restrict__ Zs, bool& good) {
    // (l is made opaque so that the per-lane constants are not hoisted out of the
    // panel loop, where they would only take registers)
    int l = threadIdx.x & 63;
    asm volatile("" : "+v"(l));
    const int r = l & 15;
    const bool lrow = l < NB;   // lanes of L; lanes 16 .. 31 carry Z (and 32 .. 63 a copy)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    R x[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c)
        x[c] = (lrow && r < jb && c <= r) ? Lt[r * kSlotLd + c] : (r == c ? R(1) : R(0));
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        const R dcc = bcast(x[c], c);
        if (c < jb && !(dcc > R(0))) good = false;
        const R inv = rsqrt_refined(dcc);
        // entries above the diagonal of the tile (l < s) are never stored or read
        // from another lane again
        x[c] = (l == c ? dcc : x[c]) * inv;
#pragma unroll
        for (int s = c + 1; s < NB; ++s) x[s] -= x[c] * bcast(x[c], s);   // L[s][c]
        __builtin_amdgcn_sched_barrier(0);
    }
    if (lrow && r < jb) {
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (c <= r) A[(size_t)(c0 + r) * ld + c0 + c] = x[c];
    }
    if (l >= NB && l < 2 * NB) {
#pragma unroll
        for (int q = 0; q < NB; ++q) Zs[q * kSlotLd + r] = x[q];
        if (r < jb) {
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (q > r && q < jb) A[(size_t)(c0 + r) * ld + c0 + q] = x[q];
        }
    }
}

// The factorisation (see the storage and algorithm notes above).  Lt: one tile and
// its padding column; part: kMaxParts x 4 tiles of k-split partial sums; pre: 2 x 4
// tiles (the prepared unit 0, double-buffered over panels); Z1, Z2, L21: one tile
// each; ctl: two unit counters, the diagonal flag and the give-up flag.
template <typename R>
__device__ __forceinline__ void chol_factor(R* __restrict__ A, int N, int ld, R* __restrict__ Lt,
                                            R* __restrict__ part, R* __restrict__ pre, R* __restrict__ Z1,
                                            R* __restrict__ Z2, R* __restrict__ L21, int* ctl, int dw, bool& ok,
                                            bool& stalled) {
    typedef Mfma<R> M;
    typedef typename M::acc Acc;
    typedef typename Vec4T<R>::type V4;
    const int tid = threadIdx.x;
    const int lane = tid & 63, nwave = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform, so are the unit indices below
    const int li = lane & 15, lk = lane >> 4;
    const int Nr = N + 3;                           // rows: B~, then d^T
    const int ntr = (Nr + NB - 1) / NB;             // row tiles
    const int npan = (N + 2 * NB - 1) / (2 * NB);   // 32-column panels
    const V4 zero = {R(0), R(0), R(0), R(0)};
    Acc zacc;
#pragma unroll
    for (int q = 0; q < 4; ++q) zacc[q] = R(0);
    // (1) the update of unit u (row tiles 2u, 2u + 1; both column tiles) of the panel
    // at column c0p (mtp row tiles from its diagonal down, a second column tile if twop)
    // with the chunks cb, cb + st, .. below ce: m[x][h] = A(2u + x, h)^T - (L_h L_t^T)^T,
    // starting from the matrix (init 0), from zero (1) or from m as given (2)
    auto update = [&](int c0p, int mtp, bool twop, int u, int cb, int st, int ce, int init, Acc(&m)[2][2]) {
        // (the lane's indices are made opaque here so that the offsets derived from
        // them are formed per call rather than held, or spilled, over the panel loop)
        int lio = li, lko = lk;
        asm volatile("" : "+v"(lio), "+v"(lko));
        bool v[2][2];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int t = 2 * u + x;
                v[x][h] = t < mtp && (h == 0 || twop) && !(t == 0 && h == 1);
                if (init != 2) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int row = c0p + NB * t + lio, col = c0p + NB * h + M::acc_row(lko, q);
                        m[x][h][q] = (init == 0 && v[x][h] && row < Nr && col < N && (t != h || row >= col))
                                         ? A[(size_t)row * ld + col] : R(0);
                    }
                }
            }
        if (cb < ce) {   // uniform
            const R* pt[2];
            const R* ph[2];
            bool okt[2], okh[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const int r = c0p + NB * (2 * u + x) + lio;
                okt[x] = 2 * u + x < mtp && r < Nr;
                pt[x] = A + (size_t)(okt[x] ? r : 0) * ld + 4 * lko;
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = c0p + NB * h + lio;
                okh[h] = (h == 0 || twop) && r < N;
                ph[h] = A + (size_t)(okh[h] ? r : 0) * ld + 4 * lko;
            }
            auto ld4 = [&](const R* base, bool okr, int c) { return (okr && c < ce) ? load4(base + NB * c) : zero; };
            // ring of kRing chunks: each chunk's registers are refilled with the chunk
            // kRing ahead right after use
            V4 rt[kRing][2], rh[kRing][2];
#pragma unroll
            for (int j = 0; j < kRing; ++j) {
#pragma unroll
                for (int x = 0; x < 2; ++x) rt[j][x] = ld4(pt[x], okt[x], cb + j * st);
#pragma unroll
                for (int h = 0; h < 2; ++h) rh[j][h] = ld4(ph[h], okh[h], cb + j * st);
            }
            for (int ch = cb; ch < ce; ch += kRing * st) {
#pragma unroll
                for (int j = 0; j < kRing; ++j) {
                    if (ch + j * st < ce) {   // uniform
#pragma unroll
                        for (int x = 0; x < 2; ++x)
#pragma unroll
                            for (int h = 0; h < 2; ++h)
                                if (v[x][h]) {   // uniform
#pragma unroll
                                    for (int e = 0; e < 4; ++e) m[x][h] = M::mma(-rh[j][h][e], rt[j][x][e], m[x][h]);
                                }
                    }
                    const int cn = ch + (j + kRing) * st;
#pragma unroll
                    for (int x = 0; x < 2; ++x) rt[j][x] = ld4(pt[x], okt[x], cn);
#pragma unroll
                    for (int h = 0; h < 2; ++h) rh[j][h] = ld4(ph[h], okh[h], cn);
                }
            }
        }
    };
    // k-split parts of panel Pq's units; and whether unit 0 of panel Pq is prepared
    // during panel Pq - 1 (all chunks but the last two) by the wavefront after the
    // diagonal one, so that the chain of Pq starts after two chunks
    auto kparts = [&](int Pq) {
        const int nuq = (ntr - 2 * Pq + 1) / 2, nchq = 2 * Pq;
        return (nuq < nwave && nchq > 1) ? min(nwave / nuq, nchq) : 1;
    };
    auto has_pre = [&](int Pq) { return Pq >= 2 && Pq < npan && kparts(Pq) == 1; };
    const int pw = (dw + 1) % nwave;
    bool good = true;
    if (tid < 4) ctl[tid] = 0;
    __syncthreads();
    for (int P = 0; P < npan; ++P) {
        const int c0 = 2 * NB * P;
        const int jb = min(2 * NB, N - c0), jb1 = min(NB, jb), jb2 = jb - jb1;
        const bool two = jb2 > 0;                   // the panel has a second column tile
        const int mt = ntr - 2 * P;                 // row tiles from the panel's diagonal down
        const int nu = (mt + 1) / 2;                // units: pairs of row tiles
        const int nch = 2 * P;                      // finished 16-column chunks
        const int S = kparts(P);                    // k-split parts
        // X^T = Z M for a tile held transposed (M = X^T before the step): the Z operand
        // row-major from LDS, the tile's registers as the right-hand operands
        auto zmul = [&](const R* Zs, const Acc& mm) {
            Acc xo = zacc;
#pragma unroll
            for (int e = 0; e < 4; ++e) xo = M::mma(Zs[li * kSlotLd + M::acc_row(lk, e)], mm[e], xo);
            return xo;
        };
        // rows rmin.. of the result X (held transposed) of row tile t, column tile h
        auto store_x = [&](const Acc& xt, int t, int h, int rmin) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = c0 + NB * t + li, col = c0 + NB * h + M::acc_row(lk, q);
                if (li >= rmin && row < Nr && col < N) A[(size_t)row * ld + col] = xt[q];
            }
        };
        // (2) unit 0, by one wavefront: the diagonal tiles and L21, published to the others
        // (the tiles of row tile 1 wait in LDS, in the first part slot, while the first
        // diagonal block is factorised; its rows of d^T, if any, stay in Lt)
        auto diag_unit = [&](Acc(&m)[2][2]) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                Lt[li * kSlotLd + M::acc_row(lk, q)] = m[0][0][q];
                part[(0 * 4 + q) * 64 + lane] = m[1][0][q];
                part[(1 * 4 + q) * 64 + lane] = m[1][1][q];
            }
            asm volatile("" ::: "memory");   // really reload them: no registers held over the chain
            // the two diagonal blocks in one loop that is not unrolled: the block's code
            // (the longest straight line of the kernel) is there once per call
            const int nblk = (mt > 1 && two) ? 2 : 1;
#pragma clang loop unroll(disable)
            for (int b = 0; b < nblk; ++b) {
                R* Zb = b == 0 ? Z1 : Z2;
                const int jbb = b == 0 ? jb1 : jb2;
                diag_block<R>(Lt, jbb, A, ld, c0 + NB * b, Zb, good);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                if (jbb < NB) {   // rows of d^T in the diagonal tile (still in Lt)
                    Acc mbb;
#pragma unroll
                    for (int q = 0; q < 4; ++q) mbb[q] = Lt[li * kSlotLd + M::acc_row(lk, q)];
                    store_x(zmul(Zb, mbb), b, b, jbb);
                }
                if (b == 0 && mt > 1) {
                    Acc m10, m11;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        m10[q] = part[(0 * 4 + q) * 64 + lane];
                        m11[q] = part[(1 * 4 + q) * 64 + lane];
                    }
                    const Acc l21 = zmul(Z1, m10);
                    store_x(l21, 1, 0, 0);
#pragma unroll
                    for (int q = 0; q < 4; ++q) L21[li * kSlotLd + M::acc_row(lk, q)] = l21[q];
                    if (two) {
                        // A22 -= L21 L21^T: the registers of L21^T are both operands
#pragma unroll
                        for (int e = 0; e < 4; ++e) m11 = M::mma(-l21[e], l21[e], m11);
#pragma unroll
                        for (int q = 0; q < 4; ++q) Lt[li * kSlotLd + M::acc_row(lk, q)] = m11[q];
                        asm volatile("" ::: "memory");
                    }
                }
            }
            // the flag orders only the LDS tiles: the wavefront does not wait for its
            // stores to the matrix, which the other wavefronts read after the panel's barrier
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
            if (lane == 0) __hip_atomic_store(ctl + 2, P + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        };
        // (3) any other unit, once the diagonal flag says panel P: X1 = A1 Z1^T,
        // A2 -= X1 L21^T, X2 = A2 Z2^T, all on the unit's registers
        auto below_unit = [&](int u, Acc(&m)[2][2]) {
            for (int it = 0;; ++it) {   // bounded wait: a wavefront that gives up flags the call
                if (__hip_atomic_load(ctl + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) > P) break;
                if (__hip_atomic_load(ctl + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0) break;
                if (it >= kSpinMax) {
                    __hip_atomic_store(ctl + 3, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    stalled = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
            R z1[4], z2[4], lr[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = li * kSlotLd + M::acc_row(lk, e);
                z1[e] = Z1[o];
                z2[e] = Z2[o];
                lr[e] = L21[o];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const int t = 2 * u + x;
                if (t >= mt) continue;   // uniform
                Acc x1 = zacc;
#pragma unroll
                for (int e = 0; e < 4; ++e) x1 = M::mma(z1[e], m[x][0][e], x1);
                store_x(x1, t, 0, 0);
                if (two) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) m[x][1] = M::mma(-lr[e], x1[e], m[x][1]);
                    Acc x2 = zacc;
#pragma unroll
                    for (int e = 0; e < 4; ++e) x2 = M::mma(z2[e], m[x][1][e], x2);
                    store_x(x2, t, 1, 0);
                }
            }
        };
        if (S == 1) {
            // the diagonal wavefront takes unit 0 and starts its chain at once; units 1..
            // go to whichever wavefront asks next
            // the chain of the diagonal tiles is the panel's critical path: its
            // wavefront issues ahead of the other workgroups' updates on its SIMD and
            // finds unit 0 prepared but for the last two chunks
            if (wave == dw) {
                __builtin_amdgcn_s_setprio(2);
                Acc m[2][2];
                if (has_pre(P)) {
                    const R* pr = pre + (P & 1) * 16 * 64;
#pragma unroll
                    for (int y = 0; y < 4; ++y)
#pragma unroll
                        for (int q = 0; q < 4; ++q) m[y >> 1][y & 1][q] = pr[(y * 4 + q) * 64 + lane];
                    update(c0, mt, two, 0, nch - 2, 1, nch, 2, m);
                } else {
                    update(c0, mt, two, 0, 0, 1, nch, 0, m);
                }
                diag_unit(m);
                __builtin_amdgcn_s_setprio(0);
            }
            if (wave == pw && has_pre(P + 1)) {   // unit 0 of the next panel with this panel's chunks
                const int c0n = c0 + 2 * NB;
                Acc m[2][2];
                update(c0n, mt - 2, N - c0n > NB, 0, 0, 1, nch, 0, m);
                R* pr = pre + ((P + 1) & 1) * 16 * 64;
#pragma unroll
                for (int y = 0; y < 4; ++y)
#pragma unroll
                    for (int q = 0; q < 4; ++q) pr[(y * 4 + q) * 64 + lane] = m[y >> 1][y & 1][q];
            }
            if (tid == 0) ctl[(P + 1) & 1] = 0;   // the next panel's counter (last used before the previous barrier)
            int* ctr = ctl + (P & 1);
            for (;;) {
                int g = 0;
                if (lane == 0) g = atomicAdd(ctr, 1);
                g = __builtin_amdgcn_readfirstlane(g);
                if (1 + g >= nu) break;
                Acc m[2][2];
                update(c0, mt, two, 1 + g, 0, 1, nch, 0, m);
                below_unit(1 + g, m);
            }
        } else {
            // few units: item g = (unit g % nu, part g / nu) on wavefront dw + g; the parts
            // s > 0 go through LDS to the wavefront of part 0, which adds them in order
            const int g = (wave - dw + nwave) % nwave;
            const bool have = g < nu * S;
            const int u = g % nu, s = g / nu;
            Acc m[2][2] = {{zacc, zacc}, {zacc, zacc}};   // defined on every path: nothing carried between panels
            if (have) update(c0, mt, two, u, s, S, nch, s == 0 ? 0 : 1, m);
            if (have && s > 0) {
#pragma unroll
                for (int y = 0; y < 4; ++y)
#pragma unroll
                    for (int q = 0; q < 4; ++q) part[(((g - nu) * 4 + y) * 4 + q) * 64 + lane] = m[y >> 1][y & 1][q];
            }
            if (tid == 0) ctl[(P + 1) & 1] = 0;
            __syncthreads();
            if (have && s == 0) {
                for (int s2 = 1; s2 < S; ++s2) {
                    const int g2 = u + s2 * nu;
#pragma unroll
                    for (int y = 0; y < 4; ++y)
#pragma unroll
                        for (int q = 0; q < 4; ++q) m[y >> 1][y & 1][q] += part[(((g2 - nu) * 4 + y) * 4 + q) * 64 + lane];
                }
                if (u == 0) {
                    __builtin_amdgcn_s_setprio(2);
                    diag_unit(m);
                    __builtin_amdgcn_s_setprio(0);
                } else {
                    below_unit(u, m);
                }
            }
        }
        __syncthreads();   // the panel's columns are in the matrix before the next panel reads them
    }
    ok = good;
}

template <typename R>
__device__ __forceinline__ void solve_row_update(const R* __restrict__ lrow, int c0, int jb, int i, R* Y) {
    R s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        if (q < jb) {  // rows past N hold no solution values
            s0 += lrow[q] * Y[(c0 + q) * 3 + 0];
            s1 += lrow[q] * Y[(c0 + q) * 3 + 1];
            s2 += lrow[q] * Y[(c0 + q) * 3 + 2];
        }
    }
    Y[i * 3 + 0] -= s0;
    Y[i * 3 + 1] -= s1;
    Y[i * 3 + 2] -= s2;
}

// Triangular solves with the stored factor: L L^T x = b (fwd) or L^T x = y,
// three right-hand sides in Y (N x 3, LDS), one row (forward) or column
// (backward) per thread and slot: thread t takes t, t + blockDim, ..
// (NS slots, NS * blockDim >= N).  The first NP slots load the next block's
// segment a block ahead, the others load the segment they use at the start of
// its step.  Each row's sums are formed in the same order whatever NS, NP and
// blockDim are.
template <typename R, int NS, int NP>
__device__ __forceinline__ void chol_solve3(const R* __restrict__ A, int N, int ld, R* Y, R* zbuf, bool fwd) {
    static_assert(NP >= 1 && NP <= NS, "slot 0 always loads ahead");
    typedef typename Vec4T<R>::type V4;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int nt = (N + NB - 1) / NB;
    const int r = tid & 15, c = tid >> 4;
    const bool blk = tid < 48;   // threads of the block step (wavefront 0)
    const V4 zero = {R(0), R(0), R(0), R(0)};
    constexpr int kZ = NB * NB / 64;   // staged block entries per lane of wavefront 1
    // block-step operators, staged by wavefront 1 into LDS one block ahead:
    // forward Z[r][q] (q <= r), backward Z^T[r][q] = Z[q][r] (q >= r); Z[r][r] = 1 / L[r][r]
    auto zload = [&](int p, bool fwd, R* zr) {
        const int c0 = p * NB;
        const int jb = (p >= 0 && p < nt) ? min(NB, N - c0) : 0;
#pragma unroll
        for (int t = 0; t < kZ; ++t) {
            const int e = lane + 64 * t, rr = e / NB, q = e % NB;
            R v = R(0);
            if (wave == 1 && rr < jb && q < jb) {
                if (q == rr) v = A[(size_t)(c0 + rr) * ld + c0 + rr];
                else if (fwd && q < rr) v = A[(size_t)(c0 + q) * ld + c0 + rr];
                else if (!fwd && q > rr) v = A[(size_t)(c0 + rr) * ld + c0 + q];
            }
            zr[t] = v;
        }
    };
    auto zstore = [&](R* zb, const R* zr) {
        if (wave == 1) {
#pragma unroll
            for (int t = 0; t < kZ; ++t) {
                const int e = lane + 64 * t, rr = e / NB, q = e % NB;
                zb[rr * kSlotLd + q] = (q == rr && zr[t] != R(0)) ? R(1) / zr[t] : zr[t];
            }
        }
    };
    // row `row`'s segment of block column p (forward)
    auto rowseg = [&](R* dst, int row, int p, bool ok) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const V4 t4 = ok ? load4(A + (size_t)row * ld + p * NB + 4 * v) : zero;
#pragma unroll
            for (int e = 0; e < 4; ++e) dst[4 * v + e] = t4[e];
        }
    };
    // column `col`'s segment of block row p (backward; jb rows)
    auto colseg = [&](R* dst, int col, int p, int jb, bool ok) {
#pragma unroll
        for (int q = 0; q < NB; ++q) dst[q] = (ok && q < jb) ? A[(size_t)(p * NB + q) * ld + col] : R(0);
    };
    R zr[kZ];
    R cur[NS][NB], nxt[NP][NB];
    if (fwd) {
        // forward: L y = b
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int row = tid + s * nthr;
            rowseg(cur[s], row, 0, row >= NB && row < N);
        }
        zload(0, true, zr);
        zstore(zbuf, zr);
        zload(1, true, zr);
        __syncthreads();
        for (int p = 0; p < nt; ++p) {
            const int c0 = p * NB;
            const int jb = min(NB, N - c0);
            R* zb = zbuf + (p & 1) * NB * kSlotLd;
            zstore(zbuf + ((p + 1) & 1) * NB * kSlotLd, zr);   // block p + 1 (loaded during block p - 1)
            zload(p + 2, true, zr);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int row = tid + s * nthr;
                if (s < NP) rowseg(nxt[s < NP ? s : 0], row, p + 1, row >= c0 + 2 * NB && row < N);   // row follows block p + 1
                else if (p > 0) rowseg(cur[s], row, p, row >= c0 + NB && row < N);
            }
            if (blk && r < jb) {
                R v = 0;
#pragma unroll
                for (int q = 0; q < NB; ++q)
                    if (q < jb) v += zb[r * kSlotLd + q] * Y[(c0 + q) * 3 + c];  // rows past N hold no values
                Y[(c0 + r) * 3 + c] = v;  // one wavefront: all reads of the block precede this write
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int row = tid + s * nthr;
                if (row >= c0 + NB && row < N) solve_row_update(cur[s], c0, NB, row, Y);  // jb = 16 when rows follow
            }
            __syncthreads();
#pragma unroll
            for (int s = 0; s < NP; ++s)
#pragma unroll
                for (int q = 0; q < NB; ++q) cur[s][q] = nxt[s][q];
        }
    }
    // backward: L^T x = y
    {
        const int c0 = (nt - 1) * NB, jb = N - c0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int col = tid + s * nthr;
            colseg(cur[s], col, nt - 1, jb, col < c0);
        }
    }
    zload(nt - 1, false, zr);
    zstore(zbuf + ((nt - 1) & 1) * NB * kSlotLd, zr);
    zload(nt - 2, false, zr);
    __syncthreads();
    for (int p = nt - 1; p >= 0; --p) {
        const int c0 = p * NB;
        const int jb = min(NB, N - c0);
        R* zb = zbuf + (p & 1) * NB * kSlotLd;
        zstore(zbuf + ((p + 1) & 1) * NB * kSlotLd, zr);   // block p - 1
        zload(p - 2, false, zr);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int col = tid + s * nthr;
            if (s < NP) colseg(nxt[s < NP ? s : 0], col, p - 1, NB, p > 0 && col < c0 - NB);
            else if (p < nt - 1) colseg(cur[s], col, p, jb, col < c0);
        }
        if (blk && r < jb) {
            R v = 0;
#pragma unroll
            for (int q = 0; q < NB; ++q)
                if (q < jb) v += zb[r * kSlotLd + q] * Y[(c0 + q) * 3 + c];  // rows past N hold no values
            Y[(c0 + r) * 3 + c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int col = tid + s * nthr;
            if (col < c0) solve_row_update(cur[s], c0, jb, col, Y);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < NP; ++s)
#pragma unroll
            for (int q = 0; q < NB; ++q) cur[s][q] = nxt[s][q];
    }
}

// ---------------------------------------------------------------------------
// Sums over runs of equal key in a chunk of kChunk values (one per thread,
// keys ascending through the chunk, -1 for no value): each run's sum is added
// to acc[NV key ..] (global memory).  Within a wavefront by segmented prefix sums over the lanes
// with DPP moves (row shifts by 1, 2, 4, 8 inside rows of 16 lanes, then the
// last lane of a row broadcast to the rows after it; a lane adds what it
// receives when the sending lane has its key), so the run's last lane holds
// the run's sum and adds it; the part of a run that continues into the next
// wavefront goes to carry[] instead and is added by thread 0, in wavefront
// order, in add_carries() after the next barrier.  The order of every addition
// is fixed, so the sums do not depend on scheduling.  keys[] holds the chunk's
// keys (written before the barrier that precedes).
// ---------------------------------------------------------------------------
constexpr int kChunk = 256;              // threads of the chunked pair kernels = values per chunk
constexpr int kChunkWaves = kChunk / 64;

template <int CTRL, int RMASK>
__device__ __forceinline__ int dpp_int(int old, int src) {
    return __builtin_amdgcn_update_dpp(old, src, CTRL, RMASK, 0xF, false);
}
template <int CTRL, int RMASK>
__device__ __forceinline__ double dpp_dbl(double src) {   // lanes without a source read 0
    const long long b = __double_as_longlong(src);
    const int lo = dpp_int<CTRL, RMASK>(0, (int)b), hi = dpp_int<CTRL, RMASK>(0, (int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL, int RMASK, int NV>
__device__ __forceinline__ void seg_step(int key, double (&h)[NV]) {
    const int kd = dpp_int<CTRL, RMASK>(-2, key);
    double u[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = dpp_dbl<CTRL, RMASK>(h[v]);
    if (kd == key) {
#pragma unroll
        for (int v = 0; v < NV; ++v) h[v] += u[v];
    }
}

// acc (global memory) += v.  An address never has two additions in flight
// (within a chunk each key is added once, and the chunks and carries are
// separated by barriers), so the order of the additions is fixed; the
// hardware add at the cache saves the round trip of a read-modify-write.
__device__ __forceinline__ void acc_add(double* acc, double v) { (void)unsafeAtomicAdd(acc, v); }

template <int NV>
__device__ __forceinline__ void run_sums(int key, double (&h)[NV], const int32_t* keys, double* acc, double* carry,
                                         int* carry_key) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    seg_step<0x111, 0xF>(key, h);   // row_shr:1
    seg_step<0x112, 0xF>(key, h);   // row_shr:2
    seg_step<0x114, 0xF>(key, h);   // row_shr:4
    seg_step<0x118, 0xF>(key, h);   // row_shr:8
    seg_step<0x142, 0xA>(key, h);   // row_bcast:15 to rows 1 and 3
    seg_step<0x143, 0xC>(key, h);   // row_bcast:31 to rows 2 and 3
    const int knext = t + 1 < kChunk ? keys[t + 1] : -2;
    const bool cont = lane == 63 && wave + 1 < kChunkWaves && key >= 0 && knext == key;
    if (lane == 63) carry_key[wave] = cont ? key : -1;
    if (cont) {
#pragma unroll
        for (int v = 0; v < NV; ++v) carry[NV * wave + v] = h[v];
    } else if (key >= 0 && (lane == 63 || knext != key)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) acc_add(&acc[NV * key + v], h[v]);
    }
}

template <int NV>
__device__ __forceinline__ void add_carries(double* acc, const double* carry, const int* carry_key) {
    if (threadIdx.x != 0) return;
    for (int w = 0; w + 1 < kChunkWaves; ++w) {
        const int key = carry_key[w];
        if (key < 0) continue;
        for (int v = 0; v < NV; ++v) acc_add(&acc[NV * key + v], carry[NV * w + v]);
    }
}

// ---------------------------------------------------------------------------
// LDS layout of the pair kernels.  K1 sites, right-hand sides / solutions
// (FP64), the solve buffer in the matrix type, shell sites and a per-site
// reduction area.
// ---------------------------------------------------------------------------
struct ScsLds {
    double *px, *py, *pz, *ab, *sg, *R;        // K1 sites
    double *qx, *qy, *qz, *qab, *qsg, *qR;     // shell sites
    double *Y, *X;                             // adjoint: lambda and X, 3N x 3 each
    double* H;                                 // adjoint: pair terms of one chunk, 3 per thread
    double* gk;                                // d: sums; B~: pair values
    int32_t* key;                              // adjoint: reduction key of each thread's pair
};

static_assert(kChunk >= kMaxN1, "the adjoint gives every K1 site a thread of its own");

// Adjoint LDS: K1 sites, lambda (Y), the chunk's pair terms (H) and keys, then
// X for the K1 x K1 pairs, whose space the shell sites take for the K1 x shell
// pairs.  (The per-site sums are formed in the output slice in global memory.)
__device__ inline ScsLds scs_lds(double* base, int n1max, int n2max) {
    const int N = 3 * n1max;
    ScsLds L = {};
    L.px = base;
    L.py = L.px + n1max;
    L.pz = L.py + n1max;
    L.ab = L.pz + n1max;
    L.sg = L.ab + n1max;
    L.R = L.sg + n1max;
    L.Y = L.R + n1max;
    L.H = L.Y + 3 * N;
    L.key = reinterpret_cast<int32_t*>(L.H + 3 * kChunk);
    double* u = reinterpret_cast<double*>(L.key + kChunk);
    L.X = u;
    L.qx = u;
    L.qy = L.qx + n2max;
    L.qz = L.qy + n2max;
    L.qab = L.qz + n2max;
    L.qsg = L.qab + n2max;
    L.qR = L.qsg + n2max;
    return L;
}

size_t scs_lds_bytes(int n1max, int n2max, bool) {
    const size_t N = 3 * (size_t)n1max;
    return sizeof(double) * (6 * (size_t)n1max + 3 * N + 3 * kChunk + std::max(3 * N, 6 * (size_t)n2max)) +
           sizeof(int32_t) * kChunk;
}

// CSR offsets of the pair lists of atom k (i, q, a, b; see ScsArgs)
__device__ inline int32_t* pair_segs(const ScsArgs& a, int k) {
    return const_cast<int32_t*>(a.pl_seg) + 3 * (a.site_off[k] + 2 * (int64_t)k);
}

// sites only (assembly): K1 sites then shell sites
// assembly of d: K1 sites and shell sites; assembly of B~: K1 sites, one
// chunk of slots, word counts and a bit per K1 pair (coupled)
__host__ __device__ inline int assemble_mask_words(int n1max) { return (n1max * (n1max + 1) / 2 + 31) / 32; }

static size_t dvec_lds_bytes(int n1max, int n2max) { return sizeof(double) * 6 * ((size_t)n1max + n2max); }
static size_t matrix_lds_bytes(int n1max) {
    return sizeof(double) * 6 * (size_t)n1max + sizeof(int32_t) * (2 * kChunk + (size_t)assemble_mask_words(n1max));
}
size_t scs_assemble_lds_bytes(int n1max, int n2max) {
    return std::max(dvec_lds_bytes(n1max, n2max), matrix_lds_bytes(n1max));
}

__device__ inline ScsLds scs_assemble_lds(double* base, int n1max, int n2max, bool matrix) {
    ScsLds L = {};
    L.px = base;
    L.py = L.px + n1max;
    L.pz = L.py + n1max;
    L.ab = L.pz + n1max;
    L.sg = L.ab + n1max;
    L.R = L.sg + n1max;
    L.qx = L.R + n1max;
    L.qy = L.qx + n2max;
    L.qz = L.qy + n2max;
    L.qab = L.qz + n2max;
    L.qsg = L.qab + n2max;
    L.qR = L.qsg + n2max;
    L.gk = L.qR + n2max;          // d: sums
    L.key = reinterpret_cast<int32_t*>(L.gk + (matrix ? 0 : 6 * n1max));
    return L;
}

// sites s0 .. n12-1 of atom k (K1 sites below n1, then the shell) to LDS
__device__ inline void load_sites(const ScsArgs& a, int k, int w, int n1, int n12, const ScsLds& L, int s0 = 0) {
    const Site* S = a.sites + a.site_off[k];
    for (int s = s0 + threadIdx.x; s < n12; s += blockDim.x) {
        const Site st = S[s];
        const double ab = a.abar[(size_t)st.base * a.nw + w];
        const double sg = a.sigma[(size_t)st.base * a.nw + w];
        const double R = a.Rv[st.base];
        if (s < n1) {
            L.px[s] = st.x; L.py[s] = st.y; L.pz[s] = st.z;
            L.ab[s] = ab; L.sg[s] = sg; L.R[s] = R;
        } else {
            const int q = s - n1;
            L.qx[q] = st.x; L.qy[q] = st.y; L.qz[q] = st.z;
            L.qab[q] = ab; L.qsg[q] = sg; L.qR[q] = R;
        }
    }
}

// T_SR of K1 pair (i, j) as (A, B) in the arithmetic type P, with rhat in double
template <typename P>
__device__ inline SrPair<P> k1_pair(const ScsArgs& a, const ScsLds& L, int i, int j, double rc, double rh[3],
                                    double& r) {
    const double v[3] = {L.px[i] - L.px[j], L.py[i] - L.py[j], L.pz[i] - L.pz[j]};
    r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double ir = 1.0 / r;
    rh[0] = v[0] * ir; rh[1] = v[1] * ir; rh[2] = v[2] * ir;
    const double s_ij = sqrt(L.sg[i] * L.sg[i] + L.sg[j] * L.sg[j]);
    return sr_pair<P>(P(r), P(ir), P(s_ij), P(a.beta * (L.R[i] + L.R[j])), P(a.damp_d), P(rc), P(a.r_buf),
                      P(1), P(0));
}

// T_SR of the coupling of K1 site i to shell site q (with f_inner), arithmetic type P
template <typename P>
__device__ inline SrPair<P> k2_pair(const ScsArgs& a, const ScsLds& L, int i, int q, double rc, double rh[3],
                                    double& r) {
    const double v[3] = {L.px[i] - L.qx[q], L.py[i] - L.qy[q], L.pz[i] - L.qz[q]};
    r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double ir = 1.0 / r;
    rh[0] = v[0] * ir; rh[1] = v[1] * ir; rh[2] = v[2] * ir;
    const double s_ij = sqrt(L.sg[i] * L.sg[i] + L.qsg[q] * L.qsg[q]);
    double fin, dfin;
    inner_buffer(r, a.r_inner, fin, dfin);
    return sr_pair<P>(P(r), P(ir), P(s_ij), P(a.beta * (L.R[i] + L.qR[q])), P(a.damp_d), P(rc), P(a.r_buf),
                      P(fin), P(dfin));
}

// Assembly of d (into the solution slot), one workgroup per (atom, frequency):
// d_i = I - sum_q alpha_q T_SR(i, q) over the coupled shell sites.  Sixteen
// lanes per K1 site take its pairs of the i-major list in turn (lane l the
// pairs l, l + 16, ...), and a fixed exchange tree over the sixteen lanes sums
// the 6 components of the symmetric 3x3 terms: no barriers, a fixed order.
constexpr int kSiteLanes = 16;

template <typename R>
__global__ void __launch_bounds__(kChunk) k_scs_dvec(ScsArgs a, int n1max, int n2max) {
    extern __shared__ double lds[];
    constexpr bool mixed = sizeof(R) == 4;
    const int k = a.order[blockIdx.x];
    const int w = blockIdx.y;
    const int t = threadIdx.x;
    const Counts cnt = a.counts[k];
    const int n1 = cnt.n1, n12 = cnt.n12;
    const int N = 3 * n1;
    const int ld = a.fac_ld[k];
    const double rc = a.sinfo[a.atom_struct[k]].r_scs;
    ScsLds L = scs_assemble_lds(lds, n1max, n2max, false);
    double* D = (mixed ? a.dvec : a.xsol) + a.x_off[k] + (size_t)w * N * 3;
    const int32_t* seg_i = pair_segs(a, k);
    const int32_t* li = a.pl_i + a.pl_off[k];
    const int32_t* lq = a.pl_q + a.pl_off[k];
    load_sites(a, k, w, n1, n12, L);
    __syncthreads();
    // d (N x 3) to its slot, and d^T as the three rows appended to B~, so that the
    // factorisation carries out the forward substitution
    R* Dt = static_cast<R*>(a.fac) + a.fac_off[k] + (size_t)w * ld * (N + 3) + (size_t)N * ld;
    const int g = t / kSiteLanes, gl = t % kSiteLanes;
    for (int i = g; i < n1; i += kChunk / kSiteLanes) {
        double h[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int e = seg_i[i] + gl; e < seg_i[i + 1]; e += kSiteLanes) {
            const int q = lq[li[e]] >> 16;
            double rh[3], r;
            const SrPair<R> tp = k2_pair<R>(a, L, i, q, rc, rh, r);
            const double A_ = tp.A, B_ = tp.B, ab = L.qab[q];
            h[0] += ab * (A_ * rh[0] * rh[0] + B_);
            h[1] += ab * (A_ * rh[0] * rh[1]);
            h[2] += ab * (A_ * rh[0] * rh[2]);
            h[3] += ab * (A_ * rh[1] * rh[1] + B_);
            h[4] += ab * (A_ * rh[1] * rh[2]);
            h[5] += ab * (A_ * rh[2] * rh[2] + B_);
        }
#pragma unroll
        for (int m = 1; m < kSiteLanes; m <<= 1)
#pragma unroll
            for (int v = 0; v < 6; ++v) h[v] += __shfl_xor(h[v], m);
        if (gl == 0) {
            const double d[9] = {1.0 - h[0], -h[1], -h[2], -h[1], 1.0 - h[3], -h[4], -h[2], -h[4], 1.0 - h[5]};
            for (int e = 0; e < 9; ++e) D[(3 * i + e / 3) * 3 + e % 3] = d[e];
            for (int q = 0; q < 3; ++q)
                for (int c = 0; c < 3; ++c) Dt[(size_t)c * ld + 3 * i + q] = R(d[3 * q + c]);
        }
    }
}

// Assembly of the lower triangle of B~ (into the factor slot) by the workgroup
// of (atom, frequency) that then factorises it, pairs in triangle order in
// chunks of kChunk: the
// coupled pairs of a chunk (from the a-major list) are evaluated compactly,
// one per thread, into LDS; then each pair of the chunk is written by its own
// thread (rows of atom i in contiguous 3-element runs), zero blocks for
// uncoupled pairs.  The mixed path also keeps the FP32 pair coefficients for
// the refinement residual.
template <typename R>
__device__ __forceinline__ void assemble_matrix(const ScsArgs& a, int k, int w, int n1max, double* lds) {
    constexpr bool mixed = sizeof(R) == 4;
    const int t = threadIdx.x;
    const Counts cnt = a.counts[k];
    const int n1 = cnt.n1, n12 = cnt.n12, n2 = n12 - n1;
    const int N = 3 * n1;
    const int ld = a.fac_ld[k];
    const double rc = a.sinfo[a.atom_struct[k]].r_scs;
    ScsLds L = scs_assemble_lds(lds, n1max, 0, true);
    int32_t* slot = L.key;                                  // kChunk
    int32_t* wcnt = L.key + kChunk;                         // kChunk / 32
    uint32_t* mask = reinterpret_cast<uint32_t*>(L.key + 2 * kChunk);
    R* A = static_cast<R*>(a.fac) + a.fac_off[k] + (size_t)w * ld * (N + 3);
    const int npairs = n1 * (n1 + 1) / 2;
    float* coef = mixed ? a.coef + a.coef_off[k] + (size_t)w * 2 * npairs : nullptr;
    const int32_t* seg_a = pair_segs(a, k) + (n12 + 2);
    const int32_t* la = a.pl_i + a.pl_off[k] + (int64_t)n1 * n2;
    load_sites(a, k, w, n1, n1, L);
    for (int e = t; e < assemble_mask_words(n1); e += kChunk) mask[e] = 0u;
    __syncthreads();
    const int P11 = seg_a[n1];
    for (int e = t; e < P11; e += kChunk) {   // coupled K1 pairs (a < b) -> bit of lower-triangle pair (b, a)
        const int32_t ent = la[e];
        const int i = ent & 0xFFFF, j = ent >> 16;
        const int p = i * (i + 1) / 2 + j;
        atomicOr(&mask[p >> 5], 1u << (p & 31));
    }
    __syncthreads();
    for (int p0 = 0; p0 < npairs; p0 += kChunk) {
        const int w0 = p0 >> 5;
        if (t < kChunk / 32) wcnt[t] = (p0 + 32 * t < npairs) ? __popc(mask[w0 + t]) : 0;
        __syncthreads();
        int total = 0;
        for (int x = 0; x < kChunk / 32; ++x) total += wcnt[x];
        const int p = p0 + t;
        int rank = -1;
        if (p < npairs) {
            const int wd = p >> 5;
            const uint32_t m = mask[wd];
            if ((m >> (p & 31)) & 1u) {
                int r = __popc(m & ((1u << (p & 31)) - 1u));
                for (int x = w0; x < wd; ++x) r += wcnt[x - w0];
                rank = r;
                slot[r] = p;
            }
        }
        __syncthreads();
        // coupled pairs, compacted: T_SR and its block of B~
        if (t < total) {
            const int pp = slot[t];
            int i, j;
            tri_decode(pp, i, j);
            double rh[3], rr;
            const SrPair<R> tp = k1_pair<R>(a, L, i, j, rc, rh, rr);
            if (mixed) {
                coef[2 * pp] = (float)tp.A;
                coef[2 * pp + 1] = (float)tp.B;
            }
            const double Av = double(tp.A), Bv = double(tp.B);
            R* blk = A + (size_t)(3 * i) * ld + 3 * j;
            for (int q = 0; q < 3; ++q)
                for (int c = 0; c < 3; ++c) blk[(size_t)q * ld + c] = R(Av * rh[q] * rh[c] + (q == c ? Bv : 0.0));
        }
        // every other pair of the chunk: diagonal blocks and uncoupled zeros
        if (p < npairs && rank < 0) {
            int i, j;
            tri_decode(p, i, j);
            R* blk = A + (size_t)(3 * i) * ld + 3 * j;
            if (i == j) {
                const R inv = R(1.0 / L.ab[i]);
                for (int q = 0; q < 3; ++q)
                    for (int c = 0; c <= q; ++c) blk[(size_t)q * ld + c] = (q == c) ? inv : R(0);
            } else {
                for (int q = 0; q < 3; ++q)
                    for (int c = 0; c < 3; ++c) blk[(size_t)q * ld + c] = R(0);
            }
            if (mixed) { coef[2 * p] = 0.f; coef[2 * p + 1] = 0.f; }
        }
        // (no barrier here: the next chunk's first barrier separates these reads of
        // slot from its writes, and wcnt was last read before the barrier above)
    }
    __syncthreads();
}

// Triangular solves with the stored factor, one workgroup per (atom,
// frequency), NS rows per thread.  Right-hand side and result by mode:
//   kSolveD      : y = L^{-1} d (left by the factorisation) -> X (solution
//                  slot) and Tr(X_i)/3                                       [FP64]
//   kSolveFirst  : y = L^{-1} d -> X                                         [mixed]
//   kSolveCorr   : residual -> X += correction, then Tr(X_i)/3               [mixed]
//   kSolveLambda : Xbar_i = xbar_i I / 3 from the polarisability adjoints -> lambda
enum { kSolveD = 0, kSolveFirst = 1, kSolveCorr = 2, kSolveLambda = 3 };

template <typename R, int NS, int NP>
__device__ __forceinline__ void solve_slot(const ScsArgs& a, int k, int w, int n1max, int mode, double* lds) {
    const int n1 = a.counts[k].n1;
    const int N = 3 * n1;
    const int ld = a.fac_ld[k];
    const R* A = static_cast<const R*>(a.fac) + a.fac_off[k] + (size_t)w * ld * (N + 3);
    const size_t xo = a.x_off[k] + (size_t)w * N * 3;
    R* Y = reinterpret_cast<R*>(lds);
    R* zbuf = Y + 9 * n1max;
    if (mode == kSolveLambda) {
        const double* abl = a.abar_loc + a.aloc_off[k];
        for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) {
            const int s = e / 9, q = (e / 3) % 3, c = e % 3;
            double xb = abl[(size_t)s * a.nw + w];
            if (s == 0) xb += a.abar_cen[(size_t)k * a.nw + w];
            Y[e] = (q == c) ? R(xb / 3.0) : R(0);
        }
    } else if (mode == kSolveCorr) {
        for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) Y[e] = R(a.resid[xo + e]);
    } else {
        // the factorisation left y = L^{-1} d in the rows appended to B~
        for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) Y[e] = A[(size_t)(N + e % 3) * ld + e / 3];
    }
    __syncthreads();
    chol_solve3<R, NS, NP>(A, N, ld, Y, zbuf, mode == kSolveCorr || mode == kSolveLambda);
    if (mode == kSolveLambda) {
        for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) a.lam[xo + e] = double(Y[e]);
        return;
    }
    double* X = a.xsol + xo;
    for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) X[e] = (mode == kSolveCorr ? X[e] : 0.0) + double(Y[e]);
    if (mode == kSolveFirst) return;
    __syncthreads();
    double* al = a.alpha_loc + a.aloc_off[k];
    for (int s = threadIdx.x; s < n1; s += blockDim.x)
        al[(size_t)s * a.nw + w] = (X[(3 * s) * 3 + 0] + X[(3 * s + 1) * 3 + 1] + X[(3 * s + 2) * 3 + 2]) / 3.0;
}

// The standalone solves (adjoint lambda; correction of the mixed path): two
// rows per thread, 256 threads, the first slot loading a block ahead.  Against
// one row per thread in 512-thread workgroups this keeps three workgroups on a
// compute unit instead of two (more independent block chains, more loads in
// flight): 3.45 -> 3.19 ms for the FP64 lambda solve of 1,728 C atoms.
// Systems of more than 2 x 256 rows (K1 above 170 sites, e.g. r_SCS = 8 A at carbon
// density) take three rows per thread; the rows' sums are the same either way.
constexpr int kSolveThreads = 256;
static_assert(3 * kSolveThreads >= 3 * kMaxN1, "three rows per thread cover the largest system");
__host__ __device__ inline int solve_slots(int n1max) { return 3 * n1max <= 2 * kSolveThreads ? 2 : 3; }
template <typename R, int NS>
__global__ void __launch_bounds__(kSolveThreads, NS == 2 ? 3 : 2) k_scs_solve(ScsArgs a, int n1max, int mode) {
    extern __shared__ double lds[];
    solve_slot<R, NS, 1>(a, a.order[blockIdx.x], blockIdx.y, n1max, mode, lds);
}

size_t scs_solve_lds_bytes(int n1max, bool mixed) {
    const size_t r = mixed ? sizeof(float) : sizeof(double);
    return r * (9 * (size_t)n1max + 2 * NB * kSlotLd);
}

// Refinement residual of the mixed path: resid = d - B~ X in FP64, with B~
// rebuilt from its FP32 pair coefficients; partner ranges split over kRes
// threads and recombined in a fixed order.
__device__ __forceinline__ void residual_slot(const ScsArgs& a, int k, int w, int n1max, double* lds) {
    constexpr int kRes = 2;
    const int n1 = a.counts[k].n1;
    const int N = 3 * n1;
    const size_t xo = a.x_off[k] + (size_t)w * N * 3;
    double* X = lds;
    double* px = X + 9 * n1max;
    double* py = px + n1max;
    double* pz = py + n1max;
    double* ab = pz + n1max;
    double* red = ab + n1max;   // kRes * n1max * 9
    const Site* S = a.sites + a.site_off[k];
    for (int s = threadIdx.x; s < n1; s += blockDim.x) {
        px[s] = S[s].x;
        py[s] = S[s].y;
        pz[s] = S[s].z;
        ab[s] = a.abar[(size_t)S[s].base * a.nw + w];
    }
    for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) X[e] = a.xsol[xo + e];
    const int npairs = n1 * (n1 + 1) / 2;
    const float* coef = a.coef + a.coef_off[k] + (size_t)w * 2 * npairs;
    __syncthreads();
    for (int t = threadIdx.x; t < n1 * kRes; t += blockDim.x) {
        const int i = t % n1, part = t / n1;
        double acc[9] = {};
        for (int j = part; j < n1; j += kRes) {
            if (j == i) continue;
            const int pj = i > j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
            const double cA = coef[2 * pj], cB = coef[2 * pj + 1];
            if (cA == 0.0 && cB == 0.0) continue;
            const double v[3] = {px[i] - px[j], py[i] - py[j], pz[i] - pz[j]};
            const double ir = rsqrt_refined(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);   // (a few ulp: far below the FP32 coefficients' error)
            const double rh[3] = {v[0] * ir, v[1] * ir, v[2] * ir};
            for (int c = 0; c < 3; ++c) {
                const double x0 = X[(3 * j + 0) * 3 + c], x1 = X[(3 * j + 1) * 3 + c], x2 = X[(3 * j + 2) * 3 + c];
                const double rx = rh[0] * x0 + rh[1] * x1 + rh[2] * x2;
                acc[0 * 3 + c] += cA * rh[0] * rx + cB * x0;
                acc[1 * 3 + c] += cA * rh[1] * rx + cB * x1;
                acc[2 * 3 + c] += cA * rh[2] * rx + cB * x2;
            }
        }
        for (int e = 0; e < 9; ++e) red[(size_t)(part * n1 + i) * 9 + e] = acc[e];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n1; i += blockDim.x) {
        for (int e = 0; e < 9; ++e) {
            const int idx = (3 * i + e / 3) * 3 + e % 3;
            double r = a.dvec[xo + idx] - X[idx] / ab[i];
            for (int part = 0; part < kRes; ++part) r -= red[(size_t)(part * n1 + i) * 9 + e];
            a.resid[xo + idx] = r;
        }
    }
}

static size_t scs_residual_lds_bytes(int n1max) { return sizeof(double) * (9 * (size_t)n1max + 4 * (size_t)n1max + 2 * 9 * (size_t)n1max); }

// Assembly, factorisation and first solve of B~ in place, one workgroup per
// (atom, frequency): the matrix written just before it is read back stays in
// the caches, as does the factor for the solve (and, in the mixed path, for the
// correction solve of the refinement), and the write-bound assembly of one
// workgroup overlaps the factorisations of the others on the compute unit.
// The diagonal tile and the k-split parts are dynamic LDS (the assembly, the
// solves and the residual use the same space before and after); Z1, Z2 and L21 are a separate
// static array so that the compiler sees they cannot alias it.
static_assert(kChunk == 256, "the 256 threads of the factorisation kernel run the assembly's chunks");
static_assert(3 * 256 >= 3 * kMaxN1, "three rows per thread of the factorisation kernel cover its first solve");
static_assert(256 / 64 - 1 <= kMaxParts, "k-split parts of four wavefronts");
template <typename R, int NS>
__global__ void __launch_bounds__(256, NS == 2 ? 3 : 2) k_scs_factor(ScsArgs a, int n1max) {
    extern __shared__ double lds[];
    __shared__ R Zsh[3 * NB * kSlotLd];
    __shared__ int ctl[4];
    R* Lt = reinterpret_cast<R*>(lds);
    const int k = a.order[blockIdx.x];
    const int w = blockIdx.y;
    assemble_matrix<R>(a, k, w, n1max, lds);   // ends with a barrier
    const int N = 3 * a.counts[k].n1;
    const int ld = a.fac_ld[k];
    R* A = static_cast<R*>(a.fac) + a.fac_off[k] + (size_t)w * ld * (N + 3);
    // the wave that factorises the diagonal blocks rotates over the workgroups
    const int dw = (k + w) % (blockDim.x >> 6);
    bool ok = true, stalled = false;
    R* part = Lt + NB * kSlotLd;
    chol_factor<R>(A, N, ld, Lt, part, part + kMaxParts * 16 * 64, Zsh, Zsh + NB * kSlotLd, Zsh + 2 * NB * kSlotLd,
                   ctl, dw, ok, stalled);   // ends with a barrier
    if (!ok && (threadIdx.x & 63) == 0) {   // only lanes of the diagonal wave can fail
        atomicOr(a.err, 4);
        atomicMin(a.err_atom, k);
    }
    if (stalled && (threadIdx.x & 63) == 0) {
        atomicOr(a.err, 64);
        atomicMin(a.err_atom, k);
    }
    // the first solve (backward: the forward substitution was carried by the
    // factorisation) while the factor is still in the caches
    solve_slot<R, NS, 1>(a, k, w, n1max, sizeof(R) == 4 ? kSolveFirst : kSolveD, lds);
    if constexpr (sizeof(R) == 4) {
        // the mixed path's refinement in the same launch, the FP32 factor still in
        // the caches for the correction solve
        for (int it = 0; it < a.n_refine; ++it) {
            __syncthreads();   // X written; the LDS of the solve free
            residual_slot(a, k, w, n1max, lds);
            __syncthreads();   // the residual written
            solve_slot<R, NS, 1>(a, k, w, n1max, kSolveCorr, lds);
        }
    }
}

// dynamic LDS of the factorisation: the diagonal tile, the k-split parts and the two
// buffers of the prepared unit 0
static size_t factor_panel_bytes(bool mixed) {
    const size_t r = mixed ? sizeof(float) : sizeof(double);
    return r * ((size_t)NB * kSlotLd + (size_t)(kMaxParts + 2) * 16 * 64);
}

// dynamic LDS of the assembly and factorisation kernel
static size_t factor_dynamic_bytes(int n1max, bool mixed) {
    const size_t solve = scs_solve_lds_bytes(n1max, mixed);
    return std::max(std::max(factor_panel_bytes(mixed), matrix_lds_bytes(n1max)),
                    mixed ? std::max(solve, scs_residual_lds_bytes(n1max)) : solve);
}

// all LDS of the assembly and factorisation: the dynamic part and Z1, Z2, L21
size_t scs_factor_lds_bytes(int n1max, bool mixed) {
    const size_t r = mixed ? sizeof(float) : sizeof(double);
    return factor_dynamic_bytes(n1max, mixed) + r * 3 * NB * kSlotLd;
}


// ---------------------------------------------------------------------------
// Adjoint.  With X = B~^{-1} d and seeds xbar_i (adjoint of alpha~_iso_i =
// Tr X_i / 3): lambda = B~^{-1} Xbar with Xbar_i = xbar_i I / 3, then
//   dE = -<lambda X^T, dB~> + <lambda, dd>.
// Each coupled pair is evaluated once: the gradient of its term with respect
// to the first site is h, with respect to the second -h.  The pairs are taken
// in chunks of one per thread; h goes to LDS, the first sites' sums are formed
// over the runs of equal first site in the chunk (by the run's first thread),
// and each K1 site's thread walks its index list over the other side.  Sums
// are thus formed in a fixed order, independent of scheduling.  The mixed path
// solves for lambda in FP32 and evaluates the pair-tensor derivatives in FP32;
// contractions and sums are FP64.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(kChunk, 3) k_scs_adjoint(ScsArgs a, int n1max, int n2max) {
    extern __shared__ double lds[];
    const int k = a.order[blockIdx.x];
    const int w = blockIdx.y;
    const int t = threadIdx.x;
    const Counts cnt = a.counts[k];
    const int n1 = cnt.n1, n12 = cnt.n12, n2 = n12 - n1, nall = cnt.n_all;
    const int N = 3 * n1;
    const StructInfo& SI = a.sinfo[a.atom_struct[k]];
    const double rc = SI.r_scs;
    ScsLds L = scs_lds(lds, n1max, n2max);
    const double* Xg = a.xsol + a.x_off[k] + (size_t)w * N * 3;
    const double* Lg = a.lam + a.x_off[k] + (size_t)w * N * 3;
    load_sites(a, k, w, n1, n1, L);   // the shell sites follow once X is no longer needed
    for (int e = t; e < 3 * N; e += kChunk) {
        L.X[e] = Xg[e];
        L.Y[e] = Lg[e];
    }
    // this (atom, frequency)'s slice of the contributions: the per-site sums are
    // formed in it (K1 sites gk, then shell sites gq), then scaled to forces
    double* out = a.cf + (size_t)w * a.cf_slice + a.site_off[k] * 3;
    double* gk = out;
    double* gq = out + 3 * n1;
    for (int e = t; e < 3 * n12; e += kChunk) out[e] = 0.0;
    const int32_t* seg = pair_segs(a, k);
    const int32_t* seg_i = seg;
    const int32_t* seg_q = seg + (n1 + 1);
    const int32_t* seg_a = seg + (n12 + 2);
    const int32_t* seg_b = seg + (n12 + n1 + 3);
    const int32_t* li = a.pl_i + a.pl_off[k];
    const int32_t* lq = a.pl_q + a.pl_off[k];
    const int32_t* la = li + (int64_t)n1 * n2;
    const int32_t* lb = lq + (int64_t)n1 * n2;
    __syncthreads();

    __shared__ double carry[3 * kChunkWaves];
    __shared__ int carry_key[kChunkWaves];
    // K1 site's index list over the other side, walked by ws threads (entries
    // part, part + ws, ...; two per site when n1 <= kChunk / 2): the next
    // entries are loaded before the chunk's pair is evaluated, and the terms of
    // the pairs in this chunk are subtracted from g after the barrier
    const int ws = 2 * n1 <= kChunk ? 2 : 1;
    const int site = t / ws, part = t % ws;
    const bool walker = site < n1;
    constexpr int kAhead = 8;
    int ahead[kAhead];
    auto prefetch = [&](const int32_t* lst, int p, int pe) {
#pragma unroll
        for (int j = 0; j < kAhead; ++j) ahead[j] = p + j * ws < pe ? lst[p + j * ws] : 0x7fffffff;
    };
    auto consume = [&](const int32_t* lst, int& p, int pe, int e1, double* g) {
        bool more = true;
#pragma unroll
        for (int j = 0; j < kAhead; ++j) {
            more = more && ahead[j] < e1;
            if (more) {
                const int u = ahead[j] - (e1 - kChunk);
                g[0] -= L.H[3 * u + 0];
                g[1] -= L.H[3 * u + 1];
                g[2] -= L.H[3 * u + 2];
                p += ws;
            }
        }
        if (more) {
            for (; p < pe && lst[p] < e1; p += ws) {
                const int u = lst[p] - (e1 - kChunk);
                g[0] -= L.H[3 * u + 0];
                g[1] -= L.H[3 * u + 1];
                g[2] -= L.H[3 * u + 2];
            }
        }
    };

    double gb[3] = {0.0, 0.0, 0.0};   // the walked K1 site as the second site of K1 x K1 pairs
    double gi[3] = {0.0, 0.0, 0.0};   // the walked K1 site against the shell
    // K1 x K1 pairs a < b: h = gradient of the pair's term with respect to r_a
    {
        const int P = seg_a[n1];
        int p = walker ? seg_b[site] + part : 0;
        const int pe = walker ? seg_b[site + 1] : 0;
        int32_t ent_next = t < P ? la[t] : 0;   // list entries a chunk ahead
        for (int e0 = 0; e0 < P; e0 += kChunk) {
            prefetch(lb, p, pe);
            const int e = e0 + t;
            const int32_t ent = ent_next;
            if (e + kChunk < P) ent_next = la[e + kChunk];
            int key = -1;
            double h[3] = {0.0, 0.0, 0.0};
            if (e < P) {
                const int i = ent >> 16, j = ent & 0xFFFF;
                key = i;
                double rh[3], r;
                const SrPair<R> tp = k1_pair<R>(a, L, i, j, rc, rh, r);
                const double* Xi = L.X + 9 * i;
                const double* Yi = L.Y + 9 * i;
                const double* Xj = L.X + 9 * j;
                const double* Yj = L.Y + 9 * j;
                double Cs[9];
                for (int q = 0; q < 3; ++q)
                    for (int c = q; c < 3; ++c) {
                        double s1 = 0.0, s2 = 0.0;
                        for (int m = 0; m < 3; ++m) {
                            s1 += Yi[3 * q + m] * Xj[3 * c + m] + Yi[3 * c + m] * Xj[3 * q + m];
                            s2 += Xi[3 * q + m] * Yj[3 * c + m] + Xi[3 * c + m] * Yj[3 * q + m];
                        }
                        Cs[3 * q + c] = -0.5 * (s1 + s2);
                        Cs[3 * c + q] = Cs[3 * q + c];
                    }
                radial_tensor_grad(rh, r, double(tp.A), double(tp.dA), double(tp.dB), Cs, h);
            }
            L.key[t] = key;
            L.H[3 * t + 0] = h[0];
            L.H[3 * t + 1] = h[1];
            L.H[3 * t + 2] = h[2];
            __syncthreads();
            run_sums<3>(key, h, L.key, gk, carry, carry_key);
            if (walker) consume(lb, p, pe, e0 + kChunk, gb);
            __syncthreads();
            add_carries<3>(gk, carry, carry_key);
        }
    }
    __syncthreads();   // X is no longer needed: the shell sites take its space
    load_sites(a, k, w, n1, n12, L, n1);
    __syncthreads();
    // K1 x shell pairs, shell-major: h = qab_q * (gradient of the lambda_i : dd_i
    // term with respect to r_i); the shell site gains h, the K1 site loses it
    {
        const int P = seg_q[n2];
        int p = walker ? seg_i[site] + part : 0;
        const int pe = walker ? seg_i[site + 1] : 0;
        int32_t ent_next = t < P ? lq[t] : 0;   // list entries a chunk ahead
        for (int e0 = 0; e0 < P; e0 += kChunk) {
            prefetch(li, p, pe);
            const int e = e0 + t;
            const int32_t ent = ent_next;
            if (e + kChunk < P) ent_next = lq[e + kChunk];
            int key = -1;
            double h[3] = {0.0, 0.0, 0.0};
            if (e < P) {
                const int q = ent >> 16, i = ent & 0xFFFF;
                key = q;
                double rh[3], r;
                const SrPair<R> tp = k2_pair<R>(a, L, i, q, rc, rh, r);
                const double* Yi = L.Y + 9 * i;
                double lam[9];
                for (int e2 = 0; e2 < 3; ++e2)
                    for (int c = 0; c < 3; ++c) lam[3 * e2 + c] = 0.5 * (Yi[3 * e2 + c] + Yi[3 * c + e2]);
                double gp[3];
                radial_tensor_grad(rh, r, double(tp.A), double(tp.dA), double(tp.dB), lam, gp);
                const double ab = L.qab[q];
                h[0] = ab * gp[0];
                h[1] = ab * gp[1];
                h[2] = ab * gp[2];
            }
            L.key[t] = key;
            L.H[3 * t + 0] = h[0];
            L.H[3 * t + 1] = h[1];
            L.H[3 * t + 2] = h[2];
            __syncthreads();
            run_sums<3>(key, h, L.key, gq, carry, carry_key);
            if (walker) consume(li, p, pe, e0 + kChunk, gi);
            __syncthreads();
            add_carries<3>(gq, carry, carry_key);
        }
    }
    __syncthreads();

    const double fconv = -1.0 / kBohr;  // force = -dE/dx, per Angstrom
    if (ws == 2) {   // the two walkers of a site are adjacent lanes
        for (int c = 0; c < 3; ++c) {
            gb[c] += __shfl_xor(gb[c], 1);
            gi[c] += __shfl_xor(gi[c], 1);
        }
    }
    if (walker && part == 0) {
        for (int c = 0; c < 3; ++c) out[3 * site + c] = fconv * ((gk[3 * site + c] + gb[c]) + gi[c]);
    }
    for (int q = t; q < n2; q += kChunk)
        for (int c = 0; c < 3; ++c) gq[3 * q + c] = fconv * gq[3 * q + c];
    for (int s = n12 + t; s < nall; s += kChunk)
        for (int c = 0; c < 3; ++c) out[3 * s + c] = 0.0;
}

// ---------------------------------------------------------------------------
// Adjoint of the Hirshfeld-volume ratios.  nu_b enters the local SCS system
// through the TS values of its sites (Sec. II.B): abar = alpha0 nu / (1 +
// (w/w_i)^2), sigma = (sqrt(2/pi) abar / 3)^(1/3) and R = R0 nu^(1/3), so
//   nu_b dE/dnu_b = sum over the sites s of b, in every frame and frequency, of
//   g_s = abar_s Abar_s + sigma_s Sbar_s / 3 + R_s Rbar_s / 3,
// with Abar, Sbar, Rbar the adjoints of the site's abar, sigma and R.  With
// lambda and X as in the force adjoint (B~ X = d, B~ lambda = Xbar):
//   diagonal 1/abar_i of B~:           Abar_i += <lambda_i, X_i> / abar_i^2
//   K1 pair T_SR(i, j) in B~:          with C the pair's adjoint contraction,
//       sbar = <C, dT/ds>, Sbar = <C, dT/dS> (s = sqrt(sigma_i^2 + sigma_j^2),
//       S = beta (R_i + R_j));         Sbar_i += sbar sigma_i / s, Rbar_i += beta Sbar
//   shell pair T_SR(i, q) abar_q in d: Abar_q -= <lambda_i, T>, and the same
//       sigma/R terms with C = -abar_q sym(lambda_i).
// One thread per site of the frame (K1 sites, then shell sites) forms its g_s
// from its own pair lists in list order, so the sums have a fixed order.
// Evaluated in FP64 on both paths.
// ---------------------------------------------------------------------------
struct SrPairNu {
    double A, B;     // T = A rhat rhat^T + B I
    double As, Bs;   // dT/ds
    double AS, BS;   // dT/dS
};

__device__ inline SrPairNu sr_pair_nu(double r, double s, double S, double damp_d, double rc, double rb, double wmul) {
    const double c = kTwoOverSqrtPi;
    const double u = r / s;
    const double e = exp(-u * u);
    const double g = erf(u) - c * u * e;
    const double ir3 = 1.0 / (r * r * r);
    const double u3e = u * u * u * e;
    const double Ac = -(3.0 * g - 2.0 * c * u3e) * ir3, Bc = g * ir3;
    // d/ds at fixed r (u = r/s): dA/ds = 4 c u^5 e / (s r^3), dB/ds = -2 c u^3 e / (s r^3)
    const double Acs = 4.0 * c * u3e * u * u * ir3 / s, Bcs = -2.0 * c * u3e * ir3 / s;
    double dfdr, dfdS, dcut;
    const double f = fermi<double>(r, S, damp_d, dfdr, dfdS);
    const double fc = cutoff_poly<double>(r, rc, rb, dcut);
    const double w = wmul * fc * (1.0 - f), wS = -wmul * fc * dfdS;
    return SrPairNu{w * Ac, w * Bc, w * Acs, w * Bcs, wS * Ac, wS * Bc};
}

// <C, a rhat rhat^T + b I> for a symmetric C
__device__ inline double radial_contract(const double C[9], const double rh[3], double a, double b) {
    double rCr = 0.0;
    for (int q = 0; q < 3; ++q)
        for (int m = 0; m < 3; ++m) rCr += rh[q] * C[3 * q + m] * rh[m];
    return a * rCr + b * (C[0] + C[4] + C[8]);
}

__global__ void __launch_bounds__(256) k_scs_nu(ScsArgs a, int n1max, int n2max) {
    extern __shared__ double lds[];
    const int k = a.order[blockIdx.x];
    const int w = blockIdx.y;
    const Counts cnt = a.counts[k];
    const int n1 = cnt.n1, n12 = cnt.n12, n2 = n12 - n1, nall = cnt.n_all;
    const int N = 3 * n1;
    const double rc = a.sinfo[a.atom_struct[k]].r_scs;
    ScsLds L = scs_assemble_lds(lds, n1max, n2max, false);
    const double* X = a.xsol + a.x_off[k] + (size_t)w * N * 3;
    const double* Y = a.lam + a.x_off[k] + (size_t)w * N * 3;
    const int32_t* seg = pair_segs(a, k);
    const int32_t* seg_i = seg;
    const int32_t* seg_q = seg + (n1 + 1);
    const int32_t* seg_a = seg + (n12 + 2);
    const int32_t* seg_b = seg + (n12 + n1 + 3);
    const int32_t* li = a.pl_i + a.pl_off[k];
    const int32_t* lq = a.pl_q + a.pl_off[k];
    const int32_t* la = li + (int64_t)n1 * n2;
    const int32_t* lb = lq + (int64_t)n1 * n2;
    double* out = a.cnu + a.site_off[k] * a.nw + w;
    load_sites(a, k, w, n1, n12, L);
    __syncthreads();
    // sbar and Sbar of one pair to the sigma/R part of a site's g
    auto sr_share = [&](double sig, double Rs, double s, double sbar, double Sbar) {
        return sbar * sig * sig / (3.0 * s) + a.beta * Sbar * Rs / 3.0;
    };
    for (int t = threadIdx.x; t < nall; t += blockDim.x) {
        double g = 0.0;
        if (t < n1) {
            const int i = t;
            double Xi[9], Yi[9], lam[9];
            for (int e = 0; e < 9; ++e) {
                Xi[e] = X[9 * i + e];
                Yi[e] = Y[9 * i + e];
            }
            double yx = 0.0;
            for (int e = 0; e < 9; ++e) yx += Yi[e] * Xi[e];
            g += yx / L.ab[i];
            // K1 x K1 pairs (i, j): first those with i < j (i's run of the a-major list,
            // whose majors are in scrambled order, so the run ends where the major
            // changes), then those with j < i (i's segment of the b-side index list)
            for (int side = 0; side < 2; ++side) {
                const int pb = side == 0 ? seg_a[i] : seg_b[i], pe = side == 0 ? seg_a[n1] : seg_b[i + 1];
                for (int p = pb; p < pe; ++p) {
                    if (side == 0 && (la[p] >> 16) != i) break;
                    const int32_t ent = side == 0 ? la[p] : la[lb[p]];
                    const int j = side == 0 ? (ent & 0xFFFF) : (ent >> 16);
                    const double v[3] = {L.px[i] - L.px[j], L.py[i] - L.py[j], L.pz[i] - L.pz[j]};
                    const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                    const double rh[3] = {v[0] / r, v[1] / r, v[2] / r};
                    const double s = sqrt(L.sg[i] * L.sg[i] + L.sg[j] * L.sg[j]);
                    const SrPairNu tp = sr_pair_nu(r, s, a.beta * (L.R[i] + L.R[j]), a.damp_d, rc, a.r_buf, 1.0);
                    double C[9];
                    for (int q = 0; q < 3; ++q)
                        for (int c = 0; c < 3; ++c) {
                            double s1 = 0.0;
                            for (int m = 0; m < 3; ++m)
                                s1 += Yi[3 * q + m] * X[9 * j + 3 * c + m] + Yi[3 * c + m] * X[9 * j + 3 * q + m] +
                                      Xi[3 * q + m] * Y[9 * j + 3 * c + m] + Xi[3 * c + m] * Y[9 * j + 3 * q + m];
                            C[3 * q + c] = -0.5 * s1;
                        }
                    g += sr_share(L.sg[i], L.R[i], s, radial_contract(C, rh, tp.As, tp.Bs),
                                  radial_contract(C, rh, tp.AS, tp.BS));
                }
            }
            // K1 x shell pairs (i, q)
            for (int e = 0; e < 3; ++e)
                for (int c = 0; c < 3; ++c) lam[3 * e + c] = 0.5 * (Yi[3 * e + c] + Yi[3 * c + e]);
            for (int p = seg_i[i]; p < seg_i[i + 1]; ++p) {
                const int q = lq[li[p]] >> 16;
                const double v[3] = {L.px[i] - L.qx[q], L.py[i] - L.qy[q], L.pz[i] - L.qz[q]};
                const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                const double rh[3] = {v[0] / r, v[1] / r, v[2] / r};
                const double s = sqrt(L.sg[i] * L.sg[i] + L.qsg[q] * L.qsg[q]);
                double fin, dfin;
                inner_buffer(r, a.r_inner, fin, dfin);
                const SrPairNu tp = sr_pair_nu(r, s, a.beta * (L.R[i] + L.qR[q]), a.damp_d, rc, a.r_buf, fin);
                const double m = -L.qab[q];
                g += sr_share(L.sg[i], L.R[i], s, m * radial_contract(lam, rh, tp.As, tp.Bs),
                              m * radial_contract(lam, rh, tp.AS, tp.BS));
            }
        } else if (t < n12) {
            const int q = t - n1;
            // q's run of the shell-major list (majors in scrambled order: the run ends
            // where the major changes)
            for (int p = seg_q[q]; p < seg_q[n2] && (lq[p] >> 16) == q; ++p) {
                const int i = lq[p] & 0xFFFF;
                const double v[3] = {L.px[i] - L.qx[q], L.py[i] - L.qy[q], L.pz[i] - L.qz[q]};
                const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                const double rh[3] = {v[0] / r, v[1] / r, v[2] / r};
                const double s = sqrt(L.sg[i] * L.sg[i] + L.qsg[q] * L.qsg[q]);
                double fin, dfin;
                inner_buffer(r, a.r_inner, fin, dfin);
                const SrPairNu tp = sr_pair_nu(r, s, a.beta * (L.R[i] + L.qR[q]), a.damp_d, rc, a.r_buf, fin);
                double lam[9];
                for (int e = 0; e < 3; ++e)
                    for (int c = 0; c < 3; ++c) lam[3 * e + c] = 0.5 * (Y[9 * i + 3 * e + c] + Y[9 * i + 3 * c + e]);
                const double m = -L.qab[q];
                g += -L.qab[q] * radial_contract(lam, rh, tp.A, tp.B);   // abar_q Abar_q
                g += sr_share(L.qsg[q], L.qR[q], s, m * radial_contract(lam, rh, tp.As, tp.Bs),
                              m * radial_contract(lam, rh, tp.AS, tp.BS));
            }
        }
        out[(size_t)t * a.nw] = g;   // sites beyond the SCS shell take no share
    }
}

// ---------------------------------------------------------------------------
// Pair lists of one atom (frequency independent).  A shell site q couples to a
// K1 site i when r_iq < r_scs, two K1 sites a < b when r_ab < r_scs (beyond,
// f_SR vanishes).  Each coupling appears once; the second list of each kind
// holds, per minor site, the indices of its pairs in the first list, so that a
// pass over one list can also reduce over the other side without atomics.
// The shell-major and a-major lists take their major sites in a scrambled
// order (a fixed stride coprime with the count), so that a site's pairs on the
// other side spread evenly over any run of the list instead of clustering in
// the part where spatially close sites sit.  All orders are deterministic (one
// thread per major index, minors ascending).
// ---------------------------------------------------------------------------
__device__ inline int gcd_int(int x, int y) {
    while (y) { const int r = x % y; x = y; y = r; }
    return x;
}

// stride of the scrambled order of n items: about 0.618 n, coprime with n
__device__ inline int scramble_stride(int n) {
    if (n <= 2) return 1;
    int s = (int)(0.6180339887 * n);
    if (s < 1) s = 1;
    while (gcd_int(s, n) != 1) ++s;
    return s;
}

// LDS of the pair-list kernel: positions, then coupling bit rows: per K1 site
// over the shell in scrambled order (wq words) and over K1 (a > i natural,
// a < i scrambled; wa words each), per shell site over K1 (wa words), then
// counts and offsets
struct PairlistLds {
    double *px, *py, *pz, *qx, *qy, *qz;
    uint32_t *bq, *na, *nb, *cq;
    int32_t *cnt_i, *cnt_q, *cnt_a, *cnt_b;
    int wq, wa;
};

__host__ __device__ inline size_t pairlist_lds_words(int n1max, int n2max) {
    const size_t wq = (n2max + 31) / 32, wa = (n1max + 31) / 32;
    return (size_t)n1max * wq + 2 * (size_t)n1max * wa + (size_t)n2max * wa + 3 * ((size_t)n1max + 1) +
           ((size_t)n2max + 1);
}

__device__ inline PairlistLds pairlist_lds(double* base, int n1max, int n2max) {
    PairlistLds L;
    L.px = base;
    L.py = L.px + n1max;
    L.pz = L.py + n1max;
    L.qx = L.pz + n1max;
    L.qy = L.qx + n2max;
    L.qz = L.qy + n2max;
    L.wq = (n2max + 31) / 32;
    L.wa = (n1max + 31) / 32;
    L.bq = reinterpret_cast<uint32_t*>(L.qz + n2max);
    L.na = L.bq + (size_t)n1max * L.wq;
    L.nb = L.na + (size_t)n1max * L.wa;
    L.cq = L.nb + (size_t)n1max * L.wa;
    L.cnt_i = reinterpret_cast<int32_t*>(L.cq + (size_t)n2max * L.wa);
    L.cnt_q = L.cnt_i + (n1max + 1);
    L.cnt_a = L.cnt_q + (n2max + 1);
    L.cnt_b = L.cnt_a + (n1max + 1);
    return L;
}

// number of set bits of a bit row below position x
__device__ inline int bits_below(const uint32_t* row, int x) {
    int c = 0;
    for (int w = 0; w < (x >> 5); ++w) c += __popc(row[w]);
    if (x & 31) c += __popc(row[x >> 5] & ((1u << (x & 31)) - 1u));
    return c;
}

__global__ void __launch_bounds__(256) k_pairlist(ScsArgs a, int n1max, int n2max) {
    extern __shared__ double lds[];
    const int k = a.order[blockIdx.x];
    const int t = threadIdx.x, nt = blockDim.x;
    const Counts cnt = a.counts[k];
    const int n1 = cnt.n1, n12 = cnt.n12, n2 = n12 - n1;
    const StructInfo& SI = a.sinfo[a.atom_struct[k]];
    const double rc2 = SI.r_scs * SI.r_scs;
    PairlistLds L = pairlist_lds(lds, n1max, n2max);
    const int wq = L.wq, wa = L.wa;
    const Site* S = a.sites + a.site_off[k];
    for (int s = t; s < n12; s += nt) {
        if (s < n1) { L.px[s] = S[s].x; L.py[s] = S[s].y; L.pz[s] = S[s].z; }
        else { L.qx[s - n1] = S[s].x; L.qy[s - n1] = S[s].y; L.qz[s - n1] = S[s].z; }
    }
    const int nwords = n1max * wq + 2 * n1max * wa + n2max * wa;
    for (int e = t; e < nwords; e += nt) L.bq[e] = 0u;
    __syncthreads();
    const int sq = scramble_stride(n2), sa = scramble_stride(n1);
    // every coupling tested once: K1 x shell (i, x = scrambled shell position,
    // q = x sq mod n2); e = i n2 + x advances by nt, and i, x and q follow it
    // by additions (x sq mod n2 does not change when x wraps by n2)
    if (n2 > 0) {
        int i = t / n2, x = t % n2;
        int q = (int)(((int64_t)x * sq) % n2);
        const int dq = (int)(((int64_t)(nt % n2) * sq) % n2), di = nt / n2, dx0 = nt % n2;
        for (int e = t; e < n1 * n2; e += nt) {
            const double dx = L.px[i] - L.qx[q], dy = L.py[i] - L.qy[q], dz = L.pz[i] - L.qz[q];
            if (dx * dx + dy * dy + dz * dz < rc2) {
                atomicOr(&L.bq[(size_t)i * wq + (x >> 5)], 1u << (x & 31));
                atomicOr(&L.cq[(size_t)q * wa + (i >> 5)], 1u << (i & 31));
            }
            i += di;
            x += dx0;
            q += dq;
            if (q >= n2) q -= n2;
            if (x >= n2) {
                x -= n2;
                ++i;
            }
        }
    }
    // K1 x K1 (i, x = scrambled K1 position of j): j > i in natural order for
    // i's a-major entries, j < i in scrambled order for i's b-side list
    int ii = t / n1, xx = t % n1;
    int jj = (int)(((int64_t)xx * sa) % n1);
    const int dj = (int)(((int64_t)(nt % n1) * sa) % n1), dii = nt / n1, dxx = nt % n1;
    for (int e = t; e < n1 * n1; e += nt) {
        const int i = ii, x = xx, j = jj;
        ii += dii;
        xx += dxx;
        jj += dj;
        if (jj >= n1) jj -= n1;
        if (xx >= n1) {
            xx -= n1;
            ++ii;
        }
        if (j == i) continue;
        const double dx = L.px[i] - L.px[j], dy = L.py[i] - L.py[j], dz = L.pz[i] - L.pz[j];
        if (dx * dx + dy * dy + dz * dz < rc2) {
            if (j > i) atomicOr(&L.na[(size_t)i * wa + (j >> 5)], 1u << (j & 31));
            else atomicOr(&L.nb[(size_t)i * wa + (x >> 5)], 1u << (x & 31));
        }
    }
    __syncthreads();
    for (int i = t; i < n1; i += nt) {
        int ci = 0, ca = 0, cb = 0;
        for (int w = 0; w < wq; ++w) ci += __popc(L.bq[(size_t)i * wq + w]);
        for (int w = 0; w < wa; ++w) {
            ca += __popc(L.na[(size_t)i * wa + w]);
            cb += __popc(L.nb[(size_t)i * wa + w]);
        }
        L.cnt_i[i] = ci;
        L.cnt_a[i] = ca;
        L.cnt_b[i] = cb;
    }
    for (int q = t; q < n2; q += nt) {
        int c = 0;
        for (int w = 0; w < wa; ++w) c += __popc(L.cq[(size_t)q * wa + w]);
        L.cnt_q[q] = c;
    }
    __syncthreads();
    int32_t* seg = pair_segs(a, k);
    // exclusive prefix sums, one thread per list, into LDS and the segment
    // table (i, q, a, b); q and a in their scrambled order, with the total last
    {
        int32_t* c = nullptr;
        int len = 0, at = 0, stride = 1;
        switch (t) {
            case 0: c = L.cnt_i; len = n1; at = 0; break;
            case 64: c = L.cnt_q; len = n2; at = n1 + 1; stride = sq; break;
            case 128: c = L.cnt_a; len = n1; at = n12 + 2; stride = sa; break;
            case 192: c = L.cnt_b; len = n1; at = n12 + n1 + 3; break;
            default: break;
        }
        if (c) {
            int acc = 0;
            for (int x = 0, y = 0; x < len; ++x) {   // y = x stride mod len
                const int v = c[y];
                c[y] = acc;
                seg[at + y] = acc;
                acc += v;
                y += stride;
                if (y >= len) y -= len;
            }
            c[len] = acc;
            seg[at + len] = acc;
        }
    }
    __syncthreads();
    int32_t* li = const_cast<int32_t*>(a.pl_i) + a.pl_off[k];
    int32_t* lq = const_cast<int32_t*>(a.pl_q) + a.pl_off[k];
    int32_t* la = li + (int64_t)n1 * n2;
    int32_t* lb = lq + (int64_t)n1 * n2;
    // list entries, one (major site, 32-bit word of its bit row) per thread: the
    // word's first position is the row's offset plus the set bits before it
    for (int it = t; it < n2 * wa; it += nt) {   // shell-major entries (q << 16) | i, i ascending
        const int q = it / wa, w = it % wa;
        const uint32_t* row = L.cq + (size_t)q * wa;
        int pos = L.cnt_q[q] + bits_below(row, 32 * w);
        for (uint32_t m = row[w]; m; m &= m - 1) lq[pos++] = (q << 16) | (32 * w + __ffs(m) - 1);
    }
    for (int it = t; it < n1 * wa; it += nt) {   // a-major entries (i << 16) | j, j > i ascending
        const int i = it / wa, w = it % wa;
        const uint32_t* row = L.na + (size_t)i * wa;
        int pos = L.cnt_a[i] + bits_below(row, 32 * w);
        for (uint32_t m = row[w]; m; m &= m - 1) la[pos++] = (i << 16) | (32 * w + __ffs(m) - 1);
    }
    // i-major index list: shell partners in scrambled order, each the index of
    // (q, i) in the shell-major list
    for (int it = t; it < n1 * wq; it += nt) {
        const int i = it / wq, w = it % wq;
        const uint32_t* row = L.bq + (size_t)i * wq;
        int pos = L.cnt_i[i] + bits_below(row, 32 * w);
        for (uint32_t m = row[w]; m; m &= m - 1) {
            const int x = 32 * w + __ffs(m) - 1;
            const int q = (int)((uint32_t)(x * sq) % (uint32_t)n2);   // x sq < n2^2 < 2^31
            li[pos++] = L.cnt_q[q] + bits_below(L.cq + (size_t)q * wa, i);
        }
    }
    // b-side index list: K1 partners j < i in scrambled order, each the index of
    // (j, i) in the a-major list
    for (int it = t; it < n1 * wa; it += nt) {
        const int i = it / wa, w = it % wa;
        const uint32_t* row = L.nb + (size_t)i * wa;
        int pos = L.cnt_b[i] + bits_below(row, 32 * w);
        for (uint32_t m = row[w]; m; m &= m - 1) {
            const int x = 32 * w + __ffs(m) - 1;
            const int j = (int)((uint32_t)(x * sa) % (uint32_t)n1);   // x sa < n1^2 < 2^31
            lb[pos++] = L.cnt_a[j] + bits_below(L.na + (size_t)j * wa, i);
        }
    }
}


size_t pairlist_lds_bytes(int n1max, int n2max) {
    return sizeof(double) * 3 * ((size_t)n1max + n2max) + sizeof(uint32_t) * pairlist_lds_words(n1max, n2max);
}

hipError_t launch_pairlist(hipStream_t st, const ScsArgs& a, int n1max, int n2max) {
    hipLaunchKernelGGL(k_pairlist, dim3(a.n), dim3(256), pairlist_lds_bytes(n1max, n2max), st, a, n1max, n2max);
    return hipGetLastError();
}

hipError_t launch_scs_rhs(hipStream_t st, const ScsArgs& a, int n1max, int n2max, bool mixed) {
    const dim3 grid(a.n, a.nw);
    // d and the rows of d^T; B~ itself is assembled by the factorisation kernel
    const size_t ld = dvec_lds_bytes(n1max, n2max);
    if (mixed) hipLaunchKernelGGL(k_scs_dvec<float>, grid, dim3(kChunk), ld, st, a, n1max, n2max);
    else hipLaunchKernelGGL(k_scs_dvec<double>, grid, dim3(kChunk), ld, st, a, n1max, n2max);
    return hipGetLastError();
}

hipError_t launch_scs_factor(hipStream_t st, const ScsArgs& a, int n1max, bool mixed) {
    const dim3 grid(a.n, a.nw);
    const size_t lf = factor_dynamic_bytes(n1max, mixed);
    const bool three = solve_slots(n1max) == 3;
    if (mixed) {
        if (three) hipLaunchKernelGGL((k_scs_factor<float, 3>), grid, dim3(256), lf, st, a, n1max);
        else hipLaunchKernelGGL((k_scs_factor<float, 2>), grid, dim3(256), lf, st, a, n1max);
    } else {
        if (three) hipLaunchKernelGGL((k_scs_factor<double, 3>), grid, dim3(256), lf, st, a, n1max);
        else hipLaunchKernelGGL((k_scs_factor<double, 2>), grid, dim3(256), lf, st, a, n1max);
    }
    return hipGetLastError();
}

hipError_t launch_scs_lambda(hipStream_t st, const ScsArgs& a, int n1max, bool mixed) {
    const dim3 grid(a.n, a.nw);
    const size_t ls = scs_solve_lds_bytes(n1max, mixed);
    const bool three = solve_slots(n1max) == 3;
    if (mixed) {
        if (three) hipLaunchKernelGGL((k_scs_solve<float, 3>), grid, dim3(kSolveThreads), ls, st, a, n1max, (int)kSolveLambda);
        else hipLaunchKernelGGL((k_scs_solve<float, 2>), grid, dim3(kSolveThreads), ls, st, a, n1max, (int)kSolveLambda);
    } else {
        if (three) hipLaunchKernelGGL((k_scs_solve<double, 3>), grid, dim3(kSolveThreads), ls, st, a, n1max, (int)kSolveLambda);
        else hipLaunchKernelGGL((k_scs_solve<double, 2>), grid, dim3(kSolveThreads), ls, st, a, n1max, (int)kSolveLambda);
    }
    return hipGetLastError();
}

hipError_t launch_scs_nu(hipStream_t st, const ScsArgs& a, int n1max, int n2max) {
    hipLaunchKernelGGL(k_scs_nu, dim3(a.n, a.nw), dim3(256), dvec_lds_bytes(n1max, n2max), st, a, n1max, n2max);
    return hipGetLastError();
}

hipError_t launch_scs_adjoint(hipStream_t st, const ScsArgs& a, int n1max, int n2max, bool mixed) {
    const dim3 grid(a.n, a.nw);
    const size_t lds = scs_lds_bytes(n1max, n2max, mixed);
    if (mixed) hipLaunchKernelGGL(k_scs_adjoint<float>, grid, dim3(kChunk), lds, st, a, n1max, n2max);
    else hipLaunchKernelGGL(k_scs_adjoint<double>, grid, dim3(kChunk), lds, st, a, n1max, n2max);
    return hipGetLastError();
}

}  // namespace lmbd
