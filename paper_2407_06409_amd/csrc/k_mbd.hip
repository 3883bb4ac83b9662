// Local MBD energy of every atom and its adjoint (Sec. III.A and III.B).
//
// For central atom k with neighbourhood K (central atom first):
//   alpha~_i(w) = (1 - f_SCS(r_ik)) alpha~_K,i(w) + f_SCS(r_ik) alpha~_I,i(w)  (r_ik < r_scs)
//               = alpha~_I,i(w)                                              (otherwise)
//   R~_i = R0_i (alpha~_i(0) / alpha0_i)^(1/3),  S~_ij = beta (R~_i + R~_j)
//   T_LR,ij = f_LR(r_ij; p) f(r_ij, S~_ij) T_ij      (frequency independent)
//   G~(w) = D T_LR D,  D = diag(sqrt(alpha~_i(w)))
//   E_k = (1/2pi) sum_q w_q sum_{n=2}^{n_max} c_n Tr[G~(w_q)^n]_kk.
// With u_m = G~^m e_k (e_k = the three columns of the central atom),
// Tr[G~^n]_kk = <u_a, u_b> for any a + b = n, so only ceil(n_max/2) products
// with G~ are needed for the energy; all quadrature nodes are stacked as
// columns (3 per node) so each product is one (3n x 3n) x (3n x 3 n_q) GEMM.
//
// Adjoint (seed w_k on E_k):
//   dE/d alpha~_i(w_q) = (W_q / alpha~_i) sum_n c_n sum_{a=0}^{n-1} <u_a, u_{n-a}>_i
//   Tbar = sum_q W_q D Gbar_q D,  Gbar_q = sum_n c_n sum_{a=0}^{n-1} u_a u_{n-1-a}^T
// then contracted pair by pair with dT_LR/dr and dT_LR/dS~, and pushed
// through the blend (local part to this atom's SCS, central part scattered to
// the neighbours' own SCS through a per-site contribution buffer).
//
// Approximate forces of Sec. III.D (a.paper): the seed is the functional of the
// frame whose r_k-gradient is the paper's force, int dw/2pi [c_2 Tr(G~^2) + sum_{n>=3}
// c_n n Tr(g~_k B_n g~_k^T)] (B_n = G~^(n-2) fixed), so that
//   Gbar_q = 2 c_2 G~ + sum_{n>=3} c_n n (u_{n-1} e_k^T + e_k u_{n-1}^T):
// the low-rank part keeps the Tbar product with Z_0 = sum_{n>=3} c_n n u_{n-1} and
// Z_{n-1} = c_n n e_k, the full n = 2 part is added to Tbar element by element, and
//   dE/d alpha~_i(w_q) = W_q [2 c_2 sum_j alpha~_j |T_ij|^2 + sum_{n>=3} c_n n
//                             (<u_{n-1}, u_1>_i + delta_ik mu_n) / alpha~_i];
// the central polarisabilities are held fixed (nothing is scattered to the
// neighbours), and the host keeps only the gradient of the frame's own atom.
//
// Two-body radii (Sec. III.A; SI.two_body): the n = 2 term takes a T_LR of its own, cut
// at r_2b1 on the pairs touching k and r_2b2 on the others.  Its moment is formed
// directly, mu_2 = sum_j alpha~_k alpha~_j |T2_kj|^2 (the central block row), its
// polarisability adjoint likewise, it leaves the Krylov coefficients of Tbar, and its
// pair derivative C2_kj = 2 w_k sum_q W_q c_2 alpha~_k alpha~_j T2_kj is contracted with
// dT2/dr where the pair visits of the contraction meet it (the sparse lists hold the
// central pairs out to max(r_mbd1, r_2b1)).  The approximate forces take the n = 2
// trace of the whole frame with T2: |T2_ij|^2 in the polarisability adjoint and
// C2_ij = 4 w_k sum_q W_q c_2 alpha~_i alpha~_j T2_ij on every pair within the two-body radii.
//
// Eigenvalue-bounded coefficients (Sec. III.A, Eqs. diagonal_appr, eigendecomp and
// polynomial-fit; a.fit): per atom and node, a.lz_steps Lanczos steps on G~ (all nodes
// side by side as columns: each step one (3n x 3n) x (3n x nq) product) give the
// tridiagonal matrix whose extreme eigenvalues (bisection on its Sturm counts) bound
// the spectrum; c_0 .. c_n_max are the least-squares polynomial of ln(1 - x) on that
// interval over the 32 Gauss-Legendre points, formed as the Legendre projection (the
// rule makes the discrete inner product exact for the Legendre polynomials up to
// degree 2 n_max) and converted to powers of x.  The adjoint holds them fixed.
//
// Two-point frequency model (Sec. III.C, Eqs. alpha_SCS_freq and char-freq):
// the SCS is solved at 0 and w_ref only; the blend gives a0 = alpha~_i(0) and
// ar = alpha~_i(w_ref), and alpha~_i(w) = a0 / (1 + (w / w~_i)^2) with
// w~_i = w_ref / sqrt(a0 / ar - 1), evaluated as a0 ar / (rho a0 + (1 - rho) ar),
// rho = (w / w_ref)^2.  Its adjoint: d alpha/d a0 = (1 - rho) (alpha / a0)^2 and
// d alpha/d ar = rho (alpha / ar)^2.
#include <algorithm>
#include <type_traits>

#include "lmbd_internal.h"

namespace lmbd {


__host__ __device__ inline size_t al4(size_t x) { return (x + 3) / 4 * 4; }

// Per-site arrays (LDS, or the workspace) and the small per-atom arrays (LDS).  The
// pair sums g of the force stage take the place of sqrt(alpha~), whose last use (the
// operands of Tbar) precedes them.
struct MbdLds {
    double *px, *py, *pz, *sa, *sqa, *Rt, *fs, *dfs, *ab, *g, *rb, *fg, *mu, *cf, *lz;
};
// sa and ab hold every frequency of the energy: 0 and the nq nodes.  cf (fitted
// coefficients, [nq][kMaxNmax + 1] and [kMaxNmax + 1][nq]) and lz (Lanczos: alpha and beta [steps][nq], the steps
// taken and the two bounds per node) exist only when used.  The site arrays take
// mbd_site_doubles(nk, nq) from b, the small ones start at sm.
__device__ inline MbdLds mbd_lds(double* b, int nk, int nq, double* sm, int n_max, bool fit) {
    const int nw = nq + 1;
    MbdLds L;
    L.px = b;
    L.py = L.px + nk;
    L.pz = L.py + nk;
    L.sa = L.pz + nk;
    L.sqa = L.sa + (size_t)nk * nw;   // [nk][nq]
    L.g = L.sqa;                      // [4 parts][nk][3], nq >= 12 (force stage only)
    L.Rt = L.sqa + (size_t)nk * max(nq, 12);
    L.fs = L.Rt + nk;
    L.dfs = L.fs + nk;
    L.ab = L.dfs + nk;
    L.rb = L.ab + (size_t)nk * nw;    // [4 parts][nk]
    L.fg = L.rb + 4 * (size_t)nk;     // [nk][3]
    L.mu = sm;
    L.cf = L.mu + (size_t)(n_max + 1) * nq;
    L.lz = L.cf + (fit ? 2 * (size_t)(kMaxNmax + 1) * nq : 0);
    return L;
}

// (nkmax = 0: the sparse form with the site arrays in the workspace)
size_t mbd_lds_bytes(int nkmax, int nq, int n_max, int lz_steps, bool fit) {
    return sizeof(double) * (mbd_site_doubles((size_t)nkmax, nq) + mbd_small_doubles(nq, n_max, lz_steps, fit));
}

// The output function of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) on a 64-bit counter.
__device__ inline uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Coefficients c_0 .. c_n_max (c_0 = c_1 = 0 on return) of the least-squares polynomial
// of ln(1 - x) on [lo, hi] over the Gauss-Legendre points x_i of [-1, 1] mapped to it:
// the Legendre coefficients a_j = (2 j + 1) / 2 sum_i w_i ln(1 - lambda_i) P_j(x_i),
// then sum_j a_j P_j(t), t = (x - mid) / half, in powers of x by Clenshaw's recurrence
// b_j = a_j + (2j+1)/(j+1) t b_{j+1} - (j+1)/(j+2) b_{j+2} carried out on coefficient
// arrays (b_0 is the polynomial).  No width (hi - lo <= 1e-12): the Taylor
// coefficients -1/n.
__host__ __device__ inline void log_fit(double lo, double hi, int n_max, const double* gx, const double* gw,
                                        double (&c)[kMaxNmax + 1]) {
#pragma unroll
    for (int n = 0; n <= kMaxNmax; ++n) c[n] = n >= 2 ? -1.0 / n : 0.0;
    if (!(hi - lo > 1e-12)) return;
    const double h = 0.5 * (hi - lo), m = 0.5 * (hi + lo), ih = 1.0 / h;
    double cl[kMaxNmax + 1];
#pragma unroll
    for (int j = 0; j <= kMaxNmax; ++j) cl[j] = 0.0;
    for (int i = 0; i < kFitNodes; ++i) {
        const double x = gx[i];
        const double f = gw[i] * log1p(-(m + h * x));
        double p0 = 1.0, p1 = x;
        cl[0] += f;
        cl[1] += f * x;
#pragma unroll
        for (int j = 2; j <= kMaxNmax; ++j) {
            const double p2 = ((2 * j - 1) * x * p1 - (j - 1) * p0) / j;
            cl[j] += f * p2;
            p0 = p1;
            p1 = p2;
        }
    }
    // b1 = b_{j+1}, b2 = b_{j+2}; b_j overwrites b2, then the two swap roles
    double b1[kMaxNmax + 1], b2[kMaxNmax + 1];
#pragma unroll
    for (int t = 0; t <= kMaxNmax; ++t) b1[t] = b2[t] = 0.0;
#pragma unroll
    for (int j = kMaxNmax; j >= 0; --j) {
        if (j > n_max) continue;
        const double aj = 0.5 * (2 * j + 1) * cl[j];
        const double al = (2.0 * j + 1.0) / (j + 1.0) * ih, be = -(j + 1.0) / (j + 2.0);
#pragma unroll
        for (int t = kMaxNmax; t >= 0; --t)
            b2[t] = (t == 0 ? aj : 0.0) + al * ((t > 0 ? b1[t - 1] : 0.0) - m * b1[t]) + be * b2[t];
#pragma unroll
        for (int t = 0; t <= kMaxNmax; ++t) {
            const double x = b1[t];
            b1[t] = b2[t];
            b2[t] = x;
        }
    }
#pragma unroll
    for (int n = 0; n <= kMaxNmax; ++n) c[n] = n >= 2 ? b1[n] : 0.0;
}

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// MFMA 16x16x4 in the workspace type (lane layouts as measured on gfx950: A[i][k]
// <- lane i + 16k, B[k][j] <- lane j + 16k; D[i][j] in lane j + 16 (i % 4), register
// i / 4 for f64 and lane j + 16 (i / 4), register i % 4 for f32).
template <typename W> struct MfmaW;
template <> struct MfmaW<double> {
    typedef d4_t acc;
    static __device__ inline acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int acc_row(int g, int q) { return g + 4 * q; }
};
template <> struct MfmaW<float> {
    typedef f4_t acc;
    static __device__ inline acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int acc_row(int g, int q) { return 4 * g + q; }
};

// Workgroup GEMM on the matrix cores: out(m, n) = sum_k A[m][k] B[n][k] with both operands k-contiguous
// (row-major, lda/ldb multiples of 4, K a multiple of 4).  Lane (i, g) of an MFMA
// operand reads the 4-vector k = 16 c + 4 g .. + 3 and feeds element e to k-step e,
// the same permutation of k for both operands; 16 k per chunk, the next chunk in
// flight.  Each wavefront takes MR 16-row strips times up to NVMAX 16-column tiles.
// With `lower` set, only items holding entries on or below the diagonal are
// computed (for a product known to be symmetric; the rest of the output is left
// as it was).
template <int MR, int NVMAX, typename W, typename ST>
__device__ __forceinline__ void mfma_gemm_nt(int M, int N, int K, const W* __restrict__ A, int lda,
                                             const W* __restrict__ B, int ldb, bool lower, ST st) {
    typedef MfmaW<W> Mf;
    typedef W V4 __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int mt = (M + 16 * MR - 1) / (16 * MR);   // items of MR 16-row strips
    const int nt = (N + 15) / 16;
    const int ng = (nt + NVMAX - 1) / NVMAX;
    const int nch = (K + 15) / 16;
    const V4 zero = {W(0), W(0), W(0), W(0)};
    auto kin = [&](int ch) { return ch < nch && 16 * ch + 4 * lk < K; };
    // MR 16-row strips times NV column tiles (NV = the tiles of the group inside N)
    auto item = [&](int m0, int tc0, auto nvc) {
        constexpr int NV = decltype(nvc)::value;
        typename Mf::acc acc[MR][NV];
#pragma unroll
        for (int x = 0; x < MR; ++x)
#pragma unroll
            for (int c = 0; c < NV; ++c)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[x][c][q] = W(0);
        const W* pa[MR];
        bool aok[MR];
#pragma unroll
        for (int x = 0; x < MR; ++x) {
            const int am = m0 + 16 * x + li;
            aok[x] = am < M;
            pa[x] = A + (size_t)(aok[x] ? am : 0) * lda + 4 * lk;
        }
        const W* pb[NV];
        bool bok[NV];
        int bn[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            bn[c] = (tc0 + c) * 16 + li;
            bok[c] = bn[c] < N;
            pb[c] = B + (size_t)(bok[c] ? bn[c] : 0) * ldb + 4 * lk;
        }
        V4 a[MR], b[NV];
#pragma unroll
        for (int x = 0; x < MR; ++x) a[x] = (aok[x] && kin(0)) ? *reinterpret_cast<const V4*>(pa[x]) : zero;
#pragma unroll
        for (int c = 0; c < NV; ++c) b[c] = (bok[c] && kin(0)) ? *reinterpret_cast<const V4*>(pb[c]) : zero;
        for (int ch = 0; ch < nch; ++ch) {
            const bool kn = kin(ch + 1);
            V4 na[MR], nb[NV];
#pragma unroll
            for (int x = 0; x < MR; ++x)
                na[x] = (aok[x] && kn) ? *reinterpret_cast<const V4*>(pa[x] + 16 * (ch + 1)) : zero;
#pragma unroll
            for (int c = 0; c < NV; ++c)
                nb[c] = (bok[c] && kn) ? *reinterpret_cast<const V4*>(pb[c] + 16 * (ch + 1)) : zero;
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int x = 0; x < MR; ++x)
#pragma unroll
                    for (int c = 0; c < NV; ++c) acc[x][c] = Mf::mma(a[x][e], b[c][e], acc[x][c]);
#pragma unroll
            for (int x = 0; x < MR; ++x) a[x] = na[x];
#pragma unroll
            for (int c = 0; c < NV; ++c) b[c] = nb[c];
        }
#pragma unroll
        for (int x = 0; x < MR; ++x)
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                if (bok[c]) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int m = m0 + 16 * x + Mf::acc_row(lk, q);
                        if (m < M) st(m, bn[c], acc[x][c][q]);
                    }
                }
            }
    };
    for (int t = wave; t < mt * ng; t += nwave) {
        const int m0 = (t / ng) * 16 * MR;
        const int tc0 = (t % ng) * NVMAX;
        if (lower && 16 * tc0 > m0 + 16 * MR - 1) continue;   // wholly above the diagonal
        const int nv = min(NVMAX, nt - tc0);   // uniform over the wavefront
        if (nv >= 4) item(m0, tc0, std::integral_constant<int, NVMAX >= 4 ? 4 : 1>());
        else if (nv == 3) item(m0, tc0, std::integral_constant<int, NVMAX >= 3 ? 3 : 1>());
        else if (nv == 2) item(m0, tc0, std::integral_constant<int, NVMAX >= 2 ? 2 : 1>());
        else item(m0, tc0, std::integral_constant<int, 1>());
    }
    __syncthreads();
}

// T_LR pair coefficients: T_LR = A rhat rhat^T + B I with radial derivatives,
// and dT_LR/dS~ = fLR (df/dS~) T.
template <typename P>
struct LrPair {
    P A, B, dA, dB, dfS, fLR;
};
template <typename P>
__device__ inline LrPair<P> lr_pair(P r, P S, P damp_d, P rcut, P rb) {
    P dfdr, dfdS, dcut;
    const P f = fermi<P>(r, S, damp_d, dfdr, dfdS);
    const P fc = cutoff_poly<P>(r, rcut, rb, dcut);
    const P w = fc * f;
    const P dw = dcut * f + fc * dfdr;
    const P ir = P(1) / r;
    const P ir3 = ir * ir * ir;
    LrPair<P> p;
    p.A = P(3) * w * ir3;
    p.B = -w * ir3;
    p.dA = P(3) * dw * ir3 - P(9) * w * ir3 * ir;
    p.dB = -dw * ir3 + P(3) * w * ir3 * ir;
    p.dfS = dfdS;
    p.fLR = fc;
    return p;
}

// 512 threads: the eight wavefronts share the GEMM items of an atom (six
// 48-row items per Krylov product, 21 lower-triangle items of Tbar), which
// balances them better than four (measured 4.55 -> 4.42 ms FP64, 3.07 -> 2.62
// ms FP32 on 1,728 C atoms; 384, 768 and 1,024 threads were slower)
constexpr int kMbdThreads = 512;

// Value of `x` in lane l (l uniform over the wavefront).
__device__ inline double read_lane(double x, int l) {
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ inline float read_lane(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
template <typename W>
__device__ inline W lane_value(W x, int l) { return read_lane(x, l); }

// Sums over the 64 lanes of nine per-lane values, returned to every lane.  A
// transposed butterfly: at the exchanges over lane bits 5, 4, 3 and 2 a lane keeps
// half of the (zero-padded to 16) values it carries and sends the other half, so
// lane l ends with value 8 b5 + 4 b4 + 2 b3 + b2 (b_n: bit n of l) summed over its
// 16 partners; two plain exchanges finish the sum and one lane per value gives it
// out: 17 exchanges instead of 54.
__device__ inline void wave_sum9(const double (&v)[9], double (&out)[9]) {
    const int lane = threadIdx.x & 63;
    double a[8], b[4], c[2];
    bool hi = lane & 32;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const double lo_v = v[t], hi_v = (t == 0) ? v[8] : 0.0;
        a[t] = (hi ? hi_v : lo_v) + __shfl_xor(hi ? lo_v : hi_v, 32);
    }
    hi = lane & 16;
#pragma unroll
    for (int t = 0; t < 4; ++t) b[t] = (hi ? a[4 + t] : a[t]) + __shfl_xor(hi ? a[t] : a[4 + t], 16);
    hi = lane & 8;
#pragma unroll
    for (int t = 0; t < 2; ++t) c[t] = (hi ? b[2 + t] : b[t]) + __shfl_xor(hi ? b[t] : b[2 + t], 8);
    hi = lane & 4;
    double d = (hi ? c[1] : c[0]) + __shfl_xor(hi ? c[0] : c[1], 4);
    d += __shfl_xor(d, 2);
    d += __shfl_xor(d, 1);
#pragma unroll
    for (int x = 0; x < 9; ++x)
        out[x] = read_lane(d, ((x >> 3) & 1) << 5 | ((x >> 2) & 1) << 4 | ((x >> 1) & 1) << 3 | (x & 1) << 2);
}

// SP = false: T_LR is stored dense and every product runs on the matrix cores.
// SP = true (two-radius regime, Sec. III.A: a site couples to the central atom up
// to r_MBD,1 but to the others only up to r_MBD,2, so block rows other than the
// central one are sparse): T_LR is never stored.  The coupled sites of every block
// row and their coefficients are listed once per atom (a wavefront per row, its
// lanes testing 64 candidates at a time); each Krylov product walks a row's list
// with the whole wavefront (lanes over the Krylov columns), and Tbar is formed only
// for coupled pairs, each 3x3 block as nine dot products over eight lanes.
// The sparse form is bound by the latency of its gathers rather than by arithmetic:
// it runs 1,024 threads (four wavefronts per SIMD at its register count) to hide it.
constexpr int kMbdThreadsSparse = 1024;
// TB: the atoms' structures have two-body radii of their own (a separate instantiation,
// so that the other kernels carry none of its registers)
template <typename W, int FORM, bool TB>
__global__ void __launch_bounds__(FORM != kMbdDense ? kMbdThreadsSparse : kMbdThreads, 1) k_mbd(MbdArgs a, int nkmax) {
    constexpr bool SP = FORM != kMbdDense, GS = FORM == kMbdSparseGlobal;
    extern __shared__ double lds[];
    const int k = a.order[blockIdx.x];
    const int tid = threadIdx.x;
    const Counts cnt = a.counts[k];
    const int nK = cnt.nK, n1 = cnt.n1, nall = cnt.n_all;
    const int N3 = 3 * nK;
    const int nw = a.nw, nq = a.nq, ncol = a.ncol, n_max = a.n_max;
    const int nwe = nq + 1;   // row stride of L.sa and L.ab (nw is that of the SCS arrays)
    const StructInfo& SI = a.sinfo[a.atom_struct[k]];
    const double rs = SI.r_scs;
    const bool fit = a.fit != 0;
    constexpr bool has2b = TB;
    W* const wbase = static_cast<W*>(a.work) + a.work_off[k];
    const int64_t lcap = GS ? mbd_list_cap(nK, SI.m2max) : (int64_t)nK * nK;   // list entries
    const MbdGlobalLayout G = mbd_global_layout(nK, nq, n_max, a.mmax, lcap, (int64_t)sizeof(W), a.forces != 0);
    MbdLds L = GS ? mbd_lds(reinterpret_cast<double*>(wbase + G.sites), nK, nq, lds, n_max, fit)
                  : mbd_lds(lds, nkmax, nq, lds + mbd_site_doubles((size_t)nkmax, nq), n_max, fit);
    // c_n at node q: fitted per atom and node, or the common series
    // (fitted: two copies in LDS, [kMaxNmax + 1][nq] here and [nq][kMaxNmax + 1] for the adjoint operands,
    // whose per-element loop keeps one node's coefficients at fixed offsets)
    double* const cfn = L.cf + (size_t)(kMaxNmax + 1) * nq;
    auto cfq = [&](int n, int q) -> double { return fit ? cfn[n * nq + q] : a.coef[n]; };
    const int lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
    const Site* S = a.sites + a.site_off[k];
    const double* aloc = a.alpha_loc + a.aloc_off[k];
    // sub-arrays start on multiples of 4 elements (aligned 4-vector loads)
    const int KK = n_max * ncol, KKp = (KK + 3) / 4 * 4;
    const int N3p = (int)al4(N3);                            // row stride of T and of V^T (zero padded)
    W* T = wbase;                                            // dense T_LR (the sparse form's lists in its space)
    W* U = T + al4((size_t)N3 * N3p);                        // u_1 .. u_mmax
    W* V = U + al4((size_t)a.mmax * N3 * ncol);              // (D u_m)^T, the next product's operand, ncol x N3p,
    W* V2 = V + al4((size_t)ncol * N3p);                     //   in two buffers used in turn
    W* Pm = V2 + al4((size_t)ncol * N3p);                    // D u_a side by side, a = 0 .. n_max-1
    W* Qm = Pm + (size_t)N3 * KKp;                           // W D Z_a side by side
    if constexpr (GS) {   // no dense T: the parts of the global-site layout
        T = wbase + G.lists;
        U = wbase + G.U;
        V = wbase + G.V;
        V2 = wbase + G.V2;
        Pm = wbase + G.P;
        Qm = wbase + G.Q;
    }
    auto Uat = [&](int m) { return U + (size_t)(m - 1) * N3 * ncol; };

    // --- blend (Sec. III.B, central/local combination) and SCS radii
    for (int s = tid; s < nK; s += blockDim.x) {
        const Site st = S[s];
        L.px[s] = st.x;
        L.py[s] = st.y;
        L.pz[s] = st.z;
        const double r = sqrt(st.x * st.x + st.y * st.y + st.z * st.z);
        const double* cen = a.alpha_loc + a.aloc_off[st.base];  // row 0 = central value
        double fsv = 1.0, dfsv = 0.0;
        if (s == 0) {
            fsv = 0.0;
        } else if (s < n1) {
            const double x = r / rs;
            fsv = 3.0 * x * x - 2.0 * x * x * x;
            dfsv = (6.0 * x - 6.0 * x * x) / rs;
        }
        L.fs[s] = fsv;
        L.dfs[s] = dfsv;
        if (a.lorentz) {
            const double a0 = (s == 0) ? aloc[0] : (s < n1) ? (1.0 - fsv) * aloc[(size_t)s * nw] + fsv * cen[0] : cen[0];
            const double ar = (s == 0) ? aloc[1] : (s < n1) ? (1.0 - fsv) * aloc[(size_t)s * nw + 1] + fsv * cen[1] : cen[1];
            if (!(ar > 0.0 && a0 >= ar)) {   // no real characteristic frequency
                atomicOr(a.err, 8);
                atomicMin(a.err_atom, k);
            }
            L.sa[(size_t)s * nwe] = a0;
            for (int q = 0; q < nq; ++q) {
                const double v = a0 * ar / (a.rho[q] * a0 + (1.0 - a.rho[q]) * ar);
                L.sa[(size_t)s * nwe + 1 + q] = v;
                L.sqa[(size_t)s * nq + q] = sqrt(v);
            }
        } else {
            for (int w = 0; w < nw; ++w) {
                const double al = (s < n1) ? aloc[(size_t)s * nw + w] : 0.0;
                const double v = (s == 0) ? al : (1.0 - fsv) * al + fsv * cen[w];
                L.sa[(size_t)s * nwe + w] = v;
                if (w > 0) L.sqa[(size_t)s * nq + (w - 1)] = sqrt(v);
            }
        }
        L.Rt[s] = a.r0v[st.base] * cbrt(L.sa[(size_t)s * nwe] / a.a0v[st.base]);
    }
    __syncthreads();

    // --- T_LR (row-major, symmetric, zero diagonal blocks).  One block (i, j)
    // per thread, consecutive threads along a block row, so that the rows are
    // written in contiguous runs (each unordered pair is evaluated from both
    // ends: the block is the same for (i, j) and (j, i)).
    if constexpr (!SP) {
    for (int p = tid; p < nK * nK; p += blockDim.x) {
        const int i = p / nK, j = p % nK;
        double blk[9] = {};
        if (i != j) {
            const double v[3] = {L.px[i] - L.px[j], L.py[i] - L.py[j], L.pz[i] - L.pz[j]};
            const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            const double rcut = (i == 0 || j == 0) ? SI.r_mbd1 : SI.r_mbd2;
            if (r < rcut) {
                const LrPair<W> t = lr_pair<W>(W(r), W(a.beta * (L.Rt[i] + L.Rt[j])), W(a.damp_d), W(rcut),
                                               W(a.r_buf));
                const double rh[3] = {v[0] / r, v[1] / r, v[2] / r};
                for (int q = 0; q < 3; ++q)
                    for (int c = 0; c < 3; ++c)
                        blk[3 * q + c] = double(t.A) * rh[q] * rh[c] + (q == c ? double(t.B) : 0.0);
            }
        }
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c) T[(size_t)(3 * i + q) * N3p + 3 * j + c] = W(blk[3 * q + c]);
    }
    for (int e = tid; e < N3 * (N3p - N3); e += blockDim.x) T[(size_t)(e / (N3p - N3)) * N3p + N3 + e % (N3p - N3)] = W(0);
    for (int e = tid; e < ncol * (N3p - N3); e += blockDim.x) {
        V[(size_t)(e / (N3p - N3)) * N3p + N3 + e % (N3p - N3)] = W(0);
        V2[(size_t)(e / (N3p - N3)) * N3p + N3 + e % (N3p - N3)] = W(0);
    }
    __syncthreads();
    }

    // sparse form: whether the pair (i, j) couples, and its coefficients T_LR,ij = A rhat rhat^T + B I
    auto coupled = [&](int i, int j, double v[3], double& r) -> bool {
        if (j >= nK || j == i) return false;
        v[0] = L.px[i] - L.px[j];
        v[1] = L.py[i] - L.py[j];
        v[2] = L.pz[i] - L.pz[j];
        r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        // (central pairs out to the two-body radius too: their MBD coefficients are 0 there)
        return r < ((i == 0 || j == 0) ? (has2b ? fmax(SI.r_mbd1, SI.r_2b1) : SI.r_mbd1) : SI.r_mbd2);
    };
    auto couple = [&](int i, int j, W& A, W& B, double rh[3]) -> bool {
        double v[3], r;
        if (!coupled(i, j, v, r)) return false;
        const double rcut = (i == 0 || j == 0) ? SI.r_mbd1 : SI.r_mbd2;
        const LrPair<W> t = lr_pair<W>(W(r), W(a.beta * (L.Rt[i] + L.Rt[j])), W(a.damp_d), W(rcut), W(a.r_buf));
        A = t.A;
        B = t.B;
        rh[0] = v[0] / r;
        rh[1] = v[1] / r;
        rh[2] = v[2] / r;
        return true;
    };
    // sparse form: the coupled sites of every block row and their coefficients, found
    // once per atom: row i at [roff[i], roff[i + 1]) of NN entries (site index, A, B, rhat).
    // With the site arrays in LDS they sit in the space of the dense T (unused here):
    // (4 + 5 sizeof(W)) nK^2 + 4 (nK + 1) bytes fit in its 9 nK^2 sizeof(W); else in a part of
    // their own, sized from the structure's largest count of sites within r_mbd2.
    const size_t NN = (size_t)lcap;
    W* const pA = T;
    W* const pB = pA + NN;
    W* const pR0 = pB + NN;
    W* const pR1 = pR0 + NN;
    W* const pR2 = pR1 + NN;
    int* const pj = reinterpret_cast<int*>(pR2 + NN);
    int* const roff = pj + NN;
    if constexpr (SP) {
        // counts per row (into roff[i + 1]), then their running sum over the rows
        for (int i = wave; i < nK; i += nwave) {
            int n = 0;
            for (int j0 = 0; j0 < nK; j0 += 64) {
                double v[3], r;
                n += __popcll(__ballot(coupled(i, j0 + lane, v, r)));
            }
            if (lane == 0) roff[i + 1] = n;
        }
        __syncthreads();
        if (wave == 0) {
            int carry = 0;
            for (int i0 = 0; i0 < nK; i0 += 64) {
                const bool in = i0 + lane < nK;
                int x = in ? roff[i0 + lane + 1] : 0;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int t = __shfl_up(x, o);
                    if (lane >= o) x += t;
                }
                if (in) roff[i0 + lane + 1] = carry + x;
                carry += __shfl(x, 63);
            }
            if (lane == 0) roff[0] = 0;
        }
        __syncthreads();
        if (tid == 0 && (size_t)roff[nK] > NN) {   // a row outgrew the bound: refuse the call
            atomicOr(a.err, 32);
            atomicMin(a.err_atom, k);
        }
        for (int i = wave; i < nK; i += nwave) {
            int n = roff[i];
            for (int j0 = 0; j0 < nK; j0 += 64) {
                W A = W(0), B = W(0);
                double rh[3] = {0.0, 0.0, 0.0};
                const bool in = couple(i, j0 + lane, A, B, rh);
                const unsigned long long mask = __ballot(in);
                const size_t e = (size_t)n + __popcll(mask & ((1ull << lane) - 1ull));
                if (in && e < NN) {
                    pj[e] = j0 + lane;
                    pA[e] = A;
                    pB[e] = B;
                    pR0[e] = W(rh[0]);
                    pR1[e] = W(rh[1]);
                    pR2[e] = W(rh[2]);
                }
                n += __popcll(mask);
            }
        }
        __syncthreads();
    }
    // entries of row i: [roff[i], roff[i] + row_len(i)), within the capacity
    auto row_len = [&](int i) -> int {
        const int e1 = roff[i + 1] < (int)NN ? roff[i + 1] : (int)NN;
        return e1 > roff[i] ? e1 - roff[i] : 0;
    };
    // sparse form: Uout = D T D Uin, one block row (and 64 columns) per wavefront, lanes over
    // the columns, four coupled sites per step; the loads use in-bounds indices (entry 0 of the
    // row, column 0) with a zero factor instead of a branch, so that they overlap
    auto sparse_product = [&](const W* __restrict__ Uin, W* __restrict__ Uout) {
        for (int it = wave; it < nK * ((ncol + 63) / 64); it += nwave) {
            const int i = it % nK, col = (it / nK) * 64 + lane, q = col / 3;
            const int cs = col < ncol ? col : 0, qs = cs / 3;
            const int n = row_len(i);
            const size_t e0 = (size_t)roff[i];
            W acc0 = W(0), acc1 = W(0), acc2 = W(0);
            for (int s0 = 0; s0 < n; s0 += 4) {
                // the four entries are loaded cooperatively (lane 4 f + u holds field f of entry
                // s0 + u: A, B, rhat) and handed to every lane through scalar registers
                const int fu = lane & 3, ff = min(lane >> 2, 4);
                const size_t ec = e0 + (s0 + fu < n ? s0 + fu : 0);
                const W fv = pA[(size_t)ff * NN + ec];
                const int jv = pj[ec];
                W x[4][3], Aj[4], Bj[4], r0[4], r1[4], r2[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool ok = s0 + u < n;
                    const int j = __builtin_amdgcn_readlane(jv, u);
                    Aj[u] = lane_value(fv, u);
                    Bj[u] = lane_value(fv, 4 + u);
                    r0[u] = lane_value(fv, 8 + u);
                    r1[u] = lane_value(fv, 12 + u);
                    r2[u] = lane_value(fv, 16 + u);
                    const W sj = (ok && col < ncol) ? W(L.sqa[(size_t)j * nq + qs]) : W(0);
#pragma unroll
                    for (int c = 0; c < 3; ++c) x[u][c] = sj * Uin[(size_t)(3 * j + c) * ncol + cs];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const W ax = Aj[u] * (r0[u] * x[u][0] + r1[u] * x[u][1] + r2[u] * x[u][2]);
                    acc0 += ax * r0[u] + Bj[u] * x[u][0];
                    acc1 += ax * r1[u] + Bj[u] * x[u][1];
                    acc2 += ax * r2[u] + Bj[u] * x[u][2];
                }
            }
            if (col < ncol) {
                const W si = W(L.sqa[(size_t)i * nq + q]);
                Uout[(size_t)(3 * i) * ncol + col] = si * acc0;
                Uout[(size_t)(3 * i + 1) * ncol + col] = si * acc1;
                Uout[(size_t)(3 * i + 2) * ncol + col] = si * acc2;
            }
        }
        __syncthreads();
    };

    // sparse form, Lanczos vectors (column-major [nq][N3p], one column per node):
    // Vout = D T D Vin, one block row per wavefront, lanes over the nodes, the row's
    // coupled sites in order
    auto sparse_product_lz = [&](const W* __restrict__ Vin, W* __restrict__ Vout) {
        const int q = lane < nq ? lane : 0;
        for (int i = wave; i < nK; i += nwave) {
            const int n = row_len(i);
            const size_t e0 = (size_t)roff[i];
            W acc0 = W(0), acc1 = W(0), acc2 = W(0);
            for (int t = 0; t < n; ++t) {
                const size_t e = e0 + t;
                const int j = pj[e];
                const W Aj = pA[e], Bj = pB[e], r0 = pR0[e], r1 = pR1[e], r2 = pR2[e];
                const W sj = W(L.sqa[(size_t)j * nq + q]);
                const W* x = Vin + (size_t)q * N3p + 3 * j;
                const W x0 = sj * x[0], x1 = sj * x[1], x2 = sj * x[2];
                const W ax = Aj * (r0 * x0 + r1 * x1 + r2 * x2);
                acc0 += ax * r0 + Bj * x0;
                acc1 += ax * r1 + Bj * x1;
                acc2 += ax * r2 + Bj * x2;
            }
            if (lane < nq) {
                const W si = W(L.sqa[(size_t)i * nq + q]);
                W* y = Vout + (size_t)q * N3p + 3 * i;
                y[0] = si * acc0;
                y[1] = si * acc1;
                y[2] = si * acc2;
            }
        }
        __syncthreads();
    };

    // --- u_1 = D T D e_k, V = D u_1
    W* U1 = Uat(1);
    if constexpr (SP) {
        // u_1 = D T D e_k needs the block column of the central atom only
        for (int e = tid; e < nK * ncol; e += blockDim.x) {
            const int i = e / ncol, col = e % ncol, q = col / 3, c = col % 3;
            W A = W(0), B = W(0);
            double rh[3] = {0.0, 0.0, 0.0};
            const bool in = couple(i, 0, A, B, rh);
            const double s = L.sqa[(size_t)i * nq + q] * L.sqa[q];
            for (int r = 0; r < 3; ++r)
                U1[(size_t)(3 * i + r) * ncol + col] =
                    in ? W(s * (double(A) * rh[r] * rh[c] + (r == c ? double(B) : 0.0))) : W(0);
        }
        __syncthreads();
    } else {
    for (int e = tid; e < N3 * ncol; e += blockDim.x) {
        const int row = e / ncol, col = e % ncol;
        const int q = col / 3, c = col % 3;
        const double sq = L.sqa[(size_t)(row / 3) * nq + q];
        const double u = sq * double(T[(size_t)row * N3p + c]) * L.sqa[q];
        U1[e] = W(u);
        V[(size_t)col * N3p + row] = W(sq * u);
    }
    __syncthreads();
    }
    // --- u_{m+1} = D (T V), V' = D u_{m+1}  (T symmetric, so it is its own K-major
    // operand); the product's stores write both, V' into the other buffer
    for (int m = 1; m < a.mmax; ++m) {
        W* Un = Uat(m + 1);
        if constexpr (SP) {
            sparse_product(Uat(m), Un);
            continue;
        }
        const W* Vin = (m & 1) ? V : V2;
        W* Vout = (m & 1) ? V2 : V;
        mfma_gemm_nt<3, 3, W>(N3, ncol, N3, T, N3p, Vin, N3p, false, [&](int r, int col, W v) {
            const W sq = W(L.sqa[(size_t)(r / 3) * nq + col / 3]);
            const W un = sq * v;
            Un[(size_t)r * ncol + col] = un;
            Vout[(size_t)col * N3p + r] = sq * un;
        });   // ends with a barrier
    }

    // --- spectrum bounds of G~ at every node (Lanczos) and, with a.fit, the fitted c_n
    if (a.lz_steps > 0) {
        const int m = a.lz_steps;
        // three vectors per node, column-major ([nq][N3p]), in the space of V; the dense
        // products' operand D v (rows 0 .. nq-1, zero padded) in V2
        W* vb[3] = {V, V + (size_t)nq * N3p, V + 2 * (size_t)nq * N3p};
        double* la = L.lz;                            // alpha_j of node q at [j nq + q]
        double* lb = la + (size_t)m * nq;             // beta_{j+1} at [j nq + q]
        double* lm = lb + (size_t)m * nq;             // steps taken per node
        double* bnd = lm + nq;                        // [nq][2] bounds
        auto wave_total = [&](double x) -> double {   // same order, same value in every lane
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
            return x;
        };
        // start vector, keyed on (k, base atom, lattice shift, component) in the structure's numbering
        const uint64_t kl = (uint64_t)(k - SI.atom_offset);
        auto start = [&](int r) -> double {
            const Site st = S[r / 3];
            const uint64_t h = splitmix64((kl << 32) + (uint64_t)(st.base - SI.atom_offset));
            const uint64_t z = splitmix64(h + 4ull * (uint64_t)(uint32_t)st.shift + (uint64_t)(r % 3));
            return (double)(z >> 11) * 0x1.0p-53 - 0.5;
        };
        for (int q = wave; q < nq; q += nwave) {
            double s2 = 0.0;
            for (int r = lane; r < N3; r += 64) {
                const double x = start(r);
                s2 += x * x;
            }
            const double inv = 1.0 / sqrt(wave_total(s2));
            W* v1 = vb[1] + (size_t)q * N3p;
            W* v0 = vb[0] + (size_t)q * N3p;
            for (int r = lane; r < N3; r += 64) {
                const W v = W(start(r) * inv);
                v1[r] = v;
                v0[r] = W(0);
                if constexpr (!SP) V2[(size_t)q * N3p + r] = W(L.sqa[(size_t)(r / 3) * nq + q]) * v;
            }
            if (lane == 0) lm[q] = m;
        }
        __syncthreads();
        int ip = 0, ic = 1, iw = 2;
        for (int j = 0; j < m; ++j) {
            // w = G~ v_j at every node (a node that has stopped has v_j = 0)
            if constexpr (SP) {
                sparse_product_lz(vb[ic], vb[iw]);
            } else {
                W* wv = vb[iw];
                mfma_gemm_nt<1, 2, W>(N3, nq, N3, T, N3p, V2, N3p, false, [&](int r, int q, W v) {
                    wv[(size_t)q * N3p + r] = W(L.sqa[(size_t)(r / 3) * nq + q]) * v;
                });   // ends with a barrier
            }
            // w -= beta_j v_{j-1}; alpha_j = <v_j, w>; w -= alpha_j v_j; beta_{j+1} = |w|;
            // v_{j+1} = w / beta_{j+1} (zero once the node stops)
            for (int q = wave; q < nq; q += nwave) {
                if (lm[q] <= j) continue;
                const W* vp = vb[ip] + (size_t)q * N3p;
                const W* vc = vb[ic] + (size_t)q * N3p;
                W* w = vb[iw] + (size_t)q * N3p;
                const double bj = j > 0 ? lb[(size_t)(j - 1) * nq + q] : 0.0;
                double s = 0.0;
                for (int r = lane; r < N3; r += 64) {
                    const double t = double(w[r]) - bj * double(vp[r]);
                    w[r] = W(t);
                    s += double(vc[r]) * t;
                }
                const double al = wave_total(s);
                double s2 = 0.0;
                for (int r = lane; r < N3; r += 64) {
                    const double t = double(w[r]) - al * double(vc[r]);
                    w[r] = W(t);
                    s2 += t * t;
                }
                const double bn = sqrt(wave_total(s2));
                const bool stop = j == m - 1 || !(bn > 1e-10 * (fabs(al) + bj));
                const double inv = stop ? 0.0 : 1.0 / bn;
                for (int r = lane; r < N3; r += 64) {
                    const W v = W(double(w[r]) * inv);
                    w[r] = v;
                    if constexpr (!SP) V2[(size_t)q * N3p + r] = W(L.sqa[(size_t)(r / 3) * nq + q]) * v;
                }
                if (lane == 0) {
                    la[(size_t)j * nq + q] = al;
                    lb[(size_t)j * nq + q] = bn;
                    if (stop) lm[q] = j + 1;
                }
            }
            __syncthreads();
            const int t = ip;
            ip = ic;
            ic = iw;
            iw = t;
        }
        // extreme eigenvalues of each node's tridiagonal matrix: bisection on the number
        // of eigenvalues below x (the negative pivots of T - x I = L D L^T), one lane per end
        if (tid < 2 * nq) {
            const int q = tid >> 1, top = tid & 1;
            const int me = (int)lm[q];
            double glo = 0.0, ghi = 0.0;
            for (int j = 0; j < me; ++j) {
                const double b0 = j > 0 ? fabs(lb[(size_t)(j - 1) * nq + q]) : 0.0;
                const double b1 = j + 1 < me ? fabs(lb[(size_t)j * nq + q]) : 0.0;
                const double aj = la[(size_t)j * nq + q];
                glo = j == 0 ? aj - b0 - b1 : fmin(glo, aj - b0 - b1);
                ghi = j == 0 ? aj + b0 + b1 : fmax(ghi, aj + b0 + b1);
            }
            const double pad = 1e-14 * (fabs(glo) + fabs(ghi)) + 1e-300;
            double lo = glo - pad, hi = ghi + pad;
            const int target = top ? me : 1;   // count(lo) < target <= count(hi)
            for (int it = 0; it < 256; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (!(mid > lo && mid < hi)) break;
                int cnt = 0;
                double d = 1.0;
                for (int j = 0; j < me; ++j) {
                    const double bb = j > 0 ? lb[(size_t)(j - 1) * nq + q] : 0.0;
                    d = la[(size_t)j * nq + q] - mid - (j > 0 ? bb * bb / d : 0.0);
                    if (fabs(d) < 1e-300) d = -1e-300;
                    cnt += d < 0.0 ? 1 : 0;
                }
                if (cnt >= target)
                    hi = mid;
                else
                    lo = mid;
            }
            bnd[tid] = hi;
            if (a.spectrum) a.spectrum[((size_t)k * nq + q) * 2 + top] = hi;
        }
        __syncthreads();
        if (fit && tid < nq) {
            const int q = tid;
            const double lo = bnd[2 * q], hi = bnd[2 * q + 1];
            double c[kMaxNmax + 1];
            if (!(hi < 1.0)) {   // polarisation catastrophe: ln(1 - x) has no fit
                atomicOr(a.err, 16);
                atomicMin(a.err_atom, k);
#pragma unroll
                for (int n = 0; n <= kMaxNmax; ++n) c[n] = 0.0;
            } else {
                log_fit(lo, hi, n_max, a.gl_x, a.gl_w, c);
            }
#pragma unroll
            for (int n = 0; n <= kMaxNmax; ++n) {
                L.cf[q * (kMaxNmax + 1) + n] = c[n];
                cfn[n * nq + q] = c[n];
            }
        }
        __syncthreads();
    }

    // --- moments mu_n(q) = <u_a, u_b>, a + b = n: eight moments (consecutive in the
    // node, so that a row's reads are contiguous) per wavefront, eight lanes per moment
    // over rows r = part (mod 8), combined by lane exchanges in a fixed order
    const int nmom = (n_max - 1) * nq;
    for (int g0 = 8 * wave; g0 < nmom; g0 += 8 * nwave) {
        const int t = g0 + (lane & 7), part = lane >> 3;
        double s = 0.0;
        if (t < nmom) {
            const int n = 2 + t / nq, q = t % nq;
            const int ia = n / 2, ib = n - ia;
            const W* ua = Uat(ia);
            const W* ub = Uat(ib);
            for (int row = part; row < N3; row += 8)
                for (int c = 0; c < 3; ++c)
                    s += double(ua[(size_t)row * ncol + 3 * q + c]) * double(ub[(size_t)row * ncol + 3 * q + c]);
        }
        s += __shfl_xor(s, 8);
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        if (t < nmom && part == 0) L.mu[(2 + t / nq) * nq + t % nq] = s;
    }
    __syncthreads();
    // two-body radii: t2_j = |T2_kj|^2 (into the space of the blend gradients, unused until
    // the force stage), then mu_2 = alpha~_k sum_j alpha~_j t2_j per node, in site order
    // over the lanes of one wavefront per node
    auto t2pair = [&](int i, int j, double& r, double rh[3], LrPair<double>& t) -> bool {
        const double v[3] = {L.px[i] - L.px[j], L.py[i] - L.py[j], L.pz[i] - L.pz[j]};
        r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        const double rc = (i == 0 || j == 0) ? SI.r_2b1 : SI.r_2b2;
        if (i == j || !(r < rc)) return false;
        t = lr_pair<double>(r, a.beta * (L.Rt[i] + L.Rt[j]), a.damp_d, rc, a.r_buf);
        rh[0] = v[0] / r;
        rh[1] = v[1] / r;
        rh[2] = v[2] / r;
        return true;
    };
    if (has2b) {
        for (int j = tid; j < nK; j += blockDim.x) {
            double r, rh[3];
            LrPair<double> t;
            L.fg[j] = t2pair(0, j, r, rh, t) ? (t.A + t.B) * (t.A + t.B) + 2.0 * t.B * t.B : 0.0;
        }
        __syncthreads();
        for (int q = wave; q < nq; q += nwave) {
            double x = 0.0;
            for (int j = lane; j < nK; j += 64) x += L.sa[(size_t)j * nwe + 1 + q] * L.fg[j];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
            if (lane == 0) L.mu[2 * nq + q] = L.sa[1 + q] * x;
        }
        __syncthreads();
    }
    const double wk = a.e_weight ? a.e_weight[k] : 1.0;
    if (tid == 0) {
        double e = 0.0;
        for (int q = 0; q < nq; ++q) {
            double eq = 0.0;
            for (int n = 2; n <= n_max; ++n) eq += cfq(n, q) * L.mu[n * nq + q];
            e += a.wq[q] * eq;
        }
        a.e_atom[k] = e;
    }
    if (!a.forces) return;

    // --- dE/d alpha~_i(w_q) from the moments (row-local Krylov products)
    if (a.paper) {
        // the full n = 2 trace: 2 c_2 sum_j alpha~_j |T_ij|^2, one site per thread over
        // its block row; the central terms of n >= 3 from u_{n-1} and u_1 (the dense form
        // only: the host never runs the approximate forces with the sparse products)
        for (int i = tid; i < nK; i += blockDim.x) {
            L.ab[(size_t)i * nwe] = 0.0;
            for (int q0 = 0; q0 < nq; q0 += 4) {   // four nodes at a time, |T_ij|^2 formed again for each group
                double acc2[4] = {0.0, 0.0, 0.0, 0.0};
                for (int j = 0; j < nK; ++j) {
                    if (j == i) continue;
                    double nrm = 0.0;
                    if (has2b) {   // |T2_ij|^2 = (A + B)^2 + 2 B^2 of the two-body tensor
                        double r, rh[3];
                        LrPair<double> t;
                        if (t2pair(i, j, r, rh, t)) nrm = (t.A + t.B) * (t.A + t.B) + 2.0 * t.B * t.B;
                    } else {
                        for (int r = 0; r < 3; ++r)
                            for (int c = 0; c < 3; ++c) {
                                const double x = double(T[(size_t)(3 * i + r) * N3p + 3 * j + c]);
                                nrm += x * x;
                            }
                    }
#pragma unroll
                    for (int x = 0; x < 4; ++x)
                        if (q0 + x < nq) acc2[x] += L.sa[(size_t)j * nwe + 1 + q0 + x] * nrm;
                }
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const int q = q0 + x;
                    if (q >= nq) continue;
                    double s = 2.0 * cfq(2, q) * acc2[x];
                    double sn = 0.0;
                    for (int n = 3; n <= n_max; ++n) {
                        const W* ua = Uat(n - 1);
                        const W* u1 = Uat(1);
                        double d = (i == 0) ? L.mu[n * nq + q] : 0.0;
                        for (int r = 3 * i; r < 3 * i + 3; ++r)
                            for (int c = 0; c < 3; ++c)
                                d += double(ua[(size_t)r * ncol + 3 * q + c]) * double(u1[(size_t)r * ncol + 3 * q + c]);
                        sn += cfq(n, q) * n * d;
                    }
                    s += sn / L.sa[(size_t)i * nwe + 1 + q];
                    L.ab[(size_t)i * nwe + 1 + q] = wk * a.wq[q] * s;
                }
            }
        }
    } else
    for (int t = tid; t < nK * nwe; t += blockDim.x) {
        const int i = t / nwe, w = t % nwe;
        double v = 0.0;
        if (w > 0) {
            const int q = w - 1;
            double s = 0.0;
            for (int n = 2; n <= n_max; ++n) {
                double sn = (i == 0) ? L.mu[n * nq + q] : 0.0;
                if (n == 2 && has2b) {   // alpha~_k alpha~_i t2_i (the central term is mu_2 itself)
                    if (i > 0) sn = L.sa[1 + q] * L.sa[(size_t)i * nwe + 1 + q] * L.fg[i];
                    s += cfq(n, q) * sn;
                    continue;
                }
                // sum over a = 1 .. n-1 of the row block of u_a u_{n-a}^T: the terms a and
                // n - a are equal, so each unordered pair is formed once
                double pr = 0.0;
                for (int aa = 1; 2 * aa <= n; ++aa) {
                    const W* ua = Uat(aa);
                    const W* ub = Uat(n - aa);
                    double d = 0.0;
                    for (int r = 3 * i; r < 3 * i + 3; ++r)
                        for (int c = 0; c < 3; ++c)
                            d += double(ua[(size_t)r * ncol + 3 * q + c]) * double(ub[(size_t)r * ncol + 3 * q + c]);
                    pr += (2 * aa == n) ? d : 2.0 * d;
                }
                s += cfq(n, q) * (sn + pr);
            }
            v = wk * a.wq[q] * s / L.sa[(size_t)i * nwe + w];
        }
        L.ab[t] = v;
    }
    // --- operands of Tbar = sum_a (D u_a)(W D Z_a)^T, Z_a = sum_b c_{a+b+1} u_b (u_0 = e_k),
    // k-contiguous: P[r][a ncol + col] = sqrt(alpha~_r) u_a[r][col] and
    // Q[s][a ncol + col] = w_k W_q sqrt(alpha~_s) Z_a[s][col]
    // one (row, column) of the Krylov blocks per thread: u_0 .. u_{n_max-1} read
    // once, all n_max column blocks of P and Q written
    // (two instantiations: the common series coefficients are kernel arguments at
    // fixed offsets, the fitted ones LDS entries of the column's node)
    auto build_pq = [&](auto coef) {
        for (int e = tid; e < N3 * ncol; e += blockDim.x) {
            const int r = e / ncol, col = e % ncol, q = col / 3;
            const double sq = L.sqa[(size_t)(r / 3) * nq + q];
            const double scale = wk * a.wq[q] * sq;
            double u[kMaxNmax];
            u[0] = (r == col % 3) ? 1.0 : 0.0;
#pragma unroll
            for (int b = 1; b < kMaxNmax; ++b) u[b] = (b < n_max) ? double(Uat(b)[(size_t)r * ncol + col]) : 0.0;
            W* pr = Pm + (size_t)r * KKp + col;
            W* qr = Qm + (size_t)r * KKp + col;
#pragma unroll
            for (int aa = 0; aa < kMaxNmax; ++aa) {
                if (aa >= n_max) break;
                double z = 0.0;
                if (a.paper) {   // Z_0 = sum_{n>=3} c_n n u_{n-1}; Z_{n-1} = c_n n e_k
#pragma unroll
                    for (int b = 2; b < kMaxNmax; ++b)
                        if (aa == 0 && b <= n_max - 1) z += coef(b + 1, q) * (b + 1) * u[b];
                    if (aa >= 2) z = coef(aa + 1, q) * (aa + 1) * u[0];
                } else {
#pragma unroll
                    for (int b = 0; b < kMaxNmax; ++b)
                        if ((b > 0 || aa >= 1) && b <= n_max - 1 - aa) z += coef(min(aa + b + 1, kMaxNmax), q) * u[b];
                }
                pr[(size_t)aa * ncol] = W(sq * u[aa]);
                qr[(size_t)aa * ncol] = W(scale * z);
            }
        }
    };
    if (fit)
        build_pq([&](int n, int q) { return (has2b && n == 2) ? 0.0 : L.cf[q * (kMaxNmax + 1) + n]; });
    else
        build_pq([&](int n, int) { return (has2b && n == 2) ? 0.0 : a.coef[n]; });
    for (int e = tid; e < N3 * (KKp - KK); e += blockDim.x) {   // padding columns
        const int r = e / (KKp - KK), kk = KK + e % (KKp - KK);
        Pm[(size_t)r * KKp + kk] = W(0);
        Qm[(size_t)r * KKp + kk] = W(0);
    }
    __syncthreads();
    // --- Tbar (overwrites T).  Tbar is symmetric (the terms a, b and b, a of
    // Gbar are transposes of each other), so only blocks on or below the
    // diagonal are formed and read.
    if constexpr (!SP) {
        if (a.paper && !has2b) {   // Tbar += 2 w_k sum_q c_2(q) W_q D_q^2 T D_q^2, read from T before it is overwritten
            const double c2 = 2.0 * wk;
            mfma_gemm_nt<3, 3, W>(N3, N3, KKp, Pm, KKp, Qm, KKp, true, [&](int r, int s, W v) {
                const size_t e = (size_t)r * N3p + s;
                const double t = double(T[e]);
                double f = 0.0;
                if (t != 0.0)
                    for (int q = 0; q < nq; ++q)
                        f += a.wq[q] * cfq(2, q) * L.sa[(size_t)(r / 3) * nwe + 1 + q] *
                             L.sa[(size_t)(s / 3) * nwe + 1 + q];
                T[e] = W(double(v) + c2 * t * f);
            });
        } else {
            mfma_gemm_nt<3, 3, W>(N3, N3, KKp, Pm, KKp, Qm, KKp, true, [&](int r, int s, W v) { T[(size_t)r * N3p + s] = v; });
        }
    }

    // --- pair contraction: dE/dp_i and dE/dR~_i (each unordered pair from both ends)
    const int parts = SP ? 1 : max(1, min(4, (int)blockDim.x / max(nK, 1)));
    // the two-body term's pair derivative C2 = kappa T2_ij, kappa = 2 w_k sum_q W_q c_2
    // alpha~_i alpha~_j (central pairs; 4 and every pair for the approximate forces),
    // contracted with dT2/dp_i and, through S~, with dT2/dR~
    auto add2b = [&](int i, int j, double g[3], double& Rb) {
        if (!has2b || (!a.paper && i != 0 && j != 0)) return;
        double r, rh[3];
        LrPair<double> t;
        if (!t2pair(i, j, r, rh, t)) return;
        double kap = 0.0;
        for (int q = 0; q < nq; ++q)
            kap += a.wq[q] * cfq(2, q) * L.sa[(size_t)i * nwe + 1 + q] * L.sa[(size_t)j * nwe + 1 + q];
        kap *= (a.paper ? 4.0 : 2.0) * wk;
        double C[9];
        for (int x = 0; x < 3; ++x)
            for (int c = 0; c < 3; ++c) C[3 * x + c] = kap * (t.A * rh[x] * rh[c] + (x == c ? t.B : 0.0));
        double gp[3];
        radial_tensor_grad(rh, r, t.A, t.dA, t.dB, C, gp);
        g[0] += gp[0];
        g[1] += gp[1];
        g[2] += gp[2];
        Rb += a.beta * t.fLR * t.dfS * 2.0 * kap * t.A / (r * r * r);   // <C2, T_dip> = 2 kappa A / r^3
    };
    if constexpr (GS) {
        // Each unordered coupled pair once (the neighbourhoods of this form are large and
        // the contraction is bound by the gathers of P and Q rows): pass 1, one block row
        // i per wavefront over its partners j < i (a prefix of the sorted row), forms
        // Tbar_ij = P_i Q_j^T, C = Tbar_ij + Tbar_ij^T and the pair's terms (its gradient
        // with respect to r_i and its R~ term) into the entry's slot of a pair buffer.
        // Pass 2 sums every row over its partners in list order, reading the partner's
        // slot (found by binary search in the partner's sorted row) with the gradient's
        // sign turned for j > i: the gradient of a pair term is odd in rhat, the R~ term
        // even.  The sums have a fixed order, as in the other forms.  The buffer (four
        // values of the arithmetic type per entry) takes the place of the entries' T_LR
        // coefficients, which the products before have used for the last time.
        W* const pbuf = pA;
        constexpr int VW = 16 / sizeof(W);
        typedef W VV __attribute__((ext_vector_type(VW)));
        const int pu = lane >> 3, pt = lane & 7;
        for (int i = wave; i < nK; i += nwave) {
            const int n = row_len(i);
            const size_t e0 = (size_t)roff[i];
            int nlo = 0;   // partners below i
            for (int s0 = 0; s0 < n; s0 += 64) nlo += __popcll(__ballot(s0 + lane < n && pj[e0 + s0 + lane] < i));
            // eight pairs per step, eight lanes per pair (as in the LDS form)
            for (int s0 = 0; s0 < nlo; s0 += 8) {
                const bool okp = s0 + pu < nlo;
                const int j = pj[e0 + (okp ? s0 + pu : s0)];
                double sb[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                for (int kb = 0; kb < KKp; kb += 8 * VW) {
                    const int kk = kb + VW * pt;
                    const int ks = kk < KKp ? kk : 0;
                    const double z = kk < KKp ? 1.0 : 0.0;
                    VV pv[3], qv[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        pv[c] = *reinterpret_cast<const VV*>(Pm + (size_t)(3 * i + c) * KKp + ks);
                        qv[c] = *reinterpret_cast<const VV*>(Qm + (size_t)(3 * j + c) * KKp + ks);
                    }
#pragma unroll
                    for (int x = 0; x < 3; ++x)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            double d = 0.0;
#pragma unroll
                            for (int v = 0; v < VW; ++v) d += double(pv[x][v]) * double(qv[c][v]);
                            sb[3 * x + c] += z * d;
                        }
                }
#pragma unroll
                for (int x = 0; x < 9; ++x) {
                    sb[x] += __shfl_xor(sb[x], 1);
                    sb[x] += __shfl_xor(sb[x], 2);
                    sb[x] += __shfl_xor(sb[x], 4);
                }
                if (okp && pt == 0) {
                    double C[9];
                    for (int x = 0; x < 3; ++x)
                        for (int c = 0; c < 3; ++c) C[3 * x + c] = sb[3 * x + c] + sb[3 * c + x];
                    const double v[3] = {L.px[i] - L.px[j], L.py[i] - L.py[j], L.pz[i] - L.pz[j]};
                    const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                    const double rcut = (i == 0 || j == 0) ? SI.r_mbd1 : SI.r_mbd2;
                    const double rh[3] = {v[0] / r, v[1] / r, v[2] / r};
                    const LrPair<W> lp = lr_pair<W>(W(r), W(a.beta * (L.Rt[i] + L.Rt[j])), W(a.damp_d), W(rcut),
                                                    W(a.r_buf));
                    double gp[3];
                    radial_tensor_grad(rh, r, double(lp.A), double(lp.dA), double(lp.dB), C, gp);
                    double rCr = 0.0;
                    for (int x = 0; x < 3; ++x)
                        for (int c = 0; c < 3; ++c) rCr += rh[x] * C[3 * x + c] * rh[c];
                    const double ct = (3.0 * rCr - (C[0] + C[4] + C[8])) / (r * r * r);
                    W* slot = pbuf + (e0 + s0 + pu) * 4;
                    slot[0] = W(gp[0]);
                    slot[1] = W(gp[1]);
                    slot[2] = W(gp[2]);
                    slot[3] = W(a.beta * double(lp.fLR) * double(lp.dfS) * ct);
                }
            }
        }
        __syncthreads();   // the pair buffer is complete
        for (int i = wave; i < nK; i += nwave) {
            double g[3] = {0.0, 0.0, 0.0};
            double Rb = 0.0;
            const int n = row_len(i);
            const size_t e0 = (size_t)roff[i];
            for (int s0 = 0; s0 < n; s0 += 64) {
                // the slot of entry s0 + lane (every lane), then the sums in the order of
                // eight pairs per step, pair u of a step on lane 8u
                long long src = -1;
                bool neg = false;
                if (s0 + lane < n) {
                    const int j = pj[e0 + s0 + lane];
                    if (j < i) {
                        src = (long long)(e0 + s0 + lane);
                    } else {
                        int lo = roff[j], hi = roff[j] + row_len(j);
                        const int end = hi;
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (pj[mid] < i) lo = mid + 1;
                            else hi = mid;
                        }
                        if (lo < end && pj[lo] == i) {
                            src = lo;
                            neg = true;
                        } else {   // the coupling relation is symmetric: never taken
                            atomicOr(a.err, 32);
                            atomicMin(a.err_atom, k);
                        }
                    }
                }
                for (int t = 0; t < 8; ++t) {
                    const int from = 8 * t + pu;
                    const long long sr = __shfl(src, from);
                    const bool ng = __shfl((int)neg, from) != 0;
                    if (pt == 0 && s0 + from < n && sr >= 0) {
                        const W* slot = pbuf + (size_t)sr * 4;
                        const double sg = ng ? -1.0 : 1.0;
                        g[0] += sg * double(slot[0]);
                        g[1] += sg * double(slot[1]);
                        g[2] += sg * double(slot[2]);
                        Rb += double(slot[3]);
                    }
                }
            }
            {   // the lanes' partial sums, in a fixed order
                const double part[9] = {g[0], g[1], g[2], Rb, 0.0, 0.0, 0.0, 0.0, 0.0};
                double tot[9];
                wave_sum9(part, tot);
                if (lane == 0) {
                    L.g[(size_t)i * 3 + 0] = tot[0];
                    L.g[(size_t)i * 3 + 1] = tot[1];
                    L.g[(size_t)i * 3 + 2] = tot[2];
                    L.rb[i] = tot[3];
                }
            }
        }
    } else if constexpr (SP) {
        // one block row per wavefront; Tbar_IJ (I > J) of a coupled pair from P and Q
        for (int i = wave; i < nK; i += nwave) {
            double g[3] = {0.0, 0.0, 0.0};
            double Rb = 0.0;
            const int n = row_len(i);
            // eight coupled pairs per step, eight lanes per pair: lane 8u + t sums columns
            // t, t + 8, ... (16 bytes each) of pair u's nine dot products; the eight lanes of
            // a pair then combine their sums and the pair's first lane takes its tail
            constexpr int VW = 16 / sizeof(W);
            typedef W VV __attribute__((ext_vector_type(VW)));
            const int pu = lane >> 3, pt = lane & 7;
            for (int s0 = 0; s0 < n; s0 += 8) {
                const bool okp = s0 + pu < n;
                const int j = pj[(size_t)roff[i] + (okp ? s0 + pu : s0)];
                const int I = max(i, j), J = min(i, j);
                double sb[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                for (int kb = 0; kb < KKp; kb += 8 * VW) {
                    const int kk = kb + VW * pt;
                    const int ks = kk < KKp ? kk : 0;
                    const double z = kk < KKp ? 1.0 : 0.0;
                    VV pv[3], qv[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        pv[c] = *reinterpret_cast<const VV*>(Pm + (size_t)(3 * I + c) * KKp + ks);
                        qv[c] = *reinterpret_cast<const VV*>(Qm + (size_t)(3 * J + c) * KKp + ks);
                    }
#pragma unroll
                    for (int x = 0; x < 3; ++x)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            double d = 0.0;
#pragma unroll
                            for (int v = 0; v < VW; ++v) d += double(pv[x][v]) * double(qv[c][v]);
                            sb[3 * x + c] += z * d;
                        }
                }
#pragma unroll
                for (int x = 0; x < 9; ++x) {
                    sb[x] += __shfl_xor(sb[x], 1);
                    sb[x] += __shfl_xor(sb[x], 2);
                    sb[x] += __shfl_xor(sb[x], 4);
                }
                double myC[9];
                for (int x = 0; x < 3; ++x)
                    for (int c = 0; c < 3; ++c) myC[3 * x + c] = sb[3 * x + c] + sb[3 * c + x];
                const int myj = (okp && pt == 0) ? j : -1;
                if (myj >= 0) {
                    const int j = myj;
                    const double* C = myC;
                    const double v[3] = {L.px[i] - L.px[j], L.py[i] - L.py[j], L.pz[i] - L.pz[j]};
                    const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                    const double rcut = (i == 0 || j == 0) ? SI.r_mbd1 : SI.r_mbd2;
                    const double rh[3] = {v[0] / r, v[1] / r, v[2] / r};
                    const LrPair<W> lp = lr_pair<W>(W(r), W(a.beta * (L.Rt[i] + L.Rt[j])), W(a.damp_d), W(rcut),
                                                    W(a.r_buf));
                    double gp[3];
                    radial_tensor_grad(rh, r, double(lp.A), double(lp.dA), double(lp.dB), C, gp);
                    g[0] += gp[0];
                    g[1] += gp[1];
                    g[2] += gp[2];
                    double rCr = 0.0;
                    for (int x = 0; x < 3; ++x)
                        for (int c = 0; c < 3; ++c) rCr += rh[x] * C[3 * x + c] * rh[c];
                    const double ct = (3.0 * rCr - (C[0] + C[4] + C[8])) / (r * r * r);
                    Rb += a.beta * double(lp.fLR) * double(lp.dfS) * ct;
                }
            }
            {   // the lanes' partial sums, in a fixed order
                const double part[9] = {g[0], g[1], g[2], Rb, 0.0, 0.0, 0.0, 0.0, 0.0};
                double tot[9];
                wave_sum9(part, tot);
                g[0] = tot[0];
                g[1] = tot[1];
                g[2] = tot[2];
                Rb = tot[3];
            }
            if (lane == 0) {
                L.g[(size_t)i * 3 + 0] = g[0];
                L.g[(size_t)i * 3 + 1] = g[1];
                L.g[(size_t)i * 3 + 2] = g[2];
                L.rb[i] = Rb;
            }
        }
    } else
    for (int t = tid; t < nK * parts; t += blockDim.x) {
        const int i = t % nK, part = t / nK;
        double g[3] = {0.0, 0.0, 0.0};
        double Rb = 0.0;
        for (int j = part; j < nK; j += parts) {
            if (j == i) continue;
            const double v[3] = {L.px[i] - L.px[j], L.py[i] - L.py[j], L.pz[i] - L.pz[j]};
            const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            const double rcut = (i == 0 || j == 0) ? SI.r_mbd1 : SI.r_mbd2;
            if (!(r < rcut)) continue;
            const double rh[3] = {v[0] / r, v[1] / r, v[2] / r};
            const LrPair<W> lp = lr_pair<W>(W(r), W(a.beta * (L.Rt[i] + L.Rt[j])), W(a.damp_d), W(rcut),
                                            W(a.r_buf));
            // C = Tbar_ij + Tbar_ji = Tbar_IJ + Tbar_IJ^T with I > J
            const int I = max(i, j), J = min(i, j);
            double C[9];
            for (int q = 0; q < 3; ++q)
                for (int c = 0; c < 3; ++c)
                    C[3 * q + c] = double(T[(size_t)(3 * I + q) * N3p + 3 * J + c]) +
                                   double(T[(size_t)(3 * I + c) * N3p + 3 * J + q]);
            double gp[3];
            radial_tensor_grad(rh, r, double(lp.A), double(lp.dA), double(lp.dB), C, gp);
            g[0] += gp[0];
            g[1] += gp[1];
            g[2] += gp[2];
            // <C, T_ij> with T = (3 rhat rhat^T - I)/r^3, times fLR df/dS~
            double rCr = 0.0;
            for (int q = 0; q < 3; ++q)
                for (int c = 0; c < 3; ++c) rCr += rh[q] * C[3 * q + c] * rh[c];
            const double ct = (3.0 * rCr - (C[0] + C[4] + C[8])) / (r * r * r);
            Rb += a.beta * double(lp.fLR) * double(lp.dfS) * ct;
        }
        L.g[(size_t)(part * nK + i) * 3 + 0] = g[0];
        L.g[(size_t)(part * nK + i) * 3 + 1] = g[1];
        L.g[(size_t)(part * nK + i) * 3 + 2] = g[2];
        L.rb[(size_t)part * nK + i] = Rb;
    }
    __syncthreads();
    if (has2b) {   // the two-body term's pairs, each from both ends, one site per thread
        for (int i = tid; i < nK; i += blockDim.x) {
            double g[3] = {0.0, 0.0, 0.0}, Rb = 0.0;
            if (a.paper || i == 0)
                for (int j = 0; j < nK; ++j) add2b(i, j, g, Rb);
            else
                add2b(i, 0, g, Rb);
            L.g[(size_t)i * 3 + 0] += g[0];
            L.g[(size_t)i * 3 + 1] += g[1];
            L.g[(size_t)i * 3 + 2] += g[2];
            L.rb[i] += Rb;
        }
        __syncthreads();
    }
    // reduce the parts in a fixed order; R~ adjoint into alpha~(0); blend adjoint
    double* abl = a.abar_loc + a.aloc_off[k];
    double* cap = a.ca + a.site_off[k] * nw;
    for (int i = tid; i < nK; i += blockDim.x) {
        double g0 = 0.0, g1 = 0.0, g2 = 0.0, Rb = 0.0;
        for (int part = 0; part < parts; ++part) {
            g0 += L.g[(size_t)(part * nK + i) * 3 + 0];
            g1 += L.g[(size_t)(part * nK + i) * 3 + 1];
            g2 += L.g[(size_t)(part * nK + i) * 3 + 2];
            Rb += L.rb[(size_t)part * nK + i];
        }
        // R~_i = R0 (alpha~_i(0)/alpha0)^(1/3): dR~/d alpha~(0) = R~ / (3 alpha~(0))
        L.ab[(size_t)i * nwe] += Rb * L.Rt[i] / (3.0 * L.sa[(size_t)i * nwe]);
        const Site st = S[i];
        const double* cen = a.alpha_loc + a.aloc_off[st.base];
        if (a.lorentz) {
            // back through the two-point model onto alpha~_i(0) and alpha~_i(w_ref)
            const double fsv = L.fs[i];
            const double a0 = L.sa[(size_t)i * nwe];
            const double ar = (i == 0) ? aloc[1] : (i < n1) ? (1.0 - fsv) * aloc[(size_t)i * nw + 1] + fsv * cen[1] : cen[1];
            double b0 = L.ab[(size_t)i * nwe], br = 0.0;
            for (int q = 0; q < nq; ++q) {
                const double v = L.sa[(size_t)i * nwe + 1 + q], g = L.ab[(size_t)i * nwe + 1 + q];
                b0 += g * (1.0 - a.rho[q]) * (v / a0) * (v / a0);
                br += g * a.rho[q] * (v / ar) * (v / ar);
            }
            L.ab[(size_t)i * nwe] = b0;
            L.ab[(size_t)i * nwe + 1] = br;
        }
        double gf = 0.0;  // sum_w abar_i(w) (alpha~_I,i(w) - alpha~_K,i(w))
        for (int w = 0; w < nw; ++w) {
            const double ai = L.ab[(size_t)i * nwe + w];
            // (the approximate forces hold the central polarisabilities fixed: nothing is scattered)
            if (i == 0) {
                abl[w] = ai;
                cap[w] = 0.0;
            } else if (i < n1) {
                abl[(size_t)i * nw + w] = (1.0 - L.fs[i]) * ai;
                cap[(size_t)i * nw + w] = a.paper ? 0.0 : L.fs[i] * ai;
                gf += ai * (cen[w] - aloc[(size_t)i * nw + w]);
            } else {
                cap[(size_t)i * nw + w] = a.paper ? 0.0 : ai;
            }
        }
        // f_SCS(r_ik), r_ik = |p_i| (the central atom sits at the origin)
        double fg[3] = {0.0, 0.0, 0.0};
        if (i > 0 && i < n1) {
            const double r = sqrt(L.px[i] * L.px[i] + L.py[i] * L.py[i] + L.pz[i] * L.pz[i]);
            const double c = L.dfs[i] * gf / r;
            fg[0] = c * L.px[i];
            fg[1] = c * L.py[i];
            fg[2] = c * L.pz[i];
        }
        L.fg[(size_t)i * 3 + 0] = fg[0];
        L.fg[(size_t)i * 3 + 1] = fg[1];
        L.fg[(size_t)i * 3 + 2] = fg[2];
        L.g[(size_t)i * 3 + 0] = g0 + fg[0];
        L.g[(size_t)i * 3 + 1] = g1 + fg[1];
        L.g[(size_t)i * 3 + 2] = g2 + fg[2];
    }
    // local polarisabilities of K1 sites outside K carry no energy adjoint
    for (int e = tid; e < (n1 > nK ? (n1 - nK) * nw : 0); e += blockDim.x) abl[(size_t)nK * nw + e] = 0.0;
    __syncthreads();
    double* out = a.cf0 + a.site_off[k] * 3;
    const double fconv = -1.0 / kBohr;  // force = -dE/dx per Angstrom
    if (tid == 0) {
        // moving the central atom changes every r_ik of the blend
        double c0 = 0.0, c1 = 0.0, c2 = 0.0;
        for (int i = 1; i < nK; ++i) {
            c0 += L.fg[(size_t)i * 3 + 0];
            c1 += L.fg[(size_t)i * 3 + 1];
            c2 += L.fg[(size_t)i * 3 + 2];
        }
        out[0] = fconv * (L.g[0] - c0);
        out[1] = fconv * (L.g[1] - c1);
        out[2] = fconv * (L.g[2] - c2);
    }
    for (int s = 1 + tid; s < nall; s += blockDim.x) {
        const bool in = s < nK;
        out[3 * s + 0] = in ? fconv * L.g[(size_t)s * 3 + 0] : 0.0;
        out[3 * s + 1] = in ? fconv * L.g[(size_t)s * 3 + 1] : 0.0;
        out[3 * s + 2] = in ? fconv * L.g[(size_t)s * 3 + 2] : 0.0;
    }
    for (int e = tid; e < (nall - nK) * nw; e += blockDim.x) cap[(size_t)nK * nw + e] = 0.0;
}

template <typename W, bool TB>
static void launch_mbd_t(hipStream_t st, const MbdArgs& a, int nk_lds, size_t lds, int form) {
    const dim3 grid(a.n), blk(form == kMbdDense ? kMbdThreads : kMbdThreadsSparse);
    if (form == kMbdDense)
        hipLaunchKernelGGL((k_mbd<W, kMbdDense, TB>), grid, blk, lds, st, a, nk_lds);
    else if (form == kMbdSparse)
        hipLaunchKernelGGL((k_mbd<W, kMbdSparse, TB>), grid, blk, lds, st, a, nk_lds);
    else
        hipLaunchKernelGGL((k_mbd<W, kMbdSparseGlobal, TB>), grid, blk, lds, st, a, nk_lds);
}

hipError_t launch_mbd(hipStream_t st, const MbdArgs& a, int nkmax, bool mixed, int form, bool two_body) {
    const int nk_lds = form == kMbdSparseGlobal ? 0 : nkmax;   // per-site arrays in LDS or not
    const size_t lds = mbd_lds_bytes(nk_lds, a.nq, a.n_max, a.lz_steps, a.fit != 0);
    if (mixed) {
        if (two_body) launch_mbd_t<float, true>(st, a, nk_lds, lds, form);
        else launch_mbd_t<float, false>(st, a, nk_lds, lds, form);
    } else {
        if (two_body) launch_mbd_t<double, true>(st, a, nk_lds, lds, form);
        else launch_mbd_t<double, false>(st, a, nk_lds, lds, form);
    }
    return hipGetLastError();
}

}  // namespace lmbd
