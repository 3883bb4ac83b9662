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
// breakdown reported to the host.
//
// Precision: the kernels are templated on the matrix type R.  R = double is the
// plain FP64 path.  R = float is the mixed path: pair tensors, the matrix and
// its factor in FP32 (MFMA f32), the forward solve refined in FP64 against the
// matrix rebuilt from its FP32 pair coefficients, solutions and all sums in FP64.
#include "lmbd_internal.h"

namespace lmbd {

constexpr int NB = 16;      // block size of the factorisation
constexpr int kParts = 4;   // partner-range splits of the per-site pair loops (adjoint)
constexpr int kPartsD = 2;  // partner-range splits of the right-hand-side assembly

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
    int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
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
// Left-looking blocked Cholesky of the N x N lower triangle of A (column-major,
// leading dimension ld) by one workgroup, 16-column panels:
//   A[c0:N, c0:c0+16] -= L[c0:N, 0:c0] L[c0:c0+16, 0:c0]^T     (MFMA 16x16x4)
//   L_pp = chol(A_pp)                                          (one wavefront, shuffles)
//   L[c0+16:N, c0:c0+16] = A[c0+16:N, c0:c0+16] L_pp^{-T}       (one row per thread)
// The update reads the finished columns with coalesced row segments and writes
// each panel element once; the strict upper triangle is never touched.  D is a
// 16x16 LDS block.
// ---------------------------------------------------------------------------
template <typename R>
__device__ void chol_factor(R* __restrict__ A, int N, int ld, R* D, bool& ok) {
    typedef Mfma<R> M;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwave = nthr >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nt = (N + NB - 1) / NB;
    bool good = true;
    for (int p = 0; p < nt; ++p) {
        const int c0 = p * NB;
        const int jb = min(NB, N - c0);
        // (1) panel update, one 16x16 row tile per wavefront at a time
        if (c0 > 0) {
            for (int r = p + wave; r < nt; r += nwave) {
                const int R0 = r * NB;
                typename M::acc acc;
                const int col = c0 + li;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = R0 + M::acc_row(lk, q);
                    acc[q] = (row < N && col < N && row >= col) ? A[(size_t)col * ld + row] : R(0);
                }
                const int arow = R0 + li;
                const bool arow_ok = arow < N;
                const bool bcol_ok = col < N;
#pragma unroll 4
                for (int k0 = 0; k0 < c0; k0 += 4) {
                    const size_t kc = (size_t)(k0 + lk) * ld;
                    const R a = arow_ok ? -A[kc + arow] : R(0);
                    const R b = bcol_ok ? A[kc + col] : R(0);
                    acc = M::mma(a, b, acc);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = R0 + M::acc_row(lk, q);
                    if (row < N && col < N && row >= col) A[(size_t)col * ld + row] = acc[q];
                }
            }
            __syncthreads();
        }
        // (2) diagonal block: wavefront 0, lane l holds row l of the block
        if (tid < 64) {
            const int l = tid;
            R row[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const bool valid = (l < jb) && (c <= l);
                row[c] = valid ? A[(size_t)(c0 + c) * ld + c0 + l] : (l == c ? R(1) : R(0));
            }
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const R dcc = __shfl(row[c], c, 64);
                if (c < jb && !(dcc > R(0))) good = false;
                const R sq = m_sqrt(dcc);
                const R inv = R(1) / sq;
                if (l == c) row[c] = sq;
                else if (l > c) row[c] *= inv;
#pragma unroll
                for (int s = c + 1; s < NB; ++s) {
                    const R lsc = __shfl(row[c], s, 64);
                    if (l >= s) row[s] -= row[c] * lsc;
                }
            }
            if (l < NB) {
#pragma unroll
                for (int c = 0; c < NB; ++c) D[l * NB + c] = (c <= l) ? row[c] : R(0);
            }
            if (l < jb) {
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    if (c <= l) A[(size_t)(c0 + c) * ld + c0 + l] = row[c];
            }
        }
        __syncthreads();
        // (3) rows below the block: X L_pp^T = A_panel, one row per thread
        for (int i = c0 + jb + tid; i < N; i += nthr) {
            R x[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) x[c] = (c < jb) ? A[(size_t)(c0 + c) * ld + i] : R(0);
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                if (c < jb) {
                    R s = x[c];
#pragma unroll
                    for (int q = 0; q < c; ++q) s -= x[q] * D[c * NB + q];
                    x[c] = s / D[c * NB + c];
                }
            }
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < jb) A[(size_t)(c0 + c) * ld + i] = x[c];
        }
        __syncthreads();
    }
    ok = good;
}

// Solve L L^T Y = Y in place for 3 right-hand sides (Y: LDS, row-major N x 3).
// Each 16x16 diagonal block is solved by one wavefront with shuffles (lane
// r + 16 c holds row r, right-hand side c); the coupling to the other rows is
// one row per thread.
template <typename R>
__device__ void chol_solve3(const R* __restrict__ A, int N, int ld, R* Y) {
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int nt = (N + NB - 1) / NB;
    for (int p = 0; p < nt; ++p) {  // forward: L y = b
        const int c0 = p * NB;
        const int jb = min(NB, N - c0);
        if (tid < 64) {
            const int r = tid & 15, c = tid >> 4;
            const bool act = (c < 3) && (r < jb);
            R Lrow[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) Lrow[q] = (act && q <= r) ? A[(size_t)(c0 + q) * ld + c0 + r] : R(0);
            R y = act ? Y[(c0 + r) * 3 + c] : R(0);
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const R diag = __shfl(Lrow[j], (tid & 48) + j, 64);
                const R xj = __shfl(y, (tid & 48) + j, 64) / diag;
                if (r == j) y = xj;
                else if (r > j) y -= Lrow[j] * xj;
            }
            if (act) Y[(c0 + r) * 3 + c] = y;
        }
        __syncthreads();
        for (int i = c0 + jb + tid; i < N; i += nthr) {
            R s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                if (q < jb) {
                    const R l = A[(size_t)(c0 + q) * ld + i];
                    s0 += l * Y[(c0 + q) * 3 + 0];
                    s1 += l * Y[(c0 + q) * 3 + 1];
                    s2 += l * Y[(c0 + q) * 3 + 2];
                }
            }
            Y[i * 3 + 0] -= s0;
            Y[i * 3 + 1] -= s1;
            Y[i * 3 + 2] -= s2;
        }
        __syncthreads();
    }
    for (int p = nt - 1; p >= 0; --p) {  // backward: L^T x = y
        const int c0 = p * NB;
        const int jb = min(NB, N - c0);
        if (tid < 64) {
            const int r = tid & 15, c = tid >> 4;
            const bool act = (c < 3) && (r < jb);
            R Lcol[NB];  // column r of the block: L[c0 + q][c0 + r]
#pragma unroll
            for (int q = 0; q < NB; ++q) Lcol[q] = (act && q >= r && q < jb) ? A[(size_t)(c0 + r) * ld + c0 + q] : R(0);
            R y = act ? Y[(c0 + r) * 3 + c] : R(0);
#pragma unroll
            for (int j = NB - 1; j >= 0; --j) {
                const R diag = __shfl(Lcol[j], (tid & 48) + j, 64);
                const R xj = __shfl(y, (tid & 48) + j, 64) / diag;
                if (j < jb) {
                    if (r == j) y = xj;
                    else if (r < j) y -= Lcol[j] * xj;
                }
            }
            if (act) Y[(c0 + r) * 3 + c] = y;
        }
        __syncthreads();
        for (int i = tid; i < c0; i += nthr) {
            R s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                if (q < jb) {
                    const R l = A[(size_t)i * ld + c0 + q];
                    s0 += l * Y[(c0 + q) * 3 + 0];
                    s1 += l * Y[(c0 + q) * 3 + 1];
                    s2 += l * Y[(c0 + q) * 3 + 2];
                }
            }
            Y[i * 3 + 0] -= s0;
            Y[i * 3 + 1] -= s1;
            Y[i * 3 + 2] -= s2;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// LDS layout.  K1 sites, then a union region (shell sites and the per-site
// reduction area during the right-hand-side assembly; FP32 pair coefficients
// of B~ afterwards, mixed path only), right-hand sides / solutions (FP64), the
// solve buffer in the matrix type, and the 16x16 diagonal block.
// ---------------------------------------------------------------------------
struct ScsLds {
    double *px, *py, *pz, *ab, *sg, *R;        // K1 sites
    double *qx, *qy, *qz, *qab, *qsg, *qR;     // shell sites (union region)
    double* red;                               // reduction area (union region)
    float* coef;                               // pair coefficients (A, B) of B~ (union region)
    double *Y, *X;
    void* Yr;                                  // solve buffer (matrix type)
    void* D;                                   // 16x16 block (matrix type)
};

__device__ __host__ inline size_t scs_union_doubles(int n1max, int n2max, bool mixed) {
    const size_t red = (kParts * 3 > kPartsD * 9 ? kParts * 3 : kPartsD * 9) * (size_t)n1max;
    const size_t a = 6 * (size_t)n2max + red;
    const size_t coef = mixed ? ((size_t)n1max * (n1max + 1) / 2) : 0;  // 2 floats = 1 double each
    return a > coef ? a : coef;
}

__device__ inline ScsLds scs_lds(double* base, int n1max, int n2max, bool mixed) {
    const int N = 3 * n1max;
    ScsLds L;
    L.px = base;
    L.py = L.px + n1max;
    L.pz = L.py + n1max;
    L.ab = L.pz + n1max;
    L.sg = L.ab + n1max;
    L.R = L.sg + n1max;
    double* u = L.R + n1max;
    L.qx = u;
    L.qy = L.qx + n2max;
    L.qz = L.qy + n2max;
    L.qab = L.qz + n2max;
    L.qsg = L.qab + n2max;
    L.qR = L.qsg + n2max;
    L.red = L.qR + n2max;
    L.coef = reinterpret_cast<float*>(u);
    L.Y = u + scs_union_doubles(n1max, n2max, mixed);
    L.X = L.Y + 3 * N;
    L.Yr = L.X + 3 * N;
    L.D = L.X + 6 * N;   // Yr takes at most 3N doubles
    return L;
}

size_t scs_lds_bytes(int n1max, int n2max, bool mixed) {
    const size_t N = 3 * (size_t)n1max;
    return sizeof(double) * (6 * (size_t)n1max + scs_union_doubles(n1max, n2max, mixed) + 9 * N + NB * NB);
}

__device__ inline void load_sites(const ScsArgs& a, int k, int w, int n1, int n12, const ScsLds& L) {
    const Site* S = a.sites + a.site_off[k];
    for (int s = threadIdx.x; s < n12; s += blockDim.x) {
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

template <typename R>
__global__ void __launch_bounds__(256) k_scs_forward(ScsArgs a, int n1max, int n2max) {
    extern __shared__ double lds[];
    constexpr bool mixed = sizeof(R) == 4;
    const int k = blockIdx.x;
    const int w = blockIdx.y;
    const Counts cnt = a.counts[k];
    const int n1 = cnt.n1, n12 = cnt.n12;
    const int N = 3 * n1;
    const int ld = a.fac_ld[k];
    const StructInfo& SI = a.sinfo[a.atom_struct[k]];
    const double rc = SI.r_scs;
    ScsLds L = scs_lds(lds, n1max, n2max, mixed);
    R* A = static_cast<R*>(a.fac) + a.fac_off[k] + (size_t)w * ld * N;
    R* Yr = static_cast<R*>(L.Yr);
    R* D = static_cast<R*>(L.D);
    load_sites(a, k, w, n1, n12, L);
    __syncthreads();

    // d: the shell K2 (TS polarisabilities, f_inner), over the compact list of
    // coupled (K1 site, shell site) pairs; each site's segment is split over
    // kPartsD threads and recombined in a fixed order.
    const int32_t* seg_i = a.pl_seg + a.site_off[k] + 2 * (int64_t)k;
    const int32_t* li = a.pl_i + a.pl_off[k];
    for (int t = threadIdx.x; t < n1 * kPartsD; t += blockDim.x) {
        const int i = t % n1, part = t / n1;
        double d[9] = {};
        for (int e = seg_i[i] + part; e < seg_i[i + 1]; e += kPartsD) {
            const int q = li[e] & 0xFFFF;
            double rh[3], r;
            const SrPair<R> tp = k2_pair<R>(a, L, i, q, rc, rh, r);
            const double A_ = tp.A, B_ = tp.B, ab = L.qab[q];
            for (int e2 = 0; e2 < 3; ++e2)
                for (int c = 0; c < 3; ++c) d[3 * e2 + c] -= ab * (A_ * rh[e2] * rh[c] + (e2 == c ? B_ : 0.0));
        }
        for (int e = 0; e < 9; ++e) L.red[(size_t)(part * n1 + i) * 9 + e] = d[e];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n1; i += blockDim.x) {
        for (int e = 0; e < 9; ++e) {
            double v = (e == 0 || e == 4 || e == 8) ? 1.0 : 0.0;
            for (int part = 0; part < kPartsD; ++part) v += L.red[(size_t)(part * n1 + i) * 9 + e];
            L.Y[(3 * i + e / 3) * 3 + e % 3] = v;
        }
    }
    __syncthreads();  // the union region is free from here on

    // B~ (lower triangle, block by block); the mixed path keeps the FP32 pair
    // coefficients in LDS for the refinement residual
    const int npairs = n1 * (n1 + 1) / 2;
    for (int p = threadIdx.x; p < npairs; p += blockDim.x) {
        int i, j;
        tri_decode(p, i, j);
        if (i == j) {
            const R inv = R(1.0 / L.ab[i]);
            for (int q = 0; q < 3; ++q)
                for (int r = q; r < 3; ++r) A[(size_t)(3 * i + q) * ld + 3 * i + r] = (q == r) ? inv : R(0);
            if (mixed) { L.coef[2 * p] = 0.f; L.coef[2 * p + 1] = 0.f; }
            continue;
        }
        double rh[3], r;
        const SrPair<R> t = k1_pair<R>(a, L, i, j, rc, rh, r);
        if (mixed) {
            L.coef[2 * p] = (float)t.A;
            L.coef[2 * p + 1] = (float)t.B;
        }
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c)
                A[(size_t)(3 * j + c) * ld + 3 * i + q] = R(double(t.A) * rh[q] * rh[c] + (q == c ? double(t.B) : 0.0));
    }
    __syncthreads();

    bool ok = true;
    chol_factor<R>(A, N, ld, D, ok);
    if (!ok && threadIdx.x == 0) {
        atomicOr(a.err, 4);
        atomicMin(a.err_atom, k);
    }
    if (!mixed) {
        chol_solve3<double>(reinterpret_cast<const double*>(A), N, ld, L.Y);
    } else {
        // X = 0; repeat: residual r = d - B~ X in FP64 with B~ rebuilt from its
        // FP32 pair coefficients, FP32 solve of r, X += correction
        for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) L.X[e] = 0.0;
        __syncthreads();
        for (int it = 0; it <= a.n_refine; ++it) {
            for (int i = threadIdx.x; i < n1; i += blockDim.x) {
                double res[9];
                for (int e = 0; e < 9; ++e) res[e] = L.Y[(3 * i + e / 3) * 3 + e % 3];
                if (it > 0) {
                    for (int e = 0; e < 9; ++e) res[e] -= L.X[(3 * i + e / 3) * 3 + e % 3] / L.ab[i];
                    for (int j = 0; j < n1; ++j) {
                        if (j == i) continue;
                        const int pj = i > j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
                        const double cA = L.coef[2 * pj], cB = L.coef[2 * pj + 1];
                        if (cA == 0.0 && cB == 0.0) continue;
                        const double v[3] = {L.px[i] - L.px[j], L.py[i] - L.py[j], L.pz[i] - L.pz[j]};
                        const double ir = 1.0 / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                        const double rh[3] = {v[0] * ir, v[1] * ir, v[2] * ir};
                        for (int c = 0; c < 3; ++c) {
                            const double x0 = L.X[(3 * j + 0) * 3 + c], x1 = L.X[(3 * j + 1) * 3 + c],
                                         x2 = L.X[(3 * j + 2) * 3 + c];
                            const double rx = rh[0] * x0 + rh[1] * x1 + rh[2] * x2;
                            res[0 * 3 + c] -= cA * rh[0] * rx + cB * x0;
                            res[1 * 3 + c] -= cA * rh[1] * rx + cB * x1;
                            res[2 * 3 + c] -= cA * rh[2] * rx + cB * x2;
                        }
                    }
                }
                for (int e = 0; e < 9; ++e) Yr[(3 * i + e / 3) * 3 + e % 3] = R(res[e]);
            }
            __syncthreads();
            chol_solve3<R>(A, N, ld, Yr);
            for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) L.X[e] += double(Yr[e]);
            __syncthreads();
        }
        for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) L.Y[e] = L.X[e];
        __syncthreads();
    }
    double* X = a.xsol + a.x_off[k] + (size_t)w * N * 3;
    for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) X[e] = L.Y[e];
    double* al = a.alpha_loc + a.aloc_off[k];
    for (int s = threadIdx.x; s < n1; s += blockDim.x)
        al[(size_t)s * a.nw + w] = (L.Y[(3 * s) * 3 + 0] + L.Y[(3 * s + 1) * 3 + 1] + L.Y[(3 * s + 2) * 3 + 2]) / 3.0;
}

// ---------------------------------------------------------------------------
// Adjoint.  With X = B~^{-1} d and seeds xbar_i (adjoint of alpha~_iso_i =
// Tr X_i / 3): lambda = B~^{-1} Xbar with Xbar_i = xbar_i I / 3, then
//   dE = -<lambda X^T, dB~> + <lambda, dd>.
// Per site, the gradient sums over its partners (each pair is evaluated from
// both ends; partner ranges are split over kParts threads and recombined in a
// fixed order), so the result does not depend on scheduling.  The mixed path
// solves for lambda in FP32 and evaluates the pair-tensor derivatives in FP32;
// contractions and sums are FP64.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) k_scs_adjoint(ScsArgs a, int n1max, int n2max) {
    extern __shared__ double lds[];
    constexpr bool mixed = sizeof(R) == 4;
    const int k = blockIdx.x;
    const int w = blockIdx.y;
    const Counts cnt = a.counts[k];
    const int n1 = cnt.n1, n12 = cnt.n12, n2 = n12 - n1, nall = cnt.n_all;
    const int N = 3 * n1;
    const int ld = a.fac_ld[k];
    const StructInfo& SI = a.sinfo[a.atom_struct[k]];
    const double rc = SI.r_scs;
    ScsLds L = scs_lds(lds, n1max, n2max, mixed);
    const R* A = static_cast<const R*>(a.fac) + a.fac_off[k] + (size_t)w * ld * N;
    R* Yr = static_cast<R*>(L.Yr);
    const double* Xg = a.xsol + a.x_off[k] + (size_t)w * N * 3;
    load_sites(a, k, w, n1, n12, L);
    const double* abl = a.abar_loc + a.aloc_off[k];
    for (int s = threadIdx.x; s < n1; s += blockDim.x) {
        double xb = abl[(size_t)s * a.nw + w];
        if (s == 0) xb += a.abar_cen[(size_t)k * a.nw + w];
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c) Yr[(3 * s + q) * 3 + c] = (q == c) ? R(xb / 3.0) : R(0);
    }
    for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) L.X[e] = Xg[e];
    __syncthreads();
    chol_solve3<R>(A, N, ld, Yr);  // lambda
    for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) L.Y[e] = double(Yr[e]);
    __syncthreads();

    double* out = a.cf + (size_t)w * a.cf_slice + a.site_off[k] * 3;
    const double fconv = -1.0 / kBohr;  // force = -dE/dx, per Angstrom
    const int32_t* seg_i = a.pl_seg + a.site_off[k] + 2 * (int64_t)k;
    const int32_t* li = a.pl_i + a.pl_off[k];
    // K1 sites: couplings inside B~ and to the shell through d
    for (int t = threadIdx.x; t < n1 * kParts; t += blockDim.x) {
        const int i = t % n1, part = t / n1;
        double g[3] = {0.0, 0.0, 0.0};
        double Yi[9], Xi[9];
        for (int e = 0; e < 9; ++e) {
            Yi[e] = L.Y[(3 * i + e / 3) * 3 + e % 3];
            Xi[e] = L.X[(3 * i + e / 3) * 3 + e % 3];
        }
        for (int j = part; j < n1; j += kParts) {
            if (j == i) continue;
            const double v[3] = {L.px[i] - L.px[j], L.py[i] - L.py[j], L.pz[i] - L.pz[j]};
            if (!(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] < rc * rc)) continue;
            double rh[3], r;
            const SrPair<R> tp = k1_pair<R>(a, L, i, j, rc, rh, r);
            double Yj[9], Xj[9];
            for (int e = 0; e < 9; ++e) {
                Yj[e] = L.Y[(3 * j + e / 3) * 3 + e % 3];
                Xj[e] = L.X[(3 * j + e / 3) * 3 + e % 3];
            }
            double Cs[9];
            for (int q = 0; q < 3; ++q)
                for (int c = 0; c < 3; ++c) {
                    double s1 = 0.0, s2 = 0.0;
                    for (int m = 0; m < 3; ++m) {
                        s1 += Yi[3 * q + m] * Xj[3 * c + m] + Yi[3 * c + m] * Xj[3 * q + m];
                        s2 += Xi[3 * q + m] * Yj[3 * c + m] + Xi[3 * c + m] * Yj[3 * q + m];
                    }
                    Cs[3 * q + c] = -0.5 * (s1 + s2);
                }
            double gp[3];
            radial_tensor_grad(rh, r, double(tp.A), double(tp.dA), double(tp.dB), Cs, gp);
            g[0] += gp[0];
            g[1] += gp[1];
            g[2] += gp[2];
        }
        double lam[9];
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c) lam[3 * q + c] = 0.5 * (Yi[3 * q + c] + Yi[3 * c + q]);
        for (int e = seg_i[i] + part; e < seg_i[i + 1]; e += kParts) {
            const int q = li[e] & 0xFFFF;
            double rh[3], r;
            const SrPair<R> tp = k2_pair<R>(a, L, i, q, rc, rh, r);
            double gp[3];
            radial_tensor_grad(rh, r, double(tp.A), double(tp.dA), double(tp.dB), lam, gp);
            g[0] -= L.qab[q] * gp[0];
            g[1] -= L.qab[q] * gp[1];
            g[2] -= L.qab[q] * gp[2];
        }
        L.red[(size_t)(part * n1 + i) * 3 + 0] = g[0];
        L.red[(size_t)(part * n1 + i) * 3 + 1] = g[1];
        L.red[(size_t)(part * n1 + i) * 3 + 2] = g[2];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n1; i += blockDim.x) {
        double g0 = 0.0, g1 = 0.0, g2 = 0.0;
        for (int part = 0; part < kParts; ++part) {
            g0 += L.red[(size_t)(part * n1 + i) * 3 + 0];
            g1 += L.red[(size_t)(part * n1 + i) * 3 + 1];
            g2 += L.red[(size_t)(part * n1 + i) * 3 + 2];
        }
        out[3 * i + 0] = fconv * g0;
        out[3 * i + 1] = fconv * g1;
        out[3 * i + 2] = fconv * g2;
    }
    // shell sites K2: their coupling to K1 through d (one thread per shell site,
    // over its segment of the shell-major list)
    const int32_t* seg_q = seg_i + (n1 + 1);
    const int32_t* lq = a.pl_q + a.pl_off[k];
    for (int q = threadIdx.x; q < n2; q += blockDim.x) {
        double g[3] = {0.0, 0.0, 0.0};
        for (int e = seg_q[q]; e < seg_q[q + 1]; ++e) {
            const int i = lq[e] & 0xFFFF;
            double rh[3], r;
            const SrPair<R> tp = k2_pair<R>(a, L, i, q, rc, rh, r);
            double lam[9];
            for (int e2 = 0; e2 < 3; ++e2)
                for (int c = 0; c < 3; ++c)
                    lam[3 * e2 + c] = 0.5 * (L.Y[(3 * i + e2) * 3 + c] + L.Y[(3 * i + c) * 3 + e2]);
            double gp[3];
            radial_tensor_grad(rh, r, double(tp.A), double(tp.dA), double(tp.dB), lam, gp);
            g[0] += L.qab[q] * gp[0];
            g[1] += L.qab[q] * gp[1];
            g[2] += L.qab[q] * gp[2];
        }
        out[3 * (n1 + q) + 0] = fconv * g[0];
        out[3 * (n1 + q) + 1] = fconv * g[1];
        out[3 * (n1 + q) + 2] = fconv * g[2];
    }
    for (int s = n12 + threadIdx.x; s < nall; s += blockDim.x) {
        out[3 * s + 0] = 0.0;
        out[3 * s + 1] = 0.0;
        out[3 * s + 2] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// K1 x K2 coupling lists of one atom (frequency independent).  A shell site q
// couples to a K1 site i when r_iq < r_scs (beyond, f_SR vanishes).  The lists
// are written in i-major and shell-major order with CSR offsets; both orders
// are deterministic (one thread per major index, minors in increasing order).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_pairlist(ScsArgs a, int n1max, int n2max) {
    extern __shared__ double lds[];
    const int k = blockIdx.x;
    const Counts cnt = a.counts[k];
    const int n1 = cnt.n1, n12 = cnt.n12, n2 = n12 - n1;
    const StructInfo& SI = a.sinfo[a.atom_struct[k]];
    const double rc2 = SI.r_scs * SI.r_scs;
    double* px = lds;
    double* py = px + n1max;
    double* pz = py + n1max;
    double* qx = pz + n1max;
    double* qy = qx + n2max;
    double* qz = qy + n2max;
    int32_t* cnt_i = reinterpret_cast<int32_t*>(qz + n2max);   // n1max + 1
    int32_t* cnt_q = cnt_i + (n1max + 1);                        // n2max + 1
    const Site* S = a.sites + a.site_off[k];
    for (int s = threadIdx.x; s < n12; s += blockDim.x) {
        if (s < n1) { px[s] = S[s].x; py[s] = S[s].y; pz[s] = S[s].z; }
        else { qx[s - n1] = S[s].x; qy[s - n1] = S[s].y; qz[s - n1] = S[s].z; }
    }
    __syncthreads();
    auto coupled = [&](int i, int q) {
        const double dx = px[i] - qx[q], dy = py[i] - qy[q], dz = pz[i] - qz[q];
        return dx * dx + dy * dy + dz * dz < rc2;
    };
    for (int i = threadIdx.x; i < n1; i += blockDim.x) {
        int c = 0;
        for (int q = 0; q < n2; ++q) c += coupled(i, q);
        cnt_i[i] = c;
    }
    for (int q = threadIdx.x; q < n2; q += blockDim.x) {
        int c = 0;
        for (int i = 0; i < n1; ++i) c += coupled(i, q);
        cnt_q[q] = c;
    }
    __syncthreads();
    int32_t* seg = const_cast<int32_t*>(a.pl_seg) + a.site_off[k] + 2 * (int64_t)k;
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < n1; ++i) { const int c = cnt_i[i]; cnt_i[i] = acc; seg[i] = acc; acc += c; }
        seg[n1] = acc;
        cnt_i[n1] = acc;
    }
    if (threadIdx.x == 64) {
        int acc = 0;
        for (int q = 0; q < n2; ++q) { const int c = cnt_q[q]; cnt_q[q] = acc; seg[n1 + 1 + q] = acc; acc += c; }
        seg[n1 + 1 + n2] = acc;
        cnt_q[n2] = acc;
    }
    __syncthreads();
    int32_t* lio = const_cast<int32_t*>(a.pl_i) + a.pl_off[k];
    int32_t* lqo = const_cast<int32_t*>(a.pl_q) + a.pl_off[k];
    for (int i = threadIdx.x; i < n1; i += blockDim.x) {
        int pos = cnt_i[i];
        for (int q = 0; q < n2; ++q)
            if (coupled(i, q)) lio[pos++] = (i << 16) | q;
    }
    for (int q = threadIdx.x; q < n2; q += blockDim.x) {
        int pos = cnt_q[q];
        for (int i = 0; i < n1; ++i)
            if (coupled(i, q)) lqo[pos++] = (q << 16) | i;
    }
}

size_t pairlist_lds_bytes(int n1max, int n2max) {
    return sizeof(double) * 3 * ((size_t)n1max + n2max) + sizeof(int32_t) * ((size_t)n1max + n2max + 2);
}

hipError_t launch_pairlist(hipStream_t st, const ScsArgs& a, int n1max, int n2max) {
    hipLaunchKernelGGL(k_pairlist, dim3(a.n), dim3(256), pairlist_lds_bytes(n1max, n2max), st, a, n1max, n2max);
    return hipGetLastError();
}

hipError_t launch_scs_forward(hipStream_t st, const ScsArgs& a, int n1max, int n2max, bool mixed) {
    const size_t lds = scs_lds_bytes(n1max, n2max, mixed);
    if (mixed)
        hipLaunchKernelGGL(k_scs_forward<float>, dim3(a.n, a.nw), dim3(256), lds, st, a, n1max, n2max);
    else
        hipLaunchKernelGGL(k_scs_forward<double>, dim3(a.n, a.nw), dim3(256), lds, st, a, n1max, n2max);
    return hipGetLastError();
}

hipError_t launch_scs_adjoint(hipStream_t st, const ScsArgs& a, int n1max, int n2max, bool mixed) {
    const size_t lds = scs_lds_bytes(n1max, n2max, mixed);
    if (mixed)
        hipLaunchKernelGGL(k_scs_adjoint<float>, dim3(a.n, a.nw), dim3(256), lds, st, a, n1max, n2max);
    else
        hipLaunchKernelGGL(k_scs_adjoint<double>, dim3(a.n, a.nw), dim3(256), lds, st, a, n1max, n2max);
    return hipGetLastError();
}

}  // namespace lmbd
