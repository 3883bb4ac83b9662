// Local SCS: assembly, Cholesky factorisation and solves of
//   B~_K alpha~_K = d_K                         (Sec. III.B, local polarisability system)
//   B~_K,ij = delta_ij / abar_i + T_SR,K,ij     (i, j in K1)
//   d_K,i   = I - sum_{j in K2} T_SR,K,ij abar_j
//   T_SR,K,ij = f_inner f_SR (1 - f(r, S)) (-T g + h)     (Sec. II.B and III.B)
// and the adjoint of the isotropic polarisabilities alpha~_iso = Tr(X_i)/3.
//
// One workgroup per (atom, frequency).  B~_K is symmetric positive definite on
// the workloads (measured: diagonally scaled condition numbers below 12), so it
// is factorised by a right-looking blocked Cholesky in its own slot of device
// memory; the factor is kept for the adjoint solve.  A non-positive pivot is a
// breakdown reported to the host.
#include "lmbd_internal.h"

namespace lmbd {

constexpr int NB = 16;  // block size of the factorisation


// T_SR,K for one pair as A rhat rhat^T + B I, with radial derivatives.
struct SrPair {
    double A, B, dA, dB;
};

__device__ inline SrPair sr_pair(double r, double s_ij, double S, double damp_d, double rc,
                                 double rb, double wmul, double dwmul) {
    double A, B, dA, dB;
    sr_core(r, s_ij, A, B, dA, dB);
    double dfdr, dfdS, dcut;
    const double f = fermi(r, S, damp_d, dfdr, dfdS);
    const double fc = cutoff_poly(r, rc, rb, dcut);
    const double w = wmul * fc * (1.0 - f);
    const double dw = dwmul * fc * (1.0 - f) + wmul * dcut * (1.0 - f) - wmul * fc * dfdr;
    return SrPair{w * A, w * B, dw * A + w * dA, dw * B + w * dB};
}

__device__ inline void tri_decode(int t, int& i, int& j) {
    int a = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((a + 1) * (a + 2) / 2 <= t) ++a;
    while (a * (a + 1) / 2 > t) --a;
    i = a;
    j = t - a * (a + 1) / 2;
}

// ---------------------------------------------------------------------------
// Blocked Cholesky of the N x N lower triangle of A (column-major, leading
// dimension ld) by one workgroup.  P is an LDS panel of at least N*NB doubles,
// D an LDS 16x16 block.  Returns false in `ok` on a non-positive pivot.
// ---------------------------------------------------------------------------
__device__ void chol_factor(double* __restrict__ A, int N, int ld, double* P, double* D, bool& ok) {
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    bool good = true;
    for (int j0 = 0; j0 < N; j0 += NB) {
        const int jb = min(NB, N - j0);
        // (a) diagonal block: wave 0, lane l holds row l of the block
        if (tid < 64) {
            const int l = tid;
            double row[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const bool valid = (l < jb) && (c <= l);
                row[c] = valid ? A[(size_t)(j0 + c) * ld + j0 + l] : (l == c ? 1.0 : 0.0);
            }
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const double dcc = __shfl(row[c], c, 64);
                if (c < jb && !(dcc > 0.0)) good = false;
                const double sq = sqrt(dcc);
                const double inv = 1.0 / sq;
                if (l == c) row[c] = sq;
                else if (l > c) row[c] *= inv;
#pragma unroll
                for (int s = c + 1; s < NB; ++s) {
                    const double lsc = __shfl(row[c], s, 64);
                    if (l >= s) row[s] -= row[c] * lsc;
                }
            }
            if (l < NB) {
#pragma unroll
                for (int c = 0; c < NB; ++c) D[l * NB + c] = (c <= l) ? row[c] : 0.0;
            }
            if (l < jb) {
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    if (c <= l) A[(size_t)(j0 + c) * ld + j0 + l] = row[c];
            }
        }
        __syncthreads();
        // (b) panel below the block: X L_bb^T = A_panel, row by row
        const int r0 = j0 + jb;
        for (int i = r0 + tid; i < N; i += nthr) {
            double x[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) x[c] = (c < jb) ? A[(size_t)(j0 + c) * ld + i] : 0.0;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                if (c < jb) {
                    double s = x[c];
#pragma unroll
                    for (int q = 0; q < c; ++q) s -= x[q] * D[c * NB + q];
                    x[c] = s / D[c * NB + c];
                }
            }
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                if (c < jb) A[(size_t)(j0 + c) * ld + i] = x[c];
                P[(size_t)(i - r0) * NB + c] = x[c];
            }
        }
        __syncthreads();
        // (c) trailing update A22 -= P P^T on 4x4 tiles of the lower triangle
        const int m = N - r0;
        if (m > 0) {
            const int nt = (m + 3) / 4;
            const int ntiles = nt * (nt + 1) / 2;
            for (int t = tid; t < ntiles; t += nthr) {
                int ti, tj;
                tri_decode(t, ti, tj);
                const int i0 = ti * 4, c0 = tj * 4;
                double acc[4][4] = {};
                for (int c = 0; c < jb; ++c) {
                    double a[4], b[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        a[r] = (i0 + r < m) ? P[(size_t)(i0 + r) * NB + c] : 0.0;
                        b[r] = (c0 + r < m) ? P[(size_t)(c0 + r) * NB + c] : 0.0;
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int q = 0; q < 4; ++q) acc[r][q] += a[r] * b[q];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int j = c0 + q;
                    if (j >= m) continue;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = i0 + r;
                        if (i < m && i >= j) A[(size_t)(r0 + j) * ld + r0 + i] -= acc[r][q];
                    }
                }
            }
        }
        __syncthreads();
    }
    ok = good;
}

// Solve L L^T Y = Y in place for 3 right-hand sides (Y: LDS, row-major N x 3).
__device__ void chol_solve3(const double* __restrict__ A, int N, int ld, double* Y) {
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    // forward: L y = b
    for (int j0 = 0; j0 < N; j0 += NB) {
        const int jb = min(NB, N - j0);
        if (tid < 3) {
            const int c = tid;
            for (int r = 0; r < jb; ++r) {
                double y = Y[(j0 + r) * 3 + c];
                for (int q = 0; q < r; ++q) y -= A[(size_t)(j0 + q) * ld + j0 + r] * Y[(j0 + q) * 3 + c];
                Y[(j0 + r) * 3 + c] = y / A[(size_t)(j0 + r) * ld + j0 + r];
            }
        }
        __syncthreads();
        for (int i = j0 + jb + tid; i < N; i += nthr) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int q = 0; q < jb; ++q) {
                const double l = A[(size_t)(j0 + q) * ld + i];
                s0 += l * Y[(j0 + q) * 3 + 0];
                s1 += l * Y[(j0 + q) * 3 + 1];
                s2 += l * Y[(j0 + q) * 3 + 2];
            }
            Y[i * 3 + 0] -= s0;
            Y[i * 3 + 1] -= s1;
            Y[i * 3 + 2] -= s2;
        }
        __syncthreads();
    }
    // backward: L^T x = y
    const int nblk = (N + NB - 1) / NB;
    for (int b = nblk - 1; b >= 0; --b) {
        const int j0 = b * NB;
        const int jb = min(NB, N - j0);
        if (tid < 3) {
            const int c = tid;
            for (int r = jb - 1; r >= 0; --r) {
                double x = Y[(j0 + r) * 3 + c];
                for (int q = r + 1; q < jb; ++q) x -= A[(size_t)(j0 + r) * ld + j0 + q] * Y[(j0 + q) * 3 + c];
                Y[(j0 + r) * 3 + c] = x / A[(size_t)(j0 + r) * ld + j0 + r];
            }
        }
        __syncthreads();
        for (int i = tid; i < j0; i += nthr) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int q = 0; q < jb; ++q) {
                const double l = A[(size_t)i * ld + j0 + q];
                s0 += l * Y[(j0 + q) * 3 + 0];
                s1 += l * Y[(j0 + q) * 3 + 1];
                s2 += l * Y[(j0 + q) * 3 + 2];
            }
            Y[i * 3 + 0] -= s0;
            Y[i * 3 + 1] -= s1;
            Y[i * 3 + 2] -= s2;
        }
        __syncthreads();
    }
}

// LDS layout shared by the forward and adjoint kernels
struct ScsLds {
    double *px, *py, *pz, *ab, *sg, *R, *Y, *D, *P, *X;
};
__device__ inline ScsLds scs_lds(double* base, int n1max) {
    const int N = 3 * n1max;
    ScsLds L;
    L.px = base;
    L.py = L.px + n1max;
    L.pz = L.py + n1max;
    L.ab = L.pz + n1max;
    L.sg = L.ab + n1max;
    L.R = L.sg + n1max;
    L.Y = L.R + n1max;
    L.D = L.Y + 3 * N;
    L.P = L.D + NB * NB;
    L.X = L.P + (size_t)N * NB;
    return L;
}

__device__ inline void load_k1(const ScsArgs& a, int k, int w, int n1, const ScsLds& L) {
    const Site* S = a.sites + a.site_off[k];
    for (int s = threadIdx.x; s < n1; s += blockDim.x) {
        const Site st = S[s];
        L.px[s] = st.x;
        L.py[s] = st.y;
        L.pz[s] = st.z;
        L.ab[s] = a.abar[(size_t)st.base * a.nw + w];
        L.sg[s] = a.sigma[(size_t)st.base * a.nw + w];
        L.R[s] = a.Rv[st.base];
    }
}

__global__ void __launch_bounds__(256) k_scs_forward(ScsArgs a, int n1max) {
    extern __shared__ double lds[];
    const int k = blockIdx.x;
    const int w = blockIdx.y;
    const Counts cnt = a.counts[k];
    const int n1 = cnt.n1, n12 = cnt.n12;
    const int N = 3 * n1;
    const int ld = a.fac_ld[k];
    const StructInfo& SI = a.sinfo[a.atom_struct[k]];
    const double rc = SI.r_scs;
    ScsLds L = scs_lds(lds, n1max);
    double* A = a.fac + a.fac_off[k] + (size_t)w * ld * N;
    load_k1(a, k, w, n1, L);
    __syncthreads();

    // B~ (lower triangle, block by block)
    const int npairs = n1 * (n1 + 1) / 2;
    for (int p = threadIdx.x; p < npairs; p += blockDim.x) {
        int i, j;
        tri_decode(p, i, j);
        if (i == j) {
            const double inv = 1.0 / L.ab[i];
            for (int q = 0; q < 3; ++q)
                for (int r = q; r < 3; ++r) A[(size_t)(3 * i + q) * ld + 3 * i + r] = (q == r) ? inv : 0.0;
            continue;
        }
        const double v[3] = {L.px[i] - L.px[j], L.py[i] - L.py[j], L.pz[i] - L.pz[j]};
        const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        const double rh[3] = {v[0] / r, v[1] / r, v[2] / r};
        const double s_ij = sqrt(L.sg[i] * L.sg[i] + L.sg[j] * L.sg[j]);
        const SrPair t = sr_pair(r, s_ij, a.beta * (L.R[i] + L.R[j]), a.damp_d, rc, a.r_buf, 1.0, 0.0);
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c)
                A[(size_t)(3 * j + c) * ld + 3 * i + q] = t.A * rh[q] * rh[c] + (q == c ? t.B : 0.0);
    }
    // d: identity minus the uncoupled shell K2 with TS polarisabilities and f_inner
    const Site* S = a.sites + a.site_off[k];
    for (int i = threadIdx.x; i < n1; i += blockDim.x) {
        double d[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
        for (int jj = n1; jj < n12; ++jj) {
            const Site sj = S[jj];
            const double v[3] = {L.px[i] - sj.x, L.py[i] - sj.y, L.pz[i] - sj.z};
            const double r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            if (!(r2 < rc * rc)) continue;
            const double r = sqrt(r2);
            const double rh[3] = {v[0] / r, v[1] / r, v[2] / r};
            const double abj = a.abar[(size_t)sj.base * a.nw + w];
            const double sgj = a.sigma[(size_t)sj.base * a.nw + w];
            const double s_ij = sqrt(L.sg[i] * L.sg[i] + sgj * sgj);
            double fin = 1.0, dfin = 0.0;
            if (r < a.r_inner) {
                const double x = r / a.r_inner;
                fin = 3.0 * x * x - 2.0 * x * x * x;
                dfin = (6.0 * x - 6.0 * x * x) / a.r_inner;
            }
            const SrPair t = sr_pair(r, s_ij, a.beta * (L.R[i] + a.Rv[sj.base]), a.damp_d, rc, a.r_buf,
                                     fin, dfin);
            for (int q = 0; q < 3; ++q)
                for (int c = 0; c < 3; ++c)
                    d[3 * q + c] -= abj * (t.A * rh[q] * rh[c] + (q == c ? t.B : 0.0));
        }
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c) L.Y[(3 * i + q) * 3 + c] = d[3 * q + c];
    }
    __threadfence_block();
    __syncthreads();

    bool ok = true;
    chol_factor(A, N, ld, L.P, L.D, ok);
    if (!ok && threadIdx.x == 0) {
        atomicOr(a.err, 4);
        atomicMin(a.err_atom, k);
    }
    chol_solve3(A, N, ld, L.Y);
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
// both ends, so the order of summation is fixed).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_scs_adjoint(ScsArgs a, int n1max) {
    extern __shared__ double lds[];
    const int k = blockIdx.x;
    const int w = blockIdx.y;
    const Counts cnt = a.counts[k];
    const int n1 = cnt.n1, n12 = cnt.n12, nall = cnt.n_all;
    const int N = 3 * n1;
    const int ld = a.fac_ld[k];
    const StructInfo& SI = a.sinfo[a.atom_struct[k]];
    const double rc = SI.r_scs;
    ScsLds L = scs_lds(lds, n1max);
    const double* A = a.fac + a.fac_off[k] + (size_t)w * ld * N;
    const double* Xg = a.xsol + a.x_off[k] + (size_t)w * N * 3;
    load_k1(a, k, w, n1, L);
    const double* abl = a.abar_loc + a.aloc_off[k];
    for (int s = threadIdx.x; s < n1; s += blockDim.x) {
        double xb = abl[(size_t)s * a.nw + w];
        if (s == 0) xb += a.abar_cen[(size_t)k * a.nw + w];
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c) L.Y[(3 * s + q) * 3 + c] = (q == c) ? xb / 3.0 : 0.0;
    }
    for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) L.X[e] = Xg[e];
    __syncthreads();
    chol_solve3(A, N, ld, L.Y);  // Y = lambda

    const Site* S = a.sites + a.site_off[k];
    double* out = a.cf + (size_t)w * a.cf_slice + a.site_off[k] * 3;
    const double fconv = -1.0 / kBohr;  // force = -dE/dx, per Angstrom
    // K1 sites: couplings inside B~ and to the shell through d
    for (int i = threadIdx.x; i < n1; i += blockDim.x) {
        double g[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < n1; ++j) {
            if (j == i) continue;
            const double v[3] = {L.px[i] - L.px[j], L.py[i] - L.py[j], L.pz[i] - L.pz[j]};
            const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (!(r < rc)) continue;
            const double rh[3] = {v[0] / r, v[1] / r, v[2] / r};
            const double s_ij = sqrt(L.sg[i] * L.sg[i] + L.sg[j] * L.sg[j]);
            const SrPair t = sr_pair(r, s_ij, a.beta * (L.R[i] + L.R[j]), a.damp_d, rc, a.r_buf, 1.0, 0.0);
            double C[9];
            for (int q = 0; q < 3; ++q)
                for (int c = 0; c < 3; ++c) {
                    double s1 = 0.0, s2 = 0.0;
                    for (int m = 0; m < 3; ++m) {
                        s1 += L.Y[(3 * i + q) * 3 + m] * L.X[(3 * j + c) * 3 + m];
                        s2 += L.X[(3 * i + q) * 3 + m] * L.Y[(3 * j + c) * 3 + m];
                    }
                    C[3 * q + c] = -(s1 + s2);
                }
            double Cs[9];
            for (int q = 0; q < 3; ++q)
                for (int c = 0; c < 3; ++c) Cs[3 * q + c] = 0.5 * (C[3 * q + c] + C[3 * c + q]);
            double gp[3];
            radial_tensor_grad(rh, r, t.A, t.dA, t.dB, Cs, gp);
            g[0] += gp[0];
            g[1] += gp[1];
            g[2] += gp[2];
        }
        double lam[9];
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c)
                lam[3 * q + c] = 0.5 * (L.Y[(3 * i + q) * 3 + c] + L.Y[(3 * i + c) * 3 + q]);
        for (int jj = n1; jj < n12; ++jj) {
            const Site sj = S[jj];
            const double v[3] = {L.px[i] - sj.x, L.py[i] - sj.y, L.pz[i] - sj.z};
            const double r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            if (!(r2 < rc * rc)) continue;
            const double r = sqrt(r2);
            const double rh[3] = {v[0] / r, v[1] / r, v[2] / r};
            const double abj = a.abar[(size_t)sj.base * a.nw + w];
            const double sgj = a.sigma[(size_t)sj.base * a.nw + w];
            const double s_ij = sqrt(L.sg[i] * L.sg[i] + sgj * sgj);
            double fin = 1.0, dfin = 0.0;
            if (r < a.r_inner) {
                const double x = r / a.r_inner;
                fin = 3.0 * x * x - 2.0 * x * x * x;
                dfin = (6.0 * x - 6.0 * x * x) / a.r_inner;
            }
            const SrPair t = sr_pair(r, s_ij, a.beta * (L.R[i] + a.Rv[sj.base]), a.damp_d, rc, a.r_buf,
                                     fin, dfin);
            double gp[3];
            radial_tensor_grad(rh, r, t.A, t.dA, t.dB, lam, gp);
            g[0] -= abj * gp[0];
            g[1] -= abj * gp[1];
            g[2] -= abj * gp[2];
        }
        out[3 * i + 0] = fconv * g[0];
        out[3 * i + 1] = fconv * g[1];
        out[3 * i + 2] = fconv * g[2];
    }
    // shell sites K2: their coupling to K1 through d
    for (int jj = n1 + threadIdx.x; jj < n12; jj += blockDim.x) {
        const Site sj = S[jj];
        const double abj = a.abar[(size_t)sj.base * a.nw + w];
        const double sgj = a.sigma[(size_t)sj.base * a.nw + w];
        const double Rj = a.Rv[sj.base];
        double g[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < n1; ++i) {
            const double v[3] = {L.px[i] - sj.x, L.py[i] - sj.y, L.pz[i] - sj.z};
            const double r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            if (!(r2 < rc * rc)) continue;
            const double r = sqrt(r2);
            const double rh[3] = {v[0] / r, v[1] / r, v[2] / r};
            const double s_ij = sqrt(L.sg[i] * L.sg[i] + sgj * sgj);
            double fin = 1.0, dfin = 0.0;
            if (r < a.r_inner) {
                const double x = r / a.r_inner;
                fin = 3.0 * x * x - 2.0 * x * x * x;
                dfin = (6.0 * x - 6.0 * x * x) / a.r_inner;
            }
            const SrPair t = sr_pair(r, s_ij, a.beta * (L.R[i] + Rj), a.damp_d, rc, a.r_buf, fin, dfin);
            double lam[9];
            for (int q = 0; q < 3; ++q)
                for (int c = 0; c < 3; ++c)
                    lam[3 * q + c] = 0.5 * (L.Y[(3 * i + q) * 3 + c] + L.Y[(3 * i + c) * 3 + q]);
            double gp[3];
            radial_tensor_grad(rh, r, t.A, t.dA, t.dB, lam, gp);
            g[0] += abj * gp[0];
            g[1] += abj * gp[1];
            g[2] += abj * gp[2];
        }
        out[3 * jj + 0] = fconv * g[0];
        out[3 * jj + 1] = fconv * g[1];
        out[3 * jj + 2] = fconv * g[2];
    }
    for (int s = n12 + threadIdx.x; s < nall; s += blockDim.x) {
        out[3 * s + 0] = 0.0;
        out[3 * s + 1] = 0.0;
        out[3 * s + 2] = 0.0;
    }
}

size_t scs_lds_bytes(int n1max) {
    const size_t N = 3 * (size_t)n1max;
    return sizeof(double) * (6 * (size_t)n1max + 3 * N + NB * NB + N * NB + 3 * N);
}

hipError_t launch_scs_forward(hipStream_t st, const ScsArgs& a, int n1max) {
    hipLaunchKernelGGL(k_scs_forward, dim3(a.n, a.nw), dim3(256), scs_lds_bytes(n1max), st, a, n1max);
    return hipGetLastError();
}

hipError_t launch_scs_adjoint(hipStream_t st, const ScsArgs& a, int n1max) {
    hipLaunchKernelGGL(k_scs_adjoint, dim3(a.n, a.nw), dim3(256), scs_lds_bytes(n1max), st, a, n1max);
    return hipGetLastError();
}

}  // namespace lmbd
