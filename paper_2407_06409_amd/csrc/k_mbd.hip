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
#include "lmbd_internal.h"

namespace lmbd {


// LDS layout
struct MbdLds {
    double *px, *py, *pz, *sa, *sqa, *Rt, *fs, *dfs, *ab, *g, *rb, *fg, *mu, *tA, *tB;
};
__device__ inline MbdLds mbd_lds(double* b, int nk, int nw, int nq, int n_max) {
    MbdLds L;
    L.px = b;
    L.py = L.px + nk;
    L.pz = L.py + nk;
    L.sa = L.pz + nk;
    L.sqa = L.sa + (size_t)nk * nw;
    L.Rt = L.sqa + (size_t)nk * nq;
    L.fs = L.Rt + nk;
    L.dfs = L.fs + nk;
    L.ab = L.dfs + nk;
    L.g = L.ab + (size_t)nk * nw;     // [4 parts][nk][3]
    L.rb = L.g + 12 * (size_t)nk;     // [4 parts][nk]
    L.fg = L.rb + 4 * (size_t)nk;     // [nk][3]
    L.mu = L.fg + 3 * (size_t)nk;
    L.tA = L.mu + (size_t)(n_max + 1) * nq;
    L.tB = L.tA + 16 * 65;
    return L;
}

size_t mbd_lds_bytes(int nkmax, int nw, int nq, int n_max) {
    const size_t nk = nkmax;
    return sizeof(double) * (3 * nk + nk * nw + nk * nq + 3 * nk + nk * nw + 12 * nk + 4 * nk +
                             3 * nk + (size_t)(n_max + 1) * nq + 2 * 16 * 65);
}

// Workgroup GEMM: out(m, n) = sum_k A(m, k) B(k, n), 64x64 tiles, 4x4 per thread,
// k staged through LDS in chunks of 16.  Loaders return 0 outside the range.
template <typename LA, typename LB, typename ST>
__device__ void wg_gemm(int M, int N, int K, LA la, LB lb, ST st, double* tA, double* tB) {
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    for (int m0 = 0; m0 < M; m0 += 64)
        for (int n0 = 0; n0 < N; n0 += 64) {
            double acc[4][4] = {};
            for (int k0 = 0; k0 < K; k0 += 16) {
                for (int e = tid; e < 16 * 64; e += 256) {
                    const int kk = e >> 6, mm = e & 63;
                    tA[kk * 65 + mm] = (m0 + mm < M && k0 + kk < K) ? la(m0 + mm, k0 + kk) : 0.0;
                    tB[kk * 65 + mm] = (n0 + mm < N && k0 + kk < K) ? lb(k0 + kk, n0 + mm) : 0.0;
                }
                __syncthreads();
#pragma unroll 4
                for (int kk = 0; kk < 16; ++kk) {
                    double a[4], b[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        a[i] = tA[kk * 65 + ty + 16 * i];
                        b[i] = tB[kk * 65 + tx + 16 * i];
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
                }
                __syncthreads();
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int m = m0 + ty + 16 * i, nn = n0 + tx + 16 * j;
                    if (m < M && nn < N) st(m, nn, acc[i][j]);
                }
        }
    __syncthreads();
}

// T_LR pair coefficients: T_LR = A rhat rhat^T + B I with radial derivatives,
// and dT_LR/dS~ = fLR (df/dS~) T.
struct LrPair {
    double A, B, dA, dB, dfS, fLR;
};
__device__ inline LrPair lr_pair(double r, double S, double damp_d, double rcut, double rb) {
    double dfdr, dfdS, dcut;
    const double f = fermi(r, S, damp_d, dfdr, dfdS);
    const double fc = cutoff_poly(r, rcut, rb, dcut);
    const double w = fc * f;
    const double dw = dcut * f + fc * dfdr;
    const double r3 = r * r * r;
    LrPair p;
    p.A = 3.0 * w / r3;
    p.B = -w / r3;
    p.dA = 3.0 * dw / r3 - 9.0 * w / (r3 * r);
    p.dB = -dw / r3 + 3.0 * w / (r3 * r);
    p.dfS = dfdS;
    p.fLR = fc;
    return p;
}

__global__ void __launch_bounds__(256) k_mbd(MbdArgs a, int nkmax) {
    extern __shared__ double lds[];
    const int k = blockIdx.x;
    const int tid = threadIdx.x;
    const Counts cnt = a.counts[k];
    const int nK = cnt.nK, n1 = cnt.n1, nall = cnt.n_all;
    const int N3 = 3 * nK;
    const int nw = a.nw, nq = a.nq, ncol = a.ncol, n_max = a.n_max;
    const StructInfo& SI = a.sinfo[a.atom_struct[k]];
    const double rs = SI.r_scs;
    MbdLds L = mbd_lds(lds, nkmax, nw, nq, n_max);
    const Site* S = a.sites + a.site_off[k];
    const double* aloc = a.alpha_loc + a.aloc_off[k];
    double* T = a.work + a.work_off[k];
    double* U = T + (size_t)N3 * N3;                         // u_1 .. u_mmax
    double* Z = U + (size_t)a.mmax * N3 * ncol;              // Z_0 .. Z_{n_max-1}
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
        for (int w = 0; w < nw; ++w) {
            const double al = (s < n1) ? aloc[(size_t)s * nw + w] : 0.0;
            const double v = (s == 0) ? al : (1.0 - fsv) * al + fsv * cen[w];
            L.sa[(size_t)s * nw + w] = v;
            if (w > 0) L.sqa[(size_t)s * nq + (w - 1)] = sqrt(v);
        }
        L.Rt[s] = a.r0v[st.base] * cbrt(L.sa[(size_t)s * nw] / a.a0v[st.base]);
    }
    __syncthreads();

    // --- T_LR (row-major, symmetric, zero diagonal blocks)
    for (int p = tid; p < nK * nK; p += blockDim.x) {
        const int i = p / nK, j = p % nK;
        double blk[9] = {};
        if (i != j) {
            const double v[3] = {L.px[i] - L.px[j], L.py[i] - L.py[j], L.pz[i] - L.pz[j]};
            const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            const double rcut = (i == 0 || j == 0) ? SI.r_mbd1 : SI.r_mbd2;
            if (r < rcut) {
                const LrPair t = lr_pair(r, a.beta * (L.Rt[i] + L.Rt[j]), a.damp_d, rcut, a.r_buf);
                const double rh[3] = {v[0] / r, v[1] / r, v[2] / r};
                for (int q = 0; q < 3; ++q)
                    for (int c = 0; c < 3; ++c) blk[3 * q + c] = t.A * rh[q] * rh[c] + (q == c ? t.B : 0.0);
            }
        }
        for (int q = 0; q < 3; ++q)
            for (int c = 0; c < 3; ++c) T[(size_t)(3 * i + q) * N3 + 3 * j + c] = blk[3 * q + c];
    }
    __syncthreads();

    // --- u_1 = D T D e_k
    double* U1 = Uat(1);
    for (int e = tid; e < N3 * ncol; e += blockDim.x) {
        const int row = e / ncol, col = e % ncol;
        const int q = col / 3, c = col % 3;
        U1[e] = L.sqa[(size_t)(row / 3) * nq + q] * T[(size_t)row * N3 + c] * L.sqa[q];
    }
    __syncthreads();
    // --- u_{m+1} = D T (D u_m)
    for (int m = 1; m < a.mmax; ++m) {
        const double* Um = Uat(m);
        double* Un = Uat(m + 1);
        wg_gemm(
            N3, ncol, N3, [&](int r, int l) { return T[(size_t)r * N3 + l]; },
            [&](int l, int col) { return L.sqa[(size_t)(l / 3) * nq + col / 3] * Um[(size_t)l * ncol + col]; },
            [&](int r, int col, double v) { Un[(size_t)r * ncol + col] = L.sqa[(size_t)(r / 3) * nq + col / 3] * v; },
            L.tA, L.tB);
    }

    // --- moments mu_n(q) = <u_a, u_b>, a + b = n
    const int nmom = (n_max - 1) * nq;
    for (int t = tid; t < nmom; t += blockDim.x) {
        const int n = 2 + t / nq, q = t % nq;
        const int ia = n / 2, ib = n - ia;
        const double* ua = Uat(ia);
        const double* ub = Uat(ib);
        double s = 0.0;
        for (int row = 0; row < N3; ++row)
            for (int c = 0; c < 3; ++c) s += ua[(size_t)row * ncol + 3 * q + c] * ub[(size_t)row * ncol + 3 * q + c];
        L.mu[n * nq + q] = s;
    }
    __syncthreads();
    const double wk = a.e_weight ? a.e_weight[k] : 1.0;
    if (tid == 0) {
        double e = 0.0;
        for (int q = 0; q < nq; ++q) {
            double eq = 0.0;
            for (int n = 2; n <= n_max; ++n) eq += a.coef[n] * L.mu[n * nq + q];
            e += a.wq[q] * eq;
        }
        a.e_atom[k] = e;
    }
    if (!a.forces) return;

    // --- dE/d alpha~_i(w_q) from the moments (row-local Krylov products)
    for (int t = tid; t < nK * nw; t += blockDim.x) {
        const int i = t / nw, w = t % nw;
        double v = 0.0;
        if (w > 0) {
            const int q = w - 1;
            double s = 0.0;
            for (int n = 2; n <= n_max; ++n) {
                double sn = (i == 0) ? L.mu[n * nq + q] : 0.0;
                for (int aa = 1; aa < n; ++aa) {
                    const double* ua = Uat(aa);
                    const double* ub = Uat(n - aa);
                    for (int r = 3 * i; r < 3 * i + 3; ++r)
                        for (int c = 0; c < 3; ++c)
                            sn += ua[(size_t)r * ncol + 3 * q + c] * ub[(size_t)r * ncol + 3 * q + c];
                }
                s += a.coef[n] * sn;
            }
            v = wk * a.wq[q] * s / L.sa[(size_t)i * nw + w];
        }
        L.ab[t] = v;
    }
    // --- Z_a = sum_b c_{a+b+1} u_b (u_0 = e_k)
    for (int e = tid; e < n_max * N3 * ncol; e += blockDim.x) {
        const int aa = e / (N3 * ncol);
        const int rem = e % (N3 * ncol);
        const int row = rem / ncol, col = rem % ncol;
        double s = (row == col % 3) ? a.coef[aa + 1] : 0.0;   // b = 0 term, c_1 = 0 anyway
        if (aa + 1 < 2) s = 0.0;
        for (int b = 1; b <= n_max - 1 - aa; ++b) s += a.coef[aa + b + 1] * Uat(b)[(size_t)row * ncol + col];
        Z[e] = s;
    }
    __syncthreads();
    // --- Tbar = sum_a (D u_a)(W D Z_a)^T  (overwrites T)
    const int KK = n_max * ncol;
    wg_gemm(
        N3, N3, KK,
        [&](int r, int kk) {
            const int aa = kk / ncol, col = kk % ncol;
            double u;
            if (aa == 0) u = (r == col % 3) ? 1.0 : 0.0;
            else u = Uat(aa)[(size_t)r * ncol + col];
            return L.sqa[(size_t)(r / 3) * nq + col / 3] * u;
        },
        [&](int kk, int s) {
            const int aa = kk / ncol, col = kk % ncol;
            return wk * a.wq[col / 3] * L.sqa[(size_t)(s / 3) * nq + col / 3] * Z[(size_t)aa * N3 * ncol + (size_t)s * ncol + col];
        },
        [&](int r, int s, double v) { T[(size_t)r * N3 + s] = v; }, L.tA, L.tB);

    // --- pair contraction: dE/dp_i and dE/dR~_i (each unordered pair from both ends)
    const int parts = max(1, min(4, (int)blockDim.x / max(nK, 1)));
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
            const LrPair lp = lr_pair(r, a.beta * (L.Rt[i] + L.Rt[j]), a.damp_d, rcut, a.r_buf);
            double C[9];
            for (int q = 0; q < 3; ++q)
                for (int c = 0; c < 3; ++c)
                    C[3 * q + c] = T[(size_t)(3 * i + q) * N3 + 3 * j + c] + T[(size_t)(3 * i + c) * N3 + 3 * j + q];
            double gp[3];
            radial_tensor_grad(rh, r, lp.A, lp.dA, lp.dB, C, gp);
            g[0] += gp[0];
            g[1] += gp[1];
            g[2] += gp[2];
            // <C, T_ij> with T = (3 rhat rhat^T - I)/r^3, times fLR df/dS~
            double rCr = 0.0;
            for (int q = 0; q < 3; ++q)
                for (int c = 0; c < 3; ++c) rCr += rh[q] * C[3 * q + c] * rh[c];
            const double ct = (3.0 * rCr - (C[0] + C[4] + C[8])) / (r * r * r);
            Rb += a.beta * lp.fLR * lp.dfS * ct;
        }
        L.g[(size_t)(part * nK + i) * 3 + 0] = g[0];
        L.g[(size_t)(part * nK + i) * 3 + 1] = g[1];
        L.g[(size_t)(part * nK + i) * 3 + 2] = g[2];
        L.rb[(size_t)part * nK + i] = Rb;
    }
    __syncthreads();
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
        L.ab[(size_t)i * nw] += Rb * L.Rt[i] / (3.0 * L.sa[(size_t)i * nw]);
        const Site st = S[i];
        const double* cen = a.alpha_loc + a.aloc_off[st.base];
        double gf = 0.0;  // sum_w abar_i(w) (alpha~_I,i(w) - alpha~_K,i(w))
        for (int w = 0; w < nw; ++w) {
            const double ai = L.ab[(size_t)i * nw + w];
            if (i == 0) {
                abl[w] = ai;
                cap[w] = 0.0;
            } else if (i < n1) {
                abl[(size_t)i * nw + w] = (1.0 - L.fs[i]) * ai;
                cap[(size_t)i * nw + w] = L.fs[i] * ai;
                gf += ai * (cen[w] - aloc[(size_t)i * nw + w]);
            } else {
                cap[(size_t)i * nw + w] = ai;
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

hipError_t launch_mbd(hipStream_t st, const MbdArgs& a, int nkmax) {
    hipLaunchKernelGGL(k_mbd, dim3(a.n), dim3(256), mbd_lds_bytes(nkmax, a.nw, a.nq, a.n_max), st, a,
                       nkmax);
    return hipGetLastError();
}

}  // namespace lmbd
