// Internal definitions shared by the lMBD HIP kernels and the host driver.
// Not part of the public ABI (see include/lmbd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace lmbd {

// CODATA 2018
constexpr double kBohr = 0.529177210903;      // Angstrom per bohr
constexpr double kHartree = 27.211386245988;  // eV per hartree
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoOverSqrtPi = 1.12837916709551257390;  // 2/sqrt(pi)
constexpr double kSqrt2OverPi = 0.79788456080286535588;    // sqrt(2/pi)

// Kernel size limits (checked on the host before any launch).
constexpr int kMaxFreq = 33;       // omega = 0 plus up to 32 quadrature nodes
constexpr int kMaxNmax = 12;       // highest body order
constexpr int kMaxN1 = 256;        // atoms in K1 (r < r_scs), central atom included
constexpr double kSparseMbdRatio = 0.45;  // automatic sparse MBD products when r_mbd2 <= this * r_nbr
constexpr int kMaxNK = 400;        // sites in K (r < r_nbr), central atom included; the MBD kernel's LDS,
                                   // 8 (3 nq + 15) bytes per site for nq >= 12 nodes, caps it lower for
                                   // long grids (the host checks that limit too)
constexpr int kMaxSites = 32768;   // sites in the largest ball, central atom included (20 + 14 A at carbon density)
constexpr int kFitNodes = 32;      // Gauss-Legendre points of the least-squares fit of ln(1 - x)
constexpr int kMaxLanczos = 64;    // Lanczos steps for the spectrum bounds

// One site of a neighbourhood: an atom or one of its periodic images, stored
// relative to the central atom.  32 bytes.
struct Site {
    double x, y, z;   // position relative to the central atom, bohr
    int32_t base;     // batch-global index of the atom it is an image of
    int32_t shift;    // lattice shift packed as 3 x 8 bits, each biased by 128
};

__host__ __device__ inline int32_t pack_shift(int a, int b, int c) {
    return ((a + 128) << 16) | ((b + 128) << 8) | (c + 128);
}
__host__ __device__ inline void unpack_shift(int32_t s, int& a, int& b, int& c) {
    a = ((s >> 16) & 255) - 128;
    b = ((s >> 8) & 255) - 128;
    c = (s & 255) - 128;
}

// Per-structure data on the device.
struct StructInfo {
    double cell[9];      // rows = lattice vectors, bohr (open: diagonal grid box)
    double inv[9];       // inverse of cell: frac = pos @ inv
    double origin[3];    // open structures: lower corner of the bounding box, bohr
    double flo[3];       // periodic structures, non-periodic directions: lowest fractional coordinate
    double fext[3];      //   and the extent of the fractional coordinates (cells span it)
    int periodic;        // 1 = periodic along at least one lattice direction, 0 = open
    int pbc[3];          // periodic along lattice direction d
    int ncell[3];        // cell-list grid
    int reach[3];        // cells to visit on each side
    int cell_offset;     // first batch-global cell index
    int atom_offset;     // first batch-global atom index
    int n_atoms;
    int m2max;           // largest Counts::n_m2 of the structure's atoms (bounds the sparse rows)
    int two_body;        // the n = 2 term has radii of its own (r_2b1, r_2b2 differ from r_mbd1, r_mbd2)
    double r_scs, r_nbr, r_mbd1, r_mbd2, r_big;  // bohr
    double r_2b1, r_2b2;                          // bohr (equal to r_mbd1, r_mbd2 unless set)
};

// Per-atom neighbourhood counts (central atom included in every count).
struct Counts {
    int32_t n_all;   // sites with r < r_big = max(2 r_scs, r_nbr)
    int32_t n1;      // r < r_scs       (K1 of the SCS)
    int32_t nK;      // r < r_nbr       (K of the energy)
    int32_t n12;     // r < 2 r_scs     (K1 plus the uncoupled shell K2)
    int32_t n_m2;    // r < r_mbd2      (the sites a block row other than the central one couples to)
};

// ---------------------------------------------------------------------------
// Pair functions (device), templated on the arithmetic type P (double, or float
// for the mixed-precision path).  r in bohr.
// ---------------------------------------------------------------------------
__device__ inline double m_exp(double x) { return exp(x); }
__device__ inline float m_exp(float x) { return expf(x); }
__device__ inline double m_erf(double x) { return erf(x); }
__device__ inline float m_erf(float x) { return erff(x); }
__device__ inline double m_sqrt(double x) { return sqrt(x); }
__device__ inline float m_sqrt(float x) { return sqrtf(x); }

// Fermi damping f(r, S) = 1 / (1 + exp(-d (r / S - 1))) and its partial
// derivatives: df/dr = d f (1 - f) / S, df/dS = -d r f (1 - f) / S^2.
template <typename P>
__device__ inline P fermi(P r, P S, P d, P& dfdr, P& dfdS) {
    const P iS = P(1) / S;
    const P f = P(1) / (P(1) + m_exp(-d * (r * iS - P(1))));
    const P g = d * f * (P(1) - f) * iS;
    dfdr = g;
    dfdS = -g * r * iS;
    return f;
}

// Smooth cutoff: 1 below rc - rb, 1 - 3x^2 + 2x^3 with x = (r - rc + rb)/rb in
// the buffer, 0 from rc on; returns value and d/dr.
template <typename P>
__device__ inline P cutoff_poly(P r, P rc, P rb, P& dcdr) {
    if (r < rc - rb) { dcdr = P(0); return P(1); }
    if (r >= rc) { dcdr = P(0); return P(0); }
    const P irb = P(1) / rb;
    const P x = (r - rc + rb) * irb;
    dcdr = (P(-6) * x + P(6) * x * x) * irb;
    return P(1) - P(3) * x * x + P(2) * x * x * x;
}

// Radial decomposition of a symmetric pair tensor M(r_vec) = A(r) rhat rhat^T + B(r) I.
// Its gradient contracted with a symmetric 3x3 matrix C is
//   sum_ab C_ab dM_ab/dr_g = (A' - 2A/r)(rhat.C.rhat) rhat_g + (2A/r)(C rhat)_g + B' tr(C) rhat_g,
// using d rhat_a / dr_g = (delta_ag - rhat_a rhat_g) / r.
__device__ inline void radial_tensor_grad(const double rh[3], double r, double A, double dA,
                                          double dB, const double C[9], double g[3]) {
    const double Cr0 = C[0] * rh[0] + C[1] * rh[1] + C[2] * rh[2];
    const double Cr1 = C[3] * rh[0] + C[4] * rh[1] + C[5] * rh[2];
    const double Cr2 = C[6] * rh[0] + C[7] * rh[1] + C[8] * rh[2];
    const double rCr = rh[0] * Cr0 + rh[1] * Cr1 + rh[2] * Cr2;
    const double tr = C[0] + C[4] + C[8];
    const double a = (dA - 2.0 * A / r) * rCr + dB * tr;
    const double b = 2.0 * A / r;
    g[0] = a * rh[0] + b * Cr0;
    g[1] = a * rh[1] + b * Cr1;
    g[2] = a * rh[2] + b * Cr2;
}

// Coefficients of the short-range core H = -T g + h = -(Hessian of erf(r/s)/r)
// written as A rhat rhat^T + B I:
//   A = -(3 g - 2 c u^3 e) / r^3,  B = g / r^3,  c = 2/sqrt(pi), u = r/s, e = exp(-u^2)
// with g = erf(u) - c u e (Sec. II.B, T_SR with the g and h functions).
template <typename P>
__device__ inline void sr_core(P r, P ir, P s, P& A, P& B, P& dA, P& dB) {
    const P c = P(kTwoOverSqrtPi);
    const P u = r / s;
    const P e = m_exp(-u * u);
    const P g = m_erf(u) - c * u * e;
    const P u3e = u * u * u * e;
    const P ir3 = ir * ir * ir;
    const P ir4 = ir3 * ir;
    const P Pc = P(3) * g - P(2) * c * u3e;       // A = -Pc / r^3
    // dPc/dr = 4 c u^5 e / r  (from g' = 2 c u^3 e / r and (u^3 e)' = (3 - 2u^2) u^3 e / r)
    const P dP = P(4) * c * u3e * u * u * ir;
    A = -Pc * ir3;
    dA = -dP * ir3 + P(3) * Pc * ir4;
    B = g * ir3;
    dB = P(2) * c * u3e * ir4 - P(3) * g * ir4;
}

// ---------------------------------------------------------------------------
// Kernel argument blocks and host launchers
// ---------------------------------------------------------------------------
struct NbrArgs {
    int n;
    const double* pos_b;
    const int32_t* atom_struct;
    const StructInfo* sinfo;
    const int32_t* cell_id;
    const int32_t* wrap;
    const int32_t* cell_start;
    const int32_t* cell_end;
    const int32_t* sorted_atoms;
    int32_t* wcounts;   // per atom and wavefront of the search: counts (all, r_scs, r_nbr, 2 r_scs)
};
constexpr int kNbrWaves = 4;   // wavefronts per atom in the neighbour search (each a block of the cell stencil)

struct ScsArgs {
    int n, nw;
    int n_refine;            // refinement steps of the FP32 solve (mixed precision)
    const Counts* counts;
    const int32_t* order;    // per-atom launches: workgroup x takes atom order[x] (largest neighbourhoods first)
    const int64_t* site_off;
    const Site* sites;
    const double* abar;      // [n][nw]
    const double* sigma;     // [n][nw]
    const double* Rv;        // [n]
    const int32_t* atom_struct;
    const StructInfo* sinfo;
    double beta, damp_d, r_buf, r_inner;   // bohr
    void* fac;               // factor slots (double or float): per atom nw * N * ld, row-major lower,
                             // inverses of the 16x16 diagonal blocks in their strict upper parts
    const int64_t* fac_off;
    const int32_t* fac_ld;   // ld >= N, a multiple of 4; per (atom, frequency) N + 3 rows: B~, then d^T
    float* coef;             // mixed path: FP32 pair coefficients (A, B) of B~, per atom nw * n1 (n1 + 1) / 2 pairs
    const int64_t* coef_off; // per atom, in floats
    double* xsol;            // per atom nw * N * 3 (row-major): d, then the solution X
    double* dvec;            // mixed path: d (same layout)
    double* resid;           // mixed path: refinement residual (same layout)
    double* lam;             // forces: adjoint solution lambda (same layout)
    const int64_t* x_off;
    double* alpha_loc;       // per atom n1 * nw
    const int64_t* aloc_off;
    // pair lists of one atom (frequency independent), per atom a block of
    // n1 n2 + n1 (n1 - 1) / 2 entries in each of pl_i and pl_q:
    //   K1 x K2 (r_iq < r_scs): pl_q[0 ..) shell-major, entries (q << 16) | i;
    //                           pl_i[0 ..) i-major, entries = index into the shell-major list
    //   K1 x K1 (a < b, r_ab < r_scs), from n1 n2 on:
    //                           pl_i a-major, entries (a << 16) | b;
    //                           pl_q b-major, entries = index into the a-major list
    // each list is ordered by major site (shell-major and a-major lists in a
    // scrambled order of the majors), then minor index; index lists ascend
    const int32_t* pl_i;
    const int32_t* pl_q;
    const int64_t* pl_off;   // per atom: first entry of the block
    const int32_t* pl_seg;   // per atom at 3 (site_off[k] + 2k): segment starts per major site, then
                             //   the total: i (n1 + 1), q (n2 + 1), a (n1 + 1), b (n1 + 1)
    int* err;
    int* err_atom;
    // adjoint only
    const double* abar_loc;  // per atom n1 * nw: adjoint of the local polarisabilities
    const double* abar_cen;  // [n][nw]: adjoint of the central polarisabilities
    double* cf;              // force contributions [nw][total_sites][3] (slice base)
    int64_t cf_slice;        // stride between frequency slices
    double* cnu;             // volume-ratio adjoint numerators [total_sites][nw] (dE_dv)
};

struct MbdArgs {
    int n, nw, nq, n_max, ncol, mmax;   // nw: SCS frequencies (stride of the polarisability arrays)
    const Counts* counts;
    const int32_t* order;      // workgroup x takes atom order[x] (largest neighbourhoods first)
    const int64_t* site_off;
    const Site* sites;
    const double* alpha_loc;   // per atom n1 * nw
    const int64_t* aloc_off;
    const double* a0v;
    const double* r0v;
    const int32_t* atom_struct;
    const StructInfo* sinfo;
    double beta, damp_d, r_buf;
    double coef[kMaxNmax + 1];
    double wq[kMaxFreq];       // quadrature weight * Hartree / (2 pi): eV per unit integrand
    int lorentz;               // SCS solved at 0 and omega_ref only (nw = 2): two-point Lorentzian at the nodes
    int paper;                 // adjoint of the approximate forces of Sec. III.D instead of the exact one
    double rho[kMaxFreq];      // two-point model: (omega_q / omega_ref)^2
    int fit;                   // c_n per atom and node: least-squares polynomial of ln(1 - x) on the
                               // Lanczos bounds of the spectrum of G~ (Sec. III.A)
    int lz_steps;              // Lanczos steps (0: no Lanczos iteration)
    double gl_x[kFitNodes];    // Gauss-Legendre nodes and weights on [-1, 1] of the fit
    double gl_w[kFitNodes];
    double* spectrum;          // [n][nq][2] Lanczos bounds (batch-global atom index), or null
    int* err;                  // bit 8: a polarisability rises between 0 and omega_ref;
                               // bit 16: a spectrum bound reaches 1 with the fitted c_n;
                               // bit 32: the coupled-site lists outgrew their capacity
    int* err_atom;             // lowest atom whose frame raised an error
    const double* e_weight;    // [n] or null
    double* e_atom;            // [n]
    void* work;                // per atom T (N3^2), U (mmax N3 ncol), V (N3 ncol), with forces P^T and
                               // Q^T (n_max ncol x N3 each): double or float
    const int64_t* work_off;
    int forces;
    double* abar_loc;          // per atom n1 * nw (aloc_off)
    double* ca;                // [total_sites][nw]
    double* cf0;               // [total_sites][3]
};

hipError_t launch_prep(hipStream_t st, int n, const double* pos_A, const int32_t* species,
                       const double* nu, const int32_t* atom_struct, const StructInfo* sinfo,
                       const double* sp_table, int n_species, const double* omegas, int nw,
                       double* pos_b, double* abar, double* sigma, double* Rv, double* a0v,
                       double* r0v, int32_t* cell_id, int32_t* wrap, int* err);
hipError_t sort_cells(hipStream_t st, int n, int n_cells, const int32_t* cell_id,
                      const int32_t* iota, int32_t* sorted_cell, int32_t* sorted_atoms,
                      void* temp, size_t* temp_bytes, int32_t* cell_start, int32_t* cell_end);
hipError_t launch_nbr_count(hipStream_t st, const NbrArgs& a, Counts* counts);
hipError_t launch_nbr_fill(hipStream_t st, const NbrArgs& a, const Counts* counts,
                           const int64_t* site_off, Site* sites);
hipError_t launch_rev_map(hipStream_t st, int n, const Counts* counts, const int64_t* site_off,
                          const Site* sites, const int64_t* hash_off, const int32_t* hash_cap,
                          int32_t* table, size_t table_len, int32_t* rev, int* err);
size_t scs_lds_bytes(int n1max, int n2max, bool mixed);
size_t scs_assemble_lds_bytes(int n1max, int n2max);
size_t pairlist_lds_bytes(int n1max, int n2max);
// d (to its slot) and d^T (the rows appended to B~); B~ itself is assembled by the factorisation kernel
hipError_t launch_scs_rhs(hipStream_t st, const ScsArgs& a, int n1max, int n2max, bool mixed);
hipError_t launch_scs_factor(hipStream_t st, const ScsArgs& a, int n1max, bool mixed);
size_t scs_factor_lds_bytes(int n1max, bool mixed);
hipError_t launch_scs_lambda(hipStream_t st, const ScsArgs& a, int n1max, bool mixed);
hipError_t launch_pairlist(hipStream_t st, const ScsArgs& a, int n1max, int n2max);
hipError_t launch_scs_adjoint(hipStream_t st, const ScsArgs& a, int n1max, int n2max, bool mixed);
// per (atom, frequency) and site: the numerator of the site's share of d E / d nu (into a.cnu)
hipError_t launch_scs_nu(hipStream_t st, const ScsArgs& a, int n1max, int n2max);
// dE_dv[a] = (sum over the slots that refer to a, over frequencies) / nu_a
hipError_t launch_gather_nu(hipStream_t st, int n, int nw, const Counts* counts, const int64_t* site_off,
                            const Site* sites, const int32_t* rev, const double* cnu, const double* nu,
                            double* dv);
// Doubles of the MBD stage's per-site arrays for nk sites and nq nodes: positions (3),
// blended polarisabilities at 0 and the nodes (nq + 1), their square roots at the nodes
// (max(nq, 12): the force stage's pair sums take their place), SCS radii, f_SCS and its
// derivative (3), polarisability adjoints (nq + 1), radius-adjoint parts (4), blend
// gradients (3).  In LDS, or in the workspace for the sparse form with global site arrays.
__host__ __device__ inline size_t mbd_site_doubles(size_t nk, int nq) {
    const size_t nw = (size_t)nq + 1;
    return 3 * nk + nk * nw + nk * (size_t)(nq > 12 ? nq : 12) + 3 * nk + nk * nw + 4 * nk + 3 * nk;
}
// Doubles of the small per-atom LDS arrays: moments, fitted coefficients, Lanczos state.
__host__ __device__ inline size_t mbd_small_doubles(int nq, int n_max, int lz_steps, bool fit) {
    return (size_t)(n_max + 1) * nq + (fit ? 2 * (size_t)(kMaxNmax + 1) * nq : 0) +
           (lz_steps > 0 ? (2 * (size_t)lz_steps + 3) * nq : 0);
}
// Capacity (entries) of the coupled-site lists of an atom with nK sites in the sparse form
// with global site arrays: the central row couples to at most nK - 1 sites, every other row
// to at most m2max - 1 sites within r_mbd2 plus the central atom (m2max: the structure's
// largest count of sites within r_mbd2, itself included); two entries of slack per row.
__host__ __device__ inline int64_t mbd_list_cap(int nK, int m2max) {
    return (int64_t)(nK - 1) * (m2max + 2) + nK;
}
// Per-atom workspace of that form, offsets in elements of the workspace type (size wsz),
// each part on a 16-byte boundary: site arrays (double), the lists (cap entries of five
// coefficients A, B, rhat of type W and one int32 site index; nK + 1 int32 row offsets),
// the Krylov blocks, the two Lanczos/operand buffers and, with forces, P and Q.
struct MbdGlobalLayout {
    int64_t sites, lists, U, V, V2, P, Q, total;
};
__host__ __device__ inline MbdGlobalLayout mbd_global_layout(int nK, int nq, int n_max, int mmax, int64_t cap,
                                                             int64_t wsz, bool forces) {
    const int64_t N3 = 3 * (int64_t)nK, N3p = (N3 + 3) / 4 * 4, ncol = 3 * (int64_t)nq;
    const int64_t KKp = ((int64_t)n_max * ncol + 3) / 4 * 4;
    int64_t o = 0;
    MbdGlobalLayout g;
    auto take = [&](int64_t bytes) {
        const int64_t at = o;
        o += (bytes + 15) / 16 * 16;
        return at / wsz;
    };
    g.sites = take(8 * (int64_t)mbd_site_doubles((size_t)nK, nq));
    g.lists = take(cap * (5 * wsz + 4) + 4 * ((int64_t)nK + 1));
    g.U = take(wsz * mmax * N3 * ncol);
    g.V = take(wsz * ncol * N3p);
    g.V2 = take(wsz * ncol * N3p);
    g.P = take(forces ? wsz * N3 * KKp : 0);
    g.Q = take(forces ? wsz * N3 * KKp : 0);
    g.total = o / wsz;
    return g;
}
// MBD kernel forms: dense T_LR on the matrix cores; sparse products with the per-site
// arrays in LDS; sparse products with them in the workspace (neighbourhoods too large for LDS)
enum { kMbdDense = 0, kMbdSparse = 1, kMbdSparseGlobal = 2 };
constexpr size_t kLdsBytes = 160 * 1024;   // LDS of a gfx950 workgroup
size_t mbd_lds_bytes(int nkmax, int nq, int n_max, int lz_steps, bool fit);
// two_body: every atom of the launch belongs to a structure with two-body radii of its own
hipError_t launch_mbd(hipStream_t st, const MbdArgs& a, int nkmax, bool mixed, int form, bool two_body);
hipError_t launch_gather_central(hipStream_t st, int n, int nw, const Counts* counts,
                                 const int64_t* site_off, const Site* sites, const int32_t* rev,
                                 const double* ca, double* abar_cen);
// out[0 .. n) = v
hipError_t launch_fill(hipStream_t st, int n, double v, double* out);
hipError_t launch_gather_forces(hipStream_t st, int n, int nslices, int64_t slice_stride,
                                const Counts* counts, const int64_t* site_off, const Site* sites,
                                const int32_t* rev, double* cf, double* forces);
// F[a] = sum over the sites s of a's own list with base(s) = a of the slot sums (the
// gradient of a's own frame with respect to r_a; approximate forces of Sec. III.D)
hipError_t launch_gather_self(hipStream_t st, int n, int nslices, int64_t slice_stride, const Counts* counts,
                              const int64_t* site_off, const Site* sites, double* cf, double* forces);
hipError_t launch_central_static(hipStream_t st, int n, int nw, const double* alpha_loc,
                                 const int64_t* aloc_off, double* out);

}  // namespace lmbd
