// Per-atom preparation and neighbourhood construction.
//
// For every atom k the library needs the ball of sites (atoms and periodic
// images) of radius r_big = max(2 r_scs, r_nbr) around it, split into
//   K1 = B(r_scs), K2 = B(2 r_scs) \ B(r_scs)   (local SCS, Sec. III.B)
//   K  = B(r_nbr)                               (local energy, Sec. III.A)
// Each list starts with the central atom; the remaining sites are grouped by
// the distance intervals cut at the sorted radii, so K1, K1 u K2 and K are all
// prefixes of the list.  Within a group the order is the deterministic
// traversal order of the cell list (cells in fixed order, atoms by index).
//
// Pair vectors are computed in a canonical orientation (from the lower to the
// higher atom index) so that site j of atom k and site k of atom j have bitwise
// equal distances: membership is symmetric, which the reverse-slot map needs.
#include "lmbd_internal.h"

#include <hipcub/hipcub.hpp>

namespace lmbd {

// lattice translation t . cell with a fixed evaluation order
__device__ inline void lattice_vec(const double* c, int t0, int t1, int t2, double out[3]) {
    out[0] = fma((double)t2, c[6], fma((double)t1, c[3], (double)t0 * c[0]));
    out[1] = fma((double)t2, c[7], fma((double)t1, c[4], (double)t0 * c[1]));
    out[2] = fma((double)t2, c[8], fma((double)t1, c[5], (double)t0 * c[2]));
}

__device__ inline bool lex_positive(int a, int b, int c) {
    return a > 0 || (a == 0 && (b > 0 || (b == 0 && c > 0)));
}

// Vector from the central atom kc to site (j, t) in the canonical orientation.
__device__ inline void canonical_rel(const double* __restrict__ pos, const double* cell, int kc,
                                     int j, int t0, int t1, int t2, double v[3]) {
    if (j > kc || (j == kc && lex_positive(t0, t1, t2))) {
        double T[3];
        lattice_vec(cell, t0, t1, t2, T);
        v[0] = (pos[3 * j + 0] + T[0]) - pos[3 * kc + 0];
        v[1] = (pos[3 * j + 1] + T[1]) - pos[3 * kc + 1];
        v[2] = (pos[3 * j + 2] + T[2]) - pos[3 * kc + 2];
    } else {
        double T[3];
        lattice_vec(cell, -t0, -t1, -t2, T);
        v[0] = -((pos[3 * kc + 0] + T[0]) - pos[3 * j + 0]);
        v[1] = -((pos[3 * kc + 1] + T[1]) - pos[3 * j + 1]);
        v[2] = -((pos[3 * kc + 2] + T[2]) - pos[3 * j + 2]);
    }
}

__device__ inline double norm2(const double v[3]) {
    return fma(v[2], v[2], fma(v[1], v[1], v[0] * v[0]));
}

// ---------------------------------------------------------------------------
// k_prep: positions to bohr, free-atom tables (Sec. II.B), cell assignment.
//   omega_i = 4 C6 / (3 alpha0^2); abar_i(w) = alpha0 nu / (1 + (w/omega_i)^2);
//   sigma_i(w) = (sqrt(2/pi) abar_i(w) / 3)^(1/3); R_i = R0 nu^(1/3).
// ---------------------------------------------------------------------------
__global__ void k_prep(int n, const double* __restrict__ pos_A, const int32_t* __restrict__ species,
                       const double* __restrict__ nu, const int32_t* __restrict__ atom_struct,
                       const StructInfo* __restrict__ sinfo, const double* __restrict__ sp_table,
                       int n_species, const double* __restrict__ omegas, int nw,
                       double* __restrict__ pos_b, double* __restrict__ abar,
                       double* __restrict__ sigma, double* __restrict__ Rv,
                       double* __restrict__ a0v, double* __restrict__ r0v,
                       int32_t* __restrict__ cell_id, int32_t* __restrict__ wrap,
                       int* __restrict__ err) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const StructInfo& S = sinfo[atom_struct[g]];
    double p[3];
    bool ok = true;
    for (int d = 0; d < 3; ++d) {
        p[d] = pos_A[3 * g + d] / kBohr;
        ok = ok && isfinite(p[d]);
        pos_b[3 * g + d] = p[d];
    }
    const int sp = species[g];
    const double v = nu[g];
    if (sp < 0 || sp >= n_species || !(v > 0.0) || !isfinite(v) || !ok) {
        atomicOr(err, 1);
        cell_id[g] = S.cell_offset;
        for (int d = 0; d < 3; ++d) wrap[3 * g + d] = 0;
        return;
    }
    const double al0 = sp_table[3 * sp + 0];
    const double c6 = sp_table[3 * sp + 1];
    const double rr0 = sp_table[3 * sp + 2];
    const double om = 4.0 * c6 / (3.0 * al0 * al0);
    for (int w = 0; w < nw; ++w) {
        const double x = omegas[w] / om;
        const double a = al0 * v / (1.0 + x * x);
        abar[(size_t)g * nw + w] = a;
        sigma[(size_t)g * nw + w] = cbrt(kSqrt2OverPi * a / 3.0);
    }
    Rv[g] = rr0 * cbrt(v);
    a0v[g] = al0;
    r0v[g] = rr0;

    int c[3], wr[3];
    if (S.periodic) {
        for (int d = 0; d < 3; ++d) {
            const double f = p[0] * S.inv[d] + p[1] * S.inv[3 + d] + p[2] * S.inv[6 + d];
            int cc;
            if (S.pbc[d]) {
                const double fl = floor(f);
                wr[d] = (int)fl;
                cc = (int)((f - fl) * S.ncell[d]);
            } else {   // a non-periodic direction of a periodic structure: cells over the atoms' extent
                wr[d] = 0;
                cc = (int)((f - S.flo[d]) / S.fext[d] * S.ncell[d]);
            }
            c[d] = cc < 0 ? 0 : (cc >= S.ncell[d] ? S.ncell[d] - 1 : cc);
        }
    } else {
        for (int d = 0; d < 3; ++d) {
            const double h = S.cell[4 * d] / S.ncell[d];
            int cc = (int)((p[d] - S.origin[d]) / h);
            c[d] = cc < 0 ? 0 : (cc >= S.ncell[d] ? S.ncell[d] - 1 : cc);
            wr[d] = 0;
        }
    }
    cell_id[g] = S.cell_offset + (c[0] * S.ncell[1] + c[1]) * S.ncell[2] + c[2];
    for (int d = 0; d < 3; ++d) wrap[3 * g + d] = wr[d];
}

// cell_start/cell_end from the sorted cell ids
__global__ void k_cell_ranges(int n, const int32_t* __restrict__ sorted_cell,
                              int32_t* __restrict__ cell_start, int32_t* __restrict__ cell_end) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = sorted_cell[i];
    if (i == 0 || sorted_cell[i - 1] != c) cell_start[c] = i;
    if (i == n - 1 || sorted_cell[i + 1] != c) cell_end[c] = i + 1;
}


// number of cells in the search stencil of a structure
__device__ inline int stencil_cells(const StructInfo& S) {
    return (2 * S.reach[0] + 1) * (2 * S.reach[1] + 1) * (2 * S.reach[2] + 1);
}

// Visit the candidate sites of atom k in the stencil cells [c_begin, c_end)
// (dx slowest, dz fastest; one wavefront) in a fixed order; `fn(valid, j, t0,
// t1, t2, v, d2)` is called once per chunk of 64 lanes.  Consecutive blocks of
// the stencil visited one after the other give the order of the whole stencil.
template <typename F>
__device__ inline void visit_candidates(const NbrArgs& a, int k, int lane, int c_begin, int c_end, F fn) {
    const StructInfo& S = a.sinfo[a.atom_struct[k]];
    const int local = a.cell_id[k] - S.cell_offset;
    const int ck[3] = {local / (S.ncell[1] * S.ncell[2]), (local / S.ncell[2]) % S.ncell[1],
                       local % S.ncell[2]};
    const int wk0 = a.wrap[3 * k], wk1 = a.wrap[3 * k + 1], wk2 = a.wrap[3 * k + 2];
    const int ny = 2 * S.reach[1] + 1, nz = 2 * S.reach[2] + 1;
    for (int c = c_begin; c < c_end; ++c) {
                const int dx = c / (ny * nz) - S.reach[0], dy = (c / nz) % ny - S.reach[1], dz = c % nz - S.reach[2];
                int cc[3] = {ck[0] + dx, ck[1] + dy, ck[2] + dz};
                int sh[3] = {0, 0, 0};
                bool inside = true;
                for (int d = 0; d < 3; ++d) {
                    if (S.pbc[d]) {
                        const int m = S.ncell[d];
                        const int q = (cc[d] >= 0) ? cc[d] / m : -((-cc[d] + m - 1) / m);
                        sh[d] = q;
                        cc[d] -= q * m;
                    } else if (cc[d] < 0 || cc[d] >= S.ncell[d]) {
                        inside = false;
                    }
                }
                if (!inside) continue;
                const int gc = S.cell_offset + (cc[0] * S.ncell[1] + cc[1]) * S.ncell[2] + cc[2];
                const int beg = a.cell_start[gc], end = a.cell_end[gc];
                for (int b0 = beg; b0 < end; b0 += 64) {
                    const int i = b0 + lane;
                    const bool in = i < end;
                    int j = k, t0 = 0, t1 = 0, t2 = 0;
                    double v[3] = {0.0, 0.0, 0.0};
                    double d2 = 0.0;
                    if (in) {
                        j = a.sorted_atoms[i];
                        t0 = sh[0] - a.wrap[3 * j] + wk0;
                        t1 = sh[1] - a.wrap[3 * j + 1] + wk1;
                        t2 = sh[2] - a.wrap[3 * j + 2] + wk2;
                        canonical_rel(a.pos_b, S.cell, k, j, t0, t1, t2, v);
                        d2 = norm2(v);
                    }
                    const bool self = (j == k && t0 == 0 && t1 == 0 && t2 == 0);
                    fn(in && !self && d2 < S.r_big * S.r_big, j, t0, t1, t2, v, d2);
                }
            }
}

// one atom per workgroup, wavefront w counting the w-th block of the stencil
__device__ inline void stencil_block(const StructInfo& S, int w, int& c0, int& c1) {
    const int C = stencil_cells(S);
    c0 = (int)((int64_t)C * w / kNbrWaves);
    c1 = (int)((int64_t)C * (w + 1) / kNbrWaves);
}

__global__ void __launch_bounds__(64 * kNbrWaves) k_nbr_count(NbrArgs a, Counts* __restrict__ counts) {
    __shared__ int part[kNbrWaves][5];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int k = blockIdx.x;
    const StructInfo& S = a.sinfo[a.atom_struct[k]];
    const double r1 = S.r_scs * S.r_scs, rK = S.r_nbr * S.r_nbr, r2 = 4.0 * S.r_scs * S.r_scs,
                 rM2 = S.r_mbd2 * S.r_mbd2;
    int c_all = 0, c1 = 0, cK = 0, c12 = 0, cM2 = 0;
    int cb, ce;
    stencil_block(S, wave, cb, ce);
    visit_candidates(a, k, lane, cb, ce, [&](bool valid, int, int, int, int, const double*, double d2) {
        if (valid) {
            c_all += 1;
            c1 += d2 < r1;
            cK += d2 < rK;
            c12 += d2 < r2;
            cM2 += d2 < rM2;
        }
    });
    for (int off = 32; off > 0; off >>= 1) {
        c_all += __shfl_xor(c_all, off);
        c1 += __shfl_xor(c1, off);
        cK += __shfl_xor(cK, off);
        c12 += __shfl_xor(c12, off);
        cM2 += __shfl_xor(cM2, off);
    }
    if (lane == 0) {
        int32_t* wc = a.wcounts + ((size_t)k * kNbrWaves + wave) * 4;
        wc[0] = c_all;
        wc[1] = c1;
        wc[2] = cK;
        wc[3] = c12;
        part[wave][0] = c_all;
        part[wave][1] = c1;
        part[wave][2] = cK;
        part[wave][3] = c12;
        part[wave][4] = cM2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int t[5] = {0, 0, 0, 0, 0};
        for (int w = 0; w < kNbrWaves; ++w)
            for (int q = 0; q < 5; ++q) t[q] += part[w][q];
        counts[k] = Counts{1 + t[0], 1 + t[1], 1 + t[2], 1 + t[3], 1 + t[4]};
    }
}

// one atom per workgroup: wavefront w fills from the w-th block of the
// stencil, each of its site classes starting after the sites the blocks before
// it found (their counts come from k_nbr_count), so the order is that of one
// pass over the whole stencil
__global__ void __launch_bounds__(64 * kNbrWaves) k_nbr_fill(NbrArgs a, const Counts* __restrict__ counts,
                                                  const int64_t* __restrict__ site_off,
                                                  Site* __restrict__ sites) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int k = blockIdx.x;
    const StructInfo& S = a.sinfo[a.atom_struct[k]];
    Site* out = sites + site_off[k];
    const Counts c = counts[k];
    // sorted thresholds and the counts below each (whole stencil, and in the
    // blocks before this wavefront's); counts index 1, 2, 3 = r_scs, r_nbr, 2 r_scs
    double th[3] = {S.r_scs, S.r_nbr, 2.0 * S.r_scs};
    int below[3] = {c.n1 - 1, c.nK - 1, c.n12 - 1};
    int idx[3] = {1, 2, 3};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (th[j] < th[i]) {
                double t = th[i]; th[i] = th[j]; th[j] = t;
                int b = below[i]; below[i] = below[j]; below[j] = b;
                int x = idx[i]; idx[i] = idx[j]; idx[j] = x;
            }
    int before[3] = {0, 0, 0};   // sites of each class found by the earlier blocks
    for (int w = 0; w < wave; ++w) {
        const int32_t* wc = a.wcounts + ((size_t)k * kNbrWaves + w) * 4;
        before[0] += wc[idx[0]];
        before[1] += wc[idx[1]] - wc[idx[0]];
        before[2] += wc[0] - wc[idx[1]];
    }
    const double t0s = th[0] * th[0], t1s = th[1] * th[1];
    int cursor[3] = {1 + before[0], 1 + below[0] + before[1], 1 + below[1] + before[2]};
    if (lane == 0 && wave == 0) out[0] = Site{0.0, 0.0, 0.0, k, pack_shift(0, 0, 0)};
    int cb, ce;
    stencil_block(S, wave, cb, ce);
    visit_candidates(a, k, lane, cb, ce, [&](bool valid, int j, int t0, int t1, int t2, const double* v,
                                     double d2) {
        const int cls = d2 < t0s ? 0 : (d2 < t1s ? 1 : 2);
        const uint64_t below_me = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const uint64_t m = __ballot(valid && cls == q);
            if (valid && cls == q) {
                const int slot = cursor[q] + __popcll(m & below_me);
                out[slot] = Site{v[0], v[1], v[2], j, pack_shift(t0, t1, t2)};
            }
            cursor[q] += __popcll(m);
        }
    });
}

// ---------------------------------------------------------------------------
// Reverse-slot map: for entry s of atom a (site (j, t)), the slot of (a, -t) in
// the list of j.  Built with one open-addressing hash table per atom.
// ---------------------------------------------------------------------------
__device__ inline uint64_t site_key(int base, int32_t shift) {
    return ((uint64_t)(uint32_t)base << 24) | (uint64_t)(shift & 0xFFFFFF);
}
__device__ inline uint32_t hash_key(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return (uint32_t)x;
}

__global__ void __launch_bounds__(256) k_hash_build(int n, const Counts* __restrict__ counts,
                                                    const int64_t* __restrict__ site_off,
                                                    const Site* __restrict__ sites,
                                                    const int64_t* __restrict__ hash_off,
                                                    const int32_t* __restrict__ hash_cap,
                                                    int32_t* __restrict__ table) {
    const int k = blockIdx.x;
    if (k >= n) return;
    const Site* L = sites + site_off[k];
    int32_t* T = table + hash_off[k];
    const uint32_t mask = (uint32_t)hash_cap[k] - 1u;
    for (int s = threadIdx.x; s < counts[k].n_all; s += blockDim.x) {
        uint32_t h = hash_key(site_key(L[s].base, L[s].shift)) & mask;
        while (atomicCAS(&T[h], -1, s) != -1) h = (h + 1) & mask;
    }
}

__global__ void __launch_bounds__(256) k_rev_map(int n, const Counts* __restrict__ counts,
                                                 const int64_t* __restrict__ site_off,
                                                 const Site* __restrict__ sites,
                                                 const int64_t* __restrict__ hash_off,
                                                 const int32_t* __restrict__ hash_cap,
                                                 const int32_t* __restrict__ table,
                                                 int32_t* __restrict__ rev, int* __restrict__ err) {
    const int a = blockIdx.x;
    if (a >= n) return;
    const Site* L = sites + site_off[a];
    for (int s = threadIdx.x; s < counts[a].n_all; s += blockDim.x) {
        const int j = L[s].base;
        int t0, t1, t2;
        unpack_shift(L[s].shift, t0, t1, t2);
        const uint64_t key = site_key(a, pack_shift(-t0, -t1, -t2));
        const Site* Lj = sites + site_off[j];
        const int32_t* T = table + hash_off[j];
        const uint32_t cap = (uint32_t)hash_cap[j];
        uint32_t h = hash_key(key) & (cap - 1u);
        int found = -1;
        for (uint32_t probe = 0; probe < cap; ++probe) {
            const int slot = T[h];
            if (slot < 0) break;
            if (site_key(Lj[slot].base, Lj[slot].shift) == key) { found = slot; break; }
            h = (h + 1) & (cap - 1u);
        }
        if (found < 0) atomicOr(err, 2);
        rev[site_off[a] + s] = found < 0 ? 0 : found;
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t launch_prep(hipStream_t st, int n, const double* pos_A, const int32_t* species,
                       const double* nu, const int32_t* atom_struct, const StructInfo* sinfo,
                       const double* sp_table, int n_species, const double* omegas, int nw,
                       double* pos_b, double* abar, double* sigma, double* Rv, double* a0v,
                       double* r0v, int32_t* cell_id, int32_t* wrap, int* err) {
    hipLaunchKernelGGL(k_prep, dim3((n + 255) / 256), dim3(256), 0, st, n, pos_A, species, nu,
                       atom_struct, sinfo, sp_table, n_species, omegas, nw, pos_b, abar, sigma, Rv,
                       a0v, r0v, cell_id, wrap, err);
    return hipGetLastError();
}

// Sort atoms by cell id (stable radix sort: atoms of one cell stay in index order).
hipError_t sort_cells(hipStream_t st, int n, int n_cells, const int32_t* cell_id,
                      const int32_t* iota, int32_t* sorted_cell, int32_t* sorted_atoms,
                      void* temp, size_t* temp_bytes, int32_t* cell_start, int32_t* cell_end) {
    int end_bit = 1;
    while ((1 << end_bit) < n_cells + 1 && end_bit < 31) ++end_bit;
    if (temp == nullptr)
        return hipcub::DeviceRadixSort::SortPairs(nullptr, *temp_bytes, cell_id, sorted_cell, iota,
                                                  sorted_atoms, n, 0, end_bit, st);
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(temp, *temp_bytes, cell_id, sorted_cell, iota,
                                                      sorted_atoms, n, 0, end_bit, st);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(cell_start, 0, sizeof(int32_t) * n_cells, st);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(cell_end, 0, sizeof(int32_t) * n_cells, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cell_ranges, dim3((n + 255) / 256), dim3(256), 0, st, n, sorted_cell,
                       cell_start, cell_end);
    return hipGetLastError();
}

hipError_t launch_nbr_count(hipStream_t st, const NbrArgs& a, Counts* counts) {
    hipLaunchKernelGGL(k_nbr_count, dim3(a.n), dim3(64 * kNbrWaves), 0, st, a, counts);
    return hipGetLastError();
}

hipError_t launch_nbr_fill(hipStream_t st, const NbrArgs& a, const Counts* counts,
                           const int64_t* site_off, Site* sites) {
    hipLaunchKernelGGL(k_nbr_fill, dim3(a.n), dim3(64 * kNbrWaves), 0, st, a, counts, site_off, sites);
    return hipGetLastError();
}

hipError_t launch_rev_map(hipStream_t st, int n, const Counts* counts, const int64_t* site_off,
                          const Site* sites, const int64_t* hash_off, const int32_t* hash_cap,
                          int32_t* table, size_t table_len, int32_t* rev, int* err) {
    hipError_t e = hipMemsetAsync(table, 0xFF, sizeof(int32_t) * table_len, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hash_build, dim3(n), dim3(256), 0, st, n, counts, site_off, sites, hash_off,
                       hash_cap, table);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rev_map, dim3(n), dim3(256), 0, st, n, counts, site_off, sites, hash_off,
                       hash_cap, table, rev, err);
    return hipGetLastError();
}

}  // namespace lmbd
