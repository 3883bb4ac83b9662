// Deterministic per-destination gathers.
//
// Every contribution that one atom's local problem makes to another atom (a
// force on a neighbour, the adjoint of a neighbour's central polarisability)
// is written into a per-(central atom, site) slot.  Atom a then collects the
// slots that refer to it: for each site s of its own list (base j, shift t) the
// matching slot is rev[a][s] in the list of j (site (a, -t)), because neighbour
// membership is symmetric.  The order of summation is fixed by a's list, so
// results are bitwise reproducible and independent of the other structures in
// a batch.
#include "lmbd_internal.h"

namespace lmbd {

// abar_cen[a][w] = sum_{s in K(a)} ca[slot(base s, rev)][w]
__global__ void __launch_bounds__(256) k_gather_central(int n, int nw, const Counts* __restrict__ counts,
                                                        const int64_t* __restrict__ site_off,
                                                        const Site* __restrict__ sites,
                                                        const int32_t* __restrict__ rev,
                                                        const double* __restrict__ ca,
                                                        double* __restrict__ abar_cen) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nw) return;
    const int a = t / nw, w = t % nw;
    const int64_t off = site_off[a];
    const int nK = counts[a].nK;
    double s = 0.0;
    for (int e = 0; e < nK; ++e) {
        const int j = sites[off + e].base;
        s += ca[(site_off[j] + rev[off + e]) * nw + w];
    }
    abar_cen[(size_t)a * nw + w] = s;
}

// F[a] = sum_{s in list(a)} sum_slices cf[slice][slot(base s, rev)]; one wavefront per atom,
// lanes take sites round robin and a fixed xor tree combines the lanes.
__global__ void __launch_bounds__(256) k_gather_forces(int n, int nslices, int64_t slice_stride,
                                                       const Counts* __restrict__ counts,
                                                       const int64_t* __restrict__ site_off,
                                                       const Site* __restrict__ sites,
                                                       const int32_t* __restrict__ rev,
                                                       const double* __restrict__ cf,
                                                       double* __restrict__ forces) {
    const int lane = threadIdx.x & 63;
    const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (a >= n) return;
    const int64_t off = site_off[a];
    const int nall = counts[a].n_all;
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    for (int e = lane; e < nall; e += 64) {
        const int j = sites[off + e].base;
        const int64_t slot = site_off[j] + rev[off + e];
        for (int sl = 0; sl < nslices; ++sl) {
            const double* c = cf + sl * slice_stride + slot * 3;
            f0 += c[0];
            f1 += c[1];
            f2 += c[2];
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        f0 += __shfl_xor(f0, o);
        f1 += __shfl_xor(f1, o);
        f2 += __shfl_xor(f2, o);
    }
    if (lane == 0) {
        forces[3 * a + 0] = f0;
        forces[3 * a + 1] = f1;
        forces[3 * a + 2] = f2;
    }
}

__global__ void k_slice_sum(int64_t len, int nslices, int64_t slice_stride, double* __restrict__ cf);

// dv[a] = (sum_{s in list(a)} sum_w cnu[slot(base s, rev)][w]) / nu_a; one wavefront per
// atom, lanes over sites, a fixed xor tree over the lanes
__global__ void __launch_bounds__(256) k_gather_nu(int n, int nw, const Counts* __restrict__ counts,
                                                   const int64_t* __restrict__ site_off,
                                                   const Site* __restrict__ sites,
                                                   const int32_t* __restrict__ rev,
                                                   const double* __restrict__ cnu,
                                                   const double* __restrict__ nu, double* __restrict__ dv) {
    const int lane = threadIdx.x & 63;
    const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (a >= n) return;
    const int64_t off = site_off[a];
    const int nall = counts[a].n_all;
    double s = 0.0;
    for (int e = lane; e < nall; e += 64) {
        const int j = sites[off + e].base;
        const double* c = cnu + (site_off[j] + rev[off + e]) * nw;
        for (int w = 0; w < nw; ++w) s += c[w];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) dv[a] = s / nu[a];
}

hipError_t launch_gather_nu(hipStream_t st, int n, int nw, const Counts* counts, const int64_t* site_off,
                            const Site* sites, const int32_t* rev, const double* cnu, const double* nu,
                            double* dv) {
    hipLaunchKernelGGL(k_gather_nu, dim3((n + 3) / 4), dim3(256), 0, st, n, nw, counts, site_off, sites, rev,
                       cnu, nu, dv);
    return hipGetLastError();
}

// F[a] = sum of the slots of a's own frame whose site is a or one of its images; one
// wavefront per atom, a fixed xor tree over the lanes
__global__ void __launch_bounds__(256) k_gather_self(int n, const Counts* __restrict__ counts,
                                                     const int64_t* __restrict__ site_off,
                                                     const Site* __restrict__ sites, const double* __restrict__ cf,
                                                     double* __restrict__ forces) {
    const int lane = threadIdx.x & 63;
    const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (a >= n) return;
    const int64_t off = site_off[a];
    const int nall = counts[a].n_all;
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    for (int e = lane; e < nall; e += 64) {
        if (sites[off + e].base != a) continue;
        const double* c = cf + (off + e) * 3;
        f0 += c[0];
        f1 += c[1];
        f2 += c[2];
    }
    for (int o = 32; o > 0; o >>= 1) {
        f0 += __shfl_xor(f0, o);
        f1 += __shfl_xor(f1, o);
        f2 += __shfl_xor(f2, o);
    }
    if (lane == 0) {
        forces[3 * a + 0] = f0;
        forces[3 * a + 1] = f1;
        forces[3 * a + 2] = f2;
    }
}

hipError_t launch_gather_self(hipStream_t st, int n, int nslices, int64_t slice_stride, const Counts* counts,
                              const int64_t* site_off, const Site* sites, double* cf, double* forces) {
    hipLaunchKernelGGL(k_slice_sum, dim3((unsigned)((slice_stride + 255) / 256)), dim3(256), 0, st, slice_stride,
                       nslices, slice_stride, cf);
    hipLaunchKernelGGL(k_gather_self, dim3((n + 3) / 4), dim3(256), 0, st, n, counts, site_off, sites, cf, forces);
    return hipGetLastError();
}

// cf[0][x] = sum over slices sl = 0 .. nslices-1 of cf[sl][x] (in slice order), so
// that the force gather reads one slice
__global__ void __launch_bounds__(256) k_slice_sum(int64_t len, int nslices, int64_t slice_stride,
                                                   double* __restrict__ cf) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= len) return;
    double s = cf[x];
    for (int sl = 1; sl < nslices; ++sl) s += cf[sl * slice_stride + x];
    cf[x] = s;
}

// central static SCS polarisability alpha~_I,k(0): row 0, frequency 0 of each local solve
__global__ void k_central_static(int n, int nw, const double* __restrict__ alpha_loc,
                                 const int64_t* __restrict__ aloc_off, double* __restrict__ out) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < n) out[a] = alpha_loc[aloc_off[a]];
}

hipError_t launch_gather_central(hipStream_t st, int n, int nw, const Counts* counts,
                                 const int64_t* site_off, const Site* sites, const int32_t* rev,
                                 const double* ca, double* abar_cen) {
    hipLaunchKernelGGL(k_gather_central, dim3((n * nw + 255) / 256), dim3(256), 0, st, n, nw, counts,
                       site_off, sites, rev, ca, abar_cen);
    return hipGetLastError();
}

hipError_t launch_gather_forces(hipStream_t st, int n, int nslices, int64_t slice_stride,
                                const Counts* counts, const int64_t* site_off, const Site* sites,
                                const int32_t* rev, double* cf, double* forces) {
    // slices first summed in place into slice 0 (coalesced), then one gathered read per site
    hipLaunchKernelGGL(k_slice_sum, dim3((unsigned)((slice_stride + 255) / 256)), dim3(256), 0, st, slice_stride,
                       nslices, slice_stride, cf);
    hipLaunchKernelGGL(k_gather_forces, dim3((n + 3) / 4), dim3(256), 0, st, n, 1, slice_stride,
                       counts, site_off, sites, rev, cf, forces);
    return hipGetLastError();
}

__global__ void k_fill(int n, double v, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

hipError_t launch_fill(hipStream_t st, int n, double v, double* out) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((n + 255) / 256), dim3(256), 0, st, n, v, out);
    return hipGetLastError();
}

hipError_t launch_central_static(hipStream_t st, int n, int nw, const double* alpha_loc,
                                 const int64_t* aloc_off, double* out) {
    hipLaunchKernelGGL(k_central_static, dim3((n + 255) / 256), dim3(256), 0, st, n, nw, alpha_loc,
                       aloc_off, out);
    return hipGetLastError();
}

}  // namespace lmbd
