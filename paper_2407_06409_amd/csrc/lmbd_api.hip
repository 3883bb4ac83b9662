// Host driver of the lMBD library: validation, batch layout, memory plan and
// the launch sequence of the hot path on one HIP stream.
//
//   prep -> cell sort -> neighbour counts  (one host read-back: counts)
//   -> neighbour lists, reverse-slot map
//   -> local SCS per (atom, frequency)                   [all central values ready]
//   -> local MBD energy per atom (+ its adjoint)
//   -> gather central-polarisability adjoints -> SCS adjoint per (atom, frequency)
//   -> gather forces -> outputs
//
// The device-wide dependency between the SCS stage and the MBD stage is the
// single-GPU form of the exchange of central polarisabilities between the two
// stages of the paper's flowchart (Sec. III.A).
#include "lmbd.h"
#include "lmbd_host.h"
#include "lmbd_internal.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

using namespace lmbd;

namespace {

struct DBuf {
    void* p = nullptr;
    size_t cap = 0;
    bool owned = false;  // false: a slice of a caller-provided workspace
};

struct Plan {
    int64_t n_atoms = 0;
    int64_t total_sites = 0;
    int64_t table_len = 0;
    int64_t fac_len = 0, x_len = 0, aloc_len = 0, work_len = 0, coef_len = 0;
    int n1max = 0, nkmax = 0, nallmax = 0, n2max = 0;
    int nkmax_lds = 0;            // largest nK among the atoms whose MBD site arrays sit in LDS
    std::vector<int64_t> site_off, hash_off, fac_off, x_off, aloc_off, work_off, pl_off, coef_off;
    int64_t pl_len = 0;
    std::vector<int32_t> hash_cap, fac_ld;
    std::vector<int32_t> order;   // dispatch order of the per-atom workgroups: largest neighbourhoods first
};

}  // namespace

struct lmbd_context {
    int device = 0;
    size_t budget = 0;
    std::string err;
    DBuf in_pos, in_sp, in_nu, in_w, atom_struct, sinfo, sp_table, omegas;
    DBuf pos_b, abar, sigma, Rv, a0v, r0v, cell_id, wrap, iota, sorted_cell, sorted_atoms;
    DBuf cell_start, cell_end, sort_temp, counts, flags, wcounts;
    DBuf site_off, sites, hash_off, hash_cap, table, rev;
    DBuf fac_off, fac_ld, x_off, aloc_off, work_off;
    DBuf fac, xsol, alpha_loc, abar_loc, abar_cen, work, ca, cf;
    DBuf pl_i, pl_q, pl_off, pl_seg, coef, coef_off, dvec, resid, lam;
    DBuf e_out, f_out, a_out, dv_out, sp_out, order;
    DBuf tabs;   // one buffer holding the per-atom plan tables (pl_off .. order are views into it)
    // caller-provided workspace: every buffer of a call is carved from it in a
    // fixed order (nothing is allocated while it is set)
    char* arena = nullptr;
    size_t arena_size = 0, arena_used = 0;
    // pinned host staging of the small host <-> device copies of a call (plan
    // tables, counts, flags), allocated once with the context; a call whose
    // copies do not fit uses pageable memory instead
    char* pin = nullptr;
    size_t pin_cap = 0, pin_used = 0;
    bool pin_pending = false;       // copies from the staging area may still be queued
    int lds_limit = 0;              // LDS bytes per workgroup of the device
    bool profiling = false;
    int mbd_product = LMBD_MBD_AUTO;
    hipEvent_t ev[2 * LMBD_N_STAGES] = {};
    bool ev_used[LMBD_N_STAGES] = {};
    double stage_ms[LMBD_N_STAGES] = {};
    char* scratch = nullptr;   // device address of this device's static scratch array (set at creation)
};

// ---------------------------------------------------------------------------
// Static scratch for lmbd_compute_batch_static: one file-scope device array per
// GPU, held until the process ends.  Host code never passes the array's name to
// a kernel: the device address of each GPU's copy is taken once per device with
// hipGetSymbolAddress (the device current) and kept in g_scratch_ptr.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;                   // guards g_scratch_ptr
char* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_use[kMaxDevices];     // one call at a time per device uses the array
}  // namespace

static __device__ __align__(256) char scratch[kStaticScratchBytes];

#define ALL_BUFFERS(c)                                                                                     \
    &c->in_pos, &c->in_sp, &c->in_nu, &c->in_w, &c->atom_struct, &c->sinfo, &c->sp_table, &c->omegas, &c->pos_b,  \
        &c->abar, &c->sigma, &c->Rv, &c->a0v, &c->r0v, &c->cell_id, &c->wrap, &c->iota, &c->sorted_cell,           \
        &c->sorted_atoms, &c->cell_start, &c->cell_end, &c->sort_temp, &c->counts, &c->flags, &c->site_off,        \
        &c->sites, &c->hash_off, &c->hash_cap, &c->table, &c->rev, &c->fac_off, &c->fac_ld, &c->x_off,             \
        &c->aloc_off, &c->work_off, &c->fac, &c->xsol, &c->alpha_loc, &c->abar_loc, &c->abar_cen, &c->work,        \
        &c->ca, &c->cf, &c->e_out, &c->f_out, &c->a_out, &c->dv_out, &c->sp_out, &c->pl_i, &c->pl_q, &c->pl_off, &c->pl_seg, &c->coef, &c->coef_off, &c->dvec, &c->resid, &c->lam, \
        &c->order, &c->tabs, &c->wcounts

namespace {

constexpr size_t kAlign = 256;

size_t aligned(size_t bytes) {
    if (bytes == 0) bytes = 8;
    return (bytes + kAlign - 1) / kAlign * kAlign;
}

void release(DBuf& b) {
    if (b.p && b.owned) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    b.owned = false;
}

// Make b hold at least `bytes`: a slice of the context's workspace when one is
// set, else an owned allocation that grows and is cached between calls.
hipError_t ensure(lmbd_context* ctx, DBuf& b, size_t bytes) {
    if (ctx->arena) {
        const size_t need = aligned(bytes);
        if (ctx->arena_used + need > ctx->arena_size) return hipErrorOutOfMemory;
        release(b);
        b.p = ctx->arena + ctx->arena_used;
        b.cap = need;
        ctx->arena_used += need;
        return hipSuccess;
    }
    if (bytes == 0) bytes = 8;
    if (b.owned && bytes <= b.cap) return hipSuccess;
    release(b);
    const size_t nb = bytes + bytes / 8 + 256;
    hipError_t e = hipMalloc(&b.p, nb);
    if (e == hipSuccess) {
        b.cap = nb;
        b.owned = true;
    } else {
        b.p = nullptr;
    }
    return e;
}

template <typename T>
T* as(DBuf& b) {
    return static_cast<T*>(b.p);
}

lmbd_status fail(lmbd_context* ctx, lmbd_status s, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(ctx, e_ == hipErrorOutOfMemory ? LMBD_E_OOM : LMBD_E_DEVICE,    \
                        std::string(#expr) + ": " + hipGetErrorString(e_));             \
    } while (0)

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// number of frequencies at which the local SCS systems are solved
int scs_freq_count(const lmbd_params* p) { return p->scs_freq == LMBD_SCS_LORENTZ ? 2 : p->n_freq + 1; }

lmbd_status check_params(lmbd_context* ctx, const lmbd_params* p) {
    if (!p) return fail(ctx, LMBD_E_INVALID_ARG, "params is NULL");
    if (!finite_pos(p->beta) || !finite_pos(p->damp_d) || !finite_pos(p->r_buf) || !finite_pos(p->r_inner))
        return fail(ctx, LMBD_E_INVALID_ARG, "beta, damp_d, r_buf and r_inner must be positive");
    if (p->n_max < 2 || p->n_max > kMaxNmax) return fail(ctx, LMBD_E_INVALID_ARG, "n_max out of range [2, 12]");
    if (p->n_freq < 1 || p->n_freq > kMaxFreq - 1)
        return fail(ctx, LMBD_E_INVALID_ARG, "n_freq out of range [1, 32]");
    if (!p->omega || !p->weight) return fail(ctx, LMBD_E_INVALID_ARG, "omega/weight is NULL");
    for (int i = 0; i < p->n_freq; ++i)
        if (!std::isfinite(p->omega[i]) || p->omega[i] < 0.0 || !std::isfinite(p->weight[i]))
            return fail(ctx, LMBD_E_INVALID_ARG, "non-finite or negative quadrature node");
    if (p->c_n)
        for (int i = 0; i <= p->n_max; ++i)
            if (!std::isfinite(p->c_n[i])) return fail(ctx, LMBD_E_INVALID_ARG, "non-finite c_n");
    if (p->precision != LMBD_FP64 && p->precision != LMBD_MIXED)
        return fail(ctx, LMBD_E_INVALID_ARG, "unknown precision");
    if (p->scs_freq != LMBD_SCS_EXACT && p->scs_freq != LMBD_SCS_LORENTZ)
        return fail(ctx, LMBD_E_INVALID_ARG, "unknown SCS frequency treatment");
    if (p->scs_freq == LMBD_SCS_LORENTZ && !finite_pos(p->omega_ref))
        return fail(ctx, LMBD_E_INVALID_ARG, "omega_ref must be positive");
    if (p->force_model != LMBD_FORCES_EXACT && p->force_model != LMBD_FORCES_PAPER)
        return fail(ctx, LMBD_E_INVALID_ARG, "unknown force model");
    if (p->cn_mode != LMBD_CN_SERIES && p->cn_mode != LMBD_CN_FIT)
        return fail(ctx, LMBD_E_INVALID_ARG, "unknown c_n mode");
    if (p->cn_mode == LMBD_CN_FIT && p->c_n) return fail(ctx, LMBD_E_INVALID_ARG, "fitted c_n: c_n must be NULL");
    if (p->lanczos_steps != 0 && (p->lanczos_steps < 2 || p->lanczos_steps > kMaxLanczos))
        return fail(ctx, LMBD_E_INVALID_ARG, "lanczos_steps out of range [2, 64] (0 = 20)");
    return LMBD_OK;
}

lmbd_status check_struct(lmbd_context* ctx, const lmbd_params* p, const lmbd_structure& s) {
    if (s.n_atoms < 1 || s.n_atoms > INT32_MAX / 4) return fail(ctx, LMBD_E_INVALID_ARG, "bad n_atoms");
    if (!s.pos || !s.species || !s.v_ratio) return fail(ctx, LMBD_E_INVALID_ARG, "NULL input array");
    if (!finite_pos(s.r_scs) || !finite_pos(s.r_nbr) || !finite_pos(s.r_mbd1) || !finite_pos(s.r_mbd2))
        return fail(ctx, LMBD_E_INVALID_ARG, "cutoffs must be positive");
    if (!(p->r_buf < s.r_scs) || !(p->r_buf < s.r_mbd1) || !(p->r_buf < s.r_mbd2))
        return fail(ctx, LMBD_E_INVALID_ARG, "r_buf must be smaller than every cutoff");
    // Sec. III.A: the central atom's radius is the larger one, and K = B(r_nbr) must hold
    // every pair that f_LR couples (else a site leaving K would cut a coupled pair)
    if (s.r_mbd1 < s.r_mbd2) return fail(ctx, LMBD_E_INVALID_ARG, "r_mbd1 must not be smaller than r_mbd2");
    if (s.r_nbr < s.r_mbd1) return fail(ctx, LMBD_E_INVALID_ARG, "r_nbr must not be smaller than r_mbd1");
    {
        const double b1 = s.r_2b1 != 0.0 ? s.r_2b1 : s.r_mbd1, b2 = s.r_2b2 != 0.0 ? s.r_2b2 : s.r_mbd2;
        if (!finite_pos(b1) || !finite_pos(b2) || !(p->r_buf < b2) || b1 < b2 || s.r_nbr < b1)
            return fail(ctx, LMBD_E_INVALID_ARG, "two-body radii need r_nbr >= r_2b1 >= r_2b2 > r_buf");
    }
    const int npbc = (s.pbc[0] != 0) + (s.pbc[1] != 0) + (s.pbc[2] != 0);
    if (npbc > 0) {
        if (!s.cell) return fail(ctx, LMBD_E_INVALID_ARG, "periodic structure without a cell");
        for (int i = 0; i < 9; ++i)
            if (!std::isfinite(s.cell[i])) return fail(ctx, LMBD_E_INVALID_ARG, "non-finite cell");
    }
    return LMBD_OK;
}

void inv3(const double* m, double* o, double& det) {
    det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
          m[2] * (m[3] * m[7] - m[4] * m[6]);
    const double id = 1.0 / det;
    o[0] = (m[4] * m[8] - m[5] * m[7]) * id;
    o[1] = (m[2] * m[7] - m[1] * m[8]) * id;
    o[2] = (m[1] * m[5] - m[2] * m[4]) * id;
    o[3] = (m[5] * m[6] - m[3] * m[8]) * id;
    o[4] = (m[0] * m[8] - m[2] * m[6]) * id;
    o[5] = (m[2] * m[3] - m[0] * m[5]) * id;
    o[6] = (m[3] * m[7] - m[4] * m[6]) * id;
    o[7] = (m[1] * m[6] - m[0] * m[7]) * id;
    o[8] = (m[0] * m[4] - m[1] * m[3]) * id;
}

// Cell-list geometry of one structure (positions: host, Angstrom).
lmbd_status make_struct_info(lmbd_context* ctx, const lmbd_structure& s, const double* pos_host,
                             int atom_offset, int cell_offset, StructInfo& si) {
    std::memset(&si, 0, sizeof(si));
    si.r_scs = s.r_scs / kBohr;
    si.r_nbr = s.r_nbr / kBohr;
    si.r_mbd1 = s.r_mbd1 / kBohr;
    si.r_mbd2 = s.r_mbd2 / kBohr;
    si.r_2b1 = (s.r_2b1 != 0.0 ? s.r_2b1 : s.r_mbd1) / kBohr;
    si.r_2b2 = (s.r_2b2 != 0.0 ? s.r_2b2 : s.r_mbd2) / kBohr;
    si.two_body = (si.r_2b1 != si.r_mbd1 || si.r_2b2 != si.r_mbd2) ? 1 : 0;
    si.r_big = std::max(2.0 * si.r_scs, si.r_nbr);
    si.atom_offset = atom_offset;
    si.cell_offset = cell_offset;
    si.n_atoms = (int)s.n_atoms;
    const int n = (int)s.n_atoms;
    if (s.pbc[0] || s.pbc[1] || s.pbc[2]) {
        si.periodic = 1;
        for (int d = 0; d < 3; ++d) si.pbc[d] = s.pbc[d] != 0;
        for (int i = 0; i < 9; ++i) si.cell[i] = s.cell[i] / kBohr;
        double det;
        inv3(si.cell, si.inv, det);
        if (!(std::fabs(det) > 1e-12)) return fail(ctx, LMBD_E_INVALID_ARG, "singular cell");
        const double vol = std::fabs(det);
        for (int d = 0; d < 3; ++d) {
            const double* a = si.cell + 3 * ((d + 1) % 3);
            const double* b = si.cell + 3 * ((d + 2) % 3);
            const double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2],
                         cz = a[0] * b[1] - a[1] * b[0];
            const double perp = vol / std::sqrt(cx * cx + cy * cy + cz * cz);   // spacing of the lattice planes
            if (si.pbc[d]) {
                int nc = (int)std::floor(2.0 * perp / si.r_big);
                nc = std::max(1, std::min(nc, 64));
                si.ncell[d] = nc;
                si.reach[d] = (int)std::ceil(si.r_big * nc / perp * (1.0 + 1e-9));
                if (si.reach[d] > 60) return fail(ctx, LMBD_E_UNSUPPORTED, "cutoff too large for the cell");
            } else {
                // no images along d: cells of at least r_big over the atoms' extent
                double lo = 1e300, hi = -1e300;
                for (int i = 0; i < n; ++i) {
                    const double x = pos_host[3 * i] / kBohr, y = pos_host[3 * i + 1] / kBohr,
                                 z = pos_host[3 * i + 2] / kBohr;
                    if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z))
                        return fail(ctx, LMBD_E_INVALID_ARG, "non-finite position");
                    const double f = x * si.inv[d] + y * si.inv[3 + d] + z * si.inv[6 + d];
                    lo = std::min(lo, f);
                    hi = std::max(hi, f);
                }
                si.flo[d] = lo;
                si.fext[d] = std::max(hi - lo, 1e-9);
                int nc = (int)std::floor(si.fext[d] * perp / si.r_big);
                si.ncell[d] = std::max(1, std::min(nc, 64));
                si.reach[d] = 1;
            }
        }
    } else {
        si.periodic = 0;
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) {
                const double x = pos_host[3 * i + d] / kBohr;
                if (!std::isfinite(x)) return fail(ctx, LMBD_E_INVALID_ARG, "non-finite position");
                lo[d] = std::min(lo[d], x);
                hi[d] = std::max(hi[d], x);
            }
        for (int d = 0; d < 3; ++d) {
            const double ext = std::max(hi[d] - lo[d], 1e-6);
            int nc = (int)std::floor(ext / si.r_big);
            nc = std::max(1, std::min(nc, 64));
            si.ncell[d] = nc;
            si.reach[d] = 1;
            si.origin[d] = lo[d];
            si.cell[4 * d] = ext;
        }
    }
    return LMBD_OK;
}

int64_t next_pow2(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Atoms whose MBD stage keeps its per-site arrays in the workspace (the sparse form with
// global site arrays): those of structures whose largest neighbourhood K exceeds the LDS
// forms, in sites or in LDS bytes (with room for the Lanczos state, so that the choice does
// not depend on the outputs requested).  Per atom also the structure's largest count of
// sites within r_mbd2 (the bound of the sparse rows).  struct_begin: first atom of each
// structure, then the total.
void mbd_global_sites(const lmbd_params* p, const std::vector<Counts>& cnt, const std::vector<int64_t>& struct_begin,
                      std::vector<char>& gs, std::vector<int32_t>& m2max) {
    const int lz = p->lanczos_steps ? p->lanczos_steps : 20;
    gs.assign(cnt.size(), 0);
    m2max.assign(cnt.size(), 0);
    for (size_t s = 0; s + 1 < struct_begin.size(); ++s) {
        int nk = 0, m2 = 0;
        for (int64_t k = struct_begin[s]; k < struct_begin[s + 1]; ++k) {
            nk = std::max(nk, cnt[k].nK);
            m2 = std::max(m2, cnt[k].n_m2);
        }
        const bool g = nk > kMaxNK || mbd_lds_bytes(nk, p->n_freq, p->n_max, lz, p->cn_mode == LMBD_CN_FIT) > kLdsBytes;
        for (int64_t k = struct_begin[s]; k < struct_begin[s + 1]; ++k) {
            gs[k] = g ? 1 : 0;
            m2max[k] = m2;
        }
    }
}

void build_plan(const std::vector<Counts>& cnt, const std::vector<char>& gs, const std::vector<int32_t>& m2max, int nw,
                int ncol, int n_max, bool forces, bool mixed, Plan& P) {
    const int64_t n = (int64_t)cnt.size();
    P.n_atoms = n;
    P.site_off.resize(n + 1);
    P.hash_off.resize(n + 1);
    P.fac_off.resize(n + 1);
    P.x_off.resize(n + 1);
    P.aloc_off.resize(n + 1);
    P.work_off.resize(n + 1);
    P.pl_off.resize(n + 1);
    P.coef_off.resize(n + 1);
    P.hash_cap.resize(n);
    P.fac_ld.resize(n);
    const int mmax = forces ? std::max(1, n_max - 1) : std::max(1, (n_max + 1) / 2);
    int64_t so = 0, ho = 0, fo = 0, xo = 0, ao = 0, wo = 0, po = 0, co = 0;
    P.n1max = P.nkmax = P.nallmax = P.n2max = P.nkmax_lds = 0;
    for (int64_t k = 0; k < n; ++k) {
        const Counts& c = cnt[k];
        P.site_off[k] = so;
        P.hash_off[k] = ho;
        P.fac_off[k] = fo;
        P.x_off[k] = xo;
        P.aloc_off[k] = ao;
        P.work_off[k] = wo;
        P.pl_off[k] = po;
        P.coef_off[k] = co;
        po += (int64_t)c.n1 * (c.n12 - c.n1) + (int64_t)c.n1 * (c.n1 - 1) / 2;
        if (mixed) co += (int64_t)nw * c.n1 * (c.n1 + 1);
        const int64_t N1 = 3 * (int64_t)c.n1, N3 = 3 * (int64_t)c.nK;
        P.hash_cap[k] = (int32_t)next_pow2(2 * (int64_t)c.n_all);
        P.fac_ld[k] = (int32_t)((N1 + 3) / 4 * 4);
        so += c.n_all;
        ho += P.hash_cap[k];
        fo += (int64_t)nw * (N1 + 3) * P.fac_ld[k];   // B~ and, appended, the three rows of d^T
        xo += (int64_t)nw * N1 * 3;
        ao += (int64_t)c.n1 * nw;
        auto al4 = [](int64_t x) { return (x + 3) / 4 * 4; };  // as the MBD kernel lays out its workspace
        if (gs[k])
            wo += mbd_global_layout(c.nK, ncol / 3, n_max, mmax, mbd_list_cap(c.nK, m2max[k]), mixed ? 4 : 8, forces)
                      .total;
        else
            wo += al4(N3 * al4(N3)) + al4((int64_t)mmax * N3 * ncol) + 2 * al4(ncol * al4(N3)) +
                  (forces ? 2 * N3 * al4((int64_t)n_max * ncol) : 0);
        if (!gs[k]) P.nkmax_lds = std::max(P.nkmax_lds, c.nK);
        P.n1max = std::max(P.n1max, c.n1);
        P.nkmax = std::max(P.nkmax, c.nK);
        P.nallmax = std::max(P.nallmax, c.n_all);
        P.n2max = std::max(P.n2max, c.n12 - c.n1);
    }
    P.site_off[n] = so;
    P.total_sites = so;
    P.table_len = ho;
    P.fac_len = fo;
    P.x_len = xo;
    P.aloc_len = ao;
    P.work_len = wo;
    P.pl_len = po;
    P.coef_len = co;
    // the work of an atom's workgroups grows with its neighbourhood: taking the
    // largest first leaves the shortest ones for the end of each launch
    P.order.resize(n);
    for (int64_t k = 0; k < n; ++k) P.order[k] = (int32_t)k;
    std::stable_sort(P.order.begin(), P.order.end(), [&](int32_t x, int32_t y) {
        if (cnt[x].n1 != cnt[y].n1) return cnt[x].n1 > cnt[y].n1;
        return cnt[x].nK > cnt[y].nK;
    });
}

// A slice of the pinned staging area (nullptr when it has no room left).
void* pin_take(lmbd_context* ctx, size_t bytes) {
    const size_t need = (bytes + 255) / 256 * 256;
    if (!ctx->pin || ctx->pin_used + need > ctx->pin_cap) return nullptr;
    void* p = ctx->pin + ctx->pin_used;
    ctx->pin_used += need;
    ctx->pin_pending = true;
    return p;
}

// Host array -> device, asynchronously from the pinned staging area when it has
// room (the host array may then be reused at once), else from pageable memory.
hipError_t copy_h2d(lmbd_context* ctx, void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    if (void* p = pin_take(ctx, bytes)) {
        std::memcpy(p, src, bytes);
        return hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, st);
    }
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
}

template <typename T>
lmbd_status upload(lmbd_context* ctx, DBuf& b, const std::vector<T>& v, hipStream_t st) {
    if (sizeof(T) * v.size() > b.cap) return fail(ctx, LMBD_E_DEVICE, "workspace layout mismatch");
    HIP_TRY(copy_h2d(ctx, b.p, v.data(), sizeof(T) * v.size(), st));
    return LMBD_OK;
}

// Device -> host array through the staging area when it has room; the stream
// is synchronised before returning either way.
hipError_t copy_d2h_sync(lmbd_context* ctx, void* dst, const void* src, size_t bytes, hipStream_t st) {
    void* p = pin_take(ctx, bytes);
    hipError_t e = hipMemcpyAsync(p ? p : dst, src, bytes, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess && p) std::memcpy(dst, p, bytes);
    return e;
}

// Sizes that fix the buffers needed before the neighbour counts are known.
struct PreDims {
    int64_t N = 0;
    int n_structs = 0, n_cells = 0, nw = 0, n_species = 0;
    size_t sort_temp = 0;
};

// Every workspace buffer of a call, in the order it is laid out.  `get(buf,
// bytes)` allocates (or, for a footprint estimate, only counts) one buffer.
template <class F>
hipError_t layout_pre(lmbd_context* c, const PreDims& d, F&& get) {
    const size_t N = (size_t)d.N, D = sizeof(double), I = sizeof(int32_t), nw = (size_t)d.nw;
    const std::pair<DBuf*, size_t> L[] = {
        {&c->in_pos, 3 * N * D}, {&c->in_sp, N * I}, {&c->in_nu, N * D}, {&c->in_w, N * D},
        {&c->atom_struct, N * I}, {&c->sinfo, (size_t)d.n_structs * sizeof(StructInfo)},
        {&c->omegas, nw * D}, {&c->sp_table, 3 * (size_t)std::max(d.n_species, 64) * D}, {&c->iota, N * I},
        {&c->pos_b, 3 * N * D}, {&c->abar, N * nw * D}, {&c->sigma, N * nw * D}, {&c->Rv, N * D},
        {&c->a0v, N * D}, {&c->r0v, N * D}, {&c->cell_id, N * I}, {&c->wrap, 3 * N * I},
        {&c->sorted_cell, N * I}, {&c->sorted_atoms, N * I}, {&c->cell_start, (size_t)d.n_cells * I},
        {&c->cell_end, (size_t)d.n_cells * I}, {&c->counts, N * sizeof(Counts)}, {&c->flags, 4 * sizeof(int)},
        {&c->wcounts, N * kNbrWaves * 4 * I},
        {&c->sort_temp, d.sort_temp}};
    for (const auto& e : L) {
        const hipError_t r = get(*e.first, e.second);
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

// The per-atom plan tables, in this order, as slices of one buffer (one upload):
// eight int64 tables, then three int32 tables, each on a 256-byte boundary.
// Returns the bytes of the whole; with `set`, points the table buffers into
// c->tabs (views: the memory belongs to c->tabs).
size_t table_views(lmbd_context* c, int64_t n, bool set) {
    DBuf* t64[] = {&c->pl_off, &c->site_off, &c->hash_off, &c->fac_off, &c->x_off, &c->aloc_off, &c->work_off,
                   &c->coef_off};
    DBuf* t32[] = {&c->hash_cap, &c->fac_ld, &c->order};
    const size_t b64 = ((size_t)n * sizeof(int64_t) + 255) / 256 * 256;
    const size_t b32 = ((size_t)n * sizeof(int32_t) + 255) / 256 * 256;
    size_t off = 0;
    for (DBuf* b : t64) {
        if (set) {
            release(*b);
            b->p = static_cast<char*>(c->tabs.p) + off;
            b->cap = b64;
        }
        off += b64;
    }
    for (DBuf* b : t32) {
        if (set) {
            release(*b);
            b->p = static_cast<char*>(c->tabs.p) + off;
            b->cap = b32;
        }
        off += b32;
    }
    return off;
}

template <class F>
hipError_t layout_post(lmbd_context* c, const Plan& P, int nw, int nq, bool forces, size_t wsz, F&& get) {
    const bool mixed = wsz == sizeof(float);
    const size_t N = (size_t)P.n_atoms, D = sizeof(double), I = sizeof(int32_t);
    const size_t TS = (size_t)P.total_sites;
    const std::pair<DBuf*, size_t> L[] = {
        {&c->tabs, table_views(c, P.n_atoms, false)}, {&c->sites, TS * sizeof(Site)}, {&c->table, (size_t)P.table_len * I},
        {&c->rev, TS * I}, {&c->fac, (size_t)P.fac_len * wsz}, {&c->xsol, (size_t)P.x_len * D},
        {&c->alpha_loc, (size_t)P.aloc_len * D}, {&c->abar_loc, (size_t)P.aloc_len * D},
        {&c->abar_cen, N * nw * D}, {&c->work, (size_t)P.work_len * wsz}, {&c->e_out, N * D},
        {&c->a_out, N * D}, {&c->pl_i, (size_t)P.pl_len * I}, {&c->pl_q, (size_t)P.pl_len * I},
        {&c->pl_seg, 3 * (TS + 2 * N) * I}, {&c->coef, (size_t)P.coef_len * sizeof(float)},
        {&c->sp_out, N * (size_t)nq * 2 * D}};
    for (const auto& e : L) {
        const hipError_t r = get(*e.first, e.second);
        if (r != hipSuccess) return r;
    }
    if (mixed) {
        const std::pair<DBuf*, size_t> M2[] = {{&c->dvec, (size_t)P.x_len * D}, {&c->resid, (size_t)P.x_len * D}};
        for (const auto& e : M2) {
            const hipError_t r = get(*e.first, e.second);
            if (r != hipSuccess) return r;
        }
    }
    if (forces) {
        const std::pair<DBuf*, size_t> F2[] = {
            {&c->ca, TS * nw * D}, {&c->cf, (size_t)(1 + nw) * TS * 3 * D}, {&c->f_out, 3 * N * D},
            {&c->lam, (size_t)P.x_len * D}, {&c->dv_out, N * D}};
        for (const auto& e : F2) {
            const hipError_t r = get(*e.first, e.second);
            if (r != hipSuccess) return r;
        }
    }
    return hipSuccess;
}

struct Measure {
    size_t total = 0;
    hipError_t operator()(DBuf&, size_t bytes) {
        total += aligned(bytes);
        return hipSuccess;
    }
};

}  // namespace

extern "C" {

int32_t lmbd_abi_version(void) { return LMBD_ABI_VERSION; }

const char* lmbd_status_string(lmbd_status s) {
    switch (s) {
        case LMBD_OK: return "ok";
        case LMBD_E_INVALID_ARG: return "invalid argument";
        case LMBD_E_OOM: return "out of device memory";
        case LMBD_E_OOM_ADMISSION: return "request exceeds the memory budget";
        case LMBD_E_DEVICE: return "HIP runtime error";
        case LMBD_E_SCS_BREAKDOWN: return "local SCS matrix is not positive definite";
        case LMBD_E_UNSUPPORTED: return "unsupported size or option";
        case LMBD_E_CANCELLED: return "request cancelled";
        case LMBD_E_POLARISATION: return "a spectrum bound of G~ reaches 1 (polarisation catastrophe)";
    }
    return "unknown status";
}

const char* lmbd_last_error(const lmbd_context* ctx) { return ctx ? ctx->err.c_str() : ""; }

lmbd_status lmbd_create(int32_t device, lmbd_context** out) {
    if (!out) return LMBD_E_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return LMBD_E_INVALID_ARG;
    lmbd_context* ctx = new lmbd_context();
    ctx->device = device;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) == hipSuccess) {
        (void)hipDeviceGetAttribute(&ctx->lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
        constexpr size_t kPinBytes = 4u << 20;   // the plan tables of ~30k atoms
        if (hipHostMalloc(reinterpret_cast<void**>(&ctx->pin), kPinBytes, hipHostMallocDefault) == hipSuccess)
            ctx->pin_cap = kPinBytes;
        else
            ctx->pin = nullptr;
    }
    if (device < kMaxDevices && hipSetDevice(device) == hipSuccess) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void* ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess && ptr)
                g_scratch_ptr[device] = static_cast<char*>(ptr);
        }
        ctx->scratch = g_scratch_ptr[device];
    }
    (void)hipSetDevice(prev);
    *out = ctx;
    return LMBD_OK;
}

void lmbd_destroy(lmbd_context* ctx) {
    if (!ctx) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (hipEvent_t& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    DBuf* all[] = {ALL_BUFFERS(ctx)};
    for (DBuf* b : all) release(*b);
    if (ctx->pin) (void)hipHostFree(ctx->pin);
    (void)hipSetDevice(prev);
    delete ctx;
}

static const char* kStageNames[LMBD_N_STAGES] = {"prep_sort_count", "nbr_fill_revmap", "scs_rhs",
                                                  "scs_assemble_factor_solve", "scs_refine", "mbd",
                                                  "gather_central",  "scs_lambda",      "scs_adjoint",
                                                  "gather_forces"};

const char* lmbd_stage_name(int32_t i) { return (i >= 0 && i < LMBD_N_STAGES) ? kStageNames[i] : nullptr; }

lmbd_status lmbd_set_profiling(lmbd_context* ctx, int32_t enable) {
    if (!ctx) return LMBD_E_INVALID_ARG;
    if (enable && !ctx->ev[0]) {
        HIP_TRY(hipSetDevice(ctx->device));
        for (hipEvent_t& e : ctx->ev) HIP_TRY(hipEventCreate(&e));
    }
    ctx->profiling = enable != 0;
    return LMBD_OK;
}

lmbd_status lmbd_set_mbd_product(lmbd_context* ctx, int32_t mode) {
    if (!ctx || mode < LMBD_MBD_AUTO || mode > LMBD_MBD_SPARSE) return LMBD_E_INVALID_ARG;
    ctx->mbd_product = mode;
    return LMBD_OK;
}

lmbd_status lmbd_stage_times(const lmbd_context* ctx, double* ms) {
    if (!ctx || !ms) return LMBD_E_INVALID_ARG;
    for (int i = 0; i < LMBD_N_STAGES; ++i) ms[i] = ctx->stage_ms[i];
    return LMBD_OK;
}

lmbd_status lmbd_set_memory_budget(lmbd_context* ctx, size_t bytes) {
    if (!ctx) return LMBD_E_INVALID_ARG;
    ctx->budget = bytes;
    return LMBD_OK;
}

}  // extern "C"

// Host-side neighbour counts for footprint estimates: the cell list of the
// device (same grid, same traversal) and the same pair vectors, evaluated with
// the same operations, so the counts equal the device's.
namespace {

void h_lattice_vec(const double* c, int t0, int t1, int t2, double out[3]) {
    out[0] = std::fma((double)t2, c[6], std::fma((double)t1, c[3], (double)t0 * c[0]));
    out[1] = std::fma((double)t2, c[7], std::fma((double)t1, c[4], (double)t0 * c[1]));
    out[2] = std::fma((double)t2, c[8], std::fma((double)t1, c[5], (double)t0 * c[2]));
}

void h_canonical_rel(const double* pos, const double* cell, int kc, int j, int t0, int t1, int t2, double v[3]) {
    const bool pos_dir = j > kc || (j == kc && (t0 > 0 || (t0 == 0 && (t1 > 0 || (t1 == 0 && t2 > 0)))));
    double T[3];
    if (pos_dir) {
        h_lattice_vec(cell, t0, t1, t2, T);
        for (int d = 0; d < 3; ++d) v[d] = (pos[3 * j + d] + T[d]) - pos[3 * kc + d];
    } else {
        h_lattice_vec(cell, -t0, -t1, -t2, T);
        for (int d = 0; d < 3; ++d) v[d] = -((pos[3 * kc + d] + T[d]) - pos[3 * j + d]);
    }
}

lmbd_status host_counts(lmbd_context* ctx, const lmbd_structure& s, std::vector<Counts>& out, int& n_cells) {
    StructInfo S;
    lmbd_status st = make_struct_info(ctx, s, s.pos, 0, 0, S);
    if (st != LMBD_OK) return st;
    const int n = (int)s.n_atoms;
    const int nc = S.ncell[0] * S.ncell[1] * S.ncell[2];
    n_cells = nc;
    std::vector<double> p(3 * (size_t)n);
    std::vector<int> cell(n), wrap(3 * (size_t)n);
    for (int g = 0; g < n; ++g) {
        for (int d = 0; d < 3; ++d) p[3 * g + d] = s.pos[3 * g + d] / kBohr;
        int c[3];
        for (int d = 0; d < 3; ++d) {
            if (S.periodic) {
                const double f = p[3 * g] * S.inv[d] + p[3 * g + 1] * S.inv[3 + d] + p[3 * g + 2] * S.inv[6 + d];
                int cc;
                if (S.pbc[d]) {
                    const double fl = std::floor(f);
                    wrap[3 * g + d] = (int)fl;
                    cc = (int)((f - fl) * S.ncell[d]);
                } else {
                    wrap[3 * g + d] = 0;
                    cc = (int)((f - S.flo[d]) / S.fext[d] * S.ncell[d]);
                }
                c[d] = std::min(std::max(cc, 0), S.ncell[d] - 1);
            } else {
                const double h = S.cell[4 * d] / S.ncell[d];
                c[d] = std::min(std::max((int)((p[3 * g + d] - S.origin[d]) / h), 0), S.ncell[d] - 1);
                wrap[3 * g + d] = 0;
            }
        }
        cell[g] = (c[0] * S.ncell[1] + c[1]) * S.ncell[2] + c[2];
    }
    std::vector<int> start(nc + 1, 0), order(n);
    for (int g = 0; g < n; ++g) start[cell[g] + 1]++;
    for (int c = 0; c < nc; ++c) start[c + 1] += start[c];
    {
        std::vector<int> fill(start.begin(), start.end() - 1);
        for (int g = 0; g < n; ++g) order[fill[cell[g]]++] = g;
    }
    const double r1 = S.r_scs * S.r_scs, rK = S.r_nbr * S.r_nbr, r2 = 4.0 * S.r_scs * S.r_scs,
                 rb = S.r_big * S.r_big, rM2 = S.r_mbd2 * S.r_mbd2;
    auto count_one = [&](int k) {
        Counts c{1, 1, 1, 1, 1};
        const int ck[3] = {cell[k] / (S.ncell[1] * S.ncell[2]), (cell[k] / S.ncell[2]) % S.ncell[1],
                           cell[k] % S.ncell[2]};
        for (int dx = -S.reach[0]; dx <= S.reach[0]; ++dx)
            for (int dy = -S.reach[1]; dy <= S.reach[1]; ++dy)
                for (int dz = -S.reach[2]; dz <= S.reach[2]; ++dz) {
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
                    const int gc = (cc[0] * S.ncell[1] + cc[1]) * S.ncell[2] + cc[2];
                    for (int i = start[gc]; i < start[gc + 1]; ++i) {
                        const int j = order[i];
                        const int t0 = sh[0] - wrap[3 * j] + wrap[3 * k];
                        const int t1 = sh[1] - wrap[3 * j + 1] + wrap[3 * k + 1];
                        const int t2 = sh[2] - wrap[3 * j + 2] + wrap[3 * k + 2];
                        if (j == k && t0 == 0 && t1 == 0 && t2 == 0) continue;
                        double v[3];
                        h_canonical_rel(p.data(), S.cell, k, j, t0, t1, t2, v);
                        const double d2 = std::fma(v[2], v[2], std::fma(v[1], v[1], v[0] * v[0]));
                        if (!(d2 < rb)) continue;
                        c.n_all++;
                        c.n1 += d2 < r1;
                        c.nK += d2 < rK;
                        c.n12 += d2 < r2;
                        c.n_m2 += d2 < rM2;
                    }
                }
        return c;
    };
    // atoms are independent: split them over host threads (each writes its own entries)
    const size_t base = out.size();
    out.resize(base + (size_t)n);
    const int nthreads = (int)std::max<unsigned>(1u, std::min<unsigned>(16u, std::thread::hardware_concurrency()));
    const int nt = n >= 512 ? nthreads : 1;
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&, t] {
            for (int k = t; k < n; k += nt) out[base + k] = count_one(k);
        });
    for (std::thread& th : pool) th.join();
    return LMBD_OK;
}

}  // namespace

namespace lmbd {

lmbd_status analyse_structure(const lmbd_params* params, const lmbd_structure& s, StructCounts& out) {
    lmbd_context* ctx = nullptr;
    lmbd_status st = check_struct(ctx, params, s);
    if (st != LMBD_OK) return st;
    for (int64_t i = 0; i < s.n_atoms; ++i) {
        if (!finite_pos(s.v_ratio[i]) || s.species[i] < 0) return LMBD_E_INVALID_ARG;
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(s.pos[3 * i + d])) return LMBD_E_INVALID_ARG;
    }
    out.cnt.clear();
    out.cnt.reserve((size_t)s.n_atoms);
    out.forces = s.forces != nullptr || s.dE_dv != nullptr;   // both need the adjoint passes
    return host_counts(ctx, s, out.cnt, out.n_cells);
}

lmbd_status layout_bytes(const lmbd_params* params, int n_species, const std::vector<const StructCounts*>& parts,
                         size_t* bytes) {
    std::vector<Counts> cnt;
    std::vector<int64_t> begin(1, 0);
    bool forces = false;
    int n_cells = 0;
    for (const StructCounts* p : parts) {
        cnt.insert(cnt.end(), p->cnt.begin(), p->cnt.end());
        begin.push_back((int64_t)cnt.size());
        n_cells += p->n_cells;
        forces = forces || p->forces;
    }
    if (cnt.empty() || cnt.size() > (size_t)(INT32_MAX / 8)) return LMBD_E_UNSUPPORTED;
    const int nw = scs_freq_count(params);
    PreDims pd;
    pd.N = (int64_t)cnt.size();
    pd.n_structs = (int)parts.size();
    pd.n_cells = n_cells;
    pd.nw = nw;
    pd.n_species = n_species;
    if (sort_cells(nullptr, (int)pd.N, n_cells, nullptr, nullptr, nullptr, nullptr, nullptr, &pd.sort_temp,
                   nullptr, nullptr) != hipSuccess)
        return LMBD_E_DEVICE;
    lmbd_context layout;  // only its buffer descriptors are named; nothing is allocated
    Measure m;
    (void)layout_pre(&layout, pd, m);
    Plan P;
    std::vector<char> gs;
    std::vector<int32_t> m2max;
    mbd_global_sites(params, cnt, begin, gs, m2max);
    build_plan(cnt, gs, m2max, nw, 3 * params->n_freq, params->n_max, forces, params->precision == LMBD_MIXED, P);
    (void)layout_post(&layout, P, nw, params->n_freq, forces,
                      params->precision == LMBD_MIXED ? sizeof(float) : sizeof(double), m);
    *bytes = m.total;
    return LMBD_OK;
}

// Gauss-Legendre nodes (ascending) and weights of order n on [-1, 1]: Newton's method on
// P_n from the asymptotic guess cos(pi (i + 3/4) / (n + 1/2)) for the i-th largest root,
// P_n by its three-term recurrence, P_n' = n (x P_n - P_{n-1}) / (x^2 - 1), and the
// weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, double* x, double* w) {
    auto eval = [n](double z, double& dp) {
        double p0 = 1.0, p1 = z;
        for (int j = 2; j <= n; ++j) {
            const double p2 = ((2 * j - 1) * z * p1 - (j - 1) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        return p1;
    };
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            const double dz = eval(z, dp) / dp;
            z -= dz;
            if (std::fabs(dz) <= 1e-16) break;
        }
        (void)eval(z, dp);
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

void set_workspace(lmbd_context* ctx, void* base, size_t bytes) {
    DBuf* all[] = {ALL_BUFFERS(ctx)};
    for (DBuf* b : all) release(*b);
    ctx->arena = static_cast<char*>(base);
    ctx->arena_size = base ? bytes : 0;
    ctx->arena_used = 0;
}

}  // namespace lmbd

extern "C" {

lmbd_status lmbd_estimate_footprint(const lmbd_params* params, int32_t n_structs, const lmbd_structure* structs,
                                    size_t* bytes) {
    if (!bytes || !structs || n_structs < 1) return LMBD_E_INVALID_ARG;
    lmbd_status st = check_params(nullptr, params);
    if (st != LMBD_OK) return st;
    std::vector<StructCounts> sc(n_structs);
    std::vector<const StructCounts*> parts;
    int max_sp = 0;
    for (int s = 0; s < n_structs; ++s) {
        if ((st = analyse_structure(params, structs[s], sc[s])) != LMBD_OK) return st;
        for (int64_t i = 0; i < structs[s].n_atoms; ++i) max_sp = std::max(max_sp, structs[s].species[i]);
        parts.push_back(&sc[s]);
    }
    return layout_bytes(params, std::max(64, max_sp + 1), parts, bytes);
}

lmbd_status lmbd_compute_batch(lmbd_context* ctx, const lmbd_params* params, int32_t n_species,
                               const lmbd_species* species_table, int32_t n_structs,
                               const lmbd_structure* structs, int32_t mem, void* hip_stream) {
    if (!ctx) return LMBD_E_INVALID_ARG;
    ctx->err.clear();
    lmbd_status st = check_params(ctx, params);
    if (st != LMBD_OK) return st;
    if (!species_table || n_species < 1) return fail(ctx, LMBD_E_INVALID_ARG, "empty species table");
    for (int i = 0; i < n_species; ++i)
        if (!finite_pos(species_table[i].alpha0) || !finite_pos(species_table[i].c6) ||
            !finite_pos(species_table[i].r0))
            return fail(ctx, LMBD_E_INVALID_ARG, "species data must be positive");
    if (!structs || n_structs < 1) return fail(ctx, LMBD_E_INVALID_ARG, "no structures");
    if (mem != LMBD_HOST && mem != LMBD_DEVICE) return fail(ctx, LMBD_E_INVALID_ARG, "bad mem");
    bool forces = false;   // the adjoint passes run (forces or volume-ratio derivatives requested)
    bool want_dv = false;
    bool want_spec = false;
    int64_t N64 = 0;
    for (int s = 0; s < n_structs; ++s) {
        st = check_struct(ctx, params, structs[s]);
        if (st != LMBD_OK) return st;
        forces = forces || structs[s].forces != nullptr || structs[s].dE_dv != nullptr;
        want_dv = want_dv || structs[s].dE_dv != nullptr;
        want_spec = want_spec || structs[s].spectrum != nullptr;
        if (structs[s].dE_dv && params->force_model == LMBD_FORCES_PAPER)
            return fail(ctx, LMBD_E_INVALID_ARG, "dE_dv is the exact derivative: not with the approximate forces");
        N64 += structs[s].n_atoms;
    }
    if (N64 > INT32_MAX / 8) return fail(ctx, LMBD_E_UNSUPPORTED, "too many atoms in one call");
    const int N = (int)N64;
    const int nq = params->n_freq, nw = scs_freq_count(params), ncol = 3 * nq, n_max = params->n_max;
    const bool lorentz = params->scs_freq == LMBD_SCS_LORENTZ;
    const bool mixed = params->precision == LMBD_MIXED;
    const size_t wsz = mixed ? sizeof(float) : sizeof(double);  // matrix and workspace element size
    const bool fit = params->cn_mode == LMBD_CN_FIT;
    const int lz_steps = (fit || want_spec) ? (params->lanczos_steps ? params->lanczos_steps : 20) : 0;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (ctx->pin_pending) {   // a call that ended early may have left copies from the staging area queued
        HIP_TRY(hipDeviceSynchronize());
        ctx->pin_pending = false;
    }
    ctx->pin_used = 0;
    for (int i = 0; i < LMBD_N_STAGES; ++i) {
        ctx->ev_used[i] = false;
        ctx->stage_ms[i] = 0.0;
    }
    auto mark = [&](int stage, int which) -> hipError_t {
        if (!ctx->profiling) return hipSuccess;
        if (which == 1) ctx->ev_used[stage] = true;
        return hipEventRecord(ctx->ev[2 * stage + which], stream);
    };
    const hipMemcpyKind h2d = mem == LMBD_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    const hipMemcpyKind d2o = mem == LMBD_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;

    // --- workspace of the stages before the memory plan
    int n_cells = 0;
    std::vector<StructInfo> sinfo(n_structs);
    std::vector<std::vector<double>> pos_host(n_structs);
    for (int s = 0, off = 0, coff = 0; s < n_structs; ++s) {
        const lmbd_structure& S = structs[s];
        const int n = (int)S.n_atoms;
        const double* ph = S.pos;
        if (mem == LMBD_DEVICE && !(S.pbc[0] && S.pbc[1] && S.pbc[2])) {   // extents of the non-periodic directions
            pos_host[s].resize(3 * (size_t)n);
            HIP_TRY(hipMemcpyAsync(pos_host[s].data(), S.pos, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            ph = pos_host[s].data();
        }
        if (mem == LMBD_HOST) {
            for (int i = 0; i < n; ++i) {
                if (S.species[i] < 0 || S.species[i] >= n_species)
                    return fail(ctx, LMBD_E_INVALID_ARG, "species index out of range");
                if (!finite_pos(S.v_ratio[i])) return fail(ctx, LMBD_E_INVALID_ARG, "non-positive volume ratio");
                for (int d = 0; d < 3; ++d)
                    if (!std::isfinite(S.pos[3 * i + d])) return fail(ctx, LMBD_E_INVALID_ARG, "non-finite position");
            }
        }
        st = make_struct_info(ctx, S, ph, off, coff, sinfo[s]);
        if (st != LMBD_OK) return st;
        off += n;
        coff += sinfo[s].ncell[0] * sinfo[s].ncell[1] * sinfo[s].ncell[2];
        n_cells = coff;
    }
    PreDims pd;
    pd.N = N;
    pd.n_structs = n_structs;
    pd.n_cells = n_cells;
    pd.nw = nw;
    pd.n_species = n_species;
    HIP_TRY(sort_cells(stream, N, n_cells, nullptr, nullptr, nullptr, nullptr, nullptr, &pd.sort_temp, nullptr,
                       nullptr));
    Measure pre_bytes;
    (void)layout_pre(ctx, pd, pre_bytes);
    if (ctx->budget && pre_bytes.total > ctx->budget)
        return fail(ctx, LMBD_E_OOM_ADMISSION, "footprint over the memory budget");
    if (ctx->arena && pre_bytes.total > ctx->arena_size)
        return fail(ctx, LMBD_E_OOM_ADMISSION, "footprint over the workspace size");
    ctx->arena_used = 0;
    HIP_TRY(layout_pre(ctx, pd, [&](DBuf& b, size_t n) { return ensure(ctx, b, n); }));
    std::vector<int32_t> atom_struct(N);
    for (int s = 0, off = 0; s < n_structs; ++s) {
        const lmbd_structure& S = structs[s];
        const int n = (int)S.n_atoms;
        HIP_TRY(hipMemcpyAsync(as<double>(ctx->in_pos) + 3 * (size_t)off, S.pos, sizeof(double) * 3 * n, h2d, stream));
        HIP_TRY(hipMemcpyAsync(as<int32_t>(ctx->in_sp) + off, S.species, sizeof(int32_t) * n, h2d, stream));
        HIP_TRY(hipMemcpyAsync(as<double>(ctx->in_nu) + off, S.v_ratio, sizeof(double) * n, h2d, stream));
        if (S.e_weight) {
            HIP_TRY(hipMemcpyAsync(as<double>(ctx->in_w) + off, S.e_weight, sizeof(double) * n, h2d, stream));
        } else {
            HIP_TRY(launch_fill(stream, n, 1.0, as<double>(ctx->in_w) + off));   // no weights: 1 per atom
        }
        for (int i = 0; i < n; ++i) atom_struct[off + i] = s;
        off += n;
    }
    std::vector<double> omegas(nw);   // SCS frequencies: 0, then omega_ref or every node
    omegas[0] = 0.0;
    if (lorentz)
        omegas[1] = params->omega_ref;
    else
        for (int q = 0; q < nq; ++q) omegas[q + 1] = params->omega[q];
    std::vector<double> tab(3 * (size_t)n_species);
    for (int i = 0; i < n_species; ++i) {
        tab[3 * i] = species_table[i].alpha0;
        tab[3 * i + 1] = species_table[i].c6;
        tab[3 * i + 2] = species_table[i].r0;
    }
    std::vector<int32_t> iota(N);
    for (int i = 0; i < N; ++i) iota[i] = i;
    if ((st = upload(ctx, ctx->atom_struct, atom_struct, stream)) != LMBD_OK) return st;
    if ((st = upload(ctx, ctx->sinfo, sinfo, stream)) != LMBD_OK) return st;
    if ((st = upload(ctx, ctx->omegas, omegas, stream)) != LMBD_OK) return st;
    if ((st = upload(ctx, ctx->sp_table, tab, stream)) != LMBD_OK) return st;
    if ((st = upload(ctx, ctx->iota, iota, stream)) != LMBD_OK) return st;

    // --- per-atom tables and cell list
    int flags_init[4] = {0, INT_MAX, 0, 0};
    HIP_TRY(copy_h2d(ctx, ctx->flags.p, flags_init, sizeof(flags_init), stream));
    int* err = as<int>(ctx->flags);
    int* err_atom = err + 1;
    HIP_TRY(mark(0, 0));
    HIP_TRY(launch_prep(stream, N, as<double>(ctx->in_pos), as<int32_t>(ctx->in_sp), as<double>(ctx->in_nu),
                        as<int32_t>(ctx->atom_struct), as<StructInfo>(ctx->sinfo), as<double>(ctx->sp_table),
                        n_species, as<double>(ctx->omegas), nw, as<double>(ctx->pos_b), as<double>(ctx->abar),
                        as<double>(ctx->sigma), as<double>(ctx->Rv), as<double>(ctx->a0v), as<double>(ctx->r0v),
                        as<int32_t>(ctx->cell_id), as<int32_t>(ctx->wrap), err));
    size_t temp_bytes = ctx->sort_temp.cap;
    HIP_TRY(sort_cells(stream, N, n_cells, as<int32_t>(ctx->cell_id), as<int32_t>(ctx->iota),
                       as<int32_t>(ctx->sorted_cell), as<int32_t>(ctx->sorted_atoms), ctx->sort_temp.p,
                       &temp_bytes, as<int32_t>(ctx->cell_start), as<int32_t>(ctx->cell_end)));
    NbrArgs na;
    na.n = N;
    na.pos_b = as<double>(ctx->pos_b);
    na.atom_struct = as<int32_t>(ctx->atom_struct);
    na.sinfo = as<StructInfo>(ctx->sinfo);
    na.cell_id = as<int32_t>(ctx->cell_id);
    na.wrap = as<int32_t>(ctx->wrap);
    na.cell_start = as<int32_t>(ctx->cell_start);
    na.cell_end = as<int32_t>(ctx->cell_end);
    na.sorted_atoms = as<int32_t>(ctx->sorted_atoms);
    na.wcounts = as<int32_t>(ctx->wcounts);
    HIP_TRY(launch_nbr_count(stream, na, as<Counts>(ctx->counts)));
    HIP_TRY(mark(0, 1));
    std::vector<Counts> cnt(N);
    int flags[4];
    {
        // counts and flags in one staged copy when the staging area has room
        Counts* pc = static_cast<Counts*>(pin_take(ctx, sizeof(Counts) * N));
        int* pf = static_cast<int*>(pin_take(ctx, sizeof(flags)));
        HIP_TRY(hipMemcpyAsync(pc ? (void*)pc : (void*)cnt.data(), ctx->counts.p, sizeof(Counts) * N,
                               hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipMemcpyAsync(pf ? (void*)pf : (void*)flags, ctx->flags.p, sizeof(flags), hipMemcpyDeviceToHost,
                               stream));
        HIP_TRY(hipStreamSynchronize(stream));
        if (pc) std::memcpy(cnt.data(), pc, sizeof(Counts) * N);
        if (pf) std::memcpy(flags, pf, sizeof(flags));
    }
    if (flags[0] & 1) return fail(ctx, LMBD_E_INVALID_ARG, "invalid species, volume ratio or position");

    // --- memory plan
    std::vector<int64_t> sbegin(n_structs + 1, 0);
    for (int s = 0; s < n_structs; ++s) sbegin[s + 1] = sbegin[s] + structs[s].n_atoms;
    std::vector<char> gsites;
    std::vector<int32_t> m2max;
    mbd_global_sites(params, cnt, sbegin, gsites, m2max);
    for (int s = 0; s < n_structs; ++s) sinfo[s].m2max = m2max[sbegin[s]];
    if ((st = upload(ctx, ctx->sinfo, sinfo, stream)) != LMBD_OK) return st;
    Plan P;
    build_plan(cnt, gsites, m2max, nw, ncol, n_max, forces, mixed, P);
    // MBD kernel form per structure, not per call, so that a structure's results do not
    // depend on what it shares a call with: dense-form atoms first, then sparse-form atoms
    // with the site arrays in LDS, then those with them in the workspace, each part still
    // largest first
    std::vector<int> form(n_structs);
    for (int s = 0; s < n_structs; ++s) {
        const bool sparse = params->force_model == LMBD_FORCES_EXACT &&   // the approximate forces use dense products
                            (ctx->mbd_product == LMBD_MBD_SPARSE ||
                             (ctx->mbd_product == LMBD_MBD_AUTO && structs[s].r_mbd2 <= kSparseMbdRatio * structs[s].r_nbr));
        form[s] = gsites[sbegin[s]] ? kMbdSparseGlobal : sparse ? kMbdSparse : kMbdDense;
        if (form[s] == kMbdSparseGlobal && (params->force_model != LMBD_FORCES_EXACT || ctx->mbd_product == LMBD_MBD_DENSE))
            return fail(ctx, LMBD_E_UNSUPPORTED, "neighbourhood too large for the dense MBD products (nK up to " +
                                                     std::to_string(kMaxNK) + "; larger ones need the sparse form)");
    }
    // launch groups: MBD form, then whether the structure has two-body radii of its own
    auto group = [&](int32_t k) { return 2 * form[atom_struct[k]] + sinfo[atom_struct[k]].two_body; };
    std::stable_sort(P.order.begin(), P.order.end(), [&](int32_t x, int32_t y) { return group(x) < group(y); });
    int n_group[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < N; ++k) n_group[group(k)]++;
    if (P.n1max > kMaxN1 || P.nkmax_lds > kMaxNK || P.nallmax > kMaxSites)
        return fail(ctx, LMBD_E_UNSUPPORTED,
                    "neighbourhood too large (n1 " + std::to_string(P.n1max) + ", nK " + std::to_string(P.nkmax) +
                        ", sites " + std::to_string(P.nallmax) + ")");
    int lds_limit = ctx->lds_limit;
    if (lds_limit <= 0) {
        HIP_TRY(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
        ctx->lds_limit = lds_limit;
    }
    if (scs_lds_bytes(P.n1max, P.n2max, mixed) > (size_t)lds_limit || mbd_lds_bytes(P.nkmax_lds, nq, n_max, lz_steps, fit) > (size_t)lds_limit ||
        scs_factor_lds_bytes(P.n1max, mixed) > (size_t)lds_limit || scs_assemble_lds_bytes(P.n1max, P.n2max) > (size_t)lds_limit ||
        pairlist_lds_bytes(P.n1max, P.n2max) > (size_t)lds_limit)
        return fail(ctx, LMBD_E_UNSUPPORTED, "neighbourhood needs more LDS than the device offers (" +
                                                 std::to_string(lds_limit) + " bytes)");
    Measure post_bytes;
    (void)layout_post(ctx, P, nw, nq, forces, wsz, post_bytes);
    if (ctx->budget && pre_bytes.total + post_bytes.total > ctx->budget)
        return fail(ctx, LMBD_E_OOM_ADMISSION,
                    "footprint " + std::to_string(pre_bytes.total + post_bytes.total) + " bytes over the memory budget");
    if (ctx->arena && ctx->arena_used + post_bytes.total > ctx->arena_size)
        return fail(ctx, LMBD_E_OOM_ADMISSION, "footprint over the workspace size");
    HIP_TRY(layout_post(ctx, P, nw, nq, forces, wsz, [&](DBuf& b, size_t n) { return ensure(ctx, b, n); }));
    {
        // all per-atom plan tables in one image, one copy
        const size_t tb = table_views(ctx, N, true);
        std::vector<char> img(tb);
        size_t off = 0;
        const size_t b64 = ((size_t)N * sizeof(int64_t) + 255) / 256 * 256;
        const size_t b32 = ((size_t)N * sizeof(int32_t) + 255) / 256 * 256;
        const std::vector<int64_t>* v64[] = {&P.pl_off, &P.site_off, &P.hash_off, &P.fac_off, &P.x_off, &P.aloc_off,
                                             &P.work_off, &P.coef_off};
        for (const std::vector<int64_t>* v : v64) {   // the first N entries (the last is the total)
            std::memcpy(img.data() + off, v->data(), sizeof(int64_t) * (size_t)N);
            off += b64;
        }
        const std::vector<int32_t>* v32[] = {&P.hash_cap, &P.fac_ld, &P.order};
        for (const std::vector<int32_t>* v : v32) {
            std::memcpy(img.data() + off, v->data(), sizeof(int32_t) * (size_t)N);
            off += b32;
        }
        if (tb > ctx->tabs.cap) return fail(ctx, LMBD_E_DEVICE, "workspace layout mismatch");
        HIP_TRY(copy_h2d(ctx, ctx->tabs.p, img.data(), tb, stream));
    }
    const int64_t TS = P.total_sites;

    // --- neighbour lists and the reverse-slot map
    HIP_TRY(mark(1, 0));
    HIP_TRY(launch_nbr_fill(stream, na, as<Counts>(ctx->counts), as<int64_t>(ctx->site_off), as<Site>(ctx->sites)));
    HIP_TRY(launch_rev_map(stream, N, as<Counts>(ctx->counts), as<int64_t>(ctx->site_off), as<Site>(ctx->sites),
                           as<int64_t>(ctx->hash_off), as<int32_t>(ctx->hash_cap), as<int32_t>(ctx->table),
                           (size_t)P.table_len, as<int32_t>(ctx->rev), err));

    // --- local SCS at omega = 0 and every node
    ScsArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.n = N;
    sa.nw = nw;
    sa.counts = as<Counts>(ctx->counts);
    sa.order = as<int32_t>(ctx->order);
    sa.site_off = as<int64_t>(ctx->site_off);
    sa.sites = as<Site>(ctx->sites);
    sa.abar = as<double>(ctx->abar);
    sa.sigma = as<double>(ctx->sigma);
    sa.Rv = as<double>(ctx->Rv);
    sa.atom_struct = as<int32_t>(ctx->atom_struct);
    sa.sinfo = as<StructInfo>(ctx->sinfo);
    sa.beta = params->beta;
    sa.damp_d = params->damp_d;
    sa.r_buf = params->r_buf / kBohr;
    sa.r_inner = params->r_inner / kBohr;
    sa.fac = ctx->fac.p;
    sa.n_refine = 1;
    sa.fac_off = as<int64_t>(ctx->fac_off);
    sa.fac_ld = as<int32_t>(ctx->fac_ld);
    sa.coef = mixed ? as<float>(ctx->coef) : nullptr;
    sa.coef_off = as<int64_t>(ctx->coef_off);
    sa.xsol = as<double>(ctx->xsol);
    sa.dvec = mixed ? as<double>(ctx->dvec) : nullptr;
    sa.resid = mixed ? as<double>(ctx->resid) : nullptr;
    sa.lam = forces ? as<double>(ctx->lam) : nullptr;
    sa.x_off = as<int64_t>(ctx->x_off);
    sa.alpha_loc = as<double>(ctx->alpha_loc);
    sa.aloc_off = as<int64_t>(ctx->aloc_off);
    sa.err = err;
    sa.err_atom = err_atom;
    sa.pl_i = as<int32_t>(ctx->pl_i);
    sa.pl_q = as<int32_t>(ctx->pl_q);
    sa.pl_off = as<int64_t>(ctx->pl_off);
    sa.pl_seg = as<int32_t>(ctx->pl_seg);
    HIP_TRY(launch_pairlist(stream, sa, P.n1max, P.n2max));
    HIP_TRY(mark(1, 1));
    HIP_TRY(mark(2, 0));
    HIP_TRY(launch_scs_rhs(stream, sa, P.n1max, P.n2max, mixed));
    HIP_TRY(mark(2, 1));
    HIP_TRY(mark(3, 0));
    HIP_TRY(launch_scs_factor(stream, sa, P.n1max, mixed));   // assembles B~, factorises it, solves (and refines)
    HIP_TRY(mark(3, 1));   // (stage 4, the refinement's former kernels, is not recorded)

    // --- local MBD energy (+ adjoint)
    MbdArgs ma;
    std::memset(&ma, 0, sizeof(ma));
    ma.n = N;
    ma.nw = nw;
    ma.nq = nq;
    ma.n_max = n_max;
    ma.ncol = ncol;
    ma.mmax = forces ? std::max(1, n_max - 1) : std::max(1, (n_max + 1) / 2);
    ma.counts = sa.counts;
    ma.order = sa.order;
    ma.site_off = sa.site_off;
    ma.sites = sa.sites;
    ma.alpha_loc = sa.alpha_loc;
    ma.aloc_off = sa.aloc_off;
    ma.a0v = as<double>(ctx->a0v);
    ma.r0v = as<double>(ctx->r0v);
    ma.atom_struct = sa.atom_struct;
    ma.sinfo = sa.sinfo;
    ma.beta = params->beta;
    ma.damp_d = params->damp_d;
    ma.r_buf = sa.r_buf;
    for (int i = 0; i <= n_max; ++i) ma.coef[i] = (i < 2) ? 0.0 : (params->c_n ? params->c_n[i] : -1.0 / i);
    for (int q = 0; q < nq; ++q) ma.wq[q] = params->weight[q] * kHartree / (2.0 * kPi);
    ma.lorentz = lorentz ? 1 : 0;
    ma.paper = params->force_model == LMBD_FORCES_PAPER ? 1 : 0;
    if (lorentz)
        for (int q = 0; q < nq; ++q) ma.rho[q] = (params->omega[q] / params->omega_ref) * (params->omega[q] / params->omega_ref);
    ma.fit = fit ? 1 : 0;
    ma.lz_steps = lz_steps;
    gauss_legendre(kFitNodes, ma.gl_x, ma.gl_w);
    ma.spectrum = want_spec ? as<double>(ctx->sp_out) : nullptr;
    ma.err = err;
    ma.err_atom = err_atom;
    ma.e_weight = as<double>(ctx->in_w);
    ma.e_atom = as<double>(ctx->e_out);
    ma.work = ctx->work.p;
    ma.work_off = as<int64_t>(ctx->work_off);
    ma.forces = forces ? 1 : 0;
    ma.abar_loc = as<double>(ctx->abar_loc);
    ma.ca = forces ? as<double>(ctx->ca) : nullptr;
    ma.cf0 = forces ? as<double>(ctx->cf) : nullptr;
    HIP_TRY(mark(5, 0));
    for (int gi = 0, first = 0; gi < 6; first += n_group[gi], ++gi) {   // the sparse forms pay once block
        if (n_group[gi] == 0) continue;                                      // rows couple to a small part of K
        MbdArgs mf = ma;
        mf.n = n_group[gi];
        mf.order = ma.order + first;
        HIP_TRY(launch_mbd(stream, mf, P.nkmax_lds, mixed, gi / 2, (gi & 1) != 0));
    }
    HIP_TRY(mark(5, 1));

    if (forces) {
        HIP_TRY(mark(6, 0));
        if (ma.paper)   // the central polarisabilities are held fixed
            HIP_TRY(launch_fill(stream, N * nw, 0.0, as<double>(ctx->abar_cen)));
        else
            HIP_TRY(launch_gather_central(stream, N, nw, sa.counts, sa.site_off, sa.sites, as<int32_t>(ctx->rev),
                                          as<double>(ctx->ca), as<double>(ctx->abar_cen)));
        HIP_TRY(mark(6, 1));
        sa.abar_loc = as<double>(ctx->abar_loc);
        sa.abar_cen = as<double>(ctx->abar_cen);
        sa.cf_slice = TS * 3;
        sa.cf = as<double>(ctx->cf) + sa.cf_slice;  // slices 1..nw
        HIP_TRY(mark(7, 0));
        HIP_TRY(launch_scs_lambda(stream, sa, P.n1max, mixed));
        HIP_TRY(mark(7, 1));
        HIP_TRY(mark(8, 0));
        HIP_TRY(launch_scs_adjoint(stream, sa, P.n1max, P.n2max, mixed));
        if (want_dv) {   // the central adjoints are gathered: their slots take the volume-ratio shares
            sa.cnu = as<double>(ctx->ca);
            HIP_TRY(launch_scs_nu(stream, sa, P.n1max, P.n2max));
            HIP_TRY(launch_gather_nu(stream, N, nw, sa.counts, sa.site_off, sa.sites, as<int32_t>(ctx->rev),
                                     sa.cnu, as<double>(ctx->in_nu), as<double>(ctx->dv_out)));
        }
        HIP_TRY(mark(8, 1));
        HIP_TRY(mark(9, 0));
        if (ma.paper)   // each atom's force from its own frame
            HIP_TRY(launch_gather_self(stream, N, 1 + nw, TS * 3, sa.counts, sa.site_off, sa.sites,
                                       as<double>(ctx->cf), as<double>(ctx->f_out)));
        else
            HIP_TRY(launch_gather_forces(stream, N, 1 + nw, TS * 3, sa.counts, sa.site_off, sa.sites,
                                         as<int32_t>(ctx->rev), as<double>(ctx->cf), as<double>(ctx->f_out)));
        HIP_TRY(mark(9, 1));
    }
    HIP_TRY(launch_central_static(stream, N, nw, sa.alpha_loc, sa.aloc_off, as<double>(ctx->a_out)));

    // --- outputs
    for (int s = 0, off = 0; s < n_structs; ++s) {
        const lmbd_structure& S = structs[s];
        const int n = (int)S.n_atoms;
        if (S.e_atom)
            HIP_TRY(hipMemcpyAsync(S.e_atom, as<double>(ctx->e_out) + off, sizeof(double) * n, d2o, stream));
        if (S.forces)
            HIP_TRY(hipMemcpyAsync(S.forces, as<double>(ctx->f_out) + 3 * (size_t)off, sizeof(double) * 3 * n, d2o,
                                   stream));
        if (S.alpha_scs0)
            HIP_TRY(hipMemcpyAsync(S.alpha_scs0, as<double>(ctx->a_out) + off, sizeof(double) * n, d2o, stream));
        if (S.dE_dv)
            HIP_TRY(hipMemcpyAsync(S.dE_dv, as<double>(ctx->dv_out) + off, sizeof(double) * n, d2o, stream));
        if (S.spectrum)
            HIP_TRY(hipMemcpyAsync(S.spectrum, as<double>(ctx->sp_out) + (size_t)off * nq * 2,
                                   sizeof(double) * n * nq * 2, d2o, stream));
        off += n;
    }
    HIP_TRY(copy_d2h_sync(ctx, flags, ctx->flags.p, sizeof(flags), stream));
    ctx->pin_pending = false;
    if (ctx->profiling)
        for (int i = 0; i < LMBD_N_STAGES; ++i)
            if (ctx->ev_used[i]) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[2 * i], ctx->ev[2 * i + 1]));
                ctx->stage_ms[i] = ms;
            }
    if (flags[0] & 2) return fail(ctx, LMBD_E_DEVICE, "reverse neighbour slot not found");
    if (flags[0] & 4)
        return fail(ctx, LMBD_E_SCS_BREAKDOWN,
                    "non-positive pivot in the local SCS matrix of atom " + std::to_string(flags[1]));
    if (flags[0] & 8)
        return fail(ctx, LMBD_E_SCS_BREAKDOWN,
                    "SCS polarisability not decreasing between 0 and omega_ref in the frame of atom " +
                        std::to_string(flags[1]));
    if (flags[0] & 64)
        return fail(ctx, LMBD_E_DEVICE, "a wavefront of the SCS factorisation of atom " + std::to_string(flags[1]) +
                                            " gave up waiting for its diagonal block");
    if (flags[0] & 32)
        return fail(ctx, LMBD_E_DEVICE, "coupled-site lists of atom " + std::to_string(flags[1]) + " outgrew their bound");
    if (flags[0] & 16)
        return fail(ctx, LMBD_E_POLARISATION,
                    "largest eigenvalue bound of G~ >= 1 in the frame of atom " + std::to_string(flags[1]));
    return LMBD_OK;
}

lmbd_status lmbd_compute_batch_static(lmbd_context* ctx, const lmbd_params* params, int32_t n_species,
                                      const lmbd_species* species_table, int32_t n_structs,
                                      const lmbd_structure* structs, int32_t mem, void* hip_stream) {
    if (!ctx) return LMBD_E_INVALID_ARG;
    if (!ctx->scratch || ctx->device >= kMaxDevices)
        return fail(ctx, LMBD_E_DEVICE, "the static scratch array of the device is not available");
    std::lock_guard<std::mutex> lk(g_scratch_use[ctx->device]);
    // A call context that owns nothing: every buffer is carved from the static
    // array, so neither the call nor its end allocates or frees device memory
    // (the caller's context keeps its own cached buffers untouched).  It borrows
    // the context's pinned staging area and stage-timer events.
    lmbd_context tmp;
    tmp.device = ctx->device;
    tmp.budget = ctx->budget;
    tmp.pin = ctx->pin;
    tmp.pin_cap = ctx->pin_cap;
    tmp.pin_pending = ctx->pin_pending;
    tmp.lds_limit = ctx->lds_limit;
    tmp.profiling = ctx->profiling;
    tmp.mbd_product = ctx->mbd_product;
    for (int i = 0; i < 2 * LMBD_N_STAGES; ++i) tmp.ev[i] = ctx->ev[i];
    tmp.arena = ctx->scratch;
    tmp.arena_size = kStaticScratchBytes;
    const lmbd_status st = lmbd_compute_batch(&tmp, params, n_species, species_table, n_structs, structs, mem,
                                              hip_stream);
    ctx->pin_pending = tmp.pin_pending;
    ctx->err = tmp.err;
    for (int i = 0; i < LMBD_N_STAGES; ++i) {
        ctx->ev_used[i] = tmp.ev_used[i];
        ctx->stage_ms[i] = tmp.stage_ms[i];
    }
    if (st == LMBD_E_OOM_ADMISSION)
        ctx->err = "footprint over the static scratch of " + std::to_string(kStaticScratchBytes) + " bytes (" +
                   tmp.err + ")";
    return st;
}

size_t lmbd_static_scratch_bytes(void) { return kStaticScratchBytes; }

lmbd_status lmbd_compute(lmbd_context* ctx, const lmbd_params* params, int32_t n_species,
                         const lmbd_species* species_table, const lmbd_structure* structure, int32_t mem,
                         void* hip_stream) {
    return lmbd_compute_batch(ctx, params, n_species, species_table, 1, structure, mem, hip_stream);
}

}  // extern "C"
