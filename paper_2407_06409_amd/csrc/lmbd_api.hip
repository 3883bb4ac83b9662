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
#include "lmbd_internal.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace lmbd;

namespace {

struct DBuf {
    void* p = nullptr;
    size_t cap = 0;
};

struct Plan {
    int64_t n_atoms = 0;
    int64_t total_sites = 0;
    int64_t table_len = 0;
    int64_t fac_len = 0, x_len = 0, aloc_len = 0, work_len = 0;
    int n1max = 0, nkmax = 0, nallmax = 0, n2max = 0;
    std::vector<int64_t> site_off, hash_off, fac_off, x_off, aloc_off, work_off, pl_off;
    int64_t pl_len = 0;
    std::vector<int32_t> hash_cap, fac_ld;
    size_t bytes = 0;
};

}  // namespace

struct lmbd_context {
    int device = 0;
    size_t budget = 0;
    std::string err;
    DBuf in_pos, in_sp, in_nu, in_w, atom_struct, sinfo, sp_table, omegas;
    DBuf pos_b, abar, sigma, Rv, a0v, r0v, cell_id, wrap, iota, sorted_cell, sorted_atoms;
    DBuf cell_start, cell_end, sort_temp, counts, flags;
    DBuf site_off, sites, hash_off, hash_cap, table, rev;
    DBuf fac_off, fac_ld, x_off, aloc_off, work_off;
    DBuf fac, xsol, alpha_loc, abar_loc, abar_cen, work, ca, cf;
    DBuf pl_i, pl_q, pl_off, pl_seg;
    DBuf e_out, f_out, a_out;
    bool profiling = false;
    hipEvent_t ev[2 * LMBD_N_STAGES] = {};
    bool ev_used[LMBD_N_STAGES] = {};
    double stage_ms[LMBD_N_STAGES] = {};
};

namespace {

hipError_t ensure(DBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (bytes <= b.cap) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        if (e != hipSuccess) return e;
    }
    const size_t nb = bytes + bytes / 8 + 256;
    hipError_t e = hipMalloc(&b.p, nb);
    if (e == hipSuccess) b.cap = nb;
    return e;
}

void release(DBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
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
    return LMBD_OK;
}

lmbd_status check_struct(lmbd_context* ctx, const lmbd_params* p, const lmbd_structure& s) {
    if (s.n_atoms < 1 || s.n_atoms > INT32_MAX / 4) return fail(ctx, LMBD_E_INVALID_ARG, "bad n_atoms");
    if (!s.pos || !s.species || !s.v_ratio) return fail(ctx, LMBD_E_INVALID_ARG, "NULL input array");
    if (!finite_pos(s.r_scs) || !finite_pos(s.r_nbr) || !finite_pos(s.r_mbd1) || !finite_pos(s.r_mbd2))
        return fail(ctx, LMBD_E_INVALID_ARG, "cutoffs must be positive");
    if (!(p->r_buf < s.r_scs) || !(p->r_buf < s.r_mbd1) || !(p->r_buf < s.r_mbd2))
        return fail(ctx, LMBD_E_INVALID_ARG, "r_buf must be smaller than every cutoff");
    const int npbc = (s.pbc[0] != 0) + (s.pbc[1] != 0) + (s.pbc[2] != 0);
    if (npbc != 0 && npbc != 3) return fail(ctx, LMBD_E_UNSUPPORTED, "mixed periodicity is not supported");
    if (npbc == 3) {
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
    si.r_big = std::max(2.0 * si.r_scs, si.r_nbr);
    si.atom_offset = atom_offset;
    si.cell_offset = cell_offset;
    si.n_atoms = (int)s.n_atoms;
    const int n = (int)s.n_atoms;
    if (s.pbc[0] && s.pbc[1] && s.pbc[2]) {
        si.periodic = 1;
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
            const double perp = vol / std::sqrt(cx * cx + cy * cy + cz * cz);
            int nc = (int)std::floor(2.0 * perp / si.r_big);
            nc = std::max(1, std::min(nc, 64));
            si.ncell[d] = nc;
            si.reach[d] = (int)std::ceil(si.r_big * nc / perp * (1.0 + 1e-9));
            if (si.reach[d] > 60) return fail(ctx, LMBD_E_UNSUPPORTED, "cutoff too large for the cell");
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

void build_plan(const std::vector<Counts>& cnt, int nw, int ncol, int n_max, bool forces, bool mixed, Plan& P) {
    const int64_t n = (int64_t)cnt.size();
    P.n_atoms = n;
    P.site_off.resize(n + 1);
    P.hash_off.resize(n + 1);
    P.fac_off.resize(n + 1);
    P.x_off.resize(n + 1);
    P.aloc_off.resize(n + 1);
    P.work_off.resize(n + 1);
    P.pl_off.resize(n + 1);
    P.hash_cap.resize(n);
    P.fac_ld.resize(n);
    const int mmax = forces ? std::max(1, n_max - 1) : std::max(1, (n_max + 1) / 2);
    int64_t so = 0, ho = 0, fo = 0, xo = 0, ao = 0, wo = 0, po = 0;
    P.n1max = P.nkmax = P.nallmax = P.n2max = 0;
    for (int64_t k = 0; k < n; ++k) {
        const Counts& c = cnt[k];
        P.site_off[k] = so;
        P.hash_off[k] = ho;
        P.fac_off[k] = fo;
        P.x_off[k] = xo;
        P.aloc_off[k] = ao;
        P.work_off[k] = wo;
        P.pl_off[k] = po;
        po += (int64_t)c.n1 * (c.n12 - c.n1);
        const int64_t N1 = 3 * (int64_t)c.n1, N3 = 3 * (int64_t)c.nK;
        P.hash_cap[k] = (int32_t)next_pow2(2 * (int64_t)c.n_all);
        P.fac_ld[k] = (int32_t)N1;
        so += c.n_all;
        ho += P.hash_cap[k];
        fo += (int64_t)nw * N1 * N1;
        xo += (int64_t)nw * N1 * 3;
        ao += (int64_t)c.n1 * nw;
        wo += N3 * N3 + (int64_t)mmax * N3 * ncol + (forces ? (int64_t)n_max * N3 * ncol : 0);
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
    const size_t d = sizeof(double);
    size_t b = 0;
    b += (size_t)so * sizeof(Site) + (size_t)so * 4 /*rev*/ + (size_t)ho * 4 /*hash*/;
    const size_t wsz = mixed ? sizeof(float) : sizeof(double);
    b += (size_t)(fo + wo) * wsz + (size_t)(xo + 2 * ao) * d;
    b += (size_t)n * nw * d /*abar_cen*/;
    if (forces) b += (size_t)so * nw * d /*ca*/ + (size_t)(1 + nw) * so * 3 * d /*cf*/;
    b += (size_t)n * (8 * d + 64);  // per-atom tables and offsets
    b += (size_t)po * 8 + (size_t)(so + 2 * n) * 4;  // coupling lists
    P.bytes = b;
}

template <typename T>
lmbd_status upload(lmbd_context* ctx, DBuf& b, const std::vector<T>& v, hipStream_t st) {
    HIP_TRY(ensure(b, sizeof(T) * v.size()));
    HIP_TRY(hipMemcpyAsync(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
    return LMBD_OK;
}

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
    DBuf* all[] = {&ctx->in_pos, &ctx->in_sp, &ctx->in_nu, &ctx->in_w, &ctx->atom_struct, &ctx->sinfo,
                   &ctx->sp_table, &ctx->omegas, &ctx->pos_b, &ctx->abar, &ctx->sigma, &ctx->Rv,
                   &ctx->a0v, &ctx->r0v, &ctx->cell_id, &ctx->wrap, &ctx->iota, &ctx->sorted_cell,
                   &ctx->sorted_atoms, &ctx->cell_start, &ctx->cell_end, &ctx->sort_temp, &ctx->counts,
                   &ctx->flags, &ctx->site_off, &ctx->sites, &ctx->hash_off, &ctx->hash_cap, &ctx->table,
                   &ctx->rev, &ctx->fac_off, &ctx->fac_ld, &ctx->x_off, &ctx->aloc_off, &ctx->work_off,
                   &ctx->fac, &ctx->xsol, &ctx->alpha_loc, &ctx->abar_loc, &ctx->abar_cen, &ctx->work,
                   &ctx->ca, &ctx->cf, &ctx->e_out, &ctx->f_out, &ctx->a_out, &ctx->pl_i, &ctx->pl_q,
                   &ctx->pl_off, &ctx->pl_seg};
    for (DBuf* b : all) release(*b);
    (void)hipSetDevice(prev);
    delete ctx;
}

static const char* kStageNames[LMBD_N_STAGES] = {"prep_sort_count", "nbr_fill_revmap", "scs_forward",
                                                  "mbd",  "gather_central", "scs_adjoint", "gather_forces"};

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

// Host-side neighbour counting for the footprint estimate (same radii and the
// same cell geometry as the device, plain loops).
static lmbd_status host_counts(lmbd_context* ctx, const lmbd_structure& s, std::vector<Counts>& out) {
    StructInfo si;
    lmbd_status st = make_struct_info(ctx, s, s.pos, 0, 0, si);
    if (st != LMBD_OK) return st;
    const int n = (int)s.n_atoms;
    std::vector<double> p(3 * (size_t)n);
    for (int i = 0; i < 3 * n; ++i) p[i] = s.pos[i] / kBohr;
    int range[3];
    for (int d = 0; d < 3; ++d) range[d] = si.periodic ? si.reach[d] + 1 : 0;
    const double r1 = si.r_scs * si.r_scs, rK = si.r_nbr * si.r_nbr, r2 = 4 * si.r_scs * si.r_scs,
                 rb = si.r_big * si.r_big;
    for (int k = 0; k < n; ++k) {
        Counts c{1, 1, 1, 1};
        for (int a = -range[0]; a <= range[0]; ++a)
            for (int b = -range[1]; b <= range[1]; ++b)
                for (int e = -range[2]; e <= range[2]; ++e)
                    for (int j = 0; j < n; ++j) {
                        if (j == k && a == 0 && b == 0 && e == 0) continue;
                        double v[3];
                        for (int d = 0; d < 3; ++d)
                            v[d] = p[3 * j + d] - p[3 * k + d] +
                                   (si.periodic ? a * si.cell[d] + b * si.cell[3 + d] + e * si.cell[6 + d] : 0.0);
                        const double d2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
                        if (d2 >= rb) continue;
                        c.n_all++;
                        c.n1 += d2 < r1;
                        c.nK += d2 < rK;
                        c.n12 += d2 < r2;
                    }
        out.push_back(c);
    }
    return LMBD_OK;
}

lmbd_status lmbd_estimate_footprint(const lmbd_params* params, int32_t n_structs,
                                    const lmbd_structure* structs, size_t* bytes) {
    lmbd_context* ctx = nullptr;
    if (!bytes || !structs || n_structs < 1) return LMBD_E_INVALID_ARG;
    lmbd_status st = check_params(ctx, params);
    if (st != LMBD_OK) return st;
    std::vector<Counts> cnt;
    bool forces = false;
    for (int s = 0; s < n_structs; ++s) {
        st = check_struct(ctx, params, structs[s]);
        if (st != LMBD_OK) return st;
        st = host_counts(ctx, structs[s], cnt);
        if (st != LMBD_OK) return st;
        forces = forces || structs[s].forces != nullptr;
    }
    Plan P;
    build_plan(cnt, params->n_freq + 1, 3 * params->n_freq, params->n_max, forces,
               params->precision == LMBD_MIXED, P);
    *bytes = P.bytes;
    return LMBD_OK;
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
    bool forces = false;
    int64_t N64 = 0;
    for (int s = 0; s < n_structs; ++s) {
        st = check_struct(ctx, params, structs[s]);
        if (st != LMBD_OK) return st;
        forces = forces || structs[s].forces != nullptr;
        N64 += structs[s].n_atoms;
    }
    if (N64 > INT32_MAX / 8) return fail(ctx, LMBD_E_UNSUPPORTED, "too many atoms in one call");
    const int N = (int)N64;
    const int nq = params->n_freq, nw = nq + 1, ncol = 3 * nq, n_max = params->n_max;
    const bool mixed = params->precision == LMBD_MIXED;
    const size_t wsz = mixed ? sizeof(float) : sizeof(double);  // matrix and workspace element size
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
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

    // --- inputs into contiguous batch arrays
    HIP_TRY(ensure(ctx->in_pos, sizeof(double) * 3 * N));
    HIP_TRY(ensure(ctx->in_sp, sizeof(int32_t) * N));
    HIP_TRY(ensure(ctx->in_nu, sizeof(double) * N));
    HIP_TRY(ensure(ctx->in_w, sizeof(double) * N));
    std::vector<int32_t> atom_struct(N);
    std::vector<double> pos_host;
    std::vector<double> ones;
    std::vector<StructInfo> sinfo(n_structs);
    int off = 0, coff = 0;
    for (int s = 0; s < n_structs; ++s) {
        const lmbd_structure& S = structs[s];
        const int n = (int)S.n_atoms;
        HIP_TRY(hipMemcpyAsync(as<double>(ctx->in_pos) + 3 * (size_t)off, S.pos, sizeof(double) * 3 * n, h2d, stream));
        HIP_TRY(hipMemcpyAsync(as<int32_t>(ctx->in_sp) + off, S.species, sizeof(int32_t) * n, h2d, stream));
        HIP_TRY(hipMemcpyAsync(as<double>(ctx->in_nu) + off, S.v_ratio, sizeof(double) * n, h2d, stream));
        if (S.e_weight) {
            HIP_TRY(hipMemcpyAsync(as<double>(ctx->in_w) + off, S.e_weight, sizeof(double) * n, h2d, stream));
        } else {
            ones.assign(n, 1.0);
            HIP_TRY(hipMemcpyAsync(as<double>(ctx->in_w) + off, ones.data(), sizeof(double) * n,
                                   hipMemcpyHostToDevice, stream));
            HIP_TRY(hipStreamSynchronize(stream));
        }
        const double* ph = S.pos;
        if (mem == LMBD_DEVICE && !(S.pbc[0] && S.pbc[1] && S.pbc[2])) {
            pos_host.resize(3 * (size_t)n);
            HIP_TRY(hipMemcpyAsync(pos_host.data(), S.pos, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            ph = pos_host.data();
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
        for (int i = 0; i < n; ++i) atom_struct[off + i] = s;
        off += n;
        coff += sinfo[s].ncell[0] * sinfo[s].ncell[1] * sinfo[s].ncell[2];
    }
    const int n_cells = coff;
    std::vector<double> omegas(nw);
    omegas[0] = 0.0;
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
    HIP_TRY(ensure(ctx->pos_b, sizeof(double) * 3 * N));
    HIP_TRY(ensure(ctx->abar, sizeof(double) * (size_t)N * nw));
    HIP_TRY(ensure(ctx->sigma, sizeof(double) * (size_t)N * nw));
    HIP_TRY(ensure(ctx->Rv, sizeof(double) * N));
    HIP_TRY(ensure(ctx->a0v, sizeof(double) * N));
    HIP_TRY(ensure(ctx->r0v, sizeof(double) * N));
    HIP_TRY(ensure(ctx->cell_id, sizeof(int32_t) * N));
    HIP_TRY(ensure(ctx->wrap, sizeof(int32_t) * 3 * N));
    HIP_TRY(ensure(ctx->sorted_cell, sizeof(int32_t) * N));
    HIP_TRY(ensure(ctx->sorted_atoms, sizeof(int32_t) * N));
    HIP_TRY(ensure(ctx->cell_start, sizeof(int32_t) * n_cells));
    HIP_TRY(ensure(ctx->cell_end, sizeof(int32_t) * n_cells));
    HIP_TRY(ensure(ctx->counts, sizeof(Counts) * N));
    HIP_TRY(ensure(ctx->flags, sizeof(int) * 4));
    int flags_init[4] = {0, INT_MAX, 0, 0};
    HIP_TRY(hipMemcpyAsync(ctx->flags.p, flags_init, sizeof(flags_init), hipMemcpyHostToDevice, stream));
    int* err = as<int>(ctx->flags);
    int* err_atom = err + 1;
    HIP_TRY(mark(0, 0));
    HIP_TRY(launch_prep(stream, N, as<double>(ctx->in_pos), as<int32_t>(ctx->in_sp), as<double>(ctx->in_nu),
                        as<int32_t>(ctx->atom_struct), as<StructInfo>(ctx->sinfo), as<double>(ctx->sp_table),
                        n_species, as<double>(ctx->omegas), nw, as<double>(ctx->pos_b), as<double>(ctx->abar),
                        as<double>(ctx->sigma), as<double>(ctx->Rv), as<double>(ctx->a0v), as<double>(ctx->r0v),
                        as<int32_t>(ctx->cell_id), as<int32_t>(ctx->wrap), err));
    size_t temp_bytes = 0;
    HIP_TRY(sort_cells(stream, N, n_cells, nullptr, nullptr, nullptr, nullptr, nullptr, &temp_bytes, nullptr,
                       nullptr));
    HIP_TRY(ensure(ctx->sort_temp, temp_bytes));
    temp_bytes = ctx->sort_temp.cap;
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
    HIP_TRY(launch_nbr_count(stream, na, as<Counts>(ctx->counts)));
    HIP_TRY(mark(0, 1));
    std::vector<Counts> cnt(N);
    int flags[4];
    HIP_TRY(hipMemcpyAsync(cnt.data(), ctx->counts.p, sizeof(Counts) * N, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(flags, ctx->flags.p, sizeof(flags), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (flags[0] & 1) return fail(ctx, LMBD_E_INVALID_ARG, "invalid species, volume ratio or position");

    // --- memory plan
    Plan P;
    build_plan(cnt, nw, ncol, n_max, forces, mixed, P);
    if (P.n1max > kMaxN1 || P.nkmax > kMaxNK || P.nallmax > kMaxSites)
        return fail(ctx, LMBD_E_UNSUPPORTED,
                    "neighbourhood too large (n1 " + std::to_string(P.n1max) + ", nK " + std::to_string(P.nkmax) +
                        ", sites " + std::to_string(P.nallmax) + ")");
    int lds_limit = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    if (scs_lds_bytes(P.n1max, P.n2max, mixed) > (size_t)lds_limit || mbd_lds_bytes(P.nkmax, nw, nq, n_max) > (size_t)lds_limit)
        return fail(ctx, LMBD_E_UNSUPPORTED, "neighbourhood needs more LDS than the device offers (" +
                                                 std::to_string(lds_limit) + " bytes)");
    if (ctx->budget && P.bytes > ctx->budget)
        return fail(ctx, LMBD_E_OOM_ADMISSION, "footprint " + std::to_string(P.bytes) + " bytes over budget");
    std::vector<int64_t> so(P.site_off.begin(), P.site_off.end() - 1);
    std::vector<int64_t> ho(P.hash_off.begin(), P.hash_off.end() - 1);
    std::vector<int64_t> fo(P.fac_off.begin(), P.fac_off.end() - 1);
    std::vector<int64_t> xo(P.x_off.begin(), P.x_off.end() - 1);
    std::vector<int64_t> ao(P.aloc_off.begin(), P.aloc_off.end() - 1);
    std::vector<int64_t> wo(P.work_off.begin(), P.work_off.end() - 1);
    std::vector<int64_t> plo(P.pl_off.begin(), P.pl_off.end() - 1);
    if ((st = upload(ctx, ctx->pl_off, plo, stream)) != LMBD_OK) return st;
    if ((st = upload(ctx, ctx->site_off, so, stream)) != LMBD_OK) return st;
    if ((st = upload(ctx, ctx->hash_off, ho, stream)) != LMBD_OK) return st;
    if ((st = upload(ctx, ctx->hash_cap, P.hash_cap, stream)) != LMBD_OK) return st;
    if ((st = upload(ctx, ctx->fac_off, fo, stream)) != LMBD_OK) return st;
    if ((st = upload(ctx, ctx->fac_ld, P.fac_ld, stream)) != LMBD_OK) return st;
    if ((st = upload(ctx, ctx->x_off, xo, stream)) != LMBD_OK) return st;
    if ((st = upload(ctx, ctx->aloc_off, ao, stream)) != LMBD_OK) return st;
    if ((st = upload(ctx, ctx->work_off, wo, stream)) != LMBD_OK) return st;
    const int64_t TS = P.total_sites;
    HIP_TRY(ensure(ctx->sites, sizeof(Site) * TS));
    HIP_TRY(ensure(ctx->table, sizeof(int32_t) * P.table_len));
    HIP_TRY(ensure(ctx->rev, sizeof(int32_t) * TS));
    HIP_TRY(ensure(ctx->fac, wsz * P.fac_len));
    HIP_TRY(ensure(ctx->xsol, sizeof(double) * P.x_len));
    HIP_TRY(ensure(ctx->alpha_loc, sizeof(double) * P.aloc_len));
    HIP_TRY(ensure(ctx->abar_loc, sizeof(double) * P.aloc_len));
    HIP_TRY(ensure(ctx->abar_cen, sizeof(double) * (size_t)N * nw));
    HIP_TRY(ensure(ctx->work, wsz * P.work_len));
    HIP_TRY(ensure(ctx->e_out, sizeof(double) * N));
    if (forces) {
        HIP_TRY(ensure(ctx->ca, sizeof(double) * TS * nw));
        HIP_TRY(ensure(ctx->cf, sizeof(double) * (size_t)(1 + nw) * TS * 3));
        HIP_TRY(ensure(ctx->f_out, sizeof(double) * 3 * N));
    }
    HIP_TRY(ensure(ctx->a_out, sizeof(double) * N));
    HIP_TRY(ensure(ctx->pl_i, sizeof(int32_t) * P.pl_len));
    HIP_TRY(ensure(ctx->pl_q, sizeof(int32_t) * P.pl_len));
    HIP_TRY(ensure(ctx->pl_seg, sizeof(int32_t) * (TS + 2 * (int64_t)N)));

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
    sa.n_refine = 2;
    sa.fac_off = as<int64_t>(ctx->fac_off);
    sa.fac_ld = as<int32_t>(ctx->fac_ld);
    sa.xsol = as<double>(ctx->xsol);
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
    HIP_TRY(launch_scs_forward(stream, sa, P.n1max, P.n2max, mixed));
    HIP_TRY(mark(2, 1));

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
    ma.e_weight = as<double>(ctx->in_w);
    ma.e_atom = as<double>(ctx->e_out);
    ma.work = ctx->work.p;
    ma.work_off = as<int64_t>(ctx->work_off);
    ma.forces = forces ? 1 : 0;
    ma.abar_loc = as<double>(ctx->abar_loc);
    ma.ca = forces ? as<double>(ctx->ca) : nullptr;
    ma.cf0 = forces ? as<double>(ctx->cf) : nullptr;
    HIP_TRY(mark(3, 0));
    HIP_TRY(launch_mbd(stream, ma, P.nkmax, mixed));
    HIP_TRY(mark(3, 1));

    if (forces) {
        HIP_TRY(mark(4, 0));
        HIP_TRY(launch_gather_central(stream, N, nw, sa.counts, sa.site_off, sa.sites, as<int32_t>(ctx->rev),
                                      as<double>(ctx->ca), as<double>(ctx->abar_cen)));
        HIP_TRY(mark(4, 1));
        sa.abar_loc = as<double>(ctx->abar_loc);
        sa.abar_cen = as<double>(ctx->abar_cen);
        sa.cf_slice = TS * 3;
        sa.cf = as<double>(ctx->cf) + sa.cf_slice;  // slices 1..nw
        HIP_TRY(mark(5, 0));
        HIP_TRY(launch_scs_adjoint(stream, sa, P.n1max, P.n2max, mixed));
        HIP_TRY(mark(5, 1));
        HIP_TRY(mark(6, 0));
        HIP_TRY(launch_gather_forces(stream, N, 1 + nw, TS * 3, sa.counts, sa.site_off, sa.sites,
                                     as<int32_t>(ctx->rev), as<double>(ctx->cf), as<double>(ctx->f_out)));
        HIP_TRY(mark(6, 1));
    }
    HIP_TRY(launch_central_static(stream, N, nw, sa.alpha_loc, sa.aloc_off, as<double>(ctx->a_out)));

    // --- outputs
    off = 0;
    for (int s = 0; s < n_structs; ++s) {
        const lmbd_structure& S = structs[s];
        const int n = (int)S.n_atoms;
        if (S.e_atom)
            HIP_TRY(hipMemcpyAsync(S.e_atom, as<double>(ctx->e_out) + off, sizeof(double) * n, d2o, stream));
        if (S.forces)
            HIP_TRY(hipMemcpyAsync(S.forces, as<double>(ctx->f_out) + 3 * (size_t)off, sizeof(double) * 3 * n, d2o,
                                   stream));
        if (S.alpha_scs0)
            HIP_TRY(hipMemcpyAsync(S.alpha_scs0, as<double>(ctx->a_out) + off, sizeof(double) * n, d2o, stream));
        off += n;
    }
    HIP_TRY(hipMemcpyAsync(flags, ctx->flags.p, sizeof(flags), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
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
    return LMBD_OK;
}

lmbd_status lmbd_compute(lmbd_context* ctx, const lmbd_params* params, int32_t n_species,
                         const lmbd_species* species_table, const lmbd_structure* structure, int32_t mem,
                         void* hip_stream) {
    return lmbd_compute_batch(ctx, params, n_species, species_table, 1, structure, mem, hip_stream);
}

}  // extern "C"
