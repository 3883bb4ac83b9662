/*
 * lmbd.h -- C ABI of the atom-wise linear many-body dispersion (lMBD) library
 * for AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, for every atom k of one or more structures, the
 * atom-wise MBD energy of Muhli, Ala-Nissila & Caro (2024), "Atom-wise
 * formulation of the many-body dispersion problem for linear-scaling van der
 * Waals corrections":
 *
 *   E_k = (1/2pi) sum_q w_q sum_{n=2}^{n_max} c_n Tr[ G~_K(w_q)^n ]_kk     (Sec. III.A,
 *         symmetrised local energy), G~_K = sqrt(A_K) T_LR,K sqrt(A_K),
 *
 * where A_K holds the blended SCS polarisabilities of the neighbourhood of k
 * (Sec. III.B, local polarisability system B~_K alpha~_K = d_K and the
 * central/local combination), and the exact forces
 *
 *   F_a = -d( sum_k w_k E_k ) / d R_a       (Hirshfeld ratios held fixed),
 *
 * from hand-written adjoint kernels.  Units: positions and lengths in Angstrom,
 * frequencies in hartree, free-atom data in atomic units (bohr^3, Ha bohr^6,
 * bohr), energies in eV, forces in eV/Angstrom.  Internally everything is in
 * Hartree atomic units (CODATA 2018 bohr and hartree).
 *
 * Plain C99; no C++ or torch types cross this boundary.  Every array is owned
 * by the caller; the library keeps no caller pointer after a call returns.
 */
#ifndef LMBD_H
#define LMBD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LMBD_ABI_VERSION 7

typedef enum lmbd_status {
    LMBD_OK = 0,
    LMBD_E_INVALID_ARG = 1,    /* bad pointer, size, NaN/Inf input, inconsistent cutoffs */
    LMBD_E_OOM = 2,            /* device allocation failed */
    LMBD_E_OOM_ADMISSION = 3,  /* request larger than the memory budget of the context */
    LMBD_E_DEVICE = 4,         /* a HIP runtime call failed; see lmbd_last_error */
    LMBD_E_SCS_BREAKDOWN = 5,  /* a local SCS matrix B~_K is not positive definite */
    LMBD_E_UNSUPPORTED = 6,    /* a size limit of the kernels is exceeded: K1 (r < r_scs) above 256
                                  sites, an SCS shell whose coupling rows outgrow the pair-list
                                  kernel's LDS, or the largest ball of an atom above 32,768 sites
                                  (K above 400 sites is served by the global-site MBD form) */
    LMBD_E_CANCELLED = 7,      /* a queued request was dropped when its server was destroyed */
    LMBD_E_POLARISATION = 8    /* LMBD_CN_FIT: a spectrum bound of G~_K reaches 1 (polarisation
                                  catastrophe, Sec. III.A): ln(1 - x) has no fit there */
} lmbd_status;

/* precision of the hot path */
enum { LMBD_FP64 = 0, LMBD_MIXED = 1 };
/* frequency treatment of the SCS polarisabilities */
enum { LMBD_SCS_EXACT = 0, LMBD_SCS_LORENTZ = 1 };
/* where the caller's arrays live */
enum { LMBD_HOST = 0, LMBD_DEVICE = 1 };
/* what the forces output holds */
enum { LMBD_FORCES_EXACT = 0, LMBD_FORCES_PAPER = 1 };
/* where the body-order coefficients c_n come from */
enum { LMBD_CN_SERIES = 0, LMBD_CN_FIT = 1 };

/* Free-atom reference data of one species (Sec. II.B: the TS polarisability,
 * its characteristic frequency omega = 4 C6 / (3 alpha0^2), and vdW radius). */
typedef struct lmbd_species {
    double alpha0;   /* static free-atom polarisability, bohr^3 (> 0) */
    double c6;       /* free-atom C6 coefficient, Ha bohr^6 (> 0) */
    double r0;       /* free-atom vdW radius, bohr (> 0) */
} lmbd_species;

/* Method parameters, shared by every structure of a call.
 *  beta, damp_d : Fermi damping f(r,S) = 1/(1+exp(-d (r/S - 1))), S = beta (R_i + R_j)
 *                 (Sec. II.B; defaults 0.83 and 6)
 *  r_buf        : width of the smooth cutoff buffers f_SR and f_LR (Sec. III.A/III.B), A
 *  r_inner      : inner buffer f_inner for shell atoms near K1 atoms (Sec. III.B), A
 *  n_max        : highest body order of the series (>= 2)
 *  c_n          : host array of n_max+1 series coefficients, or NULL for c_n = -1/n
 *                 (the logarithm series; c_0 and c_1 are ignored)
 *  n_freq, omega, weight : host arrays; imaginary-frequency nodes (Ha) and weights of
 *                 int_0^inf d omega; the library applies the 1/(2 pi) itself
 *  precision    : LMBD_FP64 or LMBD_MIXED
 *  scs_freq     : LMBD_SCS_EXACT solves the local SCS systems at omega = 0 and at
 *                 every node; LMBD_SCS_LORENTZ solves them at omega = 0 and omega_ref
 *                 only and gives the blended polarisability of every site the
 *                 two-point Lorentzian form of Sec. III.C (Eqs. alpha_SCS_freq,
 *                 char-freq): alpha(w) = alpha(0) / (1 + (w / w~)^2), with w~ fixed
 *                 by alpha(0) and alpha(omega_ref).  Such a site needs
 *                 alpha(0) >= alpha(omega_ref) > 0, else the call fails with
 *                 LMBD_E_SCS_BREAKDOWN.
 *  omega_ref    : reference frequency of LMBD_SCS_LORENTZ (Ha, > 0; the paper leaves
 *                 it empirical); ignored by LMBD_SCS_EXACT
 *  force_model  : LMBD_FORCES_EXACT: forces = -d( sum_k w_k E_k ) / dR, the exact
 *                 gradient.  LMBD_FORCES_PAPER: the approximate forces of Sec. III.D
 *                 (Eqs. full-pol-grad, cent-appr-step, cent-appr): each atom's force
 *                 comes from its own neighbourhood only, F_k = -w_k d E^tot_k / d r_k of
 *                 the total energy k sees, with the central polarisabilities of the
 *                 other atoms held fixed and, for n >= 3, only k's block row and column
 *                 of dG~ kept (the n = 2 term in full); the frequency integral is the
 *                 same quadrature as the energy.  Not the gradient of sum_k E_k (exact
 *                 without screening when every neighbourhood holds the whole
 *                 structure).  Uses the dense MBD products; dE_dv must be NULL.
 *  cn_mode      : LMBD_CN_SERIES: the c_n above for every atom and node.  LMBD_CN_FIT:
 *                 the eigenvalue-bounded polynomial of Sec. III.A (Eqs. diagonal_appr,
 *                 eigendecomp, polynomial-fit): for every atom k and node q the bounds
 *                 [lambda_min, lambda_max] of the spectrum of G~_K(w_q) are estimated by
 *                 `lanczos_steps` Lanczos steps, and c_0 .. c_n_max are the least-squares
 *                 polynomial of degree n_max to ln(1 - x) on that interval (sum of the
 *                 squared residuals at its 32 Gauss-Legendre points, each weighted by
 *                 its quadrature weight); the energy keeps n = 2 .. n_max.  The Lanczos
 *                 iteration starts from the vector with entry (site, c) = U(k, base atom,
 *                 lattice shift, c) of the SplitMix64 hash (Steele, Lea and Flood 2014):
 *                 with k and the base atom counted within their structure, s the lattice
 *                 shift packed as ((s0 + 128) << 16) | ((s1 + 128) << 8) | (s2 + 128) and
 *                 SM the SplitMix64 output function of a 64-bit counter,
 *                 U = (SM(SM(k 2^32 + base) + 4 s + c) >> 11) 2^-53 - 1/2; it stops early
 *                 at beta_{j+1} <= 1e-10 (|alpha_j| + beta_j) (an invariant subspace).  An
 *                 interval narrower than 1e-12 takes c_n = -1/n.  The forces hold the
 *                 fitted c_n fixed, as the force expression of Sec. III.D does (they are
 *                 not the derivative of the refitted energy).  A bound lambda_max >= 1
 *                 fails the call with LMBD_E_POLARISATION (lowest such atom in
 *                 lmbd_last_error).  c_n must be NULL.
 *  lanczos_steps: Lanczos steps of LMBD_CN_FIT and of the `spectrum` output, 2 .. 64
 *                 (0 = 20).
 * Cutoffs are per structure (lmbd_structure). */
typedef struct lmbd_params {
    double beta;
    double damp_d;
    double r_buf;
    double r_inner;
    int32_t n_max;
    const double* c_n;
    int32_t n_freq;
    const double* omega;
    const double* weight;
    int32_t precision;
    int32_t scs_freq;
    double omega_ref;
    int32_t force_model;
    int32_t cn_mode;
    int32_t lanczos_steps;
} lmbd_params;

/* One structure of a batch.  Pointers are host or device pointers according to
 * the `mem` argument of the call.
 *  n_atoms     : number of atoms (>= 1)
 *  pos         : [n_atoms][3] Cartesian positions, A
 *  species     : [n_atoms] index into the species table
 *  v_ratio     : [n_atoms] Hirshfeld-volume ratios nu (> 0)
 *  cell        : HOST array [3][3], rows = lattice vectors (A); required when any
 *                pbc[d] != 0 (non-singular; a non-periodic row only fixes the
 *                fractional frame of that direction, e.g. the normal of a slab),
 *                ignored (may be NULL) for an open structure
 *  pbc         : periodicity per lattice direction (any combination: open,
 *                slab, wire or bulk); periodic images are taken only along the
 *                directions with pbc[d] != 0
 *  r_scs       : SCS cutoff: K1 = B(r_scs), K2 = B(2 r_scs) \ B(r_scs) (Sec. III.B)
 *  r_nbr       : radius of the energy neighbourhood K = B(r_nbr) (Sec. III.A)
 *  r_mbd1/2    : f_LR cutoffs for pairs touching / not touching the central atom;
 *                the call fails with LMBD_E_INVALID_ARG unless
 *                r_nbr >= r_mbd1 >= r_mbd2 (Sec. III.A: the central atom has the
 *                larger radius, and K must hold every pair that f_LR couples)
 *  r_2b1/2     : the two-body radii of Sec. III.A: the n = 2 term of the energy uses a
 *                T_LR with f_LR cut at r_2b1 for pairs touching the central atom and at
 *                r_2b2 for the others (the terms n >= 3 keep r_mbd1/2).  The energy and
 *                the exact forces depend on r_2b1 only; r_2b2 enters the approximate
 *                forces (LMBD_FORCES_PAPER, whose n = 2 term is the frame's whole trace).
 *                0 = the MBD radius; required r_nbr >= r_2b1 >= r_2b2 > r_buf.  With
 *                radii that differ from the MBD ones n_max must be finite (always so here)
 *  e_weight    : [n_atoms] adjoint seeds w_k of the forces, or NULL for w_k = 1
 *  e_atom      : [n_atoms] output per-atom energies E_k (eV), or NULL
 *  forces      : [n_atoms][3] output forces (eV/A), or NULL for energies only
 *  alpha_scs0  : [n_atoms] output central static SCS polarisabilities (bohr^3), or NULL
 *  dE_dv       : [n_atoms] output d( sum_k w_k E_k ) / d nu_i (eV), the exact
 *                derivative with respect to the Hirshfeld-volume ratios (through
 *                the TS polarisabilities, attenuation lengths and radii of
 *                Sec. II.B), so that a caller can apply the chain rule of the
 *                volume gradients of Sec. III.D outside the library; or NULL
 *  spectrum    : [n_atoms][n_freq][2] output: the Lanczos bounds [lambda_min,
 *                lambda_max] of the spectrum of G~_K(w_q) of every atom and node (the
 *                estimates LMBD_CN_FIT fits on; lanczos_steps steps), a diagnostic of
 *                the polarisation catastrophe (lambda_max >= 1) in either cn_mode; or NULL.
 *                A Lanczos bound lies inside the true spectrum (lambda_max from below). */
typedef struct lmbd_structure {
    int64_t n_atoms;
    const double* pos;
    const int32_t* species;
    const double* v_ratio;
    const double* cell;
    int32_t pbc[3];
    double r_scs;
    double r_nbr;
    double r_mbd1;
    double r_mbd2;
    double r_2b1;
    double r_2b2;
    const double* e_weight;
    double* e_atom;
    double* forces;
    double* alpha_scs0;
    double* dE_dv;
    double* spectrum;
} lmbd_structure;

typedef struct lmbd_context lmbd_context;

/* ABI version of the loaded library (LMBD_ABI_VERSION of its build). */
int32_t lmbd_abi_version(void);

/* Create a context on HIP device `device`.  The context owns its device
 * workspaces and caches them between calls; it is not thread-safe.
 * Returns LMBD_E_INVALID_ARG for a NULL `out` or a bad device index. */
lmbd_status lmbd_create(int32_t device, lmbd_context** out);

/* Release the context and every device buffer it owns.  NULL is ignored. */
void lmbd_destroy(lmbd_context* ctx);

/* Cap the device memory (bytes) that one call may use; 0 = no cap.  A call whose
 * footprint exceeds the cap fails with LMBD_E_OOM_ADMISSION after the neighbour
 * counts and before any workspace that depends on them is allocated. */
lmbd_status lmbd_set_memory_budget(lmbd_context* ctx, size_t bytes);

/* Energies (and forces) of a batch of structures in one set of kernel launches.
 *
 * species_table: HOST array of n_species entries.  structs: HOST array of
 * n_structs descriptors.  mem = LMBD_DEVICE: every array of the descriptors is a
 * device pointer on the context's device; mem = LMBD_HOST: host arrays.  All
 * work is ordered on `hip_stream` (a hipStream_t, NULL = default stream) and
 * the call returns when the outputs are written (it synchronises the stream,
 * once after the neighbour counts and once at the end), so that a breakdown or
 * a bad input is reported by its status.  Concurrent calls on different
 * streams need one context each (one host thread per context); their kernels
 * overlap on the device.  Results of a structure are bitwise independent of the
 * other structures of the batch.  On error the outputs are unspecified. */
lmbd_status lmbd_compute_batch(lmbd_context* ctx, const lmbd_params* params,
                               int32_t n_species, const lmbd_species* species_table,
                               int32_t n_structs, const lmbd_structure* structs,
                               int32_t mem, void* hip_stream);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it): the same
 * evaluation as lmbd_compute_batch, with the same arguments, outputs and status
 * codes, but every workspace buffer is carved from a static device array of
 * lmbd_static_scratch_bytes() bytes (64 MiB) that the library holds on each GPU
 * it runs on until the process ends.  The call allocates and frees no device
 * memory, and leaves the context's own cached buffers untouched.  A call whose
 * exact footprint (lmbd_estimate_footprint) exceeds the array fails with
 * LMBD_E_OOM_ADMISSION before any kernel runs; 64 MiB holds, for example, 64
 * carbon atoms at a 5 A cutoff with forces in FP64.  Every call on one GPU
 * shares that GPU's array and its contents are those of the last call: calls
 * from several host threads on one GPU are serialised by the library, and a
 * caller must not overlap such a call with another process's use of the same
 * library copy on that GPU.  Inputs and outputs are the caller's, as in
 * lmbd_compute_batch; the call returns once the outputs are written. */
lmbd_status lmbd_compute_batch_static(lmbd_context* ctx, const lmbd_params* params,
                                      int32_t n_species, const lmbd_species* species_table,
                                      int32_t n_structs, const lmbd_structure* structs,
                                      int32_t mem, void* hip_stream);

/* Size in bytes of the static device array behind lmbd_compute_batch_static. */
size_t lmbd_static_scratch_bytes(void);

/* Single-structure convenience form of lmbd_compute_batch. */
lmbd_status lmbd_compute(lmbd_context* ctx, const lmbd_params* params,
                         int32_t n_species, const lmbd_species* species_table,
                         const lmbd_structure* structure, int32_t mem, void* hip_stream);

/* Device bytes a call on these structures would need: the exact size of the
 * workspace lmbd_compute_batch lays out, from host-side neighbour counts that
 * equal the device's (every array of the descriptors is a HOST array here,
 * whatever `mem` a later call uses).  Exact for species tables of up to 64
 * entries.  Needs the HIP runtime, not a launch. */
lmbd_status lmbd_estimate_footprint(const lmbd_params* params, int32_t n_structs,
                                    const lmbd_structure* structs, size_t* bytes);

/* Stage timers.  With profiling on, the library records a HIP event on the
 * call's stream before and after each stage of the hot path and, once the call
 * has completed, keeps the elapsed milliseconds of the last call per stage.
 * Stages: 0 prep+cell sort+neighbour counts, 1 neighbour lists+reverse map+
 * coupling lists, 2 right-hand sides d of the local SCS, 3 local SCS assembly,
 * factorisation, first solve and, in the mixed path, its refinement (one
 * kernel), 4 unused (the refinement had kernels of its own here; not recorded),
 * 5 local MBD energy
 * (+adjoint), 6 central-polarisability gather, 7 adjoint SCS solves, 8 SCS
 * pair gradients (and, when dE_dv is requested, the volume-ratio adjoint),
 * 9 force gather. */
#define LMBD_N_STAGES 10
lmbd_status lmbd_set_profiling(lmbd_context* ctx, int32_t enable);
/* ms: caller array of LMBD_N_STAGES doubles; stages not run in the last call read 0. */
lmbd_status lmbd_stage_times(const lmbd_context* ctx, double* ms);
/* Name of stage i (0 <= i < LMBD_N_STAGES), or NULL. */
const char* lmbd_stage_name(int32_t i);

/* How the local MBD stage forms its products with T_LR.  LMBD_MBD_DENSE stores
 * T_LR and runs every product on the matrix cores; LMBD_MBD_SPARSE never stores
 * it and walks only the coupled pairs (for the two-radius regime of Sec. III.A,
 * where block rows other than the central atom's couple only up to r_mbd2);
 * LMBD_MBD_AUTO (the default) takes the sparse form for each structure of a call
 * with r_mbd2 <= 0.45 r_nbr and the dense form for the others (a structure's
 * results do not depend on the batch it is in).  Both forms compute the same
 * quantities (to rounding).  LMBD_E_INVALID_ARG for a NULL context or an
 * unknown mode. */
enum { LMBD_MBD_AUTO = 0, LMBD_MBD_DENSE = 1, LMBD_MBD_SPARSE = 2 };
lmbd_status lmbd_set_mbd_product(lmbd_context* ctx, int32_t mode);

/* Static description of a status code. */
const char* lmbd_status_string(lmbd_status status);

/* Detail of the last error of a context (empty string if none). */
const char* lmbd_last_error(const lmbd_context* ctx);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent structures on one device.
 *
 * A server owns one device memory pool of `memory_budget` bytes and `n_slots`
 * slots; each slot is a host thread with its own lmbd context and HIP stream.
 * Submitted structures wait in a FIFO queue.  A free slot takes the longest
 * prefix of the queue whose exact device footprint (lmbd_estimate_footprint of
 * the batch) fits in one free block of the pool and in the batch caps, carves
 * its whole workspace from that block, and evaluates the prefix as one batch.
 * Requests that arrive while others run are admitted as soon as a slot and
 * pool memory are free, so batches of different slots overlap on the device.
 * Every result is bitwise the one the structure gets when evaluated alone.
 * --------------------------------------------------------------------------- */
typedef struct lmbd_server lmbd_server;

typedef struct lmbd_server_config {
    int32_t device;              /* HIP device index */
    int32_t n_slots;             /* batches in flight at once (1..16) */
    size_t memory_budget;        /* bytes of the device pool; 0 = 80 % of the free device memory */
    int64_t max_batch_atoms;     /* atoms per batch (0 = no cap); a larger request runs alone */
    int32_t max_batch_requests;  /* requests per batch (0 = no cap) */
} lmbd_server_config;

typedef struct lmbd_request_info {
    int32_t done;                /* 1 once the outputs are written (or the request failed) */
    lmbd_status status;          /* result of the request, valid when done */
    double t_submit;             /* seconds since server creation: submission, */
    double t_start;              /*   start of the batch that ran it, */
    double t_end;                /*   outputs written */
    size_t footprint;            /* exact device bytes of the request evaluated alone */
    uint64_t batch;              /* serial number of that batch (from 1) */
    int32_t batch_requests;      /* requests in that batch */
    int32_t slot;                /* slot that ran it */
    char detail[160];            /* error detail when status != LMBD_OK */
} lmbd_request_info;

typedef struct lmbd_server_stats {
    uint64_t submitted, completed, batches;
    int32_t max_concurrent;      /* most batches ever in flight together */
    size_t pool_bytes, pool_peak;
} lmbd_server_stats;

/* Create a server.  params (with its arrays) and the species table are copied;
 * every request of the server uses them.  The pool is allocated here. */
lmbd_status lmbd_server_create(const lmbd_server_config* config, const lmbd_params* params, int32_t n_species,
                               const lmbd_species* species_table, lmbd_server** out);

/* Drop queued requests (status LMBD_E_CANCELLED), wait for running batches,
 * release the pool, the slots and every request record.  NULL is ignored. */
void lmbd_server_destroy(lmbd_server* server);

/* Queue one structure.  Its arrays are HOST arrays owned by the caller, who
 * keeps them alive and leaves them untouched until the request is done.
 * Returns LMBD_E_OOM_ADMISSION (the structure alone needs more than the pool)
 * or LMBD_E_INVALID_ARG without issuing a ticket. */
lmbd_status lmbd_submit(lmbd_server* server, const lmbd_structure* request, uint64_t* ticket);

/* State of a request without blocking (info->done tells whether it finished). */
lmbd_status lmbd_poll(lmbd_server* server, uint64_t ticket, lmbd_request_info* info);

/* Block until the request is done; then as lmbd_poll. */
lmbd_status lmbd_wait(lmbd_server* server, uint64_t ticket, lmbd_request_info* info);

/* Forget a finished request (LMBD_E_INVALID_ARG while it is queued or running). */
lmbd_status lmbd_release(lmbd_server* server, uint64_t ticket);

lmbd_status lmbd_server_get_stats(lmbd_server* server, lmbd_server_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* LMBD_H */
