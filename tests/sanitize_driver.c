/* Host-side exercise of the C ABI for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host code (no GPU needed): argument checks,
 * status and stage strings, and the footprint estimate, which runs the host
 * neighbour counting, form choice and workspace layout of a call on every
 * structure of the input file, alone and as one batch.
 *
 * Input file (little-endian): int32 n_structs, then per structure int32 n,
 * int32 pbc[3], double cell[9], double radii[6] (r_scs, r_nbr, r_mbd1, r_mbd2,
 * r_2b1, r_2b2), double pos[3n], int32 species[n], double nu[n].
 * Prints one line per estimate; exit status 0 when every check holds. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lmbd.h"

static int fail(const char* what) {
    fprintf(stderr, "check failed: %s\n", what);
    return 1;
}

int main(int argc, char** argv) {
    if (argc < 2) return fail("usage: sanitize_driver <structures file>");
    FILE* fh = fopen(argv[1], "rb");
    if (!fh) return fail("open input");
    int32_t ns = 0;
    if (fread(&ns, 4, 1, fh) != 1 || ns < 1 || ns > 64) return fail("header");
    lmbd_structure* st = calloc((size_t)ns, sizeof(lmbd_structure));
    double* cells = calloc((size_t)ns * 9, sizeof(double));
    for (int s = 0; s < ns; ++s) {
        int32_t n = 0, pbc[3];
        double radii[6];
        if (fread(&n, 4, 1, fh) != 1 || n < 1 || fread(pbc, 4, 3, fh) != 3 || fread(cells + 9 * s, 8, 9, fh) != 9 ||
            fread(radii, 8, 6, fh) != 6)
            return fail("structure header");
        double* pos = malloc(sizeof(double) * 3 * (size_t)n);
        int32_t* sp = malloc(sizeof(int32_t) * (size_t)n);
        double* nu = malloc(sizeof(double) * (size_t)n);
        if (fread(pos, 8, 3 * (size_t)n, fh) != 3 * (size_t)n || fread(sp, 4, (size_t)n, fh) != (size_t)n ||
            fread(nu, 8, (size_t)n, fh) != (size_t)n)
            return fail("structure arrays");
        st[s].n_atoms = n;
        st[s].pos = pos;
        st[s].species = sp;
        st[s].v_ratio = nu;
        st[s].cell = (pbc[0] || pbc[1] || pbc[2]) ? cells + 9 * s : NULL;
        memcpy(st[s].pbc, pbc, sizeof(pbc));
        st[s].r_scs = radii[0];
        st[s].r_nbr = radii[1];
        st[s].r_mbd1 = radii[2];
        st[s].r_mbd2 = radii[3];
        st[s].r_2b1 = radii[4];
        st[s].r_2b2 = radii[5];
        st[s].forces = (double*)8;   /* only its being non-NULL is read by the estimate */
    }
    fclose(fh);

    int bad = 0;
    if (lmbd_abi_version() != LMBD_ABI_VERSION) bad |= fail("abi version");
    for (int c = 0; c <= 9; ++c)
        if (!lmbd_status_string((lmbd_status)c)) bad |= fail("status string");
    for (int i = 0; i < LMBD_N_STAGES; ++i)
        if (!lmbd_stage_name(i)) bad |= fail("stage name");
    if (lmbd_stage_name(LMBD_N_STAGES) != NULL || lmbd_stage_name(-1) != NULL) bad |= fail("stage name range");
    if (lmbd_create(0, NULL) != LMBD_E_INVALID_ARG) bad |= fail("create NULL");
    if (lmbd_compute_batch(NULL, NULL, 0, NULL, 0, NULL, 0, NULL) != LMBD_E_INVALID_ARG) bad |= fail("compute NULL");
    lmbd_destroy(NULL);

    double omega[12], weight[12];
    for (int q = 0; q < 12; ++q) {
        omega[q] = 0.05 * (q + 1);
        weight[q] = 0.1;
    }
    lmbd_params p;
    memset(&p, 0, sizeof(p));
    p.beta = 0.83;
    p.damp_d = 6.0;
    p.r_buf = 0.5;
    p.r_inner = 2.0;
    p.n_max = 6;
    p.n_freq = 12;
    p.omega = omega;
    p.weight = weight;
    for (int s = 0; s < ns; ++s) {
        size_t bytes = 0;
        const lmbd_status r = lmbd_estimate_footprint(&p, 1, st + s, &bytes);
        printf("structure %d: %lld atoms, status %d, %zu bytes\n", s, (long long)st[s].n_atoms, (int)r, bytes);
        if (r != LMBD_OK || bytes == 0) bad |= fail("estimate of one structure");
    }
    size_t all = 0;
    if (lmbd_estimate_footprint(&p, ns, st, &all) != LMBD_OK || all == 0) bad |= fail("estimate of the batch");
    printf("batch: %zu bytes\n", all);
    p.precision = LMBD_MIXED;
    p.cn_mode = LMBD_CN_FIT;
    size_t mixed = 0;
    if (lmbd_estimate_footprint(&p, ns, st, &mixed) != LMBD_OK || !(mixed < all)) bad |= fail("mixed estimate");
    printf("batch, mixed: %zu bytes\n", mixed);
    /* argument errors found by the host checks */
    lmbd_structure e = st[0];
    e.r_mbd2 = e.r_mbd1 + 1.0;
    size_t b = 0;
    if (lmbd_estimate_footprint(&p, 1, &e, &b) != LMBD_E_INVALID_ARG) bad |= fail("radii order");
    e = st[0];
    e.r_2b1 = e.r_nbr + 1.0;
    if (lmbd_estimate_footprint(&p, 1, &e, &b) != LMBD_E_INVALID_ARG) bad |= fail("two-body radius");
    e = st[0];
    double* pos = malloc(sizeof(double) * 3 * (size_t)e.n_atoms);
    memcpy(pos, e.pos, sizeof(double) * 3 * (size_t)e.n_atoms);
    pos[4] = 0.0 / 0.0;
    e.pos = pos;
    if (lmbd_estimate_footprint(&p, 1, &e, &b) != LMBD_E_INVALID_ARG) bad |= fail("non-finite position");
    free(pos);
    p.n_max = 99;
    if (lmbd_estimate_footprint(&p, 1, st, &b) != LMBD_E_INVALID_ARG) bad |= fail("n_max range");
    for (int s = 0; s < ns; ++s) {
        free((void*)st[s].pos);
        free((void*)st[s].species);
        free((void*)st[s].v_ratio);
    }
    free(st);
    free(cells);
    printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
