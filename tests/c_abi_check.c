/*
 * A C caller of include/cosenu.h with no Python or torch in the process:
 * creates a simulation and a two-instance batch from the default parameters
 * with a few changes, steps them, and writes the states and a few facts to
 * files the test reads back.  Test infrastructure.
 *
 * usage: c_abi_check OUT_PREFIX
 *   OUT_PREFIX.sim.bin    [8][96][128] FP64 state after 10 steps
 *   OUT_PREFIX.batch.bin  the two batch instances after 7 steps, one after the other
 *   OUT_PREFIX.txt        key = value lines
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "cosenu.h"

static int fail(const char *what, int rc, const char *detail) {
    fprintf(stderr, "%s: %s (%d) %s\n", what, cosenu_strerror(rc), rc, detail ? detail : "");
    return 1;
}

static int write_doubles(const char *path, const double *x, size_t n, const char *mode) {
    FILE *f = fopen(path, mode);
    if (!f) return 1;
    size_t w = fwrite(x, sizeof(double), n, f);
    fclose(f);
    return w == n ? 0 : 1;
}

int main(int argc, char **argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s OUT_PREFIX\n", argv[0]);
        return 2;
    }
    char path[4096];
    cosenu_params p;
    int rc = cosenu_params_default(&p);
    if (rc) return fail("cosenu_params_default", rc, NULL);
    p.nz = 96;
    p.nv = 128;
    p.L = 75.0;
    p.omega = 0.1;
    p.lambda = 0.2;
    p.pert_amp = 0.3;
    p.precision = COSENU_FP64;

    cosenu_sim *s = NULL;
    rc = cosenu_create(&p, &s);
    if (rc) return fail("cosenu_create", rc, NULL);
    rc = cosenu_step(s, 10);
    if (!rc) rc = cosenu_sync(s);
    if (rc) return fail("cosenu_step", rc, cosenu_last_error(s));
    const size_t n = (size_t)8 * p.nz * p.nv;
    double *y = (double *)malloc(n * sizeof(double));
    if (!y) return 1;
    rc = cosenu_get_state(s, y, n);
    if (rc) return fail("cosenu_get_state", rc, cosenu_last_error(s));
    snprintf(path, sizeof path, "%s.sim.bin", argv[1]);
    if (write_doubles(path, y, n, "wb")) return fail("write", 0, path);
    cosenu_conserved_t c;
    rc = cosenu_conserved(s, &c);
    if (rc) return fail("cosenu_conserved", rc, cosenu_last_error(s));
    cosenu_info_t info;
    rc = cosenu_info(s, &info);
    if (rc) return fail("cosenu_info", rc, cosenu_last_error(s));
    snprintf(path, sizeof path, "%s.txt", argv[1]);
    FILE *f = fopen(path, "w");
    if (!f) return fail("write", 0, path);
    fprintf(f, "step = %lld\nt = %.17g\ndt = %.17g\nlaunches_per_step = %d\nN_nu = %.17g\nnonfinite = %lld\n",
            (long long)c.step, c.t, info.dt, info.launches_per_step, c.N_nu, (long long)c.nonfinite);
    cosenu_destroy(s);

    /* a batch: the same instance and a WENO7 one with Simpson's rule */
    cosenu_params q[2] = {p, p};
    q[1].scheme = COSENU_FV_WENO7;
    q[1].nz = 64;
    q[1].nv = 33;
    q[1].quadrature = COSENU_QUAD_SIMPSON;
    cosenu_batch *b = NULL;
    rc = cosenu_batch_create(q, 2, &b);
    if (rc) return fail("cosenu_batch_create", rc, NULL);
    rc = cosenu_batch_step(b, 7);
    if (!rc) rc = cosenu_batch_sync(b);
    if (rc) return fail("cosenu_batch_step", rc, cosenu_batch_last_error(b));
    snprintf(path, sizeof path, "%s.batch.bin", argv[1]);
    for (int i = 0; i < 2; ++i) {
        const size_t m = (size_t)8 * q[i].nz * q[i].nv;
        double *x = (double *)malloc(m * sizeof(double));
        if (!x) return 1;
        rc = cosenu_batch_get_state(b, i, x, m);
        if (rc) return fail("cosenu_batch_get_state", rc, cosenu_batch_last_error(b));
        if (write_doubles(path, x, m, i == 0 ? "wb" : "ab")) return fail("write", 0, path);
        free(x);
    }
    cosenu_batch_destroy(b);
    fprintf(f, "batch = ok\n");
    fclose(f);
    free(y);
    return 0;
}
