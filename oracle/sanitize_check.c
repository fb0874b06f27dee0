/*
 * sanitize_check.c -- runs the oracle (cosenu_oracle.c, included as one
 * translation unit) under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * TEST INFRASTRUCTURE ONLY, like the oracle itself: tests/test_oracle_sanitized.py
 * builds it with gcc -fsanitize=address,undefined, feeds it cases written by
 * the test and compares what it writes with the regular (unsanitized) build.
 *
 * Input file (native byte order):
 *   int32 ncases, then per case
 *     int32 nz, nv, scheme, ko_r, quad, steps
 *     double L, dt, mu, omega, theta, lambda, alpha, ko_eps, weno_eps
 *     double g_nu[nv], g_nubar[nv], Y[8 nz nv], stencil[7]
 * Output file, per case:
 *     double rhs(Y)[8 nz nv], moments(Y)[nz 2 4], diagnostics(Y)[12],
 *            Y after `steps` RK4 steps [8 nz nv],
 *            WENO7 parts of the stencil q[4], si[4], w[4], and its flux [1]
 * Every buffer is allocated at its exact size, so an access one element past
 * any of them is reported.
 */
#include <stdio.h>

#include "cosenu_oracle.c"

static void *xread(FILE *f, size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "sanitize_check: short input\n");
        exit(2);
    }
    return p;
}

static void xwrite(FILE *f, const double *p, size_t n) {
    if (fwrite(p, sizeof(double), n, f) != n) {
        fprintf(stderr, "sanitize_check: write failed\n");
        exit(3);
    }
}

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s input output\n", argv[0]);
        return 1;
    }
    FILE *in = fopen(argv[1], "rb"), *out = fopen(argv[2], "wb");
    if (!in || !out) {
        fprintf(stderr, "sanitize_check: cannot open files\n");
        return 1;
    }
    int32_t *nc = xread(in, sizeof(int32_t));
    const int ncases = *nc;
    free(nc);
    for (int c = 0; c < ncases; ++c) {
        int32_t *hi = xread(in, 6 * sizeof(int32_t));
        double *hd = xread(in, 9 * sizeof(double));
        const int nz = hi[0], nv = hi[1];
        const size_t cells = (size_t)nz * nv;
        double *gn = xread(in, nv * sizeof(double));
        double *gb = xread(in, nv * sizeof(double));
        double *y = xread(in, 8 * cells * sizeof(double));
        double *stencil = xread(in, 7 * sizeof(double));
        oracle_params p;
        memset(&p, 0, sizeof p);
        p.nz = nz;
        p.nv = nv;
        p.scheme = hi[2];
        p.ko_r = hi[3];
        p.quad = hi[4];
        p.L = hd[0];
        p.dt = hd[1];
        p.mu = hd[2];
        p.omega = hd[3];
        p.theta = hd[4];
        p.lambda = hd[5];
        p.alpha = hd[6];
        p.ko_eps = hd[7];
        p.weno_eps = hd[8];
        p.g_nu = gn;
        p.g_nubar = gb;

        double *k = malloc(8 * cells * sizeof(double));
        double *mom = malloc(cells / nv * 8 * sizeof(double));
        double *diag = malloc(12 * sizeof(double));
        oracle_rhs(&p, y, k);
        oracle_moments(&p, y, mom);
        oracle_diagnostics(&p, y, diag);
        xwrite(out, k, 8 * cells);
        xwrite(out, mom, (size_t)nz * 8);
        xwrite(out, diag, 12);
        if (oracle_rk4(&p, y, hi[5]) != 0) {
            fprintf(stderr, "sanitize_check: oracle_rk4 failed in case %d\n", c);
            return 4;
        }
        xwrite(out, y, 8 * cells);
        double *q = malloc(4 * sizeof(double)), *si = malloc(4 * sizeof(double)), *w = malloc(4 * sizeof(double));
        oracle_weno7_parts(stencil, p.weno_eps, q, si, w);
        double f = oracle_weno7_minus(stencil, p.weno_eps);
        xwrite(out, q, 4);
        xwrite(out, si, 4);
        xwrite(out, w, 4);
        xwrite(out, &f, 1);
        free(q);
        free(si);
        free(w);
        free(k);
        free(mom);
        free(diag);
        free(stencil);
        free(y);
        free(gb);
        free(gn);
        free(hd);
        free(hi);
    }
    fclose(in);
    if (fclose(out) != 0) return 3;
    printf("sanitize_check: %d cases\n", ncases);
    return 0;
}
