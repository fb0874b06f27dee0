/*
 * cosenu_oracle.c -- plain, slow, FP64 CPU reference solver for the hot path
 * of COSEnu (George, Lin, Wu, Liu, Xiong, arXiv:2203.12866).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header or table with the GPU
 * library: every formula below is written out again from the paper.
 *
 * It is written to be checked against the paper by eye, not to be fast:
 *   - the self-interaction integral is the literal quadrature sum of eq:ham
 *     (Riemann, trapezoid or Simpson weights) for every (z, v) pair, O(Nv)
 *     per cell, for H and for Hbar separately;
 *   - the commutators are 2x2 complex matrix products;
 *   - the Kreiss-Oliger operator is built by composing D+ and D- r times;
 *   - WENO7 follows the steps of Appendix A in order (candidates eq:f4s,
 *     smoothness indicators eq:Si4, weights eq:weight, normalised sum);
 *   - RK4 is the classic tableau, stage by stage.
 * The only parallelism is an OpenMP loop over independent z rows.
 *
 * State layout (shared convention with the caller, not code): 8 real planes
 *   c = 0 rho_ee, 1 rho_xx, 2 Re rho_ex, 3 Im rho_ex,
 *       4 rhobar_ee, 5 rhobar_xx, 6 Re rhobar_ex, 7 Im rhobar_ex,
 * each plane [nz][nv] with v fastest: index = (c*nz + z)*nv + v.
 *
 * Readings of the paper taken here (each is listed in the design notes):
 *   - alpha = n_nubar / n_nu (Sec. 5, ELN definition; the text after eq:ham
 *     states the inverse ratio, which would not produce the ELN crossing).
 *   - velocity bins are midpoints v_j = -1 + (j+1/2) dv and the velocity
 *     integral is the Riemann sum over them (Sec. 3, opening paragraph), for
 *     both schemes.  Sec. 3.1 also describes a vertex grid over [-1, 1] with
 *     the trapezoid rule, and Simpson's rule; both are available as
 *     alternatives (quad = 1, 2), with v_j = -1 + j dv, dv = 2/(nv-1), and
 *     the rule's weights w_j in every velocity integral and sum.
 *   - the angular distributions are normalised discretely: sum_j w_j g_j = 1.
 *   - Kreiss-Oliger: "d_t u -> d_t u + Q u" moves Q to the left-hand side, so
 *     du/dt = (rest) - Q u; this is the dissipative sign (Sec. 3.1).
 *   - WENO7 linear weights: the values listed after eq:f4s are in reversed
 *     order; the set consistent with eq:f7 = sum_r d_r q_r is
 *     d = (4, 18, 12, 1)/35 for r = 0..3 (Appendix A).
 *   - WENO reconstructs the flux f = v u; for v < 0 the same reconstruction is
 *     applied to the sequence mirrored about the interface (Sec. 3.2,
 *     Appendix A "similar procedure").  One flux per interface is shared by
 *     the two cells it separates (eq:cell_av).
 *   - matter term: H_m = diag(lambda, 0) for neutrinos and -diag(lambda, 0)
 *     for antineutrinos (the paper removes it by a frame rotation; footnote
 *     in Sec. 2).
 *   - dt = CFL dz / max_j |v_j| over the discrete velocity grid (Sec. 3).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Parameters.  The caller fills this struct; g_nu / g_nubar are per-bin      */
/* angular distributions (length nv), computed by oracle_angular_dist or      */
/* supplied directly by a test.                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t nz, nv;
    double L;        /* domain length, z in [-L/2, L/2), periodic            */
    double dt;       /* time step                                            */
    double mu;       /* self-interaction strength                            */
    double omega;    /* vacuum oscillation frequency                         */
    double theta;    /* vacuum mixing angle (radians)                        */
    double lambda;   /* matter potential                                     */
    double alpha;    /* n_nubar / n_nu                                       */
    int32_t scheme;  /* 0: FD4 + Kreiss-Oliger, 1: FV + WENO7                */
    int32_t ko_r;    /* Kreiss-Oliger order parameter r (paper uses 2)       */
    double ko_eps;   /* Kreiss-Oliger strength (paper uses 0.1)              */
    double weno_eps; /* WENO regulator (paper: about 1e-6)                   */
    const double *g_nu;
    const double *g_nubar;
    int32_t quad;    /* velocity grid and rule: 0 midpoint bins + Riemann sum,
                        1 vertex grid + trapezoid, 2 vertex grid + Simpson */
} oracle_params;

/* ------------------------------------------------------------------------ */
/* Complex numbers and 2x2 complex matrices.                                  */
/* ------------------------------------------------------------------------ */
typedef struct { double re, im; } cx;
typedef struct { cx a[2][2]; } mat2;

static cx cx_make(double re, double im) { cx r; r.re = re; r.im = im; return r; }
static cx cx_add(cx x, cx y) { return cx_make(x.re + y.re, x.im + y.im); }
static cx cx_sub(cx x, cx y) { return cx_make(x.re - y.re, x.im - y.im); }
static cx cx_mul(cx x, cx y) { return cx_make(x.re * y.re - x.im * y.im, x.re * y.im + x.im * y.re); }
static cx cx_scale(cx x, double s) { return cx_make(x.re * s, x.im * s); }
static cx cx_conj(cx x) { return cx_make(x.re, -x.im); }

static mat2 mat_zero(void) { mat2 m; memset(&m, 0, sizeof m); return m; }
static mat2 mat_add(mat2 x, mat2 y) {
    mat2 r; for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) r.a[i][j] = cx_add(x.a[i][j], y.a[i][j]); return r;
}
static mat2 mat_sub(mat2 x, mat2 y) {
    mat2 r; for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) r.a[i][j] = cx_sub(x.a[i][j], y.a[i][j]); return r;
}
static mat2 mat_scale(mat2 x, double s) {
    mat2 r; for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) r.a[i][j] = cx_scale(x.a[i][j], s); return r;
}
/* element-wise complex conjugate (rho^* in eq:ham, not the adjoint) */
static mat2 mat_conj(mat2 x) {
    mat2 r; for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) r.a[i][j] = cx_conj(x.a[i][j]); return r;
}
static mat2 mat_mul(mat2 x, mat2 y) {
    mat2 r;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            r.a[i][j] = cx_add(cx_mul(x.a[i][0], y.a[0][j]), cx_mul(x.a[i][1], y.a[1][j]));
    return r;
}
/* -i [H, R]: the right-hand side of eq:eom */
static mat2 minus_i_commutator(mat2 H, mat2 R) {
    mat2 c = mat_sub(mat_mul(H, R), mat_mul(R, H));
    mat2 r;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            r.a[i][j] = cx_make(c.a[i][j].im, -c.a[i][j].re); /* (-i)(x + iy) = y - ix */
    return r;
}

/* Density matrix of eq:rho from the 8 real planes.  base = 0 for rho, 4 for rhobar. */
static mat2 density_matrix(const double *Y, int base, int nz, int nv, int z, int v) {
    size_t plane = (size_t)nz * nv, at = (size_t)z * nv + v;
    double ee = Y[(base + 0) * plane + at];
    double xx = Y[(base + 1) * plane + at];
    double re = Y[(base + 2) * plane + at];
    double im = Y[(base + 3) * plane + at];
    mat2 m;
    m.a[0][0] = cx_make(ee, 0.0);
    m.a[0][1] = cx_make(re, im);
    m.a[1][0] = cx_make(re, -im);
    m.a[1][1] = cx_make(xx, 0.0);
    return m;
}

/* ------------------------------------------------------------------------ */
/* Grid (Sec. 3, opening paragraph).                                          */
/* ------------------------------------------------------------------------ */
double oracle_velocity_q(int32_t nv, int32_t quad, int32_t j) {
    if (quad == 0) {
        double dv = 2.0 / nv;
        return -1.0 + (j + 0.5) * dv; /* each bin is represented by its midpoint */
    }
    double dv = 2.0 / (nv - 1);       /* vertex grid: v_0 = -1, v_{nv-1} = +1 */
    return -1.0 + j * dv;
}

double oracle_velocity(int32_t nv, int32_t j) { return oracle_velocity_q(nv, 0, j); }

/* Quadrature weight of point j: the Riemann sum (dv), the composite trapezoid
 * rule (dv, halved at both ends) or the composite Simpson rule (dv/3 times
 * 1, 4, 2, 4, ..., 2, 4, 1; nv odd). */
double oracle_vweight(int32_t nv, int32_t quad, int32_t j) {
    if (quad == 0) return 2.0 / nv;
    double dv = 2.0 / (nv - 1);
    int end = (j == 0 || j == nv - 1);
    if (quad == 1) return end ? 0.5 * dv : dv;
    if (end) return dv / 3.0;
    return (j % 2 == 1) ? 4.0 * dv / 3.0 : 2.0 * dv / 3.0;
}

double oracle_position(int32_t nz, double L, int32_t i) {
    double dz = L / nz;
    return -0.5 * L + (i + 0.5) * dz;
}

/* dt = C_CFL dz / max |v_z|, the maximum taken over the discrete grid. */
double oracle_dt_q(int32_t nz, int32_t nv, int32_t quad, double L, double cfl) {
    double vmax = 0.0;
    for (int j = 0; j < nv; ++j) {
        double a = fabs(oracle_velocity_q(nv, quad, j));
        if (a > vmax) vmax = a;
    }
    return cfl * (L / nz) / vmax;
}

double oracle_dt(int32_t nz, int32_t nv, double L, double cfl) { return oracle_dt_q(nz, nv, 0, L, cfl); }

/* g(v) proportional to exp(-(v-1)^2 / (2 sigma^2)), normalised so that the
 * quadrature over the grid is one (Sec. 5, the Gaussian angular family). */
void oracle_angular_dist_q(int32_t nv, int32_t quad, double sigma, double *g) {
    double norm = 0.0;
    for (int j = 0; j < nv; ++j) {
        double v = oracle_velocity_q(nv, quad, j);
        g[j] = exp(-(v - 1.0) * (v - 1.0) / (2.0 * sigma * sigma));
        norm += oracle_vweight(nv, quad, j) * g[j];
    }
    for (int j = 0; j < nv; ++j) g[j] /= norm;
}

void oracle_angular_dist(int32_t nv, double sigma, double *g) { oracle_angular_dist_q(nv, 0, sigma, g); }

/* Initial data of eqs:perts: a pure flavour state perturbed by eps(z) =
 * amp exp(-z^2/width), identical in every velocity bin.  The off-diagonal
 * carries a global phase phi for rho and -phi for rhobar (phi = 0 is the
 * paper's data). */
void oracle_initial_state(int32_t nz, int32_t nv, double L, double amp, double width,
                          double phi, double *Y) {
    size_t plane = (size_t)nz * nv;
    for (int i = 0; i < nz; ++i) {
        double z = oracle_position(nz, L, i);
        double e = amp * exp(-z * z / width);
        double root = sqrt(1.0 - e * e);
        double ee = 0.5 * (1.0 + root), xx = 0.5 * (1.0 - root);
        for (int j = 0; j < nv; ++j) {
            size_t at = (size_t)i * nv + j;
            Y[0 * plane + at] = ee;
            Y[1 * plane + at] = xx;
            Y[2 * plane + at] = 0.5 * e * cos(phi);
            Y[3 * plane + at] = 0.5 * e * sin(phi);
            Y[4 * plane + at] = ee;
            Y[5 * plane + at] = xx;
            Y[6 * plane + at] = 0.5 * e * cos(phi);
            Y[7 * plane + at] = -0.5 * e * sin(phi);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* WENO7 reconstruction at the interface i+1/2 from the upwind-oriented      */
/* values a[0..6] = f_{i-3} .. f_{i+3}  (Appendix A).                         */
/* ------------------------------------------------------------------------ */
/* The intermediate quantities of the reconstruction, step by step:
 * candidates q_r (eq:f4s), smoothness indicators SI_r (eq:Si4) and the
 * un-normalised weights w_r = d_r / (SI_r + eps)^2 (eq:weight). */
void oracle_weno7_parts(const double *a, double eps, double *q, double *si, double *w) {
    const double fm3 = a[0], fm2 = a[1], fm1 = a[2], f0 = a[3], fp1 = a[4], fp2 = a[5], fp3 = a[6];
    /* fourth-order candidates on the sub-stencils S_0..S_3 (eq:f4s) */
    q[0] = (3.0 * f0 + 13.0 * fp1 - 5.0 * fp2 + 1.0 * fp3) / 12.0;
    q[1] = (-1.0 * fm1 + 7.0 * f0 + 7.0 * fp1 - 1.0 * fp2) / 12.0;
    q[2] = (1.0 * fm2 - 5.0 * fm1 + 13.0 * f0 + 3.0 * fp1) / 12.0;
    q[3] = (-3.0 * fm3 + 13.0 * fm2 - 23.0 * fm1 + 25.0 * f0) / 12.0;
    /* smoothness indicators (eq:Si4) */
    si[0] = f0 * (2107.0 * f0 - 9402.0 * fp1 + 7042.0 * fp2 - 1854.0 * fp3)
          + fp1 * (11003.0 * fp1 - 17246.0 * fp2 + 4642.0 * fp3)
          + fp2 * (7043.0 * fp2 - 3882.0 * fp3)
          + 547.0 * fp3 * fp3;
    si[1] = fm1 * (547.0 * fm1 - 2522.0 * f0 + 1922.0 * fp1 - 494.0 * fp2)
          + f0 * (3443.0 * f0 - 5966.0 * fp1 + 1602.0 * fp2)
          + fp1 * (2843.0 * fp1 - 1642.0 * fp2)
          + 267.0 * fp2 * fp2;
    si[2] = fm2 * (267.0 * fm2 - 1642.0 * fm1 + 1602.0 * f0 - 494.0 * fp1)
          + fm1 * (2843.0 * fm1 - 5966.0 * f0 + 1922.0 * fp1)
          + f0 * (3443.0 * f0 - 2522.0 * fp1)
          + 547.0 * fp1 * fp1;
    si[3] = fm3 * (547.0 * fm3 - 3882.0 * fm2 + 4642.0 * fm1 - 1854.0 * f0)
          + fm2 * (7043.0 * fm2 - 17246.0 * fm1 + 7042.0 * f0)
          + fm1 * (11003.0 * fm1 - 9402.0 * f0)
          + 2107.0 * f0 * f0;
    /* linear weights consistent with eq:f7 (see the header) */
    const double d[4] = {4.0 / 35.0, 18.0 / 35.0, 12.0 / 35.0, 1.0 / 35.0};
    for (int r = 0; r < 4; ++r) w[r] = d[r] / ((si[r] + eps) * (si[r] + eps)); /* eq:weight */
}

double oracle_weno7_minus(const double *a, double eps) {
    double q[4], si[4], w[4];
    oracle_weno7_parts(a, eps, q, si, w);
    double wsum = 0.0;
    for (int r = 0; r < 4; ++r) wsum += w[r];
    double f = 0.0;
    for (int r = 0; r < 4; ++r) f += (w[r] / wsum) * q[r]; /* eq:fn_w_lin_comb */
    return f;
}

/* ------------------------------------------------------------------------ */
/* Advection operators on one periodic line u[0..nz-1] (stride 'stride').     */
/* ------------------------------------------------------------------------ */
static int wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

/* Coefficients of (D+)^r (D-)^r times h^(2r) as a stencil over offsets
 * -r..r, obtained by composing the one-sided differences literally:
 * D- u_0 = (u_0 - u_{-1})/h,  D+ u_0 = (u_{+1} - u_0)/h  (Sec. 3.1). */
static void ko_stencil(int r, double *c /* length 2r+1, c[k+r] = coeff of u_k */) {
    int n = 2 * r + 1;
    double tmp[64];
    for (int k = 0; k < n; ++k) c[k] = 0.0;
    c[r] = 1.0; /* identity */
    for (int s = 0; s < r; ++s) { /* apply D-: (D- w)_k = w_k - w_{k-1} as operators on shifts */
        for (int k = 0; k < n; ++k) tmp[k] = 0.0;
        for (int k = 0; k < n; ++k) {
            if (c[k] == 0.0) continue;
            tmp[k] += c[k];                 /* E^k u   -> E^k u         */
            if (k - 1 >= 0) tmp[k - 1] -= c[k]; /* E^k u   -> -E^(k-1) u  */
        }
        for (int k = 0; k < n; ++k) c[k] = tmp[k];
    }
    for (int s = 0; s < r; ++s) { /* apply D+: (D+ w) -> E^(k+1) - E^k */
        for (int k = 0; k < n; ++k) tmp[k] = 0.0;
        for (int k = 0; k < n; ++k) {
            if (c[k] == 0.0) continue;
            if (k + 1 < n) tmp[k + 1] += c[k];
            tmp[k] -= c[k];
        }
        for (int k = 0; k < n; ++k) c[k] = tmp[k];
    }
}

/* d u_i / dt contribution of FD4 advection plus Kreiss-Oliger dissipation:
 *   -v (u_{i-2} - 8 u_{i-1} + 8 u_{i+1} - u_{i+2}) / (12 dz)     (4th-order central)
 *   - Q u_i,  Q = eps (-1)^r h^(2r-1) (D+)^r (D-)^r / 2^(2r)      (Sec. 3.1)      */
static void fd_ko_line(const double *u, double *out, int nz, size_t stride, double v,
                       double dz, double ko_eps, int ko_r) {
    double c[64];
    ko_stencil(ko_r, c);
    double sign = (ko_r % 2 == 0) ? 1.0 : -1.0;
    double scale = ko_eps * sign * pow(dz, 2 * ko_r - 1) / pow(2.0, 2 * ko_r) / pow(dz, 2 * ko_r);
    for (int i = 0; i < nz; ++i) {
        double um2 = u[(size_t)wrap(i - 2, nz) * stride];
        double um1 = u[(size_t)wrap(i - 1, nz) * stride];
        double up1 = u[(size_t)wrap(i + 1, nz) * stride];
        double up2 = u[(size_t)wrap(i + 2, nz) * stride];
        double adv = -v * (um2 - 8.0 * um1 + 8.0 * up1 - up2) / (12.0 * dz);
        double qu = 0.0;
        if (ko_eps != 0.0) {
            double s = 0.0;
            for (int k = -ko_r; k <= ko_r; ++k) s += c[k + ko_r] * u[(size_t)wrap(i + k, nz) * stride];
            qu = scale * s;
        }
        out[(size_t)i * stride] += adv - qu;
    }
}

/* d u_i / dt contribution of the finite-volume update eq:cell_av with WENO7
 * interface fluxes of f = v u.  F[i] holds the flux at i+1/2. */
static void fv_weno7_line(const double *u, double *out, int nz, size_t stride, double v,
                          double dz, double eps, double *F) {
    for (int i = 0; i < nz; ++i) {
        double a[7];
        for (int m = -3; m <= 3; ++m) {
            /* upwind side: for v > 0 the stencil centred on cell i, for v <= 0
             * the mirror image about the interface, centred on cell i+1 */
            int k = (v > 0.0) ? i + m : i + 1 - m;
            a[m + 3] = v * u[(size_t)wrap(k, nz) * stride];
        }
        F[i] = oracle_weno7_minus(a, eps);
    }
    for (int i = 0; i < nz; ++i) out[(size_t)i * stride] += -(F[i] - F[wrap(i - 1, nz)]) / dz;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side of eq:eom for the whole state.                            */
/* ------------------------------------------------------------------------ */
void oracle_rhs(const oracle_params *p, const double *Y, double *K) {
    const int nz = p->nz, nv = p->nv;
    const size_t plane = (size_t)nz * nv;
    const double dz = p->L / nz;

    /* H_vac = (omega/2) [[-cos 2theta, sin 2theta], [sin 2theta, cos 2theta]], same for nubar */
    mat2 Hvac = mat_zero();
    Hvac.a[0][0] = cx_make(-0.5 * p->omega * cos(2.0 * p->theta), 0.0);
    Hvac.a[0][1] = cx_make(0.5 * p->omega * sin(2.0 * p->theta), 0.0);
    Hvac.a[1][0] = cx_make(0.5 * p->omega * sin(2.0 * p->theta), 0.0);
    Hvac.a[1][1] = cx_make(0.5 * p->omega * cos(2.0 * p->theta), 0.0);
    /* matter: +diag(lambda, 0) for neutrinos, -diag(lambda, 0) for antineutrinos */
    mat2 Hm = mat_zero();
    Hm.a[0][0] = cx_make(p->lambda, 0.0);

    /* commutator part, row by row */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        for (int j = 0; j < nv; ++j) {
            double vj = oracle_velocity_q(nv, p->quad, j);
            /* velocity integrals of eq:ham with rho -> g rho, rhobar -> gbar rhobar (Sec. 5) */
            mat2 S = mat_zero(), Sb = mat_zero();
            for (int l = 0; l < nv; ++l) {
                double vl = oracle_velocity_q(nv, p->quad, l);
                double w = oracle_vweight(nv, p->quad, l) * (1.0 - vj * vl);
                mat2 r = density_matrix(Y, 0, nz, nv, z, l);
                mat2 rb = density_matrix(Y, 4, nz, nv, z, l);
                mat2 term = mat_sub(mat_scale(r, p->g_nu[l]), mat_scale(mat_conj(rb), p->alpha * p->g_nubar[l]));
                mat2 termb = mat_sub(mat_scale(mat_conj(r), p->g_nu[l]), mat_scale(rb, p->alpha * p->g_nubar[l]));
                S = mat_add(S, mat_scale(term, w));
                Sb = mat_add(Sb, mat_scale(termb, w));
            }
            mat2 H = mat_add(mat_add(Hvac, Hm), mat_scale(S, p->mu));
            mat2 Hb = mat_sub(mat_sub(Hvac, Hm), mat_scale(Sb, p->mu));
            mat2 C = minus_i_commutator(H, density_matrix(Y, 0, nz, nv, z, j));
            mat2 Cb = minus_i_commutator(Hb, density_matrix(Y, 4, nz, nv, z, j));
            size_t at = (size_t)z * nv + j;
            K[0 * plane + at] = C.a[0][0].re;
            K[1 * plane + at] = C.a[1][1].re;
            K[2 * plane + at] = C.a[0][1].re;
            K[3 * plane + at] = C.a[0][1].im;
            K[4 * plane + at] = Cb.a[0][0].re;
            K[5 * plane + at] = Cb.a[1][1].re;
            K[6 * plane + at] = Cb.a[0][1].re;
            K[7 * plane + at] = Cb.a[0][1].im;
        }
    }

    /* advection part: (d/dt + v d/dz) u = ..., one periodic line per (component, v) */
#pragma omp parallel
    {
        double *F = (double *)malloc(sizeof(double) * (size_t)nz);
#pragma omp for collapse(2) schedule(static)
        for (int c = 0; c < 8; ++c) {
            for (int j = 0; j < nv; ++j) {
                double vj = oracle_velocity_q(nv, p->quad, j);
                const double *u = Y + c * plane + j;
                double *out = K + c * plane + j;
                if (p->scheme == 0)
                    fd_ko_line(u, out, nz, (size_t)nv, vj, dz, p->ko_eps, p->ko_r);
                else
                    fv_weno7_line(u, out, nz, (size_t)nv, vj, dz, p->weno_eps, F);
            }
        }
        free(F);
    }
}

/* ------------------------------------------------------------------------ */
/* Classic fourth-order Runge-Kutta (method of lines, Sec. 3.1).              */
/* ------------------------------------------------------------------------ */
int oracle_rk4(const oracle_params *p, double *y, int64_t nsteps) {
    const size_t n = (size_t)8 * p->nz * p->nv;
    double *k1 = malloc(n * sizeof(double)), *k2 = malloc(n * sizeof(double));
    double *k3 = malloc(n * sizeof(double)), *k4 = malloc(n * sizeof(double));
    double *Ys = malloc(n * sizeof(double));
    if (!k1 || !k2 || !k3 || !k4 || !Ys) {
        free(k1); free(k2); free(k3); free(k4); free(Ys);
        return -1;
    }
    const double dt = p->dt;
    for (int64_t s = 0; s < nsteps; ++s) {
        oracle_rhs(p, y, k1);
        for (size_t i = 0; i < n; ++i) Ys[i] = y[i] + 0.5 * dt * k1[i];
        oracle_rhs(p, Ys, k2);
        for (size_t i = 0; i < n; ++i) Ys[i] = y[i] + 0.5 * dt * k2[i];
        oracle_rhs(p, Ys, k3);
        for (size_t i = 0; i < n; ++i) Ys[i] = y[i] + dt * k3[i];
        oracle_rhs(p, Ys, k4);
        for (size_t i = 0; i < n; ++i) y[i] = y[i] + dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    free(k1); free(k2); free(k3); free(k4); free(Ys);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Angular moments of D = g rho - alpha gbar rhobar^* per z row:              */
/*   out[(z*2 + m)*4 + q],  m = 0: sum_j w_j D_j,  m = 1: sum_j w_j v_j D_j,  */
/*   q = 0 D_ee, 1 D_xx, 2 Re D_ex, 3 Im D_ex.                                */
/* ------------------------------------------------------------------------ */
void oracle_moments(const oracle_params *p, const double *Y, double *out) {
    const int nz = p->nz, nv = p->nv;
    for (int z = 0; z < nz; ++z) {
        double m[2][4] = {{0}};
        for (int j = 0; j < nv; ++j) {
            double vj = oracle_velocity_q(nv, p->quad, j);
            double dv = oracle_vweight(nv, p->quad, j);
            mat2 r = density_matrix(Y, 0, nz, nv, z, j);
            mat2 rb = density_matrix(Y, 4, nz, nv, z, j);
            mat2 D = mat_sub(mat_scale(r, p->g_nu[j]), mat_scale(mat_conj(rb), p->alpha * p->g_nubar[j]));
            double q[4] = {D.a[0][0].re, D.a[1][1].re, D.a[0][1].re, D.a[0][1].im};
            for (int k = 0; k < 4; ++k) {
                m[0][k] += dv * q[k];
                m[1][k] += dv * vj * q[k];
            }
        }
        for (int k = 0; k < 4; ++k) {
            out[(z * 2 + 0) * 4 + k] = m[0][k];
            out[(z * 2 + 1) * 4 + k] = m[1][k];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Conserved quantities and error measures (Sec. 5).                         */
/* Polarisation vector: rho = (P0 + P . sigma)/2, so P = (2 Re rho_ex,        */
/* -2 Im rho_ex, rho_ee - rho_xx).  For the antineutrino the matrix entering  */
/* D is rhobar^*, whose vector is (2 Re rhob_ex, +2 Im rhob_ex, ...).         */
/* (w_j is the quadrature weight: dv for the midpoint bins)                   */
/* out[0..3]  M0 = dz sum w (g P - alpha gbar Pbar*) as (trace, x, y, z)      */
/* out[4]     N_nu    = dz sum w g Tr rho                                     */
/* out[5]     N_nubar = dz sum w gbar Tr rhobar                               */
/* out[6]     dP_max  = max over cells and species of | |P| - 1 |             */
/* out[7]     <dP>    = sum w g | |P_nu| - 1 | / sum w g                      */
/* out[8]     dz sum w g rho_ee        out[9]  dz sum w gbar rhobar_ee        */
/* out[10]    B.M0 with B = (sin 2theta, 0, -cos 2theta)                      */
/* out[11]    number of non-finite values in the state                        */
/* ------------------------------------------------------------------------ */
void oracle_diagnostics(const oracle_params *p, const double *Y, double *out) {
    const int nz = p->nz, nv = p->nv;
    const size_t plane = (size_t)nz * nv;
    const double dz = p->L / nz;
    double M[4] = {0, 0, 0, 0}, Nn = 0, Nb = 0, dpmax = 0, dpw = 0, gw = 0, een = 0, eeb = 0, bad = 0;
    for (int z = 0; z < nz; ++z) {
        for (int j = 0; j < nv; ++j) {
            const double wj = oracle_vweight(nv, p->quad, j), cell = dz * wj;
            size_t at = (size_t)z * nv + j;
            double y[8];
            for (int c = 0; c < 8; ++c) {
                y[c] = Y[c * plane + at];
                if (!isfinite(y[c])) bad += 1.0;
            }
            double g = p->g_nu[j], gb = p->g_nubar[j];
            double P0 = y[0] + y[1], P1 = 2.0 * y[2], P2 = -2.0 * y[3], P3 = y[0] - y[1];
            double Q0 = y[4] + y[5], Q1 = 2.0 * y[6], Q2 = 2.0 * y[7], Q3 = y[4] - y[5];
            M[0] += cell * (g * P0 - p->alpha * gb * Q0);
            M[1] += cell * (g * P1 - p->alpha * gb * Q1);
            M[2] += cell * (g * P2 - p->alpha * gb * Q2);
            M[3] += cell * (g * P3 - p->alpha * gb * Q3);
            Nn += cell * g * P0;
            Nb += cell * gb * Q0;
            double dpn = fabs(sqrt(P1 * P1 + P2 * P2 + P3 * P3) - 1.0);
            double dpb = fabs(sqrt(Q1 * Q1 + Q2 * Q2 + Q3 * Q3) - 1.0);
            if (dpn > dpmax) dpmax = dpn;
            if (dpb > dpmax) dpmax = dpb;
            dpw += wj * g * dpn;
            gw += wj * g;
            een += cell * g * y[0];
            eeb += cell * gb * y[4];
        }
    }
    out[0] = M[0]; out[1] = M[1]; out[2] = M[2]; out[3] = M[3];
    out[4] = Nn; out[5] = Nb;
    out[6] = dpmax; out[7] = dpw / gw;
    out[8] = een; out[9] = eeb;
    out[10] = sin(2.0 * p->theta) * M[1] - cos(2.0 * p->theta) * M[3];
    out[11] = bad;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the OpenMP thread count of later calls (n >= 1); returns the count now in force. */
int oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
