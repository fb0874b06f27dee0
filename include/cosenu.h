/*
 * cosenu.h -- C ABI of the MI355X (gfx950) hot path of the COSEnu
 * collective-oscillation solver (George, Lin, Wu, Liu, Xiong,
 * arXiv:2203.12866).
 *
 * The library advances the two-flavour quantum kinetic equations of Sec. 2
 * (eq:eom),
 *     (d/dt + v d/dz) rho    = -i [H,    rho   ],
 *     (d/dt + v d/dz) rhobar = -i [Hbar, rhobar],
 * with H = H_vac + H_m + H_nunu and Hbar = H_vac - H_m + Hbar_nunu (eq:ham),
 * on a periodic z grid times a grid of velocities v in [-1, 1] (Sec. 3),
 * by the method of lines with classic fourth-order Runge-Kutta.  Advection is
 * either the fourth-order central finite difference with Kreiss-Oliger
 * dissipation (Sec. 3.1) or the finite-volume update eq:cell_av with WENO7
 * interface fluxes (Sec. 3.2, Appendix A).
 *
 * Conventions common to every entry point:
 *  - Return value 0 on success, a negative COSENU_E* code on failure; no C++
 *    exception crosses the ABI.  cosenu_strerror() names a code and
 *    cosenu_last_error() gives the detail recorded on a handle.
 *  - The caller owns every host buffer passed in; the library owns every
 *    device buffer it allocates (freed by the matching destroy call).
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - cosenu_step / cosenu_batch_step are asynchronous on the handle's HIP
 *    stream; every call that returns host data synchronises that stream.
 *  - State arrays on the host are FP64, shape [8][nz][nv] with v fastest,
 *    component order c = 0 rho_ee, 1 rho_xx, 2 Re rho_ex, 3 Im rho_ex,
 *    4 rhobar_ee, 5 rhobar_xx, 6 Re rhobar_ex, 7 Im rhobar_ex
 *    (the density matrices of eq:rho, after the rescaling rho -> g rho of
 *    Sec. 5, i.e. the angular weight g(v) is not folded into the state).
 */
#ifndef COSENU_H
#define COSENU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define COSENU_OK 0
#define COSENU_EINVAL (-1)     /* a parameter is out of range or a buffer is too small */
#define COSENU_ENOMEM (-2)     /* device or host allocation failed                      */
#define COSENU_EDEVICE (-3)    /* a HIP runtime call failed (detail: cosenu_last_error)  */
#define COSENU_ENONFINITE (-4) /* a diagnostics call found NaN or Inf in the state       */
#define COSENU_ESTATE (-5)     /* misuse: null handle, call out of order                 */

/* ---- discretisations and arithmetic forms -------------------------------- */
enum cosenu_scheme {
    COSENU_FD_KO = 0,    /* FD4 central advection + Kreiss-Oliger of order r (Sec. 3.1)  */
    COSENU_FV_WENO7 = 1  /* finite volume eq:cell_av, WENO7 fluxes of f = v u (Sec. 3.2) */
};
enum cosenu_precision {
    COSENU_FP64 = 0,       /* everything in FP64                                          */
    COSENU_FP32_ACC64 = 1  /* advection stencils and WENO in FP32 on FP32-rounded stage
                              values; angular moments, commutators, flux differences and
                              the Runge-Kutta accumulation of the state in FP64           */
};

/* velocity grid and the rule of every velocity integral (Sec. 3 and 3.1) */
enum cosenu_quadrature {
    COSENU_QUAD_MIDPOINT = 0,  /* nv bins of width dv = 2/nv at their midpoints, Riemann sum  */
    COSENU_QUAD_TRAPEZOID = 1, /* nv vertices v_j = -1 + j dv, dv = 2/(nv-1), trapezoid rule */
    COSENU_QUAD_SIMPSON = 2    /* the same vertices (nv odd), composite Simpson rule          */
};

typedef struct cosenu_sim cosenu_sim;
typedef struct cosenu_batch cosenu_batch;

/* Problem description (Sec. 2, 3 and 5).  Units: 1/mu for t and z.
 *  nz, nv      number of z cells (periodic) and velocity points; nz >= 5 for FD
 *              (>= 7 with ko_order 3), nz >= 9 for WENO7; nv >= 2 (one bin would
 *              have max|v| = 0), odd for Simpson's rule; nz * nv <= 2^29 (per-plane
 *              byte offsets are 32 bits).  The velocity grid and the rule of the
 *              integral of eq:ham are set by quadrature.
 *  L           domain length; cells are centred at z_i = -L/2 + (i + 1/2) L/nz.
 *  cfl         dt = cfl * dz / max_j |v_j|  (Sec. 3); 0 < cfl <= 2.  max |v_j|
 *              is 1 - 1/nv for the bins and 1 on a vertex grid.
 *  mu          self-interaction strength of eq:ham.
 *  omega,theta vacuum frequency and mixing angle (radians) of H_vac (Sec. 2).
 *  lambda      matter potential: H_m = diag(lambda, 0), Hbar_m = -diag(lambda, 0)
 *              (the paper removes H_m by a frame rotation, Sec. 2 footnote).
 *  alpha       n_nubar / n_nu (Sec. 5).
 *  sigma_nu, sigma_nubar  widths of g(v) ~ exp(-(v-1)^2 / 2 sigma^2), each
 *              normalised so that sum_j w_j g_j = 1, w_j the quadrature
 *              weights (Sec. 5).
 *  pert_amp, pert_width, phase   initial data eqs:perts with
 *              eps(z) = pert_amp * exp(-z^2 / pert_width), identical in every
 *              bin; rho_ex = eps/2 e^{i phase}, rhobar_ex = eps/2 e^{-i phase}
 *              (phase = 0 is the paper's data).
 *  ko_eps      Kreiss-Oliger strength (paper: 0.1), FD only; 0 switches the
 *              dissipation off.
 *  weno_eps    WENO regulator of eq:weight (paper: about 1e-6), WENO7 only.
 *  ko_order    r of the Kreiss-Oliger operator eps (-1)^r dz^(2r-1) (D+)^r (D-)^r / 2^(2r)
 *              (Sec. 3.1): 1, 2 (the paper's choice) or 3.  FD only, but
 *              validated for both schemes.  Stage pairs are fused only for r <= 2.
 *  quadrature  enum cosenu_quadrature (default COSENU_QUAD_MIDPOINT).
 * Fields appended after weno_eps keep the offsets of the earlier ones;
 * cosenu_params_default fills every field.  */
typedef struct {
    int32_t nz, nv;
    int32_t scheme;    /* enum cosenu_scheme    */
    int32_t precision; /* enum cosenu_precision */
    double L, cfl;
    double mu, omega, theta, lambda;
    double alpha, sigma_nu, sigma_nubar;
    double pert_amp, pert_width, phase;
    double ko_eps, weno_eps;
    int32_t ko_order;   /* 1, 2 or 3                  */
    int32_t quadrature; /* enum cosenu_quadrature     */
} cosenu_params;

/* Conserved quantities and error measures of Sec. 5, from the current state.
 * Every sum over velocities carries the quadrature weight w_j (w_j = dv for
 * the midpoint bins), written dv below.
 *  M0[4]     dz dv sum (g P - alpha gbar Pbar~) as (trace, x, y, z) where
 *            rho = (P0 + P.sigma)/2 and Pbar~ is the vector of rhobar^*; M0[3]
 *            is the net lepton number of Sec. 5.
 *  N_nu, N_nubar   dz dv sum g Tr rho, dz dv sum gbar Tr rhobar.
 *  dP_max    max over cells and species of | |P| - 1 |.
 *  dP_mean   sum dv g | |P_nu| - 1 | / sum dv g (g-weighted mean over all cells).
 *  ee_nu, ee_nubar   dz dv sum g rho_ee, dz dv sum gbar rhobar_ee.
 *  Pee_nu, Pee_nubar survival probabilities: ee_* divided by its value at the
 *            last cosenu_create / cosenu_set_state (Sec. 4.2, taken g-weighted).
 *  B_dot_M0  (sin 2theta, 0, -cos 2theta) . M0[1..3].
 *  nonfinite number of NaN / Inf values found in the state.                 */
typedef struct {
    double t;
    int64_t step;
    double M0[4];
    double N_nu, N_nubar;
    double dP_max, dP_mean;
    double ee_nu, ee_nubar;
    double Pee_nu, Pee_nubar;
    double B_dot_M0;
    int64_t nonfinite;
} cosenu_conserved_t;

/* Read-only facts about a handle. */
typedef struct {
    double dt, dz, dv, t;    /* dv: spacing of the velocity grid             */
    int64_t step;
    size_t device_bytes;     /* device memory owned by the handle              */
    int32_t seg_rows;        /* z rows marched by one lane group (launch shape) */
    int32_t lanes_per_row;   /* lanes sharing one z row (power of two <= 64)   */
    int32_t v_chunks;        /* 64-bin chunks per row (1 when nv <= 64)        */
    int32_t blocks_per_stage;/* workgroups of one stage (or fused pair) launch */
    double bytes_per_step;   /* algorithmic HBM bytes of one RK4 step          */
    int32_t launches_per_step; /* 4 single stages, or 2 fused stage pairs      */
    int32_t waves_per_workgroup; /* of the single-stage launches (1, 2 or 4)  */
} cosenu_info_t;

/* Fills *p with the paper's fiducial values (Sec. 5): nz = 512, nv = 32,
 * L = 400, cfl = 0.4, mu = 1, omega = lambda = 0, theta = 37 deg,
 * alpha = 0.9, sigma = 0.6 / 0.5, eps(z) = 1e-6 exp(-z^2/50), FD + KO with
 * ko_eps = 0.1, ko_order = 2, weno_eps = 1e-6, midpoint bins, FP64.
 * Returns COSENU_EINVAL if p is NULL. */
int cosenu_params_default(cosenu_params *p);

/* Validates *p, allocates the device state on the current HIP device,
 * builds the initial data of eqs:perts, uploads it and prepares the step
 * graph.  On success *out owns everything; on failure *out is NULL. */
int cosenu_create(const cosenu_params *p, cosenu_sim **out);
void cosenu_destroy(cosenu_sim *s);

/* Enqueues nsteps RK4 steps (4 stage launches each, or 2 fused stage pairs,
 * see cosenu_set_fusion) on the handle's stream as HIP graph launches;
 * returns without waiting.  nsteps = 0 is a no-op; nsteps < 0 is EINVAL. */
int cosenu_step(cosenu_sim *s, int64_t nsteps);
/* Waits for everything enqueued on the handle's stream. */
int cosenu_sync(cosenu_sim *s);

/* Copies the FP64 state [8][nz][nv] to / from the host.  n is the number of
 * doubles in the caller's buffer (must be >= 8*nz*nv).  set_state also
 * recomputes the angular moments of the new state and makes it the reference
 * of the survival probabilities; t and step are left unchanged. */
int cosenu_get_state(cosenu_sim *s, double *out, size_t n);
int cosenu_set_state(cosenu_sim *s, const double *in, size_t n);
/* Copies the FP64 state of nrows consecutive z rows starting at row z0 to the
 * host, as [8][nrows][nv]; rows wrap periodically (z0 may be any integer,
 * 1 <= nrows <= nz).  n is the number of doubles in the caller's buffer (must
 * be >= 8*nrows*nv).  Synchronises the handle's stream.  Meant for checking
 * and inspecting a slab of a grid too large to download whole. */
int cosenu_get_rows(cosenu_sim *s, int64_t z0, int32_t nrows, double *out, size_t n);
/* Sets the simulation clock (used with set_state to resume a checkpoint). */
int cosenu_set_clock(cosenu_sim *s, double t, int64_t step);

/* Angular moments of D = g rho - alpha gbar rhobar^* of the current state,
 * per z row: out[(z*2 + m)*4 + q], m = 0: sum_j w_j D_j, m = 1: sum_j w_j v_j D_j
 * (w_j the quadrature weights, dv for the midpoint bins),
 * q = 0 D_ee, 1 D_xx, 2 Re D_ex, 3 Im D_ex (eq:ham is H_nunu(v) = mu (m0 - v m1)).
 * n must be >= 8*nz.  FP64. */
int cosenu_moments(cosenu_sim *s, double *out, size_t n);

/* Conserved quantities of the current state (FP64 reductions in a fixed
 * order).  Returns COSENU_ENONFINITE (with *out filled) if NaN/Inf found. */
int cosenu_conserved(cosenu_sim *s, cosenu_conserved_t *out);

int cosenu_info(cosenu_sim *s, cosenu_info_t *out);

/* Makes the handle enqueue its work on an existing HIP stream (for example
 * torch.cuda.current_stream().cuda_stream).  NULL restores the handle's own
 * stream.  The caller keeps ownership of the stream. */
int cosenu_set_stream(cosenu_sim *s, void *hip_stream);

/* Launch shape: z rows per lane group (>= 1).  0 restores the tuned default.
 * Results do not depend on it (bitwise). */
int cosenu_set_seg_rows(cosenu_sim *s, int32_t seg_rows);

/* Stage fusion (method of lines with classic RK4, Sec. 3.1): on = 0 runs four
 * single-stage launches per step; on = 1 (the default) fuses stages where the
 * shape allows it (FD + KO with ko_order <= 2 and 32 < nv <= 256): two
 * launches per step, stages 1 + 2 and 3 + 4, the intermediate stage values Y2
 * and Y4 on chip and their moments exchanged between the waves of a
 * workgroup, 448 (FP64) or 384 (FP32 form) algorithmic bytes per cell and step
 * against 768 or 704 for single stages; after cosenu_autotune, on = 1 takes the
 * fastest path it measured.  on = 2 runs the whole RK4 step in one launch
 * where the shape allows it (also nz >= 16): the four stages march each
 * segment together with Y2, Y3, Y4 and acc on chip, 128 bytes per cell and
 * step in both forms (the state read and written once).  Other shapes and
 * schemes fall back to what they support.  Results are bitwise those of four
 * single stages on every path.  Other values of on: COSENU_EINVAL.
 * Synchronises the handle's stream; cosenu_info reports launches_per_step
 * (4, 2 or 1). */
int cosenu_set_fusion(cosenu_sim *s, int32_t on);

/* Times nsteps steps on the handle's stream with HIP events (after the work
 * already queued) and returns the elapsed milliseconds; synchronises. */
int cosenu_time_steps(cosenu_sim *s, int64_t nsteps, double *ms);
/* Times each launch of a step separately over nsteps steps (eagerly launched,
 * one event pair around each launch); ms_stage[4] receives the summed
 * milliseconds of stages 1..4, or of the two fused stage pairs followed by two
 * zeros.  Synchronises. */
int cosenu_time_stages(cosenu_sim *s, int64_t nsteps, double *ms_stage);

/* Picks the launch shape by timing whole RK4 steps on the handle's buffers:
 * the segment length of the whole step in one launch and of the fused stage
 * pairs (where the shape allows them and fusion is on), the segment length and
 * the waves per workgroup (1, 2 or 4) of the single stages, and the fastest of
 * these paths (the fused ones recompute the halos of their intermediate stages
 * on chip; single stages re-read their stencil halo from the caches).  The
 * state, its moments and all later results
 * are unchanged (results do not depend on launch shapes).  The choice is
 * cached per device and (kernel variant, precision, nv, nz bucket) for the
 * process, and handles created later start from it; if the environment
 * variable COSENU_TUNE_CACHE names a file, the cache is also read from that
 * file on first use and written back after every tuning (so later processes
 * start tuned).  cosenu_set_fusion afterwards overrides the path.
 * *seg_rows receives the segment length (may be NULL).  Synchronises. */
int cosenu_autotune(cosenu_sim *s, int32_t *seg_rows);

const char *cosenu_strerror(int code);
const char *cosenu_last_error(const cosenu_sim *s);

/* ---- for callers that cannot allocate -------------------------------------
 * cosenu_step_noalloc is for callers that must not allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It advances a state the caller owns on the device by nsteps RK4
 * steps, exactly as cosenu_step advances a handle created from *p (same
 * kernels: fused stage pairs where the shape allows them; default launch
 * shapes; same arithmetic, so the same results bit for bit).  Every intermediate
 * buffer (stage values, the accumulator, the angular-moment partials of
 * each stage input, the per-point constants) lives in one static device
 * array of COSENU_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from
 * its first use on that GPU until the process ends.  The call allocates
 * nothing on the device or the host.
 *  p        problem (validated as by cosenu_create; pert_* and phase unused).
 *  state    device pointer to the FP64 state [8][nz][nv] (layout as above,
 *           planes contiguous, 8*nz*nv doubles), read at the start and
 *           overwritten with the state after nsteps steps.  Caller-owned.
 *  nsteps   >= 0; 0 returns at once.
 *  hip_stream  HIP stream to enqueue on (NULL: the default stream).  The call
 *           is asynchronous: it returns once the launches are enqueued.
 * Needed scratch: about 8*nz*nv*(16 + 8 or 4 bytes: FP64 or FP32 form) plus
 * 384*nz*ceil(nv/64) + 32*nv bytes (each part rounded up to 256 bytes); a
 * problem needing more than COSENU_NOALLOC_SCRATCH_BYTES returns COSENU_EINVAL
 * before anything is enqueued (for example 2048 x 128 fits, 4096 x 128 does
 * not).  Invalid parameters also give COSENU_EINVAL; a HIP error COSENU_EDEVICE.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (other threads, or other streams not ordered with this one) race and
 * corrupt each other's results.  Nothing in the array needs to start at zero:
 * every value is written before it is read within one call.  */
#define COSENU_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int cosenu_step_noalloc(const cosenu_params *p, double *state, int64_t nsteps, void *hip_stream);

/* ---- batched execution ----------------------------------------------------
 * n independent simulations of any sizes and schemes (one precision for the
 * whole batch, taken from p[0]) advanced together: per RK4 step, each kernel
 * variant present runs persistent launches walking a work list (four single
 * stages; for FD + KO with ko_order <= 2 and 32 < nv <= 256 two fused stage
 * pairs, or one whole step once the batch autotuner or a tuning of the shape
 * chose it), and steps of the whole batch are HIP graphs.  Instance i behaves
 * exactly like a cosenu_sim created from p[i] (bit for bit, whatever the
 * paths and launch shapes).                                                 */
int cosenu_batch_create(const cosenu_params *p, int32_t n, cosenu_batch **out);
void cosenu_batch_destroy(cosenu_batch *b);
int cosenu_batch_step(cosenu_batch *b, int64_t nsteps);
int cosenu_batch_sync(cosenu_batch *b);
int cosenu_batch_get_state(cosenu_batch *b, int32_t i, double *out, size_t n);
int cosenu_batch_set_state(cosenu_batch *b, int32_t i, const double *in, size_t n);
int cosenu_batch_conserved(cosenu_batch *b, int32_t i, cosenu_conserved_t *out);
/* Instance i's angular moments and z rows, as cosenu_moments and
 * cosenu_get_rows give them for a single simulation (same layouts, same
 * checks; EINVAL for i out of range).  Synchronise the handle's stream. */
int cosenu_batch_moments(cosenu_batch *b, int32_t i, double *out, size_t n);
/* Sets instance i's clock (with cosenu_batch_set_state, to resume a checkpoint). */
int cosenu_batch_set_clock(cosenu_batch *b, int32_t i, double t, int64_t step);
int cosenu_batch_get_rows(cosenu_batch *b, int32_t i, int64_t z0, int32_t nrows, double *out, size_t n);
int cosenu_batch_info(cosenu_batch *b, int32_t i, cosenu_info_t *out);
int cosenu_batch_time_steps(cosenu_batch *b, int64_t nsteps, double *ms);
/* Batch autotuner: chooses the segment length of every kernel variant of the
 * batch by timing that variant alone (single stages 1-3, or a whole step of
 * the fused pairs or the whole-step kernel) for seg in {4, 6, 8, 11, ..., 128}
 * (about sqrt(2) apart); every instance of a variant takes the same length (at
 * most its nz).  The FD + KO instances that can fuse are timed as fused pairs
 * and as whole steps, and each group with the same vchunks takes the faster
 * path.  Variants: 2*k + (nv > 32) for single stages, k = 0 FD with ko_order
 * <= 2, 1 WENO7, 2 FD with ko_order 3; 6 + vchunks - 1 for fused pairs and
 * 10 + vchunks - 1 for whole steps (vchunks = ceil(nv / 64) = 1 .. 4).  Then
 * rebuilds the task lists and re-captures the step graphs.  States, clocks
 * and results are unchanged (results do not depend on paths or segment
 * lengths).  seg_rows, if not NULL, receives 14 values (0 for variants the
 * batch does not run).  Synchronises the handle's stream.                   */
int cosenu_batch_autotune(cosenu_batch *b, int32_t *seg_rows);
const char *cosenu_batch_last_error(const cosenu_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* COSENU_H */
