// Host runtime behind the C ABI of include/cosenu.h: parameter checks, grid
// and initial data (Sec. 3 and 5), device buffers, the per-step HIP graph,
// diagnostics, timing and the launch-shape autotuner.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <stdexcept>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <unistd.h>
#include <vector>

#include "cosenu.h"
#include "cosenu_host.h"
#include "cosenu_testing.h"
#include "cosenu_internal.h"

using namespace cosenu;

namespace cosenu {

const char *strerror_code(int code) {
    switch (code) {
        case COSENU_OK: return "ok";
        case COSENU_EINVAL: return "invalid argument";
        case COSENU_ENOMEM: return "out of memory";
        case COSENU_EDEVICE: return "HIP device error";
        case COSENU_ENONFINITE: return "non-finite values in the state";
        case COSENU_ESTATE: return "invalid handle or call order";
        default: return "unknown error";
    }
}

int abi_fail(std::string *err, int code, const char *what) noexcept {
    if (err) {
        try {
            *err = what ? what : "exception";
        } catch (...) {
        }
    }
    return code;
}

namespace {
std::atomic<int> g_fail_site{0}, g_fail_after{0};
}  // namespace

bool test_fail_now(int site) {
    if (g_fail_site.load() != site) return false;
    if (g_fail_after.fetch_sub(1) > 0) return false;
    g_fail_site.store(0);
    return true;
}

bool hw_queues_below(int n) {
    const char *e = std::getenv("GPU_MAX_HW_QUEUES");
    if (!e || !*e) return false;
    const long v = std::strtol(e, nullptr, 10);
    return v > 0 && v < n;
}

// The checks of every entry point that takes parameters, without allocating:
// nullptr if p is valid, else the reason (a literal, or formatted into buf).
const char *params_problem(const cosenu_params &p, char *buf, size_t nbuf) {
    auto fin = [](double x) { return std::isfinite(x); };
    if (p.scheme != COSENU_FD_KO && p.scheme != COSENU_FV_WENO7) return "scheme must be COSENU_FD_KO or COSENU_FV_WENO7";
    if (p.precision != COSENU_FP64 && p.precision != COSENU_FP32_ACC64) return "precision must be COSENU_FP64 or COSENU_FP32_ACC64";
    if (p.ko_order < 1 || p.ko_order > 3) return "ko_order must be 1, 2 or 3";
    if (p.quadrature != COSENU_QUAD_MIDPOINT && p.quadrature != COSENU_QUAD_TRAPEZOID &&
        p.quadrature != COSENU_QUAD_SIMPSON)
        return "quadrature must be COSENU_QUAD_MIDPOINT, COSENU_QUAD_TRAPEZOID or COSENU_QUAD_SIMPSON";
    const int nzmin = p.scheme == COSENU_FD_KO ? std::max(5, 2 * p.ko_order + 1) : 9;
    if (p.nz < nzmin) {
        snprintf(buf, nbuf, "nz = %d is below the stencil width (%d)", p.nz, nzmin);
        return buf;
    }
    if (p.nv < 2) return "nv must be >= 2 (with one bin max|v| = 0 and dt is undefined)";
    if (p.quadrature == COSENU_QUAD_SIMPSON && p.nv % 2 == 0) return "Simpson's rule needs an odd nv";
    if ((double)p.nz * (double)p.nv > (double)(1u << 29)) return "nz * nv above 2^29 cells (32-bit byte offsets per plane)";
    if (!(fin(p.L) && p.L > 0)) return "L must be finite and > 0";
    if (!(fin(p.cfl) && p.cfl > 0 && p.cfl <= 2.0)) return "cfl must be in (0, 2]";
    if (!(fin(p.mu) && fin(p.omega) && fin(p.theta) && fin(p.lambda))) return "mu, omega, theta, lambda must be finite";
    if (!(fin(p.alpha) && p.alpha >= 0)) return "alpha must be finite and >= 0";
    if (!(fin(p.sigma_nu) && p.sigma_nu > 0 && fin(p.sigma_nubar) && p.sigma_nubar > 0)) return "sigmas must be > 0";
    if (!(fin(p.pert_amp) && std::fabs(p.pert_amp) <= 1.0)) return "|pert_amp| must be <= 1";
    if (!(fin(p.pert_width) && p.pert_width > 0)) return "pert_width must be > 0";
    if (!fin(p.phase)) return "phase must be finite";
    if (!(fin(p.ko_eps) && p.ko_eps >= 0)) return "ko_eps must be >= 0";
    if (!(fin(p.weno_eps) && p.weno_eps > 0)) return "weno_eps must be > 0";
    return nullptr;
}

std::string validate_params(const cosenu_params &p) {
    if (test_fail_now(kFailThrowBadAlloc)) throw std::bad_alloc();
    if (test_fail_now(kFailThrowOther)) throw std::runtime_error("injected exception (test hook)");
    char buf[256];
    const char *why = params_problem(p, buf, sizeof buf);
    return why ? std::string(why) : std::string();
}

// Velocity grid spacing: bins of width 2/nv, or nv vertices spanning [-1, 1].
double grid_dv(int nv, int quad) { return quad == COSENU_QUAD_MIDPOINT ? 2.0 / nv : 2.0 / (nv - 1); }

// Bin midpoint v_j = -1 + (j + 1/2) dv (Sec. 3), or vertex v_j = -1 + j dv
// (Sec. 3.1).
double point_velocity(int nv, int quad, int j) {
    const double first = quad == COSENU_QUAD_MIDPOINT ? 0.5 : 0.0;
    return -1.0 + (j + first) * grid_dv(nv, quad);
}

// Quadrature weight of point j in the velocity integral (Sec. 3 and 3.1): dv
// per bin (Riemann sum), the composite trapezoid rule (ends halved) or the
// composite Simpson rule (dv/3 times 1, 4, 2, 4, ..., 4, 1).
double point_weight(int nv, int quad, int j) {
    const double dv = grid_dv(nv, quad);
    if (quad == COSENU_QUAD_TRAPEZOID) return (j == 0 || j == nv - 1) ? 0.5 * dv : dv;
    if (quad == COSENU_QUAD_SIMPSON) return (j == 0 || j == nv - 1) ? dv / 3.0 : (j % 2 ? 4.0 : 2.0) * dv / 3.0;
    return dv;
}

// Unnormalised g(v) ~ exp(-(v-1)^2 / 2 sigma^2) (Sec. 5).
double gaussian_raw(double v, double sigma) { return std::exp(-(v - 1.0) * (v - 1.0) / (2.0 * sigma * sigma)); }

// sum_j w_j exp(-(v_j-1)^2 / 2 sigma^2), summed in j order: g is divided by it
// so that sum_j w_j g_j = 1.
double gaussian_norm(int nv, int quad, double sigma) {
    double s = 0.0;
    for (int j = 0; j < nv; ++j) s += gaussian_raw(point_velocity(nv, quad, j), sigma) * point_weight(nv, quad, j);
    return s;
}

std::vector<double> bin_velocities(int nv, int quad) {
    std::vector<double> v(nv);
    for (int j = 0; j < nv; ++j) v[j] = point_velocity(nv, quad, j);
    return v;
}

std::vector<double> quadrature_weights(int nv, int quad) {
    std::vector<double> w(nv);
    for (int j = 0; j < nv; ++j) w[j] = point_weight(nv, quad, j);
    return w;
}

// g(v) ~ exp(-(v-1)^2 / 2 sigma^2) with sum_j w_j g_j = 1 (Sec. 5).
std::vector<double> gaussian_distribution(int nv, int quad, double sigma) {
    const double s = gaussian_norm(nv, quad, sigma);
    std::vector<double> g(nv);
    for (int j = 0; j < nv; ++j) g[j] = gaussian_raw(point_velocity(nv, quad, j), sigma) / s;
    return g;
}

// Element k of the per-point constants as the kernels read them, [4][nv]: v_j,
// then g_j, gbar_j and alpha gbar_j, each times w_j / dv (s_nu, s_nubar: the
// normalisation sums of gaussian_norm).  The kernels form every velocity
// integral as dv times a plain sum over the grid, so the rule's weights travel
// inside the distributions (a factor of exactly one for the bins).  Allocates
// nothing, so the non-allocating entry point computes the same table.
double bin_constant_at(const cosenu_params &p, int k, double s_nu, double s_nubar) {
    const int nv = p.nv, quad = p.quadrature;
    const int q = k / nv, j = k % nv;
    const double v = point_velocity(nv, quad, j);
    if (q == 0) return v;
    const double f = quad == COSENU_QUAD_MIDPOINT ? 1.0 : point_weight(nv, quad, j) / grid_dv(nv, quad);
    if (q == 1) return (gaussian_raw(v, p.sigma_nu) / s_nu) * f;
    const double gb = gaussian_raw(v, p.sigma_nubar) / s_nubar;
    return q == 2 ? gb * f : p.alpha * (gb * f);
}

std::vector<double> bin_constants(const cosenu_params &p) {
    const double s_nu = gaussian_norm(p.nv, p.quadrature, p.sigma_nu);
    const double s_nubar = gaussian_norm(p.nv, p.quadrature, p.sigma_nubar);
    std::vector<double> c(4 * (size_t)p.nv);
    for (size_t k = 0; k < c.size(); ++k) c[k] = bin_constant_at(p, (int)k, s_nu, s_nubar);
    return c;
}

// Per-row moments of the state in d.y into out[nz][2][4] (scratch holds the
// per-chunk partials [nz][vchunks][8]); synchronises st.
hipError_t moments_to_host(const InstDesc &d, double *scratch, hipStream_t st, double *out) {
    const int nz = d.nz, vch = d.vchunks;
    hipError_t e = launch_moments_out(d, scratch, row_blocks_for(d), st);
    std::vector<double> part((size_t)nz * vch * 8);
    if (e == hipSuccess)
        e = hipMemcpyAsync(part.data(), scratch, part.size() * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    for (int z = 0; z < nz; ++z) {
        for (int q = 0; q < 8; ++q) {
            double acc = 0.0;
            for (int c = 0; c < vch; ++c) acc += part[((size_t)z * vch + c) * 8 + q];
            // part holds (D_ee, D_xx, ReD, ImD, v D_ee, ...); out is [z][m][q]
            out[(size_t)z * 8 + q] = d.dv * acc;
        }
    }
    return hipSuccess;
}

// nrows z rows of the state in d.y from row z0 (periodic) into out[8][nrows][nv];
// synchronises st.
hipError_t rows_to_host(const InstDesc &d, int64_t z0, int nrows, hipStream_t st, double *out) {
    const int nz = d.nz, nv = d.nv;
    const int first = (int)(((z0 % nz) + nz) % nz);
    const int n1 = std::min(nrows, nz - first);  // rows before the periodic seam
    const size_t rowb = (size_t)nv * sizeof(double);
    const size_t dpitch = (size_t)nrows * rowb, spitch = d.ps * sizeof(double);
    hipError_t e = hipMemcpy2DAsync(out, dpitch, d.y + (size_t)first * nv, spitch, (size_t)n1 * rowb, 8,
                                    hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && n1 < nrows)
        e = hipMemcpy2DAsync(out + (size_t)n1 * nv, dpitch, d.y, spitch, (size_t)(nrows - n1) * rowb, 8,
                             hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

double time_step(const cosenu_params &p) {
    // largest |v| over the grid: the outer midpoint, or 1 on a vertex grid
    const double vmax = p.quadrature == COSENU_QUAD_MIDPOINT ? 1.0 - 0.5 * (2.0 / p.nv) : 1.0;
    return p.cfl * (p.L / p.nz) / vmax;
}

int lr_log2_for(int nv) {
    int lr = 1, lg = 0;
    const int want = std::min(nv, kWave);
    while (lr < want) { lr <<= 1; ++lg; }
    return lg;
}

int default_seg_rows(int nz, int nv) {
    const int lg = lr_log2_for(nv);
    const int G = kWave >> lg;
    const int vch = nv > kWave ? (nv + kWave - 1) / kWave : 1;
    // aim at ~2048 waves per stage launch (two species per row group), segments of 4 .. 64 rows
    long long target = 2LL * nz * vch / ((long long)G * 2048);
    int s = 4;
    while (s * 2 <= target && s < 64) s *= 2;
    return s;
}

void set_shape(InstDesc &d, int seg) {
    d.seg = std::max(1, std::min(seg, d.nz));
    d.nseg = (d.nz + d.seg - 1) / d.seg;
    d.nrowtasks = d.nseg * d.vchunks;
    const int G = kWave >> d.lr_log2;
    d.tps = (d.nrowtasks + G - 1) / G * G;
    d.ntasks = 2 * d.tps;
}

double bytes_per_cell_step(int form) {
    // 12 FP64 streams of 8 components; in the FP32 form Y3 is written and read in FP32
    return form == COSENU_FP64 ? 12.0 * 64.0 : 10.0 * 64.0 + 2.0 * 32.0;
}

double bytes_per_cell_step_whole(int) {
    // one launch per step reads the state and writes the new state, FP64 in both forms
    return 2.0 * 64.0;
}

double bytes_per_cell_step_fused(int form) {
    // pair 0 reads y, writes Y3 and acc; pair 1 reads Y3, y and acc, writes y
    return form == COSENU_FP64 ? 7.0 * 64.0 : 5.0 * 64.0 + 2.0 * 32.0;
}

void fill_desc_constants(const cosenu_params &p, InstDesc &d) {
    std::memset(&d, 0, sizeof d);
    d.nz = p.nz;
    d.nv = p.nv;
    // kernel variant: FD with the 4-row stencil (KO r = 1, 2), WENO7, FD with
    // the 6-row stencil (KO r = 3)
    d.scheme = p.scheme == COSENU_FD_KO && p.ko_order == 3 ? 2 : p.scheme;
    d.form = p.precision;
    d.lr_log2 = lr_log2_for(p.nv);
    d.vchunks = p.nv > kWave ? (p.nv + kWave - 1) / kWave : 1;
    d.dz_inv = p.nz / p.L;
    d.dt = time_step(p);
    d.dv = grid_dv(p.nv, p.quadrature);
    d.mudv = p.mu * d.dv;
    d.h3vac = -p.omega * std::cos(2.0 * p.theta);
    d.hexvac = 0.5 * p.omega * std::sin(2.0 * p.theta);
    d.lam = p.lambda;
    // Kreiss-Oliger flux -(-1)^r (eps / 2^(2r)) (delta^(2r-1) u)_{i+1/2} (Sec. 3.1),
    // written as ko[0] (u_i - u_{i+1}) + ko[1] (u_{i+2} - u_{i-1}) + ko[2] (u_{i-2} - u_{i+3})
    const double e = p.ko_eps;
    if (p.ko_order == 1) {
        d.ko[0] = e / 4.0;
    } else if (p.ko_order == 2) {
        d.ko[0] = 3.0 * e / 16.0;
        d.ko[1] = e / 16.0;
    } else {
        d.ko[0] = 10.0 * e / 64.0;
        d.ko[1] = 5.0 * e / 64.0;
        d.ko[2] = e / 64.0;
    }
    d.weno_eps = p.weno_eps;
    d.ps = (size_t)p.nz * p.nv + kPlanePad;
    d.wpb = kWavesPerBlock;
    set_shape(d, default_seg_rows(p.nz, p.nv));
}

// The diagnostics reduce over a fixed decomposition of the grid (kDiagSeg rows
// per task), whatever launch shape the stage kernels use.
InstDesc diag_desc(const InstDesc &d) {
    InstDesc dd = d;
    set_shape(dd, kDiagSeg);
    return dd;
}

// Sum of the per-task diagnostic partials (task order, compensated) into the
// public struct; dd is the descriptor the partials were reduced with.
void finish_conserved(const cosenu_params &p, const InstDesc &dd, const std::vector<double> &part, double ee0n,
                      double ee0b, double t, int64_t step, cosenu_conserved_t *out) {
    double a[kDiagQ] = {0}, ac[kDiagQ] = {0};
    auto comp_add = [](double &s, double &c, double x) {
        const double u = s + x;
        c += std::fabs(s) >= std::fabs(x) ? (s - u) + x : (x - u) + s;
        s = u;
    };
    for (int task = 0; task < dd.nrowtasks; ++task) {
        const double *q = &part[(size_t)task * kDiagPartial];
        for (int k = 0; k < kDiagQ; ++k) {
            if (k == 10) {
                a[k] = std::max(a[k], q[k]);
            } else if (k == 11) {
                a[k] += q[k];
            } else {
                comp_add(a[k], ac[k], q[k]);
                comp_add(a[k], ac[k], q[kDiagQ + k]);
            }
        }
    }
    for (int k = 0; k < 10; ++k) a[k] += ac[k];
    const double cell = (p.L / p.nz) * dd.dv;
    std::memset(out, 0, sizeof *out);
    out->t = t;
    out->step = step;
    for (int k = 0; k < 4; ++k) out->M0[k] = cell * a[k];
    out->N_nu = cell * a[4];
    out->N_nubar = cell * a[5];
    out->dP_mean = a[7] > 0 ? a[6] / a[7] : 0.0;
    out->dP_max = a[10];
    out->ee_nu = cell * a[8];
    out->ee_nubar = cell * a[9];
    out->Pee_nu = ee0n != 0 ? out->ee_nu / ee0n : 0.0;
    out->Pee_nubar = ee0b != 0 ? out->ee_nubar / ee0b : 0.0;
    out->B_dot_M0 = std::sin(2.0 * p.theta) * out->M0[1] - std::cos(2.0 * p.theta) * out->M0[3];
    out->nonfinite = (int64_t)a[11];
}

// Launch-shape cache shared by single instances, batches and the
// non-allocating entry point: per device and (kernel variant, form, nv,
// nz bucket), the tuned shapes of both paths and the faster path.  With
// COSENU_TUNE_CACHE naming a file, entries are read from it on first use and
// the whole cache is written back (to a temporary file, then renamed) after
// every tuning, so that later processes on the same kind of device start tuned.
namespace {
std::mutex g_tune_mu;
bool g_tune_loaded = false;
std::map<std::string, TuneEntry> g_tune_cache;  // key: "device scheme form nv bucket"

int nz_bucket(int nz) {
    int bucket = 0;
    while ((1 << (bucket + 1)) <= nz) ++bucket;
    return bucket;
}

// The current device's architecture and compute-unit count: shapes tuned on
// one kind of GPU are not reused on another.
std::string device_tag() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return arch + "/" + std::to_string(prop.multiProcessorCount);
}

std::string tune_key(int scheme, int form, int nz, int nv) {
    return device_tag() + " " + std::to_string(scheme) + " " + std::to_string(form) + " " + std::to_string(nv) + " " +
           std::to_string(nz_bucket(nz));
}

const char *tune_file() {
    const char *f = std::getenv("COSENU_TUNE_CACHE");
    return f && *f ? f : nullptr;
}

// One line per entry: device scheme form nv bucket seg_pairs seg_quad seg_single wpb path.
void load_tune_file_locked() {
    g_tune_loaded = true;
    const char *path = tune_file();
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char dev[128];
    int scheme, form, nv, bucket, sp, sq, ss, wpb, pth;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        if (std::sscanf(line, "%127s %d %d %d %d %d %d %d %d %d", dev, &scheme, &form, &nv, &bucket, &sp, &sq, &ss,
                        &wpb, &pth) != 10)
            continue;
        if (sp < 0 || sq < 0 || ss < 0 || (wpb != 0 && wpb != 1 && wpb != 2 && wpb != 4) || pth < -1 || pth > 2)
            continue;
        TuneEntry e;
        e.seg_pairs = sp;
        e.seg_quad = sq;
        e.seg_single = ss;
        e.wpb = wpb;
        e.path = pth;
        g_tune_cache[std::string(dev) + " " + std::to_string(scheme) + " " + std::to_string(form) + " " +
                     std::to_string(nv) + " " + std::to_string(bucket)] = e;
    }
    std::fclose(f);
}

void save_tune_file_locked() {
    const char *path = tune_file();
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "# cosenu launch-shape cache: device scheme form nv nz_bucket seg_pairs seg_whole_step "
                    "seg_single waves_per_workgroup path(0 single stages, 1 fused pairs, 2 whole step, -1 unknown)\n");
    for (const auto &kv : g_tune_cache)
        std::fprintf(f, "%s %d %d %d %d %d\n", kv.first.c_str(), kv.second.seg_pairs, kv.second.seg_quad,
                     kv.second.seg_single, kv.second.wpb, kv.second.path);
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0) std::remove(tmp.c_str());
}
}  // namespace

TuneEntry tuned_entry(int scheme, int form, int nz, int nv) {
    const std::string key = tune_key(scheme, form, nz, nv);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) load_tune_file_locked();
    auto it = g_tune_cache.find(key);
    return it == g_tune_cache.end() ? TuneEntry() : it->second;
}

void store_tuned_entry(int scheme, int form, int nz, int nv, const TuneEntry &e) {
    const std::string key = tune_key(scheme, form, nz, nv);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) load_tune_file_locked();
    g_tune_cache[key] = e;
    save_tune_file_locked();
}

int tuned_seg(int scheme, int form, int nz, int nv, bool pairs) {
    const TuneEntry e = tuned_entry(scheme, form, nz, nv);
    return pairs ? e.seg_pairs : e.seg_single;
}

}  // namespace cosenu

// ---------------------------------------------------------------------------
struct cosenu_sim {
    cosenu_params prm;
    InstDesc d;
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    // step graphs for a state held in buffer 0 or 1 (g1: one step, gN: gN_steps)
    hipGraphExec_t g1[2] = {nullptr, nullptr}, gN[2] = {nullptr, nullptr};
    int gN_steps = 16;
    // The fused paths write the new state into the other of two buffers (a
    // fused launch still reads the old state on the halo rows of its segments,
    // which neighbouring workgroups are rewriting); d.y is the buffer holding
    // the current state, d.ya the other one.  The whole-step path also
    // alternates the moment partials of the state between mom_buf[0] and
    // mom_buf[1] (the other paths keep them in mom_buf[0]).
    double *state_buf[2] = {nullptr, nullptr};
    double *mom_buf[4] = {nullptr, nullptr, nullptr, nullptr};
    int parity = 0;
    bool graphs_ok = false;
    double t = 0.0;
    int64_t step = 0;
    double ee0_nu = 0.0, ee0_nubar = 0.0;
    size_t bytes = 0;
    std::vector<void *> allocs;
    double *diag_part = nullptr;   // [max tasks][kDiagPartial]
    size_t diag_cap = 0;           // in tasks
    double *mom_out = nullptr;     // [nz][vchunks][8]
    int fusion = 1;                // cosenu_set_fusion: 0 single stages, 1 fused (default), 2 whole step preferred
    int tuned_path = -1;           // the autotuner's (or the cache's) faster path: 0, 1 or 2; -1 none
    std::string err;
};

namespace {
// The path a step takes: 0 four single stages, 1 two fused stage pairs, 2 one
// whole-step launch.  Fusion off means single stages; otherwise the tuned path
// (or, untuned, fused pairs, or the whole step when preferred), falling back to
// what the shape supports.
int path_of(const cosenu_sim *s, const InstDesc &d) {
    if (s->fusion == 0) return 0;
    const int want = s->tuned_path >= 0 ? s->tuned_path : (s->fusion == 2 ? 2 : 1);
    if (want == 2 && quad_supported(d)) return 2;
    if (want >= 1 && pair_supported(d)) return 1;
    return 0;
}
int path_of(const cosenu_sim *s) { return path_of(s, s->d); }
bool fused(const cosenu_sim *s) { return path_of(s) != 0; }
void point_state(InstDesc &d, const cosenu_sim *s, int p, int path) {
    d.y = s->state_buf[p];
    d.ya = s->state_buf[1 - p];
    const int m = path == 2 ? p : 0;
    d.mom[0] = s->mom_buf[m];
    d.mom[1] = s->mom_buf[1 - m];
}
void set_parity(cosenu_sim *s, int p) {
    s->parity = p;
    point_state(s->d, s, p, path_of(s));
}
int launches_per_step(const cosenu_sim *s) {
    const int path = path_of(s);
    return path == 2 ? 1 : path == 1 ? 2 : 4;
}
// launch k of a step: the whole step, a fused stage pair, or one single stage
hipError_t launch_k(const cosenu_sim *s, int k, hipStream_t st) {
    const int path = path_of(s);
    if (path == 2) return launch_quad(s->d, st);
    return path == 1 ? launch_pair(s->d, k, st) : launch_stage(s->d, k, blocks_for(s->d), st);
}
double bytes_per_step_of(const cosenu_sim *s) {
    const int path = path_of(s);
    const double per_cell = path == 2 ? bytes_per_cell_step_whole(s->prm.precision)
                          : path == 1 ? bytes_per_cell_step_fused(s->prm.precision)
                                      : bytes_per_cell_step(s->prm.precision);
    return per_cell * (double)s->d.nz * s->d.nv;
}
}  // namespace

#define SIM_CHECK(s)                                   \
    do {                                               \
        if (!(s)) return COSENU_ESTATE;                \
    } while (0)

#define HIPCHK(s, call)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            (s)->err = std::string(#call) + ": " + hipGetErrorString(e_);                  \
            return e_ == hipErrorOutOfMemory ? COSENU_ENOMEM : COSENU_EDEVICE;             \
        }                                                                                  \
    } while (0)

namespace {

int sim_alloc(cosenu_sim *s, void **p, size_t bytes) {
    HIPCHK(s, hipMalloc(p, bytes));
    s->allocs.push_back(*p);
    s->bytes += bytes;
    return COSENU_OK;
}

void destroy_graphs(cosenu_sim *s) {
    for (int p = 0; p < 2; ++p) {
        if (s->g1[p]) (void)hipGraphExecDestroy(s->g1[p]);
        if (s->gN[p]) (void)hipGraphExecDestroy(s->gN[p]);
        s->g1[p] = s->gN[p] = nullptr;
    }
    s->graphs_ok = false;
}

// nsteps steps from a state in buffer p: four single stages per step (the
// state stays in place), two fused pairs or one whole-step launch (the state
// changes buffer)
int enqueue_steps(cosenu_sim *s, hipStream_t st, int nsteps, int p) {
    InstDesc d = s->d;
    const int path = path_of(s);
    for (int k = 0; k < nsteps; ++k) {
        point_state(d, s, p, path);
        if (path == 2) {
            HIPCHK(s, launch_quad(d, st));
            p ^= 1;
        } else if (path == 1) {
            HIPCHK(s, launch_pair(d, 0, st));
            HIPCHK(s, launch_pair(d, 1, st));
            p ^= 1;
        } else {
            for (int stage = 0; stage < 4; ++stage) HIPCHK(s, launch_stage(d, stage, blocks_for(d), st));
        }
    }
    return COSENU_OK;
}

int capture(cosenu_sim *s, int nsteps, int p, hipGraphExec_t *out) {
    hipGraph_t graph = nullptr;
    HIPCHK(s, hipStreamBeginCapture(s->own_stream, hipStreamCaptureModeRelaxed));
    int rc = enqueue_steps(s, s->own_stream, nsteps, p);
    hipError_t e = hipStreamEndCapture(s->own_stream, &graph);
    if (rc != COSENU_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) {
        s->err = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
        return COSENU_EDEVICE;
    }
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        s->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
        return COSENU_EDEVICE;
    }
    return COSENU_OK;
}

int build_graphs(cosenu_sim *s) {
    destroy_graphs(s);
    for (int p = 0; p < 2; ++p) {
        int rc = capture(s, 1, p, &s->g1[p]);
        if (rc) return rc;
        rc = capture(s, s->gN_steps, p, &s->gN[p]);
        if (rc) return rc;
    }
    s->graphs_ok = true;
    return COSENU_OK;
}

int ensure_diag_capacity(cosenu_sim *s, const InstDesc &dd) {
    if ((size_t)dd.nrowtasks <= s->diag_cap) return COSENU_OK;
    size_t need = (size_t)dd.nrowtasks;
    void *p = nullptr;
    int rc = sim_alloc(s, &p, need * kDiagPartial * sizeof(double));
    if (rc) return rc;
    s->diag_part = (double *)p;
    s->diag_cap = need;
    return COSENU_OK;
}

int compute_conserved(cosenu_sim *s, cosenu_conserved_t *out) {
    const InstDesc dd = diag_desc(s->d);
    int rc = ensure_diag_capacity(s, dd);
    if (rc) return rc;
    HIPCHK(s, launch_diag(dd, s->diag_part, row_blocks_for(dd), s->stream));
    std::vector<double> part((size_t)dd.nrowtasks * kDiagPartial);
    HIPCHK(s, hipMemcpyAsync(part.data(), s->diag_part, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                             s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    finish_conserved(s->prm, dd, part, s->ee0_nu, s->ee0_nubar, s->t, s->step, out);
    return COSENU_OK;
}

// After a new state is in d.y: moments of the stage-1 input and the
// reference of the survival probabilities.
int state_changed(cosenu_sim *s) {
    HIPCHK(s, launch_moments_init(s->d, blocks_for(s->d), s->stream));
    cosenu_conserved_t c;
    int rc = compute_conserved(s, &c);
    if (rc) return rc;
    s->ee0_nu = c.ee_nu;
    s->ee0_nubar = c.ee_nubar;
    return COSENU_OK;
}

int upload_state(cosenu_sim *s, const double *host) {
    const size_t row = (size_t)s->d.nz * s->d.nv * sizeof(double);
    HIPCHK(s, hipMemcpy2DAsync(s->d.y, s->d.ps * sizeof(double), host, row, row, 8, hipMemcpyHostToDevice,
                               s->stream));
    return state_changed(s);
}

}  // namespace

// ---------------------------------------------------------------------------
extern "C" {

const char *cosenu_strerror(int code) { return strerror_code(code); }

int cosenu_test_inject_failure(int32_t site, int32_t after) {
    if (site < 0 || site >= kFailSites || after < 0) return COSENU_EINVAL;
    g_fail_after.store(after);
    g_fail_site.store(site);
    return COSENU_OK;
}

const char *cosenu_last_error(const cosenu_sim *s) { return s ? s->err.c_str() : "null handle"; }

int cosenu_params_default(cosenu_params *p) try {
    if (!p) return COSENU_EINVAL;
    std::memset(p, 0, sizeof *p);
    p->nz = 512;
    p->nv = 32;
    p->scheme = COSENU_FD_KO;
    p->precision = COSENU_FP64;
    p->L = 400.0;
    p->cfl = 0.4;
    p->mu = 1.0;
    p->omega = 0.0;
    p->theta = 37.0 * 3.14159265358979323846 / 180.0;
    p->lambda = 0.0;
    p->alpha = 0.9;
    p->sigma_nu = 0.6;
    p->sigma_nubar = 0.5;
    p->pert_amp = 1e-6;
    p->pert_width = 50.0;
    p->phase = 0.0;
    p->ko_eps = 0.1;
    p->weno_eps = 1e-6;
    p->ko_order = 2;
    p->quadrature = COSENU_QUAD_MIDPOINT;
    return COSENU_OK;
} COSENU_ABI_CATCH(nullptr)

void cosenu_destroy(cosenu_sim *s) try {
    if (!s) return;
    if (s->own_stream) (void)hipStreamSynchronize(s->own_stream);
    if (s->stream && s->stream != s->own_stream) (void)hipStreamSynchronize(s->stream);
    destroy_graphs(s);
    for (void *p : s->allocs) (void)hipFree(p);
    if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
    delete s;
} catch (...) {
}

int cosenu_create(const cosenu_params *p, cosenu_sim **out) try {
    if (!p || !out) return COSENU_EINVAL;
    *out = nullptr;
    if (!validate_params(*p).empty()) return COSENU_EINVAL;
    cosenu_sim *s = new (std::nothrow) cosenu_sim();
    if (!s) return COSENU_ENOMEM;
    // destroys the partly built handle on every early return, and on an
    // exception (which the ABI guard below then turns into a code)
    struct Owner {
        cosenu_sim *h;
        ~Owner() { if (h) cosenu_destroy(h); }
    } own{s};
    s->prm = *p;
    auto fail = [&](int rc) { return rc; };
    if (hipGetDevice(&s->device) != hipSuccess) return fail(COSENU_EDEVICE);
    if (hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking) != hipSuccess) return fail(COSENU_EDEVICE);
    s->stream = s->own_stream;

    fill_desc_constants(*p, s->d);
    {
        // launch shapes from the tuning cache, if this shape was tuned before
        const TuneEntry e = tuned_entry(s->d.scheme, p->precision, p->nz, p->nv);
        s->tuned_path = e.path;
        if (e.wpb > 0) s->d.wpb = e.wpb;
        const int path = path_of(s);
        const int tuned = path == 2 ? e.seg_quad : path == 1 ? e.seg_pairs : e.seg_single;
        if (tuned > 0) set_shape(s->d, tuned);
    }

    const int nz = p->nz, nv = p->nv;
    const size_t f64 = 8 * s->d.ps * sizeof(double);
    const size_t ybbytes = 8 * s->d.ps * (p->precision == COSENU_FP64 ? sizeof(double) : sizeof(float));
    void *ptr = nullptr;
    int rc;
    if ((rc = sim_alloc(s, &ptr, f64))) return fail(rc);
    s->state_buf[0] = (double *)ptr;
    if ((rc = sim_alloc(s, &ptr, f64))) return fail(rc);
    s->d.acc = (double *)ptr;
    if ((rc = sim_alloc(s, &ptr, f64))) return fail(rc);
    s->state_buf[1] = (double *)ptr;
    if ((rc = sim_alloc(s, &ptr, ybbytes))) return fail(rc);
    s->d.yb = ptr;
    const size_t mom_bytes = (size_t)nz * s->d.vchunks * 2 * kMomQ * sizeof(double);
    for (int k = 0; k < 4; ++k) {
        if ((rc = sim_alloc(s, &ptr, mom_bytes))) return fail(rc);
        s->mom_buf[k] = (double *)ptr;
        s->d.mom[k] = (double *)ptr;
    }
    set_parity(s, 0);
    // per-bin constants
    const std::vector<double> hostc = bin_constants(*p);
    double *consts = nullptr;
    if ((rc = sim_alloc(s, (void **)&consts, hostc.size() * sizeof(double)))) return fail(rc);
    if (hipMemcpy(consts, hostc.data(), hostc.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return fail(COSENU_EDEVICE);
    s->d.vel = consts;
    s->d.g = consts + nv;
    s->d.gb = consts + 2 * nv;
    s->d.agb = consts + 3 * nv;
    // scratch buffers that never move (so captured graphs stay valid)
    if ((rc = sim_alloc(s, &ptr, (size_t)nz * s->d.vchunks * 8 * sizeof(double)))) return fail(rc);
    s->mom_out = (double *)ptr;
    {
        // diagnostics partials sized for the finest launch shape the tuner may pick (seg >= 1)
        const size_t cap = (size_t)nz * s->d.vchunks;
        if ((rc = sim_alloc(s, &ptr, cap * kDiagPartial * sizeof(double)))) return fail(rc);
        s->diag_part = (double *)ptr;
        s->diag_cap = cap;
    }
    // initial data (eqs:perts), computed on the device
    if (launch_init_state(s->d, p->L, p->pert_amp, p->pert_width, p->phase, s->stream) != hipSuccess)
        return fail(COSENU_EDEVICE);
    if ((rc = state_changed(s))) return fail(rc);
    if ((rc = build_graphs(s))) return fail(rc);
    own.h = nullptr;
    *out = s;
    return COSENU_OK;
} COSENU_ABI_CATCH(nullptr)

int cosenu_step(cosenu_sim *s, int64_t nsteps) try {
    SIM_CHECK(s);
    if (nsteps < 0) return COSENU_EINVAL;
    if (nsteps == 0) return COSENU_OK;
    if (!s->graphs_ok) {
        int rc = build_graphs(s);
        if (rc) return rc;
    }
    const bool moves = fused(s);  // the fused paths move the state to the other buffer every step
    int64_t big = nsteps / s->gN_steps, rem = nsteps % s->gN_steps;
    for (int64_t k = 0; k < big; ++k) {
        HIPCHK(s, hipGraphLaunch(s->gN[s->parity], s->stream));
        if (moves && (s->gN_steps & 1)) set_parity(s, s->parity ^ 1);
    }
    for (int64_t k = 0; k < rem; ++k) {
        HIPCHK(s, hipGraphLaunch(s->g1[s->parity], s->stream));
        if (moves) set_parity(s, s->parity ^ 1);
    }
    s->step += nsteps;
    s->t += (double)nsteps * s->d.dt;
    return COSENU_OK;
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_sync(cosenu_sim *s) try {
    SIM_CHECK(s);
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return COSENU_OK;
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_get_state(cosenu_sim *s, double *out, size_t n) try {
    SIM_CHECK(s);
    const size_t need = (size_t)8 * s->d.nz * s->d.nv;
    if (!out || n < need) return COSENU_EINVAL;
    const size_t row = (size_t)s->d.nz * s->d.nv * sizeof(double);
    HIPCHK(s, hipMemcpy2DAsync(out, row, s->d.y, s->d.ps * sizeof(double), row, 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return COSENU_OK;
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_get_rows(cosenu_sim *s, int64_t z0, int32_t nrows, double *out, size_t n) try {
    SIM_CHECK(s);
    if (!out || nrows < 1 || nrows > s->d.nz || n < (size_t)8 * nrows * s->d.nv) return COSENU_EINVAL;
    HIPCHK(s, rows_to_host(s->d, z0, nrows, s->stream, out));
    return COSENU_OK;
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_set_state(cosenu_sim *s, const double *in, size_t n) try {
    SIM_CHECK(s);
    const size_t need = (size_t)8 * s->d.nz * s->d.nv;
    if (!in || n < need) return COSENU_EINVAL;
    return upload_state(s, in);
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_set_clock(cosenu_sim *s, double t, int64_t step) try {
    SIM_CHECK(s);
    if (!std::isfinite(t) || step < 0) return COSENU_EINVAL;
    s->t = t;
    s->step = step;
    return COSENU_OK;
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_moments(cosenu_sim *s, double *out, size_t n) try {
    SIM_CHECK(s);
    if (!out || n < (size_t)8 * s->d.nz) return COSENU_EINVAL;
    HIPCHK(s, moments_to_host(s->d, s->mom_out, s->stream, out));
    return COSENU_OK;
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_conserved(cosenu_sim *s, cosenu_conserved_t *out) try {
    SIM_CHECK(s);
    if (!out) return COSENU_EINVAL;
    int rc = compute_conserved(s, out);
    if (rc) return rc;
    return out->nonfinite ? COSENU_ENONFINITE : COSENU_OK;
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_info(cosenu_sim *s, cosenu_info_t *out) try {
    SIM_CHECK(s);
    if (!out) return COSENU_EINVAL;
    std::memset(out, 0, sizeof *out);
    out->dt = s->d.dt;
    out->dz = s->prm.L / s->prm.nz;
    out->dv = s->d.dv;
    out->t = s->t;
    out->step = s->step;
    out->device_bytes = s->bytes;
    out->seg_rows = s->d.seg;
    out->lanes_per_row = 1 << s->d.lr_log2;
    out->v_chunks = s->d.vchunks;
    out->blocks_per_stage = fused(s) ? s->d.nseg : blocks_for(s->d);
    out->bytes_per_step = bytes_per_step_of(s);
    out->launches_per_step = launches_per_step(s);
    out->waves_per_workgroup = s->d.wpb;
    return COSENU_OK;
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_set_stream(cosenu_sim *s, void *hip_stream) try {
    SIM_CHECK(s);
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->stream = hip_stream ? (hipStream_t)hip_stream : s->own_stream;
    return COSENU_OK;
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_set_seg_rows(cosenu_sim *s, int32_t seg_rows) try {
    SIM_CHECK(s);
    if (seg_rows < 0) return COSENU_EINVAL;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    int seg = seg_rows;
    if (seg == 0) {
        const TuneEntry e = tuned_entry(s->d.scheme, s->prm.precision, s->prm.nz, s->prm.nv);
        const int path = path_of(s);
        seg = path == 2 ? e.seg_quad : path == 1 ? e.seg_pairs : e.seg_single;
        if (seg == 0) seg = default_seg_rows(s->prm.nz, s->prm.nv);
    }
    set_shape(s->d, seg);
    return build_graphs(s);
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_set_fusion(cosenu_sim *s, int32_t on) try {
    SIM_CHECK(s);
    if (on < 0 || on > 2) return COSENU_EINVAL;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->fusion = on;
    s->tuned_path = -1;
    // the moments of the state may live in another buffer on the new path
    set_parity(s, s->parity);
    HIPCHK(s, launch_moments_init(s->d, blocks_for(s->d), s->stream));
    return build_graphs(s);
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_time_steps(cosenu_sim *s, int64_t nsteps, double *ms) try {
    SIM_CHECK(s);
    if (!ms || nsteps < 0) return COSENU_EINVAL;
    hipEvent_t a, b;
    HIPCHK(s, hipEventCreate(&a));
    HIPCHK(s, hipEventCreate(&b));
    int rc = COSENU_OK;
    if (hipEventRecord(a, s->stream) != hipSuccess) rc = COSENU_EDEVICE;
    if (!rc) rc = cosenu_step(s, nsteps);
    if (!rc && hipEventRecord(b, s->stream) != hipSuccess) rc = COSENU_EDEVICE;
    if (!rc && hipEventSynchronize(b) != hipSuccess) rc = COSENU_EDEVICE;
    float f = 0.f;
    if (!rc && hipEventElapsedTime(&f, a, b) != hipSuccess) rc = COSENU_EDEVICE;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = f;
    if (rc == COSENU_EDEVICE && s->err.empty()) s->err = "event timing failed";
    return rc;
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_time_stages(cosenu_sim *s, int64_t nsteps, double *ms_stage) try {
    SIM_CHECK(s);
    if (!ms_stage || nsteps < 0) return COSENU_EINVAL;
    std::vector<hipEvent_t> ev(8);
    for (auto &e : ev) HIPCHK(s, hipEventCreate(&e));
    for (int k = 0; k < 4; ++k) ms_stage[k] = 0.0;
    const int nl = launches_per_step(s);
    int rc = COSENU_OK;
    for (int64_t n = 0; n < nsteps && !rc; ++n) {
        for (int stage = 0; stage < nl; ++stage) {
            if (hipEventRecord(ev[2 * stage], s->stream) != hipSuccess) rc = COSENU_EDEVICE;
            if (!rc && launch_k(s, stage, s->stream) != hipSuccess) rc = COSENU_EDEVICE;
            if (!rc && hipEventRecord(ev[2 * stage + 1], s->stream) != hipSuccess) rc = COSENU_EDEVICE;
        }
        if (!rc && nl <= 2) set_parity(s, s->parity ^ 1);  // the fused paths moved the state
        if (!rc && hipEventSynchronize(ev[2 * nl - 1]) != hipSuccess) rc = COSENU_EDEVICE;
        for (int stage = 0; stage < nl && !rc; ++stage) {
            float f = 0.f;
            if (hipEventElapsedTime(&f, ev[2 * stage], ev[2 * stage + 1]) != hipSuccess) rc = COSENU_EDEVICE;
            ms_stage[stage] += f;
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (!rc) {
        s->step += nsteps;
        s->t += (double)nsteps * s->d.dt;
    } else if (s->err.empty()) {
        s->err = "stage timing failed";
    }
    return rc;
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

int cosenu_autotune(cosenu_sim *s, int32_t *seg_rows) try {
    SIM_CHECK(s);
    HIPCHK(s, hipStreamSynchronize(s->stream));
    // Every candidate is timed over whole RK4 steps on the handle's buffers,
    // leaving the state untouched: stages 1-3 write only scratch (Y2, Y3, Y4,
    // acc and the moments of those stage values); stage 4 is timed with its
    // output redirected onto acc, which it reads point by point (each value is
    // read before it is overwritten, by the same lane); the second fused pair
    // writes the other state buffer, scratch until a step is taken.  Stage 4 and
    // the fused pairs overwrite the moments of the current state, which are
    // rebuilt afterwards from the state with the producer's own arithmetic.
    //
    // Search: the segment length of the fused pairs (where the shape allows
    // them and fusion is on), the segment length of the single stages with 4
    // waves per workgroup, then 1 and 2 waves per workgroup at that length,
    // then the faster of the two paths.  Segment lengths are about sqrt(2)
    // apart: the workgroup count of the fused pairs (one per segment) has to
    // land just under a whole number of resident rounds.
    const int cands[] = {4, 6, 8, 11, 16, 22, 32, 45, 64, 90, 128, 181, 256};
    const InstDesc keep = s->d;
    const bool try_pairs = s->fusion != 0 && pair_supported(s->d);
    const bool try_quad = s->fusion != 0 && quad_supported(s->d);
    hipEvent_t a, b;
    HIPCHK(s, hipEventCreate(&a));
    HIPCHK(s, hipEventCreate(&b));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{a, b};
    // one pass = one RK4 step of the given path (0 single stages, 1 fused
    // pairs, 2 whole step) and shape
    auto pass = [&](const InstDesc &d, int path) -> bool {
        if (path == 2) {
            // the whole step writes the other state buffer and the other moment buffer
            InstDesc dq = d;
            point_state(dq, s, s->parity, 2);
            return launch_quad(dq, s->stream) == hipSuccess;
        }
        if (path == 1) return launch_pair(d, 0, s->stream) == hipSuccess && launch_pair(d, 1, s->stream) == hipSuccess;
        InstDesc d4 = d;
        d4.y = d.acc;  // stage 4 writes over acc (scratch) instead of the state
        const int nb = blocks_for(d);
        return launch_stage(d, 0, nb, s->stream) == hipSuccess && launch_stage(d, 1, nb, s->stream) == hipSuccess &&
               launch_stage(d, 2, nb, s->stream) == hipSuccess && launch_stage(d4, 3, nb, s->stream) == hipSuccess;
    };
    // milliseconds per step: the fastest of several repetitions (after one to
    // warm up), so candidates a few percent apart are told apart through
    // run-to-run jitter; fewer repetitions for long steps
    auto time_step = [&](const InstDesc &d, int path, double *ms) -> bool {
        float f = 0.f;
        if (!(hipEventRecord(a, s->stream) == hipSuccess && pass(d, path) &&
              hipEventRecord(b, s->stream) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
              hipEventElapsedTime(&f, a, b) == hipSuccess))
            return false;
        const int reps = f > 20.f ? 2 : 5, passes = f > 5.f ? 1 : 3;
        double best = 1e300;
        for (int rep = 0; rep < reps; ++rep) {
            bool ok = hipEventRecord(a, s->stream) == hipSuccess;
            for (int k = 0; k < passes && ok; ++k) ok = pass(d, path);
            ok = ok && hipEventRecord(b, s->stream) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
                 hipEventElapsedTime(&f, a, b) == hipSuccess;
            if (!ok) return false;
            best = std::min(best, (double)f / passes);
        }
        *ms = best;
        return true;
    };
    auto fail = [&]() {
        s->d = keep;
        set_parity(s, s->parity);
        (void)launch_moments_init(s->d, blocks_for(s->d), s->stream);
        (void)hipStreamSynchronize(s->stream);
        s->err = "autotune launch failed";
        return COSENU_EDEVICE;
    };
    // the fastest segment length of one path at the given waves per workgroup
    auto sweep = [&](int path, int wpb, int *seg_out, double *ms_out) -> bool {
        *ms_out = 1e300;
        for (int c : cands) {
            if (c > keep.nz) break;
            InstDesc d = keep;
            d.wpb = wpb;
            set_shape(d, c);
            double ms;
            if (!time_step(d, path, &ms)) return false;
            if (ms < *ms_out) {
                *ms_out = ms;
                *seg_out = c;
            }
        }
        return true;
    };
    TuneEntry e = tuned_entry(keep.scheme, s->prm.precision, s->prm.nz, s->prm.nv);
    double ms_pairs = 1e300, ms_single = 1e300, ms_quad = 1e300;
    int seg_pairs = keep.seg, seg_single = keep.seg, seg_quad = keep.seg, wpb = kWavesPerBlock;
    if (try_quad && !sweep(2, kWavesPerBlock, &seg_quad, &ms_quad)) return fail();
    if (try_pairs && !sweep(1, kWavesPerBlock, &seg_pairs, &ms_pairs)) return fail();
    if (!sweep(0, kWavesPerBlock, &seg_single, &ms_single)) return fail();
    for (int w : {2, 1}) {
        InstDesc d = keep;
        d.wpb = w;
        set_shape(d, seg_single);
        double ms;
        if (!time_step(d, 0, &ms)) return fail();
        if (ms < ms_single) {
            ms_single = ms;
            wpb = w;
        }
    }
    int path = 0;
    double best = ms_single;
    if (try_pairs && ms_pairs <= best) {
        path = 1;
        best = ms_pairs;
    }
    if (try_quad && ms_quad <= best) path = 2;
    e.seg_single = seg_single;
    e.wpb = wpb;
    if (try_pairs) e.seg_pairs = seg_pairs;
    if (try_quad) e.seg_quad = seg_quad;
    if (try_pairs || try_quad) e.path = path;
    s->d = keep;
    s->d.wpb = wpb;
    if (try_pairs || try_quad) s->tuned_path = path;
    set_shape(s->d, path == 2 ? seg_quad : path == 1 ? seg_pairs : seg_single);
    set_parity(s, s->parity);  // the moments of the state live where the chosen path keeps them
    HIPCHK(s, launch_moments_init(s->d, blocks_for(s->d), s->stream));
    store_tuned_entry(keep.scheme, s->prm.precision, s->prm.nz, s->prm.nv, e);
    if (seg_rows) *seg_rows = s->d.seg;
    return build_graphs(s);
} COSENU_ABI_CATCH(s ? &s->err : nullptr)

}  // extern "C"
