// Host-side helpers shared by the single-instance and batched runtimes.
#pragma once

#include <exception>
#include <new>
#include <string>
#include <vector>

#include "cosenu.h"
#include "cosenu_internal.h"

namespace cosenu {

const char *strerror_code(int code);
std::string validate_params(const cosenu_params &p);
const char *params_problem(const cosenu_params &p, char *buf, size_t nbuf);
double grid_dv(int nv, int quad);
double point_velocity(int nv, int quad, int j);
double point_weight(int nv, int quad, int j);
double gaussian_raw(double v, double sigma);
double gaussian_norm(int nv, int quad, double sigma);
double bin_constant_at(const cosenu_params &p, int k, double s_nu, double s_nubar);
std::vector<double> bin_velocities(int nv, int quad);
std::vector<double> quadrature_weights(int nv, int quad);
std::vector<double> gaussian_distribution(int nv, int quad, double sigma);
std::vector<double> bin_constants(const cosenu_params &p);
double time_step(const cosenu_params &p);
int lr_log2_for(int nv);
int default_seg_rows(int nz, int nv);
void set_shape(InstDesc &d, int seg);
double bytes_per_cell_step(int form);
double bytes_per_cell_step_fused(int form);
double bytes_per_cell_step_whole(int form);
void fill_desc_constants(const cosenu_params &p, InstDesc &d);
hipError_t moments_to_host(const InstDesc &d, double *scratch, hipStream_t st, double *out);
hipError_t rows_to_host(const InstDesc &d, int64_t z0, int nrows, hipStream_t st, double *out);
// the descriptor of the diagnostics reduction: a fixed decomposition (kDiagSeg rows per task)
InstDesc diag_desc(const InstDesc &d);
void finish_conserved(const cosenu_params &p, const InstDesc &dd, const std::vector<double> &part, double ee0n,
                      double ee0b, double t, int64_t step, cosenu_conserved_t *out);
// Tuned launch shapes per device and (kernel variant, form, nv, nz bucket);
// zeros where not tuned.  Kept for the process, and in the file named by
// COSENU_TUNE_CACHE when that is set.
struct TuneEntry {
    int seg_pairs = 0;   // fused stage pairs: rows per segment
    int seg_quad = 0;    // whole step in one launch: rows per segment
    int seg_single = 0;  // single stages: rows per segment
    int wpb = 0;         // single stages: waves per workgroup (1, 2 or 4)
    int path = -1;       // the fastest full step: 0 single stages, 1 fused pairs, 2 whole step, -1 not compared
};
TuneEntry tuned_entry(int scheme, int form, int nz, int nv);
void store_tuned_entry(int scheme, int form, int nz, int nv, const TuneEntry &e);
// the tuned segment length of one path, 0 if none
int tuned_seg(int scheme, int form, int nz, int nv, bool pairs);

// ---- no C++ exception crosses the C ABI ------------------------------------
// Every extern "C" entry point returning a code is a function-try-block that
// ends in COSENU_ABI_CATCH(err): std::bad_alloc becomes COSENU_ENOMEM, any other
// exception COSENU_EDEVICE, with a message kept in *err when a handle exists.
int abi_fail(std::string *err, int code, const char *what) noexcept;
#define COSENU_ABI_CATCH(errp)                                                                     \
    catch (const std::bad_alloc &) {                                                               \
        return ::cosenu::abi_fail((errp), COSENU_ENOMEM, "host allocation failed");                \
    }                                                                                              \
    catch (const std::exception &e_) {                                                             \
        return ::cosenu::abi_fail((errp), COSENU_EDEVICE, e_.what());                              \
    }                                                                                              \
    catch (...) {                                                                                  \
        return ::cosenu::abi_fail((errp), COSENU_EDEVICE, "unexpected C++ exception");             \
    }

// ---- failure injection for the test-suite (cosenu_testing.h) ---------------
enum {
    kFailThrowBadAlloc = 1,    // parameter validation throws std::bad_alloc
    kFailThrowOther = 2,       // parameter validation throws std::runtime_error
    kFailBatchBuildTasks = 3,  // a batch task-list rebuild returns COSENU_EDEVICE
    kFailSites = 4
};
// true once, when the failure armed for this site is due
bool test_fail_now(int site);

// GPU_MAX_HW_QUEUES is set to a positive value below n
bool hw_queues_below(int n);

}  // namespace cosenu
