// Host-side helpers shared by the single-instance and batched runtimes.
#pragma once

#include <string>
#include <vector>

#include "cosenu.h"
#include "cosenu_internal.h"

namespace cosenu {

const char *strerror_code(int code);
std::string validate_params(const cosenu_params &p);
double grid_dv(int nv, int quad);
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
void fill_desc_constants(const cosenu_params &p, InstDesc &d);
hipError_t moments_to_host(const InstDesc &d, double *scratch, hipStream_t st, double *out);
hipError_t rows_to_host(const InstDesc &d, int64_t z0, int nrows, hipStream_t st, double *out);
void finish_conserved(const cosenu_params &p, const InstDesc &d, const std::vector<double> &part, double ee0n,
                      double ee0b, double t, int64_t step, cosenu_conserved_t *out);
// tuned segment length per (kernel variant, form, nv, nz bucket) and path (fused stage pairs or single stages); 0 if none
int tuned_seg(int scheme, int form, int nz, int nv, bool pairs);
void store_tuned_seg(int scheme, int form, int nz, int nv, bool pairs, int seg);

}  // namespace cosenu
