// Internal interface between the host runtime and the gfx950 kernels.
// Not part of the public ABI (see include/cosenu.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cosenu {

constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kWavesPerBlock = 4;   // default (and largest) waves per stage workgroup; diagnostics and
                                    // batch kernels always run 4 (256 threads)
constexpr int kMomQ = 6;            // reduced quantities per row and part:
                                    //   sum D3, sum ReDex, sum ImDex, and the same times v
constexpr int kDiagQ = 12;         // per-task quantities of the conserved-quantity kernel
constexpr int kDiagPartial = 22;   // per-task doubles it writes: kDiagQ values, then the compensations
                                   //   of the 10 compensated sums
constexpr int kDiagSeg = 16;       // rows per task of the conserved-quantity reduction, fixed so that
                                   //   results do not depend on the stage kernels' launch shape
constexpr int kPlanePad = 544;      // elements between planes beyond nz*nv (4352 B in FP64, 2176 B
                                    // in FP32: 128-byte aligned, off the power-of-two strides)
constexpr int kLdsQStride = 68;     // doubles between quantity rows of a wave's moment scratch
constexpr int kLdsPerWave = 8 * kLdsQStride;  // LDS doubles per wave (6 quantities + 2 pad rows)

// Everything one stage launch needs about one simulation.  Passed by value to
// the single-instance kernels and stored in device memory for the batch.
struct InstDesc {
    int32_t nz, nv;
    int32_t scheme;    // kernel variant: 0 FD (KO r = 1, 2), 1 WENO7, 2 FD (KO r = 3)
    int32_t form;
    int32_t lr_log2;   // lanes per row group = 1 << lr_log2 (<= 64)
    int32_t vchunks;   // 64-bin chunks per row (1 when nv <= 64); = moment parts per row
    int32_t seg;       // rows per lane group
    int32_t nseg;      // ceil(nz / seg)
    int32_t nrowtasks; // nseg * vchunks: (segment, chunk) pairs
    int32_t tps;       // stage tasks per species: nrowtasks padded to a multiple of the groups per wave
    int32_t ntasks;    // stage tasks: 2 * tps (neutrinos, then antineutrinos)
    int32_t wpb;       // waves per workgroup of the single-instance stage and moment kernels: 1, 2 or 4
    double dz_inv;     // 1 / dz
    double dt;
    double mudv;       // mu * dv
    double h3vac;      // (H_vac)_ee - (H_vac)_xx = -omega cos 2theta
    double hexvac;     // (H_vac)_ex = omega/2 sin 2theta
    double lam;        // matter potential
    double ko[3];      // Kreiss-Oliger flux coefficients of u_i - u_{i+1}, u_{i+2} - u_{i-1}, u_{i-2} - u_{i+3}
    double weno_eps;
    double dv;
    size_t ps;         // plane stride in elements: nz * nv + kPlanePad
    const double *g;   // g_nu per point times w_j / dv         [nv]
    const double *gb;  // g_nubar per point times w_j / dv      [nv]
    const double *agb; // alpha * gb                            [nv]
    const double *vel; // velocity grid                         [nv]
    double *y;         // state, FP64                        [8][ps], plane = [nz][nv]
    double *acc;       // RK4 accumulator, FP64              [8][nz][nv]
    void *ya;          // Y2 / Y4 stage values, FP64         [8][nz][nv]
    void *yb;          // Y3 stage values, FP64 or FP32      [8][nz][nv]
    double *mom[4];    // row moment partials of the stage inputs y, Y2, Y3, Y4
                       //   [nz][vchunks][2 species][kMomQ]
};

// One wave's work item in a batched launch: instance and first task.
struct WaveTask {
    int32_t inst;
    int32_t task0;
};

// ---- launchers (stage_kernels.hip) -----------------------------------------
// single-instance launches run blocks workgroups of d.wpb waves
hipError_t launch_stage(const InstDesc &d, int stage, int blocks, hipStream_t st);
hipError_t launch_moments_init(const InstDesc &d, int blocks, hipStream_t st);
// wave_rows: every instance of the task list has nv > 32 (one row group per wave)
hipError_t launch_batch_stage(const InstDesc *d_descs, const WaveTask *d_tasks, int nwaves, int scheme, int form,
                              bool wave_rows, int stage, int blocks, hipStream_t st);
// resident waves per CU of the batch stage kernels of one variant (the least over the four stages)
int batch_waves_per_cu(int scheme, int form, bool wave_rows);
// fused stage pairs (FD + KO, 32 < nv <= 256): pair 0 = stages 1 and 2, pair 1 = stages 3 and 4;
// one workgroup of 2 vchunks waves per segment (d.nseg workgroups)
bool pair_supported(const InstDesc &d);
hipError_t launch_pair(const InstDesc &d, int pair, hipStream_t st);
// a whole RK4 step in one launch (FD + KO, 32 < nv <= 256, nz >= 16): reads the
// state in d.y and its moment partials in d.mom[0], writes the new state into
// d.ya and its moment partials into d.mom[1]; one workgroup of 2 vchunks waves
// per segment (d.nseg workgroups)
bool quad_supported(const InstDesc &d);
hipError_t launch_quad(const InstDesc &d, hipStream_t st);
// batched fused stage pairs: W = 2 vchunks waves per workgroup, one (instance,
// segment) task per workgroup and turn (WaveTask.task0 = segment)
hipError_t launch_batch_pair(const InstDesc *d_descs, const WaveTask *d_tasks, int ntasks, int form, int pair, int W,
                             int blocks, hipStream_t st);
int batch_pair_blocks_per_cu(int form, int W);
// batched whole steps, the same task lists as the fused pairs
hipError_t launch_batch_quad(const InstDesc *d_descs, const WaveTask *d_tasks, int ntasks, int form, int W, int blocks,
                             hipStream_t st);
int batch_quad_blocks_per_cu(int form, int W);
// ---- diagnostics (diag_kernels.hip) ----------------------------------------
// per (segment, chunk) partials [nrowtasks][kDiagPartial] (sums with their
// Neumaier compensations in slots kDiagQ ..):
//   0..3 M0 (trace, x, y, z) summed g P - alpha gbar Pbar~ (without dz dv)
//   4 N_nu, 5 N_nubar (sum g Tr rho, sum gbar Tr rhobar), 6 sum g |dP_nu|, 7 sum g,
//   8 sum g rho_ee, 9 sum gbar rhobar_ee, 10 max |dP| over both species, 11 non-finite count
hipError_t launch_diag(const InstDesc &d, double *partials, int blocks, hipStream_t st);
// initial data of eqs:perts written into d.y
hipError_t launch_init_state(const InstDesc &d, double L, double amp, double width, double phase, hipStream_t st);
// per row and chunk [nz][vchunks][8]: dv sum D_q and dv sum v D_q, q = ee, xx, Re ex, Im ex
hipError_t launch_moments_out(const InstDesc &d, double *out, int blocks, hipStream_t st);

// number of workgroups covering all stage tasks (d.wpb waves each) / all
// (segment, chunk) tasks (kWavesPerBlock waves each)
int blocks_for(const InstDesc &d);
int row_blocks_for(const InstDesc &d);
int groups_per_wave(const InstDesc &d);

}  // namespace cosenu
