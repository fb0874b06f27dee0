// Off-path reductions over the state (FP64, fixed summation order):
// conserved quantities and error measures of Sec. 5, and the per-row angular
// moments of D = g rho - alpha gbar rhobar^*.  Same task decomposition as the
// stage kernels (row groups of lanes over v, segments of rows over z); each
// lane accumulates its bin down the segment, then the group reduces with an
// xor butterfly and lane 0 writes one partial per task.  The sums of the
// conserved quantities are compensated (Neumaier): a drift of 1e-15 relative
// has to be measurable over 5e8 cells, where plain FP64 summation would leave
// rounding noise near 1e-13.
#include <algorithm>
#include <cmath>

#include "cosenu_internal.h"

namespace cosenu {
namespace {

__device__ __forceinline__ double group_sum(double x, int lr_log2) {
    for (int off = (1 << lr_log2) >> 1; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}
// Compensated accumulation: s + c carries the sum to about twice FP64
// precision (Neumaier's variant of Kahan summation).
__device__ __forceinline__ void comp_add(double &s, double &c, double x) {
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
}
// the same over the lanes of a row group: every lane ends with the group's (s, c)
__device__ __forceinline__ void group_comp_sum(double &s, double &c, int lr_log2) {
    for (int off = (1 << lr_log2) >> 1; off > 0; off >>= 1) {
        const double so = __shfl_xor(s, off, kWave), co = __shfl_xor(c, off, kWave);
        // both lanes of a pair form the same sum (operands in lane order)
        const bool lo = (threadIdx.x & off) == 0;
        double a = lo ? s : so, ca = lo ? c : co;
        const double b = lo ? so : s, cb = lo ? co : c;
        comp_add(a, ca, b);
        s = a;
        c = ca + cb;
    }
}
__device__ __forceinline__ double group_max(double x, int lr_log2) {
    for (int off = (1 << lr_log2) >> 1; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, kWave));
    return x;
}

__global__ __launch_bounds__(kWave *kWavesPerBlock) void diag_kernel(InstDesc d, double *partials) {
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    const int G = kWave >> d.lr_log2;
    const int task = wave * G + (lane >> d.lr_log2);
    if (wave * G >= d.nrowtasks) return;
    const int l = lane & ((1 << d.lr_log2) - 1);
    const bool task_ok = task < d.nrowtasks;
    const int nz = d.nz, nv = d.nv, vchunks = d.vchunks;
    const int vc = task_ok ? task % vchunks : 0;
    const int segi = task_ok ? task / vchunks : 0;
    const int j = vc * kWave + l;
    const bool lane_on = task_ok && j < nv;
    const int jl = j < nv ? j : nv - 1;
    const int z0 = segi * d.seg;
    const int z1 = task_ok ? min(nz, z0 + d.seg) : z0;
    const double g = d.g[jl], gb = d.gb[jl], ag = d.agb[jl];
    const size_t plane = d.ps;
    double a[kDiagQ], ac[kDiagQ];  // sums (or max / count) and their compensations
#pragma unroll
    for (int q = 0; q < kDiagQ; ++q) a[q] = ac[q] = 0.0;
    if (lane_on) {
        for (int i = z0; i < z1; ++i) {
            const size_t at = (size_t)i * nv + jl;
            double o[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                o[c] = d.y[c * plane + at];
                if (!isfinite(o[c])) a[11] += 1.0;
            }
            // polarisation vectors: rho = (P0 + P.sigma)/2; Pbar~ belongs to rhobar^*
            const double P0 = o[0] + o[1], P1 = 2.0 * o[2], P2 = -2.0 * o[3], P3 = o[0] - o[1];
            const double Q0 = o[4] + o[5], Q1 = 2.0 * o[6], Q2 = 2.0 * o[7], Q3 = o[4] - o[5];
            comp_add(a[0], ac[0], g * P0 - ag * Q0);
            comp_add(a[1], ac[1], g * P1 - ag * Q1);
            comp_add(a[2], ac[2], g * P2 - ag * Q2);
            comp_add(a[3], ac[3], g * P3 - ag * Q3);
            comp_add(a[4], ac[4], g * P0);
            comp_add(a[5], ac[5], gb * Q0);
            const double dpn = fabs(sqrt(P1 * P1 + P2 * P2 + P3 * P3) - 1.0);
            const double dpb = fabs(sqrt(Q1 * Q1 + Q2 * Q2 + Q3 * Q3) - 1.0);
            comp_add(a[6], ac[6], g * dpn);
            comp_add(a[7], ac[7], g);
            comp_add(a[8], ac[8], g * o[0]);
            comp_add(a[9], ac[9], gb * o[4]);
            a[10] = fmax(a[10], fmax(dpn, dpb));
        }
    }
#pragma unroll
    for (int q = 0; q < kDiagQ; ++q) {
        if (q == 10) a[q] = group_max(a[q], d.lr_log2);
        else if (q == 11) a[q] = group_sum(a[q], d.lr_log2);  // a count: exact
        else group_comp_sum(a[q], ac[q], d.lr_log2);
    }
    if (task_ok && l == 0) {
        // sums as (value, compensation) pairs: kDiagQ values, then the compensations of the first 10
#pragma unroll
        for (int q = 0; q < kDiagQ; ++q) partials[(size_t)task * kDiagPartial + q] = a[q];
#pragma unroll
        for (int q = 0; q < 10; ++q) partials[(size_t)task * kDiagPartial + kDiagQ + q] = ac[q];
    }
}

__global__ __launch_bounds__(kWave *kWavesPerBlock) void moments_out_kernel(InstDesc d, double *out) {
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    const int G = kWave >> d.lr_log2;
    const int task = wave * G + (lane >> d.lr_log2);
    if (wave * G >= d.nrowtasks) return;
    const int l = lane & ((1 << d.lr_log2) - 1);
    const bool task_ok = task < d.nrowtasks;
    const int nz = d.nz, nv = d.nv, vchunks = d.vchunks;
    const int vc = task_ok ? task % vchunks : 0;
    const int segi = task_ok ? task / vchunks : 0;
    const int j = vc * kWave + l;
    const bool lane_on = task_ok && j < nv;
    const int jl = j < nv ? j : nv - 1;
    const int z0 = segi * d.seg;
    const int z1 = task_ok ? min(nz, z0 + d.seg) : z0;
    const double g = d.g[jl], ag = d.agb[jl], v = d.vel[jl];
    const size_t plane = d.ps;
    for (int i = z0; i < z0 + d.seg; ++i) {
        const bool row_in = i < z1;
        const int irow = min(i, nz - 1);
        const size_t at = (size_t)irow * nv + jl;
        double m[8];
        if (row_in && lane_on) {
            const double Dee = g * d.y[0 * plane + at] - ag * d.y[4 * plane + at];
            const double Dxx = g * d.y[1 * plane + at] - ag * d.y[5 * plane + at];
            const double Dre = g * d.y[2 * plane + at] - ag * d.y[6 * plane + at];
            const double Dim = g * d.y[3 * plane + at] + ag * d.y[7 * plane + at];
            m[0] = Dee; m[1] = Dxx; m[2] = Dre; m[3] = Dim;
            m[4] = v * Dee; m[5] = v * Dxx; m[6] = v * Dre; m[7] = v * Dim;
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) m[q] = 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) m[q] = group_sum(m[q], d.lr_log2);
        if (row_in && l == 0) {
#pragma unroll
            for (int q = 0; q < 8; ++q) out[((size_t)irow * vchunks + vc) * 8 + q] = m[q];
        }
    }
}

// Initial data of eqs:perts on the device: eps(z) = amp exp(-z^2/width),
// rho_ee = (1 + sqrt(1 - eps^2))/2, rho_xx = (1 - sqrt(1 - eps^2))/2,
// rho_ex = eps/2 e^{i phase}, rhobar = rho^*, identical in every bin.
__global__ void init_state_kernel(InstDesc d, double L, double amp, double width, double cph, double sph) {
    const size_t cells = (size_t)d.nz * d.nv;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t at = blockIdx.x * (size_t)blockDim.x + threadIdx.x; at < cells; at += stride) {
        const int i = (int)(at / (size_t)d.nv);
        const double z = -0.5 * L + (i + 0.5) * (L / d.nz);
        const double e = amp * exp(-z * z / width);
        const double r = sqrt(1.0 - e * e);
        const double vals[8] = {0.5 * (1.0 + r), 0.5 * (1.0 - r), 0.5 * e * cph, 0.5 * e * sph,
                                0.5 * (1.0 + r), 0.5 * (1.0 - r), 0.5 * e * cph, -0.5 * e * sph};
#pragma unroll
        for (int c = 0; c < 8; ++c) d.y[c * d.ps + at] = vals[c];
    }
}

}  // namespace

hipError_t launch_init_state(const InstDesc &d, double L, double amp, double width, double phase, hipStream_t st) {
    const size_t cells = (size_t)d.nz * d.nv;
    const int blocks = (int)std::min<size_t>((cells + 255) / 256, 65536);
    hipLaunchKernelGGL(init_state_kernel, dim3(blocks), dim3(256), 0, st, d, L, amp, width, cos(phase), sin(phase));
    return hipGetLastError();
}

hipError_t launch_diag(const InstDesc &d, double *partials, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(diag_kernel, dim3(blocks), dim3(kWave * kWavesPerBlock), 0, st, d, partials);
    return hipGetLastError();
}

hipError_t launch_moments_out(const InstDesc &d, double *out, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(moments_out_kernel, dim3(blocks), dim3(kWave * kWavesPerBlock), 0, st, d, out);
    return hipGetLastError();
}

}  // namespace cosenu
