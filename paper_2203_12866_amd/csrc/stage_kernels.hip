// RK4 stage kernels of the QKE hot path for gfx950 (CDNA4).
//
// One launch evaluates the right-hand side of eq:eom at one Runge-Kutta stage
// input for every (z, v) cell and fuses the stage combine into the same pass.
//
// Layout: every array is 8 real planes [c][z][v] with v fastest, so a z row of
// one component is nv contiguous values and a wavefront reads whole rows.
//
// Work decomposition: the v bins of a row are spread over a "row group" of
// LR = min(64, pow2ceil(nv)) lanes (nv > 64: several 64-bin chunks, each its own
// group); a group marches down a segment of `seg` consecutive z rows.  The z
// stencil is a register window that slides with the march (FD: rows i-1..i+2,
// WENO7: rows i-3..i+4), so every stage input value is read from memory once
// per group plus a halo at the segment ends.  The interface flux F_{i+1/2} is
// formed once and reused for both neighbouring cells (conservative form for
// both schemes).
//
// The self-interaction needs two angular moments of every input row
// (eq:ham: the kernel 1 - v v' is separable, so H_nunu(v) = mu (M0 - v M1)).
// They are produced by the kernel that writes that row: after the stage
// combine, each group reduces its 64 bins with an xor butterfly in FP64 and
// writes one partial per (row, chunk); the consumer adds the chunk partials in
// chunk order.  The reduction order depends only on nv, so results are
// bitwise independent of the launch shape.
//
// Runge-Kutta storage (classic RK4, y_new = y + dt/6 (k1 + 2k2 + 2k3 + k4)):
//   stage 1: in y   -> Y2 = y + dt/2 k1                              (ya)
//   stage 2: in Y2  -> Y3 = y + dt/2 k2 (yb), acc = (y + Y2 + dt k2)/3
//   stage 3: in Y3  -> Y4 = y + dt k3                                 (ya)
//   stage 4: in Y4  -> y_new = acc + Y4/3 + dt/6 k4                   (y)
// which uses dt k1 = 2 (Y2 - y) and dt k3 = Y4 - y: twelve FP64 streams of
// 8 components per cell and step.  In the FP32 form Y3 is stored in FP32 (Y2
// and Y4 carry k1 and k3 and stay FP64) and every stage input is rounded to
// FP32 before the stencil, so its right-hand side is evaluated on FP32 values.
#include <type_traits>

#include "cosenu_internal.h"

namespace cosenu {
namespace {

__device__ __forceinline__ int wrap_row(int r, int nz) { return r < 0 ? r + nz : (r >= nz ? r - nz : r); }

// Sum over the lanes of a row group (xor butterfly: every lane ends with the
// same bits, since IEEE addition is commutative).
__device__ __forceinline__ double group_sum(double x, int lr_log2) {
    for (int off = (1 << lr_log2) >> 1; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    return x;
}

// Interface flux at i+1/2 whose difference gives, for cell i,
//   v (u_{i-2} - 8u_{i-1} + 8u_{i+1} - u_{i+2}) / 12  +  eps/16 (u_{i-2} - 4u_{i-1} + 6u_i - 4u_{i+1} + u_{i+2}),
// i.e. dz times the FD4 central derivative term plus the Kreiss-Oliger r = 2
// term of Sec. 3.1 (cv = v/12, ce = eps/16).
template <typename T>
__device__ __forceinline__ T fd_ko_flux(T um1, T u0, T up1, T up2, T cv, T ce) {
    const T s_in = u0 + up1, s_out = um1 + up2;
    const T d_in = u0 - up1, d_out = up2 - um1;
    return cv * (T(7) * s_in - s_out) + ce * (T(3) * d_in + d_out);
}

// Normalised WENO combination sum_r w_r q_r / sum_r w_r with w_r = d_r / s_r,
// s_r = (SI_r + eps)^2 and d = (4, 18, 12, 1)/35 (Appendix A).
template <typename T>
__device__ __forceinline__ T weno_combine(T s0, T s1, T s2, T s3, T q0, T q1, T q2, T q3);

// FP64: one division, by multiplying every weight by s0 s1 s2 s3.
template <>
__device__ __forceinline__ double weno_combine<double>(double s0, double s1, double s2, double s3, double q0,
                                                       double q1, double q2, double q3) {
    const double p01 = s0 * s1, p23 = s2 * s3;
    const double e0 = 4.0 * (s1 * p23);
    const double e1 = 18.0 * (s0 * p23);
    const double e2 = 12.0 * (p01 * s3);
    const double e3 = p01 * s2;
    const double num = (e0 * q0 + e1 * q1) + (e2 * q2 + e3 * q3);
    const double den = (e0 + e1) + (e2 + e3);
    return num / den;
}

// FP32: hardware reciprocals (the products of three s_r could leave FP32 range).
template <>
__device__ __forceinline__ float weno_combine<float>(float s0, float s1, float s2, float s3, float q0, float q1,
                                                     float q2, float q3) {
    const float w0 = 4.0f * __builtin_amdgcn_rcpf(s0);
    const float w1 = 18.0f * __builtin_amdgcn_rcpf(s1);
    const float w2 = 12.0f * __builtin_amdgcn_rcpf(s2);
    const float w3 = __builtin_amdgcn_rcpf(s3);
    const float num = (w0 * q0 + w1 * q1) + (w2 * q2 + w3 * q3);
    const float den = (w0 + w1) + (w2 + w3);
    return num * __builtin_amdgcn_rcpf(den);
}

// WENO7 reconstruction at i+1/2 from a_k = f_{i-3+k}, k = 0..6 (Appendix A).
// Computed on the stencil shifted by its centre value a_3: the smoothness
// indicators annihilate constants and every candidate reproduces them, so the
// shift is exact algebra; it removes the large common part before the
// quadratic forms (essential in FP32) and drops the terms in a_3.
template <typename T>
__device__ __forceinline__ T weno7_flux(T a0, T a1, T a2, T a3, T a4, T a5, T a6, T eps) {
    const T b0 = a0 - a3, b1 = a1 - a3, b2 = a2 - a3;
    const T b4 = a4 - a3, b5 = a5 - a3, b6 = a6 - a3;
    const T k12 = T(1.0 / 12.0);
    // fourth-order candidates on S_0..S_3 (eq:f4s), minus a_3
    const T q0 = (T(13) * b4 - T(5) * b5 + b6) * k12;
    const T q1 = (T(7) * b4 - b2 - b5) * k12;
    const T q2 = (b1 - T(5) * b2 + T(3) * b4) * k12;
    const T q3 = (T(13) * b1 - T(3) * b0 - T(23) * b2) * k12;
    // smoothness indicators (eq:Si4) with the centre value removed
    const T si0 = b4 * (T(11003) * b4 - T(17246) * b5 + T(4642) * b6) + b5 * (T(7043) * b5 - T(3882) * b6) +
                  T(547) * (b6 * b6);
    const T si1 = b2 * (T(547) * b2 + T(1922) * b4 - T(494) * b5) + b4 * (T(2843) * b4 - T(1642) * b5) +
                  T(267) * (b5 * b5);
    const T si2 = b1 * (T(267) * b1 - T(1642) * b2 - T(494) * b4) + b2 * (T(2843) * b2 + T(1922) * b4) +
                  T(547) * (b4 * b4);
    const T si3 = b0 * (T(547) * b0 - T(3882) * b1 + T(4642) * b2) + b1 * (T(7043) * b1 - T(17246) * b2) +
                  T(11003) * (b2 * b2);
    const T e0 = si0 + eps, e1 = si1 + eps, e2 = si2 + eps, e3 = si3 + eps;
    return a3 + weno_combine<T>(e0 * e0, e1 * e1, e2 * e2, e3 * e3, q0, q1, q2, q3);
}

// -i [H, rho] for a 2x2 Hermitian H = [[h_ee, h_ex], [h_ex^*, h_xx]] given by
// h3 = h_ee - h_xx and h_ex = hr + i hi (the trace of H drops out), and
// rho = [[a, b], [b^*, d]], b = br + i bi  (eq:eom).
__device__ __forceinline__ void minus_i_commutator(double h3, double hr, double hi, double a, double d, double br,
                                                   double bi, double &cee, double &cxx, double &cr, double &ci) {
    const double t = 2.0 * (hi * br - hr * bi);
    cee = t;
    cxx = -t;
    const double ad = a - d;
    cr = h3 * bi - ad * hi;
    ci = ad * hr - h3 * br;
}

// Row-moment integrands of D = g rho - alpha gbar rhobar^* for one bin:
// (D_ee - D_xx, Re D_ex, Im D_ex) and the same times v.
__device__ __forceinline__ void moment_terms(const double o[8], double g, double ag, double v, double m[kMomQ]) {
    const double d0 = g * (o[0] - o[1]) - ag * (o[4] - o[5]);
    const double d1 = g * o[2] - ag * o[6];
    const double d2 = g * o[3] + ag * o[7];
    m[0] = d0;
    m[1] = d1;
    m[2] = d2;
    m[3] = v * d0;
    m[4] = v * d1;
    m[5] = v * d2;
}

// Reduce the per-lane integrands over the group and let lane 0 write them.
__device__ __forceinline__ void write_row_moments(double m[kMomQ], int lr_log2, bool writer, double *dst) {
#pragma unroll
    for (int q = 0; q < kMomQ; ++q) m[q] = group_sum(m[q], lr_log2);
    if (writer) {
#pragma unroll
        for (int q = 0; q < kMomQ; ++q) dst[q] = m[q];
    }
}

template <typename T>
__device__ __forceinline__ T load_as(const void *base, size_t idx, bool f32) {
    if (f32) return (T)(static_cast<const float *>(base)[idx]);
    return (T)(static_cast<const double *>(base)[idx]);
}

// One row group: task -> (segment, 64-bin chunk); lane l of the group owns bin
// j = 64*chunk + l.  All lanes of a group run the same number of iterations.
template <int SCHEME, int FORM>
__device__ __forceinline__ void stage_group(const InstDesc &d, int stage, int task, int l) {
    using T = typename std::conditional<FORM == 0, double, float>::type;
    constexpr int R = SCHEME == 0 ? 4 : 8;  // window rows i-H+1 .. i+H
    constexpr int H = R / 2;

    const bool task_ok = task < d.ntasks;
    const int nz = d.nz, nv = d.nv, vchunks = d.vchunks;
    const int vc = task_ok ? task % vchunks : 0;
    const int segi = task_ok ? task / vchunks : 0;
    const int j = vc * kWave + l;
    const bool lane_on = task_ok && (j < nv);
    const int jl = j < nv ? j : nv - 1;
    const int z0 = segi * d.seg;
    const int z1 = task_ok ? min(nz, z0 + d.seg) : z0;

    const double v = d.vel[jl];
    const double g = lane_on ? d.g[jl] : 0.0;
    const double ag = lane_on ? d.agb[jl] : 0.0;
    const T tv = (T)v;
    const T cv = (T)(v * (1.0 / 12.0));
    const T ce = (T)d.ko16;
    const T weps = (T)d.weno_eps;
    const bool vpos = v > 0.0;

    // stage-dependent buffers
    const void *in;
    bool in_f32 = false;
    if (stage == 0) in = d.y;
    else if (stage == 2) { in = d.yb; in_f32 = (FORM == 1); }
    else in = d.ya;
    // (selects rather than an indexed load keep the descriptor in scalar registers)
    const double *m_in = stage == 0 ? d.mom[0] : stage == 1 ? d.mom[1] : stage == 2 ? d.mom[2] : d.mom[3];
    double *m_out = stage == 0 ? d.mom[1] : stage == 1 ? d.mom[2] : stage == 2 ? d.mom[3] : d.mom[0];

    const double dz_inv = d.dz_inv, dt = d.dt, hdt = 0.5 * d.dt, dt6 = d.dt * (1.0 / 6.0);
    const double third = 1.0 / 3.0;
    const double mudv = d.mudv, h3vac = d.h3vac, hexvac = d.hexvac, lam = d.lam;

    const size_t plane = (size_t)nz * nv;
    T w[8][R];
    T fprev[8];

    // prologue: rows z0-H .. z0+H-2 into slots 0 .. R-2
#pragma unroll
    for (int m = 0; m < R - 1; ++m) {
        const int row = wrap_row(z0 - H + m, nz);
        const size_t at = (size_t)row * nv + jl;
#pragma unroll
        for (int c = 0; c < 8; ++c) w[c][m] = load_as<T>(in, c * plane + at, in_f32);
    }

    const int iters = d.seg + 1;  // the first iteration only forms the left flux of row z0
    for (int base = 0; base < iters; base += R) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int it = base + k;
            if (it >= iters) break;
            const int i = z0 - 1 + it;  // this iteration forms F_{i+1/2} and produces row i
            {
                const int snew = (k + R - 1) % R;
                // rows past the end of a ragged segment are not produced: keep
                // their look-ahead on the last produced row (stays in [0, 2 nz))
                const int ahead = min(i + H, z1 - 1 + H);
                const size_t at = (size_t)wrap_row(ahead, nz) * nv + jl;
#pragma unroll
                for (int c = 0; c < 8; ++c) w[c][snew] = load_as<T>(in, c * plane + at, in_f32);
            }
            T fnew[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if (SCHEME == 0) {
                    fnew[c] = fd_ko_flux<T>(w[c][(k + 0) % R], w[c][(k + 1) % R], w[c][(k + 2) % R],
                                            w[c][(k + 3) % R], cv, ce);
                } else {
                    // rows i-3..i+4 are window slots (k+0..7) % R; upwind orientation by the sign of v
                    T a[7];
#pragma unroll
                    for (int q = 0; q < 7; ++q) {
                        const T up = w[c][(k + q) % R];
                        const T dn = w[c][(k + 7 - q) % R];
                        a[q] = tv * (vpos ? up : dn);
                    }
                    fnew[c] = weno7_flux<T>(a[0], a[1], a[2], a[3], a[4], a[5], a[6], weps);
                }
            }
            if (it > 0) {
                const bool row_in = i < z1;
                const bool on = row_in && lane_on;
                const int irow = min(i, nz - 1);
                const size_t at = (size_t)irow * nv + jl;
                // Hamiltonian of this row and bin (eq:ham; vacuum and matter terms per Sec. 2)
                double S[kMomQ] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                for (int p = 0; p < vchunks; ++p) {
                    const double *mp = m_in + ((size_t)irow * vchunks + p) * kMomQ;
#pragma unroll
                    for (int q = 0; q < kMomQ; ++q) S[q] += mp[q];
                }
                const double A0 = S[0] - v * S[3], A1 = S[1] - v * S[4], A2 = S[2] - v * S[5];
                const double hn3 = h3vac + lam + mudv * A0, hnr = hexvac + mudv * A1, hni = mudv * A2;
                const double hb3 = h3vac - lam - mudv * A0, hbr = hexvac - mudv * A1, hbi = mudv * A2;
                const int sc = (k + H - 1) % R;
                double u[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) u[c] = (double)w[c][sc];
                double kk[8];
                minus_i_commutator(hn3, hnr, hni, u[0], u[1], u[2], u[3], kk[0], kk[1], kk[2], kk[3]);
                minus_i_commutator(hb3, hbr, hbi, u[4], u[5], u[6], u[7], kk[4], kk[5], kk[6], kk[7]);
#pragma unroll
                for (int c = 0; c < 8; ++c) kk[c] -= ((double)fnew[c] - (double)fprev[c]) * dz_inv;

                double o[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) o[c] = 0.0;
                if (on) {
                    if (stage == 0) {
                        double *ya = static_cast<double *>(d.ya);
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            const double yc = FORM == 0 ? u[c] : d.y[c * plane + at];
                            o[c] = yc + hdt * kk[c];
                            ya[c * plane + at] = o[c];
                        }
                    } else if (stage == 1) {
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            const double yv = d.y[c * plane + at];
                            const double y2 = FORM == 0 ? u[c] : static_cast<const double *>(d.ya)[c * plane + at];
                            o[c] = yv + hdt * kk[c];
                            d.acc[c * plane + at] = ((yv + y2) + dt * kk[c]) * third;
                            if (FORM == 0) static_cast<double *>(d.yb)[c * plane + at] = o[c];
                            else static_cast<float *>(d.yb)[c * plane + at] = (float)o[c];
                        }
                    } else if (stage == 2) {
                        double *ya = static_cast<double *>(d.ya);
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            const double yv = d.y[c * plane + at];
                            o[c] = yv + dt * kk[c];
                            ya[c * plane + at] = o[c];
                        }
                    } else {
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            const double av = d.acc[c * plane + at];
                            const double y4 = FORM == 0 ? u[c] : static_cast<const double *>(d.ya)[c * plane + at];
                            o[c] = (av + y4 * third) + dt6 * kk[c];
                            d.y[c * plane + at] = o[c];
                        }
                    }
                    if (FORM == 1) {
#pragma unroll
                        for (int c = 0; c < 8; ++c) o[c] = (double)(float)o[c];  // the next stage sees FP32 values
                    }
                }
                double mt[kMomQ];
                moment_terms(o, g, ag, v, mt);
                write_row_moments(mt, d.lr_log2, row_in && l == 0,
                                  m_out + ((size_t)irow * vchunks + vc) * kMomQ);
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) fprev[c] = fnew[c];
        }
    }
}

// Moments of the stage-1 input (the state y) for a freshly set state.
template <int FORM>
__device__ __forceinline__ void moments_group(const InstDesc &d, int task, int l) {
    const bool task_ok = task < d.ntasks;
    const int nz = d.nz, nv = d.nv, vchunks = d.vchunks;
    const int vc = task_ok ? task % vchunks : 0;
    const int segi = task_ok ? task / vchunks : 0;
    const int j = vc * kWave + l;
    const bool lane_on = task_ok && (j < nv);
    const int jl = j < nv ? j : nv - 1;
    const int z0 = segi * d.seg;
    const int z1 = task_ok ? min(nz, z0 + d.seg) : z0;
    const double v = d.vel[jl];
    const double g = lane_on ? d.g[jl] : 0.0;
    const double ag = lane_on ? d.agb[jl] : 0.0;
    const size_t plane = (size_t)nz * nv;
    for (int i = z0; i < z0 + d.seg; ++i) {
        const bool row_in = i < z1;
        const int irow = min(i, nz - 1);
        const size_t at = (size_t)irow * nv + jl;
        double o[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            double x = (row_in && lane_on) ? d.y[c * plane + at] : 0.0;
            o[c] = FORM == 1 ? (double)(float)x : x;
        }
        double mt[kMomQ];
        moment_terms(o, g, ag, v, mt);
        write_row_moments(mt, d.lr_log2, row_in && l == 0, d.mom[0] + ((size_t)irow * vchunks + vc) * kMomQ);
    }
}

// XCD-aware block order: the hardware deals workgroups round-robin to the 8
// XCDs; renumber so that each XCD receives a contiguous range of tasks and
// neighbouring segments (which share halo rows) meet in the same L2.
__device__ __forceinline__ int xcd_block(int bid, int nblk) {
    const int q = nblk >> 3, r = nblk & 7;
    const int x = bid & 7, kk = bid >> 3;
    const int start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return start + kk;
}

template <int SCHEME, int FORM>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void stage_kernel(InstDesc d, int stage) {
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int wave = __builtin_amdgcn_readfirstlane(lb * kWavesPerBlock + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    const int G = kWave >> d.lr_log2;
    const int task = wave * G + (lane >> d.lr_log2);
    if (wave * G >= d.ntasks) return;  // whole wave idle (uniform)
    stage_group<SCHEME, FORM>(d, stage, task, lane & ((1 << d.lr_log2) - 1));
}

template <int FORM>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void moments_init_kernel(InstDesc d) {
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int wave = __builtin_amdgcn_readfirstlane(lb * kWavesPerBlock + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    const int G = kWave >> d.lr_log2;
    const int task = wave * G + (lane >> d.lr_log2);
    if (wave * G >= d.ntasks) return;
    moments_group<FORM>(d, task, lane & ((1 << d.lr_log2) - 1));
}

// Batched launch: a fixed grid of waves walks the wave-task list round-robin
// (the list is sorted by decreasing cost on the host).  Every wave reads its
// instance descriptor, then runs the same group code as a single instance.
// One kernel per scheme, so each gets its own register budget.
template <int SCHEME, int FORM>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void batch_stage_kernel(const InstDesc *__restrict__ descs,
                                                                           const WaveTask *__restrict__ tasks,
                                                                           int nwt, int stage) {
    const int nwaves = gridDim.x * kWavesPerBlock;
    const int lane = threadIdx.x & (kWave - 1);
    const int first = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6));
    for (int wt = first; wt < nwt; wt += nwaves) {
        const WaveTask t = tasks[wt];
        const InstDesc &d = descs[t.inst];
        stage_group<SCHEME, FORM>(d, stage, t.task0 + (lane >> d.lr_log2), lane & ((1 << d.lr_log2) - 1));
    }
}

}  // namespace

int groups_per_wave(const InstDesc &d) { return kWave >> d.lr_log2; }

int blocks_for(const InstDesc &d) {
    const int G = groups_per_wave(d);
    const int waves = (d.ntasks + G - 1) / G;
    return (waves + kWavesPerBlock - 1) / kWavesPerBlock;
}

hipError_t launch_stage(const InstDesc &d, int stage, int blocks, hipStream_t st) {
    const dim3 grid(blocks), block(kWave * kWavesPerBlock);
    if (d.scheme == 0) {
        if (d.form == 0) hipLaunchKernelGGL((stage_kernel<0, 0>), grid, block, 0, st, d, stage);
        else hipLaunchKernelGGL((stage_kernel<0, 1>), grid, block, 0, st, d, stage);
    } else {
        if (d.form == 0) hipLaunchKernelGGL((stage_kernel<1, 0>), grid, block, 0, st, d, stage);
        else hipLaunchKernelGGL((stage_kernel<1, 1>), grid, block, 0, st, d, stage);
    }
    return hipGetLastError();
}

hipError_t launch_moments_init(const InstDesc &d, int blocks, hipStream_t st) {
    const dim3 grid(blocks), block(kWave * kWavesPerBlock);
    if (d.form == 0) hipLaunchKernelGGL((moments_init_kernel<0>), grid, block, 0, st, d);
    else hipLaunchKernelGGL((moments_init_kernel<1>), grid, block, 0, st, d);
    return hipGetLastError();
}

hipError_t launch_batch_stage(const InstDesc *d_descs, const WaveTask *d_tasks, int nwt, int scheme, int form,
                              int stage, int blocks, hipStream_t st) {
    const dim3 grid(blocks), block(kWave * kWavesPerBlock);
    if (scheme == 0) {
        if (form == 0) hipLaunchKernelGGL((batch_stage_kernel<0, 0>), grid, block, 0, st, d_descs, d_tasks, nwt, stage);
        else hipLaunchKernelGGL((batch_stage_kernel<0, 1>), grid, block, 0, st, d_descs, d_tasks, nwt, stage);
    } else {
        if (form == 0) hipLaunchKernelGGL((batch_stage_kernel<1, 0>), grid, block, 0, st, d_descs, d_tasks, nwt, stage);
        else hipLaunchKernelGGL((batch_stage_kernel<1, 1>), grid, block, 0, st, d_descs, d_tasks, nwt, stage);
    }
    return hipGetLastError();
}

}  // namespace cosenu
