// RK4 stage kernels of the QKE hot path for gfx950 (CDNA4).
//
// One launch evaluates the right-hand side of eq:eom at one Runge-Kutta stage
// input for every (z, v) cell and fuses the stage combine into the same pass.
//
// Layout: every array is 8 real planes [c][z][v] with v fastest, so a z row of
// one component is nv contiguous values and a wavefront reads whole rows.
// Planes are d.ps elements apart (nz*nv plus a pad that keeps concurrently
// streamed planes off a power-of-two stride).
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

// Cross-lane move of an FP64 value with a fixed DPP pattern (two 32-bit
// halves); lanes of rows outside ROW_MASK receive 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 2^lr_log2 lanes of a row group, entirely in VALU cross-lane
// moves: pairs and quads (quad_perm), eights (row_half_mirror) and sixteens
// (row_mirror) leave every lane of a 16-lane row with the same total; rows are
// then combined with row_bcast15 / row_bcast31.  The group total ends in the
// group's last lane; the association order depends only on lr_log2.
__device__ __forceinline__ double group_sum(double x, int lr_log2) {
    if (lr_log2 >= 1) x += dpp_f64<0xB1, 0xF>(x);   // quad_perm [1,0,3,2]
    if (lr_log2 >= 2) x += dpp_f64<0x4E, 0xF>(x);   // quad_perm [2,3,0,1]
    if (lr_log2 >= 3) x += dpp_f64<0x141, 0xF>(x);  // row_half_mirror
    if (lr_log2 >= 4) x += dpp_f64<0x140, 0xF>(x);  // row_mirror
    if (lr_log2 >= 5) x += dpp_f64<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
    if (lr_log2 >= 6) x += dpp_f64<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
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

// Reduce the per-lane integrands over the group; the writer is the group's
// last lane, which holds the totals.
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

// Byte-offset loads and stores from a wave-uniform base: the per-lane offset
// is 32 bits (planes are limited to 2^29 cells), so the address is formed by
// the memory unit from a scalar base plus one VGPR.
template <typename T>
__device__ __forceinline__ T ld(const char *base, uint32_t off) {
    return *reinterpret_cast<const T *>(base + off);
}
template <typename T>
__device__ __forceinline__ void st(char *base, uint32_t off, T v) {
    *reinterpret_cast<T *>(base + off) = v;
}

// Moment integrands of one species' four components for one bin: the
// neutrino part of D = g rho - alpha gbar rhobar^* is g rho, the antineutrino
// part -alpha gbar rhobar^*, so (D_ee - D_xx, Re D_ex, Im D_ex) receive
// (ca (o0 - o1), ca o2, cb o3) with ca = cb = g, or ca = -alpha gbar, cb = +alpha gbar.
__device__ __forceinline__ void species_moment_terms(const double o[4], double ca, double cb, double v,
                                                     double m[kMomQ]) {
    const double d0 = ca * (o[0] - o[1]);
    const double d1 = ca * o[2];
    const double d2 = cb * o[3];
    m[0] = d0;
    m[1] = d1;
    m[2] = d2;
    m[3] = v * d0;
    m[4] = v * d1;
    m[5] = v * d2;
}

// Interface flux from the R window rows around it (FD: rows i-1..i+2, WENO7:
// rows i-3..i+4); the upwind side of WENO7 follows the sign of v.
template <int SCHEME, typename T>
__device__ __forceinline__ T interface_flux(const T (&u)[SCHEME == 0 ? 4 : 8], T tv, bool vpos, T cv, T ce, T weps) {
    if constexpr (SCHEME == 0) {
        return fd_ko_flux<T>(u[0], u[1], u[2], u[3], cv, ce);
    } else {
        T a[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) a[q] = tv * (vpos ? u[q] : u[7 - q]);
        return weno7_flux<T>(a[0], a[1], a[2], a[3], a[4], a[5], a[6], weps);
    }
}

// Task numbering: the first d.tps tasks are neutrino groups, the next d.tps
// antineutrino groups; within a species, task = segment * vchunks + chunk.
// d.tps is padded to a multiple of the groups per wave, so a wave never mixes
// species and its component planes are wave-uniform.
struct GroupGeom {
    int sp, vc, segi, j, jl, z0, z1;
    bool task_ok, lane_on;
};

__device__ __forceinline__ GroupGeom group_geom(const InstDesc &d, int task, int l) {
    GroupGeom q;
    q.sp = task >= d.tps ? 1 : 0;
    const int t2 = task - q.sp * d.tps;
    q.task_ok = task < d.ntasks && t2 < d.nrowtasks;
    q.vc = q.task_ok ? t2 % d.vchunks : 0;
    q.segi = q.task_ok ? t2 / d.vchunks : 0;
    q.j = q.vc * kWave + l;
    q.lane_on = q.task_ok && q.j < d.nv;
    q.jl = q.j < d.nv ? q.j : d.nv - 1;
    q.z0 = q.segi * d.seg;
    q.z1 = q.task_ok ? min(d.nz, q.z0 + d.seg) : q.z0;
    return q;
}

// Everything one chunk of B rows needs from memory, loaded ahead of use.
template <typename T, int B, int NC, bool AUX0, bool AUX1>
struct ChunkBuf {
    T nw[NC][B];           // the B window rows entering with this chunk
    double a0[B][NC];      // y (or acc in stage 4) of the B produced rows
    double a1[B][NC];      // the FP64 stage input of the B rows (FP32 form, stages 2 and 4)
    double S[B][kMomQ];    // summed moment partials of the B input rows
};

// One row group of one species: march down the segment in chunks of B rows,
// software-pipelined one chunk deep.  Two chunk buffers alternate: while
// chunk c is computed, the loads of chunk c+1 (its new window rows, the FP64
// operands of its stage combine and its moment partials) are in flight, and
// the arithmetic reads straight from the buffer registers so that no copy
// forces an early wait.
template <int SCHEME, int FORM, int STAGE, int B, bool WR>
__device__ __forceinline__ void stage_body(const InstDesc &d, const GroupGeom &q, int l) {
    constexpr bool IN32 = FORM == 1 && STAGE == 2;  // Y3 of the FP32 form is stored in FP32
    using T = typename std::conditional<FORM == 0, double, float>::type;   // stencil arithmetic
    using TI = typename std::conditional<IN32, float, double>::type;      // stage input as stored
    constexpr int R = SCHEME == 0 ? 4 : 8;  // window rows of one interface flux
    constexpr int H = R / 2;
    constexpr int NC = 4;                   // components of one species
    constexpr bool AUX0 = STAGE != 0;       // y, or acc in stage 4
    constexpr bool AUX1 = false;
    // The window keeps the stage input as stored; the FP32 form rounds it to
    // FP32 where the right-hand side consumes it, and its stage combine uses
    // the exact FP64 centre value.
    using Buf = ChunkBuf<TI, B, NC, AUX0, AUX1>;

    const int nz = d.nz, nv = d.nv, vchunks = d.vchunks;
    const int sp = q.sp, z0 = q.z0, z1 = q.z1, jl = q.jl;
    const double v = d.vel[jl];
    const double gl = q.lane_on ? d.g[jl] : 0.0;
    const double agl = q.lane_on ? d.agb[jl] : 0.0;
    const double ca = sp ? -agl : gl, cb = sp ? agl : gl;
    const double sgn = sp ? -1.0 : 1.0;
    const T tv = (T)v;
    const T cv = (T)(v * (1.0 / 12.0));
    const T ce = (T)d.ko16;
    const T weps = (T)d.weno_eps;
    const bool vpos = v > 0.0;

    const size_t plane = d.ps;  // plane stride in elements (padded)
    const int cofs = sp * NC;
    const void *in = STAGE == 0 ? (const void *)d.y : (STAGE == 2 ? d.yb : d.ya);
    const char *inb = static_cast<const char *>(in) + (size_t)cofs * plane * sizeof(TI);
    const char *aux0b = reinterpret_cast<const char *>(STAGE == 3 ? d.acc : d.y) + (size_t)cofs * plane * 8;
    constexpr uint32_t out_es = (STAGE == 1 && FORM == 1) ? 4 : 8;  // element size of the stage output
    char *outb = STAGE == 0 ? static_cast<char *>(d.ya)
               : STAGE == 1 ? static_cast<char *>(d.yb)
               : STAGE == 2 ? static_cast<char *>(d.ya) : reinterpret_cast<char *>(d.y);
    outb += (size_t)cofs * plane * out_es;
    char *accw = reinterpret_cast<char *>(d.acc) + (size_t)cofs * plane * 8;
    const size_t pin = plane * sizeof(TI);   // plane strides in bytes
    const size_t p64 = plane * 8;
    const size_t pout = plane * out_es;
    const double *m_in = STAGE == 0 ? d.mom[0] : STAGE == 1 ? d.mom[1] : STAGE == 2 ? d.mom[2] : d.mom[3];
    double *m_out = STAGE == 0 ? d.mom[1] : STAGE == 1 ? d.mom[2] : STAGE == 2 ? d.mom[3] : d.mom[0];
    const int nparts = 2 * vchunks;
    // WR: one row group per wave (nv > 32), so rows and their moment partials
    // are wave-uniform and live in scalar registers

    const double dz_inv = d.dz_inv, dt = d.dt, hdt = 0.5 * d.dt, dt6 = d.dt * (1.0 / 6.0);
    const double third = 1.0 / 3.0;
    const double mudv = d.mudv, h3vac = d.h3vac, hexvac = d.hexvac, lam = d.lam;
    const int zend = z0 + d.seg;

    auto load_row = [&](int row, TI (&dst)[NC]) {
        const uint32_t off = (uint32_t)(row * nv + jl) * (uint32_t)sizeof(TI);
#pragma unroll
        for (int c = 0; c < NC; ++c) dst[c] = ld<TI>(inb + (size_t)c * pin, off);
    };

    // issue every load of the chunk starting at row i0
    auto issue = [&](int i0, Buf &cb_) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            int irow = min(i0 + b, nz - 1);
            if constexpr (WR) irow = __builtin_amdgcn_readfirstlane(irow);
            const double *mp = m_in + (size_t)irow * nparts * kMomQ;
#pragma unroll
            for (int k = 0; k < kMomQ; ++k) cb_.S[b][k] = mp[k] + mp[kMomQ + k];
            for (int p = 2; p < nparts; ++p) {
#pragma unroll
                for (int k = 0; k < kMomQ; ++k) cb_.S[b][k] += mp[p * kMomQ + k];
            }
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            // rows past a ragged segment end are not produced; their look-ahead
            // stays on the last produced row (always inside [0, 2 nz))
            const int ahead = min(i0 + b + H, z1 - 1 + H);
            TI tmp[NC];
            load_row(wrap_row(ahead, nz), tmp);
#pragma unroll
            for (int c = 0; c < NC; ++c) cb_.nw[c][b] = tmp[c];
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const uint32_t off = (uint32_t)(min(i0 + b, nz - 1) * nv + jl) * 8u;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if constexpr (AUX0) cb_.a0[b][c] = ld<double>(aux0b + (size_t)c * p64, off);
            }
        }
    };

    TI w[NC][R - 1];  // carried window rows i0-H+1 .. i0+H-1
    T fprev[NC];      // flux at i0-1/2

    // the B rows of a chunk: window row m of row i0+b is w (m < R-1-b) or the buffer
    auto compute = [&](int i0, const Buf &cb_) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = i0 + b;
            const bool row_in = i < z1;
            const int irow = min(i, nz - 1);
            auto win = [&](int c, int m) -> TI {  // window row i-H+1+m, as stored
                const int k = b + m;              // index in carried ++ buffer
                return k < R - 1 ? w[c][k] : cb_.nw[c][k - (R - 1)];
            };
            const double A0 = cb_.S[b][0] - v * cb_.S[b][3];
            const double A1 = cb_.S[b][1] - v * cb_.S[b][4];
            const double A2 = cb_.S[b][2] - v * cb_.S[b][5];
            const double h3 = h3vac + sgn * (lam + mudv * A0);
            const double hr = hexvac + sgn * (mudv * A1);
            const double hi = mudv * A2;
            double u[NC], kk[NC];  // centre values as the right-hand side sees them
#pragma unroll
            for (int c = 0; c < NC; ++c) u[c] = (double)(T)win(c, H - 1);
            minus_i_commutator(h3, hr, hi, u[0], u[1], u[2], u[3], kk[0], kk[1], kk[2], kk[3]);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                T uu[R];
#pragma unroll
                for (int m = 0; m < R; ++m) uu[m] = (T)win(c, m);
                const T fnew = interface_flux<SCHEME, T>(uu, tv, vpos, cv, ce, weps);
                kk[c] -= ((double)fnew - (double)fprev[c]) * dz_inv;
                fprev[c] = fnew;
            }
            double o[NC];
            const uint32_t off64 = (uint32_t)(irow * nv + jl) * 8u;
            const uint32_t offo = (uint32_t)(irow * nv + jl) * out_es;
            const bool on = row_in && q.lane_on;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double centre = (double)win(c, H - 1);  // exact stage input (FP64 except Y3)
                if constexpr (STAGE == 0) {
                    o[c] = centre + hdt * kk[c];
                } else if constexpr (STAGE == 1) {
                    const double y2 = centre;
                    o[c] = cb_.a0[b][c] + hdt * kk[c];
                    if (on) st<double>(accw + (size_t)c * p64, off64, ((cb_.a0[b][c] + y2) + dt * kk[c]) * third);
                } else if constexpr (STAGE == 2) {
                    o[c] = cb_.a0[b][c] + dt * kk[c];
                } else {
                    const double y4 = centre;
                    o[c] = (cb_.a0[b][c] + y4 * third) + dt6 * kk[c];
                }
                if (on) {
                    if constexpr (out_es == 8) st<double>(outb + (size_t)c * pout, offo, o[c]);
                    else st<float>(outb + (size_t)c * pout, offo, (float)o[c]);
                }
                if (FORM == 1) o[c] = (double)(float)o[c];  // the next stage sees FP32 values
                if (!on) o[c] = 0.0;
            }
            double mt[kMomQ];
            species_moment_terms(o, ca, cb, v, mt);
            write_row_moments(mt, d.lr_log2, row_in && l == (1 << d.lr_log2) - 1,
                              m_out + (((size_t)irow * vchunks + q.vc) * 2 + sp) * kMomQ);
        }
        // slide: the last R-1 rows of (carried ++ buffer) are carried on
#pragma unroll
        for (int m = 0; m < R - 1; ++m) {
#pragma unroll
            for (int c = 0; c < NC; ++c) w[c][m] = (m + B < R - 1) ? w[c][m + B] : cb_.nw[c][m + B - (R - 1)];
        }
    };

    // prologue: carried rows z0-H+1 .. z0+H-1 and the row below them, then the
    // first chunk's loads, then the flux at z0-1/2
    TI low[NC];
    load_row(wrap_row(z0 - H, nz), low);
#pragma unroll
    for (int m = 0; m < R - 1; ++m) {
        TI tmp[NC];
        load_row(wrap_row(z0 - H + 1 + m, nz), tmp);
#pragma unroll
        for (int c = 0; c < NC; ++c) w[c][m] = tmp[c];
    }
    Buf bufA, bufB;
    issue(z0, bufA);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        T u[R];
        u[0] = (T)low[c];
#pragma unroll
        for (int m = 1; m < R; ++m) u[m] = (T)w[c][m - 1];
        fprev[c] = interface_flux<SCHEME, T>(u, tv, vpos, cv, ce, weps);
    }
    for (int i0 = z0; i0 < zend; i0 += 2 * B) {
        if (i0 + B < zend) issue(i0 + B, bufB);
        compute(i0, bufA);
        if (i0 + B >= zend) break;
        if (i0 + 2 * B < zend) issue(i0 + 2 * B, bufA);
        compute(i0 + B, bufB);
    }
}

template <int SCHEME, int FORM, int STAGE, bool WR>
__device__ __forceinline__ void stage_group(const InstDesc &d, int task, int l) {
    const GroupGeom q = group_geom(d, task, l);
    stage_body<SCHEME, FORM, STAGE, kChunkRows[SCHEME], WR>(d, q, l);
}

// Moment partials of the stage-1 input (the state y) for a freshly set state,
// with exactly the arithmetic the stage-4 producer uses.
template <int FORM>
__device__ __forceinline__ void moments_group(const InstDesc &d, int task, int l) {
    const GroupGeom q = group_geom(d, task, l);
    const int nz = d.nz, nv = d.nv;
    const double v = d.vel[q.jl];
    const double gl = q.lane_on ? d.g[q.jl] : 0.0;
    const double agl = q.lane_on ? d.agb[q.jl] : 0.0;
    const double ca = q.sp ? -agl : gl, cb = q.sp ? agl : gl;
    const size_t plane = d.ps;
    const double *yb = d.y + (size_t)q.sp * 4 * plane;
    for (int i = q.z0; i < q.z0 + d.seg; ++i) {
        const bool row_in = i < q.z1;
        const int irow = min(i, nz - 1);
        const size_t at = (size_t)irow * nv + q.jl;
        double o[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double x = (row_in && q.lane_on) ? yb[c * plane + at] : 0.0;
            o[c] = FORM == 1 ? (double)(float)x : x;
        }
        double mt[kMomQ];
        species_moment_terms(o, ca, cb, v, mt);
        write_row_moments(mt, d.lr_log2, row_in && l == (1 << d.lr_log2) - 1,
                          d.mom[0] + (((size_t)irow * d.vchunks + q.vc) * 2 + q.sp) * kMomQ);
    }
}

// XCD-aware block order: the hardware deals workgroups round-robin to the 8
// XCDs; renumber so that each XCD receives a contiguous range of tasks and
// neighbouring segments (which share halo rows) meet in the same L2.  With
// reverse set, each XCD walks its range from the top: consecutive stages
// alternate direction so that a stage first reads the rows its producer
// wrote last, while they are still in the last-level cache.
__device__ __forceinline__ int xcd_block(int bid, int nblk, bool reverse) {
    const int q = nblk >> 3, r = nblk & 7;
    const int x = bid & 7, kk = bid >> 3;
    const int cnt = x < r ? q + 1 : q;
    const int start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return start + (reverse ? cnt - 1 - kk : kk);
}

template <int SCHEME, int FORM, int STAGE, bool WR>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void stage_kernel(InstDesc d) {
    const int lb = xcd_block(blockIdx.x, gridDim.x, (STAGE & 1) != 0);
    const int wave = __builtin_amdgcn_readfirstlane(lb * kWavesPerBlock + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    const int G = kWave >> d.lr_log2;
    const int task = wave * G + (lane >> d.lr_log2);
    if (wave * G >= d.ntasks) return;  // whole wave idle (uniform)
    if constexpr (WR) stage_group<SCHEME, FORM, STAGE, true>(d, wave, lane);
    else stage_group<SCHEME, FORM, STAGE, false>(d, task, lane & ((1 << d.lr_log2) - 1));
}

template <int FORM>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void moments_init_kernel(InstDesc d) {
    const int lb = xcd_block(blockIdx.x, gridDim.x, false);
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
template <int SCHEME, int FORM, int STAGE, bool WR>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void batch_stage_kernel(const InstDesc *__restrict__ descs,
                                                                           const WaveTask *__restrict__ tasks,
                                                                           int nwt) {
    const int nwaves = gridDim.x * kWavesPerBlock;
    const int lane = threadIdx.x & (kWave - 1);
    const int first = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6));
    for (int wt = first; wt < nwt; wt += nwaves) {
        const WaveTask t = tasks[wt];
        const InstDesc &d = descs[t.inst];
        if constexpr (WR) stage_group<SCHEME, FORM, STAGE, true>(d, t.task0, lane);
        else stage_group<SCHEME, FORM, STAGE, false>(d, t.task0 + (lane >> d.lr_log2), lane & ((1 << d.lr_log2) - 1));
    }
}

}  // namespace

int groups_per_wave(const InstDesc &d) { return kWave >> d.lr_log2; }

int blocks_for(const InstDesc &d) {
    const int G = groups_per_wave(d);
    const int waves = (d.ntasks + G - 1) / G;
    return (waves + kWavesPerBlock - 1) / kWavesPerBlock;
}

int row_blocks_for(const InstDesc &d) {
    const int G = groups_per_wave(d);
    const int waves = (d.nrowtasks + G - 1) / G;
    return (waves + kWavesPerBlock - 1) / kWavesPerBlock;
}

namespace {
template <int SCHEME, int FORM, bool WR>
hipError_t launch_stage_t(const InstDesc &d, int stage, dim3 grid, dim3 block, hipStream_t st) {
    switch (stage) {
        case 0: hipLaunchKernelGGL((stage_kernel<SCHEME, FORM, 0, WR>), grid, block, 0, st, d); break;
        case 1: hipLaunchKernelGGL((stage_kernel<SCHEME, FORM, 1, WR>), grid, block, 0, st, d); break;
        case 2: hipLaunchKernelGGL((stage_kernel<SCHEME, FORM, 2, WR>), grid, block, 0, st, d); break;
        default: hipLaunchKernelGGL((stage_kernel<SCHEME, FORM, 3, WR>), grid, block, 0, st, d); break;
    }
    return hipGetLastError();
}
template <int SCHEME, int FORM, bool WR>
hipError_t launch_batch_t(const InstDesc *dd, const WaveTask *tk, int nwt, int stage, dim3 grid, dim3 block,
                          hipStream_t st) {
    switch (stage) {
        case 0: hipLaunchKernelGGL((batch_stage_kernel<SCHEME, FORM, 0, WR>), grid, block, 0, st, dd, tk, nwt); break;
        case 1: hipLaunchKernelGGL((batch_stage_kernel<SCHEME, FORM, 1, WR>), grid, block, 0, st, dd, tk, nwt); break;
        case 2: hipLaunchKernelGGL((batch_stage_kernel<SCHEME, FORM, 2, WR>), grid, block, 0, st, dd, tk, nwt); break;
        default: hipLaunchKernelGGL((batch_stage_kernel<SCHEME, FORM, 3, WR>), grid, block, 0, st, dd, tk, nwt); break;
    }
    return hipGetLastError();
}
template <bool WR>
hipError_t launch_stage_w(const InstDesc &d, int stage, dim3 grid, dim3 block, hipStream_t st) {
    if (d.scheme == 0) return d.form == 0 ? launch_stage_t<0, 0, WR>(d, stage, grid, block, st)
                                          : launch_stage_t<0, 1, WR>(d, stage, grid, block, st);
    return d.form == 0 ? launch_stage_t<1, 0, WR>(d, stage, grid, block, st)
                       : launch_stage_t<1, 1, WR>(d, stage, grid, block, st);
}
template <bool WR>
hipError_t launch_batch_w(const InstDesc *dd, const WaveTask *tk, int nwt, int scheme, int form, int stage, dim3 grid,
                          dim3 block, hipStream_t st) {
    if (scheme == 0) return form == 0 ? launch_batch_t<0, 0, WR>(dd, tk, nwt, stage, grid, block, st)
                                      : launch_batch_t<0, 1, WR>(dd, tk, nwt, stage, grid, block, st);
    return form == 0 ? launch_batch_t<1, 0, WR>(dd, tk, nwt, stage, grid, block, st)
                     : launch_batch_t<1, 1, WR>(dd, tk, nwt, stage, grid, block, st);
}
}  // namespace

hipError_t launch_stage(const InstDesc &d, int stage, int blocks, hipStream_t st) {
    const dim3 grid(blocks), block(kWave * kWavesPerBlock);
    return d.lr_log2 == 6 ? launch_stage_w<true>(d, stage, grid, block, st)
                          : launch_stage_w<false>(d, stage, grid, block, st);
}

hipError_t launch_moments_init(const InstDesc &d, int blocks, hipStream_t st) {
    const dim3 grid(blocks), block(kWave * kWavesPerBlock);
    if (d.form == 0) hipLaunchKernelGGL((moments_init_kernel<0>), grid, block, 0, st, d);
    else hipLaunchKernelGGL((moments_init_kernel<1>), grid, block, 0, st, d);
    return hipGetLastError();
}

hipError_t launch_batch_stage(const InstDesc *d_descs, const WaveTask *d_tasks, int nwt, int scheme, int form,
                              bool wave_rows, int stage, int blocks, hipStream_t st) {
    const dim3 grid(blocks), block(kWave * kWavesPerBlock);
    return wave_rows ? launch_batch_w<true>(d_descs, d_tasks, nwt, scheme, form, stage, grid, block, st)
                     : launch_batch_w<false>(d_descs, d_tasks, nwt, scheme, form, stage, grid, block, st);
}

}  // namespace cosenu
