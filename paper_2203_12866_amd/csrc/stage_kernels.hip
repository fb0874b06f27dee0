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
// or i-2..i+3 with Kreiss-Oliger r = 3; WENO7: rows i-3..i+4), so every stage
// input value is read from memory once
// per group plus a halo at the segment ends.  The interface flux F_{i+1/2} is
// formed once and reused for both neighbouring cells (conservative form for
// both schemes).
//
// The self-interaction needs two angular moments of every input row
// (eq:ham: the kernel 1 - v v' is separable, so H_nunu(v) = mu (M0 - v M1)).
// They are produced by the kernel that writes that row: after the stage
// combine, each group reduces its bins in FP64 (through LDS and DPP when a
// row group fills a wave, by a DPP tree otherwise) and writes one partial per
// (row, chunk, species); the consumer adds the partials in a fixed order.
// The reduction order depends only on nv, so results are bitwise independent
// of the launch shape, of single versus fused stages and of batching.
//
// FD + KO with 32 < nv <= 256 also runs as fused stage pairs (pair_body):
// stages 1 + 2 and 3 + 4 each in one launch, the intermediate stage kept in
// registers and its moments exchanged between the waves of a workgroup.
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
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "cosenu_internal.h"

namespace cosenu {
namespace {

// Global-address-space views.  Pointers read from a descriptor in memory (the
// batch kernels) are otherwise generic, and generic (flat) loads also count
// against the LDS wait counter, which would tie the row prefetch to the LDS
// moment reduction.
using gchar = __attribute__((address_space(1))) char;
using gdouble = __attribute__((address_space(1))) double;

__device__ __forceinline__ int wrap_row(int r, int nz) { return r < 0 ? r + nz : (r >= nz ? r - nz : r); }

// Cross-lane move of an FP64 value with a fixed DPP pattern (two 32-bit
// halves); lanes of rows outside ROW_MASK receive 0.  With every row enabled
// no lane keeps its old value, so the move takes none (bound_ctrl set: a
// source lane out of range would read 0, as with an old value of 0), which
// spares the compiler an instruction that zeroes the destination first.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    int lo, hi;
    if constexpr (ROW_MASK == 0xF) {
        lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, true);
        hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    } else {
        lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, ROW_MASK, 0xF, false);
        hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF, false);
    }
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
// The same with the group size known at compile time (no branches).
template <int LOG>
__device__ __forceinline__ double group_sum_c(double x) {
    if constexpr (LOG >= 1) x += dpp_f64<0xB1, 0xF>(x);
    if constexpr (LOG >= 2) x += dpp_f64<0x4E, 0xF>(x);
    if constexpr (LOG >= 3) x += dpp_f64<0x141, 0xF>(x);
    if constexpr (LOG >= 4) x += dpp_f64<0x140, 0xF>(x);
    return x;
}

// Interface flux at i+1/2 whose difference gives, for cell i, dz times the
// FD4 central derivative term v (u_{i-2} - 8u_{i-1} + 8u_{i+1} - u_{i+2}) / 12
// plus the Kreiss-Oliger term Q u of Sec. 3.1.  Q u = -(-1)^r eps/2^(2r)
// delta^(2r) u / dz is the difference of the flux -(-1)^r eps/2^(2r)
// (delta^(2r-1) u)_{i+1/2}: k0 (u_i - u_{i+1}) + k1 (u_{i+2} - u_{i-1}) with
// k = (eps/4, 0) for r = 1 and (3 eps/16, eps/16) for r = 2 (cv = v/12).
template <typename T>
__device__ __forceinline__ T fd_ko_flux(T um1, T u0, T up1, T up2, T cv, T k0, T k1) {
    const T s_in = u0 + up1, s_out = um1 + up2;
    const T d_in = u0 - up1, d_out = up2 - um1;
    return cv * (T(7) * s_in - s_out) + (k0 * d_in + k1 * d_out);
}

// The same for r = 3, from six rows i-2..i+3: the KO flux is
// k0 (u_i - u_{i+1}) + k1 (u_{i+2} - u_{i-1}) + k2 (u_{i-2} - u_{i+3}) with
// k = (10, 5, 1) eps/64.
template <typename T>
__device__ __forceinline__ T fd_ko3_flux(T um2, T um1, T u0, T up1, T up2, T up3, T cv, T k0, T k1, T k2) {
    const T s_in = u0 + up1, s_out = um1 + up2;
    const T d_in = u0 - up1, d_mid = up2 - um1, d_out = um2 - up3;
    return cv * (T(7) * s_in - s_out) + ((k0 * d_in + k1 * d_mid) + k2 * d_out);
}

// Normalised WENO combination sum_r w_r q_r / sum_r w_r with w_r = d_r / s_r,
// s_r = (SI_r + eps)^2 and d = (4, 18, 12, 1)/35 (Appendix A).
template <typename T>
__device__ __forceinline__ T weno_combine(T s0, T s1, T s2, T s3, T q0, T q1, T q2, T q3);

// FP64: every weight is multiplied by s0 s1 s2 s3, which leaves one quotient.
// It is formed from the hardware reciprocal refined by one Newton step and one
// residual correction: within a few ulp, with no correctly rounded division.
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
    double r = __builtin_amdgcn_rcp(den);
    r = __builtin_fma(__builtin_fma(-den, r, 1.0), r, r);
    const double x = num * r;
    return __builtin_fma(__builtin_fma(-den, x, num), r, x);
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

// WENO7 reconstruction at i+1/2 from a_k = u_{i-3+k}, k = 0..6 (Appendix A),
// returned times v: v a_3 + (v/12) * combine(12 q_r), with tv = v, tv12 = v/12.
// Computed on the stencil shifted by its centre value a_3: the smoothness
// indicators annihilate constants and every candidate reproduces them, so the
// shift is exact algebra; it removes the large common part before the
// quadratic forms (essential in FP32) and drops the terms in a_3.  The
// candidates' common factor 1/12 leaves the normalised combination and joins
// v in the final scaling, and eps enters each indicator's last fused
// multiply-add.
template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c);
template <>
__device__ __forceinline__ double fma_t<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// One smoothness indicator plus eps, for the quadratic form
// x (c0 x + c1 y + c2 z) + y (c3 y + c4 z) + c5 z^2 of eq:Si4 written as a
// chain of fused multiply-adds.
template <typename T>
__device__ __forceinline__ T indicator(T x, T y, T z, T c0, T c1, T c2, T c3, T c4, T c5, T eps) {
    const T ix = fma_t<T>(c2, z, fma_t<T>(c1, y, c0 * x));
    const T iy = fma_t<T>(c4, z, c3 * y);
    return fma_t<T>(x, ix, fma_t<T>(y, iy, fma_t<T>(c5 * z, z, eps)));
}

template <typename T>
__device__ __forceinline__ T weno7_flux(T a0, T a1, T a2, T a3, T a4, T a5, T a6, T eps, T tv, T tv12) {
    const T b0 = a0 - a3, b1 = a1 - a3, b2 = a2 - a3;
    const T b4 = a4 - a3, b5 = a5 - a3, b6 = a6 - a3;
    // twelve times the fourth-order candidates on S_0..S_3 (eq:f4s), minus 12 a_3
    const T q0 = fma_t<T>(T(13), b4, fma_t<T>(T(-5), b5, b6));
    const T q1 = fma_t<T>(T(7), b4, -(b2 + b5));
    const T q2 = fma_t<T>(T(3), b4, fma_t<T>(T(-5), b2, b1));
    const T q3 = fma_t<T>(T(13), b1, fma_t<T>(T(-3), b0, T(-23) * b2));
    // smoothness indicators (eq:Si4) with the centre value removed, plus eps
    const T e0 = indicator<T>(b4, b5, b6, T(11003), T(-17246), T(4642), T(7043), T(-3882), T(547), eps);
    const T e1 = indicator<T>(b2, b4, b5, T(547), T(1922), T(-494), T(2843), T(-1642), T(267), eps);
    const T e2 = indicator<T>(b1, b2, b4, T(267), T(-1642), T(-494), T(2843), T(1922), T(547), eps);
    const T e3 = indicator<T>(b0, b1, b2, T(547), T(-3882), T(4642), T(7043), T(-17246), T(11003), eps);
    const T r = weno_combine<T>(e0 * e0, e1 * e1, e2 * e2, e3 * e3, q0, q1, q2, q3);
    return fma_t<T>(tv12, r, tv * a3);
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
__device__ __forceinline__ void write_row_moments(double m[kMomQ], int lr_log2, bool writer, gdouble *dst) {
#pragma unroll
    for (int q = 0; q < kMomQ; ++q) m[q] = group_sum(m[q], lr_log2);
    if (writer) {
#pragma unroll
        for (int q = 0; q < kMomQ; ++q) dst[q] = m[q];
    }
}

// Byte-offset loads and stores from a wave-uniform base: the per-lane offset
// is 32 bits (planes are limited to 2^29 cells), so the address is formed by
// the memory unit from a scalar base plus one VGPR.
template <typename T>
__device__ __forceinline__ T ld(const gchar *base, uint32_t off) {
    return *reinterpret_cast<const __attribute__((address_space(1))) T *>(base + off);
}
template <typename T>
__device__ __forceinline__ void st(gchar *base, uint32_t off, T v) {
    *reinterpret_cast<__attribute__((address_space(1))) T *>(base + off) = v;
}
// The same with the non-temporal hint, for the streams that a kernel touches
// once per cell: every stage output (read only by the next launch) and, in the
// second fused pair, acc and the y operand of stage 3.  Marked as streaming,
// they do not displace the window rows that a workgroup and its neighbours
// re-read from the caches (+7% for four single stages, +10% for the fused
// pairs on FD + KO 16384 x 128, measured; a non-temporal load of the y operand
// of a single stage was slower, so those keep the plain load).
template <typename T>
__device__ __forceinline__ void st_nt(gchar *base, uint32_t off, T v) {
    __builtin_nontemporal_store(v, reinterpret_cast<__attribute__((address_space(1))) T *>(base + off));
}
template <typename T>
__device__ __forceinline__ T ld_nt(const gchar *base, uint32_t off) {
    return __builtin_nontemporal_load(reinterpret_cast<const __attribute__((address_space(1))) T *>(base + off));
}

// Row totals of the six integrands over the 64 lanes of a wave (one row group
// per wave) through the wave's LDS scratch: every lane stores its six values;
// lane 8q + p adds the eight values of quantity q held by lanes 8p .. 8p+7;
// three DPP steps combine the eight partial sums of q (every lane of the
// eight ends with the same total) and lane 8q writes it.  The association
// order is fixed.  LDS operations of one wave complete in program order, so
// the only ordering needed is the compiler's (signal fences).  Returns, in
// lane 8q (q < 6), total q.
__device__ __forceinline__ double wave_row_totals(const double m[kMomQ], double *lds, int lane) {
#pragma unroll
    for (int q = 0; q < kMomQ; ++q) lds[q * kLdsQStride + lane] = m[q];
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    const int qq = lane >> 3, part = lane & 7;
    const double2 *src = reinterpret_cast<const double2 *>(lds + qq * kLdsQStride + part * 8);
    const double2 x0 = src[0], x1 = src[1], x2 = src[2], x3 = src[3];
    double s = ((x0.x + x0.y) + (x1.x + x1.y)) + ((x2.x + x2.y) + (x3.x + x3.y));
    s += dpp_f64<0xB1, 0xF>(s);   // quad_perm [1,0,3,2]
    s += dpp_f64<0x4E, 0xF>(s);   // quad_perm [2,3,0,1]
    s += dpp_f64<0x141, 0xF>(s);  // row_half_mirror
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return s;
}
// dst is wave-uniform: the store takes it as a scalar base with a 32-bit lane
// offset.  The empty asm keeps the compiler from folding the lane offset into a
// per-lane 64-bit pointer that lives across the march (one that did was
// spilled, and each reload waited for every store still in flight).
__device__ __forceinline__ void wave_row_moments(const double m[kMomQ], double *lds, int lane, gdouble *dst) {
    const double s = wave_row_totals(m, lds, lane);
    if ((lane & 7) == 0 && (lane >> 3) < kMomQ) {
        uint32_t off = (uint32_t)(lane >> 3) * 8u;
        asm volatile("" : "+v"(off));
        st<double>((gchar *)dst, off, s);
    }
}

// A register copy the compiler cannot coalesce with its source (the output
// operand is early-clobber, so it gets a register of its own).
__device__ __forceinline__ double fresh_copy(double x) {
    double y;
    asm("v_mov_b64 %0, %1" : "=&v"(y) : "v"(x));
    return y;
}
__device__ __forceinline__ float fresh_copy(float x) {
    float y;
    asm("v_mov_b32 %0, %1" : "=&v"(y) : "v"(x));
    return y;
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

// Interface flux from the R window rows around it (FD: rows i-1..i+2 of the
// interface i+1/2, or i-2..i+3 for KO r = 3; WENO7: rows i-3..i+4), in
// window order.
// WENO7 reconstructs f = v u.  Scaling eps by 1/v^2 makes it homogeneous of
// degree one in f, WENO7(v u; eps) = v WENO7(u; eps / v^2), so the products
// v u drop out (epsv is eps / v^2, or eps for v = 0, where the flux is 0).
// The upwind side follows the sign of v (Appendix A; v < 0 takes the stencil
// mirrored about the interface).  With MIX the lanes of a wave may upwind to
// either side and select per lane; otherwise the wave marches in its upwind
// direction, its window is already in upwind order, and nothing is selected.
// The window rows are scalar arguments (FD uses u0..u3): selecting between
// elements of an array would be lowered to an indexed read.
template <int SCHEME, bool MIX, typename T>
__device__ __forceinline__ T interface_flux(T u0, T u1, T u2, T u3, T u4, T u5, T u6, T u7, T tv, bool vpos, T cv,
                                            const T (&ko)[3], T epsv) {
    if constexpr (SCHEME == 0) {
        return fd_ko_flux<T>(u0, u1, u2, u3, cv, ko[0], ko[1]);
    } else if constexpr (SCHEME == 2) {
        return fd_ko3_flux<T>(u0, u1, u2, u3, u4, u5, cv, ko[0], ko[1], ko[2]);
    } else if constexpr (MIX) {  // cv = v/12
        return weno7_flux<T>(vpos ? u0 : u7, vpos ? u1 : u6, vpos ? u2 : u5, vpos ? u3 : u4, vpos ? u4 : u3,
                             vpos ? u5 : u2, vpos ? u6 : u1, epsv, tv, cv);
    } else {
        return weno7_flux<T>(u0, u1, u2, u3, u4, u5, u6, epsv, tv, cv);
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

// Everything one row needs from memory, loaded one row ahead of its use.
template <typename TI, int NC>
struct RowBuf {
    TI nw[NC];        // the window row entering with this row (the look-ahead row)
    double a0[NC];    // y (or acc in stage 4) of the produced row
    double S[kMomQ];  // summed moment partials of the input row
    double pv[2];     // or, with one row group per wave, its lane's two partials
};

// The moment partials of an input row come from nparts = 2 vchunks producer
// groups.  With one row group per wave they are read lane-distributed: lane
// 16 g + p holds part p of quantities g and g + 3 (zero past the parts; parts
// p + 16, p + 32, ... are added to it at load time, which only nv > 512 needs),
// one load per lane and quantity pair, and they are summed only where they are
// used, so that their load never forces an early wait on the loads issued
// after it.  A DPP sum over the 16 lanes of each g (p in pairs, then pairs of
// pairs; a fixed order) leaves every lane of the group with the totals, which
// are then read as wave-uniform values.
constexpr int kPartLanes = 16;

__device__ __forceinline__ double readlane_f64(double x, int lane) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ void sum_row_parts(const double pv[2], int plog, double S[kMomQ]) {
    const double t0 = group_sum(pv[0], plog), t1 = group_sum(pv[1], plog);
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        S[g] = readlane_f64(t0, kPartLanes * g);
        S[g + 3] = readlane_f64(t1, kPartLanes * g);
    }
}
template <int PLOG>
__device__ __forceinline__ void sum_row_parts_c(const double pv[2], double S[kMomQ]) {
    const double t0 = group_sum_c<PLOG>(pv[0]), t1 = group_sum_c<PLOG>(pv[1]);
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        S[g] = readlane_f64(t0, kPartLanes * g);
        S[g + 3] = readlane_f64(t1, kPartLanes * g);
    }
}

// One row group of one species marches through its segment, one row per step,
// software-pipelined one row deep: while row k is computed, the loads of row
// k+1 (its look-ahead window row, the FP64 operand of its stage combine and its
// moment partials) are in flight; two buffers alternate so that the arithmetic
// reads straight from the buffer registers and no copy forces an early wait.
// Step k handles row start + dir k.  dir = +1 marches up z from z0; dir = -1
// marches down from z1 - 1 with the window mirrored (WENO7 waves whose bins all
// have v < 0, so that the window is in upwind order; FD waves of odd segments,
// whose flux then takes its arguments in reverse, REV).  The flux produced at
// each step is the one on the face ahead in the march, hence the sign of dzs.
//
// XP: a row has more than 16 moment parts (nv > 512), which lanes add up in a
// loop.  Only that copy carries the loop: inside the march, the loop's extra
// control flow made the compiler wait for the loads just issued.
template <int SCHEME, int FORM, int STAGE, bool WR, bool MIX, bool REV, bool XP>
__device__ __forceinline__ void stage_body(const InstDesc &d, const GroupGeom &q, int l, int dir, double *lds) {
    constexpr bool IN32 = FORM == 1 && STAGE == 2;  // Y3 of the FP32 form is stored in FP32
    using T = typename std::conditional<FORM == 0, double, float>::type;   // stencil arithmetic
    using TI = typename std::conditional<IN32, float, double>::type;      // stage input as stored
    // Window: R rows around the current one, slot m holding row r + dir (m - CTR).
    // FD needs rows i-1..i+2 of the face i+1/2 (i-2..i+3 with KO r = 3,
    // SCHEME 2).  WENO7 needs rows i-3..i+3 of
    // the upwind-ordered stencil when it marches upwind; with MIX a lane may
    // need the mirrored one, and against the upwind direction (REV) every lane
    // does, rows i-2..i+4, so the window reaches one row further.
    constexpr int CTR = SCHEME == 0 ? 1 : SCHEME == 2 ? 2 : 3;
    constexpr int R = SCHEME == 0 ? 4 : SCHEME == 2 ? 6 : (MIX || REV ? 8 : 7);
    constexpr int AH = R - 1 - CTR;  // look-ahead distance
    constexpr int NC = 4;                   // components of one species
    constexpr bool AUX0 = STAGE != 0;       // y, or acc in stage 4
    // The window keeps the stage input as stored; the FP32 form rounds it to
    // FP32 where the right-hand side consumes it, and its stage combine uses
    // the exact FP64 centre value.  SPLIT (FP32 form, FP64 stage input): every
    // row is rounded once as it enters an FP32 window, and only the rows from
    // the centre to the look-ahead row stay in FP64 for the combine, in the
    // same registers as a full FP64 window.  (Reading the exact centre again
    // from memory instead missed the L2: 1.32x the algorithmic bytes.)
    constexpr bool SPLIT = FORM == 1 && !IN32;
    using TW = TI;
    using Buf = RowBuf<TI, NC>;

    const int nz = d.nz, nv = d.nv, vchunks = d.vchunks;
    const int sp = q.sp, jl = q.jl;
    const double v = d.vel[jl];
    const double gl = q.lane_on ? d.g[jl] : 0.0;
    const double agl = q.lane_on ? d.agb[jl] : 0.0;
    const double ca = sp ? -agl : gl, cb = sp ? agl : gl;
    const double sgn = sp ? -1.0 : 1.0;
    const T tv = (T)v;
    const T cv = (T)(v * (1.0 / 12.0));
    const T ce[3] = {(T)d.ko[0], (T)d.ko[1], (T)d.ko[2]};
    const T epsv = (T)(v != 0.0 ? d.weno_eps / (v * v) : d.weno_eps);
    const bool vpos = v > 0.0;

    const size_t plane = d.ps;  // plane stride in elements (padded)
    const int cofs = sp * NC;
    const void *in = STAGE == 0 ? (const void *)d.y : (STAGE == 2 ? d.yb : d.ya);
    const gchar *inb = (const gchar *)in + (size_t)cofs * plane * sizeof(TI);
    const gchar *aux0b = (const gchar *)(STAGE == 3 ? d.acc : d.y) + (size_t)cofs * plane * 8;
    constexpr uint32_t out_es = (STAGE == 1 && FORM == 1) ? 4 : 8;  // element size of the stage output
    gchar *outb = STAGE == 0 ? (gchar *)d.ya
                : STAGE == 1 ? (gchar *)d.yb
                : STAGE == 2 ? (gchar *)d.ya : (gchar *)d.y;
    outb += (size_t)cofs * plane * out_es;
    gchar *accw = (gchar *)d.acc + (size_t)cofs * plane * 8;
    const size_t pin = plane * sizeof(TI);   // plane strides in bytes
    const size_t p64 = plane * 8;
    const size_t pout = plane * out_es;
    const gdouble *m_in = (const gdouble *)(STAGE == 0 ? d.mom[0] : STAGE == 1 ? d.mom[1] : STAGE == 2 ? d.mom[2] : d.mom[3]);
    gdouble *m_out = (gdouble *)(STAGE == 0 ? d.mom[1] : STAGE == 1 ? d.mom[2] : STAGE == 2 ? d.mom[3] : d.mom[0]);
    const int nparts = WR ? 2 * vchunks : 2;  // without wave rows nv <= 32: one chunk
    // lane-distributed partial reads (one row group per wave): lane 16 g + p
    // reads parts p, p + 16, ... of quantities g and g + 3
    constexpr bool lanep = WR;
    const int plog = min(4, 32 - __builtin_clz(nparts - 1));  // DPP steps: log2 of the parts per lane group
    const int pg = min(l / kPartLanes, 2), pp = min(l % kPartLanes, nparts - 1);
    const bool p_on = l < 3 * kPartLanes && l % kPartLanes < nparts;
    const int poff = pp * kMomQ + pg;

    const double dzs = dir > 0 ? d.dz_inv : -d.dz_inv;
    const double dt = d.dt, hdt = 0.5 * d.dt, dt6 = d.dt * (1.0 / 6.0);
    const double third = 1.0 / 3.0;
    const double mudv = d.mudv, h3vac = d.h3vac, hexvac = d.hexvac, lam = d.lam;
    // WR: rows are wave-uniform and exactly the segment's; otherwise every
    // group of the wave takes seg steps and rows past a ragged end are not stored
    const int nrows = q.z1 - q.z0;
    const int nsteps = WR ? nrows : d.seg;
    const int start = dir > 0 ? q.z0 : q.z1 - 1;

    auto load_row = [&](int row, TI (&dst)[NC]) {
        const uint32_t off = (uint32_t)(row * nv + jl) * (uint32_t)sizeof(TI);
#pragma unroll
        for (int c = 0; c < NC; ++c) dst[c] = ld<TI>(inb + (size_t)c * pin, off);
    };

    // the moment partials of step k's input row and the FP64 operand of its
    // stage combine
    auto issue_side = [&](int k, double (&a0)[NC], double (&S)[kMomQ], double (&pv)[2]) {
        const int r = start + dir * k;
        int irow = min(max(r, 0), nz - 1);  // r < 0 only at k = nsteps (a load nobody uses)
        if constexpr (WR) irow = __builtin_amdgcn_readfirstlane(irow);
        const gdouble *mp = m_in + (size_t)irow * nparts * kMomQ;
        if constexpr (lanep) {
            // nothing uses the loaded values before the sum (lanes past the
            // parts are zeroed there), so nothing waits for these loads here
            pv[0] = mp[poff];
            pv[1] = mp[poff + 3];
            if constexpr (XP) {
                for (int pb = kPartLanes; pb < nparts; pb += kPartLanes) {
                    const int pq = pb + l % kPartLanes;
                    const bool on2 = l < 3 * kPartLanes && pq < nparts;
                    const int o2 = min(pq, nparts - 1) * kMomQ + pg;
                    const double x0 = mp[o2], x1 = mp[o2 + 3];
                    pv[0] += on2 ? x0 : 0.0;
                    pv[1] += on2 ? x1 : 0.0;
                }
            }
        } else {
#pragma unroll
            for (int m = 0; m < kMomQ; ++m) S[m] = mp[m] + mp[kMomQ + m];
            for (int p = 2; p < nparts; ++p) {
#pragma unroll
                for (int m = 0; m < kMomQ; ++m) S[m] += mp[p * kMomQ + m];
            }
        }
        const uint32_t off = (uint32_t)(irow * nv + jl) * 8u;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (AUX0) a0[c] = ld<double>(aux0b + (size_t)c * p64, off);
        }
    };
    // the window row entering at step k
    auto issue_ahead = [&](int k, TI (&nw)[NC]) {
        const int r = start + dir * k;
        // WR: the look-ahead row lies in [z0 - 1 - AH, z1 + AH] (the ends at
        // k = nsteps, loads nobody uses).  Otherwise rows past a ragged segment
        // end are not produced and their look-ahead stays on the last produced
        // row.  Both stay inside (-nz, 2 nz), since nz > AH + 1 for every scheme.
        const int ahead = WR ? r + dir * AH : min(r + AH, q.z1 - 1 + AH);
        load_row(wrap_row(ahead, nz), nw);
    };
    // every load of step k, issued one step ahead
    auto issue = [&](int k, Buf &b) {
        issue_ahead(k, b.nw);
        issue_side(k, b.a0, b.S, b.pv);
    };

    // carried window rows: w[.][m] is row r + dir (m - CTR); with SPLIT, wf
    // holds them in FP32 and wd the rows m = CTR .. R - 2 in FP64
    constexpr int NW = SPLIT ? 1 : R - 1;
    constexpr int ND = SPLIT ? R - 1 - CTR : 1;
    TW w[NC][NW];
    T wf[NC][SPLIT ? R - 1 : 1];
    double wd[NC][ND];
    T fprev[NC];      // flux on the face behind the current row

    auto compute = [&](int k, const Buf &b) {
        const int r = start + dir * k;
        const bool row_in = WR || k < nrows;
        const int irow = min(r, nz - 1);
        auto win = [&](int c, int m) -> TW {  // window row m of this step (exact; with SPLIT m >= CTR)
            if constexpr (SPLIT) return m < R - 1 ? wd[c][m - CTR] : (TW)b.nw[c];
            else return m < R - 1 ? w[c][m] : (TW)b.nw[c];
        };
        auto wlo = [&](int c, int m) -> T {  // window row m as the right-hand side sees it
            if constexpr (SPLIT) return m < R - 1 ? wf[c][m] : (T)b.nw[c];
            else return (T)win(c, m);
        };
        const double(&a0)[NC] = b.a0;
        const double(&S0)[kMomQ] = b.S;
        const double(&pv)[2] = b.pv;
        double adv[NC];  // flux differences times dir / dz
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            auto x = [&](int m) -> T { return m < R ? wlo(c, REV ? R - 1 - m : m) : T(0); };
            const T fnew = interface_flux<SCHEME, MIX, T>(x(0), x(1), x(2), x(3), x(4), x(5), x(6), x(7), tv, vpos, cv,
                                                          ce, epsv);
            adv[c] = ((double)fnew - (double)fprev[c]) * dzs;
            fprev[c] = fnew;
        }
        double S[kMomQ];
        if constexpr (lanep) {
            const double pz[2] = {p_on ? pv[0] : 0.0, p_on ? pv[1] : 0.0};
            sum_row_parts(pz, plog, S);
        } else {
#pragma unroll
            for (int m = 0; m < kMomQ; ++m) S[m] = S0[m];
        }
        const double A0 = S[0] - v * S[3];
        const double A1 = S[1] - v * S[4];
        const double A2 = S[2] - v * S[5];
        const double h3 = h3vac + sgn * (lam + mudv * A0);
        const double hr = hexvac + sgn * (mudv * A1);
        const double hi = mudv * A2;
        double u[NC], kk[NC];  // centre values as the right-hand side sees them
#pragma unroll
        for (int c = 0; c < NC; ++c) u[c] = (double)wlo(c, CTR);
        minus_i_commutator(h3, hr, hi, u[0], u[1], u[2], u[3], kk[0], kk[1], kk[2], kk[3]);
#pragma unroll
        for (int c = 0; c < NC; ++c) kk[c] -= adv[c];
        double o[NC];
        const uint32_t off64 = (uint32_t)(irow * nv + jl) * 8u;
        const uint32_t offo = (uint32_t)(irow * nv + jl) * out_es;
        const bool on = row_in && q.lane_on;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double centre = (double)win(c, CTR);  // exact stage input (FP64 except Y3)
            if constexpr (STAGE == 0) {
                o[c] = centre + hdt * kk[c];
            } else if constexpr (STAGE == 1) {
                const double y2 = centre;
                o[c] = a0[c] + hdt * kk[c];
                if (on) st_nt<double>(accw + (size_t)c * p64, off64, ((a0[c] + y2) + dt * kk[c]) * third);
            } else if constexpr (STAGE == 2) {
                o[c] = a0[c] + dt * kk[c];
            } else {
                const double y4 = centre;
                o[c] = (a0[c] + y4 * third) + dt6 * kk[c];
            }
            if (on) {
                if constexpr (out_es == 8) st_nt<double>(outb + (size_t)c * pout, offo, o[c]);
                else st_nt<float>(outb + (size_t)c * pout, offo, (float)o[c]);
            }
            if (FORM == 1) o[c] = (double)(float)o[c];  // the next stage sees FP32 values
            if (!on) o[c] = 0.0;
        }
        double mt[kMomQ];
        species_moment_terms(o, ca, cb, v, mt);
        gdouble *dst = m_out + (((size_t)irow * vchunks + q.vc) * 2 + sp) * kMomQ;
        if constexpr (WR) wave_row_moments(mt, lds, l, dst);
        else write_row_moments(mt, d.lr_log2, row_in && l == (1 << d.lr_log2) - 1, dst);
        // slide the window by one row; the entering row is copied into fresh
        // registers so that the buffer's registers are free for the next load
        // into it (else the buffer would be moved, after waiting for its
        // loads, at the loop's back edge)
        if constexpr (SPLIT) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
#pragma unroll
                for (int m = 0; m < R - 1; ++m) wf[c][m] = m < R - 2 ? wf[c][m + 1] : (T)b.nw[c];
#pragma unroll
                for (int j = 0; j < ND; ++j) wd[c][j] = j < ND - 1 ? wd[c][j + 1] : fresh_copy(b.nw[c]);
            }
        } else {
#pragma unroll
            for (int m = 0; m < R - 1; ++m) {
#pragma unroll
                for (int c = 0; c < NC; ++c) w[c][m] = m < R - 2 ? w[c][m + 1] : fresh_copy(b.nw[c]);
            }
        }
    };

    // prologue: the carried rows and the row behind them, then the first
    // step's loads, then the flux on the face behind the first row
    TI low[NC];
    load_row(wrap_row(start - dir * (CTR + 1), nz), low);
#pragma unroll
    for (int m = 0; m < R - 1; ++m) {
        TI tmp[NC];
        load_row(wrap_row(start + dir * (m - CTR), nz), tmp);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (SPLIT) {
                wf[c][m] = (T)tmp[c];
                if (m >= CTR) wd[c][m - CTR] = (double)tmp[c];
            } else {
                w[c][m] = (TW)tmp[c];
            }
        }
    }
    Buf bufA, bufB;
    issue(0, bufA);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        auto y = [&](int m) -> T {
            if constexpr (SPLIT) return m == 0 ? (T)low[c] : wf[c][m - 1];
            else return m == 0 ? (T)low[c] : (T)w[c][m - 1];
        };
        auto x = [&](int m) -> T { return m < R ? y(REV ? R - 1 - m : m) : T(0); };
        fprev[c] = interface_flux<SCHEME, MIX, T>(x(0), x(1), x(2), x(3), x(4), x(5), x(6), x(7), tv, vpos, cv, ce,
                                                  epsv);
    }
    // The loads of the next step are issued unconditionally (at k = nsteps they
    // read rows nobody uses, inside the grid): a conditional issue leaves a
    // path without them, and the compiler's wait counts, merged over both
    // paths, then wait for the loads just issued.
    for (int k = 0; k < nsteps; k += 2) {
        issue(k + 1, bufB);
        compute(k, bufA);
        if (k + 1 >= nsteps) break;
        issue(k + 2, bufA);
        compute(k + 1, bufB);
    }
}

// Direction of march.  Waves of neighbouring segments march in opposite
// directions, so that they reach their shared boundary rows at the same time
// (both at the start or both at the end of their march) and the halo rows are
// re-read from L2.  FD: even segments march up z, odd ones down (the flux then
// takes its window arguments in reverse).  WENO7 waves whose bins all share
// one sign of v: even segments march upwind (window in upwind order, 7 rows),
// odd ones against it (8 rows, arguments in reverse).  WENO7 waves whose bins
// straddle v = 0 (and every wave of a small-nv grid, whose row groups span all
// bins) march up z and select the stencil per lane.
constexpr bool kAltDir = true;
template <int SCHEME, int FORM, int STAGE, bool WR>
__device__ __forceinline__ void stage_group(const InstDesc &d, int task, int l, double *lds) {
    const GroupGeom q = group_geom(d, task, l);
    if constexpr (WR) {
        if (q.z1 <= q.z0) return;  // wave-uniform
        if (2 * d.vchunks > kPartLanes) {  // nv > 512: one copy, marching up with per-lane stencils (same fluxes)
            stage_body<SCHEME, FORM, STAGE, true, SCHEME == 1, false, true>(d, q, l, 1, lds);
            return;
        }
        if constexpr (SCHEME == 1) {
            const double v = d.vel[q.jl];
            const bool any_pos = __ballot(q.lane_on && v > 0.0) != 0;
            const bool any_neg = __ballot(q.lane_on && v < 0.0) != 0;
            const int up = any_neg ? -1 : 1;
            if (any_pos && any_neg) stage_body<SCHEME, FORM, STAGE, true, true, false, false>(d, q, l, 1, lds);
            else if (kAltDir && (q.segi & 1)) stage_body<SCHEME, FORM, STAGE, true, false, true, false>(d, q, l, -up, lds);
            else stage_body<SCHEME, FORM, STAGE, true, false, false, false>(d, q, l, up, lds);
        } else if (kAltDir && (q.segi & 1)) {
            stage_body<SCHEME, FORM, STAGE, true, false, true, false>(d, q, l, -1, lds);
        } else {
            stage_body<SCHEME, FORM, STAGE, true, false, false, false>(d, q, l, 1, lds);
        }
    } else {
        stage_body<SCHEME, FORM, STAGE, false, SCHEME == 1, false, false>(d, q, l, 1, lds);
    }
}

// Moment partials of the stage-1 input (the state y) for a freshly set state,
// with exactly the arithmetic the stage-4 producer uses.
template <int FORM, bool WR>
__device__ __forceinline__ void moments_group(const InstDesc &d, int task, int l, double *lds) {
    const GroupGeom q = group_geom(d, task, l);
    const int nz = d.nz, nv = d.nv;
    const double v = d.vel[q.jl];
    const double gl = q.lane_on ? d.g[q.jl] : 0.0;
    const double agl = q.lane_on ? d.agb[q.jl] : 0.0;
    const double ca = q.sp ? -agl : gl, cb = q.sp ? agl : gl;
    const size_t plane = d.ps;
    const gdouble *yb = (const gdouble *)d.y + (size_t)q.sp * 4 * plane;
    const int zend = WR ? q.z1 : q.z0 + d.seg;
    for (int i = q.z0; i < zend; ++i) {
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
        gdouble *dst = (gdouble *)d.mom[0] + (((size_t)irow * d.vchunks + q.vc) * 2 + q.sp) * kMomQ;
        if constexpr (WR) wave_row_moments(mt, lds, l, dst);
        else write_row_moments(mt, d.lr_log2, row_in && l == (1 << d.lr_log2) - 1, dst);
    }
}

// ---------------------------------------------------------------------------
// Fused stage pairs for FD + KO with one row group per wave (32 < nv <= 256).  Pair 0 runs stages 1 and 2, pair 1 stages 3 and 4; the
// intermediate stage value Z (Y2, or Y4) is never stored.
//
// One workgroup holds every (chunk, species) wave of one segment.  At step s
// stage A produces Z row a = start + dir (s - 2) from its input X (y, or Y3),
// and stage B produces row b = a - 2 dir of the pair's output from the last
// four Z rows, kept in registers.  Stage B needs the angular moments of Z row
// b over every chunk and species: each wave stores its six totals of row a in
// a ring of LDS slots, a barrier after every second step makes them visible,
// and two steps later every wave reads the slot lane-distributed and sums it exactly as the
// unfused stage reads the moment partials from memory.  So every value, and
// every moment partial written, is bitwise the one the four single stages
// produce.  Z covers the segment and two rows on either side (its halo for
// stage B), X four rows on either side.  Pair 1 writes the new state into the
// second state buffer (d.ya); the host swaps the two after every step.
//
// Bytes per cell and step (8 components): FP64 form 192 + 256 = 448, FP32
// form 160 + 224 = 384, against 768 and 704 for four single stages.
// ---------------------------------------------------------------------------
// LDS ring of Z moment totals: [slot][part][6].  The barrier sits between the
// slot writes and reads of every odd step.  A slot written at step s is read
// at step s + 2, after the barrier of step s or s + 1; it is rewritten at
// step s + 8, after the barrier of an odd step in s + 3 .. s + 7, which
// every wave reaches only once its read at step s + 2 is done.
constexpr int kXchSlots = 8;

// FULL (for nv a multiple of 64 with exactly 2^PLOG moment parts): bit 0
// drops the lane masks (every lane holds a bin), bit 1 the part masks (every
// lane of a part group holds a part).
template <int FORM, int PAIR, bool REV, int PLOG, int FULL>
__device__ __forceinline__ void pair_body(const InstDesc &d, int vc, int sp, int segi, int l, int dir, double *lds,
                                          double *xch) {
    constexpr bool XIN32 = FORM == 1 && PAIR == 1;  // X = Y3, stored in FP32 by the FP32 form
    using T = typename std::conditional<FORM == 0, double, float>::type;
    using TI = typename std::conditional<XIN32, float, double>::type;
    constexpr int NC = 4, R = 4, CTR = 1, AH = 2;
    const int nz = d.nz, nv = d.nv, vchunks = d.vchunks;
    const int j = vc * kWave + l;
    const bool lane_on = (FULL & 1) || j < nv;
    const int jl = lane_on ? j : nv - 1;
    const int z0 = segi * d.seg, z1 = min(nz, z0 + d.seg);
    const int nrows = z1 - z0;
    const int start = dir > 0 ? z0 : z1 - 1;  // first row of stage B
    const int nsteps = nrows + 4;

    const double v = d.vel[jl];
    const double gl = lane_on ? d.g[jl] : 0.0;
    const double agl = lane_on ? d.agb[jl] : 0.0;
    const double ca = sp ? -agl : gl, cb = sp ? agl : gl;
    const double sgn = sp ? -1.0 : 1.0;
    const T cv = (T)(v * (1.0 / 12.0));
    const T k0 = (T)d.ko[0], k1 = (T)d.ko[1];
    const size_t plane = d.ps;
    const int cofs = sp * NC;
    const gchar *xb = (const gchar *)(PAIR == 0 ? (const void *)d.y : d.yb) + (size_t)cofs * plane * sizeof(TI);
    const gchar *yb8 = (const gchar *)d.y + (size_t)cofs * plane * 8;      // y (aux of stage 3)
    const gchar *accb = (const gchar *)d.acc + (size_t)cofs * plane * 8;   // acc
    constexpr uint32_t out_es = (PAIR == 0 && FORM == 1) ? 4 : 8;          // Y3 of the FP32 form is FP32
    // pair 1 writes the new state into the other state buffer: its stage 3
    // still reads the old state on the halo rows of the segment, which the
    // neighbouring workgroups are rewriting
    gchar *outb = (PAIR == 0 ? (gchar *)d.yb : (gchar *)d.ya) + (size_t)cofs * plane * out_es;
    gchar *accw = (gchar *)d.acc + (size_t)cofs * plane * 8;
    const size_t pin = plane * sizeof(TI), p64 = plane * 8, pout = plane * out_es;
    const gdouble *m_in = (const gdouble *)(PAIR == 0 ? d.mom[0] : d.mom[2]);
    gdouble *m_out = (gdouble *)(PAIR == 0 ? d.mom[2] : d.mom[0]);
    const int nparts = 2 * vchunks;
    const int part = vc * 2 + sp;
    const int pg = min(l / kPartLanes, 2), pp = min(l % kPartLanes, nparts - 1);
    // FULL: lanes outside the three read groups sum parts that nobody reads
    const bool p_on = (FULL & 2) || (l < 3 * kPartLanes && l % kPartLanes < nparts);
    const int poff = pp * kMomQ + pg;
    // the part sums with a compile-time number of DPP steps, except in the
    // FP64 form's second pair, whose register budget the freer schedule
    // overruns (same arithmetic either way)
    constexpr bool CPLOG = !(FORM == 0 && PAIR == 1);
    const int plog = 32 - __builtin_clz(nparts - 1);
    auto part_sums = [&](const double(&pz)[2], double(&S)[kMomQ]) {
        if constexpr (CPLOG) sum_row_parts_c<PLOG>(pz, S);
        else sum_row_parts(pz, plog, S);
    };

    const double dzs = dir > 0 ? d.dz_inv : -d.dz_inv;
    const double dt = d.dt, hdt = 0.5 * d.dt, dt6 = d.dt * (1.0 / 6.0);
    const double third = 1.0 / 3.0;
    const double mudv = d.mudv, h3vac = d.h3vac, hexvac = d.hexvac, lam = d.lam;

    auto row_a = [&](int s) { return start + dir * (s - 2); };
    auto load_x = [&](int row, TI (&dst)[NC]) {
        const uint32_t off = (uint32_t)(row * nv + jl) * (uint32_t)sizeof(TI);
#pragma unroll
        for (int c = 0; c < NC; ++c) dst[c] = ld<TI>(xb + (size_t)c * pin, off);
    };
    // pair 1: acc at the stage B row.  The FP32 form loads it with the other
    // operands of its step, one step ahead into the alternating buffers; the
    // FP64 form has no registers to spare for that and loads it at the start
    // of its own step instead.
    constexpr bool ACC_AHEAD = FORM == 1;
    struct Buf {
        TI nw[NC];     // X look-ahead row a + 2 dir
        double pv[2];  // lane-distributed moment partials of X row a
        double ya[NC]; // pair 1: y at row a (stage 3 combine)
        double ac[NC]; // pair 1, FP32 form: acc at the stage B row
    };
    auto issue = [&](int s, Buf &b) {
        const int a = wrap_row(row_a(s), nz);
        load_x(wrap_row(row_a(s) + dir * AH, nz), b.nw);
        const int ar = __builtin_amdgcn_readfirstlane(a);
        const gdouble *mp = m_in + (size_t)ar * nparts * kMomQ;
        b.pv[0] = mp[poff];
        b.pv[1] = mp[poff + 3];
        if constexpr (PAIR == 1) {
            const uint32_t offa = (uint32_t)(ar * nv + jl) * 8u;
#pragma unroll
            for (int c = 0; c < NC; ++c) b.ya[c] = ld_nt<double>(yb8 + (size_t)c * p64, offa);
            if constexpr (ACC_AHEAD) {
                const int br = s >= 4 && s < nsteps ? row_a(s) - 2 * dir : start;  // in [z0, z1)
                const uint32_t offb = (uint32_t)(br * nv + jl) * 8u;
#pragma unroll
                for (int c = 0; c < NC; ++c) b.ac[c] = ld_nt<double>(accb + (size_t)c * p64, offb);
            }
        }
    };

    TI xw[NC][R - 1];   // carried X rows a - dir, a, a + dir
    double lag[NC];     // X row a - 2 dir (pair 0: y at the stage B row)
    double zw[NC][R];   // Z rows a - 3 dir .. a (dir order)
    T fA[NC], fB[NC];   // fluxes on the faces behind rows a and b

    auto flux = [&](auto x) -> T {  // FD + KO interface flux from four window rows in dir order
        return REV ? fd_ko_flux<T>(x(3), x(2), x(1), x(0), cv, k0, k1) : fd_ko_flux<T>(x(0), x(1), x(2), x(3), cv, k0, k1);
    };
    auto hamiltonian = [&](const double S[kMomQ], double &h3, double &hr, double &hi) {
        const double A0 = S[0] - v * S[3];
        const double A1 = S[1] - v * S[4];
        const double A2 = S[2] - v * S[5];
        h3 = h3vac + sgn * (lam + mudv * A0);
        hr = hexvac + sgn * (mudv * A1);
        hi = mudv * A2;
    };

    // pair 1, FP64 form: acc at the stage B row of step s, loaded at the start
    // of the step
    auto load_acc = [&](int s, double (&dst)[NC]) {
        if constexpr (PAIR == 1) {
            const int br = s >= 4 && s < nsteps ? row_a(s) - 2 * dir : start;  // stage B row (in [z0, z1) from s = 4)
            const uint32_t offb = (uint32_t)(br * nv + jl) * 8u;
#pragma unroll
            for (int c = 0; c < NC; ++c) dst[c] = ld_nt<double>(accb + (size_t)c * p64, offb);
        }
    };
    auto compute = [&](int s, const Buf &b, bool sync) {
        const int a = row_a(s);
        double abl[NC];
        if (!ACC_AHEAD && s >= 4) load_acc(s, abl);
        const double(&ab)[NC] = ACC_AHEAD ? b.ac : abl;
        // ---- stage A: Z row a
        auto win = [&](int c, int m) -> TI { return m < R - 1 ? xw[c][m] : b.nw[c]; };
        double adv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const T fn = flux([&](int m) -> T { return (T)win(c, m); });
            adv[c] = ((double)fn - (double)fA[c]) * dzs;
            fA[c] = fn;
        }
        double S[kMomQ];
        {
            const double pz[2] = {p_on ? b.pv[0] : 0.0, p_on ? b.pv[1] : 0.0};
            part_sums(pz, S);
        }
        double h3, hr, hi, u[NC], kk[NC];
        hamiltonian(S, h3, hr, hi);
#pragma unroll
        for (int c = 0; c < NC; ++c) u[c] = (double)(T)win(c, CTR);
        minus_i_commutator(h3, hr, hi, u[0], u[1], u[2], u[3], kk[0], kk[1], kk[2], kk[3]);
        double z[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            kk[c] -= adv[c];
            if constexpr (PAIR == 0) z[c] = (double)win(c, CTR) + hdt * kk[c];  // stage 1: Y2
            else z[c] = b.ya[c] + dt * kk[c];                                   // stage 3: Y4
        }
        // slide X at the end of the step (the dropped row is kept: pair 0 needs
        // y at the stage B row of the next step)
        auto slide_x = [&]() {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                lag[c] = (double)xw[c][0];
                xw[c][0] = xw[c][1];
                xw[c][1] = xw[c][2];
                xw[c][2] = fresh_copy(b.nw[c]);
            }
        };
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            zw[c][0] = zw[c][1];
            zw[c][1] = zw[c][2];
            zw[c][2] = zw[c][3];
            zw[c][3] = z[c];
        }
        // moments of Z row a for stage B (rows of the segment only)
        const bool a_in = s >= 2 && s < nrows + 2;
        if (a_in) {
            double o[NC], mt[kMomQ];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                o[c] = FORM == 1 ? (double)(float)z[c] : z[c];  // the next stage sees FP32 values
                if (!lane_on) o[c] = 0.0;
            }
            species_moment_terms(o, ca, cb, v, mt);
            const double t = wave_row_totals(mt, lds, l);
            if ((l & 7) == 0 && (l >> 3) < kMomQ) xch[((s % kXchSlots) * nparts + part) * kMomQ + (l >> 3)] = t;
        }
        if (sync) __syncthreads();
        if (s == 3) {  // flux on the face behind the first stage B row, from Z rows start - 2 dir .. start + dir
#pragma unroll
            for (int c = 0; c < NC; ++c) fB[c] = flux([&](int m) -> T { return (T)zw[c][m]; });
        }
        if (s < 4) {
            slide_x();
            return;
        }
        // ---- stage B: output row b
        const int brow = a - 2 * dir;
        double SB[kMomQ];
        {
            const double *xs = xch + ((s - 2) % kXchSlots) * nparts * kMomQ;
            const double pz[2] = {p_on ? xs[poff] : 0.0, p_on ? xs[poff + 3] : 0.0};
            part_sums(pz, SB);
        }
        // Z window of row b: rows b - dir .. b + 2 dir = zw[0..3]
        double advB[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const T fn = flux([&](int m) -> T { return (T)zw[c][m]; });
            advB[c] = ((double)fn - (double)fB[c]) * dzs;
            fB[c] = fn;
        }
        hamiltonian(SB, h3, hr, hi);
#pragma unroll
        for (int c = 0; c < NC; ++c) u[c] = (double)(T)zw[c][1];
        minus_i_commutator(h3, hr, hi, u[0], u[1], u[2], u[3], kk[0], kk[1], kk[2], kk[3]);
        const uint32_t off64 = (uint32_t)(brow * nv + jl) * 8u;
        const uint32_t offo = (uint32_t)(brow * nv + jl) * out_es;
        double o[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            kk[c] -= advB[c];
            const double zc = zw[c][1];  // exact Z at row b
            if constexpr (PAIR == 0) {   // stage 2: Y3 and acc
                o[c] = lag[c] + hdt * kk[c];
                if (lane_on) st_nt<double>(accw + (size_t)c * p64, off64, ((lag[c] + zc) + dt * kk[c]) * third);
            } else {                     // stage 4: the new state
                o[c] = (ab[c] + zc * third) + dt6 * kk[c];
            }
            if (lane_on) {
                if constexpr (out_es == 8) st_nt<double>(outb + (size_t)c * pout, offo, o[c]);
                else st_nt<float>(outb + (size_t)c * pout, offo, (float)o[c]);
            }
            if (FORM == 1) o[c] = (double)(float)o[c];
            if (!lane_on) o[c] = 0.0;
        }
        double mt[kMomQ];
        species_moment_terms(o, ca, cb, v, mt);
        wave_row_moments(mt, lds, l, m_out + (((size_t)brow * vchunks + vc) * 2 + sp) * kMomQ);
        slide_x();
    };

    // prologue: X rows a(0) - 2 dir .. a(0) + dir, then the loads of step 0,
    // then the flux on the face behind row a(0)
    const int a0 = row_a(0);
    TI low[NC];
    load_x(wrap_row(a0 - 2 * dir, nz), low);
#pragma unroll
    for (int m = 0; m < R - 1; ++m) {
        TI tmp[NC];
        load_x(wrap_row(a0 + dir * (m - CTR), nz), tmp);
#pragma unroll
        for (int c = 0; c < NC; ++c) xw[c][m] = tmp[c];
    }
    Buf bufA, bufB;
    issue(0, bufA);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        fA[c] = flux([&](int m) -> T { return m == 0 ? (T)low[c] : (T)xw[c][m - 1]; });
        lag[c] = 0.0;
        fB[c] = T(0);
#pragma unroll
        for (int m = 0; m < R; ++m) zw[c][m] = 0.0;
    }
    // The loads of the next step are issued unconditionally (past the last
    // step they read rows nobody uses, at most five rows beyond the segment,
    // which one periodic wrap keeps inside the grid since nz >= 5).  A
    // conditional issue leaves a path without those loads, and the compiler's
    // wait counts, merged over both paths, then wait for the loads just issued.
    for (int s = 0; s < nsteps; s += 2) {
        issue(s + 1, bufB);
        compute(s, bufA, false);
        if (s + 1 >= nsteps) break;
        issue(s + 2, bufA);
        compute(s + 1, bufB, true);
    }
}

// ---------------------------------------------------------------------------
// A whole RK4 step in one launch for FD + KO with one row group per wave
// (32 < nv <= 256, KO r <= 2).  The four stages march through one segment
// together, each two rows behind the one before it (the stencil's reach):
// at step s stage 1 produces Y2 row a1 = start + dir (s - 6), stage 2 Y3 row
// a1 - 2 dir, stage 3 Y4 row a1 - 4 dir and stage 4 the new state at row
// a1 - 6 dir.  Y2, Y3, Y4 and acc never leave the chip: each stage keeps the
// last four rows of its output in registers as the next stage's window, the
// moments of those rows are exchanged between the waves of the workgroup
// through three LDS rings (as in the fused pairs: written at step s, read at
// s + 2, one barrier per two steps), and acc, formed by stage 2 and consumed by
// stage 4 four steps later, waits in a per-wave LDS queue.  Halos: the new
// state over the segment needs Y4 two rows beyond it, Y3 four, Y2 six and y
// eight, so each segment recomputes 6 + 4 + 2 rows of intermediate stages.
// Every value and every moment partial is bitwise the one of four single
// stages (same expressions, same summation order).
//
// Bytes per cell and step: the state read and written once, 2 x 64 = 128 in
// both forms (32 per cell-velocity-stage update), plus the halo re-reads from
// the caches.  The new state goes to the other state buffer and its moments to
// the other moment buffer (d.ya, d.mom[1]): neighbouring workgroups still read
// the old ones in their halos.
// ---------------------------------------------------------------------------
constexpr int kAccQ = 5;  // acc rows in flight between stage 2 and stage 4

template <int FORM, bool REV, int PLOG>
__device__ __forceinline__ void quad_body(const InstDesc &d, int vc, int sp, int segi, int l, int dir, double *lds,
                                          double *xch, double *accq) {
    using T = typename std::conditional<FORM == 0, double, float>::type;  // stencils, and Y3 as stored
    constexpr int NC = 4, AH = 2, RING = kXchSlots;
    const int nz = d.nz, nv = d.nv, vchunks = d.vchunks;
    const int j = vc * kWave + l;
    const bool lane_on = j < nv;
    const int jl = lane_on ? j : nv - 1;
    const int z0 = segi * d.seg, z1 = min(nz, z0 + d.seg);
    const int nrows = z1 - z0;
    const int start = dir > 0 ? z0 : z1 - 1;  // first row of stage 4
    const int nsteps = nrows + 12;

    const double v = d.vel[jl];
    const double gl = lane_on ? d.g[jl] : 0.0;
    const double agl = lane_on ? d.agb[jl] : 0.0;
    const double ca = sp ? -agl : gl, cb = sp ? agl : gl;
    const double sgn = sp ? -1.0 : 1.0;
    const T cv = (T)(v * (1.0 / 12.0));
    const T k0 = (T)d.ko[0], k1 = (T)d.ko[1];
    const size_t plane = d.ps;
    const int cofs = sp * NC;
    const gchar *xb = (const gchar *)d.y + (size_t)cofs * plane * 8;  // the state
    gchar *outb = (gchar *)d.ya + (size_t)cofs * plane * 8;          // the new state
    const size_t p64 = plane * 8;
    const gdouble *m_in = (const gdouble *)d.mom[0];
    gdouble *m_out = (gdouble *)d.mom[1];
    const int nparts = 2 * vchunks;
    const int part = vc * 2 + sp;
    const int pg = min(l / kPartLanes, 2), pp = min(l % kPartLanes, nparts - 1);
    const bool p_on = l < 3 * kPartLanes && l % kPartLanes < nparts;
    const int poff = pp * kMomQ + pg;

    const double dzs = dir > 0 ? d.dz_inv : -d.dz_inv;
    const double dt = d.dt, hdt = 0.5 * d.dt, dt6 = d.dt * (1.0 / 6.0);
    const double third = 1.0 / 3.0;
    const double mudv = d.mudv, h3vac = d.h3vac, hexvac = d.hexvac, lam = d.lam;

    auto row1 = [&](int s) { return start + dir * (s - 6); };
    auto load_x = [&](int row, double (&dst)[NC]) {
        const uint32_t off = (uint32_t)(row * nv + jl) * 8u;
#pragma unroll
        for (int c = 0; c < NC; ++c) dst[c] = ld<double>(xb + (size_t)c * p64, off);
    };
    struct Buf {
        double nw[NC];  // y look-ahead row a1 + 2 dir
        double pv[2];   // lane-distributed moment partials of y row a1
        double y3[NC];  // y at the stage-3 row a1 - 4 dir (read again, from the caches)
    };
    auto issue = [&](int s, Buf &b) {
        const int a = row1(s);
        load_x(wrap_row(a + dir * AH, nz), b.nw);
        const int ar = __builtin_amdgcn_readfirstlane(wrap_row(a, nz));
        const gdouble *mp = m_in + (size_t)ar * nparts * kMomQ;
        b.pv[0] = mp[poff];
        b.pv[1] = mp[poff + 3];
        load_x(wrap_row(a - 4 * dir, nz), b.y3);
    };

    double xw[NC][3];  // y rows a1 - dir, a1, a1 + dir
    double lag[NC];    // y row a1 - 2 dir (the stage-2 row)
    double z1w[NC][4]; // Y2 rows a1 - 3 dir .. a1
    T z2w[NC][4];      // Y3 rows a2 - 3 dir .. a2, as the single stages store them
    double z3w[NC][4]; // Y4 rows a3 - 3 dir .. a3
    T f1[NC], f2[NC], f3[NC], f4[NC];  // fluxes on the faces behind the stage rows

    auto flux = [&](auto x) -> T {  // FD + KO interface flux from four rows in dir order
        return REV ? fd_ko_flux<T>(x(3), x(2), x(1), x(0), cv, k0, k1) : fd_ko_flux<T>(x(0), x(1), x(2), x(3), cv, k0, k1);
    };
    auto hamiltonian = [&](const double S[kMomQ], double &h3, double &hr, double &hi) {
        const double A0 = S[0] - v * S[3];
        const double A1 = S[1] - v * S[4];
        const double A2 = S[2] - v * S[5];
        h3 = h3vac + sgn * (lam + mudv * A0);
        hr = hexvac + sgn * (mudv * A1);
        hi = mudv * A2;
    };
    // the moments of a row, summed over the workgroup's waves from a ring slot
    auto ring_sums = [&](int ring, int slot, double (&S)[kMomQ]) {
        const double *xs = xch + (ring * RING + slot) * nparts * kMomQ;
        const double pz[2] = {p_on ? xs[poff] : 0.0, p_on ? xs[poff + 3] : 0.0};
        sum_row_parts_c<PLOG>(pz, S);
    };
    // this wave's moment totals of a produced row (the next stage sees FP32
    // values in the FP32 form) into a ring slot
    auto ring_put = [&](int ring, int slot, const double (&o)[NC]) {
        double oo[NC], mt[kMomQ];
#pragma unroll
        for (int c = 0; c < NC; ++c) oo[c] = lane_on ? (FORM == 1 ? (double)(float)o[c] : o[c]) : 0.0;
        species_moment_terms(oo, ca, cb, v, mt);
        const double t = wave_row_totals(mt, lds, l);
        if ((l & 7) == 0 && (l >> 3) < kMomQ) xch[((ring * RING + slot) * nparts + part) * kMomQ + (l >> 3)] = t;
    };
    // one right-hand side: -i [H, rho] - (flux difference) / dz at the centre u.
    // The flux difference is rounded in a statement of its own, as the single
    // stages round it (one expression would let the compiler fuse it into the
    // subtraction, and the results would differ in the last bit).
    auto rhs = [&](const double (&S)[kMomQ], const T (&fn)[NC], T (&fprev)[NC], const double (&u)[NC],
                   double (&kk)[NC]) {
        double adv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            adv[c] = ((double)fn[c] - (double)fprev[c]) * dzs;
            fprev[c] = fn[c];
        }
        double h3, hr, hi;
        hamiltonian(S, h3, hr, hi);
        minus_i_commutator(h3, hr, hi, u[0], u[1], u[2], u[3], kk[0], kk[1], kk[2], kk[3]);
#pragma unroll
        for (int c = 0; c < NC; ++c) kk[c] -= adv[c];
    };

    auto compute = [&](int s, const Buf &b, bool sync) {
        // ---- stage 1: Y2 row a1 = y + dt/2 k1
        {
            T fn[NC];
            double u[NC], kk[NC], S[kMomQ], z[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                fn[c] = flux([&](int m) -> T { return (T)(m < 3 ? xw[c][m] : b.nw[c]); });
                u[c] = (double)(T)xw[c][1];
            }
            const double pz[2] = {p_on ? b.pv[0] : 0.0, p_on ? b.pv[1] : 0.0};
            sum_row_parts_c<PLOG>(pz, S);
            rhs(S, fn, f1, u, kk);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                z[c] = xw[c][1] + hdt * kk[c];
                z1w[c][0] = z1w[c][1];
                z1w[c][1] = z1w[c][2];
                z1w[c][2] = z1w[c][3];
                z1w[c][3] = z[c];
            }
            if (s >= 2 && s < nrows + 10) ring_put(0, s % RING, z);
        }
        if (sync) __syncthreads();
        if (s == 3) {
#pragma unroll
            for (int c = 0; c < NC; ++c) f2[c] = flux([&](int m) -> T { return (T)z1w[c][m]; });
        }
        // ---- stage 2: Y3 row a2 = a1 - 2 dir = y + dt/2 k2; acc = (y + Y2 + dt k2) / 3
        if (s >= 4) {
            T fn[NC];
            double u[NC], kk[NC], S[kMomQ], o[NC];
            ring_sums(0, (s - 2) % RING, S);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                fn[c] = flux([&](int m) -> T { return (T)z1w[c][m]; });
                u[c] = (double)(T)z1w[c][1];
            }
            rhs(S, fn, f2, u, kk);
            double *aq = accq + (s % kAccQ) * NC * kWave + l;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                o[c] = lag[c] + hdt * kk[c];
                aq[c * kWave] = ((lag[c] + z1w[c][1]) + dt * kk[c]) * third;
                z2w[c][0] = z2w[c][1];
                z2w[c][1] = z2w[c][2];
                z2w[c][2] = z2w[c][3];
                z2w[c][3] = (T)o[c];
            }
            if (s >= 6 && s < nrows + 10) ring_put(1, s % RING, o);
        }
        if (s == 7) {
#pragma unroll
            for (int c = 0; c < NC; ++c) f3[c] = flux([&](int m) -> T { return z2w[c][m]; });
        }
        // ---- stage 3: Y4 row a3 = a1 - 4 dir = y + dt k3
        if (s >= 8) {
            T fn[NC];
            double u[NC], kk[NC], S[kMomQ], o[NC];
            ring_sums(1, (s - 2) % RING, S);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                fn[c] = flux([&](int m) -> T { return z2w[c][m]; });
                u[c] = (double)z2w[c][1];
            }
            rhs(S, fn, f3, u, kk);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                o[c] = b.y3[c] + dt * kk[c];
                z3w[c][0] = z3w[c][1];
                z3w[c][1] = z3w[c][2];
                z3w[c][2] = z3w[c][3];
                z3w[c][3] = o[c];
            }
            if (s >= 10 && s < nrows + 10) ring_put(2, s % RING, o);
        }
        if (s == 11) {
#pragma unroll
            for (int c = 0; c < NC; ++c) f4[c] = flux([&](int m) -> T { return (T)z3w[c][m]; });
        }
        // ---- stage 4: the new state at row a4 = a1 - 6 dir = (acc + Y4/3) + dt/6 k4
        if (s >= 12) {
            T fn[NC];
            double u[NC], kk[NC], S[kMomQ], o[NC];
            ring_sums(2, (s - 2) % RING, S);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                fn[c] = flux([&](int m) -> T { return (T)z3w[c][m]; });
                u[c] = (double)(T)z3w[c][1];
            }
            rhs(S, fn, f4, u, kk);
            const int brow = row1(s) - 6 * dir;  // in [z0, z1)
            const uint32_t off = (uint32_t)(brow * nv + jl) * 8u;
            const double *aq = accq + ((s - 4) % kAccQ) * NC * kWave + l;  // acc of this row, from step s - 4
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                o[c] = (aq[c * kWave] + z3w[c][1] * third) + dt6 * kk[c];
                if (lane_on) st_nt<double>(outb + (size_t)c * p64, off, o[c]);
                if (FORM == 1) o[c] = (double)(float)o[c];
                if (!lane_on) o[c] = 0.0;
            }
            double mt[kMomQ];
            species_moment_terms(o, ca, cb, v, mt);
            wave_row_moments(mt, lds, l, m_out + (((size_t)brow * vchunks + vc) * 2 + sp) * kMomQ);
        }
        // slide the y window; the dropped row is the next step's stage-2 row
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            lag[c] = xw[c][0];
            xw[c][0] = xw[c][1];
            xw[c][1] = xw[c][2];
            xw[c][2] = fresh_copy(b.nw[c]);
        }
    };

    // prologue: y rows a1(0) - 2 dir .. a1(0) + dir, the loads of step 0, and
    // the flux on the face behind row a1(0)
    const int a0 = row1(0);
    double low[NC];
    load_x(wrap_row(a0 - 2 * dir, nz), low);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        double tmp[NC];
        load_x(wrap_row(a0 + dir * (m - 1), nz), tmp);
#pragma unroll
        for (int c = 0; c < NC; ++c) xw[c][m] = tmp[c];
    }
    Buf bufA, bufB;
    issue(0, bufA);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        f1[c] = flux([&](int m) -> T { return (T)(m == 0 ? low[c] : xw[c][m - 1]); });
        f2[c] = f3[c] = f4[c] = T(0);
        lag[c] = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            z1w[c][m] = 0.0;
            z2w[c][m] = T(0);
            z3w[c][m] = 0.0;
        }
    }
    // The next step's loads are issued unconditionally (past the last step they
    // read rows nobody uses, at most eight rows beyond the segment, inside one
    // periodic wrap since nz >= 16), so the compiler's wait counts never wait
    // for loads just issued.
    for (int s = 0; s < nsteps; s += 2) {
        issue(s + 1, bufB);
        compute(s, bufA, false);
        if (s + 1 >= nsteps) break;
        issue(s + 2, bufA);
        compute(s + 1, bufB, true);
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

// LDS scratch of the wave-row moment reduction (WR kernels only).
template <bool WR>
__device__ __forceinline__ double *wave_lds(double *pool) {
    return WR ? pool + (threadIdx.x >> 6) * kLdsPerWave : nullptr;
}

// Register budgets (waves per SIMD): FD with KO r <= 2 4 (128 VGPRs) with one
// row group per wave, else 3 (168 VGPRs); WENO7 and FD with KO r = 3 (two more
// window rows) 3, else 2.
template <int SCHEME, bool WR>
constexpr int kMinWavesPerSimd = SCHEME == 0 ? (WR ? 4 : 3) : (WR ? 3 : 2);

// Single-instance launches: workgroups of d.wpb waves (1, 2 or 4, a launch
// shape the autotuner picks), with d.wpb wave scratches of dynamic LDS for the
// wave-row moment reduction.
template <int SCHEME, int FORM, int STAGE, bool WR>
__global__ __launch_bounds__(kWave *kWavesPerBlock, (kMinWavesPerSimd<SCHEME, WR>)) void stage_kernel(InstDesc d) {
    extern __shared__ __align__(16) double stage_pool[];
    const int lb = xcd_block(blockIdx.x, gridDim.x, (STAGE & 1) != 0);
    const int wave = __builtin_amdgcn_readfirstlane(lb * d.wpb + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    const int G = kWave >> d.lr_log2;
    const int task = wave * G + (lane >> d.lr_log2);
    if (wave * G >= d.ntasks) return;  // whole wave idle (uniform)
    if constexpr (WR) stage_group<SCHEME, FORM, STAGE, true>(d, wave, lane, wave_lds<true>(stage_pool));
    else stage_group<SCHEME, FORM, STAGE, false>(d, task, lane & ((1 << d.lr_log2) - 1), nullptr);
}

template <int FORM, bool WR>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void moments_init_kernel(InstDesc d) {
    extern __shared__ __align__(16) double stage_pool[];
    double *pool = stage_pool;
    const int lb = xcd_block(blockIdx.x, gridDim.x, false);
    const int wave = __builtin_amdgcn_readfirstlane(lb * d.wpb + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    const int G = kWave >> d.lr_log2;
    const int task = wave * G + (lane >> d.lr_log2);
    if (wave * G >= d.ntasks) return;
    if constexpr (WR) moments_group<FORM, true>(d, wave, lane, wave_lds<true>(pool));
    else moments_group<FORM, false>(d, task, lane & ((1 << d.lr_log2) - 1), nullptr);
}

// Batched launch: a fixed grid of waves walks the wave-task list round-robin
// (the list is sorted by decreasing cost on the host).  Every wave reads its
// instance descriptor, then runs the same group code as a single instance.
// One kernel per scheme, so each gets its own register budget.
template <int SCHEME, int FORM, int STAGE, bool WR>
__global__ __launch_bounds__(kWave *kWavesPerBlock, (kMinWavesPerSimd<SCHEME, WR>)) void batch_stage_kernel(const InstDesc *__restrict__ descs,
                                                                           const WaveTask *__restrict__ tasks,
                                                                           int nwt) {
    __shared__ __align__(16) double pool[WR ? kWavesPerBlock * kLdsPerWave : 2];
    const int nwaves = gridDim.x * kWavesPerBlock;
    const int lane = threadIdx.x & (kWave - 1);
    const int first = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6));
    for (int wt = first; wt < nwt; wt += nwaves) {
        const WaveTask t = tasks[wt];
        const InstDesc &d = descs[t.inst];
        if constexpr (WR) stage_group<SCHEME, FORM, STAGE, true>(d, t.task0, lane, wave_lds<true>(pool));
        else stage_group<SCHEME, FORM, STAGE, false>(d, t.task0 + (lane >> d.lr_log2), lane & ((1 << d.lr_log2) - 1),
                                                     nullptr);
    }
}

// Fused stage pairs: one workgroup per segment, one wave per (chunk, species);
// 2^PLOG >= 2 vchunks moment parts per row, so at most 2^PLOG waves.
template <int FORM, int PAIR, int PLOG, int FULL>
__global__ __launch_bounds__(kWave * (1 << PLOG), 3) void pair_kernel(InstDesc d) {
    extern __shared__ __align__(16) double pair_pool[];
    const int nw = blockDim.x >> 6;  // 2 vchunks
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    const int segi = xcd_block(blockIdx.x, gridDim.x, PAIR == 1);
    double *lds = pair_pool + w * kLdsPerWave;
    double *xch = pair_pool + nw * kLdsPerWave;
    const int vc = w >> 1, sp = w & 1;
    if (kAltDir && (segi & 1)) pair_body<FORM, PAIR, true, PLOG, FULL>(d, vc, sp, segi, lane, -1, lds, xch);
    else pair_body<FORM, PAIR, false, PLOG, FULL>(d, vc, sp, segi, lane, 1, lds, xch);
}

// A whole RK4 step per launch: one workgroup per segment, one wave per
// (chunk, species); LDS holds each wave's scratch, the three moment rings and
// each wave's acc queue.
template <int FORM, int PLOG>
__global__ __launch_bounds__(kWave * (1 << PLOG), 2) void quad_kernel(InstDesc d) {
    extern __shared__ __align__(16) double quad_pool[];
    const int nw = blockDim.x >> 6;  // 2 vchunks
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    const int segi = xcd_block(blockIdx.x, gridDim.x, false);
    double *lds = quad_pool + w * kLdsPerWave;
    double *xch = quad_pool + nw * kLdsPerWave;
    double *accq = xch + 3 * kXchSlots * nw * kMomQ + w * (kAccQ * 4 * kWave);
    const int vc = w >> 1, sp = w & 1;
    if (kAltDir && (segi & 1)) quad_body<FORM, true, PLOG>(d, vc, sp, segi, lane, -1, lds, xch, accq);
    else quad_body<FORM, false, PLOG>(d, vc, sp, segi, lane, 1, lds, xch, accq);
}

// Batched whole steps: a persistent grid of workgroups of 2 vchunks waves
// walks a list of (instance, segment) tasks, sorted by decreasing cost on the
// host, of instances that all have that many waves per segment.
template <int FORM, int PLOG>
__global__ __launch_bounds__(kWave * (1 << PLOG), 2) void batch_quad_kernel(const InstDesc *__restrict__ descs,
                                                                             const WaveTask *__restrict__ tasks,
                                                                             int ntasks) {
    extern __shared__ __align__(16) double quad_pool[];
    const int nw = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    double *lds = quad_pool + w * kLdsPerWave;
    double *xch = quad_pool + nw * kLdsPerWave;
    double *accq = xch + 3 * kXchSlots * nw * kMomQ + w * (kAccQ * 4 * kWave);
    const int vc = w >> 1, sp = w & 1;
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const WaveTask tk = tasks[t];
        const InstDesc &d = descs[tk.inst];
        const int segi = tk.task0;
        if (kAltDir && (segi & 1)) quad_body<FORM, true, PLOG>(d, vc, sp, segi, lane, -1, lds, xch, accq);
        else quad_body<FORM, false, PLOG>(d, vc, sp, segi, lane, 1, lds, xch, accq);
        __syncthreads();  // the next task rewrites the LDS rings and queues from their first slots
    }
}

// Batched fused stage pairs: a persistent grid of workgroups of 2 vchunks
// waves walks a list of (instance, segment) tasks, sorted by decreasing cost
// on the host, of instances that all have that many waves per segment.
template <int FORM, int PAIR, int PLOG>
__global__ __launch_bounds__(kWave * (1 << PLOG), 3) void batch_pair_kernel(const InstDesc *__restrict__ descs,
                                                                             const WaveTask *__restrict__ tasks,
                                                                             int ntasks) {
    extern __shared__ __align__(16) double pair_pool[];
    const int nw = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & (kWave - 1);
    double *lds = pair_pool + w * kLdsPerWave;
    double *xch = pair_pool + nw * kLdsPerWave;
    const int vc = w >> 1, sp = w & 1;
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const WaveTask tk = tasks[t];
        const InstDesc &d = descs[tk.inst];
        const int segi = tk.task0;
        if (kAltDir && (segi & 1)) pair_body<FORM, PAIR, true, PLOG, 0>(d, vc, sp, segi, lane, -1, lds, xch);
        else pair_body<FORM, PAIR, false, PLOG, 0>(d, vc, sp, segi, lane, 1, lds, xch);
        __syncthreads();  // the next task rewrites the LDS ring from its first slot
    }
}

}  // namespace

int groups_per_wave(const InstDesc &d) { return kWave >> d.lr_log2; }

int blocks_for(const InstDesc &d) {
    const int G = groups_per_wave(d);
    const int waves = (d.ntasks + G - 1) / G;
    return (waves + d.wpb - 1) / d.wpb;
}

int row_blocks_for(const InstDesc &d) {
    const int G = groups_per_wave(d);
    const int waves = (d.nrowtasks + G - 1) / G;
    return (waves + kWavesPerBlock - 1) / kWavesPerBlock;
}

namespace {
// dynamic LDS of a single-instance stage or moment launch: one wave scratch per
// wave with one row group per wave, none otherwise
size_t stage_shm_bytes(const InstDesc &d) {
    return d.lr_log2 == 6 ? (size_t)d.wpb * kLdsPerWave * sizeof(double) : 0;
}
template <int SCHEME, int FORM, bool WR>
hipError_t launch_stage_t(const InstDesc &d, int stage, dim3 grid, dim3 block, hipStream_t st) {
    const size_t shm = stage_shm_bytes(d);
    switch (stage) {
        case 0: hipLaunchKernelGGL((stage_kernel<SCHEME, FORM, 0, WR>), grid, block, shm, st, d); break;
        case 1: hipLaunchKernelGGL((stage_kernel<SCHEME, FORM, 1, WR>), grid, block, shm, st, d); break;
        case 2: hipLaunchKernelGGL((stage_kernel<SCHEME, FORM, 2, WR>), grid, block, shm, st, d); break;
        default: hipLaunchKernelGGL((stage_kernel<SCHEME, FORM, 3, WR>), grid, block, shm, st, d); break;
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
    if (d.scheme == 2) return d.form == 0 ? launch_stage_t<2, 0, WR>(d, stage, grid, block, st)
                                          : launch_stage_t<2, 1, WR>(d, stage, grid, block, st);
    return d.form == 0 ? launch_stage_t<1, 0, WR>(d, stage, grid, block, st)
                       : launch_stage_t<1, 1, WR>(d, stage, grid, block, st);
}
template <bool WR>
hipError_t launch_batch_w(const InstDesc *dd, const WaveTask *tk, int nwt, int scheme, int form, int stage, dim3 grid,
                          dim3 block, hipStream_t st) {
    if (scheme == 0) return form == 0 ? launch_batch_t<0, 0, WR>(dd, tk, nwt, stage, grid, block, st)
                                      : launch_batch_t<0, 1, WR>(dd, tk, nwt, stage, grid, block, st);
    if (scheme == 2) return form == 0 ? launch_batch_t<2, 0, WR>(dd, tk, nwt, stage, grid, block, st)
                                      : launch_batch_t<2, 1, WR>(dd, tk, nwt, stage, grid, block, st);
    return form == 0 ? launch_batch_t<1, 0, WR>(dd, tk, nwt, stage, grid, block, st)
                     : launch_batch_t<1, 1, WR>(dd, tk, nwt, stage, grid, block, st);
}
}  // namespace

hipError_t launch_stage(const InstDesc &d, int stage, int blocks, hipStream_t st) {
    if (d.wpb != 1 && d.wpb != 2 && d.wpb != 4) return hipErrorInvalidValue;
    const dim3 grid(blocks), block(kWave * d.wpb);
    return d.lr_log2 == 6 ? launch_stage_w<true>(d, stage, grid, block, st)
                          : launch_stage_w<false>(d, stage, grid, block, st);
}

hipError_t launch_moments_init(const InstDesc &d, int blocks, hipStream_t st) {
    if (d.wpb != 1 && d.wpb != 2 && d.wpb != 4) return hipErrorInvalidValue;
    const dim3 grid(blocks), block(kWave * d.wpb);
    const size_t shm = stage_shm_bytes(d);
    const bool wr = d.lr_log2 == 6;
    if (d.form == 0) {
        if (wr) hipLaunchKernelGGL((moments_init_kernel<0, true>), grid, block, shm, st, d);
        else hipLaunchKernelGGL((moments_init_kernel<0, false>), grid, block, shm, st, d);
    } else {
        if (wr) hipLaunchKernelGGL((moments_init_kernel<1, true>), grid, block, shm, st, d);
        else hipLaunchKernelGGL((moments_init_kernel<1, false>), grid, block, shm, st, d);
    }
    return hipGetLastError();
}

namespace {
template <int SCHEME, int FORM, bool WR>
int batch_waves_per_cu_t() {
    int lo = 1 << 30;
    auto one = [&](const void *fn) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kWave * kWavesPerBlock, 0) == hipSuccess && nb > 0)
            lo = std::min(lo, nb * kWavesPerBlock);
    };
    one(reinterpret_cast<const void *>(batch_stage_kernel<SCHEME, FORM, 0, WR>));
    one(reinterpret_cast<const void *>(batch_stage_kernel<SCHEME, FORM, 1, WR>));
    one(reinterpret_cast<const void *>(batch_stage_kernel<SCHEME, FORM, 2, WR>));
    one(reinterpret_cast<const void *>(batch_stage_kernel<SCHEME, FORM, 3, WR>));
    return lo == (1 << 30) ? 2 * kWavesPerBlock : lo;
}
template <bool WR>
int batch_waves_per_cu_w(int scheme, int form) {
    if (scheme == 0) return form == 0 ? batch_waves_per_cu_t<0, 0, WR>() : batch_waves_per_cu_t<0, 1, WR>();
    if (scheme == 2) return form == 0 ? batch_waves_per_cu_t<2, 0, WR>() : batch_waves_per_cu_t<2, 1, WR>();
    return form == 0 ? batch_waves_per_cu_t<1, 0, WR>() : batch_waves_per_cu_t<1, 1, WR>();
}
}  // namespace

int batch_waves_per_cu(int scheme, int form, bool wave_rows) {
    return wave_rows ? batch_waves_per_cu_w<true>(scheme, form) : batch_waves_per_cu_w<false>(scheme, form);
}

bool pair_supported(const InstDesc &d) { return d.scheme == 0 && d.nz >= 5 && d.lr_log2 == 6 && 2 * d.vchunks <= 8; }

namespace {
template <int FORM, int PAIR>
hipError_t launch_pair_t(const InstDesc &d, dim3 grid, dim3 block, size_t shm, hipStream_t st) {
    const int W = (int)block.x / kWave;  // moment parts per row, 2 vchunks
    // mask-free copies in the FP32 form only (both masks in its second pair,
    // the part masks in its first): elsewhere the registers they free are
    // taken by a freer schedule, which spills
    constexpr int kFull = FORM == 1 ? (PAIR == 1 ? 3 : 2) : 0;
    const bool full = kFull != 0 && d.nv % kWave == 0 && (W & (W - 1)) == 0;
    if (W <= 2) {
        if (full) hipLaunchKernelGGL((pair_kernel<FORM, PAIR, 1, kFull>), grid, block, shm, st, d);
        else hipLaunchKernelGGL((pair_kernel<FORM, PAIR, 1, 0>), grid, block, shm, st, d);
    } else if (W <= 4) {
        if (full) hipLaunchKernelGGL((pair_kernel<FORM, PAIR, 2, kFull>), grid, block, shm, st, d);
        else hipLaunchKernelGGL((pair_kernel<FORM, PAIR, 2, 0>), grid, block, shm, st, d);
    } else {
        if (full) hipLaunchKernelGGL((pair_kernel<FORM, PAIR, 3, kFull>), grid, block, shm, st, d);
        else hipLaunchKernelGGL((pair_kernel<FORM, PAIR, 3, 0>), grid, block, shm, st, d);
    }
    return hipGetLastError();
}
}  // namespace

size_t pair_shm_bytes(int W) { return (size_t)(W * kLdsPerWave + kXchSlots * W * kMomQ) * sizeof(double); }

hipError_t launch_pair(const InstDesc &d, int pair, hipStream_t st) {
    if (!pair_supported(d)) return hipErrorInvalidValue;
    const int W = 2 * d.vchunks;
    const size_t shm = pair_shm_bytes(W);
    const dim3 grid(d.nseg), block(kWave * W);
    if (d.form == 0) return pair == 0 ? launch_pair_t<0, 0>(d, grid, block, shm, st) : launch_pair_t<0, 1>(d, grid, block, shm, st);
    return pair == 0 ? launch_pair_t<1, 0>(d, grid, block, shm, st) : launch_pair_t<1, 1>(d, grid, block, shm, st);
}

size_t quad_shm_bytes(int W) {
    return (size_t)(W * kLdsPerWave + 3 * kXchSlots * W * kMomQ + W * kAccQ * 4 * kWave) * sizeof(double);
}

// The whole-step kernel needs nz >= 16 (its eight-row halos wrap once) and its
// LDS within the device's per-workgroup limit (queried once per process).
bool quad_supported(const InstDesc &d) {
    static std::atomic<int> max_shm{-1};
    if (!pair_supported(d) || d.nz < 16) return false;
    int m = max_shm.load();
    if (m < 0) {
        int dev = 0, v = 0;
        m = hipGetDevice(&dev) == hipSuccess &&
                    hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess
                ? v
                : 65536;
        max_shm.store(m);
    }
    return quad_shm_bytes(2 * d.vchunks) <= (size_t)m;
}

hipError_t launch_quad(const InstDesc &d, hipStream_t st) {
    if (!quad_supported(d)) return hipErrorInvalidValue;
    const int W = 2 * d.vchunks;
    const size_t shm = quad_shm_bytes(W);
    const dim3 grid(d.nseg), block(kWave * W);
    if (d.form == 0) {
        if (W <= 2) hipLaunchKernelGGL((quad_kernel<0, 1>), grid, block, shm, st, d);
        else if (W <= 4) hipLaunchKernelGGL((quad_kernel<0, 2>), grid, block, shm, st, d);
        else hipLaunchKernelGGL((quad_kernel<0, 3>), grid, block, shm, st, d);
    } else {
        if (W <= 2) hipLaunchKernelGGL((quad_kernel<1, 1>), grid, block, shm, st, d);
        else if (W <= 4) hipLaunchKernelGGL((quad_kernel<1, 2>), grid, block, shm, st, d);
        else hipLaunchKernelGGL((quad_kernel<1, 3>), grid, block, shm, st, d);
    }
    return hipGetLastError();
}

namespace {
template <int FORM, int PAIR, int PLOG>
const void *batch_pair_fn() {
    return reinterpret_cast<const void *>(batch_pair_kernel<FORM, PAIR, PLOG>);
}
template <int PLOG>
const void *batch_pair_fn_p(int form, int pair) {
    if (form == 0) return pair == 0 ? batch_pair_fn<0, 0, PLOG>() : batch_pair_fn<0, 1, PLOG>();
    return pair == 0 ? batch_pair_fn<1, 0, PLOG>() : batch_pair_fn<1, 1, PLOG>();
}
const void *batch_pair_fn_any(int form, int pair, int W) {
    return W <= 2 ? batch_pair_fn_p<1>(form, pair) : W <= 4 ? batch_pair_fn_p<2>(form, pair) : batch_pair_fn_p<3>(form, pair);
}
}  // namespace

namespace {
template <int FORM>
const void *batch_quad_fn(int W) {
    return W <= 2 ? reinterpret_cast<const void *>(batch_quad_kernel<FORM, 1>)
         : W <= 4 ? reinterpret_cast<const void *>(batch_quad_kernel<FORM, 2>)
                  : reinterpret_cast<const void *>(batch_quad_kernel<FORM, 3>);
}
const void *batch_quad_fn_any(int form, int W) { return form == 0 ? batch_quad_fn<0>(W) : batch_quad_fn<1>(W); }
}  // namespace

hipError_t launch_batch_quad(const InstDesc *d_descs, const WaveTask *d_tasks, int ntasks, int form, int W, int blocks,
                             hipStream_t st) {
    if (W < 2 || W > 8 || (W & 1)) return hipErrorInvalidValue;
    const void *fn = batch_quad_fn_any(form, W);
    void *args[] = {(void *)&d_descs, (void *)&d_tasks, (void *)&ntasks};
    return hipLaunchKernel(fn, dim3(blocks), dim3(kWave * W), args, quad_shm_bytes(W), st);
}

int batch_quad_blocks_per_cu(int form, int W) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_quad_fn_any(form, W), kWave * W, quad_shm_bytes(W)) ==
            hipSuccess &&
        nb > 0)
        return nb;
    return 1;
}

hipError_t launch_batch_pair(const InstDesc *d_descs, const WaveTask *d_tasks, int ntasks, int form, int pair, int W,
                             int blocks, hipStream_t st) {
    if (W < 2 || W > 8 || (W & 1)) return hipErrorInvalidValue;
    const void *fn = batch_pair_fn_any(form, pair, W);
    void *args[] = {(void *)&d_descs, (void *)&d_tasks, (void *)&ntasks};
    return hipLaunchKernel(fn, dim3(blocks), dim3(kWave * W), args, pair_shm_bytes(W), st);
}

int batch_pair_blocks_per_cu(int form, int W) {
    int lo = 1 << 30;
    for (int pair = 0; pair < 2; ++pair) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_pair_fn_any(form, pair, W), kWave * W,
                                                         pair_shm_bytes(W)) == hipSuccess &&
            nb > 0)
            lo = std::min(lo, nb);
    }
    return lo == (1 << 30) ? 1 : lo;
}

hipError_t launch_batch_stage(const InstDesc *d_descs, const WaveTask *d_tasks, int nwt, int scheme, int form,
                              bool wave_rows, int stage, int blocks, hipStream_t st) {
    const dim3 grid(blocks), block(kWave * kWavesPerBlock);
    return wave_rows ? launch_batch_w<true>(d_descs, d_tasks, nwt, scheme, form, stage, grid, block, st)
                     : launch_batch_w<false>(d_descs, d_tasks, nwt, scheme, form, stage, grid, block, st);
}

}  // namespace cosenu
