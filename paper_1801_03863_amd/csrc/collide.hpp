// collide.hpp -- per-node collision rules of MinxEnt-LBM for gfx950, held
// entirely in registers.
//
// Populations are indexed in the column order of the moment matrix T
// (Sec. IV.D): 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE.
//
// MinxEnt4 (Sec. IV.C-D).  Mass, momentum and the two stress moments
// (C1, C4, C6, C8, C9) are fixed; the moments e, eps, q_x, q_y (rows 2, 3, 5,
// 7 of T) are free and take one Newton-Raphson step on the divergence
// H(p) = sum p ln(p/W), starting from the moments of the polynomial
// equilibrium.  The step is taken here in population space f = rho p with the
// free columns of T^-1 scaled to integers:
//   a_e  = (-4,-1,-1,-1,-1, 2, 2, 2, 2)      a_eps = ( 4,-2,-2,-2,-2, 1, 1, 1, 1)
//   a_qx = ( 0,-2, 0, 2, 0, 1,-1,-1, 1)      a_qy  = ( 0, 0,-2, 0, 2, 1, 1,-1,-1)
// Newton's step is affine invariant, so with A = [a_e a_eps a_qx a_qy]:
//   g = A^T ln(f0/W),  H = A^T diag(1/f0) A,  f_post = f0 - A H^-1 g
// equals rho times the step in probability space with the paper's scaling
// (the column scales and rho cancel; the "+1" of the gradient and ln rho
// drop out because every free column sums to zero).
//
// The start point f0 = T^-1 M0 is the polynomial equilibrium plus the stress
// part of the pre-collision state scaled by (1 - 1/tau):
//   f0 = feq + (1 - 1/tau) [ (P_xx-yy - rho(ux^2-uy^2)) T^-1_col8 + (P_xy - rho ux uy) T^-1_col9 ]
// with T^-1_col8 = (0,1,-1,1,-1,0,0,0,0)/4 and T^-1_col9 = (0,0,0,0,0,1,-1,1,-1)/4.
//
// The gradient is evaluated as the logarithms of four products of population
// ratios f0_a / f0_b, each close to one near equilibrium (four logarithms per
// node instead of nine).  In single precision this is as accurate as taking
// the nine logarithms of the deviations from the weights; both are limited
// by the single-precision start point.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Rounded weights of the D2Q9 set (Table I) in compute precision.
template <class C>
struct W9 {
    static constexpr C rest = C(4.0 / 9.0);
    static constexpr C axis = C(1.0 / 9.0);
    static constexpr C diag = C(1.0 / 36.0);
};

// Fused multiply-add in the compute precision (the double builtin would
// widen float operands and round twice).
__device__ __forceinline__ double fma_c(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_c(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
    r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
    return r;
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// One Newton refinement of the hardware reciprocal (v_rcp_f64 is good to
// about 4.6e-8 relative; one step brings it to about 2e-15).
__device__ __forceinline__ double rcp1(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
}

__device__ __forceinline__ float rcp1(float x) { return __builtin_amdgcn_rcpf(x); }

// ln(1 + t) = t + t^2 Q(t) by the Taylor series through the t^N term:
// Q(t) = sum_{k=0}^{N-2} (-1)^(k+1) t^k / (k+2), by Horner's rule (N - 2
// fused multiply-adds, one product and one final fma).  For |t| < 2^-b the
// first omitted term is below 2^(-b N) |t| / (N + 1).
template <int N>
__device__ __forceinline__ double ln1p_taylor(double x)
{
    double q = ((N - 2) % 2 ? 1.0 : -1.0) / N;
#pragma unroll
    for (int k = N - 3; k >= 0; --k) q = __builtin_fma(q, x, (k % 2 ? 1.0 : -1.0) / (k + 2));
    return __builtin_fma(x * x, q, x);
}

// ln(1 + t) of four doubles t > -1 (finite), chosen per value by max |t|
// over the four:
//   |t| < 2^-16 (fluid close to rest)      Taylor through t^4  (omitted term < 2^-64 |t| / 5)
//   |t| < 2^-8  (the bulk of a smooth flow) Taylor through t^7  (< 2^-56 |t| / 8)
//   |t| < 2^-5  (developed, faster flow)    Taylor through t^11 (< 2^-55 |t| / 12)
// otherwise argument reduction y = 1 + t = m 2^k with m in [sqrt(1/2),
// sqrt(2)), then ln m = 2 atanh(s) with s = (m - 1)/(m + 1), |s| <= 0.1716,
// summed as the odd series through s^19 (truncation below 2^-54), and k ln 2
// added with ln 2 split into a 32-bit head and a tail (the Cody-Waite /
// fdlibm split).  Error <= 2-3 ulp on every path (the general path rounds
// 1 + t once more).
__device__ __forceinline__ void ln1p4(const double (&t)[4], double (&out)[4])
{
    const double mt = __builtin_fmax(__builtin_fmax(__builtin_fabs(t[0]), __builtin_fabs(t[1])),
                                     __builtin_fmax(__builtin_fabs(t[2]), __builtin_fabs(t[3])));
    if (mt < 1.52587890625e-05) {
#pragma unroll
        for (int i = 0; i < 4; ++i) out[i] = ln1p_taylor<4>(t[i]);
        return;
    }
    if (mt < 0.00390625) {
#pragma unroll
        for (int i = 0; i < 4; ++i) out[i] = ln1p_taylor<7>(t[i]);
        return;
    }
    if (mt < 0.03125) {
#pragma unroll
        for (int i = 0; i < 4; ++i) out[i] = ln1p_taylor<11>(t[i]);
        return;
    }
    // The general path is rare (steep gradients); it takes one reciprocal
    // per value rather than a shared one, which keeps few values live: the
    // register budget of the whole kernel is set by its busiest point, and
    // this path must not be it.
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double y = 1.0 + t[i];
        double m = __builtin_amdgcn_frexp_mant(y);  // [0.5, 1)
        const int k = __builtin_amdgcn_frexp_exp(y);
        const bool lo = m < 0.70710678118654752440;
        m = lo ? m + m : m;
        const double kd = (double)(lo ? k - 1 : k);
        const double s = (m - 1.0) * rcp(m + 1.0);
        const double z = s * s;
        double p = 1.0 / 19.0;
        p = __builtin_fma(p, z, 1.0 / 17.0);
        p = __builtin_fma(p, z, 1.0 / 15.0);
        p = __builtin_fma(p, z, 1.0 / 13.0);
        p = __builtin_fma(p, z, 1.0 / 11.0);
        p = __builtin_fma(p, z, 1.0 / 9.0);
        p = __builtin_fma(p, z, 1.0 / 7.0);
        p = __builtin_fma(p, z, 1.0 / 5.0);
        p = __builtin_fma(p, z, 1.0 / 3.0);
        const double tt = s + s;
        const double lnm = __builtin_fma(tt * z, p, tt);
        out[i] = __builtin_fma(kd, 6.93147180369123816490e-01, __builtin_fma(kd, 1.90821492927058770002e-10, lnm));
    }
}

// The same for a form whose populations are stored in single precision:
// the series stop once the first omitted term is below 2^-42 |t|, four
// orders of magnitude under the storage rounding (2^-24), so each tier is
// shorter:
//   |t| < 2^-14  through t^3  (omitted term < 2^-42 |t| / 4)
//   |t| < 2^-8   through t^5  (< 2^-40 |t| / 6)
//   |t| < 2^-5   through t^8  (< 2^-40 |t| / 9)
// and the general path is the full-precision one.
__device__ __forceinline__ void ln1p4_lean(const double (&t)[4], double (&out)[4])
{
    const double mt = __builtin_fmax(__builtin_fmax(__builtin_fabs(t[0]), __builtin_fabs(t[1])),
                                     __builtin_fmax(__builtin_fabs(t[2]), __builtin_fabs(t[3])));
    if (mt < 6.103515625e-05) {
#pragma unroll
        for (int i = 0; i < 4; ++i) out[i] = ln1p_taylor<3>(t[i]);
        return;
    }
    if (mt < 0.00390625) {
#pragma unroll
        for (int i = 0; i < 4; ++i) out[i] = ln1p_taylor<5>(t[i]);
        return;
    }
    if (mt < 0.03125) {
#pragma unroll
        for (int i = 0; i < 4; ++i) out[i] = ln1p_taylor<8>(t[i]);
        return;
    }
    ln1p4(t, out);
}

// Single precision, chosen per lane from the largest |t| of the four:
// |t| < 2^-12 (fluid close to rest), t - t^2/2, first omitted term below
// 2^-24 |t| / 3; |t| < 2^-8, t - t^2/2 + t^3/3, below 2^-24 |t| / 4 (two or
// three operations instead of a quarter-rate hardware logarithm and its range
// handling).  Otherwise logf(1 + t): t = y - 1 is exact for y in [1/2, 2],
// so 1 + t gives y back (outside that range one more rounding).
__device__ __forceinline__ void ln1p4(const float (&t)[4], float (&out)[4])
{
    const float mt = __builtin_fmaxf(__builtin_fmaxf(__builtin_fabsf(t[0]), __builtin_fabsf(t[1])),
                                     __builtin_fmaxf(__builtin_fabsf(t[2]), __builtin_fabsf(t[3])));
    if (mt < 0.000244140625f) {
#pragma unroll
        for (int i = 0; i < 4; ++i) out[i] = __builtin_fmaf(t[i] * t[i], -0.5f, t[i]);
        return;
    }
    if (mt < 0.00390625f) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            out[i] = __builtin_fmaf(t[i] * t[i], __builtin_fmaf(t[i], 1.0f / 3.0f, -0.5f), t[i]);
        return;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) out[i] = logf(1.0f + t[i]);
}



template <class C>
__device__ __forceinline__ bool positive_finite(C v)
{
    // false for v <= 0, NaN and +inf
    return v > C(0) && v < C(__builtin_huge_valf());
}

template <class C>
__device__ __forceinline__ bool nonneg_finite(C v)
{
    return v >= C(0) && v < C(__builtin_huge_valf());
}

// Polynomial equilibrium (Sec. IV.E) of (rho, ux, uy) in direction order.
template <class C>
__device__ __forceinline__ void equilibrium(C rho, C ux, C uy, C (&feq)[9])
{
    const C b = C(1) - C(1.5) * (ux * ux + uy * uy);
    const C wr = W9<C>::rest * rho, wa = W9<C>::axis * rho, wd = W9<C>::diag * rho;
    const C s = ux + uy, d = ux - uy;
    const C xx = C(4.5) * ux * ux + b, yy = C(4.5) * uy * uy + b;
    const C ss = C(4.5) * s * s + b, dd = C(4.5) * d * d + b;
    feq[0] = wr * b;
    feq[1] = wa * (xx + C(3) * ux);
    feq[2] = wa * (yy + C(3) * uy);
    feq[3] = wa * (xx - C(3) * ux);
    feq[4] = wa * (yy - C(3) * uy);
    feq[5] = wd * (ss + C(3) * s);
    feq[6] = wd * (dd - C(3) * d);
    feq[7] = wd * (ss - C(3) * s);
    feq[8] = wd * (dd + C(3) * d);
}

// LDL^T solve of the symmetric positive definite n x n system H x = g
// (n = 2 or 4) held in registers.  Unknown order: e, eps, qx, qy.
template <class C>
struct Sym4 {
    C ee, ep, pp, ex, px, xx, ey, py, xy, yy;
};

// Pivot reciprocal: one Newton step on the hardware estimate, or the
// estimate alone where LEAN (single-precision storage: the solve's relative
// error, a few times 1e-7, scales a correction that is itself small next to
// the populations, so it stays far below their storage rounding).
template <bool LEAN, class C>
__device__ __forceinline__ C pivot_rcp(C x)
{
    if constexpr (LEAN && sizeof(C) == 8)
        return __builtin_amdgcn_rcp(x);
    else
        return rcp1(x);
}

template <class C, bool LEAN = false>
__device__ __forceinline__ void ldlt_solve4(const Sym4<C> &h, C (&g)[4])
{
    const C d0 = h.ee, i0 = pivot_rcp<LEAN>(d0);
    const C l10 = h.ep * i0, l20 = h.ex * i0, l30 = h.ey * i0;
    const C d1 = h.pp - l10 * h.ep, i1 = pivot_rcp<LEAN>(d1);
    const C t21 = h.px - l20 * h.ep, t31 = h.py - l30 * h.ep;
    const C l21 = t21 * i1, l31 = t31 * i1;
    const C d2 = h.xx - l20 * h.ex - l21 * t21, i2 = pivot_rcp<LEAN>(d2);
    const C t32 = h.xy - l30 * h.ex - l31 * t21;
    const C l32 = t32 * i2;
    const C d3 = h.yy - l30 * h.ey - l31 * t31 - l32 * t32, i3 = pivot_rcp<LEAN>(d3);
    // forward (unit lower), diagonal, backward
    const C z0 = g[0];
    const C z1 = g[1] - l10 * z0;
    const C z2 = g[2] - l20 * z0 - l21 * z1;
    const C z3 = g[3] - l30 * z0 - l31 * z1 - l32 * z2;
    const C x3 = z3 * i3;
    const C x2 = z2 * i2 - l32 * x3;
    const C x1 = z1 * i1 - l21 * x2 - l31 * x3;
    const C x0 = z0 * i0 - l10 * x1 - l20 * x2 - l30 * x3;
    g[0] = x0;
    g[1] = x1;
    g[2] = x2;
    g[3] = x3;
}

// SRT / BGK (Sec. II.B.1): f += (feq - f) / tau.
template <class C>
__device__ __forceinline__ void collide_srt(C (&f)[9], C omega)
{
    const C rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const C jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const C jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const C irho = rcp(rho);
    C feq[9];
    equilibrium(rho, jx * irho, jy * irho, feq);
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = f[a] + omega * (feq[a] - f[a]);
}

// Multiple-relaxation-time rule (Sec. II.B.2): f += T^-1 B T (feq - f) with
// B diagonal (Table III).  The conserved rows have rate 0; be, bp relax the
// energy-like rows e and eps, bq the heat-flux rows q_x, q_y, bs the two
// stress rows.  TRT is be = bp = bs = 1/tau, bq = 1/tau2; MRT is be = 1.64,
// bp = 1.54, bq = 1/tau2, bs = 1/tau.  T^-1 = T^T diag(1/|row|^2).
template <class C>
__device__ __forceinline__ void collide_mrt(C (&f)[9], C be, C bp, C bq, C bs)
{
    const C rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const C jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const C jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const C irho = rcp(rho);
    C d[9];
    equilibrium(rho, jx * irho, jy * irho, d);
#pragma unroll
    for (int a = 0; a < 9; ++a) d[a] = d[a] - f[a];
    const C da = (d[1] + d[2]) + (d[3] + d[4]);
    const C dd = (d[5] + d[6]) + (d[7] + d[8]);
    const C se = be * C(1.0 / 36.0) * ((C(2) * dd - da) - C(4) * d[0]);
    const C sp = bp * C(1.0 / 36.0) * ((dd - C(2) * da) + C(4) * d[0]);
    const C sx = bq * C(1.0 / 12.0) * (C(2) * (d[3] - d[1]) + (d[5] + d[8]) - (d[6] + d[7]));
    const C sy = bq * C(1.0 / 12.0) * (C(2) * (d[4] - d[2]) + (d[5] + d[6]) - (d[7] + d[8]));
    const C s8 = bs * C(0.25) * ((d[1] + d[3]) - (d[2] + d[4]));
    const C s9 = bs * C(0.25) * ((d[5] + d[7]) - (d[6] + d[8]));
    const C axis = -(se + C(2) * sp);
    const C dgn = C(2) * se + sp;
    f[0] = f[0] + C(4) * (sp - se);
    f[1] = f[1] + ((axis - C(2) * sx) + s8);
    f[2] = f[2] + ((axis - C(2) * sy) - s8);
    f[3] = f[3] + ((axis + C(2) * sx) + s8);
    f[4] = f[4] + ((axis + C(2) * sy) - s8);
    f[5] = f[5] + ((dgn + (sx + sy)) + s9);
    f[6] = f[6] + ((dgn - (sx - sy)) - s9);
    f[7] = f[7] + ((dgn - (sx + sy)) + s9);
    f[8] = f[8] + ((dgn + (sx - sy)) - s9);
}

// True if any of the nine values has its sign bit set (negative values and
// -0): the minimum of the high words as signed integers is negative.  Four
// three-input integer minima instead of eight floating-point ones.
__device__ __forceinline__ bool any_sign9(const double (&v)[9])
{
    int32_t h[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) h[a] = (int32_t)(__builtin_bit_cast(uint64_t, v[a]) >> 32);
    int32_t m = h[0];
#pragma unroll
    for (int a = 1; a < 9; ++a) m = m < h[a] ? m : h[a];
    return m < 0;
}

__device__ __forceinline__ bool any_sign9(const float (&v)[9])
{
    uint32_t o = 0;
#pragma unroll
    for (int a = 0; a < 9; ++a) o |= __builtin_bit_cast(uint32_t, v[a]);
    return (int32_t)o < 0;
}

// MinxEnt collision with a single Newton step.  MX2 selects MinxEnt2 (only
// e and eps free; q_x, q_y relaxed with omega2 = 1/tau2).  Returns true if
// the node was guarded: its start point had a population <= 0 or not
// finite, in which case f holds the start point itself (no Newton step).
// `stable` is the stability criterion of Sec. IV.G for the result: every
// population finite and non-negative.  The nine reciprocals share one
// hardware reciprocal (Montgomery) in double precision, and in single
// precision when SHARED_RCP is set: a few ulp less accurate than nine
// single-precision reciprocals, which is far below the storage error of
// FP16 deviations (the form that sets it); the product of the nine start
// values must then also lie in the normal single-precision range.  LEAN (a
// double-precision step for populations stored in single precision) keeps
// the arithmetic in double but stops each refinement once it is four orders
// of magnitude below the storage rounding: one Newton step on the
// reciprocals of rho and of the product (about 1e-15), none on the four
// pivots of the solve, and the shorter log series of ln1p4_lean.
template <class C, bool MX2, bool SHARED_RCP = false, bool LEAN = false>
__device__ __forceinline__ bool collide_minxent(C (&f)[9], C omega, C omega2, bool &stable)
{
    constexpr bool lean = LEAN && sizeof(C) == 8;
    // Moments of the pre-collision populations (Sec. II.A, Sec. IV.C), from
    // shared pair sums and differences.
    const C a13 = f[1] + f[3], a24 = f[2] + f[4], m13 = f[1] - f[3], m24 = f[2] - f[4];
    const C d57 = f[5] + f[7], d68 = f[6] + f[8], n57 = f[5] - f[7], n68 = f[6] - f[8];
    const C rho = (f[0] + (a13 + a24)) + (d57 + d68);
    const C jx = m13 + (n57 - n68);
    const C jy = m24 + (n57 + n68);
    const C pxxyy = a13 - a24;  // sum f (vx^2 - vy^2)
    const C pxy = d57 - d68;    // sum f vx vy
    const C irho = lean ? rcp1(rho) : rcp(rho);
    const C ux = jx * irho, uy = jy * irho;
    // Relaxed stress constraints C8, C9 as deviations from equilibrium.
    const C k = C(1) - omega;
    const C q8 = C(0.25) * k * (pxxyy - (jx * ux - jy * uy));
    const C q9 = C(0.25) * k * (pxy - jx * uy);
    // Start point: the polynomial equilibrium
    //   W_a rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u)
    // plus the non-equilibrium corrections, with the weights folded into
    // the coefficients (rho/9 * 4.5 = rho/2, rho/36 * 4.5 = rho/8).
    const C uxx = ux * ux, uyy = uy * uy;
    const C b1 = C(1) - C(1.5) * (uxx + uyy);
    const C wa = W9<C>::axis * rho, wd = W9<C>::diag * rho;
    const C wa3 = C(1.0 / 3.0) * rho, wd3 = C(1.0 / 12.0) * rho;
    const C wa45 = C(0.5) * rho, wd45 = C(0.125) * rho;
    const C wab = wa * b1, wdb = wd * b1;
    const C s = ux + uy, d = ux - uy;
    const C ex = fma_c(wa45, uxx, wab) + q8;
    const C ey = fma_c(wa45, uyy, wab) - q8;
    const C es = fma_c(wd45, s * s, wdb) + q9;
    const C ed = fma_c(wd45, d * d, wdb) - q9;
    C f0[9];
    f0[0] = (W9<C>::rest * rho) * b1;
    if constexpr (MX2) {
        // MinxEnt2: C5 and C7 relaxed with 1/tau2 (T^-1 columns = rows / 12).
        const C k2 = C(1) - omega2;
        const C m5 = C(2) * (f[3] - f[1]) + (f[5] - f[6]) + (f[8] - f[7]);
        const C m7 = C(2) * (f[4] - f[2]) + (f[5] + f[6]) - (f[7] + f[8]);
        const C q5 = k2 * (m5 + jx) * C(1.0 / 12.0);
        const C q7 = k2 * (m7 + jy) * C(1.0 / 12.0);
        f0[1] = fma_c(wa3, ux, ex - C(2) * q5);
        f0[2] = fma_c(wa3, uy, ey - C(2) * q7);
        f0[3] = fma_c(-wa3, ux, ex + C(2) * q5);
        f0[4] = fma_c(-wa3, uy, ey + C(2) * q7);
        f0[5] = fma_c(wd3, s, es + (q5 + q7));
        f0[6] = fma_c(-wd3, d, ed - (q5 - q7));
        f0[7] = fma_c(-wd3, s, es - (q5 + q7));
        f0[8] = fma_c(wd3, d, ed + (q5 - q7));
    } else {
        f0[1] = fma_c(wa3, ux, ex);
        f0[2] = fma_c(wa3, uy, ey);
        f0[3] = fma_c(-wa3, ux, ex);
        f0[4] = fma_c(-wa3, uy, ey);
        f0[5] = fma_c(wd3, s, es);
        f0[6] = fma_c(-wd3, d, ed);
        f0[7] = fma_c(-wd3, s, es);
        f0[8] = fma_c(wd3, d, ed);
    }

    // Reciprocals r_a = 1/f0_a and the guard: every start population must be
    // positive and finite (sign bits clear, product of all nine a positive
    // normal number below infinity); otherwise the node keeps its start point.
    // The gradient g = A^T ln(f0/W) is taken as the logarithms of products
    // of population ratios, each close to one near equilibrium:
    //  g_e   = ln( 2^24 F^2 R r0^4 ),   g_eps = ln( f0^4 F R^2 )
    //  g_qx  = ln( (f3 r1)^2 f5 f8 r6 r7 ),  g_qy = ln( (f4 r2)^2 f5 f6 r7 r8 )
    // with F = f5 f6 f7 f8 and R = r1 r2 r3 r4 (2^24 = prod_a W_a^(-a_e,a),
    // the only weight term left; ln rho and the "+1" cancel because every
    // free column sums to zero).
    C r[9];
    C y[4];  // y_i - 1 for the four products
    bool ok;
    C p1, F, R;
    if constexpr (sizeof(C) == 8 || SHARED_RCP) {
        // Simultaneous inversion (Montgomery's trick) over a product tree:
        // pairs 56, 78, 12, 34, quads F = f5 f6 f7 f8 and G = f1 f2 f3 f4,
        // and the product of all nine; one reciprocal of that product is
        // taken back down the tree.  1/G is R itself.  The tree keeps fewer
        // partial products live than a running chain and its dependent
        // chains are three products deep instead of eight.
        p1 = f0[5] * f0[6];
        const C p78 = f0[7] * f0[8];
        const C p12 = f0[1] * f0[2];
        const C p34 = f0[3] * f0[4];
        F = p1 * p78;
        const C G = p12 * p34;
        const C FG = F * G;
        const C p8 = FG * f0[0];
        const C q = lean ? rcp1(p8) : rcp(p8);
        r[0] = q * FG;
        const C qa = q * f0[0];  // 1/(F G)
        const C iF = qa * G;
        R = qa * F;
        const C i56 = iF * p78, i78 = iF * p1;
        const C i12 = R * p34, i34 = R * p12;
        r[5] = i56 * f0[6];
        r[6] = i56 * f0[5];
        r[7] = i78 * f0[8];
        r[8] = i78 * f0[7];
        r[1] = i12 * f0[2];
        r[2] = i12 * f0[1];
        r[3] = i34 * f0[4];
        r[4] = i34 * f0[3];
        if constexpr (sizeof(C) == 8)
            ok = !any_sign9(f0) && p8 > 2.2250738585072014e-308 && p8 < C(__builtin_huge_val());
        else
            ok = !any_sign9(f0) && p8 > 1.17549435e-38f && p8 < C(__builtin_huge_valf());
    } else {
        // Guard on the raw bits, as unsigned integers: a negative value (or
        // -0), +inf or NaN is at least 0x7f800000, and +0 is 0.
        uint32_t hi = 0u, lo = 0xffffffffu;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const uint32_t u = __builtin_bit_cast(uint32_t, f0[a]);
            hi = hi > u ? hi : u;
            lo = lo < u ? lo : u;
        }
        ok = hi < 0x7f800000u && lo != 0u;
#pragma unroll
        for (int a = 0; a < 9; ++a) r[a] = rcp(f0[a]);
        p1 = f0[5] * f0[6];
        F = p1 * (f0[7] * f0[8]);
        R = (r[1] * r[2]) * (r[3] * r[4]);
    }
    {
        const C FR = F * R;
        const C a0 = r[0] * C(64), a2 = a0 * a0;  // (64 r0)^4 = 2^24 r0^4
        const C b0 = f0[0] * f0[0];
        const C t31 = f0[3] * r[1], t42 = f0[4] * r[2];
        // y_i - 1 with the last product fused (one rounding).
        y[0] = fma_c(FR * F, a2 * a2, C(-1));
        y[1] = fma_c(FR * R, b0 * b0, C(-1));
        y[2] = fma_c(t31 * t31, (f0[5] * f0[8]) * (r[6] * r[7]), C(-1));
        y[3] = fma_c(t42 * t42, p1 * (r[7] * r[8]), C(-1));
    }
    if (!ok) {
#pragma unroll
        for (int a = 0; a < 9; ++a) f[a] = f0[a];
        C sm = f0[0], mn = f0[0];
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            sm += f0[a];
            mn = __builtin_fmin(mn, f0[a]);
        }
        stable = __builtin_fabs(sm) < C(__builtin_huge_valf()) && mn >= C(0);  // inf and NaN fail the sum
        return true;
    }
    C g[4];
    if constexpr (lean)
        ln1p4_lean(y, g);
    else
        ln1p4(y, g);

    // Hessian H = A^T diag(r) A, from pair sums and differences of the r.
    const C r13 = r[1] + r[3], r24 = r[2] + r[4], s13 = r[1] - r[3], s24 = r[2] - r[4];
    const C r57 = r[5] + r[7], r68 = r[6] + r[8], s57 = r[5] - r[7], s68 = r[6] - r[8];
    const C Sa = r13 + r24;
    const C Sd = r57 + r68;
    Sym4<C> h;
    h.ee = C(16) * r[0] + Sa + C(4) * Sd;
    h.ep = C(2) * (Sa + Sd) - C(16) * r[0];
    h.pp = C(16) * r[0] + C(4) * Sa + Sd;

    C de, dp, dx = C(0), dy = C(0);
    if (MX2) {
        // Two free moments: closed-form 2 x 2 solve.
        const C det = h.ee * h.pp - h.ep * h.ep;
        const C idet = rcp1(det);
        de = (h.pp * g[0] - h.ep * g[1]) * idet;
        dp = (h.ee * g[1] - h.ep * g[0]) * idet;
    } else {
        const C Dx = s57 - s68;  // r5 - r6 - r7 + r8
        const C Dy = s57 + s68;  // r5 + r6 - r7 - r8
        h.ex = C(2) * (s13 + Dx);
        h.px = C(4) * s13 + Dx;
        h.ey = C(2) * (s24 + Dy);
        h.py = C(4) * s24 + Dy;
        h.xx = C(4) * r13 + Sd;
        h.yy = C(4) * r24 + Sd;
        h.xy = r57 - r68;
        ldlt_solve4<C, lean>(h, g);
        de = g[0];
        dp = g[1];
        dx = g[2];
        dy = g[3];
    }

    // f_post = f0 - A delta.
    const C axis = de + C(2) * dp;
    const C dgn = C(2) * de + dp;
    f[0] = f0[0] + C(4) * (de - dp);
    f[1] = f0[1] + (axis + C(2) * dx);
    f[2] = f0[2] + (axis + C(2) * dy);
    f[3] = f0[3] + (axis - C(2) * dx);
    f[4] = f0[4] + (axis - C(2) * dy);
    f[5] = f0[5] - (dgn + (dx + dy));
    f[6] = f0[6] - (dgn - (dx - dy));
    f[7] = f0[7] - (dgn - (dx + dy));
    f[8] = f0[8] - (dgn + (dx - dy));
    // Stable: finite (f0 is finite, so only the increments can make it
    // otherwise) and no sign bit set.  f0 > 0 here, and a sum with a
    // positive operand is never -0 under round-to-nearest, so the sign bits
    // mark exactly the negative results.
    stable = __builtin_fabs((de + dp) + (dx + dy)) < C(__builtin_huge_valf()) && !any_sign9(f);
    return false;
}

}  // namespace lbm
