// pdmi_device.h -- device helpers shared by the step and adjoint kernels.
#pragma once

#include "pdmi_internal.h"

namespace pdmi {
namespace {

// 1/sqrt(x): hardware estimate (specified to 2^29 ulp, i.e. about 2^-23 relative) and NR
// Newton steps; one step leaves a relative error near 1e-14, two reach rounding level.
template <int NR>
__device__ __forceinline__ double rsq64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const double h = x * y;
        const double e = __builtin_fma(-h, y, 1.0);
        y = __builtin_fma(0.5 * y, e, y);
    }
    return y;
}

// 1 - (1+q)^(-1/2).  Series q/2 - 3q^2/8 + 5q^3/16 - 35q^4/128 + 63q^5/256 - 231q^6/1024
// (hot loops pass the coefficients from registers: series_coef_regs());
// the first omitted term, 429q^7/2048, is below 2e-15 of the sum for |q| < 4e-3.  Larger
// |q| (strongly compressed or broken bonds) takes the closed form, whose cancellation
// costs at most 1e-16/|q| < 3e-14 relative there.
struct SeriesCoef {
    double c6 = -231.0 / 1024.0, c5 = 63.0 / 256.0, c4 = -35.0 / 128.0, c3 = 5.0 / 16.0, c2 = -3.0 / 8.0;
};

__device__ __forceinline__ double one_minus_rsqrt1p(double q, const SeriesCoef& k = SeriesCoef())
{
    if (fabs(q) < 4.0e-3) {
        double p = __builtin_fma(k.c6, q, k.c5);
        p = __builtin_fma(p, q, k.c4);
        p = __builtin_fma(p, q, k.c3);
        p = __builtin_fma(p, q, k.c2);
        p = __builtin_fma(p, q, 0.5);
        return q * p;
    }
    return 1.0 - rsq64<2>(1.0 + q);
}

// The critical-stretch decision made exactly as the oracle makes it (Eq. mu; the bond
// kernel keeps a bond only while s < s0): s = (|y| - |xi|)/|xi| with the squares summed
// as (a^2 + b^2) + c^2, every product and sum rounded once (no fused multiply-add), and
// the square roots and the division correctly rounded (the device's IEEE sequences).  The
// step kernels decide on their fast q almost always; a slot whose q lies
// within the instance's margin of the threshold (or a law's breakpoint) is decided here,
// so that two implementations reading the same x and u break the same bonds.
__device__ __forceinline__ double stretch_exact(double xi0, double xi1, double xi2, double y0, double y1, double y2)
{
#pragma clang fp contract(off)
    const double r = __builtin_sqrt((y0 * y0 + y1 * y1) + y2 * y2);
    const double L = __builtin_sqrt((xi0 * xi0 + xi1 * xi1) + xi2 * xi2);
    return (r - L) / L;
}

// The same from a neighbour record {x_j, u_j} (6 doubles) and the owner's (X, U): the
// bond vector and the deformed bond formed as the oracle forms them,
// xi = x_j - x_i and y = xi + (u_j - u_i).
__device__ __forceinline__ double stretch_exact_rec(const double2 p0, const double2 p1, const double2 p2, double X0,
                                                    double X1, double X2, double U0, double U1, double U2)
{
#pragma clang fp contract(off)
    const double xi0 = p0.x - X0, xi1 = p0.y - X1, xi2 = p1.x - X2;
    const double y0 = xi0 + (p1.y - U0), y1 = xi1 + (p2.x - U1), y2 = xi2 + (p2.y - U2);
    return stretch_exact(xi0, xi1, xi2, y0, y1, y2);
}

// Series coefficients as opaque registers: the outer ones in scalar registers (each FMA
// of the Horner chain reads one), the innermost in a vector register (the first FMA
// reads two constants).
__device__ __forceinline__ SeriesCoef series_coef_regs()
{
    SeriesCoef k;
    asm volatile("" : "+s"(k.c6), "+s"(k.c4), "+s"(k.c3), "+s"(k.c2));
    asm volatile("" : "+v"(k.c5));
    return k;
}

// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so that each XCD
// works on one contiguous range of slices (neighbouring nodes share its L2).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb)
{
    constexpr int64_t X = 8;
    const int64_t m = nb / X, r = nb % X, x = b % X, j = b / X;
    return (x < r) ? x * (m + 1) + j : r * (m + 1) + (x - r) * m + j;
}

// Time schedule g(t) of a prescribed quantity and its derivative: 0 constant, 1 linear,
// 2 the fifth-order ramp tau^3 (10 - 15 tau + 6 tau^2), tau = t/T, from 0 to 1 over [0, T]
// with zero first and second derivatives at both ends, then 1 (Secs. 6-7).  tau is
// formed with the stored reciprocal iT = 1/T (no division in the node update).
__device__ __forceinline__ double sched_g(int sc, double t, double T, double iT)
{
    if (sc == 1) return t;
    if (sc == 2) {
        if (t >= T) return 1.0;
        const double tau = t * iT;
        return tau * tau * tau * (10.0 - 15.0 * tau + 6.0 * tau * tau);
    }
    return 1.0;
}

__device__ __forceinline__ double sched_dg(int sc, double t, double T, double iT)
{
    if (sc == 1) return 1.0;
    if (sc == 2) {
        if (t >= T) return 0.0;
        const double tau = t * iT;
        return 30.0 * tau * tau * (1.0 - tau) * (1.0 - tau) * iT;
    }
    return 0.0;
}

// Prescribed velocity of component d at time t.
__device__ __forceinline__ double bc_vel(const BCRec& r, int d, double t)
{
    const int kind = (r.code >> (2 * d)) & 3, sc = (r.code >> (8 + 2 * d)) & 3;
    return kind == 1 ? r.A[d] * sched_dg(sc, t, r.T, r.iT) : r.A[d] * sched_g(sc, t, r.T, r.iT);
}

// Prescribed displacement of component d at time t; uprev one step earlier.
__device__ __forceinline__ double bc_disp(const BCRec& r, int d, double t, double uprev, double dt)
{
    const int kind = (r.code >> (2 * d)) & 3, sc = (r.code >> (8 + 2 * d)) & 3;
    const double g = sched_g(sc, t, r.T, r.iT);
    return kind == 1 ? r.A[d] * g : uprev + dt * (r.A[d] * g);
}

__device__ __forceinline__ bool constrained(const BCRec& r, int d) { return ((r.code >> (2 * d)) & 3) != 0; }

// 1/x: hardware estimate and two Newton steps (within a few ulps; x > 0, normal).
__device__ __forceinline__ double rcp64(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = __builtin_fma(__builtin_fma(-x, y, 1.0), y, y);
    y = __builtin_fma(__builtin_fma(-x, y, 1.0), y, y);
    return y;
}

// 1/x with one Newton step (relative error near 1e-14, the level of rsq64<1>; x > 0, normal).
__device__ __forceinline__ double rcp64_1(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    return __builtin_fma(__builtin_fma(-x, y, 1.0), y, y);
}

// Secant ratio of a bond softened to stretch sm under law L (s[0] < sm < s[nb-1]): the
// law's force c s[0] rho(sm), rho interpolated linearly between breakpoints, over the
// elastic force c sm.  The bond force is this ratio times c s (unloading and reloading
// follow the secant to the origin).
__device__ __forceinline__ double law_secant(const LawRec& L, double sm)
{
    // segment of sm, chosen by selects (no indexed loads: a law shared by the wavefront
    // stays in scalar registers)
    double s_lo = L.s[0], r_lo = L.r[0], sl = L.slope[0];
    for (int k = 1; k + 1 < L.nb; ++k)
        if (sm >= L.s[k]) {
            s_lo = L.s[k];
            r_lo = L.r[k];
            sl = L.slope[k];
        }
    const double rho = __builtin_fma(sl, sm - s_lo, r_lo);
    return (L.s[0] * rho) * rcp64(sm);
}

// Damage of a softened slot from its stored largest stretch.
__device__ __forceinline__ double law_damage(const LawRec& L, double sm) { return 1.0 - law_secant(L, sm); }

// Neighbour device index of a sliced slot word (intact or broken, no-failure bit dropped).
__device__ __forceinline__ uint32_t col_node(int32_t c)
{
    return static_cast<uint32_t>(c ^ (c >> 31)) & static_cast<uint32_t>(kColNode);
}

__device__ __forceinline__ int64_t wave_uniform(int64_t v)
{
    const int lo = __builtin_amdgcn_readfirstlane(static_cast<int>(v & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane(static_cast<int>(v >> 32));
    return (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo);
}

}  // namespace
}  // namespace pdmi
