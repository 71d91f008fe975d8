// pdmi_kernels.hip -- gfx950 kernels of the bond-based PMB peridynamics step.
//
// One fused kernel per time step (paper Sec. 3: the bond force, the critical-stretch
// check and the per-node reduction are fused, Algorithm 2; here the time integration
// is fused too).  It reads displacement level k from one node-record buffer and writes
// level k+1 into the other, so no wavefront can observe a half-updated field (the race
// that forces the paper to keep integration in a separate kernel, Sec. 3.3).
//
// Mapping: a wavefront serves one slice of W = 64/G nodes; each node's bonds are split
// over G lanes, each lane sums its bonds sequentially, and the G partial sums meet in a
// butterfly of cross-lane shuffles.  No atomics and no LDS: a node's force is owned by
// its slice and the result is deterministic.
//
// Bond arithmetic (per slot b = (i, j), Eqs. microelastic and simpleBond):
//   xi = x_j - x_i,  eta = u_j - u_i,  y = xi + eta
//   q  = |y|^2/|xi|^2 - 1 = (2 xi.eta + eta.eta) / |xi|^2      (no cancellation)
//   break when q >= (1 + s0)^2 - 1, i.e. s >= s0
//   f  = c s V_j y/|y| = c V_j (1/|xi|) (1 - (1+q)^(-1/2)) y
// 1 - (1+q)^(-1/2) is summed as its binomial series for |q| < 4e-3, so small stretches
// keep full relative precision instead of losing digits in |y| - |xi|.
#include "pdmi_internal.h"

namespace pdmi {
namespace {

// 1/sqrt(x): hardware estimate (about 2^-23 relative) and two Newton steps.
__device__ __forceinline__ double rsq64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double h = x * y;
    double e = __builtin_fma(-h, y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
    h = x * y;
    e = __builtin_fma(-h, y, 1.0);
    return __builtin_fma(0.5 * y, e, y);
}

// 1 - (1+q)^(-1/2).  Series q/2 - 3q^2/8 + 5q^3/16 - 35q^4/128 + 63q^5/256 - 231q^6/1024
// + 429q^7/2048; the first omitted term is below 0.2 q^8, i.e. under 1e-17 relative for
// |q| < 4e-3.
__device__ __forceinline__ double one_minus_rsqrt1p(double q)
{
    if (fabs(q) < 4.0e-3) {
        double p = 429.0 / 2048.0;
        p = __builtin_fma(p, q, -231.0 / 1024.0);
        p = __builtin_fma(p, q, 63.0 / 256.0);
        p = __builtin_fma(p, q, -35.0 / 128.0);
        p = __builtin_fma(p, q, 5.0 / 16.0);
        p = __builtin_fma(p, q, -3.0 / 8.0);
        p = __builtin_fma(p, q, 0.5);
        return q * p;
    }
    return 1.0 - rsq64(1.0 + q);
}

// Workgroups are dispatched round-robin over the 8 XCDs; renumber them so that each XCD
// works on one contiguous range of slices (neighbouring nodes share its L2).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb)
{
    constexpr int64_t X = 8;
    const int64_t m = nb / X, r = nb % X, x = b % X, j = b / X;
    return (x < r) ? x * (m + 1) + j : r * (m + 1) + (x - r) * m + j;
}

__device__ __forceinline__ double sched(int lin, double t) { return lin ? t : 1.0; }

// Prescribed velocity of component d at time t.
__device__ __forceinline__ double bc_vel(const BCRec& r, int d, double t)
{
    const int kind = (r.code >> (2 * d)) & 3, lin = (r.code >> (8 + d)) & 1;
    return kind == 1 ? r.A[d] * (lin ? 1.0 : 0.0) : r.A[d] * sched(lin, t);
}

// Prescribed displacement of component d at time t; uprev one step earlier.
__device__ __forceinline__ double bc_disp(const BCRec& r, int d, double t, double uprev, double dt)
{
    const int kind = (r.code >> (2 * d)) & 3, lin = (r.code >> (8 + d)) & 1;
    return kind == 1 ? r.A[d] * sched(lin, t) : uprev + dt * (r.A[d] * sched(lin, t));
}

__device__ __forceinline__ bool constrained(const BCRec& r, int d) { return ((r.code >> (2 * d)) & 3) != 0; }

__device__ __forceinline__ int64_t wave_uniform(int64_t v)
{
    const int lo = __builtin_amdgcn_readfirstlane(static_cast<int>(v & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane(static_cast<int>(v >> 32));
    return (static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo);
}

template <int G, int MODE, bool STIFF>
__global__ __launch_bounds__(kBlock) void step_f64(StepArgs<double> A)
{
    constexpr int W = kWave / G;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t slice =
        wave_uniform(xcd_remap(blockIdx.x, gridDim.x) * (kBlock / kWave) + (threadIdx.x >> 6));
    if (slice >= A.nslices) return;
    const int inst = A.slice_inst[slice];
    const InstParams P = A.params[inst];
    const int w = lane / G, g = lane % G;
    const int64_t node = slice * W + w;

    const double2* rin = reinterpret_cast<const double2*>(A.rec_in);
    const double2 o0 = rin[3 * node], o1 = rin[3 * node + 1], o2 = rin[3 * node + 2];
    const double X0 = o0.x, X1 = o0.y, X2 = o1.x;
    const double U0 = o1.y, U1 = o2.x, U2 = o2.y;

    const int64_t base = A.slice_ptr[slice];
    const int T = A.slice_T[slice];
    double F0 = 0.0, F1 = 0.0, F2 = 0.0;
    for (int t = 0; t < T; ++t) {
        const int64_t idx = base + static_cast<int64_t>(t) * kWave + lane;
        const int32_t c = A.col[idx];
        const int32_t j = c >= 0 ? c : ~c;
        const double2* rj = rin + 3 * static_cast<int64_t>(j);
        const double2 p0 = rj[0], p1 = rj[1], p2 = rj[2];
        const double xi0 = p0.x - X0, xi1 = p0.y - X1, xi2 = p1.x - X2;
        const double e0 = p1.y - U0, e1 = p2.x - U1, e2 = p2.y - U2;
        const double L2 = __builtin_fma(xi2, xi2, __builtin_fma(xi1, xi1, xi0 * xi0));
        const double xe = __builtin_fma(xi2, e2, __builtin_fma(xi1, e1, xi0 * e0));
        const double ee = __builtin_fma(e2, e2, __builtin_fma(e1, e1, e0 * e0));
        const double iL = rsq64(L2);
        double q = __builtin_fma(2.0, xe, ee) * (iL * iL);
        bool alive = c >= 0;
        if (alive && q >= P.q0) {
            A.col[idx] = ~c;  // irreversible; contributes nothing from this step on
            alive = false;
        }
        q = alive ? q : 0.0;
        const double gq = one_minus_rsqrt1p(q);
        const double kb = STIFF ? A.kslot[idx] : P.c;
        const double vj = A.vol ? A.vol[j] : P.volume;
        const double coef = alive ? kb * vj * iL * gq : 0.0;
        F0 = __builtin_fma(coef, xi0 + e0, F0);
        F1 = __builtin_fma(coef, xi1 + e1, F1);
        F2 = __builtin_fma(coef, xi2 + e2, F2);
    }
#pragma unroll
    for (int m = 1; m < G; m <<= 1) {
        F0 += __shfl_xor(F0, m);
        F1 += __shfl_xor(F1, m);
        F2 += __shfl_xor(F2, m);
    }
    if (g != 0) return;
    const int32_t bcid = A.bc_id[node];
    if (bcid == kNodePad) return;

    const int64_t nn = A.nn;
    const double dt = A.dt;
    const int64_t k = *A.step_base + A.step_local;
    double F[3] = {F0, F1, F2};
    if (P.has_body)
        for (int d = 0; d < 3; ++d) F[d] += P.bmag * A.bhat[d * nn + node];
    const double u[3] = {U0, U1, U2};
    double vv[3], un[3], vn[3], an[3];
    for (int d = 0; d < 3; ++d) vv[d] = A.v[d * nn + node];
    BCRec bc;
    bc.code = 0;
    if (bcid >= 0) bc = A.bc[bcid];

    if (MODE == kModeEC || MODE == kModeFE) {
        const double t1 = static_cast<double>(k + 1) * dt;
        for (int d = 0; d < 3; ++d) {
            const double acc = (F[d] - P.eta * vv[d]) / P.rho;
            if (MODE == kModeEC) {
                vn[d] = vv[d] + dt * acc;
                un[d] = u[d] + dt * vn[d];
            } else {
                un[d] = u[d] + dt * vv[d];
                vn[d] = vv[d] + dt * acc;
            }
            if (constrained(bc, d)) {
                vn[d] = bc_vel(bc, d, t1);
                un[d] = bc_disp(bc, d, t1, u[d], dt);
            }
        }
    } else if (MODE == kModeVV) {
        // u holds level k+1; v, a hold level k.  Finish step k -> k+1, then move the
        // displacement on to level k+2 (Eq. Velocity_Verlet1) for the next launch.
        const double t1 = static_cast<double>(k + 1) * dt, t2 = static_cast<double>(k + 2) * dt;
        const double hdt = 0.5 * dt, hdt2 = 0.5 * dt * dt;
        for (int d = 0; d < 3; ++d) {
            const double aa = A.a[d * nn + node];
            const double vh = vv[d] + hdt * aa;
            an[d] = (F[d] - P.eta * vh) / P.rho;
            vn[d] = vv[d] + hdt * (aa + an[d]);
            if (constrained(bc, d)) {
                vn[d] = bc_vel(bc, d, t1);
                an[d] = 0.0;
            }
            un[d] = (u[d] + dt * vn[d]) + hdt2 * an[d];
            if (constrained(bc, d)) un[d] = bc_disp(bc, d, t2, u[d], dt);
        }
    } else {  // kModeVVInit: u holds level k; acceleration of level k, then u of level k+1
        const double t1 = static_cast<double>(k + 1) * dt;
        const double hdt2 = 0.5 * dt * dt;
        for (int d = 0; d < 3; ++d) {
            an[d] = constrained(bc, d) ? 0.0 : (F[d] - P.eta * vv[d]) / P.rho;
            un[d] = (u[d] + dt * vv[d]) + hdt2 * an[d];
            if (constrained(bc, d)) un[d] = bc_disp(bc, d, t1, u[d], dt);
            vn[d] = vv[d];
        }
    }

    bool finite = true;
    for (int d = 0; d < 3; ++d) finite = finite && __builtin_isfinite(un[d]) && __builtin_isfinite(vn[d]);
    if (!finite) atomicOr(A.status, 1);
    double* ro = A.rec_out + 6 * node;
    ro[3] = un[0];
    ro[4] = un[1];
    ro[5] = un[2];
    if (MODE != kModeVVInit)
        for (int d = 0; d < 3; ++d) A.v[d * nn + node] = vn[d];
    if (MODE == kModeVV || MODE == kModeVVInit)
        for (int d = 0; d < 3; ++d) A.a[d * nn + node] = an[d];
}

// Velocity-Verlet position update u_{k+1} = u_k + dt v_k + dt^2/2 a_k with the
// displacement constraints of t_{k+1}; one thread per device node.
__global__ __launch_bounds__(kBlock) void drift_f64(StepArgs<double> A)
{
    const int64_t node = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (node >= A.nn) return;
    const int32_t bcid = A.bc_id[node];
    if (bcid == kNodePad) return;
    const int64_t nn = A.nn;
    const double dt = A.dt, hdt2 = 0.5 * dt * dt;
    const int64_t k = *A.step_base + A.step_local;
    const double t1 = static_cast<double>(k + 1) * dt;
    BCRec bc;
    bc.code = 0;
    if (bcid >= 0) bc = A.bc[bcid];
    const double* ri = A.rec_in + 6 * node;
    double* ro = A.rec_out + 6 * node;
    for (int d = 0; d < 3; ++d) {
        const double u = ri[3 + d];
        double un = (u + dt * A.v[d * nn + node]) + hdt2 * A.a[d * nn + node];
        if (constrained(bc, d)) un = bc_disp(bc, d, t1, u, dt);
        ro[3 + d] = un;
    }
}

// Local damage: 1 - sum of intact V_j / sum of V_j over the initial family.
template <int G>
__global__ __launch_bounds__(kBlock) void damage_kernel(DamageArgs A)
{
    constexpr int W = kWave / G;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t slice =
        wave_uniform(xcd_remap(blockIdx.x, gridDim.x) * (kBlock / kWave) + (threadIdx.x >> 6));
    if (slice >= A.nslices) return;
    const InstParams P = A.params[A.slice_inst[slice]];
    const int w = lane / G, g = lane % G;
    const int64_t node = slice * W + w;
    const int64_t base = A.slice_ptr[slice];
    const int T = A.slice_T[slice];
    double num = 0.0, den = 0.0;
    for (int t = 0; t < T; ++t) {
        const int32_t c = A.col[base + static_cast<int64_t>(t) * kWave + lane];
        const int32_t j = c >= 0 ? c : ~c;
        if (j == node) continue;  // padding
        const double vj = A.vol ? A.vol[j] : P.volume;
        den += vj;
        if (c >= 0) num += vj;
    }
#pragma unroll
    for (int m = 1; m < G; m <<= 1) {
        num += __shfl_xor(num, m);
        den += __shfl_xor(den, m);
    }
    if (g == 0) A.phi[node] = den > 0.0 ? 1.0 - num / den : 0.0;
}

__global__ void advance_kernel(int64_t* step_base, int64_t by)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *step_base += by;
}

template <int G>
hipError_t launch_step_g(const StepArgs<double>& a, int mode, bool stiff, hipStream_t s)
{
    const dim3 grid(static_cast<unsigned>((a.nslices + 3) / 4)), block(kBlock);
#define PD_LAUNCH(M, S) hipLaunchKernelGGL((step_f64<G, M, S>), grid, block, 0, s, a)
    if (stiff) {
        switch (mode) {
        case kModeEC: PD_LAUNCH(kModeEC, true); break;
        case kModeVV: PD_LAUNCH(kModeVV, true); break;
        case kModeVVInit: PD_LAUNCH(kModeVVInit, true); break;
        case kModeFE: PD_LAUNCH(kModeFE, true); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (mode) {
        case kModeEC: PD_LAUNCH(kModeEC, false); break;
        case kModeVV: PD_LAUNCH(kModeVV, false); break;
        case kModeVVInit: PD_LAUNCH(kModeVVInit, false); break;
        case kModeFE: PD_LAUNCH(kModeFE, false); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef PD_LAUNCH
    return hipGetLastError();
}

}  // namespace

bool lanes_supported(int lanes) { return lanes == 1 || lanes == 4 || lanes == 16 || lanes == 64; }

template <>
hipError_t launch_step<double>(const StepArgs<double>& a, int lanes, int mode, bool stiff, hipStream_t s)
{
    if (a.nslices <= 0) return hipSuccess;
    switch (lanes) {
    case 1: return launch_step_g<1>(a, mode, stiff, s);
    case 4: return launch_step_g<4>(a, mode, stiff, s);
    case 16: return launch_step_g<16>(a, mode, stiff, s);
    case 64: return launch_step_g<64>(a, mode, stiff, s);
    default: return hipErrorInvalidValue;
    }
}

template <>
hipError_t launch_drift<double>(const StepArgs<double>& a, int /*lanes*/, hipStream_t s)
{
    if (a.nn <= 0) return hipSuccess;
    hipLaunchKernelGGL(drift_f64, dim3(static_cast<unsigned>((a.nn + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, s, a);
    return hipGetLastError();
}

template <>
hipError_t launch_step<float>(const StepArgs<float>&, int, int, bool, hipStream_t)
{
    return hipErrorNotSupported;
}

template <>
hipError_t launch_drift<float>(const StepArgs<float>&, int, hipStream_t)
{
    return hipErrorNotSupported;
}

hipError_t launch_damage(const DamageArgs& a, int lanes, hipStream_t s)
{
    if (a.nslices <= 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>((a.nslices + 3) / 4)), block(kBlock);
    switch (lanes) {
    case 1: hipLaunchKernelGGL(damage_kernel<1>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(damage_kernel<4>, grid, block, 0, s, a); break;
    case 16: hipLaunchKernelGGL(damage_kernel<16>, grid, block, 0, s, a); break;
    case 64: hipLaunchKernelGGL(damage_kernel<64>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_advance(int64_t* step_base, int64_t by, hipStream_t s)
{
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, step_base, by);
    return hipGetLastError();
}

}  // namespace pdmi
