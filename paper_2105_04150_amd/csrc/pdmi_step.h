// pdmi_step.h -- the step kernels of the bond-based PMB peridynamics library (templates;
// each launcher file instantiates its share of them).
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
//   q  = |y|^2/|xi|^2 - 1, the numerator as |y|^2 - |xi|^2, both sums in the same order
//   break when s >= s0, i.e. q >= (1 + s0)^2 - 1
//   f  = c s V_j y/|y| = c V_j (1/|xi|) (1 - (1+q)^(-1/2)) y
// The FP64 numerator cancels: q carries an absolute error of a few units of 2^-53 (plus
// 1e-14 relative from 1/|xi|), the same order as the rounding of the oracle's own
// (|y| - |xi|)/|xi|, and is exactly zero for an unstretched bond (y = xi).
// 1 - (1+q)^(-1/2) is summed as its binomial series for |q| < 4e-3, so the force adds no
// second cancellation.  The FP32 kernels keep the cancellation-free numerator
// eta.(xi + y): in single precision the difference of squares would lose most digits of
// a small stretch.
// The break decision is made on q except within a narrow margin around the threshold,
// where a rare branch recomputes s = (|y| - |xi|)/|xi| in the oracle's exact order of
// operations (stretch_exact): in the FP64 build, the same x and u break the same bonds
// whatever the rounding of the fast form.
//
// Every kernel also has a force-evaluation mode (kModeForce): the same gather at the
// current level, no breaking, the bond force density written out (the reaction-force
// readout of the quasi-static examples, Sec. 6).
//
// EXT variants carry the bond-model branch: no-failure zones and n-linear damage laws
// per bond class.  Their common path adds every live bond's elastic contribution; a slot
// over the instance's threshold (or already softened) then takes a rare branch that asks
// its damage state for a weight w and moves its contribution from 1 to w (breaking:
// w = 0).  Problems without zones or laws run the plain kernels.
#pragma once

#include "pdmi_device.h"

namespace pdmi {
namespace {

// What the bond-model branch needs of a slot: its q and its elastic contribution
// coef * y to the force density (FP64 and FP32 builds).
struct SlotTerm {
    double q, coef, y0, y1, y2;
};
struct SlotTerm32 {
    double q;
    float coef, y0, y1, y2;
};

// Contribution of one slot.  live: the slot holds an intact bond; breakable: the bond may
// break in this pass (intact, outside the no-failure zones, not a force evaluation).
// (X, U) are the owner's position and displacement, p0..p2 the neighbour's node record,
// kv = stiffness times neighbour volume, q0 the lower edge of the break decision.  Adds
// the force density to F, except for a breakable slot at or above q0: for such a
// candidate the function returns true and leaves the decision (and, if the bond holds,
// its contribution) to the caller's rare branch.
__device__ __forceinline__ bool slot_force(bool live, bool breakable, const double2 p0, const double2 p1, const double2 p2,
                                           double X0, double X1, double X2, double U0, double U1, double U2,
                                           double kv, double q0, double& F0, double& F1, double& F2, SlotTerm& st,
                                           const SeriesCoef& sk = SeriesCoef(), uint64_t* cand_ballot = nullptr)
{
    const double xi0 = p0.x - X0, xi1 = p0.y - X1, xi2 = p1.x - X2;
    const double e0 = p1.y - U0, e1 = p2.x - U1, e2 = p2.y - U2;
    const double y0 = xi0 + e0, y1 = xi1 + e1, y2 = xi2 + e2;
    const double L2 = __builtin_fma(xi2, xi2, __builtin_fma(xi1, xi1, xi0 * xi0));
    // |y|^2 - |xi|^2 with both squares summed in the same order: two fewer operations than
    // eta.(xi + y), an absolute error in q below 7e-16 (six orders of magnitude inside the
    // decision margin), and exactly zero when y = xi (a body at rest or rigidly translated
    // feels no bond force)
    const double Y2 = __builtin_fma(y2, y2, __builtin_fma(y1, y1, y0 * y0));
    const double tq = Y2 - L2;
    const double iL = rsq64<1>(L2);
    const double q = tq * (iL * iL);
    // one comparison decides both ways (a NaN q, from a non-finite state, is a candidate:
    // the rare branch adds it)
    const bool below = q < q0;
    const bool cand = breakable && !below;
    const bool alive = live && !cand;
    // the lanes' candidates as a mask (each ballot of a comparison is its lane mask)
    if (cand_ballot) *cand_ballot = __builtin_amdgcn_ballot_w64(breakable) & ~__builtin_amdgcn_ballot_w64(below);
    // broken and padding slots (and candidates) evaluate g(0) = 0 and add nothing
    const double coef = (kv * iL) * one_minus_rsqrt1p(alive ? q : 0.0, sk);
    st = SlotTerm{q, coef, y0, y1, y2};
    F0 = __builtin_fma(coef, y0, F0);
    F1 = __builtin_fma(coef, y1, F1);
    F2 = __builtin_fma(coef, y2, F2);
    return cand;
}

// FP32 bond arithmetic (same formulas): the bond vector is formed in f64 from the f64
// coordinates and rounded once, displacements are the f32 values of the records.
// 1 - (1+q)^(-1/2) uses four series terms (below 1.3e-10 relative for |q| < 4e-3).
__device__ __forceinline__ bool slot_force32(bool live, bool breakable, const double2 p0, const double2 p1, const double2 p2,
                                             double X0, double X1, double X2, float U0, float U1, float U2,
                                             float kv, float q0, float& F0, float& F1, float& F2, SlotTerm32& st,
                                             uint64_t* brk_ballot = nullptr)
{
    const float xi0 = static_cast<float>(p0.x - X0), xi1 = static_cast<float>(p0.y - X1),
                xi2 = static_cast<float>(p1.x - X2);
    const uint64_t b1 = __double_as_longlong(p1.y), b2 = __double_as_longlong(p2.x);
    const float uj0 = __uint_as_float(static_cast<uint32_t>(b1)), uj1 = __uint_as_float(static_cast<uint32_t>(b1 >> 32)),
                uj2 = __uint_as_float(static_cast<uint32_t>(b2));
    const float e0 = uj0 - U0, e1 = uj1 - U1, e2 = uj2 - U2;
    const float y0 = xi0 + e0, y1 = xi1 + e1, y2 = xi2 + e2;
    const float z0 = xi0 + y0, z1 = xi1 + y1, z2 = xi2 + y2;
    const float tq = __builtin_fmaf(e2, z2, __builtin_fmaf(e1, z1, e0 * z0));
    const float L2 = __builtin_fmaf(xi2, xi2, __builtin_fmaf(xi1, xi1, xi0 * xi0));
    const float iL = __builtin_amdgcn_rsqf(L2);
    const float q = tq * (iL * iL);
    const bool brk = breakable && q >= q0;
    const bool alive = live && !brk;
    // the lanes that break as a mask (each ballot of a comparison is its lane mask)
    if (brk_ballot) *brk_ballot = __builtin_amdgcn_ballot_w64(breakable) & __builtin_amdgcn_ballot_w64(q >= q0);
    const float qa = alive ? q : 0.0f;
    float g;
    if (fabsf(qa) < 4.0e-3f) {
        float p = -35.0f / 128.0f;
        p = __builtin_fmaf(p, qa, 5.0f / 16.0f);
        p = __builtin_fmaf(p, qa, -3.0f / 8.0f);
        p = __builtin_fmaf(p, qa, 0.5f);
        g = qa * p;
    } else {
        g = 1.0f - __builtin_amdgcn_rsqf(1.0f + qa);
    }
    const float coef = (kv * iL) * g;
    st = SlotTerm32{q, coef, y0, y1, y2};
    F0 = __builtin_fmaf(coef, y0, F0);
    F1 = __builtin_fmaf(coef, y1, F1);
    F2 = __builtin_fmaf(coef, y2, F2);
    return brk;
}

// Weight of a slot in the bond-model branch (EXT kernels): the slot is live and either at
// or over the instance's lower decision edge q0, or softened.  q is its q of this pass,
// nofail / soft its word's flags, sold its stored largest stretch (prefetched by the
// caller when soft), exact_s() the slot's exact stretch (stretch_exact; the FP64 build
// decides on it near every threshold and stores it as a new maximum, the FP32 build
// decides on q).  Returns w (the bond adds w times its elastic force); sets broke when it
// breaks now and newly_soft when it softens for the first time.  A zone bond, and every
// bond in a force evaluation, keeps its damage state as it stands.
template <int MODE, bool FP32, typename ExactS>
__device__ double bond_weight(const StepArgs& A, const InstParams& P, int64_t ds, double q, bool nofail, bool soft,
                              double sold, bool& broke, bool& newly_soft, ExactS exact_s)
{
    broke = false;
    newly_soft = false;
    if (P.nlaw == 0) {  // the brittle law with the instance's s0
        if (nofail || MODE == kModeForce) return 1.0;
        if (FP32)
            broke = static_cast<float>(q) >= static_cast<float>(P.q0);
        else
            broke = q >= P.q0 && exact_s() >= P.s0;
        return broke ? 0.0 : 1.0;
    }
    // a single law per instance is the same for the whole wavefront (scalar loads)
    const LawRec& L = P.nlaw == 1 ? A.laws[P.law_off] : A.laws[P.law_off + A.cls[ds]];
    if (!soft) sold = 0.0;
    if (nofail || MODE == kModeForce) return soft ? law_secant(L, sold) : 1.0;
    // stretch from q without cancellation: s = q / (1 + sqrt(1 + q))
    const double r = rsq64<2>(1.0 + q);
    double s = q * rcp64(__builtin_fma(1.0 + q, r, 1.0));
    // the exact stretch wherever rounding could decide: at or near the stored maximum (a
    // new maximum is stored exact) or near the law's elastic limit or last breakpoint
    const double s_first = L.s[0], s_last = L.s[L.nb - 1];
    if (!FP32 && (s >= sold - decision_margin(sold) || fabs(s - s_first) <= decision_margin(s_first) ||
                  fabs(s - s_last) <= decision_margin(s_last)))
        s = exact_s();
    const double sm = s > sold ? s : sold;
    if (sm >= s_last) {
        broke = true;
        return 0.0;
    }
    if (!(sm > s_first)) return 1.0;
    if (sm > sold) A.smax[ds] = sm;
    newly_soft = !soft;
    return law_secant(L, sm);
}

// Stiffness-correction factor of a slot of reference length L (CORR kernels), in the
// order profile, partial volume, surface factor; fvi, fvj the family volumes of the two
// ends.  The flags are the instance's, the same for the whole wavefront.
__device__ __forceinline__ double corr_factor(const InstParams& P, double L, double fvi, double fvj)
{
    double f = 1.0;
    if (P.cr_flags & 1) f = fmax(__builtin_fma(-L, P.cr_idelta, 1.0), 0.0);
    if (P.cr_flags & 2) f *= fmin(fmax(__builtin_fma(-L, P.cr_idx, P.cr_pvhi), 0.0), 1.0);
    if (P.cr_flags & 4) f *= P.cr_2v0 * rcp64_1(fvi + fvj);
    return f;
}

// Integration and boundary conditions of one node given its force density F (the tail
// of every step kernel).  U is the node's displacement at the level the forces used.
template <int MODE, bool FP32 = false>
__device__ __forceinline__ void node_update(const StepArgs& A, const InstParams& P, int64_t node,
                                            double U0, double U1, double U2, double F0, double F1, double F2)
{
    const int32_t bcid = A.bc_id[node];
    if (bcid == kNodePad) return;

    const int64_t nn = A.nn;
    if (MODE == kModeForce) {  // bond force density of the current level, nothing else
        A.force[node] = F0;
        A.force[nn + node] = F1;
        A.force[2 * nn + node] = F2;
        return;
    }
    const double dt = A.dt;
    const int64_t k = *A.step_base + A.step_local;
    double F[3] = {F0, F1, F2};
    if (P.has_body)
        for (int d = 0; d < 3; ++d) F[d] += P.bmag * A.bhat[d * nn + node];
    double u[3] = {U0, U1, U2};
    if (FP32)  // the integrator advances the f64 master displacement
        for (int d = 0; d < 3; ++d) u[d] = A.um_in[d * nn + node];
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
    if (FP32) {
        float* rf = reinterpret_cast<float*>(ro + 3);
        for (int d = 0; d < 3; ++d) {
            rf[d] = static_cast<float>(un[d]);
            A.um_out[d * nn + node] = un[d];
        }
    } else {
        ro[3] = un[0];
        ro[4] = un[1];
        ro[5] = un[2];
    }
    if (MODE != kModeVVInit)
        for (int d = 0; d < 3; ++d) A.v[d * nn + node] = vn[d];
    if (MODE == kModeVV || MODE == kModeVVInit)
        for (int d = 0; d < 3; ++d) A.a[d * nn + node] = an[d];
}

template <int G, int MODE, bool STIFF, bool VOLN, bool KNODE, bool EXT>
__global__ __launch_bounds__(kBlock) void step_f64(StepArgs A)
{
    constexpr int W = kWave / G;
    constexpr int U = kRowUnroll;  // slot rows in flight per iteration
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t slice =
        wave_uniform(xcd_remap(blockIdx.x, gridDim.x) * (kBlock / kWave) + (threadIdx.x >> 6));
    if (slice >= A.nslices) return;
    const int32_t* __restrict__ slice_inst = A.slice_inst;
    const InstParams* __restrict__ params = A.params;
    const int64_t* __restrict__ slice_ptr = A.slice_ptr;
    const int32_t* __restrict__ slice_T = A.slice_T;
    const InstParams P = params[slice_inst[slice]];
    const int w = lane / G, g = lane % G;
    const int64_t node = slice * W + w;

    const double2* __restrict__ rin = reinterpret_cast<const double2*>(A.rec_in);
    const double2 o0 = rin[3 * node], o1 = rin[3 * node + 1], o2 = rin[3 * node + 2];
    const double X0 = o0.x, X1 = o0.y, X2 = o1.x;
    const double U0 = o1.y, U1 = o2.x, U2 = o2.y;
    // 32-bit byte offsets from wave-uniform bases (the host keeps every offset below 2^32)
    const char* __restrict__ recb = reinterpret_cast<const char*>(A.rec_in);
    const int64_t base = slice_ptr[slice];
    const int T = slice_T[slice];
    const char* __restrict__ colb = reinterpret_cast<const char*>(A.col + base);
    const char* __restrict__ kb = STIFF ? reinterpret_cast<const char*>(A.kslot + base) : nullptr;
    const double* __restrict__ volp = A.vol;
    const double* __restrict__ nwp = A.nw;
    const double ai = KNODE ? A.na[node] : 0.0;  // own stiffness factor
    const uint32_t lane4 = static_cast<uint32_t>(lane) * 4u;
    const double cv = P.c * P.volume;

    // Rows are fetched one iteration ahead.  T is a multiple of kRowUnroll and the slot
    // arrays end with kRowUnroll spare rows, so every prefetch is in bounds and no load
    // sits behind a branch (rows prefetched past T belong to the next slice; unused).
    double F0 = 0.0, F1 = 0.0, F2 = 0.0;
    const SeriesCoef sk = series_coef_regs();
    if (T > 0) {
        auto col_at = [&](int t) -> int32_t {
            const uint32_t off = static_cast<uint32_t>(t) * (kWave * 4u) + lane4;
            return __builtin_nontemporal_load(reinterpret_cast<const int32_t*>(colb + off));
        };
        // stiffness times neighbour volume of row t's slot with neighbour j
        auto kv_of = [&](int t, uint32_t j) -> double {
            if (KNODE) return ai * nwp[j];  // sqrt(k_i) sqrt(k_j) V_j
            if (STIFF || VOLN) {
                double k = P.c;
                if (STIFF) {
                    const uint32_t off = static_cast<uint32_t>(t) * (kWave * 8u) + 2u * lane4;
                    k = __builtin_nontemporal_load(reinterpret_cast<const double*>(kb + off));
                }
                return k * (VOLN ? volp[j] : P.volume);
            }
            return cv;
        };
        // stored stretch of softened slots, fetched with their words (EXT with damage laws)
        auto smax_at = [&](int t, int32_t cw) -> double {
            if (!EXT || P.nlaw == 0 || cw < 0 || !(cw & kColSoft)) return 0.0;
            return A.smax[base + static_cast<int64_t>(t) * kWave + lane];
        };
        // Rare branch of a flagged slot in row t (plain: a break candidate, decided on the
        // exact stretch; EXT: the bond-model branch).  It runs after a block of 32 rows, from
        // the slot's word and neighbour record read again, so the common path keeps its
        // registers.
        auto flagged = [&](int t) {
            const int64_t ds = base + static_cast<int64_t>(t) * kWave + lane;
            const int32_t step = static_cast<int32_t>(*A.step_base + A.step_local);
            const int32_t cw = col_at(t);
            const uint32_t j = col_node(cw);
            const char* rj = recb + __umul24(j, 48u);
            const double2 r0 = *reinterpret_cast<const double2*>(rj), r1 = *reinterpret_cast<const double2*>(rj + 16),
                          r2 = *reinterpret_cast<const double2*>(rj + 32);
            auto exact = [&]() { return stretch_exact_rec(r0, r1, r2, X0, X1, X2, U0, U1, U2); };
            if constexpr (EXT) {
                // the slot's terms as the common path formed them (into scratch accumulators),
                // then move its elastic contribution from weight 1 to w
                SlotTerm st;
                double d0 = 0.0, d1 = 0.0, d2 = 0.0;
                slot_force(true, false, r0, r1, r2, X0, X1, X2, U0, U1, U2, kv_of(t, j), P.q0, d0, d1, d2, st, sk);
                bool brk, newly;
                const double wt = bond_weight<MODE, false>(A, P, ds, st.q, (cw & kColNoFail) != 0, (cw & kColSoft) != 0,
                                                           smax_at(t, cw), brk, newly, exact);
                if (brk) {
                    A.col[ds] = ~cw;
                    A.bstep[ds] = step;
                } else if (newly) {
                    A.col[ds] = cw | kColSoft;
                }
                if (wt != 1.0) {
                    const double m = (wt - 1.0) * st.coef;
                    F0 = __builtin_fma(m, st.y0, F0);
                    F1 = __builtin_fma(m, st.y1, F1);
                    F2 = __builtin_fma(m, st.y2, F2);
                }
            } else if (exact() >= P.s0) {
                A.col[ds] = ~cw;  // irreversible
                A.bstep[ds] = step;
            } else {  // it holds: the contribution the common path left out
                SlotTerm sh;
                slot_force(true, false, r0, r1, r2, X0, X1, X2, U0, U1, U2, kv_of(t, j), P.q0, F0, F1, F2, sh, sk);
            }
        };
        int32_t cn[U];
#pragma unroll
        for (int u = 0; u < U; ++u) cn[u] = col_at(u);
        uint32_t flags = 0;  // flagged rows of the current block of 32 (from row tb)
        int tb = 0;
        for (int t = 0; t < T; t += U) {
            int32_t c[U];
            double2 p[U][3];
            double kv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                c[u] = cn[u];
                const uint32_t j = static_cast<uint32_t>(c[u] ^ (c[u] >> 31)) &
                                   (EXT ? static_cast<uint32_t>(kColNode) : 0xffffffffu);
                const char* rj = recb + __umul24(j, 48u);  // full-rate 24-bit multiply: j < 2^24
                p[u][0] = *reinterpret_cast<const double2*>(rj);
                p[u][1] = *reinterpret_cast<const double2*>(rj + 16);
                p[u][2] = *reinterpret_cast<const double2*>(rj + 32);
                kv[u] = kv_of(t + u, j);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) cn[u] = col_at(t + U + u);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                SlotTerm st;
                bool flag;  // plain: a break candidate; EXT: takes the bond-model branch
                if constexpr (EXT) {
                    slot_force(c[u] >= 0, false, p[u][0], p[u][1], p[u][2], X0, X1, X2, U0, U1, U2, kv[u], P.q0, F0,
                               F1, F2, st, sk);
                    const bool soft = (c[u] & kColSoft) != 0;
                    flag = c[u] >= 0 && (MODE == kModeForce ? soft : (st.q >= P.q0 || soft));
                } else {
                    flag = slot_force(c[u] >= 0, MODE != kModeForce && c[u] >= 0, p[u][0], p[u][1], p[u][2], X0, X1,
                                      X2, U0, U1, U2, kv[u], P.q0, F0, F1, F2, st, sk);
                }
                flags |= flag ? 1u << (t + u - tb) : 0u;
            }
            if (t + U - tb == 32 || t + U >= T) {  // end of a block: its rare branches
                if (__builtin_amdgcn_ballot_w64(flags != 0) != 0)
#pragma unroll 1
                    for (int k = 0; k < 32; ++k)
                        if (flags & (1u << k)) flagged(tb + k);
                flags = 0;
                tb = t + U;
            }
        }
    }
#pragma unroll
    for (int m = 1; m < G; m <<= 1) {
        F0 += __shfl_xor(F0, m);
        F1 += __shfl_xor(F1, m);
        F2 += __shfl_xor(F2, m);
    }
    if (g != 0) return;
    node_update<MODE>(A, P, node, U0, U1, U2, F0, F1, F2);
}

// Orders a wavefront's own LDS writes before its later LDS reads (no workgroup barrier).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Before a wavefront refills its LDS area with direct global-to-LDS loads: every LDS read
// it issued earlier has returned its data (s_waitcnt lgkmcnt = 0, vmcnt and expcnt at
// their no-wait maxima).  The direct loads write LDS through the vector-memory path, which
// is not ordered behind the wavefront's pending LDS reads, so without this wait a read of
// the previous piece still queued in the LDS unit could return the next piece's data.
__device__ __forceinline__ void lds_reads_done() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Staged step kernel: one workgroup of S wavefronts per 64-node slice, one lane per node.
// Wavefront w takes the slice's pieces w, w + S, w + 2S, ...  For every piece, the
// wavefront loads the range's node records and the piece's slot entries straight into
// its own LDS area (gfx950 global_load_lds_dwordx4, no staging registers, which leaves
// room for six wavefronts per SIMD to cover the load latency); per-node weights come
// through registers one piece ahead.  Every slot reads its neighbour from LDS.  Each record crosses the
// vector-memory path once per piece instead of once per slot.  Per-slot stiffness, when
// present, streams from global memory (two rows one piece ahead, the rest when the piece
// starts, which keeps the register count at four wavefronts per SIMD).  Rows are processed in pairs so
// the LDS reads of one row overlap the arithmetic of the other; an odd last row runs
// alone.  With S > 1 the partial forces meet in LDS in a fixed order (S > 1 fills the
// chip on problems with fewer slices than SIMDs).  CORR (uniform volume, no stiffness
// field): the stiffness corrections are formed per slot from the bond length and the two
// family volumes (the neighbour's staged beside its record) instead of read from a
// per-slot stiffness stream.
template <bool FP32, int MODE, bool STIFF, bool VOLN, bool KNODE, int S, bool EXT, bool CORR = false>
__global__ __launch_bounds__(kWave * S) void step_staged(StepArgs A, const int2* __restrict__ pieces,
                                                             const int32_t* __restrict__ slice_piece,
                                                             const int64_t* __restrict__ slice_ptr)
{
    constexpr int kRecChunks = kStageChunks + 3;             // staged records, then the sentinel
    constexpr int kEntChunks = kPieceRows * kWave * 2 / 16;  // 16-byte chunks of entries
    // a per-node weight staged beside the records: through registers (VOLN, KNODE), or the
    // family volumes copied straight to LDS (CORR)
    constexpr bool WREG = VOLN || KNODE;
    static_assert(!CORR || (!STIFF && !VOLN && !KNODE), "per-slot corrections: uniform stiffness and volume");
    // staged weights (doubles): the range and the sentinel's slot; CORR copies a fixed window
    // of 3 x 64 dwords (the family-volume buffer ends with spare entries)
    constexpr int kVolWords = WREG ? (kEntPad / 48 + 2) / 2 * 2 : CORR ? 3 * kWave / 2 : 0;
    static_assert(!CORR || kEntPad / 48 < kVolWords, "the sentinel's weight index lies in the copy");
    constexpr int kLds = kRecChunks + kEntChunks + kVolWords / 2;
    static_assert(kStageChunks == 4 * kWave && kEntChunks == kWave, "four record loads and one entry load");
    __shared__ double2 lds[S * kLds];
    __shared__ double red[S > 1 ? (S - 1) * 3 * kWave : 1];  // partial forces of wavefronts 1..S-1
    const int wv = S > 1 ? __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave) : 0;
    double2* const lrec = lds + wv * kLds;
    const char* const lrecb = reinterpret_cast<const char*>(lrec);
    uint16_t* const lent = reinterpret_cast<uint16_t*>(lrec + kRecChunks);
    double* const lvol = reinterpret_cast<double*>(lrec + kRecChunks + kEntChunks);

    const int lane = threadIdx.x & (kWave - 1);
    int64_t slice = wave_uniform(xcd_remap(blockIdx.x, gridDim.x));
    if (slice >= A.nslices) return;
    if (A.slice_order) slice = __builtin_amdgcn_readfirstlane(A.slice_order[slice]);
    const int32_t* __restrict__ slice_inst = A.slice_inst;
    const InstParams* __restrict__ params = A.params;
    const InstParams P = params[slice_inst[slice]];
    const int64_t node = slice * kWave + lane;
    const double2* __restrict__ rin = reinterpret_cast<const double2*>(A.rec_in);
    const double2 o0 = rin[3 * node], o1 = rin[3 * node + 1], o2 = rin[3 * node + 2];
    const double X0 = o0.x, X1 = o0.y, X2 = o1.x;
    const double U0 = o1.y, U1 = o2.x, U2 = o2.y;  // FP64 build
    const uint64_t ub1 = __double_as_longlong(o1.y), ub2 = __double_as_longlong(o2.x);
    const float Uf0 = __uint_as_float(static_cast<uint32_t>(ub1)), Uf1 = __uint_as_float(static_cast<uint32_t>(ub1 >> 32)),
                Uf2 = __uint_as_float(static_cast<uint32_t>(ub2));  // FP32 build
    const double cv = P.c * P.volume;
    // kernels with uniform c and V accumulate sum (1/|xi|) g(q) y (and the bond-model
    // branch's corrections in the same units) and apply c V once, after the sum (in f64)
    constexpr bool UNI = !STIFF && !VOLN && !KNODE && !CORR;
    const float cvf = static_cast<float>(cv), q0f = static_cast<float>(P.q0);
    uint16_t* __restrict__ entw = A.ent;
    int32_t* __restrict__ bstep = A.bstep;
    // the two innermost series coefficients stay in registers
    const SeriesCoef sk = series_coef_regs();
    const double2* __restrict__ ent2 = reinterpret_cast<const double2*>(A.ent);

    // sentinel record (padding entries point at it), volume 0
    if (lane < 3) lrec[kStageChunks + lane] = lane == 0 ? double2{1e10, 1e10} : lane == 1 ? double2{1e10, 0.0} : double2{0.0, 0.0};
    // (CORR: the copied window fills the sentinel's slot with a positive family volume,
    // which keeps 1/(V_i + V_j) finite on padding slots)
    if (WREG && lane == 0) lvol[kEntPad / 48] = 0.0;
    // staged weight: V_j, or sqrt(k_j) V_j with per-node stiffness (times the own sqrt(k_i)),
    // or the family volume V_j of the surface correction
    const double* __restrict__ wsrc = KNODE ? A.nw : CORR ? A.cfv : A.vol;
    const double ai = KNODE ? A.na[node] : 0.0;
    const double fvi = CORR ? A.cfv[node] : 0.0;
    // FP32 build: the correction constants in single precision, once
    const float cr_id = static_cast<float>(P.cr_idelta), cr_ix = static_cast<float>(P.cr_idx),
                cr_hi = static_cast<float>(P.cr_pvhi), cr_2v0 = static_cast<float>(P.cr_2v0);

    const int p0 = __builtin_amdgcn_readfirstlane(slice_piece[slice]);
    const int p1 = __builtin_amdgcn_readfirstlane(slice_piece[slice + 1]);
    auto rows_of = [&](int p) { return (pieces[__builtin_amdgcn_readfirstlane(p)].y >> 8) & 0xff; };
    int64_t ent = wave_uniform(slice_ptr[slice]);  // first entry of the current piece
    const int pa = p0 + wv;                         // this wavefront's first piece
    for (int q = p0; q < pa && q < p1; ++q) ent += static_cast<int64_t>(rows_of(q)) * kWave;
    double F0 = 0.0, F1 = 0.0, F2 = 0.0;
    float Ff0 = 0.0f, Ff1 = 0.0f, Ff2 = 0.0f;
    // the slots of a row that take the rare branch are kept as its lane mask (scalar), and
    // the rare branch finds the lanes again (the FP32 bond-model kernels keep per-lane bits)
    constexpr bool ROWMASK = !FP32 || !EXT;
    uint64_t cmask = 0;  // candidate lanes of the slot evaluated last

    // staging registers of the next piece (weights and stiffness; records and entries go
    // straight to LDS)
    double vs0 = 0.0, vs1 = 0.0;
    int vlen = 0;
    constexpr int kKPre = 2;  // stiffness rows fetched a piece ahead; the rest when the piece starts
    double kcur[kPieceRows], knext[kKPre];
    auto kcur_at = [&](int t) {  // kcur[t] for a row index only known at run time (no indexed registers)
        double k = 0.0;
#pragma unroll
        for (int u = 0; u < kPieceRows; ++u)
            if (u == t) k = kcur[u];
        return k;
    };

    // Loads of piece p (first entry e): a fixed 256-chunk window from the range start
    // (the record buffers end with kRecPad spare records) and the whole 8-row entry block
    // (rows >= T are never read); volumes from clamped addresses.
    auto issue = [&](int p, int64_t e) {
        const int2 m = pieces[__builtin_amdgcn_readfirstlane(p)];
        if (WREG) {
            const int len = m.y & 0xff;
            vlen = len;
            vs0 = wsrc[m.x + min(lane, len - 1)];
            vs1 = wsrc[m.x + min(lane + kWave, len - 1)];
        }
        if (STIFF)
#pragma unroll
            for (int t = 0; t < kKPre; ++t) knext[t] = __builtin_nontemporal_load(A.kslot + e + t * kWave + lane);
    };
    typedef __attribute__((address_space(3))) void* lds_ptr;
    auto dma = [&](int p, int64_t e) {
        const int2 m = pieces[__builtin_amdgcn_readfirstlane(p)];
        const double2* rs = rin + 3 * static_cast<int64_t>(m.x) + lane;
        // one address and one LDS base for the four 1 KB chunks: the instruction's immediate
        // offset advances the global and the LDS address alike
        __builtin_amdgcn_global_load_lds(rs, (lds_ptr)(lrec), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(rs, (lds_ptr)(lrec), 16, 16 * kWave, 0);
        __builtin_amdgcn_global_load_lds(rs, (lds_ptr)(lrec), 16, 2 * 16 * kWave, 0);
        __builtin_amdgcn_global_load_lds(rs, (lds_ptr)(lrec), 16, 3 * 16 * kWave, 0);
        __builtin_amdgcn_global_load_lds(ent2 + e / 8 + lane, (lds_ptr)(lent), 16, 0, 0);
        if (CORR) {
            const float* ws = reinterpret_cast<const float*>(A.cfv + m.x) + lane;
            float* wl = reinterpret_cast<float*>(lvol);
            __builtin_amdgcn_global_load_lds(ws, (lds_ptr)(wl), 4, 0, 0);
            __builtin_amdgcn_global_load_lds(ws + kWave, (lds_ptr)(wl + kWave), 4, 0, 0);
            __builtin_amdgcn_global_load_lds(ws + 2 * kWave, (lds_ptr)(wl + 2 * kWave), 4, 0, 0);
        }
    };
    auto commit = [&]() {
        if (WREG) {
            if (lane < vlen) lvol[lane] = vs0;
            if (lane + kWave < vlen) lvol[lane + kWave] = vs1;
        }
    };
    // One slot from its staged record into the force accumulators; returns true for a
    // break candidate (plain kernels) and what the rare branches need in st / st32.
    auto eval_into = [&](uint16_t e, double kst, bool live, bool breakable, SlotTerm& st, SlotTerm32& st32,
                         double& G0, double& G1, double& G2, float& Gf0, float& Gf1, float& Gf2) {
        const uint32_t off = e & kEntOff;  // byte offset of the neighbour's staged record
        const double2 q0 = *reinterpret_cast<const double2*>(lrecb + off);
        const double2 q1 = *reinterpret_cast<const double2*>(lrecb + off + 16);
        const double2 q2 = *reinterpret_cast<const double2*>(lrecb + off + 32);
        double kv = UNI ? 1.0 : cv;
        const uint32_t widx = (off * 0xAAABu) >> 21;  // off / 48
        if (KNODE) {
            kv = ai * lvol[widx];
        } else if (STIFF || VOLN) {
            kv = (STIFF ? kst : P.c) * (VOLN ? lvol[widx] : P.volume);
        } else if (CORR && !FP32) {  // the bond length as slot_force forms it (the compiler shares the work)
            const double xa = q0.x - X0, xb = q0.y - X1, xc = q1.x - X2;
            const double L2 = __builtin_fma(xc, xc, __builtin_fma(xb, xb, xa * xa));
            kv = cv * corr_factor(P, L2 * rsq64<1>(L2), fvi, lvol[widx]);
        }
        float kvf = UNI ? 1.0f : cvf;
        if (CORR && FP32) {  // the same factors in single precision, from slot_force32's bond vector
            const float xa = static_cast<float>(q0.x - X0), xb = static_cast<float>(q0.y - X1),
                        xc = static_cast<float>(q1.x - X2);
            const float L2 = __builtin_fmaf(xc, xc, __builtin_fmaf(xb, xb, xa * xa));
            const float L = L2 * __builtin_amdgcn_rsqf(L2);
            float f = 1.0f;
            if (P.cr_flags & 1) f = fmaxf(__builtin_fmaf(-L, cr_id, 1.0f), 0.0f);
            if (P.cr_flags & 2) f *= fminf(fmaxf(__builtin_fmaf(-L, cr_ix, cr_hi), 0.0f), 1.0f);
            if (P.cr_flags & 4) f *= cr_2v0 * __builtin_amdgcn_rcpf(static_cast<float>(fvi + lvol[widx]));
            kvf = cvf * f;
        }
        if (FP32)
            return slot_force32(live, breakable, q0, q1, q2, X0, X1, X2, Uf0, Uf1, Uf2,
                                (STIFF || VOLN || KNODE) ? static_cast<float>(kv) : kvf,
                                q0f, Gf0, Gf1, Gf2, st32, ROWMASK && !EXT ? &cmask : nullptr);
        return slot_force(live, breakable, q0, q1, q2, X0, X1, X2, U0, U1, U2, kv, P.q0, G0, G1, G2, st, sk,
                          ROWMASK && !EXT ? &cmask : nullptr);
    };
    auto eval = [&](uint16_t e, double kst, bool live, bool breakable, SlotTerm& st, SlotTerm32& st32) {
        return eval_into(e, kst, live, breakable, st, st32, F0, F1, F2, Ff0, Ff1, Ff2);
    };
    // Plain kernels: true for a break candidate (FP32: a slot that breaks now).  EXT
    // kernels: true when it takes the bond-model branch.
    auto row = [&](uint16_t e, double kst, SlotTerm& st, SlotTerm32& st32) {
        const bool live = !(e & kEntBroken);
        if constexpr (EXT) {
            const bool soft = (e & kEntSoft) != 0;
            // the condition as lane masks (each ballot of a comparison is one), the entry's
            // taken before the evaluation's branch
            const uint64_t lm = ROWMASK ? __builtin_amdgcn_ballot_w64(live) : 0;
            const uint64_t sm = ROWMASK ? __builtin_amdgcn_ballot_w64(soft) : 0;
            eval(e, kst, live, false, st, st32);
            const bool over = FP32 ? static_cast<float>(st32.q) >= q0f : st.q >= P.q0;
            if constexpr (ROWMASK)
                cmask = lm & (MODE == kModeForce ? sm : (__builtin_amdgcn_ballot_w64(over) | sm));
            return live && (MODE == kModeForce ? soft : (over || soft));
        } else {
            return eval(e, kst, live, MODE != kModeForce && live, st, st32);
        }
    };
    // a slot that broke in this pass: flag it (irreversible) and record the pass
    auto broke = [&](int64_t ds, uint16_t e) {
        entw[ds] = static_cast<uint16_t>(e | kEntBroken);
        bstep[ds] = static_cast<int32_t>(*A.step_base + A.step_local);
    };
    // the exact stretch of a slot from its staged record (FP64 build; the piece is still
    // in LDS: the rare branches run before the next piece is loaded)
    auto exact_of = [&](uint16_t e) {
        return [&, e]() {
            const uint32_t off = e & kEntOff;
            return stretch_exact_rec(*reinterpret_cast<const double2*>(lrecb + off),
                                     *reinterpret_cast<const double2*>(lrecb + off + 16),
                                     *reinterpret_cast<const double2*>(lrecb + off + 32), X0, X1, X2, U0, U1, U2);
        };
    };
    // bond-model branch (EXT): move the slot's elastic contribution from weight 1 to the
    // weight its damage state gives
    auto model = [&](int64_t ds, uint16_t e, const SlotTerm& st, const SlotTerm32& st32) {
        bool brk, newly;
        const bool soft = (e & kEntSoft) != 0;
        const double sold = soft ? A.smax[ds] : 0.0;
        const double wt = bond_weight<MODE, FP32>(A, P, ds, FP32 ? st32.q : st.q, (e & kEntNoFail) != 0, soft,
                                                  sold, brk, newly, exact_of(e));
        if (brk)
            broke(ds, e);
        else if (newly)
            entw[ds] = static_cast<uint16_t>(e | kEntSoft);
        if (wt != 1.0) {
            if (FP32) {
                const float m = static_cast<float>(wt - 1.0) * st32.coef;
                Ff0 = __builtin_fmaf(m, st32.y0, Ff0);
                Ff1 = __builtin_fmaf(m, st32.y1, Ff1);
                Ff2 = __builtin_fmaf(m, st32.y2, Ff2);
            } else {
                const double m = (wt - 1.0) * st.coef;
                F0 = __builtin_fma(m, st.y0, F0);
                F1 = __builtin_fma(m, st.y1, F1);
                F2 = __builtin_fma(m, st.y2, F2);
            }
        }
    };
    // rare branch of a flagged slot (kst: its per-slot stiffness), run once the piece's rows
    // are done (the piece is still staged)
    auto flagged = [&](int64_t ds, uint16_t e, double kst) {
        SlotTerm st;
        SlotTerm32 st32;
        if constexpr (EXT) {
            // the slot's terms as the common path formed them (evaluated again, into
            // scratch accumulators), then its damage state's weight
            double d0 = 0.0, d1 = 0.0, d2 = 0.0;
            float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
            eval_into(e, kst, true, false, st, st32, d0, d1, d2, f0, f1, f2);
            model(ds, e, st, st32);
        } else if (FP32 || exact_of(e)() >= P.s0) {  // FP64: a candidate decided on the exact stretch
            broke(ds, e);
        } else {  // it holds: the contribution the common path left out, evaluated again
            eval(e, kst, true, false, st, st32);
        }
    };

    if (pa < p1) {
        issue(pa, ent);
        for (int p = pa; p < p1; p += S) {
            const int T = rows_of(p);
            int64_t ent_next = ent + static_cast<int64_t>(T) * kWave;  // first entry of piece p + S
            for (int q = p + 1; q < p + S && q < p1; ++q) ent_next += static_cast<int64_t>(rows_of(q)) * kWave;
            wave_sync();  // the previous piece is no longer read
            lds_reads_done();
            dma(p, ent);
            // s_waitcnt with vmcnt = 0 (expcnt and lgkmcnt at their no-wait maxima): the
            // piece's direct-to-LDS loads have landed
            __builtin_amdgcn_s_waitcnt(0x0F70);
            commit();
            if (STIFF)
#pragma unroll
                for (int t = 0; t < kPieceRows; ++t)
                    kcur[t] = t < kKPre ? knext[t] : __builtin_nontemporal_load(A.kslot + ent + t * kWave + lane);
            if (p + S < p1) issue(p + S, ent_next);
            wave_sync();  // the piece's LDS copy is complete
            // rows of this piece whose slot takes the rare branch: rows in which some lane's
            // slot does, wave-uniform, or per lane (FP32 bond-model kernels)
            uint32_t flags = 0;
#pragma unroll
            for (int t = 0; t < kPieceRows; t += 2) {
                if (t >= T) break;
                const uint16_t ea = lent[t * kWave + lane];
                if (t + 1 < T) {
                    const uint16_t eb = lent[(t + 1) * kWave + lane];
                    SlotTerm sa, sb;
                    SlotTerm32 sa32, sb32;
                    const bool ba = row(ea, STIFF ? kcur[t] : 0.0, sa, sa32);
                    const uint64_t cm_a = cmask;
                    const bool bb = row(eb, STIFF ? kcur[t + 1] : 0.0, sb, sb32);
                    if constexpr (ROWMASK)
                        flags |= (cm_a != 0 ? 1u << t : 0u) | (cmask != 0 ? 2u << t : 0u);
                    else
                        flags |= (ba ? 1u << t : 0u) | (bb ? 2u << t : 0u);
                } else {
                    SlotTerm sa;
                    SlotTerm32 sa32;
                    const bool ba = row(ea, STIFF ? kcur[t] : 0.0, sa, sa32);
                    if constexpr (ROWMASK)
                        flags |= cmask != 0 ? 1u << t : 0u;
                    else
                        flags |= ba ? 1u << t : 0u;
                }
            }
            if constexpr (!ROWMASK) {
                if (__builtin_amdgcn_ballot_w64(flags != 0) != 0) {
#pragma unroll
                    for (int t = 0; t < kPieceRows; ++t)
                        if (flags & (1u << t)) flagged(ent + t * kWave + lane, lent[t * kWave + lane], STIFF ? kcur[t] : 0.0);
                }
            } else if (__builtin_amdgcn_readfirstlane(flags) != 0) {
                // the lanes of a marked row that take the rare branch, found again (the same
                // arithmetic on the same staged record decides the same way)
#pragma unroll 1
                for (int t = 0; t < T; ++t) {
                    if (!(__builtin_amdgcn_readfirstlane(flags) & (1u << t))) continue;
                    const uint16_t e = lent[t * kWave + lane];
                    const double kst = STIFF ? kcur_at(t) : 0.0;
                    SlotTerm st;
                    SlotTerm32 st32;
                    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
                    float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
                    const bool live = !(e & kEntBroken);
                    if constexpr (EXT) {
                        // the slot's terms as the common path formed them, then (for the lanes
                        // that take the branch) its damage state's weight
                        eval_into(e, kst, live, false, st, st32, d0, d1, d2, f0, f1, f2);
                        const bool soft = (e & kEntSoft) != 0;
                        if (live && (MODE == kModeForce ? soft : (st.q >= P.q0 || soft)))
                            model(ent + t * kWave + lane, e, st, st32);
                    } else if (eval_into(e, kst, live, MODE != kModeForce && live, st, st32, d0, d1, d2, f0, f1, f2)) {
                        flagged(ent + t * kWave + lane, e, kst);
                    }
                }
            }
            ent = ent_next;
        }
    }
    if (FP32) {
        F0 = Ff0;
        F1 = Ff1;
        F2 = Ff2;
    }
    if (S > 1) {  // wavefront 0 adds the partial forces of 1..S-1 in that order
        if (wv > 0) {
            double* r = red + (wv - 1) * 3 * kWave + lane;
            r[0] = F0;
            r[kWave] = F1;
            r[2 * kWave] = F2;
        }
        __syncthreads();  // every wavefront of the workgroup reaches this once
        if (wv > 0) return;
#pragma unroll
        for (int w = 1; w < S; ++w) {
            const double* r = red + (w - 1) * 3 * kWave + lane;
            F0 += r[0];
            F1 += r[kWave];
            F2 += r[2 * kWave];
        }
    }
    if (UNI) {
        F0 *= cv;
        F1 *= cv;
        F2 *= cv;
    }
    node_update<MODE, FP32>(A, P, node, U0, U1, U2, F0, F1, F2);
}

// ---------------------------------------------------------------- launch templates

template <int G, bool STIFF, bool VOLN, bool KNODE, bool EXT>
hipError_t launch_step_gsv(const StepArgs& a, int mode, hipStream_t s)
{
    const dim3 grid(static_cast<unsigned>((a.nslices + 3) / 4)), block(kBlock);
    switch (mode) {
#define PD_L(M) hipLaunchKernelGGL((step_f64<G, M, STIFF, VOLN, KNODE, EXT>), grid, block, 0, s, a)
    case kModeEC: PD_L(kModeEC); break;
    case kModeVV: PD_L(kModeVV); break;
    case kModeVVInit: PD_L(kModeVVInit); break;
    case kModeFE: PD_L(kModeFE); break;
    case kModeForce: PD_L(kModeForce); break;
#undef PD_L
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int G, bool EXT>
hipError_t launch_step_g(const StepArgs& a, int mode, bool stiff, hipStream_t s)
{
    const bool voln = a.vol != nullptr;
    if (a.nw) return launch_step_gsv<G, false, false, true, EXT>(a, mode, s);  // per-node stiffness
    if (stiff)
        return voln ? launch_step_gsv<G, true, true, false, EXT>(a, mode, s)
                    : launch_step_gsv<G, true, false, false, EXT>(a, mode, s);
    return voln ? launch_step_gsv<G, false, true, false, EXT>(a, mode, s)
                : launch_step_gsv<G, false, false, false, EXT>(a, mode, s);
}

template <bool FP32, bool STIFF, bool VOLN, bool KNODE, int S, bool EXT, bool CORR = false>
hipError_t launch_staged_svs(const StepArgs& a, int mode, hipStream_t s)
{
    const dim3 grid(static_cast<unsigned>(a.nslices)), block(kWave * S);
    switch (mode) {
#define PD_L(M)                                                                                                   \
    hipLaunchKernelGGL((step_staged<FP32, M, STIFF, VOLN, KNODE, S, EXT, CORR>), grid, block, 0, s, a, a.pieces, \
                       a.slice_piece, a.slice_ptr)
    case kModeEC: PD_L(kModeEC); break;
    case kModeVV: PD_L(kModeVV); break;
    case kModeVVInit: PD_L(kModeVVInit); break;
    case kModeFE: PD_L(kModeFE); break;
    case kModeForce: PD_L(kModeForce); break;
#undef PD_L
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool FP32, bool STIFF, bool VOLN, bool KNODE, bool EXT, bool CORR = false>
hipError_t launch_staged_sv(const StepArgs& a, int mode, int split, hipStream_t s)
{
    switch (split) {
    case 1: return launch_staged_svs<FP32, STIFF, VOLN, KNODE, 1, EXT, CORR>(a, mode, s);
    case 2: return launch_staged_svs<FP32, STIFF, VOLN, KNODE, 2, EXT, CORR>(a, mode, s);
    case 4: return launch_staged_svs<FP32, STIFF, VOLN, KNODE, 4, EXT, CORR>(a, mode, s);
    default: return hipErrorInvalidValue;
    }
}

template <bool FP32, bool EXT>
hipError_t launch_staged_n(const StepArgs& a, int mode, int split, hipStream_t s)
{
    const bool stiff = a.kslot != nullptr, voln = a.vol != nullptr;
    if (a.cfv) return launch_staged_sv<FP32, false, false, false, EXT, true>(a, mode, split, s);  // corrections per slot
    if (a.nw) return launch_staged_sv<FP32, false, false, true, EXT>(a, mode, split, s);  // per-node stiffness
    if (stiff)
        return voln ? launch_staged_sv<FP32, true, true, false, EXT>(a, mode, split, s)
                    : launch_staged_sv<FP32, true, false, false, EXT>(a, mode, split, s);
    return voln ? launch_staged_sv<FP32, false, true, false, EXT>(a, mode, split, s)
                : launch_staged_sv<FP32, false, false, false, EXT>(a, mode, split, s);
}

}  // namespace
}  // namespace pdmi
