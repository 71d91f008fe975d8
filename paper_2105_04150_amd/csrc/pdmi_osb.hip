// pdmi_osb.hip -- the ordinary state-based linear solid (Sec. 8.2): two kernels per time
// step on the staged layout.
//
// The bond force of this model depends on the dilation of both end nodes, a sum over each
// node's whole family, so one pass over the bonds cannot both form and use it (Sec. 8.2:
// two loops, hence two kernels).
//
//   pass 1 (osb_staged<0, ...>): every slot forms its stretch; a slot at or over the
//     critical stretch breaks (outside no-failure zones, not in a force evaluation); the
//     node sums |xi| e V over its intact bonds into the dilation theta_i = 3 V / m_i sum and
//     writes the node pair {theta_i / m_i, 1 / m_i}.
//   pass 2 (osb_staged<1, ...>): every intact slot adds
//       (t_ij + t_ji) y / |y| V,   t_ij + t_ji = |xi| [(3K - 5G)(A_i + A_j) + 15 G s (B_i + B_j)]
//     with A = theta / m, B = 1 / m, s = e / |xi| the stretch, then the node integrates
//     (the same tail as the bond-based step kernels).
//
// Both passes use the staged mapping of the bond-based kernels: a slice of 64 nodes, one
// lane per node, the node records of each piece's range and its slot entries copied
// straight into LDS; pass 2 copies the range's node pairs beside them.  Influence function
// 1; a uniform node volume per instance, or per-node volumes copied into LDS beside the
// records (V_j enters the dilation sum and the force term).  FP64, or the FP32 build: bond arithmetic in
// single precision from the f32 displacements of the records and the f64 coordinates, the
// node pairs and the integration (f64 master displacement) as in FP64.
//
// Per slot: xi, eta and q = (|y|^2 - |xi|^2)/|xi|^2 as in the bond-based kernels.  The
// dilation pass needs the stretch s = sqrt(1+q) - 1, the force pass g = 1 - (1+q)^(-1/2)
// = |y| - |xi| over |y|: with |xi| / |y| = 1 - g and s (1 - g) = g the force term is
//   (t_ij + t_ji) V y / |y| = V [(3K - 5G)(A_i + A_j)(1 - g) + 15 G (B_i + B_j) g] y,
// the |xi| of the scalar state cancelling the 1 / |xi| of y / |y|.  Both s and g come
// from their binomial series for small |q| (no division, no cancellation).
#include "pdmi_step.h"

namespace pdmi {
namespace {

// sqrt(1+q) - 1.  Series q/2 - q^2/8 + q^3/16 - 5q^4/128 + 7q^5/256 - 21q^6/1024; the first
// omitted term, 33q^7/2048, is below 2e-16 of the sum for |q| < 4e-3.  Larger |q| takes
// q / (1 + sqrt(1+q)), which has no cancellation.
__device__ __forceinline__ double sqrt1p_minus1(double q)
{
    if (fabs(q) < 4.0e-3) {
        double p = __builtin_fma(-21.0 / 1024.0, q, 7.0 / 256.0);
        p = __builtin_fma(p, q, -5.0 / 128.0);
        p = __builtin_fma(p, q, 1.0 / 16.0);
        p = __builtin_fma(p, q, -1.0 / 8.0);
        p = __builtin_fma(p, q, 0.5);
        return q * p;
    }
    const double r = rsq64<2>(1.0 + q);
    return q * rcp64(__builtin_fma(1.0 + q, r, 1.0));
}

// The FP32 build's sqrt(1+q) - 1: series q/2 - q^2/8 + q^3/16 - 5q^4/128 (the next term is
// below 2e-11 of the sum for |q| < 4e-3), else q / (1 + sqrt(1+q)).
__device__ __forceinline__ float sqrt1p_minus1_f32(float q)
{
    if (fabsf(q) < 4.0e-3f) {
        float p = __builtin_fmaf(-5.0f / 128.0f, q, 1.0f / 16.0f);
        p = __builtin_fmaf(p, q, -1.0f / 8.0f);
        p = __builtin_fmaf(p, q, 0.5f);
        return q * p;
    }
    return q * __builtin_amdgcn_rcpf(1.0f + __builtin_sqrtf(1.0f + q));
}

// The FP32 build's 1 - (1+q)^(-1/2): four series terms, else the closed form.
__device__ __forceinline__ float one_minus_rsqrt1p_f32(float q)
{
    if (fabsf(q) < 4.0e-3f) {
        float p = __builtin_fmaf(-35.0f / 128.0f, q, 5.0f / 16.0f);
        p = __builtin_fmaf(p, q, -3.0f / 8.0f);
        p = __builtin_fmaf(p, q, 0.5f);
        return q * p;
    }
    return 1.0f - __builtin_amdgcn_rsqf(1.0f + q);
}

template <bool FP32, int PASS, int MODE, int S, bool VOLN>
__global__ __launch_bounds__(kWave * S) void osb_staged(StepArgs A, const int2* __restrict__ pieces,
                                                        const int32_t* __restrict__ slice_piece,
                                                        const int64_t* __restrict__ slice_ptr)
{
    constexpr int kRecChunks = kStageChunks + 3;             // staged records, then the sentinel
    constexpr int kEntChunks = kPieceRows * kWave * 2 / 16;  // 16-byte chunks of entries
    constexpr int kPairChunks = PASS == 1 ? 2 * kWave : 0;   // node pairs of the range (pass 2)
    constexpr int kVolChunks = VOLN ? 3 * kWave * 4 / 16 : 0;    // node volumes of the range (3 x 64 dwords)
    constexpr int kLds = kRecChunks + kEntChunks + kPairChunks + kVolChunks;
    static_assert(!VOLN || kEntPad / 48 < 3 * kWave / 2, "the sentinel's volume index lies in the copy");
    constexpr int kRed = PASS == 1 ? 3 : 1;
    static_assert(kEntPad / 48 < kPairChunks || PASS == 0, "the sentinel's pair index lies in the copy");
    __shared__ double2 lds[S * kLds];
    __shared__ double red[S > 1 ? (S - 1) * kRed * kWave : 1];
    const int wv = S > 1 ? __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave) : 0;
    double2* const lrec = lds + wv * kLds;
    const char* const lrecb = reinterpret_cast<const char*>(lrec);
    uint16_t* const lent = reinterpret_cast<uint16_t*>(lrec + kRecChunks);
    double2* const lpair = lrec + kRecChunks + kEntChunks;
    double* const lvol = reinterpret_cast<double*>(lrec + kRecChunks + kEntChunks + kPairChunks);

    const int lane = threadIdx.x & (kWave - 1);
    int64_t slice = wave_uniform(xcd_remap(blockIdx.x, gridDim.x));
    if (slice >= A.nslices) return;
    if (A.slice_order) slice = __builtin_amdgcn_readfirstlane(A.slice_order[slice]);  // long slices first
    const InstParams P = A.params[A.slice_inst[slice]];
    const int64_t node = slice * kWave + lane;
    const double2* __restrict__ rin = reinterpret_cast<const double2*>(A.rec_in);
    const double2 o0 = rin[3 * node], o1 = rin[3 * node + 1], o2 = rin[3 * node + 2];
    const double X0 = o0.x, X1 = o0.y, X2 = o1.x;
    const double U0 = o1.y, U1 = o2.x, U2 = o2.y;  // FP64 build
    const uint64_t ub1 = __double_as_longlong(o1.y), ub2 = __double_as_longlong(o2.x);
    const float Uf0 = __uint_as_float(static_cast<uint32_t>(ub1)), Uf1 = __uint_as_float(static_cast<uint32_t>(ub1 >> 32)),
                Uf2 = __uint_as_float(static_cast<uint32_t>(ub2));  // FP32 build
    const double2* __restrict__ ent2 = reinterpret_cast<const double2*>(A.ent);
    uint16_t* __restrict__ entw = A.ent;
    const SeriesCoef sk = series_coef_regs();
    double2 own = {0.0, 0.0};
    if (PASS == 1) own = A.osb[node];
    const double Ai = own.x, Bi = own.y;
    const double ka = P.osb_a, kb = P.osb_b;
    const float Aif = static_cast<float>(Ai), Bif = static_cast<float>(Bi), kaf = static_cast<float>(ka),
                kbf = static_cast<float>(kb), q0f = static_cast<float>(P.q0);

    // sentinel record (padding entries point at it)
    if (lane < 3) lrec[kStageChunks + lane] = lane == 0 ? double2{1e10, 1e10} : lane == 1 ? double2{1e10, 0.0} : double2{0.0, 0.0};

    const int p0 = __builtin_amdgcn_readfirstlane(slice_piece[slice]);
    const int p1 = __builtin_amdgcn_readfirstlane(slice_piece[slice + 1]);
    auto rows_of = [&](int p) { return (pieces[__builtin_amdgcn_readfirstlane(p)].y >> 8) & 0xff; };
    int64_t ent = wave_uniform(slice_ptr[slice]);
    const int pa = p0 + wv;
    for (int q = p0; q < pa && q < p1; ++q) ent += static_cast<int64_t>(rows_of(q)) * kWave;

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
        if (PASS == 1) {  // the pair buffer ends with 2 x 64 spare pairs
            const double2* ps = A.osb + m.x + lane;
            __builtin_amdgcn_global_load_lds(ps, (lds_ptr)(lpair), 16, 0, 0);
            __builtin_amdgcn_global_load_lds(ps, (lds_ptr)(lpair), 16, 16 * kWave, 0);
        }
        if (VOLN) {  // per-node volumes: the volume buffer ends with spare entries
            const float* ws = reinterpret_cast<const float*>(A.vol + m.x) + lane;
            float* wl = reinterpret_cast<float*>(lvol);
            __builtin_amdgcn_global_load_lds(ws, (lds_ptr)(wl), 4, 0, 0);
            __builtin_amdgcn_global_load_lds(ws + kWave, (lds_ptr)(wl + kWave), 4, 0, 0);
            __builtin_amdgcn_global_load_lds(ws + 2 * kWave, (lds_ptr)(wl + 2 * kWave), 4, 0, 0);
        }
    };

    double D = 0.0;                    // pass 1: sum of |xi|^2 s (V_j) over intact bonds
    double F0 = 0.0, F1 = 0.0, F2 = 0.0;  // pass 2: force density (uniform volume: without the factor V)
    float Df = 0.0f, Ff0 = 0.0f, Ff1 = 0.0f, Ff2 = 0.0f;  // the same in the FP32 build
    constexpr bool BREAK = PASS == 0 && MODE != kModeForce;
    const int32_t step = static_cast<int32_t>(*A.step_base + A.step_local);

    // FP32 build: one slot in single precision (the bond vector formed in f64 and rounded
    // once, the displacements those of the f32 records)
    auto slot32 = [&](uint16_t e, int64_t ds) {
        const bool live = !(e & kEntBroken);
        const uint32_t off = e & kEntOff;
        const double2 r0 = *reinterpret_cast<const double2*>(lrecb + off);
        const double2 r1 = *reinterpret_cast<const double2*>(lrecb + off + 16);
        const double2 r2 = *reinterpret_cast<const double2*>(lrecb + off + 32);
        const float xi0 = static_cast<float>(r0.x - X0), xi1 = static_cast<float>(r0.y - X1),
                    xi2 = static_cast<float>(r1.x - X2);
        const uint64_t b1 = __double_as_longlong(r1.y), b2 = __double_as_longlong(r2.x);
        const float e0 = __uint_as_float(static_cast<uint32_t>(b1)) - Uf0,
                    e1 = __uint_as_float(static_cast<uint32_t>(b1 >> 32)) - Uf1,
                    e2 = __uint_as_float(static_cast<uint32_t>(b2)) - Uf2;
        const float y0 = xi0 + e0, y1 = xi1 + e1, y2 = xi2 + e2;
        const float z0 = xi0 + y0, z1 = xi1 + y1, z2 = xi2 + y2;
        const float tq = __builtin_fmaf(e2, z2, __builtin_fmaf(e1, z1, e0 * z0));
        const float L2 = __builtin_fmaf(xi2, xi2, __builtin_fmaf(xi1, xi1, xi0 * xi0));
        const float q = tq * __builtin_amdgcn_rcpf(L2);
        const bool brk = BREAK && live && !(e & kEntNoFail) && q >= q0f;
        const bool alive = live && !brk;
        const float vj = VOLN ? static_cast<float>(lvol[(off * 0xAAABu) >> 21]) : 1.0f;
        if (PASS == 0) {
            Df = __builtin_fmaf(VOLN ? L2 * vj : L2, sqrt1p_minus1_f32(alive ? q : 0.0f), Df);
            if (brk) {
                entw[ds] = static_cast<uint16_t>(e | kEntBroken);
                A.bstep[ds] = step;
            }
        } else {
            const float g = one_minus_rsqrt1p_f32(alive ? q : 0.0f);
            const double2 pj = lpair[(off * 0xAAABu) >> 21];
            const float a = kaf * (Aif + static_cast<float>(pj.x)), b = kbf * (Bif + static_cast<float>(pj.y));
            const float c = alive ? __builtin_fmaf(g, b - a, a) : 0.0f;
            const float coef = VOLN ? c * vj : c;
            Ff0 = __builtin_fmaf(coef, y0, Ff0);
            Ff1 = __builtin_fmaf(coef, y1, Ff1);
            Ff2 = __builtin_fmaf(coef, y2, Ff2);
        }
    };

    auto slot = [&](uint16_t e, int64_t ds) {
        if constexpr (FP32) {
            slot32(e, ds);
            return;
        }
        const bool live = !(e & kEntBroken);
        const uint32_t off = e & kEntOff;
        const double2 r0 = *reinterpret_cast<const double2*>(lrecb + off);
        const double2 r1 = *reinterpret_cast<const double2*>(lrecb + off + 16);
        const double2 r2 = *reinterpret_cast<const double2*>(lrecb + off + 32);
        const double xi0 = r0.x - X0, xi1 = r0.y - X1, xi2 = r1.x - X2;
        const double e0 = r1.y - U0, e1 = r2.x - U1, e2 = r2.y - U2;
        const double y0 = xi0 + e0, y1 = xi1 + e1, y2 = xi2 + e2;
        // |y|^2 - |xi|^2 from two sums in the same order (exactly zero for an unstretched
        // bond), as the bond-based kernels form it
        const double L2 = __builtin_fma(xi2, xi2, __builtin_fma(xi1, xi1, xi0 * xi0));
        const double tq = __builtin_fma(y2, y2, __builtin_fma(y1, y1, y0 * y0)) - L2;
        const double q = tq * rcp64_1(L2);  // neither pass needs 1/|xi| itself
        // a break candidate: q at or above the lower edge of the decision (the rare branch
        // below decides, on the exact stretch within the margin)
        const bool cand = BREAK && live && !(e & kEntNoFail) && q >= P.q0;
        const bool alive = live && !cand;
        const double vj = VOLN ? lvol[(off * 0xAAABu) >> 21] : 1.0;
        if (PASS == 0) {
            const double s = sqrt1p_minus1(alive ? q : 0.0);
            D = __builtin_fma(VOLN ? L2 * vj : L2, s, D);  // |xi| e = |xi|^2 s; 0 for broken and padding slots
            if (cand) {
                if (stretch_exact(xi0, xi1, xi2, y0, y1, y2) >= P.s0) {
                    entw[ds] = static_cast<uint16_t>(e | kEntBroken);
                    A.bstep[ds] = step;
                } else {  // holds: the term the common path left out
                    D = __builtin_fma(VOLN ? L2 * vj : L2, sqrt1p_minus1(q), D);
                }
            }
        } else {
            const double g = one_minus_rsqrt1p(alive ? q : 0.0, sk);
            const double2 pj = lpair[(off * 0xAAABu) >> 21];  // off / 48: the neighbour's pair
            const double a = ka * (Ai + pj.x), b = kb * (Bi + pj.y);
            const double c = alive ? __builtin_fma(g, b - a, a) : 0.0;
            const double coef = VOLN ? c * vj : c;
            F0 = __builtin_fma(coef, y0, F0);
            F1 = __builtin_fma(coef, y1, F1);
            F2 = __builtin_fma(coef, y2, F2);
        }
    };

    for (int p = pa; p < p1; p += S) {
        const int T = rows_of(p);
        int64_t ent_next = ent + static_cast<int64_t>(T) * kWave;
        for (int q = p + 1; q < p + S && q < p1; ++q) ent_next += static_cast<int64_t>(rows_of(q)) * kWave;
        wave_sync();  // the previous piece is no longer read
        lds_reads_done();
        dma(p, ent);
        // s_waitcnt with vmcnt = 0 (expcnt and lgkmcnt at their no-wait maxima): the
        // piece's direct-to-LDS loads have landed
        __builtin_amdgcn_s_waitcnt(0x0F70);
        wave_sync();
#pragma unroll
        for (int t = 0; t < kPieceRows; t += 2) {
            if (t >= T) break;
            const uint16_t ea = lent[t * kWave + lane];
            slot(ea, ent + t * kWave + lane);
            if (t + 1 < T) slot(lent[(t + 1) * kWave + lane], ent + (t + 1) * kWave + lane);
        }
        ent = ent_next;
    }

    if (FP32) {
        D = Df;
        F0 = Ff0;
        F1 = Ff1;
        F2 = Ff2;
    }
    if (S > 1) {  // wavefront 0 adds the partial sums of 1..S-1 in that order
        if (wv > 0) {
            double* rr = red + (wv - 1) * kRed * kWave + lane;
            if (PASS == 0) {
                rr[0] = D;
            } else {
                rr[0] = F0;
                rr[kWave] = F1;
                rr[2 * kWave] = F2;
            }
        }
        __syncthreads();  // every wavefront of the workgroup reaches this once
        if (wv > 0) return;
#pragma unroll
        for (int w = 1; w < S; ++w) {
            const double* rr = red + (w - 1) * kRed * kWave + lane;
            if (PASS == 0) {
                D += rr[0];
            } else {
                F0 += rr[0];
                F1 += rr[kWave];
                F2 += rr[2 * kWave];
            }
        }
    }
    if (PASS == 0) {
        // theta_i = 3 V D / m_i (per-node volumes: inside D); padding nodes (1/m = 0) write zeros
        const double b = A.minv[node];
        const double theta = VOLN ? 3.0 * D * b : (3.0 * P.volume) * D * b;
        A.osb[node] = double2{theta * b, b};
        return;
    }
    if (VOLN) {
        node_update<MODE, FP32>(A, P, node, U0, U1, U2, F0, F1, F2);
    } else {
        const double V = P.volume;
        node_update<MODE, FP32>(A, P, node, U0, U1, U2, V * F0, V * F1, V * F2);
    }
}

template <bool FP32, int PASS, int MODE, bool VOLN>
hipError_t launch_osb_pmv(const StepArgs& a, int split, hipStream_t s)
{
    const dim3 grid(static_cast<unsigned>(a.nslices));
    switch (split) {
    case 1: hipLaunchKernelGGL((osb_staged<FP32, PASS, MODE, 1, VOLN>), grid, dim3(kWave), 0, s, a, a.pieces, a.slice_piece, a.slice_ptr); break;
    case 2: hipLaunchKernelGGL((osb_staged<FP32, PASS, MODE, 2, VOLN>), grid, dim3(2 * kWave), 0, s, a, a.pieces, a.slice_piece, a.slice_ptr); break;
    case 4: hipLaunchKernelGGL((osb_staged<FP32, PASS, MODE, 4, VOLN>), grid, dim3(4 * kWave), 0, s, a, a.pieces, a.slice_piece, a.slice_ptr); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool FP32, int PASS, int MODE>
hipError_t launch_osb_pm(const StepArgs& a, int split, hipStream_t s)
{
    return a.vol ? launch_osb_pmv<FP32, PASS, MODE, true>(a, split, s) : launch_osb_pmv<FP32, PASS, MODE, false>(a, split, s);
}

template <bool FP32>
hipError_t launch_osb_step_p(const StepArgs& a, int mode, int split, hipStream_t s)
{
    hipError_t e = mode != kModeForce ? launch_osb_pm<FP32, 0, kModeEC>(a, split, s)
                                      : launch_osb_pm<FP32, 0, kModeForce>(a, split, s);
    if (e != hipSuccess) return e;
    switch (mode) {
    case kModeEC: return launch_osb_pm<FP32, 1, kModeEC>(a, split, s);
    case kModeVV: return launch_osb_pm<FP32, 1, kModeVV>(a, split, s);
    case kModeVVInit: return launch_osb_pm<FP32, 1, kModeVVInit>(a, split, s);
    case kModeFE: return launch_osb_pm<FP32, 1, kModeFE>(a, split, s);
    case kModeForce: return launch_osb_pm<FP32, 1, kModeForce>(a, split, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_osb_dilation(const StepArgs& a, bool breaking, bool fp32, int split, hipStream_t s)
{
    if (a.nslices <= 0) return hipSuccess;
    if (fp32)
        return breaking ? launch_osb_pm<true, 0, kModeEC>(a, split, s) : launch_osb_pm<true, 0, kModeForce>(a, split, s);
    return breaking ? launch_osb_pm<false, 0, kModeEC>(a, split, s) : launch_osb_pm<false, 0, kModeForce>(a, split, s);
}

hipError_t launch_osb_step(const StepArgs& a, int mode, bool fp32, int split, hipStream_t s)
{
    if (a.nslices <= 0) return hipSuccess;
    return fp32 ? launch_osb_step_p<true>(a, mode, split, s) : launch_osb_step_p<false>(a, mode, split, s);
}

}  // namespace pdmi
