// pdmi_adjoint.hip -- reverse pass of the Euler-Cromer step with a frozen break schedule.
//
// Forward pass k (Sec. 2, Eq. simpleBond, with the semi-implicit Euler update):
//   v^{k+1} = d v^k + h (F(u^k; k) + A bhat),  u^{k+1} = u^k + dt v^{k+1},
//   then the boundary conditions overwrite prescribed components,
// with h = dt/rho and d = 1 - dt eta/rho.  A slot acts in pass k iff k < bstep (the pass
// in which it broke).  Reverse pass k, given lam_u = dL/du^{k+1} and the adjoint nu of
// the unconstrained v^{k+1} (zero on prescribed components):
//   dL/dk_b += h V_j (s/r)_b (y_b . nu_i)          (f_b = k_b V_j (s/r) y)
//   dL/dA   += h bhat_i . nu_i
//   lam_u    = [0 on displacement-controlled components] lam_u + h J_F^T nu
//   nu'      = d nu + dt lam_u on free components, 0 on prescribed ones (pass k-1)
// The tangent of one slot is k_b K_b with K_b = (1/L - 1/r) I + y y^T / r^3, symmetric and
// even in y.  With symmetric stiffness and schedule, (J_F^T nu)_i is the gather
//   sum over the family of i of k_b K_b (V_i nu_j - V_j nu_i),
// the same shape as the force, so the reverse pass walks the forward slot layout and
// needs no reverse-slot index.  1/L - 1/r = (1/L)(1 - (1+q)^(-1/2)) uses
// q = |y|^2/|xi|^2 - 1 with the numerator formed without cancellation, eta.(xi + y), and
// 1/r is 1/L less that.
#include "pdmi_device.h"

namespace pdmi {
namespace {

// One slot: adds k_b K_b (V_i nu_j - V_j nu_i) to J and returns the slot's
// stiffness-gradient increment h V_j (s/r) (y . nu_i).  An inactive slot (broken in an
// earlier pass, or padding) evaluates q = 0 with zero weights and adds nothing.
__device__ __forceinline__ double adj_slot(bool active, const double2 p0, const double2 p1, const double2 p2,
                                           double X0, double X1, double X2, double U0, double U1, double U2,
                                           const double nj[3], const double ni[3], double Vi, double Vj, double kb,
                                           double h, double J[3])
{
    const double xi0 = p0.x - X0, xi1 = p0.y - X1, xi2 = p1.x - X2;
    const double e0 = p1.y - U0, e1 = p2.x - U1, e2 = p2.y - U2;
    const double y0 = xi0 + e0, y1 = xi1 + e1, y2 = xi2 + e2;
    const double z0 = xi0 + y0, z1 = xi1 + y1, z2 = xi2 + y2;
    const double tq = __builtin_fma(e2, z2, __builtin_fma(e1, z1, e0 * z0));
    const double L2 = __builtin_fma(xi2, xi2, __builtin_fma(xi1, xi1, xi0 * xi0));
    const double iL = rsq64<1>(L2);
    const double q = active ? tq * (iL * iL) : 0.0;
    const double sr = iL * one_minus_rsqrt1p(q);  // s/r = 1/L - 1/r
    const double ir = iL - sr;                    // 1/r, no cancellation: sr is about |s| of iL
    const double ir3 = ir * ir * ir;
    const double w0 = Vi * nj[0] - Vj * ni[0], w1 = Vi * nj[1] - Vj * ni[1], w2 = Vi * nj[2] - Vj * ni[2];
    const double yw = __builtin_fma(y2, w2, __builtin_fma(y1, w1, y0 * w0));
    const double ka = active ? kb : 0.0;
    const double a = ka * sr, b = ka * (yw * ir3);
    J[0] += a * w0 + b * y0;
    J[1] += a * w1 + b * y1;
    J[2] += a * w2 + b * y2;
    const double yn = __builtin_fma(y2, ni[2], __builtin_fma(y1, ni[1], y0 * ni[0]));
    return active ? h * Vj * sr * yn : 0.0;
}

// Node tail of a reverse pass: body-force gradient, boundary masks, lam_u and next nu.
__device__ __forceinline__ void adj_node(const AdjArgs& A, const InstParams& P, int64_t node, const double ni[3],
                                         const double J[3], double h)
{
    const int32_t bcid = A.bc_id[node];
    if (bcid == kNodePad) return;
    const int64_t nn = A.nn;
    int code = 0;
    if (bcid >= 0) code = A.bc[bcid].code;
    if (P.has_body)
        A.gacc[node] += h * (A.bhat[node] * ni[0] + A.bhat[nn + node] * ni[1] + A.bhat[2 * nn + node] * ni[2]);
    const double damp = 1.0 - A.dt * P.eta / P.rho;
    for (int d = 0; d < 3; ++d) {
        const int kind = (code >> (2 * d)) & 3;
        const double lu = A.lam_u[d * nn + node];
        const double ln = (kind == 1 ? 0.0 : lu) + h * J[d];
        A.lam_u[d * nn + node] = ln;
        A.nu_out[3 * node + d] = kind == 0 ? damp * ni[d] + A.dt * ln : 0.0;
    }
}

// Per-slot streams of one row (index ds) and the neighbour data they point at.
struct AdjRow {
    int64_t ds;
    bool active;
    double kb, g;
    double2 p0, p1, p2;
    double nj[3];
    double Vj;
};

// Stiffness of a slot: KM = kKUniform (c), kKSlot (per-slot array) or kKNode
// (sqrt(k_i) sqrt(k_j) from per-node factors; ai = sqrt(k_i) of the own node).
constexpr int kKUniform = 0, kKSlot = 1, kKNode = 2;

template <int KM, bool VOLN>
__device__ __forceinline__ void adj_load(const AdjArgs& A, const InstParams& P, double ai, int64_t ds, int64_t j,
                                         AdjRow& r)
{
    const double2* __restrict__ rec = reinterpret_cast<const double2*>(A.rec);
    r.ds = ds;
    r.active = A.k < static_cast<int64_t>(A.bstep[ds]);
    r.p0 = rec[3 * j];
    r.p1 = rec[3 * j + 1];
    r.p2 = rec[3 * j + 2];
    r.nj[0] = A.nu_in[3 * j];
    r.nj[1] = A.nu_in[3 * j + 1];
    r.nj[2] = A.nu_in[3 * j + 2];
    r.kb = KM == kKSlot ? A.kslot[ds] : KM == kKNode ? ai * A.na[j] : P.c;
    r.Vj = VOLN ? A.vol[j] : P.volume;
    r.g = A.grad[ds];
}

// Sliced layout: G lanes per node, partial sums meet in a shuffle butterfly.  Two rows
// are loaded before either is computed (every slice's row count is even and the slot
// arrays end with spare rows, so the loads stay in bounds); padding slots point at the
// sentinel record, whose adjoint velocity is zero.
template <int G, int KM, bool VOLN>
__global__ __launch_bounds__(kBlock) void adjoint_sliced(AdjArgs A)
{
    constexpr int W = kWave / G;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t slice =
        wave_uniform(xcd_remap(blockIdx.x, gridDim.x) * (kBlock / kWave) + (threadIdx.x >> 6));
    if (slice >= A.nslices) return;
    const InstParams P = A.params[A.slice_inst[slice]];
    const int w = lane / G, g = lane % G;
    const int64_t node = slice * W + w;
    const double2* __restrict__ rec = reinterpret_cast<const double2*>(A.rec);
    const double2 o0 = rec[3 * node], o1 = rec[3 * node + 1], o2 = rec[3 * node + 2];
    const double ni[3] = {A.nu_in[3 * node], A.nu_in[3 * node + 1], A.nu_in[3 * node + 2]};
    const double Vi = VOLN ? A.vol[node] : P.volume;
    const double ai = KM == kKNode ? A.na[node] : 0.0;
    const double h = A.dt / P.rho;
    const int64_t base = wave_uniform(A.slice_ptr[slice]);
    const int T = A.slice_T[slice];
    double J[3] = {0.0, 0.0, 0.0};
    for (int t = 0; t < T; t += 2) {
        AdjRow r[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t ds = base + static_cast<int64_t>(t + u) * kWave + lane;
            const int32_t c = A.col[ds];
            adj_load<KM, VOLN>(A, P, ai, ds, static_cast<int32_t>(col_node(c)), r[u]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const double d = adj_slot(r[u].active, r[u].p0, r[u].p1, r[u].p2, o0.x, o0.y, o1.x, o1.y, o2.x, o2.y,
                                      r[u].nj, ni, Vi, r[u].Vj, r[u].kb, h, J);
            if (r[u].active) A.grad[r[u].ds] = r[u].g + d;
        }
    }
#pragma unroll
    for (int m = 1; m < G; m <<= 1)
        for (int d = 0; d < 3; ++d) J[d] += __shfl_xor(J[d], m);
    if (g != 0) return;
    adj_node(A, P, node, ni, J, h);
}

// Orders a wavefront's own LDS writes before its later LDS reads (no workgroup barrier).
__device__ __forceinline__ void adj_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Staged layout: a workgroup of S wavefronts per 64-node slice, one lane per node;
// wavefront w takes the slice's pieces w, w + S, ...  For each piece the wavefront
// stages the range's records (x, u^k), adjoint velocities and per-node weights in its
// own LDS area one piece ahead (the record and adjoint-velocity buffers end with spare
// entries, so the fixed windows need no clamping); per-slot break steps, stiffness and
// the gradient stream by row.  Padding entries point at an LDS sentinel (far record,
// zero adjoint velocity and weights).  Partial sums of J meet in LDS in a fixed order.
// The layout tables come as restrict parameters: their loads are then scalar, and a
// piece's descriptor does not wait behind the vector loads in flight.
template <int KM, bool VOLN, int S>
__global__ __launch_bounds__(kWave * S) void adjoint_lds(AdjArgs A, const int2* __restrict__ pieces,
                                                         const int32_t* __restrict__ slice_piece,
                                                         const int64_t* __restrict__ slice_ptr,
                                                         const int32_t* __restrict__ slice_order)
{
    constexpr bool KNODE = KM == kKNode;
    constexpr int kW = (kEntPad / 48 + 2) / 2 * 2;  // staged weights per array (sentinel at kEntPad / 48)
    constexpr int kRecChunks = kStageChunks + 3;     // records, then the sentinel record
    constexpr int kNuChunks = kStageChunks / 2 + 2;  // 2 * kStageChunks / 3 adjoint-velocity triples + sentinel
    constexpr int kEntChunks = kWave;                // one 8-row entry block
    constexpr int kWChunks = ((VOLN ? kW : 0) + (KNODE ? kW : 0)) / 2;
    constexpr int kLds = kRecChunks + kNuChunks + kEntChunks + kWChunks;
    static_assert(kStageChunks == 4 * kWave, "four record loads per piece");
    __shared__ double2 lds[S * kLds];
    __shared__ double red[S > 1 ? (S - 1) * 3 * kWave : 1];
    const int wv = S > 1 ? __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave) : 0;
    const int lane = threadIdx.x & (kWave - 1);
    double2* const lrec = lds + wv * kLds;
    const char* const lrecb = reinterpret_cast<const char*>(lrec);
    double* const lnu = reinterpret_cast<double*>(lrec + kRecChunks);
    uint16_t* const lent = reinterpret_cast<uint16_t*>(lrec + kRecChunks + kNuChunks);
    double* const lvol = reinterpret_cast<double*>(lrec + kRecChunks + kNuChunks + kEntChunks);
    double* const lna = lvol + (VOLN ? kW : 0);

    int64_t slice = wave_uniform(xcd_remap(blockIdx.x, gridDim.x));
    if (slice >= A.nslices) return;
    // the step kernels' processing order (each XCD's share longest first): the grid
    // ends on short slices when it does not fit the chip in one round
    if (slice_order) slice = __builtin_amdgcn_readfirstlane(slice_order[slice]);
    const InstParams P = A.params[A.slice_inst[slice]];
    const int64_t node = slice * kWave + lane;
    const double2* __restrict__ rec = reinterpret_cast<const double2*>(A.rec);
    const double2 o0 = rec[3 * node], o1 = rec[3 * node + 1], o2 = rec[3 * node + 2];
    const double ni[3] = {A.nu_in[3 * node], A.nu_in[3 * node + 1], A.nu_in[3 * node + 2]};
    const double Vi = VOLN ? A.vol[node] : P.volume;
    const double ai = KNODE ? A.na[node] : 0.0;
    const double h = A.dt / P.rho;
    const double2* __restrict__ ent2 = reinterpret_cast<const double2*>(A.ent);

    // sentinels: record far from every node; zero adjoint velocity and weights
    if (lane < 3) lrec[kStageChunks + lane] = lane == 0 ? double2{1e10, 1e10} : lane == 1 ? double2{1e10, 0.0} : double2{0.0, 0.0};
    if (lane < 4) lnu[kStageChunks + lane] = 0.0;
    if (VOLN && lane == 0) lvol[kEntPad / 48] = 0.0;
    if (KNODE && lane == 0) lna[kEntPad / 48] = 0.0;

    const int p0 = __builtin_amdgcn_readfirstlane(slice_piece[slice]);
    const int p1 = __builtin_amdgcn_readfirstlane(slice_piece[slice + 1]);
    auto rows_of = [&](int p) { return (pieces[__builtin_amdgcn_readfirstlane(p)].y >> 8) & 0xff; };
    int64_t ent = wave_uniform(slice_ptr[slice]);
    const int pa = p0 + wv;
    for (int q = p0; q < pa && q < p1; ++q) ent += static_cast<int64_t>(rows_of(q)) * kWave;

    double2 r0, r1, r2, r3, e0;
    double n0, n1, n2, n3, vs0 = 0.0, vs1 = 0.0, as0 = 0.0, as1 = 0.0;
    int vlen = 0;
    auto issue = [&](int p, int64_t e) {
        const int2 m = pieces[__builtin_amdgcn_readfirstlane(p)];
        const double2* rs = rec + 3 * static_cast<int64_t>(m.x) + lane;
        r0 = rs[0];
        r1 = rs[kWave];
        r2 = rs[2 * kWave];
        r3 = rs[3 * kWave];
        const double* ns = A.nu_in + 3 * static_cast<int64_t>(m.x) + lane;
        n0 = ns[0];
        n1 = ns[kWave];
        n2 = ns[2 * kWave];
        n3 = ns[3 * kWave];
        e0 = ent2[e / 8 + lane];
        if (VOLN || KNODE) {
            const int len = m.y & 0xff;
            vlen = len;
            if (VOLN) {
                vs0 = A.vol[m.x + min(lane, len - 1)];
                vs1 = A.vol[m.x + min(lane + kWave, len - 1)];
            }
            if (KNODE) {
                as0 = A.na[m.x + min(lane, len - 1)];
                as1 = A.na[m.x + min(lane + kWave, len - 1)];
            }
        }
    };
    auto commit = [&]() {
        lrec[lane] = r0;
        lrec[lane + kWave] = r1;
        lrec[lane + 2 * kWave] = r2;
        lrec[lane + 3 * kWave] = r3;
        lnu[lane] = n0;
        lnu[lane + kWave] = n1;
        lnu[lane + 2 * kWave] = n2;
        lnu[lane + 3 * kWave] = n3;
        reinterpret_cast<double2*>(lent)[lane] = e0;
        if (VOLN) {
            if (lane < vlen) lvol[lane] = vs0;
            if (lane + kWave < vlen) lvol[lane + kWave] = vs1;
        }
        if (KNODE) {
            if (lane < vlen) lna[lane] = as0;
            if (lane + kWave < vlen) lna[lane + kWave] = as1;
        }
    };
    // one slot of row t of the current piece; its break step, gradient and stiffness were
    // loaded with the rest of the piece's rows (bs, gr, kr)
    double J[3] = {0.0, 0.0, 0.0};
    int32_t bs[kPieceRows];
    double gr[kPieceRows], kr[kPieceRows];
    auto slot = [&](int t, int64_t ds, uint16_t e) {
        const uint32_t off = e & kEntOff;  // byte offset of the record; 3 * index = off / 16 for nu
        const double2 q0 = *reinterpret_cast<const double2*>(lrecb + off);
        const double2 q1 = *reinterpret_cast<const double2*>(lrecb + off + 16);
        const double2 q2 = *reinterpret_cast<const double2*>(lrecb + off + 32);
        const double* nu = lnu + off / 16;
        const double nj[3] = {nu[0], nu[1], nu[2]};
        const uint32_t widx = (off * 0xAAABu) >> 21;  // off / 48
        const bool active = A.k < static_cast<int64_t>(bs[t]);
        const double kb = KM == kKSlot ? kr[t] : KNODE ? ai * lna[widx] : P.c;
        const double Vj = VOLN ? lvol[widx] : P.volume;
        const double d = adj_slot(active, q0, q1, q2, o0.x, o0.y, o1.x, o1.y, o2.x, o2.y, nj, ni, Vi, Vj, kb, h, J);
        if (active) A.grad[ds] = gr[t] + d;
    };

    if (pa < p1) {
        issue(pa, ent);
        for (int p = pa; p < p1; p += S) {
            const int T = rows_of(p);
            int64_t ent_next = ent + static_cast<int64_t>(T) * kWave;
            for (int q = p + 1; q < p + S && q < p1; ++q) ent_next += static_cast<int64_t>(rows_of(q)) * kWave;
            adj_wave_sync();  // the previous piece is no longer read
            commit();
            // the piece's per-slot streams, all eight rows of its block at once (rows past T
            // belong to the next piece or the spare rows and are not used), issued before
            // the next piece's prefetch: vector-memory loads complete in order, so the rows
            // wait for these only and the prefetch stays in flight behind them
#pragma unroll
            for (int t = 0; t < kPieceRows; ++t) {
                const int64_t ds = ent + t * kWave + lane;
                bs[t] = A.bstep[ds];
                gr[t] = A.grad[ds];
                if (KM == kKSlot) kr[t] = A.kslot[ds];
            }
            if (p + S < p1) issue(p + S, ent_next);
            adj_wave_sync();  // the piece's LDS copy is complete
#pragma unroll
            for (int t = 0; t < kPieceRows; ++t) {
                if (t >= T) break;
                slot(t, ent + t * kWave + lane, lent[t * kWave + lane]);
            }
            ent = ent_next;
        }
    }
    if (S > 1) {
        if (wv > 0) {
            double* r = red + (wv - 1) * 3 * kWave + lane;
            r[0] = J[0];
            r[kWave] = J[1];
            r[2 * kWave] = J[2];
        }
        __syncthreads();  // every wavefront of the workgroup reaches this once
        if (wv > 0) return;
#pragma unroll
        for (int w = 1; w < S; ++w) {
            const double* r = red + (w - 1) * 3 * kWave + lane;
            J[0] += r[0];
            J[1] += r[kWave];
            J[2] += r[2 * kWave];
        }
    }
    adj_node(A, P, node, ni, J, h);
}

__global__ __launch_bounds__(kBlock) void bstep_init_kernel(int32_t* bstep, const int32_t* col, const uint16_t* ent,
                                                            int64_t ns)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= ns) return;
    const bool broken = col ? col[i] < 0 : (ent[i] & kEntBroken) != 0;
    bstep[i] = broken ? kBrokeBefore : kNeverBroke;
}

__global__ __launch_bounds__(kBlock) void flags_at_kernel(const int32_t* bstep, int32_t* col, uint16_t* ent,
                                                          int64_t ns, int64_t step)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= ns) return;
    const bool broken = static_cast<int64_t>(bstep[i]) < step;
    if (col) {
        const int32_t c = col[i], j = c ^ (c >> 31);
        col[i] = broken ? ~j : j;
    } else {
        const uint16_t e = ent[i];
        ent[i] = static_cast<uint16_t>((e & ~kEntBroken) | (broken ? kEntBroken : 0));
    }
}

__global__ void adj_seed_kernel(double* lam_u, int64_t nn, const int64_t* sensors, const double* dldu, int64_t m)
{
    const int d = threadIdx.x;
    if (blockIdx.x != 0 || d >= 3) return;
    for (int64_t p = 0; p < m; ++p) lam_u[d * nn + sensors[p]] += dldu[3 * p + d];
}

__global__ __launch_bounds__(kBlock) void adj_nu0_kernel(double* nu, const double* lam_u, const int32_t* bc_id,
                                                         const BCRec* bc, int64_t nn, double dt)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= nn) return;
    const int32_t id = bc_id[i];
    const int code = id >= 0 ? bc[id].code : 0;
    for (int d = 0; d < 3; ++d) {
        const bool free_comp = id != kNodePad && ((code >> (2 * d)) & 3) == 0;
        nu[3 * i + d] = free_comp ? dt * lam_u[d * nn + i] : 0.0;
    }
}

// Deterministic single-workgroup sum.
__global__ __launch_bounds__(kBlock) void sum_kernel(const double* x, int64_t n, double* out)
{
    __shared__ double part[kBlock];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) acc += x[i];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (static_cast<int>(threadIdx.x) < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0];
}

__global__ void set_i64_kernel(int64_t* p, int64_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

template <int G, int KM, bool VOLN>
void adj_launch_sliced(const AdjArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL((adjoint_sliced<G, KM, VOLN>), dim3(static_cast<unsigned>((a.nslices + 3) / 4)),
                       dim3(kBlock), 0, s, a);
}

template <int KM, bool VOLN>
hipError_t adj_launch_kv(const AdjArgs& a, const int32_t* order, bool staged, int lanes, hipStream_t s)
{
    const dim3 grid(static_cast<unsigned>(a.nslices));
    if (staged) {
        switch (lanes) {  // wavefronts per slice
        case 1: hipLaunchKernelGGL((adjoint_lds<KM, VOLN, 1>), grid, dim3(kWave), 0, s, a, a.pieces, a.slice_piece, a.slice_ptr, order); break;
        case 2: hipLaunchKernelGGL((adjoint_lds<KM, VOLN, 2>), grid, dim3(2 * kWave), 0, s, a, a.pieces, a.slice_piece, a.slice_ptr, order); break;
        case 4: hipLaunchKernelGGL((adjoint_lds<KM, VOLN, 4>), grid, dim3(4 * kWave), 0, s, a, a.pieces, a.slice_piece, a.slice_ptr, order); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (lanes) {
    case 1: adj_launch_sliced<1, KM, VOLN>(a, s); break;
    case 4: adj_launch_sliced<4, KM, VOLN>(a, s); break;
    case 16: adj_launch_sliced<16, KM, VOLN>(a, s); break;
    case 64: adj_launch_sliced<64, KM, VOLN>(a, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int KM>
hipError_t adj_launch_k(const AdjArgs& a, const int32_t* order, bool staged, int lanes, hipStream_t s)
{
    return a.vol ? adj_launch_kv<KM, true>(a, order, staged, lanes, s)
                 : adj_launch_kv<KM, false>(a, order, staged, lanes, s);
}

unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_adjoint_ordered(const AdjArgs& a, const int32_t* slice_order, bool staged, int lanes,
                                  hipStream_t s)
{
    if (a.nslices <= 0) return hipSuccess;
    if (a.kslot) return adj_launch_k<kKSlot>(a, slice_order, staged, lanes, s);
    if (a.na) return adj_launch_k<kKNode>(a, slice_order, staged, lanes, s);
    return adj_launch_k<kKUniform>(a, slice_order, staged, lanes, s);
}

hipError_t launch_adjoint(const AdjArgs& a, bool staged, int lanes, hipStream_t s)
{
    return launch_adjoint_ordered(a, nullptr, staged, lanes, s);
}

hipError_t launch_bstep_init(int32_t* bstep, const int32_t* col, const uint16_t* ent, int64_t ns, hipStream_t s)
{
    if (ns <= 0) return hipSuccess;
    hipLaunchKernelGGL(bstep_init_kernel, dim3(blocks_for(ns)), dim3(kBlock), 0, s, bstep, col, ent, ns);
    return hipGetLastError();
}

hipError_t launch_flags_at(const int32_t* bstep, int32_t* col, uint16_t* ent, int64_t ns, int64_t step, hipStream_t s)
{
    if (ns <= 0) return hipSuccess;
    hipLaunchKernelGGL(flags_at_kernel, dim3(blocks_for(ns)), dim3(kBlock), 0, s, bstep, col, ent, ns, step);
    return hipGetLastError();
}

hipError_t launch_adj_seed(double* lam_u, int64_t nn, const int64_t* sensors, const double* dldu, int64_t m,
                           hipStream_t s)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(adj_seed_kernel, dim3(1), dim3(kWave), 0, s, lam_u, nn, sensors, dldu, m);
    return hipGetLastError();
}

hipError_t launch_adj_nu0(double* nu, const double* lam_u, const int32_t* bc_id, const BCRec* bc, int64_t nn,
                          double dt, hipStream_t s)
{
    if (nn <= 0) return hipSuccess;
    hipLaunchKernelGGL(adj_nu0_kernel, dim3(blocks_for(nn)), dim3(kBlock), 0, s, nu, lam_u, bc_id, bc, nn, dt);
    return hipGetLastError();
}

hipError_t launch_sum(const double* x, int64_t n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kBlock), 0, s, x, n, out);
    return hipGetLastError();
}

hipError_t launch_set_i64(int64_t* p, int64_t value, hipStream_t s)
{
    hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(kWave), 0, s, p, value);
    return hipGetLastError();
}

}  // namespace pdmi
