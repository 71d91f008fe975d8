// pdmi_kernels.hip -- gfx950 kernels around the step: local damage, the velocity-Verlet
// drift, the step counter and weighted sums over node sets; the launchers that
// dispatch to the step-kernel launcher files.
#include "pdmi_device.h"

#include <mutex>

namespace pdmi {
namespace {

// 1 - d of a slot: 0 broken, the secant ratio of its law once softened, 1 otherwise
// (local damage is 1 - sum (1 - d) V_j / sum V_j; with the brittle law d is 0 or 1).
__device__ __forceinline__ double intact_share(const DamageArgs& A, const InstParams& P, int64_t ds, bool broken,
                                               bool soft)
{
    if (broken) return 0.0;
    if (!soft || P.nlaw == 0) return 1.0;
    const LawRec& L = A.laws[P.law_off + (P.nlaw > 1 ? A.cls[ds] : 0)];
    return 1.0 - law_damage(L, A.smax[ds]);
}

// Local damage on the staged layout.
__global__ __launch_bounds__(kWave) void damage_staged(DamageArgs A)
{
    const int lane = threadIdx.x;
    const int64_t slice = wave_uniform(xcd_remap(blockIdx.x, gridDim.x));
    if (slice >= A.nslices) return;
    const InstParams P = A.params[A.slice_inst[slice]];
    const int64_t node = slice * kWave + lane;
    const int p0 = A.slice_piece[slice], p1 = A.slice_piece[slice + 1];
    int64_t ent = A.slice_ptr[slice];
    double num = 0.0, den = 0.0;
    for (int p = p0; p < p1; ++p) {
        const int2 m = A.pieces[p];
        const int T = (m.y >> 8) & 0xff;
        for (int t = 0; t < T; ++t) {
            const int64_t ds = ent + t * kWave + lane;
            const uint16_t e = A.ent[ds];
            const int off = e & kEntOff;
            if (off == kEntPad) continue;  // padding
            const double vj = A.vol ? A.vol[m.x + off / 48] : P.volume;
            den += vj;
            num += intact_share(A, P, ds, (e & kEntBroken) != 0, (e & kEntSoft) != 0) * vj;
        }
        ent += static_cast<int64_t>(T) * kWave;
    }
    A.phi[node] = den > 0.0 ? 1.0 - num / den : 0.0;
}

// Velocity-Verlet position update u_{k+1} = u_k + dt v_k + dt^2/2 a_k with the
// displacement constraints of t_{k+1}; one thread per device node.
template <bool FP32>
__global__ __launch_bounds__(kBlock) void drift_kernel(StepArgs A)
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
        const double u = FP32 ? A.um_in[d * nn + node] : ri[3 + d];
        double un = (u + dt * A.v[d * nn + node]) + hdt2 * A.a[d * nn + node];
        if (constrained(bc, d)) un = bc_disp(bc, d, t1, u, dt);
        if (FP32) {
            reinterpret_cast<float*>(ro + 3)[d] = static_cast<float>(un);
            A.um_out[d * nn + node] = un;
        } else {
            ro[3 + d] = un;
        }
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
        const int64_t ds = base + static_cast<int64_t>(t) * kWave + lane;
        const int32_t c = A.col[ds];
        const int32_t j = static_cast<int32_t>(col_node(c));
        if (j == A.sentinel) continue;  // padding
        const double vj = A.vol ? A.vol[j] : P.volume;
        den += vj;
        num += intact_share(A, P, ds, c < 0, (c & kColSoft) != 0) * vj;
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

// Weighted sum over a node set: out[d] = sum over idx[0..m) of w_i field(i, d), with
// field(i, d) = field[i * snode + d * scomp] and w_i = wv[i], or w when wv is nullptr.
// One workgroup; each thread sums a strided subsequence, then a fixed-shape tree in
// LDS (deterministic).
__global__ __launch_bounds__(kBlock) void set_sum_kernel(const double* __restrict__ field, int64_t snode,
                                                        int64_t scomp, const double* __restrict__ wv, double w,
                                                        const int64_t* __restrict__ idx, int64_t m,
                                                        double* __restrict__ out, const int64_t* __restrict__ map)
{
    __shared__ double red[3][kBlock];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t r = threadIdx.x; r < m; r += kBlock) {
        const int64_t i = map ? map[idx[r]] : idx[r];
        const double wi = wv ? wv[i] : w;
        const double* f = field + i * snode;
        s0 += wi * f[0];
        s1 += wi * f[scomp];
        s2 += wi * f[2 * scomp];
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h)
            for (int d = 0; d < 3; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

// Device-to-device readout in the caller's order: out[i * ncomp + d] =
// src[off + dnode[i] * snode + d * scomp] for i < n (dnode: device node of user node i).
__global__ __launch_bounds__(kBlock) void export_nodes_kernel(const double* __restrict__ src, int64_t snode,
                                                             int64_t scomp, int64_t off,
                                                             const int64_t* __restrict__ dnode, int64_t n,
                                                             int ncomp, double* __restrict__ out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t dn = dnode[i];
    for (int d = 0; d < ncomp; ++d) out[i * ncomp + d] = src[off + dn * snode + d * scomp];
}

}  // namespace

hipError_t launch_export_nodes(const double* src, int64_t snode, int64_t scomp, int64_t off, const int64_t* dnode,
                               int64_t n, int ncomp, double* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(export_nodes_kernel, dim3(static_cast<unsigned>((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, src, snode, scomp, off, dnode, n, ncomp, out);
    return hipGetLastError();
}

bool lanes_supported(int lanes) { return lanes == 1 || lanes == 4 || lanes == 16 || lanes == 64; }

bool split_supported(int split) { return split == 1 || split == 2 || split == 4; }

hipError_t launch_drift(const StepArgs& a, bool fp32, hipStream_t s)
{
    if (a.nn <= 0) return hipSuccess;
    const dim3 grid(static_cast<unsigned>((a.nn + kBlock - 1) / kBlock)), block(kBlock);
    if (fp32)
        hipLaunchKernelGGL(drift_kernel<true>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(drift_kernel<false>, grid, block, 0, s, a);
    return hipGetLastError();
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

hipError_t launch_step_staged(const StepArgs& a, int mode, bool fp32, int split, bool ext, hipStream_t s)
{
    return fp32 ? launch_step_staged_f32(a, mode, split, ext, s) : launch_step_staged_f64(a, mode, split, ext, s);
}

hipError_t launch_damage_staged(const DamageArgs& a, hipStream_t s)
{
    if (a.nslices <= 0) return hipSuccess;
    hipLaunchKernelGGL(damage_staged, dim3(static_cast<unsigned>(a.nslices)), dim3(kWave), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_set_sum(const double* field, int64_t snode, int64_t scomp, const double* wv, double w,
                          const int64_t* idx, int64_t m, double* out, hipStream_t s, const int64_t* map)
{
    hipLaunchKernelGGL(set_sum_kernel, dim3(1), dim3(kBlock), 0, s, field, snode, scomp, wv, w, idx, m, out, map);
    return hipGetLastError();
}

// Device scratch of the allocation-free set readout: kScratchNodes node ids, then the
// three sums (as doubles).  One array per GPU, held until the process ends.  In host code
// `scratch` names a host-side stand-in, never the device memory: kernels and copies take
// the address scratch_address() looked up on the device.
static __device__ __align__(256) int64_t scratch[kScratchNodes + 4];

hipError_t scratch_address(int device, int64_t** out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static int64_t* addr[kMaxDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        addr[device] = static_cast<int64_t*>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

// Exact stretch of m bonds (xi, y: m x 3 row-major), one work-item per bond.
__global__ __launch_bounds__(kBlock) void stretch_exact_kernel(const double* xi, const double* y, double* s, int64_t m)
{
    const int64_t b = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (b >= m) return;
    s[b] = stretch_exact(xi[3 * b], xi[3 * b + 1], xi[3 * b + 2], y[3 * b], y[3 * b + 1], y[3 * b + 2]);
}

hipError_t launch_stretch_exact(const double* xi, const double* y, double* s, int64_t m, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(stretch_exact_kernel, dim3(static_cast<unsigned>((m + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       st, xi, y, s, m);
    return hipGetLastError();
}

hipError_t launch_advance(int64_t* step_base, int64_t by, hipStream_t s)
{
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, step_base, by);
    return hipGetLastError();
}

}  // namespace pdmi
