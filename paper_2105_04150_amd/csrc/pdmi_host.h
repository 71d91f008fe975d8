// pdmi_host.h -- host runtime behind the C ABI of include/pdmi.h (private to the library).
//
// The runtime validates arguments, searches the family (cell list on the host; the family
// is built once per model, paper Sec. 3), renumbers nodes, lays the problem out on the
// device (sliced or staged), fills the boundary-condition and material tables, steps in
// stream order with hipGraph replay and reads out in the caller's node and slot order.
//
//   pdmi_layout.cpp      family search, node order, device layout, new problems
//   pdmi_upload.cpp      parameter, table and state uploads; readouts to the host
//   pdmi_run.cpp         stepping, force evaluation, damage and set sums
//   pdmi_api.cpp         C ABI: context, family, material, loads, integrator
//   pdmi_api_state.cpp   C ABI: stepping, readouts, state and checkpoints, mapping, info
//   pdmi_api_adjoint.cpp C ABI: the recorded forward run and the reverse pass
//
// Every source is built with -ffp-contract=off: host arithmetic that the oracle repeats
// (the family test ((dx^2 + dy^2) + dz^2) <= delta^2 among it) is evaluated as written.
#pragma once

#include "pdmi.h"
#include "pdmi_internal.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <limits>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

namespace pdmi {
namespace host {

constexpr int kDefaultLanes = 1;
// spare slot rows after the last slice: the sliced kernel prefetches kRowUnroll rows
// ahead, the staged kernel reads a full piece of stiffness rows
constexpr size_t kSpareRows = kRowUnroll > kPieceRows ? kRowUnroll : kPieceRows;
constexpr int64_t kMaxGap = 12;      // staged ranges absorb gaps of up to this many unused records
constexpr int64_t kGraphChunk = 64;  // steps per captured graph (even: buffer parity repeats)

struct PdError : std::exception {
    int code;
    std::string msg;
    PdError(int c, std::string m) : code(c), msg(std::move(m)) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw PdError(code, msg); }

inline void hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess) fail(e == hipErrorOutOfMemory ? PD_ENOMEM : PD_EHIP,
                              std::string(what) + ": " + hipGetErrorString(e));
}

// Owning device allocation.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t n)
    {
        release();
        if (n == 0) n = 16;
        hip_check(hipMalloc(&p, n), "hipMalloc");
        bytes = n;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

struct Inst {
    int64_t n = 0, nnz = 0;
    double horizon = 0.0;
    std::vector<double> x;           // user order, n*3
    std::vector<int64_t> row_ptr;    // user CSR
    std::vector<int32_t> col;
    // material and loads
    double rho = 1.0, c = 1.0, s0 = std::numeric_limits<double>::infinity(), eta = 0.0, volume = 1.0;
    std::vector<double> vols;        // user order; empty = uniform
    std::vector<double> kslot;       // user CSR order; empty = c
    std::vector<double> knode;       // user order, per-node stiffness (bond: sqrt(k_i k_j)); empty = none
    std::vector<double> bhat;        // user order n*3; empty = none
    double bmag = 0.0;
    std::vector<uint8_t> bc_kind, bc_sched;  // n*3
    std::vector<double> bc_val;              // n*3
    double ramp_T = 1.0;                     // duration of the fifth-order ramp schedule
    std::vector<uint8_t> nofail;             // user order, no-failure zone flags; empty = none
    std::vector<LawRec> laws;                // damage laws (bond classes); empty = the brittle law with s0
    pd_corrections corr{};                   // stiffness corrections
    bool has_corr = false;
    double corr_v0 = 0.0;                    // largest family volume (surface correction)
    std::vector<uint8_t> cls;                // user CSR order: law of every slot; empty = law 0
    int64_t user_off = 0;                    // first entry of the instance in the device node map
    bool osb = false;                        // the state-based linear solid instead of the PMB
    double osb_K = 0.0, osb_G = 0.0;         // its bulk and shear moduli
    // device layout
    std::vector<int64_t> perm;       // device-local node -> user node, -1 = padding
    std::vector<int64_t> iperm;      // user node -> device-local node
    std::vector<int32_t> dslot_user; // device slot (instance-local) -> user slot, -1 = padding
    std::vector<int64_t> s_start;    // first device slot (instance-local) of every slice
    std::vector<int64_t> s_T;        // 64-wide slot rows of every slice (sliced layout)
    std::vector<int2> pieces;        // staged layout: {first device node, len | rows << 8}
    std::vector<int32_t> slice_piece;  // staged layout: first piece of each slice (+ end), local
    std::vector<uint8_t> ent_idx;    // staged layout: range index of every device slot
    std::vector<int64_t> rev_slot;   // user slot of the reverse bond (filled on first use)
    bool k_sym = true;               // both slots of every bond carry the same stiffness
    bool br_sym = true;              // both slots of every bond share the broken flag
    int64_t node_off = 0, n_pad = 0, slice_off = 0, nslices = 0, dslot_off = 0, n_dslots = 0;
};

}  // namespace host
}  // namespace pdmi

struct pd_ctx {
    using DevBuf = pdmi::host::DevBuf;

    int device = 0;
    int precision = PD_FP64;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    std::vector<pdmi::host::Inst> inst;
    int order = PD_ORDER_NATURAL;
    bool order_auto = false;         // the autotuner may change the device node order
    int lanes = pdmi::host::kDefaultLanes;  // sliced: lanes per node; staged: wavefronts per slice
    int mapping = PD_MAP_SLICED;
    int scheme = PD_EULER_CROMER;
    double dt = 1.0e-7;
    int64_t step = 0;
    int cur = 0;                     // node-record buffer holding u of level `step`
    bool a_valid = false;            // velocity Verlet: a holds the acceleration of level `step`
    bool vv_ahead = false;           // velocity Verlet: buffer 1-cur holds u of level step+1
    bool built = false;
    bool use_graphs = true;

    int64_t nn = 0, ns = 0, nslices = 0;
    bool has_stiff = false, has_vol = false, has_body = false, has_knode = false;
    bool has_nofail = false;         // some slot carries the no-failure bit
    bool has_laws = false;           // some instance has damage laws (smax, laws allocated)
    bool has_osb = false;            // the instances run the state-based linear solid
    bool corr_k = false;             // corrections formed per slot in the kernel (no stiffness stream)
    DevBuf rec[2], um[2], v, a, col, kslot, vol, bhat, slice_ptr, slice_T, slice_inst, params, bc_id, bc,
        step_base, status, phi, pieces, slice_piece, ent;
    DevBuf force, rset, rsum;        // force readout: F (SoA), node list and sum of a resultant
    DevBuf laws, cls, smax;          // damage laws, per-slot law (several per instance), stretch state
    DevBuf osb, minv;                // state-based model: node pairs {theta/m, 1/m}, 1/m
    DevBuf cfv;                      // corrections per slot: family volume per node
    DevBuf unode;                    // device node of every user node (instances concatenated)
    DevBuf slice_order;              // staged layout: slices in processing order (locality)

    // adjoint: per-slot break steps (recorded by every step while allocated) and the
    // (u, v) checkpoints of the last recorded forward run
    DevBuf bstep, ck;
    DevBuf na, nw;                   // per-node stiffness: sqrt(k_i) and sqrt(k_j) V_j (entry nn: 0)
    bool tape_valid = false;
    int64_t tape_step0 = 0, tape_nsteps = 0, tape_every = 0;
    int64_t tape_id = 0;             // id of the last recording (unique in the process, > 0)

    // graphs: [parity][mode] for chunks of kGraphChunk steps
    hipGraphExec_t graph[2][4] = {{nullptr}};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;

    ~pd_ctx()
    {
        drop_graphs();
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
    void drop_graphs()
    {
        for (auto& row : graph)
            for (auto& g : row)
                if (g) {
                    (void)hipGraphExecDestroy(g);
                    g = nullptr;
                }
    }
};

namespace pdmi {
namespace host {

// Run f, turning a thrown failure into the ABI's status code and the context's message.
template <typename F>
int guarded(pd_ctx* ctx, F&& f)
{
    try {
        f();
        if (ctx) ctx->err.clear();
        return PD_OK;
    } catch (const PdError& e) {
        if (ctx) ctx->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        if (ctx) ctx->err = "host allocation failed";
        return PD_ENOMEM;
    } catch (const std::exception& e) {
        if (ctx) ctx->err = e.what();
        return PD_EINVAL;
    } catch (...) {
        if (ctx) ctx->err = "unknown failure";
        return PD_EINVAL;
    }
}

inline void set_device(pd_ctx* ctx) { hip_check(hipSetDevice(ctx->device), "hipSetDevice"); }

// The step kernels with the bond-model branch: no-failure zones or damage laws present.
inline bool ext_kernels(const pd_ctx* ctx) { return ctx->has_nofail || ctx->has_laws; }

inline void require_built(const pd_ctx* ctx)
{
    if (!ctx->built) fail(PD_ESTATE, "no problem: call pd_build_family first");
}

inline Inst& instance(pd_ctx* ctx, int32_t inst)
{
    require_built(ctx);
    if (inst < 0 || inst >= static_cast<int32_t>(ctx->inst.size()))
        fail(PD_EINVAL, "instance index out of range");
    return ctx->inst[inst];
}

inline unsigned n_threads()
{
    unsigned t = std::thread::hardware_concurrency();
    return std::max(1u, std::min(t, 16u));
}

template <typename F>
void parallel_for(int64_t n, F&& f)
{
    const unsigned nt = n_threads();
    if (nt <= 1 || n < 4096) {
        f(int64_t(0), n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        const int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back([&f, lo, hi] { f(lo, hi); });
    }
    for (auto& x : th) x.join();
}

// Setup-path copy from pageable host memory; returns once the source may be freed.
inline void upload(const DevBuf& b, const void* src, size_t bytes, size_t offset_bytes, hipStream_t s)
{
    if (bytes == 0) return;
    if (offset_bytes + bytes > b.bytes) fail(PD_EINVAL, "internal: upload beyond buffer");
    hip_check(hipMemcpyAsync(static_cast<char*>(b.p) + offset_bytes, src, bytes, hipMemcpyHostToDevice, s),
              "hipMemcpyAsync H2D");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

inline void download(void* dst, const DevBuf& b, size_t bytes, size_t offset_bytes, hipStream_t s)
{
    if (bytes == 0) return;
    if (offset_bytes + bytes > b.bytes) fail(PD_EINVAL, "internal: download beyond buffer");
    hip_check(hipMemcpyAsync(dst, static_cast<const char*>(b.p) + offset_bytes, bytes, hipMemcpyDeviceToHost, s),
              "hipMemcpyAsync D2H");
}

inline void sync(pd_ctx* ctx) { hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize"); }

inline bool fp32(const pd_ctx* ctx) { return ctx->precision == PD_FP32; }

// Bytes of one node-record buffer: nn records, the sentinel and kRecPad spare records.
inline size_t rec_bytes(int64_t nn) { return static_cast<size_t>(nn + 1 + kRecPad) * 48; }

// The state of every instance in user order, kept across a rebuild of the device problem.
struct HostState {
    std::vector<std::vector<double>> u, v, a;   // per instance, n*3
    std::vector<std::vector<uint8_t>> broken;   // per instance, nnz
    std::vector<std::vector<double>> smax;      // per instance, nnz (empty without damage laws)
};

// ---- pdmi_layout.cpp
void family_search(int64_t n, const double* x, double delta, std::vector<int64_t>& row_ptr,
                   std::vector<int32_t>& col);
void build_layout(pd_ctx* ctx, const HostState* S);
void validate_coords(int64_t n, const double* coords, double horizon);
double validate_family(int64_t n, const double* x, const int64_t* row_ptr, const int32_t* col);
void new_problem(pd_ctx* ctx, int32_t ninst, const int64_t* n, const double* const* coords, const double* horizon,
                 int order, const int64_t* user_row_ptr = nullptr, const int32_t* user_col = nullptr);

// ---- pdmi_upload.cpp
void upload_params(pd_ctx* ctx);
void upload_bcs(pd_ctx* ctx);
void upload_stiffness(pd_ctx* ctx, int32_t only = -1);
void upload_node_weights(pd_ctx* ctx);
void upload_volumes(pd_ctx* ctx);
void upload_osb(pd_ctx* ctx);
void osb_checks(const pd_ctx* ctx);
void upload_body(pd_ctx* ctx);
void upload_state(pd_ctx* ctx, const Inst& I, const double* u, const double* v, const double* a);
const std::vector<int64_t>& reverse_slots(Inst& I);
void init_break_steps(pd_ctx* ctx, const Inst& I);
void upload_laws(pd_ctx* ctx);
std::vector<double> smax_of(pd_ctx* ctx, const Inst& I);
void upload_col(pd_ctx* ctx, Inst& I, const uint8_t* broken, bool keep_bsteps = false,
                const double* smax = nullptr);
std::vector<uint8_t> broken_of(pd_ctx* ctx, const Inst& I);
std::vector<double> soa_of(pd_ctx* ctx, const Inst& I, const DevBuf& buf);
std::vector<double> u_of(pd_ctx* ctx, const Inst& I);
HostState snapshot(pd_ctx* ctx);

// Whether a per-slot array (nullptr: uniform) is equal on the two slots of every bond.
template <typename T>
bool bond_symmetric(Inst& I, const T* a)
{
    if (!a) return true;
    const std::vector<int64_t>& rev = reverse_slots(I);
    std::atomic<bool> ok{true};
    parallel_for(I.nnz, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b)
            if (rev[b] < 0 || a[b] != a[rev[b]]) {
                ok = false;
                return;
            }
    });
    return ok;
}

// ---- pdmi_run.cpp
StepArgs step_args(pd_ctx* ctx, int in, int out, int64_t step_local);
int step_mode(int scheme);
hipGraphExec_t chunk_graph(pd_ctx* ctx, int mode, int parity);
void launch_one(pd_ctx* ctx, int mode, int in, int out, int64_t step_local);
void eval_force(pd_ctx* ctx);
void do_steps(pd_ctx* ctx, int64_t nsteps);
void check_status(pd_ctx* ctx);
void reset_flags_after_state_change(pd_ctx* ctx, bool a_given);
void reset_laws(pd_ctx* ctx);
void adjoint_checks(pd_ctx* ctx);
void check_symmetric(const Inst& I);
void launch_ec(pd_ctx* ctx, const StepArgs& A);
void launch_damage_now(pd_ctx* ctx);
int get_nodes_dev(pd_ctx* ctx, int32_t inst, double* out, int what);
std::vector<int64_t> device_nodes(const Inst& I, int64_t m, const int64_t* nodes);
void set_sum(pd_ctx* ctx, const std::vector<int64_t>& idx, const double* field, int64_t snode, int64_t scomp,
             const double* wv, double w, double out[3]);

}  // namespace host

// the reverse pass with the staged layout's slices in the order given (nullptr: dispatch
// order; defined beside the reverse kernels)
hipError_t launch_adjoint_ordered(const AdjArgs& a, const int32_t* slice_order, bool staged, int lanes,
                                  hipStream_t s);
}  // namespace pdmi
