// pdmi_host.cpp -- host runtime behind the C ABI of include/pdmi.h.
//
// Responsibilities: argument validation, the family search (cell list on the host;
// the family is built once per model, paper Sec. 3), node renumbering, the sliced
// device layout, boundary-condition tables, stream-ordered stepping with hipGraph
// replay, and synchronising readout in the caller's node and slot order.
//
// Built with -ffp-contract=off: the family test ((dx^2 + dy^2) + dz^2) <= delta^2 is
// evaluated exactly as written, without fused multiply-add.
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

using namespace pdmi;

namespace {

constexpr int kDefaultLanes = 1;
// spare slot rows after the last slice: the sliced kernel prefetches kRowUnroll rows
// ahead, the staged kernel reads a full piece of stiffness rows
constexpr size_t kSpareRows = kRowUnroll > kPieceRows ? kRowUnroll : kPieceRows;
constexpr int64_t kMaxGap = 12;  // staged ranges absorb gaps of up to this many unused records
constexpr int64_t kGraphChunk = 64;  // steps per captured graph (even: buffer parity repeats)

struct PdError : std::exception {
    int code;
    std::string msg;
    PdError(int c, std::string m) : code(c), msg(std::move(m)) {}
};

[[noreturn]] void fail(int code, const std::string& msg) { throw PdError(code, msg); }

void hip_check(hipError_t e, const char* what)
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

}  // namespace

struct pd_ctx {
    int device = 0;
    int precision = PD_FP64;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    std::vector<Inst> inst;
    int order = PD_ORDER_NATURAL;
    bool order_auto = false;         // the autotuner may change the device node order
    int lanes = kDefaultLanes;       // sliced: lanes per node; staged: wavefronts per slice
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

namespace {

std::string g_create_error;

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

void set_device(pd_ctx* ctx) { hip_check(hipSetDevice(ctx->device), "hipSetDevice"); }

// The step kernels with the bond-model branch: no-failure zones or damage laws present.
bool ext_kernels(const pd_ctx* ctx) { return ctx->has_nofail || ctx->has_laws; }

void require_built(const pd_ctx* ctx)
{
    if (!ctx->built) fail(PD_ESTATE, "no problem: call pd_build_family first");
}

Inst& instance(pd_ctx* ctx, int32_t inst)
{
    require_built(ctx);
    if (inst < 0 || inst >= static_cast<int32_t>(ctx->inst.size()))
        fail(PD_EINVAL, "instance index out of range");
    return ctx->inst[inst];
}

unsigned n_threads()
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

// ------------------------------------------------------------------ family search

// Family of every node (Eq. family, self excluded): bin nodes into cubic cells slightly
// wider than delta, test the 27 surrounding cells, sort each row ascending.
void family_search(int64_t n, const double* x, double delta, std::vector<int64_t>& row_ptr,
                   std::vector<int32_t>& col)
{
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = x[d];
    for (int64_t i = 1; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], x[3 * i + d]);
            hi[d] = std::max(hi[d], x[3 * i + d]);
        }
    const double h = delta * (1.0 + 1e-9);
    int64_t dim[3];
    for (int d = 0; d < 3; ++d) {
        const double span = (hi[d] - lo[d]) / h;
        if (!(span < 4.0e6)) fail(PD_ERANGE, "domain spans too many horizon cells");
        dim[d] = static_cast<int64_t>(std::floor(span)) + 1;
    }
    const int64_t ncell = dim[0] * dim[1] * dim[2];
    if (ncell > (int64_t(1) << 31)) fail(PD_ERANGE, "too many cells for the family search");
    auto cell_of = [&](int64_t i, int64_t* c3) {
        for (int d = 0; d < 3; ++d) {
            int64_t c = static_cast<int64_t>(std::floor((x[3 * i + d] - lo[d]) / h));
            c3[d] = std::min(std::max<int64_t>(c, 0), dim[d] - 1);
        }
    };
    std::vector<int64_t> cstart(ncell + 1, 0), items(n);
    std::vector<int64_t> cid(n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t c3[3];
        cell_of(i, c3);
        cid[i] = (c3[2] * dim[1] + c3[1]) * dim[0] + c3[0];
        ++cstart[cid[i] + 1];
    }
    for (int64_t c = 0; c < ncell; ++c) cstart[c + 1] += cstart[c];
    {
        std::vector<int64_t> fill(cstart.begin(), cstart.end() - 1);
        for (int64_t i = 0; i < n; ++i) items[fill[cid[i]]++] = i;
    }
    const double d2max = delta * delta;
    std::vector<int64_t> count(n, 0);
    std::atomic<bool> coincident{false};  // a zero-length bond has no stretch
    // pass 1: counts; pass 2: fill and sort
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            row_ptr.assign(n + 1, 0);
            for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + count[i];
            if (row_ptr[n] > std::numeric_limits<int32_t>::max())
                fail(PD_ERANGE, "family has 2^31 or more slots");
            col.assign(static_cast<size_t>(row_ptr[n]), 0);
        }
        parallel_for(n, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                int64_t c3[3];
                cell_of(i, c3);
                int64_t w = pass ? row_ptr[i] : 0;
                for (int64_t z = std::max<int64_t>(c3[2] - 1, 0); z <= std::min(c3[2] + 1, dim[2] - 1); ++z)
                    for (int64_t y = std::max<int64_t>(c3[1] - 1, 0); y <= std::min(c3[1] + 1, dim[1] - 1); ++y)
                        for (int64_t xx = std::max<int64_t>(c3[0] - 1, 0); xx <= std::min(c3[0] + 1, dim[0] - 1);
                             ++xx) {
                            const int64_t c = (z * dim[1] + y) * dim[0] + xx;
                            for (int64_t p = cstart[c]; p < cstart[c + 1]; ++p) {
                                const int64_t j = items[p];
                                if (j == i) continue;
                                const double a = x[3 * j + 0] - x[3 * i + 0];
                                const double b = x[3 * j + 1] - x[3 * i + 1];
                                const double e = x[3 * j + 2] - x[3 * i + 2];
                                double d2 = a * a + b * b;
                                d2 = d2 + e * e;
                                if (!(d2 <= d2max)) continue;
                                if (d2 == 0.0) coincident = true;
                                if (pass) col[w] = static_cast<int32_t>(j);
                                ++w;
                            }
                        }
                if (pass)
                    std::sort(col.begin() + row_ptr[i], col.begin() + w);
                else
                    count[i] = w;
            }
        });
        if (coincident) fail(PD_EINVAL, "two nodes share a position (a zero-length bond has no stretch)");
    }
}

// ------------------------------------------------------------------ device layout

// Spacing estimate: the smallest bond length among the first rows.
double spacing_estimate(const Inst& I)
{
    double best = std::numeric_limits<double>::infinity();
    const int64_t rows = std::min<int64_t>(I.n, 4096);
    for (int64_t i = 0; i < rows; ++i)
        for (int64_t b = I.row_ptr[i]; b < I.row_ptr[i + 1]; ++b) {
            const int64_t j = I.col[b];
            double s = 0.0;
            for (int d = 0; d < 3; ++d) {
                const double t = I.x[3 * j + d] - I.x[3 * i + d];
                s += t * t;
            }
            best = std::min(best, std::sqrt(s));
        }
    if (!(best > 0.0) || !std::isfinite(best)) best = I.horizon > 0 ? I.horizon : 1.0;
    return best;
}

uint64_t spread3(uint64_t v)
{
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

// Device-local node order of one instance.
void node_order(Inst& I, int order, double h)
{
    I.iperm.assign(I.n, 0);
    std::vector<int64_t> p(I.n);
    std::iota(p.begin(), p.end(), 0);
    if (order == PD_ORDER_MORTON && I.n > 1) {
        double lo[3];
        for (int d = 0; d < 3; ++d) lo[d] = I.x[d];
        for (int64_t i = 1; i < I.n; ++i)
            for (int d = 0; d < 3; ++d) lo[d] = std::min(lo[d], I.x[3 * i + d]);
        std::vector<uint64_t> key(I.n);
        for (int64_t i = 0; i < I.n; ++i) {
            uint64_t k = 0;
            for (int d = 0; d < 3; ++d) {
                double q = std::floor((I.x[3 * i + d] - lo[d]) / h + 0.5);
                q = std::min(std::max(q, 0.0), 2097151.0);
                k |= spread3(static_cast<uint64_t>(q)) << d;
            }
            key[i] = k;
        }
        std::stable_sort(p.begin(), p.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
    }
    for (int64_t i = 0; i < I.n; ++i) I.iperm[p[i]] = i;
    I.perm = std::move(p);
}

// Order of each row's slots on the device: by the bond offset rounded to the lattice
// spacing (z, then y, then x), so lanes of neighbouring nodes visit neighbours at the
// same relative position together.  On a natural-order lattice this is ascending j.
std::vector<int32_t> slot_ranks(const Inst& I, double h)
{
    std::vector<int32_t> order(static_cast<size_t>(I.nnz));
    parallel_for(I.n, [&](int64_t i0, int64_t i1) {
        std::vector<std::pair<int64_t, int32_t>> tmp;
        for (int64_t i = i0; i < i1; ++i) {
            const int64_t b0 = I.row_ptr[i], b1 = I.row_ptr[i + 1];
            tmp.clear();
            for (int64_t b = b0; b < b1; ++b) {
                const int64_t j = I.col[b];
                int64_t q[3];
                for (int d = 0; d < 3; ++d)
                    q[d] = static_cast<int64_t>(std::llround((I.x[3 * j + d] - I.x[3 * i + d]) / h));
                const int64_t key = ((q[2] + 4096) * 8192 + (q[1] + 4096)) * 8192 + (q[0] + 4096);
                tmp.emplace_back(key, static_cast<int32_t>(b - b0));
            }
            std::sort(tmp.begin(), tmp.end());
            for (int64_t r = 0; r < b1 - b0; ++r) order[b0 + r] = tmp[r].second;
        }
    });
    return order;
}

InstParams make_params(const Inst& I, int32_t law_off)
{
    InstParams p{};
    p.c = I.c;
    const double qt = I.s0 * (2.0 + I.s0);  // (1 + s0)^2 - 1
    p.q0 = qt - decision_margin(qt);
    p.s0 = I.s0;
    p.nlaw = static_cast<int32_t>(I.laws.size());
    p.law_off = law_off;
    if (!I.laws.empty()) {
        // the kernels' threshold for the bond-model branch: just below every law's
        // elastic limit (the branch itself decides in stretch)
        double qmin = std::numeric_limits<double>::infinity();
        for (const LawRec& L : I.laws) qmin = std::min(qmin, L.s[0] * (2.0 + L.s[0]));
        p.q0 = qmin - decision_margin(qmin);
    }
    p.rho = I.rho;
    p.eta = I.eta;
    p.volume = I.volume;
    p.bmag = I.bmag;
    p.has_body = I.bhat.empty() ? 0 : 1;
    if (I.osb) {
        p.osb_a = 3.0 * I.osb_K - 5.0 * I.osb_G;
        p.osb_b = 15.0 * I.osb_G;
    }
    if (I.has_corr) {
        p.cr_flags = (I.corr.micromodulus == PD_MICRO_CONICAL ? 1 : 0) | (I.corr.partial_volumes ? 2 : 0) |
                     (I.corr.surface ? 4 : 0);
        if (I.corr.delta > 0.0) p.cr_idelta = 1.0 / I.corr.delta;
        if (I.corr.dx > 0.0) {
            p.cr_idx = 1.0 / I.corr.dx;
            p.cr_pvhi = (I.corr.delta + 0.5 * I.corr.dx) / I.corr.dx;
        }
        p.cr_2v0 = 2.0 * I.corr_v0;
    }
    return p;
}

// Setup-path copy from pageable host memory; returns once the source may be freed.
void upload(const DevBuf& b, const void* src, size_t bytes, size_t offset_bytes, hipStream_t s)
{
    if (bytes == 0) return;
    if (offset_bytes + bytes > b.bytes) fail(PD_EINVAL, "internal: upload beyond buffer");
    hip_check(hipMemcpyAsync(static_cast<char*>(b.p) + offset_bytes, src, bytes, hipMemcpyHostToDevice, s),
              "hipMemcpyAsync H2D");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

void download(void* dst, const DevBuf& b, size_t bytes, size_t offset_bytes, hipStream_t s)
{
    if (bytes == 0) return;
    if (offset_bytes + bytes > b.bytes) fail(PD_EINVAL, "internal: download beyond buffer");
    hip_check(hipMemcpyAsync(dst, static_cast<const char*>(b.p) + offset_bytes, bytes, hipMemcpyDeviceToHost, s),
              "hipMemcpyAsync D2H");
}

void sync(pd_ctx* ctx) { hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize"); }

bool fp32(const pd_ctx* ctx) { return ctx->precision == PD_FP32; }

// Bytes of one node-record buffer: nn records, the sentinel and kRecPad spare records.
size_t rec_bytes(int64_t nn) { return static_cast<size_t>(nn + 1 + kRecPad) * 48; }

// (Re)build the whole device problem for the current lanes-per-node, keeping the state
// given in user order (nullptr = zero / intact).
struct HostState {
    std::vector<std::vector<double>> u, v, a;   // per instance, n*3
    std::vector<std::vector<uint8_t>> broken;   // per instance, nnz
    std::vector<std::vector<double>> smax;      // per instance, nnz (empty without damage laws)
};

void upload_params(pd_ctx* ctx)
{
    ctx->tape_valid = false;
    std::vector<InstParams> p;
    int32_t law_off = 0;
    for (auto& I : ctx->inst) {
        p.push_back(make_params(I, law_off));
        law_off += static_cast<int32_t>(I.laws.size());
    }
    upload(ctx->params, p.data(), p.size() * sizeof(InstParams), 0, ctx->stream);
}

void upload_bcs(pd_ctx* ctx)
{
    ctx->tape_valid = false;
    std::vector<int32_t> id(static_cast<size_t>(ctx->nn), kNodePad);
    std::vector<BCRec> recs;
    for (auto& I : ctx->inst) {
        for (int64_t l = 0; l < I.n_pad; ++l) {
            const int64_t u = I.perm[l];
            if (u < 0) continue;
            int32_t code = 0;
            BCRec r{};
            for (int d = 0; d < 3; ++d) {
                const int kind = I.bc_kind[3 * u + d];
                if (!kind) continue;
                code |= kind << (2 * d);
                code |= (I.bc_sched[3 * u + d] & 3) << (8 + 2 * d);
                r.A[d] = I.bc_val[3 * u + d];
            }
            if (code == 0) {
                id[I.node_off + l] = kNodeFree;
            } else {
                r.code = code;
                r.T = I.ramp_T;
                r.iT = 1.0 / I.ramp_T;
                id[I.node_off + l] = static_cast<int32_t>(recs.size());
                recs.push_back(r);
            }
        }
    }
    upload(ctx->bc_id, id.data(), id.size() * sizeof(int32_t), 0, ctx->stream);
    ctx->bc.alloc(std::max<size_t>(recs.size(), 1) * sizeof(BCRec));
    upload(ctx->bc, recs.data(), recs.size() * sizeof(BCRec), 0, ctx->stream);
    sync(ctx);
}

// Per-slot stiffness of every instance (instances without a field get their c), or only
// of instance `only` when the array already exists.
// Correction factors of one instance applied to a slot stiffness k (user CSR order b of
// row i): micromodulus profile, partial volume, surface correction, in that order.
struct CorrectionTable {
    std::vector<double> famvol;  // per node (surface correction)
    double v0 = 0.0;
};

double partial_volume(const pd_corrections& c, double L)
{
    const double h = 0.5 * c.dx;
    if (L <= c.delta - h) return 1.0;
    if (L >= c.delta + h) return 0.0;
    return (c.delta + h - L) / c.dx;
}

double ref_length(const Inst& I, int64_t i, int64_t j)
{
    const double a = I.x[3 * j] - I.x[3 * i], b = I.x[3 * j + 1] - I.x[3 * i + 1], c = I.x[3 * j + 2] - I.x[3 * i + 2];
    return std::sqrt((a * a + b * b) + c * c);
}

CorrectionTable correction_table(const Inst& I)
{
    CorrectionTable T;
    if (!I.has_corr || !I.corr.surface) return T;
    T.famvol.assign(static_cast<size_t>(I.n), 0.0);
    parallel_for(I.n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            double v = 0.0;
            for (int64_t b = I.row_ptr[i]; b < I.row_ptr[i + 1]; ++b) {
                const int64_t j = I.col[b];
                const double vj = I.vols.empty() ? I.volume : I.vols[j];
                v += (I.corr.partial_volumes ? partial_volume(I.corr, ref_length(I, i, j)) : 1.0) * vj;
            }
            T.famvol[i] = v;
        }
    });
    for (double v : T.famvol) T.v0 = std::max(T.v0, v);
    return T;
}

double corrected(const Inst& I, const CorrectionTable& T, int64_t i, int64_t j, double k)
{
    const double L = ref_length(I, i, j);
    if (I.corr.micromodulus == PD_MICRO_CONICAL) {
        const double m = 1.0 - L / I.corr.delta;
        k = k * (m > 0.0 ? m : 0.0);
    }
    if (I.corr.partial_volumes) k = k * partial_volume(I.corr, L);
    if (I.corr.surface) k = k * ((2.0 * T.v0) / (T.famvol[i] + T.famvol[j]));
    return k;
}

// Corrections are formed per slot in the step kernel (no per-slot stiffness stream) when
// the staged kernels run and no instance has a stiffness field or per-node volumes;
// otherwise they are folded into the per-slot stiffness.
bool corrections_in_kernel(const pd_ctx* ctx)
{
    if (ctx->mapping != PD_MAP_STAGED) return false;
    bool any = false;
    for (const Inst& I : ctx->inst) {
        if (!I.kslot.empty() || !I.knode.empty() || !I.vols.empty()) return false;
        any |= I.has_corr;
    }
    return any;
}

// Family volume of every device node for the per-slot corrections (1 for padding, for the
// spare entries the kernels' fixed copy window reaches past the last node, for nodes
// without bonds and for instances without the surface correction: every entry is positive,
// so no slot divides by zero); sets each instance's V0.
void upload_family_volumes(pd_ctx* ctx)
{
    std::vector<double> fv(static_cast<size_t>(ctx->nn) + kCorrPad, 1.0);
    for (auto& I : ctx->inst) {
        const CorrectionTable T = correction_table(I);
        I.corr_v0 = T.v0;
        if (T.famvol.empty()) continue;
        for (int64_t l = 0; l < I.n_pad; ++l) {
            const int64_t u = I.perm[l];
            if (u >= 0 && T.famvol[u] > 0.0) fv[I.node_off + l] = T.famvol[u];
        }
    }
    ctx->cfv.alloc(fv.size() * sizeof(double));
    upload(ctx->cfv, fv.data(), fv.size() * sizeof(double), 0, ctx->stream);
}

void upload_stiffness(pd_ctx* ctx, int32_t only = -1)
{
    ctx->tape_valid = false;
    ctx->corr_k = corrections_in_kernel(ctx);
    if (ctx->corr_k) {
        ctx->has_stiff = false;
        ctx->kslot.release();
        upload_family_volumes(ctx);
        upload_params(ctx);
        return;
    }
    ctx->cfv.release();
    bool any = false;
    for (auto& I : ctx->inst) any |= !I.kslot.empty() || I.has_corr;
    if (!any) {
        ctx->has_stiff = false;
        ctx->kslot.release();
        return;
    }
    const bool fresh = !ctx->has_stiff || !ctx->kslot.p;
    ctx->has_stiff = true;
    if (fresh) {
        ctx->kslot.alloc((static_cast<size_t>(ctx->ns) + kSpareRows * kWave) * sizeof(double));
        hip_check(hipMemsetAsync(ctx->kslot.p, 0, ctx->kslot.bytes, ctx->stream), "hipMemsetAsync");
    }
    for (size_t ii = 0; ii < ctx->inst.size(); ++ii) {
        if (!fresh && only >= 0 && static_cast<int32_t>(ii) != only) continue;
        const Inst& I = ctx->inst[ii];
        std::vector<double> k(static_cast<size_t>(I.n_dslots), 0.0);
        std::vector<double> sq;  // a per-node field in per-slot mode: sqrt(k_i) sqrt(k_j)
        std::vector<int32_t> row;
        if ((I.kslot.empty() && !I.knode.empty()) || I.has_corr) {
            if (!I.knode.empty()) {
                sq.resize(static_cast<size_t>(I.n));
                for (int64_t i = 0; i < I.n; ++i) sq[i] = std::sqrt(I.knode[i]);
            }
            row.resize(static_cast<size_t>(I.nnz));
            for (int64_t i = 0; i < I.n; ++i)
                for (int64_t b = I.row_ptr[i]; b < I.row_ptr[i + 1]; ++b) row[b] = static_cast<int32_t>(i);
        }
        const CorrectionTable T = correction_table(I);
        parallel_for(I.n_dslots, [&](int64_t s0, int64_t s1) {
            for (int64_t s = s0; s < s1; ++s) {
                const int32_t b = I.dslot_user[s];
                if (b < 0) continue;
                double kb = !I.kslot.empty() ? I.kslot[b] : !sq.empty() ? sq[row[b]] * sq[I.col[b]] : I.c;
                if (I.has_corr) kb = corrected(I, T, row[b], I.col[b], kb);
                k[s] = kb;
            }
        });
        upload(ctx->kslot, k.data(), k.size() * sizeof(double), I.dslot_off * sizeof(double), ctx->stream);
        sync(ctx);
    }
}

// Per-node stiffness factors when no instance carries a per-slot field: na = sqrt(k_i)
// (sqrt(c) for instances without a node field), nw = na V; padding and the sentinel 0.
void upload_node_weights(pd_ctx* ctx)
{
    ctx->tape_valid = false;
    bool any = false;
    for (auto& I : ctx->inst) any |= !I.knode.empty();
    ctx->has_knode = any && !ctx->has_stiff;
    if (!ctx->has_knode) {
        ctx->na.release();
        ctx->nw.release();
        return;
    }
    std::vector<double> a(static_cast<size_t>(ctx->nn) + 1, 0.0), w(static_cast<size_t>(ctx->nn) + 1, 0.0);
    for (auto& I : ctx->inst)
        for (int64_t l = 0; l < I.n_pad; ++l) {
            const int64_t p = I.perm[l];
            if (p < 0) continue;
            const double sk = std::sqrt(I.knode.empty() ? I.c : I.knode[p]);
            a[I.node_off + l] = sk;
            w[I.node_off + l] = sk * (I.vols.empty() ? I.volume : I.vols[p]);
        }
    ctx->na.alloc(a.size() * sizeof(double));
    ctx->nw.alloc(w.size() * sizeof(double));
    upload(ctx->na, a.data(), a.size() * sizeof(double), 0, ctx->stream);
    upload(ctx->nw, w.data(), w.size() * sizeof(double), 0, ctx->stream);
}

void upload_volumes(pd_ctx* ctx)
{
    ctx->has_vol = false;
    for (auto& I : ctx->inst) ctx->has_vol |= !I.vols.empty();
    if (!ctx->has_vol) {
        ctx->vol.release();
        return;
    }
    // entry nn: the sentinel record, volume 0; then spare zero entries for the state-based
    // kernels' fixed copy window
    std::vector<double> V(static_cast<size_t>(ctx->nn) + kCorrPad, 0.0);
    for (auto& I : ctx->inst)
        for (int64_t l = 0; l < I.n_pad; ++l) {
            const int64_t u = I.perm[l];
            V[I.node_off + l] = u < 0 ? I.volume : (I.vols.empty() ? I.volume : I.vols[u]);
        }
    ctx->vol.alloc(V.size() * sizeof(double));
    upload(ctx->vol, V.data(), V.size() * sizeof(double), 0, ctx->stream);
    sync(ctx);
}

// State-based model: 1/m_i per device node, m_i = sum over the whole family of |xi|^2 V_j
// (influence function 1, reference configuration); padding 0.  The pair
// buffer {theta/m, 1/m} starts zeroed, with kOsbPad spare pairs.
void upload_osb(pd_ctx* ctx)
{
    ctx->has_osb = false;
    for (auto& I : ctx->inst) ctx->has_osb |= I.osb;
    if (!ctx->has_osb) {
        ctx->osb.release();
        ctx->minv.release();
        return;
    }
    std::vector<double> b(static_cast<size_t>(ctx->nn) + 1, 0.0);
    for (auto& I : ctx->inst) {
        if (!I.osb) continue;
        std::vector<double> m(static_cast<size_t>(I.n), 0.0);
        parallel_for(I.n, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                double acc = 0.0;
                for (int64_t q = I.row_ptr[i]; q < I.row_ptr[i + 1]; ++q) {
                    const int64_t j = I.col[q];
                    double L2 = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        const double xi = I.x[3 * j + d] - I.x[3 * i + d];
                        L2 += xi * xi;
                    }
                    acc += L2 * (I.vols.empty() ? I.volume : I.vols[j]);
                }
                m[i] = acc;
            }
        });
        for (int64_t l = 0; l < I.n_pad; ++l) {
            const int64_t u = I.perm[l];
            if (u >= 0 && m[u] > 0.0) b[I.node_off + l] = 1.0 / m[u];
        }
    }
    ctx->minv.alloc(b.size() * sizeof(double));
    upload(ctx->minv, b.data(), b.size() * sizeof(double), 0, ctx->stream);
    ctx->osb.alloc(static_cast<size_t>(ctx->nn + kOsbPad) * 2 * sizeof(double));
    hip_check(hipMemsetAsync(ctx->osb.p, 0, ctx->osb.bytes, ctx->stream), "hipMemsetAsync");
    sync(ctx);
}

// What the state-based kernels support: every instance on the model, the staged layout, the constant micromodulus replaced by (K, G): no stiffness
// fields, damage laws or corrections.
void osb_checks(const pd_ctx* ctx)
{
    if (!ctx->has_osb) return;
    for (const Inst& I : ctx->inst) {
        if (!I.osb) fail(PD_EINVAL, "state-based and bond-based instances cannot share a context");
        if (!I.laws.empty()) fail(PD_EINVAL, "the state-based model takes the brittle critical stretch only (no damage laws)");
        if (I.has_corr) fail(PD_EINVAL, "the state-based model takes no stiffness corrections");
    }
    if (ctx->mapping != PD_MAP_STAGED) fail(PD_EINVAL, "the state-based model runs in the staged mapping");
    if (ctx->has_stiff || ctx->has_knode) fail(PD_EINVAL, "the state-based model takes no stiffness field");
}

void upload_body(pd_ctx* ctx)
{
    ctx->tape_valid = false;
    ctx->has_body = false;
    for (auto& I : ctx->inst) ctx->has_body |= !I.bhat.empty();
    if (!ctx->has_body) {
        ctx->bhat.release();
        return;
    }
    const int64_t nn = ctx->nn;
    std::vector<double> B(static_cast<size_t>(3 * nn), 0.0);
    for (auto& I : ctx->inst) {
        if (I.bhat.empty()) continue;
        for (int64_t l = 0; l < I.n_pad; ++l) {
            const int64_t u = I.perm[l];
            if (u < 0) continue;
            for (int d = 0; d < 3; ++d) B[d * nn + I.node_off + l] = I.bhat[3 * u + d];
        }
    }
    ctx->bhat.alloc(B.size() * sizeof(double));
    upload(ctx->bhat, B.data(), B.size() * sizeof(double), 0, ctx->stream);
    sync(ctx);
}

// Write one instance's state (user order) into the device buffers.
void upload_state(pd_ctx* ctx, const Inst& I, const double* u, const double* v, const double* a)
{
    ctx->tape_valid = false;
    const int64_t nn = ctx->nn;
    auto soa = [&](const double* src, int d) {
        std::vector<double> h(static_cast<size_t>(I.n_pad), 0.0);
        for (int64_t l = 0; l < I.n_pad; ++l)
            if (I.perm[l] >= 0) h[l] = src[3 * I.perm[l] + d];
        return h;
    };
    if (u) {
        std::vector<double> rec(static_cast<size_t>(6 * I.n_pad), 0.0);
        for (int64_t l = 0; l < I.n_pad; ++l) {
            const int64_t p = I.perm[l];
            if (p < 0) continue;
            for (int d = 0; d < 3; ++d) rec[6 * l + d] = I.x[3 * p + d];
            if (!fp32(ctx)) {
                for (int d = 0; d < 3; ++d) rec[6 * l + 3 + d] = u[3 * p + d];
            } else {
                float f[3] = {float(u[3 * p]), float(u[3 * p + 1]), float(u[3 * p + 2])};
                std::memcpy(&rec[6 * l + 3], f, sizeof f);
            }
        }
        for (int b = 0; b < 2; ++b)
            upload(ctx->rec[b], rec.data(), rec.size() * sizeof(double), I.node_off * 48, ctx->stream);
        if (fp32(ctx))
            for (int d = 0; d < 3; ++d) {
                const std::vector<double> h = soa(u, d);
                for (int b = 0; b < 2; ++b)
                    upload(ctx->um[b], h.data(), h.size() * 8, (d * nn + I.node_off) * 8, ctx->stream);
            }
    }
    for (int d = 0; d < 3; ++d) {
        if (v) {
            const std::vector<double> h = soa(v, d);
            upload(ctx->v, h.data(), h.size() * 8, (d * nn + I.node_off) * 8, ctx->stream);
        }
        if (a) {
            const std::vector<double> h = soa(a, d);
            upload(ctx->a, h.data(), h.size() * 8, (d * nn + I.node_off) * 8, ctx->stream);
        }
    }
}

// Slot of the reverse bond (j, i) of every user slot (i, j); rows are sorted.
const std::vector<int64_t>& reverse_slots(Inst& I)
{
    if (static_cast<int64_t>(I.rev_slot.size()) == I.nnz) return I.rev_slot;
    I.rev_slot.assign(static_cast<size_t>(I.nnz), -1);
    parallel_for(I.n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i)
            for (int64_t b = I.row_ptr[i]; b < I.row_ptr[i + 1]; ++b) {
                const int32_t j = I.col[b];
                const auto first = I.col.begin() + I.row_ptr[j], last = I.col.begin() + I.row_ptr[j + 1];
                const auto it = std::lower_bound(first, last, static_cast<int32_t>(i));
                if (it != last && *it == i) I.rev_slot[b] = it - I.col.begin();
            }
    });
    return I.rev_slot;
}

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

// Break steps of one instance from its current flags: broken -> kBrokeBefore, intact ->
// kNeverBroke (padding counts as broken).
void init_break_steps(pd_ctx* ctx, const Inst& I)
{
    const int64_t off = I.dslot_off;
    hip_check(launch_bstep_init(ctx->bstep.as<int32_t>() + off, ctx->col.p ? ctx->col.as<int32_t>() + off : nullptr,
                                ctx->ent.p ? ctx->ent.as<uint16_t>() + off : nullptr, I.n_dslots, ctx->stream),
              "break-step init launch");
}

// Damage-law table of every instance, the per-slot law index (instances with several
// laws) and a zeroed stretch state; without laws all three are released.
void upload_laws(pd_ctx* ctx)
{
    ctx->tape_valid = false;
    std::vector<LawRec> all;
    bool many = false;
    for (auto& I : ctx->inst) {
        all.insert(all.end(), I.laws.begin(), I.laws.end());
        many |= I.laws.size() > 1;
    }
    ctx->has_laws = !all.empty();
    if (!ctx->has_laws) {
        ctx->laws.release();
        ctx->cls.release();
        ctx->smax.release();
        return;
    }
    ctx->laws.alloc(all.size() * sizeof(LawRec));
    upload(ctx->laws, all.data(), all.size() * sizeof(LawRec), 0, ctx->stream);
    const size_t nslot = static_cast<size_t>(ctx->ns) + kSpareRows * kWave;
    ctx->smax.alloc(nslot * sizeof(double));
    hip_check(hipMemsetAsync(ctx->smax.p, 0, ctx->smax.bytes, ctx->stream), "hipMemsetAsync");
    if (many) {
        std::vector<uint8_t> c(nslot, 0);
        for (auto& I : ctx->inst) {
            if (I.cls.empty()) continue;
            for (int64_t d = 0; d < I.n_dslots; ++d) {
                const int32_t b = I.dslot_user[d];
                if (b >= 0) c[I.dslot_off + d] = I.cls[b];
            }
        }
        ctx->cls.alloc(nslot);
        upload(ctx->cls, c.data(), nslot, 0, ctx->stream);
    } else {
        ctx->cls.release();
    }
    sync(ctx);
}

// One instance's stretch state in user CSR order (zeros without damage laws).
std::vector<double> smax_of(pd_ctx* ctx, const Inst& I)
{
    std::vector<double> out(static_cast<size_t>(I.nnz), 0.0);
    if (!ctx->has_laws) return out;
    std::vector<double> d(static_cast<size_t>(I.n_dslots));
    download(d.data(), ctx->smax, d.size() * sizeof(double), I.dslot_off * sizeof(double), ctx->stream);
    sync(ctx);
    for (int64_t k = 0; k < I.n_dslots; ++k)
        if (I.dslot_user[k] >= 0) out[I.dslot_user[k]] = d[k];
    return out;
}

// Per user slot: the bond touches a no-failure zone (empty without flags).
std::vector<uint8_t> nofail_slots(const Inst& I)
{
    std::vector<uint8_t> nf;
    if (I.nofail.empty()) return nf;
    nf.assign(static_cast<size_t>(I.nnz), 0);
    parallel_for(I.n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i)
            for (int64_t b = I.row_ptr[i]; b < I.row_ptr[i + 1]; ++b) nf[b] = I.nofail[i] || I.nofail[I.col[b]];
    });
    return nf;
}

// Slot words of one instance from its broken flags, no-failure zones and stretch state
// (smax in user CSR order, nullptr: no bond softened; a slot with smax > 0 is marked
// softened).  The recorded break steps restart from the flags unless keep_bsteps.
void upload_col(pd_ctx* ctx, Inst& I, const uint8_t* broken, bool keep_bsteps = false,
                const double* smax = nullptr)
{
    ctx->tape_valid = false;
    I.br_sym = bond_symmetric(I, broken);
    const std::vector<uint8_t> nf = nofail_slots(I);
    const bool any_nf = !nf.empty();
    if (ctx->has_laws) {
        std::vector<double> d(static_cast<size_t>(I.n_dslots), 0.0);
        if (smax)
            for (int64_t k = 0; k < I.n_dslots; ++k)
                if (I.dslot_user[k] >= 0) d[k] = smax[I.dslot_user[k]];
        upload(ctx->smax, d.data(), d.size() * sizeof(double), I.dslot_off * sizeof(double), ctx->stream);
    }
    auto soft = [&](int32_t b) { return ctx->has_laws && smax && smax[b] > 0.0; };
    if (ctx->mapping == PD_MAP_STAGED) {
        std::vector<uint16_t> e(static_cast<size_t>(I.n_dslots));
        parallel_for(I.n_dslots, [&](int64_t s0, int64_t s1) {
            for (int64_t d = s0; d < s1; ++d) {
                const int32_t b = I.dslot_user[d];
                if (b < 0)
                    e[d] = static_cast<uint16_t>(kEntBroken | kEntPad);
                else
                    e[d] = static_cast<uint16_t>((48 * I.ent_idx[d]) | ((broken && broken[b]) ? kEntBroken : 0) |
                                                 ((any_nf && nf[b]) ? kEntNoFail : 0) | (soft(b) ? kEntSoft : 0));
            }
        });
        upload(ctx->ent, e.data(), e.size() * sizeof(uint16_t), I.dslot_off * sizeof(uint16_t), ctx->stream);
        if (!keep_bsteps) init_break_steps(ctx, I);
        sync(ctx);
        return;
    }
    std::vector<int32_t> colv(static_cast<size_t>(I.n_dslots));
    parallel_for(I.nslices, [&](int64_t s0, int64_t s1) {
        for (int64_t s = s0; s < s1; ++s)
            for (int64_t t = 0; t < I.s_T[s]; ++t)
                for (int lane = 0; lane < kWave; ++lane) {
                    const int64_t ds = I.s_start[s] + t * kWave + lane;
                    const int32_t b = I.dslot_user[ds];
                    if (b < 0) {
                        colv[ds] = ~static_cast<int32_t>(ctx->nn);  // padding: the sentinel record
                    } else {
                        const int32_t j = static_cast<int32_t>(I.node_off + I.iperm[I.col[b]]) |
                                          ((any_nf && nf[b]) ? kColNoFail : 0) | (soft(b) ? kColSoft : 0);
                        colv[ds] = (broken && broken[b]) ? ~j : j;
                    }
                }
    });
    upload(ctx->col, colv.data(), colv.size() * sizeof(int32_t), I.dslot_off * sizeof(int32_t), ctx->stream);
    if (!keep_bsteps) init_break_steps(ctx, I);
    sync(ctx);
}

// Download one instance's broken mask (user CSR order).
std::vector<uint8_t> broken_of(pd_ctx* ctx, const Inst& I)
{
    if (ctx->mapping == PD_MAP_STAGED) {
        std::vector<uint16_t> e(static_cast<size_t>(I.n_dslots));
        download(e.data(), ctx->ent, e.size() * sizeof(uint16_t), I.dslot_off * sizeof(uint16_t), ctx->stream);
        sync(ctx);
        std::vector<uint8_t> out(static_cast<size_t>(I.nnz), 0);
        for (int64_t d = 0; d < I.n_dslots; ++d) {
            const int32_t b = I.dslot_user[d];
            if (b >= 0 && (e[d] & kEntBroken)) out[b] = 1;
        }
        return out;
    }
    std::vector<int32_t> colv(static_cast<size_t>(I.n_dslots));
    download(colv.data(), ctx->col, colv.size() * sizeof(int32_t), I.dslot_off * sizeof(int32_t), ctx->stream);
    sync(ctx);
    std::vector<uint8_t> out(static_cast<size_t>(I.nnz), 0);
    for (int64_t s = 0; s < I.n_dslots; ++s) {
        const int32_t b = I.dslot_user[s];
        if (b >= 0 && colv[s] < 0) out[b] = 1;
    }
    return out;
}

std::vector<double> soa_of(pd_ctx* ctx, const Inst& I, const DevBuf& buf)
{
    const int64_t nn = ctx->nn;
    std::vector<double> out(static_cast<size_t>(3 * I.n), 0.0);
    std::vector<double> h(static_cast<size_t>(I.n_pad));
    for (int d = 0; d < 3; ++d) {
        download(h.data(), buf, h.size() * 8, (d * nn + I.node_off) * 8, ctx->stream);
        sync(ctx);
        for (int64_t l = 0; l < I.n_pad; ++l)
            if (I.perm[l] >= 0) out[3 * I.perm[l] + d] = h[l];
    }
    return out;
}

std::vector<double> u_of(pd_ctx* ctx, const Inst& I)
{
    if (fp32(ctx)) return soa_of(ctx, I, ctx->um[ctx->cur]);  // the f64 master displacement
    std::vector<double> rec(static_cast<size_t>(6 * I.n_pad));
    download(rec.data(), ctx->rec[ctx->cur], rec.size() * 8, I.node_off * 48, ctx->stream);
    sync(ctx);
    std::vector<double> out(static_cast<size_t>(3 * I.n), 0.0);
    for (int64_t l = 0; l < I.n_pad; ++l) {
        const int64_t p = I.perm[l];
        if (p < 0) continue;
        for (int d = 0; d < 3; ++d) out[3 * p + d] = rec[6 * l + 3 + d];
    }
    return out;
}

HostState snapshot(pd_ctx* ctx)
{
    HostState S;
    for (auto& I : ctx->inst) {
        S.u.push_back(u_of(ctx, I));
        S.v.push_back(soa_of(ctx, I, ctx->v));
        S.a.push_back(soa_of(ctx, I, ctx->a));
        S.broken.push_back(broken_of(ctx, I));
        S.smax.push_back(ctx->has_laws ? smax_of(ctx, I) : std::vector<double>());
    }
    return S;
}

// Staged layout of one instance (one lane per node, 64 nodes per slice): per slice, the
// sorted union of neighbour device indices is cut into ranges of consecutive nodes
// (at most kSegMax long); each lane's slots in a range, in ascending neighbour order,
// fill rows of pieces of at most kPieceRows rows.  Fills start (first slot of each slice),
// pieces, slice_piece, dslot_user and ent_idx; returns the slot count.
int64_t build_staged(Inst& I, std::vector<int64_t>& start)
{
    const int64_t nsl = I.nslices;
    std::vector<std::vector<int2>> spieces(static_cast<size_t>(nsl));
    std::vector<std::vector<int32_t>> suser(static_cast<size_t>(nsl));
    std::vector<std::vector<uint8_t>> sidx(static_cast<size_t>(nsl));
    parallel_for(nsl, [&](int64_t s0, int64_t s1) {
        std::vector<std::array<int64_t, 3>> sl;  // (device neighbour, lane, user slot)
        std::vector<std::vector<std::pair<int32_t, uint8_t>>> per_lane(kWave);
        for (int64_t s = s0; s < s1; ++s) {
            sl.clear();
            for (int w = 0; w < kWave; ++w) {
                const int64_t p = I.perm[s * kWave + w];
                if (p < 0) continue;
                for (int64_t b = I.row_ptr[p]; b < I.row_ptr[p + 1]; ++b)
                    sl.push_back({I.node_off + I.iperm[I.col[b]], w, b});
            }
            std::sort(sl.begin(), sl.end());
            auto& pcs = spieces[s];
            auto& us = suser[s];
            auto& ix = sidx[s];
            size_t k = 0;
            while (k < sl.size()) {
                // one range: consecutive device nodes starting at sl[k][0]
                const int64_t r0 = sl[k][0];
                size_t e = k;
                // small gaps are loaded along (cheaper than another piece)
                while (e < sl.size() && sl[e][0] - r0 < kSegMax && sl[e][0] - sl[e == k ? k : e - 1][0] <= kMaxGap)
                    ++e;
                const int64_t len = sl[e - 1][0] - r0 + 1;
                for (auto& v : per_lane) v.clear();
                for (size_t q = k; q < e; ++q)
                    per_lane[sl[q][1]].push_back({static_cast<int32_t>(sl[q][2]), static_cast<uint8_t>(sl[q][0] - r0)});
                size_t T = 0;
                for (auto& v : per_lane) T = std::max(T, v.size());
                for (size_t t0 = 0; t0 < T; t0 += kPieceRows) {
                    const int rows = static_cast<int>(std::min<size_t>(kPieceRows, T - t0));
                    pcs.push_back(int2{static_cast<int>(r0), static_cast<int>(len | (rows << 8))});
                    for (int t = 0; t < rows; ++t)
                        for (int w = 0; w < kWave; ++w) {
                            const auto& v = per_lane[w];
                            if (t0 + t < v.size()) {
                                us.push_back(v[t0 + t].first);
                                ix.push_back(v[t0 + t].second);
                            } else {
                                us.push_back(-1);
                                ix.push_back(static_cast<uint8_t>(kSegMax));
                            }
                        }
                }
                k = e;
            }
        }
    });
    I.pieces.clear();
    I.slice_piece.assign(static_cast<size_t>(nsl) + 1, 0);
    start.assign(static_cast<size_t>(nsl), 0);
    int64_t nds = 0;
    for (int64_t s = 0; s < nsl; ++s) {
        I.slice_piece[s] = static_cast<int32_t>(I.pieces.size());
        start[s] = nds;
        I.pieces.insert(I.pieces.end(), spieces[s].begin(), spieces[s].end());
        nds += static_cast<int64_t>(suser[s].size());
    }
    I.slice_piece[nsl] = static_cast<int32_t>(I.pieces.size());
    I.dslot_user.resize(static_cast<size_t>(nds));
    I.ent_idx.resize(static_cast<size_t>(nds));
    parallel_for(nsl, [&](int64_t s0, int64_t s1) {
        for (int64_t s = s0; s < s1; ++s) {
            std::copy(suser[s].begin(), suser[s].end(), I.dslot_user.begin() + start[s]);
            std::copy(sidx[s].begin(), sidx[s].end(), I.ent_idx.begin() + start[s]);
        }
    });
    return nds;
}

// Allocate and fill the device problem for ctx->lanes from the instances' user data.
void build_layout(pd_ctx* ctx, const HostState* S)
{
    const int G = ctx->mapping == PD_MAP_STAGED ? 1 : ctx->lanes, W = kWave / G;
    ctx->drop_graphs();
    ctx->tape_valid = false;
    ctx->ck.release();
    ctx->kslot.release();  // slot layout changes: re-uploaded in full below
    int64_t nn = 0, nsl = 0, ns = 0;
    std::vector<int64_t> sp;
    std::vector<int32_t> sT, sI, spc;
    std::vector<int2> pcs;
    for (size_t ii = 0; ii < ctx->inst.size(); ++ii) {
        Inst& I = ctx->inst[ii];
        const double h = spacing_estimate(I);
        node_order(I, ctx->order, h);
        I.n_pad = (I.n + W - 1) / W * W;
        I.perm.resize(static_cast<size_t>(I.n_pad), -1);
        I.node_off = nn;
        I.nslices = I.n_pad / W;
        I.slice_off = nsl;
        I.dslot_off = ns;
        std::vector<int64_t> T(static_cast<size_t>(I.nslices), 0);
        std::vector<int64_t> start(static_cast<size_t>(I.nslices));
        int64_t nds = 0;
        if (ctx->mapping == PD_MAP_STAGED) {
            nds = build_staged(I, start);
            for (int64_t s = 0; s < I.nslices; ++s) spc.push_back(static_cast<int32_t>(pcs.size()) + I.slice_piece[s]);
            pcs.insert(pcs.end(), I.pieces.begin(), I.pieces.end());
        } else {
            const std::vector<int32_t> ranks = slot_ranks(I, h);
            // slice row counts
            for (int64_t s = 0; s < I.nslices; ++s)
                for (int w = 0; w < W; ++w) {
                    const int64_t p = I.perm[s * W + w];
                    if (p >= 0) T[s] = std::max<int64_t>(T[s], (I.row_ptr[p + 1] - I.row_ptr[p] + G - 1) / G);
                }
            for (auto& t : T) t = (t + kRowUnroll - 1) / kRowUnroll * kRowUnroll;
            for (int64_t s = 0; s < I.nslices; ++s) {
                start[s] = nds;
                nds += T[s] * kWave;
            }
            I.dslot_user.assign(static_cast<size_t>(nds), -1);
            parallel_for(I.nslices, [&](int64_t s0, int64_t s1) {
                for (int64_t s = s0; s < s1; ++s)
                    for (int w = 0; w < W; ++w) {
                        const int64_t p = I.perm[s * W + w];
                        if (p < 0) continue;
                        const int64_t b0 = I.row_ptr[p], len = I.row_ptr[p + 1] - b0;
                        for (int64_t r = 0; r < len; ++r) {
                            const int64_t t = r / G, g = r % G;
                            I.dslot_user[start[s] + t * kWave + w * G + g] = static_cast<int32_t>(b0 + ranks[b0 + r]);
                        }
                    }
            });
        }
        I.n_dslots = nds;
        I.s_start = start;
        I.s_T = T;
        for (int64_t s = 0; s < I.nslices; ++s) {
            sp.push_back(ns + start[s]);
            if (T[s] > std::numeric_limits<int32_t>::max()) fail(PD_ERANGE, "row too long");
            sT.push_back(static_cast<int32_t>(T[s]));
            sI.push_back(static_cast<int32_t>(ii));
        }
        nn += I.n_pad;
        nsl += I.nslices;
        ns += nds;
    }
    if (nn >= std::numeric_limits<int32_t>::max() || ns >= std::numeric_limits<int32_t>::max())
        fail(PD_ERANGE, "device problem needs 2^31 or more nodes or slots");
    if (nn + 1 >= (int64_t(1) << 24))
        fail(PD_ERANGE, "device problem needs 2^24 or more node records (the gather uses 24-bit indices)");
    ctx->nn = nn;
    ctx->nslices = nsl;
    ctx->ns = ns;
    for (int b = 0; b < 2; ++b) {
        ctx->rec[b].alloc(rec_bytes(nn));
        if (fp32(ctx))
            ctx->um[b].alloc(static_cast<size_t>(3 * nn) * sizeof(double));
        else
            ctx->um[b].release();
    }
    ctx->v.alloc(static_cast<size_t>(3 * nn) * sizeof(double));
    ctx->a.alloc(static_cast<size_t>(3 * nn) * sizeof(double));
    const size_t spare = kSpareRows * kWave;
    ctx->bstep.alloc((static_cast<size_t>(ns) + spare) * sizeof(int32_t));
    if (ctx->mapping == PD_MAP_STAGED) {
        ctx->col.release();
        ctx->ent.alloc((static_cast<size_t>(ns) + spare) * sizeof(uint16_t));
    } else {
        ctx->ent.release();
        ctx->col.alloc((static_cast<size_t>(ns) + spare) * sizeof(int32_t));
    }
    ctx->slice_ptr.alloc(sp.size() * sizeof(int64_t));
    ctx->slice_T.alloc(sT.size() * sizeof(int32_t));
    ctx->slice_inst.alloc(sI.size() * sizeof(int32_t));
    if (ctx->mapping == PD_MAP_STAGED) {
        spc.push_back(static_cast<int32_t>(pcs.size()));
        ctx->pieces.alloc(std::max<size_t>(pcs.size(), 1) * sizeof(int2));
        ctx->slice_piece.alloc(spc.size() * sizeof(int32_t));
    } else {
        ctx->pieces.release();
        ctx->slice_piece.release();
    }
    ctx->params.alloc(ctx->inst.size() * sizeof(InstParams));
    ctx->bc_id.alloc(static_cast<size_t>(nn) * sizeof(int32_t));
    ctx->step_base.alloc(sizeof(int64_t));
    ctx->status.alloc(sizeof(int32_t));
    ctx->phi.alloc(static_cast<size_t>(nn) * sizeof(double));
    hip_check(hipMemsetAsync(ctx->rec[0].p, 0, ctx->rec[0].bytes, ctx->stream), "hipMemsetAsync");
    hip_check(hipMemsetAsync(ctx->rec[1].p, 0, ctx->rec[1].bytes, ctx->stream), "hipMemsetAsync");
    hip_check(hipMemsetAsync(ctx->v.p, 0, ctx->v.bytes, ctx->stream), "hipMemsetAsync");
    for (int b = 0; b < 2; ++b)
        if (ctx->um[b].p) hip_check(hipMemsetAsync(ctx->um[b].p, 0, ctx->um[b].bytes, ctx->stream), "hipMemsetAsync");
    hip_check(hipMemsetAsync(ctx->a.p, 0, ctx->a.bytes, ctx->stream), "hipMemsetAsync");
    hip_check(hipMemsetAsync(ctx->status.p, 0, sizeof(int32_t), ctx->stream), "hipMemsetAsync");
    if (ctx->col.p) hip_check(hipMemsetAsync(ctx->col.p, 0, ctx->col.bytes, ctx->stream), "hipMemsetAsync");
    if (ctx->ent.p) hip_check(hipMemsetAsync(ctx->ent.p, 0, ctx->ent.bytes, ctx->stream), "hipMemsetAsync");
    upload(ctx->slice_ptr, sp.data(), sp.size() * sizeof(int64_t), 0, ctx->stream);
    upload(ctx->slice_T, sT.data(), sT.size() * sizeof(int32_t), 0, ctx->stream);
    upload(ctx->slice_inst, sI.data(), sI.size() * sizeof(int32_t), 0, ctx->stream);
    if (ctx->mapping == PD_MAP_STAGED) {
        upload(ctx->pieces, pcs.data(), pcs.size() * sizeof(int2), 0, ctx->stream);
        upload(ctx->slice_piece, spc.data(), spc.size() * sizeof(int32_t), 0, ctx->stream);
    }
    const int64_t st = ctx->step;
    upload(ctx->step_base, &st, sizeof st, 0, ctx->stream);
    const double sentinel[6] = {1e10, 1e10, 1e10, 0.0, 0.0, 0.0};
    for (int b = 0; b < 2; ++b) upload(ctx->rec[b], sentinel, sizeof sentinel, static_cast<size_t>(nn) * 48, ctx->stream);
    sync(ctx);
    upload_params(ctx);
    upload_bcs(ctx);
    upload_stiffness(ctx);
    upload_volumes(ctx);
    upload_node_weights(ctx);
    upload_body(ctx);
    upload_laws(ctx);
    upload_osb(ctx);
    for (size_t ii = 0; ii < ctx->inst.size(); ++ii) {
        Inst& I = ctx->inst[ii];
        std::vector<double> zeros(static_cast<size_t>(3 * I.n), 0.0);
        upload_state(ctx, I, S ? S->u[ii].data() : zeros.data(), S ? S->v[ii].data() : nullptr,
                     S ? S->a[ii].data() : nullptr);
        const double* sm = (S && !S->smax[ii].empty()) ? S->smax[ii].data() : nullptr;
        upload_col(ctx, I, S ? S->broken[ii].data() : nullptr, false, sm);
    }
    {  // device node of every user node, for readouts into device memory
        std::vector<int64_t> dn;
        for (auto& I : ctx->inst) {
            I.user_off = static_cast<int64_t>(dn.size());
            for (int64_t u = 0; u < I.n; ++u) dn.push_back(I.node_off + I.iperm[u]);
        }
        ctx->unode.alloc(dn.size() * sizeof(int64_t));
        upload(ctx->unode, dn.data(), dn.size() * sizeof(int64_t), 0, ctx->stream);
    }
    ctx->cur = 0;
    ctx->vv_ahead = false;
    ctx->built = true;
}

void validate_coords(int64_t n, const double* coords, double horizon)
{
    if (n < 1) fail(PD_EINVAL, "n must be >= 1");
    if (n >= std::numeric_limits<int32_t>::max()) fail(PD_ERANGE, "n must be < 2^31 - 1");
    if (!coords) fail(PD_EINVAL, "coords is NULL");
    if (!(horizon > 0.0) || !std::isfinite(horizon)) fail(PD_EINVAL, "horizon must be positive and finite");
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!std::isfinite(coords[i])) fail(PD_EINVAL, "coords must be finite");
}

// A caller's family (pd_set_family): CSR with rows strictly ascending, no self bonds,
// every bond present in both directions, no zero-length bond.  Returns the longest bond.
double validate_family(int64_t n, const double* x, const int64_t* row_ptr, const int32_t* col)
{
    if (!row_ptr || row_ptr[0] != 0) fail(PD_EINVAL, "row_ptr must start at 0");
    for (int64_t i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) fail(PD_EINVAL, "row_ptr must be non-decreasing");
    if (row_ptr[n] >= std::numeric_limits<int32_t>::max()) fail(PD_ERANGE, "family has 2^31 or more slots");
    if (row_ptr[n] > 0 && !col) fail(PD_EINVAL, "col is NULL");
    std::atomic<int> bad{0};
    std::vector<double> longest(static_cast<size_t>(n), 0.0);
    parallel_for(n, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i)
            for (int64_t b = row_ptr[i]; b < row_ptr[i + 1]; ++b) {
                const int64_t j = col[b];
                if (j < 0 || j >= n || j == i) { bad = 1; return; }
                if (b > row_ptr[i] && col[b - 1] >= col[b]) { bad = 2; return; }
                if (!std::binary_search(col + row_ptr[j], col + row_ptr[j + 1], static_cast<int32_t>(i))) {
                    bad = 3;
                    return;
                }
                double L2 = 0.0;
                for (int d = 0; d < 3; ++d) L2 += (x[3 * j + d] - x[3 * i + d]) * (x[3 * j + d] - x[3 * i + d]);
                if (!(L2 > 0.0)) { bad = 4; return; }
                longest[i] = std::max(longest[i], std::sqrt(L2));
            }
    });
    switch (bad.load()) {
    case 1: fail(PD_EINVAL, "family: neighbour id out of range or a self bond");
    case 2: fail(PD_EINVAL, "family: rows must be strictly ascending");
    case 3: fail(PD_EINVAL, "family: every bond must appear in both directions");
    case 4: fail(PD_EINVAL, "family: zero-length bond (coincident nodes)");
    default: break;
    }
    double h = 0.0;
    for (double v : longest) h = std::max(h, v);
    return h > 0.0 ? h : 1.0;
}

void new_problem(pd_ctx* ctx, int32_t ninst, const int64_t* n, const double* const* coords, const double* horizon,
                 int order, const int64_t* user_row_ptr = nullptr, const int32_t* user_col = nullptr)
{
    if (order != PD_ORDER_NATURAL && order != PD_ORDER_MORTON && order != PD_ORDER_AUTO)
        fail(PD_EINVAL, "unknown node order");
    if (ninst < 1) fail(PD_EINVAL, "need at least one instance");
    std::vector<Inst> insts(static_cast<size_t>(ninst));
    int64_t total = 0;
    for (int32_t b = 0; b < ninst; ++b) {
        validate_coords(n[b], coords[b], horizon[b]);
        Inst& I = insts[b];
        I.n = n[b];
        I.horizon = horizon[b];
        I.x.assign(coords[b], coords[b] + 3 * n[b]);
        if (user_row_ptr) {  // the caller's family (one instance), validated already
            I.row_ptr.assign(user_row_ptr, user_row_ptr + n[b] + 1);
            I.col.assign(user_col, user_col + user_row_ptr[n[b]]);
        } else {
            family_search(I.n, I.x.data(), I.horizon, I.row_ptr, I.col);
        }
        I.nnz = I.row_ptr[I.n];
        I.bc_kind.assign(static_cast<size_t>(3 * I.n), 0);
        I.bc_sched.assign(static_cast<size_t>(3 * I.n), 0);
        I.bc_val.assign(static_cast<size_t>(3 * I.n), 0.0);
        total += I.nnz;
    }
    (void)total;
    set_device(ctx);
    ctx->built = false;
    ctx->inst = std::move(insts);
    ctx->order = order == PD_ORDER_AUTO ? PD_ORDER_NATURAL : order;
    ctx->order_auto = order == PD_ORDER_AUTO;
    ctx->has_nofail = false;
    ctx->has_laws = false;
    ctx->has_osb = false;
    ctx->step = 0;
    ctx->a_valid = false;
    ctx->vv_ahead = false;
    build_layout(ctx, nullptr);
}

// ------------------------------------------------------------------ stepping

StepArgs step_args(pd_ctx* ctx, int in, int out, int64_t step_local)
{
    StepArgs A{};
    A.rec_in = ctx->rec[in].as<double>();
    A.rec_out = ctx->rec[out].as<double>();
    A.v = ctx->v.as<double>();
    A.a = ctx->a.as<double>();
    A.um_in = ctx->um[in].as<double>();
    A.um_out = ctx->um[out].as<double>();
    A.col = ctx->col.as<int32_t>();
    A.kslot = ctx->has_stiff ? ctx->kslot.as<double>() : nullptr;
    A.vol = ctx->has_vol ? ctx->vol.as<double>() : nullptr;
    A.na = ctx->has_knode ? ctx->na.as<double>() : nullptr;
    A.nw = ctx->has_knode ? ctx->nw.as<double>() : nullptr;
    A.bhat = ctx->has_body ? ctx->bhat.as<double>() : nullptr;
    A.force = ctx->force.p ? ctx->force.as<double>() : nullptr;
    A.laws = ctx->has_laws ? ctx->laws.as<LawRec>() : nullptr;
    A.cls = ctx->cls.p ? ctx->cls.as<uint8_t>() : nullptr;
    A.smax = ctx->has_laws ? ctx->smax.as<double>() : nullptr;
    A.osb = ctx->has_osb ? ctx->osb.as<double2>() : nullptr;
    A.minv = ctx->has_osb ? ctx->minv.as<double>() : nullptr;
    A.cfv = ctx->corr_k ? ctx->cfv.as<double>() : nullptr;
    A.slice_ptr = ctx->slice_ptr.as<int64_t>();
    A.slice_T = ctx->slice_T.as<int32_t>();
    A.slice_inst = ctx->slice_inst.as<int32_t>();
    A.params = ctx->params.as<InstParams>();
    A.bc_id = ctx->bc_id.as<int32_t>();
    A.bc = ctx->bc.as<BCRec>();
    A.pieces = ctx->pieces.as<int2>();
    A.slice_piece = ctx->slice_piece.as<int32_t>();
    A.ent = ctx->ent.as<uint16_t>();
    A.step_base = ctx->step_base.as<int64_t>();
    A.status = ctx->status.as<int32_t>();
    A.bstep = ctx->bstep.as<int32_t>();
    A.nn = ctx->nn;
    A.nslices = ctx->nslices;
    A.step_local = step_local;
    A.dt = ctx->dt;
    return A;
}

int step_mode(int scheme)
{
    return scheme == PD_VELOCITY_VERLET ? kModeVV : scheme == PD_EULER_FORWARD ? kModeFE : kModeEC;
}

void launch_one(pd_ctx* ctx, int mode, int in, int out, int64_t step_local)
{
    const StepArgs A = step_args(ctx, in, out, step_local);
    if (ctx->has_osb)
        hip_check(launch_osb_step(A, mode, fp32(ctx), ctx->lanes, ctx->stream), "state-based step launch");
    else if (ctx->mapping == PD_MAP_STAGED)
        hip_check(launch_step_staged(A, mode, fp32(ctx), ctx->lanes, ext_kernels(ctx), ctx->stream),
                  "step kernel launch");
    else
        hip_check(launch_step(A, ctx->lanes, mode, ctx->has_stiff, ext_kernels(ctx), ctx->stream),
                  "step kernel launch");
}

// Launch `count` consecutive steps starting at buffer parity `cur`, step_local offsets
// 0..count-1 relative to the device step base, then advance the base.
// Bond force density of the current level into ctx->force (SoA, stride nn): the step
// kernel in its force-only mode, reading the record buffer that holds level `step`.
void eval_force(pd_ctx* ctx)
{
    osb_checks(ctx);
    const size_t bytes = static_cast<size_t>(3 * ctx->nn) * sizeof(double);
    if (!ctx->force.p || ctx->force.bytes < bytes) ctx->force.alloc(bytes);
    launch_one(ctx, kModeForce, ctx->cur, 1 - ctx->cur, 0);
}

void launch_steps(pd_ctx* ctx, int mode, int cur, int64_t count)
{
    for (int64_t i = 0; i < count; ++i) {
        const int in = (mode == kModeVV) ? 1 - cur : cur;
        const int out = 1 - in;
        launch_one(ctx, mode, in, out, i);
        cur ^= 1;
    }
    hip_check(launch_advance(ctx->step_base.as<int64_t>(), count, ctx->stream), "advance launch");
}

hipGraphExec_t chunk_graph(pd_ctx* ctx, int mode, int parity)
{
    hipGraphExec_t& g = ctx->graph[parity][mode];
    if (g) return g;
    hipGraph_t graph = nullptr;
    hip_check(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
        launch_steps(ctx, mode, parity, kGraphChunk);
    } catch (...) {
        (void)hipStreamEndCapture(ctx->stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    hip_check(hipStreamEndCapture(ctx->stream, &graph), "hipStreamEndCapture");
    hipError_t e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    hip_check(e, "hipGraphInstantiate");
    return g;
}

void do_steps(pd_ctx* ctx, int64_t nsteps)
{
    osb_checks(ctx);
    const int mode = step_mode(ctx->scheme);
    ctx->tape_valid = false;
    if (!ctx->ev0) {
        hip_check(hipEventCreate(&ctx->ev0), "hipEventCreate");
        hip_check(hipEventCreate(&ctx->ev1), "hipEventCreate");
    }
    hip_check(hipEventRecord(ctx->ev0, ctx->stream), "hipEventRecord");
    if (mode == kModeVV && nsteps > 0) {
        if (!ctx->a_valid) {
            launch_one(ctx, kModeVVInit, ctx->cur, 1 - ctx->cur, 0);
            ctx->a_valid = true;
            ctx->vv_ahead = true;
        } else if (!ctx->vv_ahead) {
            hip_check(launch_drift(step_args(ctx, ctx->cur, 1 - ctx->cur, 0), fp32(ctx), ctx->stream), "drift launch");
            ctx->vv_ahead = true;
        }
    }
    int64_t left = nsteps;
    if (ctx->use_graphs) {
        while (left >= kGraphChunk) {
            hip_check(hipGraphLaunch(chunk_graph(ctx, mode, ctx->cur), ctx->stream), "hipGraphLaunch");
            left -= kGraphChunk;  // even chunk: parity unchanged
        }
    }
    if (left > 0) {
        launch_steps(ctx, mode, ctx->cur, left);
        if (left & 1) ctx->cur ^= 1;
    }
    hip_check(hipEventRecord(ctx->ev1, ctx->stream), "hipEventRecord");
    ctx->timed = true;
    ctx->step += nsteps;
}

void check_status(pd_ctx* ctx)
{
    int32_t st = 0;
    download(&st, ctx->status, sizeof st, 0, ctx->stream);
    sync(ctx);
    if (st & 1) fail(PD_ENONFINITE, "a displacement or velocity became non-finite");
}

void reset_flags_after_state_change(pd_ctx* ctx, bool a_given)
{
    ctx->a_valid = a_given;
    ctx->vv_ahead = false;
    const int32_t z = 0;
    upload(ctx->status, &z, sizeof z, 0, ctx->stream);
    sync(ctx);
}

// ------------------------------------------------------------------ adjoint

void adjoint_checks(pd_ctx* ctx)
{
    require_built(ctx);
    if (fp32(ctx)) fail(PD_EINVAL, "the adjoint runs in the FP64 build only");
    if (ctx->scheme != PD_EULER_CROMER) fail(PD_EINVAL, "the adjoint differentiates the Euler-Cromer scheme only");
    if (ctx->inst.size() != 1) fail(PD_EINVAL, "the adjoint needs a single-instance problem");
    for (const LawRec& L : ctx->inst[0].laws)
        if (L.nb > 1) fail(PD_EINVAL, "the adjoint differentiates brittle damage laws only");
    if (ctx->inst[0].has_corr) fail(PD_EINVAL, "the adjoint does not take stiffness corrections");
    if (ctx->has_osb) fail(PD_EINVAL, "the adjoint differentiates the bond-based model only");
}

// The reverse pass gathers the transposed tangent over each node's own family, which
// needs every bond's two slots to carry the same stiffness and broken flag (bonds that
// break while stepping always break on both slots in the same pass).
void check_symmetric(const Inst& I)
{
    if (!I.k_sym) fail(PD_EINVAL, "the adjoint needs symmetric bond stiffness (slots (i,j) and (j,i) equal)");
    if (!I.br_sym) fail(PD_EINVAL, "the adjoint needs both slots of a bond broken together");
}

void launch_ec(pd_ctx* ctx, const StepArgs& A)
{
    if (ctx->mapping == PD_MAP_STAGED)
        hip_check(launch_step_staged(A, kModeEC, false, ctx->lanes, ext_kernels(ctx), ctx->stream),
                  "step kernel launch");
    else
        hip_check(launch_step(A, ctx->lanes, kModeEC, ctx->has_stiff, ext_kernels(ctx), ctx->stream),
                  "step kernel launch");
}

// Local damage of every device node into ctx->phi (stream-ordered).
void launch_damage_now(pd_ctx* ctx)
{
    DamageArgs D{};
    D.col = ctx->col.as<int32_t>();
    D.sentinel = static_cast<int32_t>(ctx->nn);
    D.vol = ctx->has_vol ? ctx->vol.as<double>() : nullptr;
    D.slice_ptr = ctx->slice_ptr.as<int64_t>();
    D.slice_T = ctx->slice_T.as<int32_t>();
    D.slice_inst = ctx->slice_inst.as<int32_t>();
    D.params = ctx->params.as<InstParams>();
    D.phi = ctx->phi.as<double>();
    D.nslices = ctx->nslices;
    D.pieces = ctx->pieces.as<int2>();
    D.slice_piece = ctx->slice_piece.as<int32_t>();
    D.ent = ctx->ent.as<uint16_t>();
    D.laws = ctx->has_laws ? ctx->laws.as<LawRec>() : nullptr;
    D.cls = ctx->cls.p ? ctx->cls.as<uint8_t>() : nullptr;
    D.smax = ctx->has_laws ? ctx->smax.as<double>() : nullptr;
    if (ctx->mapping == PD_MAP_STAGED)
        hip_check(launch_damage_staged(D, ctx->stream), "damage launch");
    else
        hip_check(launch_damage(D, ctx->lanes, ctx->stream), "damage launch");
}

// A caller's device buffer for a readout: device memory of this context's device.
void require_device_buffer(const pd_ctx* ctx, const void* p)
{
    if (!p) fail(PD_EINVAL, "out is NULL");
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();  // clear the error an unknown pointer leaves
        fail(PD_EINVAL, "out is not device memory");
    }
    if (at.type != hipMemoryTypeDevice || at.device != ctx->device)
        fail(PD_EINVAL, "out is not device memory of the context's device");
}

// Readouts into device memory (user order, stream-ordered on the context's stream):
// what = 0 displacement, 1 velocity, 2 damage.
int get_nodes_dev(pd_ctx* ctx, int32_t inst, double* out, int what)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        require_device_buffer(ctx, out);
        set_device(ctx);
        const int64_t* dn = ctx->unode.as<int64_t>() + I.user_off;
        const int64_t nn = ctx->nn;
        hipError_t e;
        if (what == 0) {
            if (fp32(ctx))  // the f64 master displacement, SoA
                e = launch_export_nodes(ctx->um[ctx->cur].as<double>(), 1, nn, 0, dn, I.n, 3, out, ctx->stream);
            else            // records: x then u, 6 doubles per node
                e = launch_export_nodes(ctx->rec[ctx->cur].as<double>(), 6, 1, 3, dn, I.n, 3, out, ctx->stream);
        } else if (what == 1) {
            e = launch_export_nodes(ctx->v.as<double>(), 1, nn, 0, dn, I.n, 3, out, ctx->stream);
        } else {
            launch_damage_now(ctx);
            e = launch_export_nodes(ctx->phi.as<double>(), 1, 0, 0, dn, I.n, 1, out, ctx->stream);
        }
        hip_check(e, "readout launch");
    });
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

int pd_create(pd_ctx** out, int device, int precision, void* hip_stream)
{
    if (!out) {
        g_create_error = "out is NULL";
        return PD_EINVAL;
    }
    *out = nullptr;
    if (precision != PD_FP64 && precision != PD_FP32) {
        g_create_error = "unknown precision";
        return PD_EINVAL;
    }
    std::unique_ptr<pd_ctx> ctx(new (std::nothrow) pd_ctx);
    if (!ctx) {
        g_create_error = "host allocation failed";
        return PD_ENOMEM;
    }
    int rc = guarded(ctx.get(), [&] {
        int count = 0;
        hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
        if (device < 0 || device >= count) fail(PD_EINVAL, "device index out of range");
        ctx->device = device;
        ctx->precision = precision;
        if (precision == PD_FP32) ctx->mapping = PD_MAP_STAGED;  // FP32 bond arithmetic lives in the staged kernel
        set_device(ctx.get());
        int64_t* scr = nullptr;  // the allocation-free readout's scratch array on this GPU, looked up once
        hip_check(scratch_address(device, &scr), "scratch address");
        if (hip_stream) {
            ctx->stream = static_cast<hipStream_t>(hip_stream);
        } else {
            hip_check(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking), "hipStreamCreate");
            ctx->own_stream = true;
        }
    });
    if (rc != PD_OK) {
        g_create_error = ctx->err;
        return rc;
    }
    *out = ctx.release();
    return PD_OK;
}

int pd_destroy(pd_ctx* ctx)
{
    if (!ctx) return PD_OK;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    delete ctx;
    return PD_OK;
}

const char* pd_last_error(const pd_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

int pd_build_family(pd_ctx* ctx, int64_t n, const double* coords, double horizon, int order)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] { new_problem(ctx, 1, &n, &coords, &horizon, order); });
}

int pd_set_family(pd_ctx* ctx, int64_t n, const double* coords, const int64_t* row_ptr, const int32_t* col,
                  int order)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        validate_coords(n, coords, 1.0);
        const double longest = validate_family(n, coords, row_ptr, col);
        new_problem(ctx, 1, &n, &coords, &longest, order, row_ptr, col);
    });
}

int pd_build_family_batch(pd_ctx* ctx, int32_t ninst, const int64_t* n, const double* const* coords,
                          const double* horizon, int order)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        if (ninst < 1 || !n || !coords || !horizon) fail(PD_EINVAL, "bad batch arguments");
        new_problem(ctx, ninst, n, coords, horizon, order);
    });
}

int pd_num_instances(const pd_ctx* ctx, int32_t* ninst)
{
    if (!ctx || !ninst) return PD_EINVAL;
    *ninst = ctx->built ? static_cast<int32_t>(ctx->inst.size()) : 0;
    return PD_OK;
}

int pd_instance_size(const pd_ctx* ctx, int32_t inst, int64_t* n, int64_t* nnz)
{
    if (!ctx || !ctx->built || inst < 0 || inst >= static_cast<int32_t>(ctx->inst.size())) return PD_EINVAL;
    if (n) *n = ctx->inst[inst].n;
    if (nnz) *nnz = ctx->inst[inst].nnz;
    return PD_OK;
}

int pd_get_family(pd_ctx* ctx, int32_t inst, int64_t* row_ptr, int32_t* col, int64_t* nnz)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (nnz) *nnz = I.nnz;
        if (row_ptr) std::memcpy(row_ptr, I.row_ptr.data(), I.row_ptr.size() * sizeof(int64_t));
        if (col) std::memcpy(col, I.col.data(), I.col.size() * sizeof(int32_t));
    });
}

int pd_set_material(pd_ctx* ctx, int32_t inst, const pd_material* m)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        if (!m) fail(PD_EINVAL, "material is NULL");
        if (!(m->rho > 0.0) || !std::isfinite(m->rho)) fail(PD_EINVAL, "rho must be positive and finite");
        if (!std::isfinite(m->c)) fail(PD_EINVAL, "c must be finite");
        if (!(m->s0 > 0.0)) fail(PD_EINVAL, "s0 must be positive");
        if (!(m->eta >= 0.0) || !std::isfinite(m->eta)) fail(PD_EINVAL, "eta must be >= 0 and finite");
        std::vector<double> vols;
        if (m->volumes) {
            vols.assign(m->volumes, m->volumes + I.n);
            for (double x : vols)
                if (!(x > 0.0) || !std::isfinite(x)) fail(PD_EINVAL, "volumes must be positive and finite");
        } else if (!(m->volume > 0.0) || !std::isfinite(m->volume)) {
            fail(PD_EINVAL, "volume must be positive and finite");
        }
        set_device(ctx);
        I.rho = m->rho;
        I.c = m->c;
        I.s0 = m->s0;
        I.eta = m->eta;
        I.volume = m->volumes ? 1.0 : m->volume;
        I.vols = std::move(vols);
        upload_params(ctx);
        upload_volumes(ctx);
        bool any_corr = false;  // family volumes and the in-kernel choice depend on the volumes
        for (const Inst& J : ctx->inst) any_corr |= J.has_corr;
        if (ctx->has_stiff || any_corr) upload_stiffness(ctx, any_corr ? -1 : inst);
        upload_node_weights(ctx);
        if (I.osb) upload_osb(ctx);  // the weighted volumes scale with the node volume
        ctx->a_valid = false;
        ctx->vv_ahead = false;
        ctx->drop_graphs();
        sync(ctx);
    });
}

int pd_set_bond_stiffness(pd_ctx* ctx, int32_t inst, const double* k)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        std::vector<double> kv;
        if (k) {
            kv.assign(k, k + I.nnz);
            for (double x : kv)
                if (!std::isfinite(x)) fail(PD_EINVAL, "stiffness must be finite");
        }
        set_device(ctx);
        I.k_sym = bond_symmetric(I, kv.empty() ? static_cast<const double*>(nullptr) : kv.data());
        const bool mode_change = kv.empty() != I.kslot.empty() || !I.knode.empty();
        I.kslot = std::move(kv);
        I.knode.clear();
        upload_stiffness(ctx, mode_change ? -1 : inst);
        upload_node_weights(ctx);
        ctx->a_valid = false;
        ctx->vv_ahead = false;
        ctx->drop_graphs();
    });
}

int pd_set_node_stiffness(pd_ctx* ctx, int32_t inst, const double* k_node)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        std::vector<double> kn;
        if (k_node) {
            kn.assign(k_node, k_node + I.n);
            for (double x : kn)
                if (!(x >= 0.0) || !std::isfinite(x)) fail(PD_EINVAL, "node stiffness must be finite and >= 0");
        }
        set_device(ctx);
        I.knode = std::move(kn);
        I.kslot.clear();
        I.k_sym = true;  // sqrt(k_i k_j) is the same on both slots of a bond
        upload_stiffness(ctx);
        upload_node_weights(ctx);
        ctx->a_valid = false;
        ctx->vv_ahead = false;
        ctx->drop_graphs();
    });
}

int pd_break_bonds(pd_ctx* ctx, int32_t inst, const uint8_t* broken)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        if (!broken) fail(PD_EINVAL, "broken is NULL");
        set_device(ctx);
        std::vector<uint8_t> cur = broken_of(ctx, I);
        for (int64_t b = 0; b < I.nnz; ++b) cur[b] = cur[b] || broken[b];
        const std::vector<double> sm = smax_of(ctx, I);
        upload_col(ctx, I, cur.data(), false, sm.data());
        ctx->a_valid = false;
        ctx->vv_ahead = false;
    });
}

int pd_set_bcs(pd_ctx* ctx, int32_t inst, int64_t m, const int64_t* nodes, int comp_mask, int kind,
               const double value[3], int sched)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        if (m < 0 || (m > 0 && !nodes)) fail(PD_EINVAL, "bad node list");
        if (comp_mask < 1 || comp_mask > 7) fail(PD_EINVAL, "comp_mask must be in 1..7");
        if (kind != PD_BC_DISP && kind != PD_BC_VEL) fail(PD_EINVAL, "unknown BC kind");
        if (sched != PD_SCHED_CONST && sched != PD_SCHED_LINEAR && sched != PD_SCHED_RAMP5)
            fail(PD_EINVAL, "unknown schedule");
        if (!value) fail(PD_EINVAL, "value is NULL");
        for (int d = 0; d < 3; ++d)
            if ((comp_mask >> d & 1) && !std::isfinite(value[d])) fail(PD_EINVAL, "BC value must be finite");
        for (int64_t i = 0; i < m; ++i)
            if (nodes[i] < 0 || nodes[i] >= I.n) fail(PD_EINVAL, "BC node id out of range");
        set_device(ctx);
        for (int64_t i = 0; i < m; ++i)
            for (int d = 0; d < 3; ++d)
                if (comp_mask >> d & 1) {
                    I.bc_kind[3 * nodes[i] + d] = static_cast<uint8_t>(kind);
                    I.bc_sched[3 * nodes[i] + d] = static_cast<uint8_t>(sched);
                    I.bc_val[3 * nodes[i] + d] = value[d];
                }
        upload_bcs(ctx);
        ctx->vv_ahead = false;
        ctx->drop_graphs();
    });
}

int pd_clear_bcs(pd_ctx* ctx, int32_t inst)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        set_device(ctx);
        std::fill(I.bc_kind.begin(), I.bc_kind.end(), 0);
        std::fill(I.bc_sched.begin(), I.bc_sched.end(), 0);
        std::fill(I.bc_val.begin(), I.bc_val.end(), 0.0);
        upload_bcs(ctx);
        ctx->vv_ahead = false;
        ctx->drop_graphs();
    });
}

int pd_set_bc_ramp(pd_ctx* ctx, int32_t inst, double ramp_time)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        if (!(ramp_time > 0.0) || !std::isfinite(ramp_time)) fail(PD_EINVAL, "ramp time must be positive and finite");
        set_device(ctx);
        I.ramp_T = ramp_time;
        upload_bcs(ctx);
        ctx->vv_ahead = false;
        ctx->drop_graphs();
    });
}

int pd_set_no_fail(pd_ctx* ctx, int32_t inst, int64_t m, const int64_t* nodes)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        if (m < 0 || (m > 0 && !nodes)) fail(PD_EINVAL, "bad node list");
        for (int64_t i = 0; i < m; ++i)
            if (nodes[i] < 0 || nodes[i] >= I.n) fail(PD_EINVAL, "no-failure node id out of range");
        set_device(ctx);
        const std::vector<uint8_t> br = broken_of(ctx, I);
        const std::vector<double> sm = smax_of(ctx, I);
        I.nofail.clear();
        if (m > 0) {
            I.nofail.assign(static_cast<size_t>(I.n), 0);
            for (int64_t i = 0; i < m; ++i) I.nofail[nodes[i]] = 1;
        }
        ctx->has_nofail = false;
        for (auto& J : ctx->inst) ctx->has_nofail |= !J.nofail.empty();
        upload_col(ctx, I, br.data(), /*keep_bsteps=*/true, sm.data());
        ctx->drop_graphs();
    });
}

// After a change of damage laws or bond classes: new tables, softening state cleared
// (broken flags and recorded break steps kept).
void reset_laws(pd_ctx* ctx)
{
    std::vector<std::vector<uint8_t>> br;
    for (auto& I : ctx->inst) br.push_back(broken_of(ctx, I));
    upload_params(ctx);
    upload_laws(ctx);
    for (size_t ii = 0; ii < ctx->inst.size(); ++ii) upload_col(ctx, ctx->inst[ii], br[ii].data(), true, nullptr);
    ctx->drop_graphs();
}

int pd_set_damage_law(pd_ctx* ctx, int32_t inst, int32_t cls, int32_t nb, const double* s_break, const double* ratio)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        if (cls < 0 || cls >= kLawMaxClasses) fail(PD_EINVAL, "bond class out of range 0..7");
        if (cls > static_cast<int32_t>(I.laws.size())) fail(PD_EINVAL, "bond classes must be defined in order");
        if (nb < 1 || nb > kLawMaxB) fail(PD_EINVAL, "a damage law has 1..8 breakpoints");
        if (!s_break || !ratio) fail(PD_EINVAL, "s_break or ratio is NULL");
        LawRec L{};
        L.nb = nb;
        for (int k = 0; k < nb; ++k) {
            if (!std::isfinite(s_break[k]) || !(s_break[k] > 0.0)) fail(PD_EINVAL, "breakpoints must be positive");
            if (k > 0 && !(s_break[k] > s_break[k - 1])) fail(PD_EINVAL, "breakpoints must increase");
            if (!std::isfinite(ratio[k]) || ratio[k] < 0.0) fail(PD_EINVAL, "force ratios must be >= 0");
            L.s[k] = s_break[k];
            L.r[k] = ratio[k];
        }
        if (nb > 1 && (ratio[0] != 1.0 || ratio[nb - 1] != 0.0))
            fail(PD_EINVAL, "a softening law starts at ratio 1 and ends at ratio 0");
        for (int k = 0; k + 1 < nb; ++k) L.slope[k] = (L.r[k + 1] - L.r[k]) / (L.s[k + 1] - L.s[k]);
        set_device(ctx);
        if (cls == static_cast<int32_t>(I.laws.size()))
            I.laws.push_back(L);
        else
            I.laws[cls] = L;
        reset_laws(ctx);
    });
}

int pd_set_bond_classes(pd_ctx* ctx, int32_t inst, const uint8_t* cls)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        if (cls) {
            if (I.laws.empty()) fail(PD_EINVAL, "define the damage laws first");
            for (int64_t b = 0; b < I.nnz; ++b)
                if (cls[b] >= I.laws.size()) fail(PD_EINVAL, "bond class without a damage law");
            if (!bond_symmetric(I, cls)) fail(PD_EINVAL, "both slots of a bond must be in the same class");
        }
        set_device(ctx);
        if (cls)
            I.cls.assign(cls, cls + I.nnz);
        else
            I.cls.clear();
        reset_laws(ctx);
    });
}

int pd_clear_damage_laws(pd_ctx* ctx, int32_t inst)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        set_device(ctx);
        I.laws.clear();
        I.cls.clear();
        reset_laws(ctx);
    });
}

int pd_set_corrections(pd_ctx* ctx, int32_t inst, const pd_corrections* corr)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        if (corr) {
            if (corr->micromodulus != PD_MICRO_CONSTANT && corr->micromodulus != PD_MICRO_CONICAL)
                fail(PD_EINVAL, "unknown micromodulus profile");
            const bool need_delta = corr->micromodulus == PD_MICRO_CONICAL || corr->partial_volumes;
            if (need_delta && (!(corr->delta > 0.0) || !std::isfinite(corr->delta)))
                fail(PD_EINVAL, "delta must be positive and finite");
            if (corr->partial_volumes && (!(corr->dx > 0.0) || !std::isfinite(corr->dx)))
                fail(PD_EINVAL, "dx must be positive and finite");
        }
        set_device(ctx);
        I.has_corr = corr && (corr->micromodulus != PD_MICRO_CONSTANT || corr->partial_volumes || corr->surface);
        I.corr = corr ? *corr : pd_corrections{};
        upload_stiffness(ctx);
        upload_node_weights(ctx);
        ctx->drop_graphs();
    });
}

int pd_set_body_force(pd_ctx* ctx, int32_t inst, const double* b_hat, double magnitude)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        if (!std::isfinite(magnitude)) fail(PD_EINVAL, "magnitude must be finite");
        std::vector<double> b;
        if (b_hat) {
            b.assign(b_hat, b_hat + 3 * I.n);
            for (double x : b)
                if (!std::isfinite(x)) fail(PD_EINVAL, "b_hat must be finite");
        }
        set_device(ctx);
        I.bhat = std::move(b);
        I.bmag = b_hat ? magnitude : 0.0;
        upload_params(ctx);
        upload_body(ctx);
        ctx->a_valid = false;
        ctx->vv_ahead = false;
        ctx->drop_graphs();
    });
}

int pd_set_integrator(pd_ctx* ctx, int scheme, double dt)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        if (scheme != PD_EULER_CROMER && scheme != PD_VELOCITY_VERLET && scheme != PD_EULER_FORWARD)
            fail(PD_EINVAL, "unknown scheme");
        if (!(dt > 0.0) || !std::isfinite(dt)) fail(PD_EINVAL, "dt must be positive and finite");
        if (scheme != ctx->scheme || dt != ctx->dt) {
            ctx->tape_valid = false;
            ctx->scheme = scheme;
            ctx->dt = dt;
            ctx->a_valid = false;
            ctx->vv_ahead = false;
            ctx->drop_graphs();
        }
    });
}

int pd_step(pd_ctx* ctx, int64_t nsteps)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        require_built(ctx);
        if (nsteps < 0) fail(PD_EINVAL, "nsteps must be >= 0");
        if (ctx->step + nsteps >= std::numeric_limits<int32_t>::max())
            fail(PD_ERANGE, "step counter would exceed 2^31 - 1");
        set_device(ctx);
        do_steps(ctx, nsteps);
    });
}

int pd_prepare(pd_ctx* ctx)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        require_built(ctx);
        set_device(ctx);
        osb_checks(ctx);
        if (!ctx->use_graphs) return;
        const int mode = step_mode(ctx->scheme);
        for (int parity = 0; parity < 2; ++parity) (void)chunk_graph(ctx, mode, parity);
    });
}

int pd_sync(pd_ctx* ctx)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        set_device(ctx);
        sync(ctx);
        if (ctx->built) check_status(ctx);
    });
}

int pd_get_step(const pd_ctx* ctx, int64_t* step)
{
    if (!ctx || !step) return PD_EINVAL;
    *step = ctx->step;
    return PD_OK;
}

int pd_get_u(pd_ctx* ctx, int32_t inst, double* out)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (!out) fail(PD_EINVAL, "out is NULL");
        set_device(ctx);
        auto u = u_of(ctx, I);
        std::memcpy(out, u.data(), u.size() * sizeof(double));
        check_status(ctx);
    });
}

int pd_get_v(pd_ctx* ctx, int32_t inst, double* out)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (!out) fail(PD_EINVAL, "out is NULL");
        set_device(ctx);
        auto v = soa_of(ctx, I, ctx->v);
        std::memcpy(out, v.data(), v.size() * sizeof(double));
        check_status(ctx);
    });
}

int pd_get_a(pd_ctx* ctx, int32_t inst, double* out)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (!out) fail(PD_EINVAL, "out is NULL");
        set_device(ctx);
        auto a = soa_of(ctx, I, ctx->a);
        std::memcpy(out, a.data(), a.size() * sizeof(double));
    });
}

int pd_get_damage(pd_ctx* ctx, int32_t inst, double* out)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (!out) fail(PD_EINVAL, "out is NULL");
        set_device(ctx);
        launch_damage_now(ctx);
        std::vector<double> h(static_cast<size_t>(I.n_pad));
        download(h.data(), ctx->phi, h.size() * 8, I.node_off * 8, ctx->stream);
        sync(ctx);
        for (int64_t l = 0; l < I.n_pad; ++l)
            if (I.perm[l] >= 0) out[I.perm[l]] = h[l];
    });
}

int pd_set_model(pd_ctx* ctx, int32_t inst, int model, double K, double G)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        if (model != PD_MODEL_PMB && model != PD_MODEL_STATE_BASED) fail(PD_EINVAL, "unknown model");
        if (model == PD_MODEL_STATE_BASED) {
            if (!(K > 0.0) || !std::isfinite(K)) fail(PD_EINVAL, "K must be positive and finite");
            if (!(G >= 0.0) || !std::isfinite(G)) fail(PD_EINVAL, "G must be >= 0 and finite");
            if (ctx->mapping != PD_MAP_STAGED)
                fail(PD_EINVAL, "the state-based model runs in the staged mapping: call pd_set_mapping first");
        }
        set_device(ctx);
        I.osb = model == PD_MODEL_STATE_BASED;
        I.osb_K = I.osb ? K : 0.0;
        I.osb_G = I.osb ? G : 0.0;
        upload_params(ctx);
        upload_osb(ctx);
        ctx->a_valid = false;
        ctx->vv_ahead = false;
        ctx->drop_graphs();
        sync(ctx);
    });
}

int pd_get_dilation(pd_ctx* ctx, int32_t inst, double* out)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (!out) fail(PD_EINVAL, "out is NULL");
        if (!I.osb) fail(PD_EINVAL, "the instance does not run the state-based model");
        osb_checks(ctx);
        set_device(ctx);
        // the dilation pass at the current level, breaking nothing
        hip_check(launch_osb_dilation(step_args(ctx, ctx->cur, 1 - ctx->cur, 0), false, fp32(ctx), ctx->lanes,
                                      ctx->stream),
                  "dilation launch");
        std::vector<double> h(static_cast<size_t>(2 * I.n_pad));
        download(h.data(), ctx->osb, h.size() * 8, I.node_off * 16, ctx->stream);
        sync(ctx);
        for (int64_t l = 0; l < I.n_pad; ++l)
            if (I.perm[l] >= 0) out[I.perm[l]] = h[2 * l + 1] > 0.0 ? h[2 * l] / h[2 * l + 1] : 0.0;
    });
}

int pd_get_u_dev(pd_ctx* ctx, int32_t inst, double* out) { return get_nodes_dev(ctx, inst, out, 0); }
int pd_get_v_dev(pd_ctx* ctx, int32_t inst, double* out) { return get_nodes_dev(ctx, inst, out, 1); }
int pd_get_damage_dev(pd_ctx* ctx, int32_t inst, double* out) { return get_nodes_dev(ctx, inst, out, 2); }

int pd_get_broken(pd_ctx* ctx, int32_t inst, uint8_t* out)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (!out) fail(PD_EINVAL, "out is NULL");
        set_device(ctx);
        auto b = broken_of(ctx, I);
        std::memcpy(out, b.data(), b.size());
    });
}

int pd_get_max_stretch(pd_ctx* ctx, int32_t inst, double* out)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (!out) fail(PD_EINVAL, "out is NULL");
        set_device(ctx);
        const std::vector<double> sm = smax_of(ctx, I);
        std::memcpy(out, sm.data(), sm.size() * sizeof(double));
    });
}

int pd_set_max_stretch(pd_ctx* ctx, int32_t inst, const double* smax)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        if (!smax) fail(PD_EINVAL, "smax is NULL");
        if (!ctx->has_laws) fail(PD_ESTATE, "no damage laws");
        for (int64_t b = 0; b < I.nnz; ++b)
            if (!std::isfinite(smax[b]) || smax[b] < 0.0) fail(PD_EINVAL, "stretch state must be finite and >= 0");
        set_device(ctx);
        const std::vector<uint8_t> br = broken_of(ctx, I);
        upload_col(ctx, I, br.data(), true, smax);
        ctx->drop_graphs();
    });
}

int pd_get_force(pd_ctx* ctx, int32_t inst, double* out)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (!out) fail(PD_EINVAL, "out is NULL");
        set_device(ctx);
        eval_force(ctx);
        auto f = soa_of(ctx, I, ctx->force);
        std::memcpy(out, f.data(), f.size() * sizeof(double));
    });
}

// Device indices of a host node list of one instance (validated).
static std::vector<int64_t> device_nodes(const Inst& I, int64_t m, const int64_t* nodes)
{
    if (m < 1 || !nodes) fail(PD_EINVAL, "need at least one node");
    std::vector<int64_t> idx(static_cast<size_t>(m));
    for (int64_t i = 0; i < m; ++i) {
        if (nodes[i] < 0 || nodes[i] >= I.n) fail(PD_EINVAL, "node id out of range");
        idx[i] = I.node_off + I.iperm[nodes[i]];
    }
    return idx;
}

// out = sum over the listed device nodes of w_i field(i, .) (see launch_set_sum).
static void set_sum(pd_ctx* ctx, const std::vector<int64_t>& idx, const double* field, int64_t snode, int64_t scomp,
             const double* wv, double w, double out[3])
{
    ctx->rset.alloc(idx.size() * sizeof(int64_t));
    if (!ctx->rsum.p) ctx->rsum.alloc(3 * sizeof(double));
    upload(ctx->rset, idx.data(), idx.size() * sizeof(int64_t), 0, ctx->stream);
    hip_check(launch_set_sum(field, snode, scomp, wv, w, ctx->rset.as<int64_t>(), static_cast<int64_t>(idx.size()),
                             ctx->rsum.as<double>(), ctx->stream),
              "set-sum launch");
    download(out, ctx->rsum, 3 * sizeof(double), 0, ctx->stream);
    sync(ctx);
}

int pd_get_resultant(pd_ctx* ctx, int32_t inst, int64_t m, const int64_t* nodes, double out[3])
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (!out) fail(PD_EINVAL, "out is NULL");
        const std::vector<int64_t> idx = device_nodes(I, m, nodes);
        set_device(ctx);
        eval_force(ctx);
        set_sum(ctx, idx, ctx->force.as<double>(), 1, ctx->nn, ctx->has_vol ? ctx->vol.as<double>() : nullptr,
                I.volume, out);
    });
}

int pd_get_mean_displacement(pd_ctx* ctx, int32_t inst, int64_t m, const int64_t* nodes, double out[3])
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (!out) fail(PD_EINVAL, "out is NULL");
        const std::vector<int64_t> idx = device_nodes(I, m, nodes);
        set_device(ctx);
        const double w = 1.0 / static_cast<double>(m);
        if (fp32(ctx))  // the f64 master displacement, structure of arrays
            set_sum(ctx, idx, ctx->um[ctx->cur].as<double>(), 1, ctx->nn, nullptr, w, out);
        else            // the node records: x then u, 6 doubles per node
            set_sum(ctx, idx, ctx->rec[ctx->cur].as<double>() + 3, 6, 1, nullptr, w, out);
    });
}

int pd_get_mean_displacement_noalloc(pd_ctx* ctx, int32_t inst, int64_t m, const int64_t* nodes, double out[3])
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (!out || !nodes) fail(PD_EINVAL, "out or nodes is NULL");
        if (m < 1) fail(PD_EINVAL, "m must be >= 1");
        if (m > kScratchNodes) fail(PD_EINVAL, "at most 262144 nodes (the size of the device scratch array)");
        for (int64_t p = 0; p < m; ++p)
            if (nodes[p] < 0 || nodes[p] >= I.n) fail(PD_EINVAL, "node id out of range");
        require_built(ctx);
        set_device(ctx);
        int64_t* scr = nullptr;  // this GPU's scratch array: node ids, then the three sums
        hip_check(scratch_address(ctx->device, &scr), "scratch address");
        double* sums = reinterpret_cast<double*>(scr + kScratchNodes);
        hip_check(hipMemcpyAsync(scr, nodes, static_cast<size_t>(m) * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream),
                  "node ids to scratch");
        const double w = 1.0 / static_cast<double>(m);
        const int64_t* map = ctx->unode.as<int64_t>() + I.user_off;  // user node -> device node
        if (fp32(ctx))
            hip_check(launch_set_sum(ctx->um[ctx->cur].as<double>(), 1, ctx->nn, nullptr, w, scr, m, sums, ctx->stream,
                                     map),
                      "set-sum launch");
        else
            hip_check(launch_set_sum(ctx->rec[ctx->cur].as<double>() + 3, 6, 1, nullptr, w, scr, m, sums, ctx->stream,
                                     map),
                      "set-sum launch");
        hip_check(hipMemcpyAsync(out, sums, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream), "sums to host");
        sync(ctx);
    });
}

int pd_set_state(pd_ctx* ctx, int32_t inst, const double* u, const double* v, const double* a,
                 const uint8_t* broken)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        for (const double* p : {u, v, a})
            if (p)
                for (int64_t q = 0; q < 3 * I.n; ++q)
                    if (!std::isfinite(p[q])) fail(PD_EINVAL, "state must be finite");
        set_device(ctx);
        if (u) {
            // both buffers: the current one and the one the next step writes
            upload_state(ctx, I, u, nullptr, nullptr);
        }
        upload_state(ctx, I, nullptr, v, a);
        if (broken) {
            const std::vector<double> sm = smax_of(ctx, I);
            upload_col(ctx, I, broken, false, sm.data());
        }
        reset_flags_after_state_change(ctx, a != nullptr);
    });
}

int pd_set_step(pd_ctx* ctx, int64_t step)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        require_built(ctx);
        if (step < 0 || step >= std::numeric_limits<int32_t>::max()) fail(PD_EINVAL, "step out of range");
        set_device(ctx);
        ctx->tape_valid = false;
        ctx->step = step;
        upload(ctx->step_base, &step, sizeof step, 0, ctx->stream);
        sync(ctx);
        ctx->vv_ahead = false;
    });
}

int pd_get_state(pd_ctx* ctx, int32_t inst, pd_state* out)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (!out) fail(PD_EINVAL, "out is NULL");
        require_built(ctx);
        set_device(ctx);
        auto put = [](auto* dst, const auto& src) { std::memcpy(dst, src.data(), src.size() * sizeof(src[0])); };
        if (out->u) put(out->u, u_of(ctx, I));
        if (out->v) put(out->v, soa_of(ctx, I, ctx->v));
        if (out->a) put(out->a, soa_of(ctx, I, ctx->a));
        if (out->broken) put(out->broken, broken_of(ctx, I));
        if (out->max_stretch) put(out->max_stretch, smax_of(ctx, I));
        if (out->break_step) {
            std::vector<int32_t> h(static_cast<size_t>(I.n_dslots));
            download(h.data(), ctx->bstep, h.size() * sizeof(int32_t), static_cast<size_t>(I.dslot_off) * sizeof(int32_t),
                     ctx->stream);
            sync(ctx);
            for (int64_t d = 0; d < I.n_dslots; ++d)
                if (I.dslot_user[d] >= 0) out->break_step[I.dslot_user[d]] = h[d];
        }
        out->step = ctx->step;
        out->a_valid = ctx->a_valid ? 1 : 0;
        check_status(ctx);
    });
}

int pd_load_state(pd_ctx* ctx, int32_t inst, const pd_state* in)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        Inst& I = instance(ctx, inst);
        if (!in) fail(PD_EINVAL, "in is NULL");
        require_built(ctx);
        for (const double* p : {static_cast<const double*>(in->u), static_cast<const double*>(in->v), static_cast<const double*>(in->a)})
            if (p)
                for (int64_t q = 0; q < 3 * I.n; ++q)
                    if (!std::isfinite(p[q])) fail(PD_EINVAL, "state must be finite");
        // a stretch state: needs damage laws unless it is all zeros (what pd_get_state
        // exports for a problem without laws), which is then ignored
        const double* smax_in = in->max_stretch;
        if (smax_in) {
            bool zero = true;
            for (int64_t b = 0; b < I.nnz; ++b) {
                if (!std::isfinite(smax_in[b]) || smax_in[b] < 0.0) fail(PD_EINVAL, "stretch state must be finite and >= 0");
                zero = zero && smax_in[b] == 0.0;
            }
            if (!ctx->has_laws) {
                if (!zero) fail(PD_ESTATE, "a non-zero max_stretch given without damage laws");
                smax_in = nullptr;
            }
        }
        if (in->step < 0 || in->step >= std::numeric_limits<int32_t>::max()) fail(PD_EINVAL, "step out of range");
        set_device(ctx);
        if (in->u) upload_state(ctx, I, in->u, nullptr, nullptr);  // both displacement levels
        upload_state(ctx, I, nullptr, in->v, in->a);
        if (in->broken || smax_in) {
            const std::vector<uint8_t> br = in->broken ? std::vector<uint8_t>() : broken_of(ctx, I);
            const std::vector<double> sm = smax_in ? std::vector<double>() : smax_of(ctx, I);
            upload_col(ctx, I, in->broken ? in->broken : br.data(), !in->broken, smax_in ? smax_in : sm.data());
        }
        if (in->break_step) {
            std::vector<int32_t> h(static_cast<size_t>(I.n_dslots), kBrokeBefore);  // padding counts as broken
            for (int64_t d = 0; d < I.n_dslots; ++d)
                if (I.dslot_user[d] >= 0) h[d] = in->break_step[I.dslot_user[d]];
            upload(ctx->bstep, h.data(), h.size() * sizeof(int32_t), static_cast<size_t>(I.dslot_off) * sizeof(int32_t),
                   ctx->stream);
        }
        ctx->tape_valid = false;
        ctx->step = in->step;
        upload(ctx->step_base, &in->step, sizeof in->step, 0, ctx->stream);
        ctx->drop_graphs();
        reset_flags_after_state_change(ctx, in->a && in->a_valid);
    });
}

int pd_stretch_exact(int device, int64_t m, const double* xi, const double* y, double* s)
{
    if (m < 0 || (m > 0 && (!xi || !y || !s))) return PD_EINVAL;
    if (m == 0) return PD_OK;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return PD_EHIP;
    if (device < 0 || device >= count) return PD_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return PD_EHIP;
    const size_t v3 = static_cast<size_t>(3 * m) * sizeof(double), v1 = static_cast<size_t>(m) * sizeof(double);
    void* d = nullptr;
    if (hipMalloc(&d, 2 * v3 + v1) != hipSuccess) return PD_ENOMEM;
    char* b = static_cast<char*>(d);
    hipError_t e = hipMemcpy(b, xi, v3, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b + v3, y, v3, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = launch_stretch_exact(reinterpret_cast<const double*>(b), reinterpret_cast<const double*>(b + v3),
                                 reinterpret_cast<double*>(b + 2 * v3), m, nullptr);
    if (e == hipSuccess) e = hipMemcpy(s, b + 2 * v3, v1, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    return e == hipSuccess ? PD_OK : PD_EHIP;
}

int pd_set_mapping(pd_ctx* ctx, int mapping, int lanes)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        if (mapping != PD_MAP_SLICED && mapping != PD_MAP_STAGED) fail(PD_EINVAL, "unknown mapping");
        if (fp32(ctx) && mapping != PD_MAP_STAGED) fail(PD_EINVAL, "the FP32 build runs the staged mapping only");
        if (ctx->has_osb && mapping != PD_MAP_STAGED)
            fail(PD_EINVAL, "the state-based model runs in the staged mapping");
        if (lanes == 0) lanes = mapping == PD_MAP_STAGED ? 1 : kDefaultLanes;
        if (mapping == PD_MAP_STAGED && !split_supported(lanes))
            fail(PD_EINVAL, "unsupported wavefronts per slice (staged mapping: 1, 2 or 4)");
        if (mapping == PD_MAP_SLICED && !lanes_supported(lanes)) fail(PD_EINVAL, "unsupported lanes-per-node");
        if (!ctx->built) {
            ctx->mapping = mapping;
            ctx->lanes = lanes;
            return;
        }
        if (lanes == ctx->lanes && mapping == ctx->mapping) return;
        set_device(ctx);
        if (mapping == ctx->mapping && mapping == PD_MAP_STAGED) {  // same layout, other launch shape
            ctx->lanes = lanes;
            ctx->drop_graphs();
            ctx->tape_valid = false;  // a recompute would sum partial forces in another order
            return;
        }
        HostState S = snapshot(ctx);
        const bool av = ctx->a_valid;
        ctx->mapping = mapping;
        ctx->lanes = lanes;
        build_layout(ctx, &S);
        ctx->a_valid = av;
    });
}

int pd_set_lanes_per_node(pd_ctx* ctx, int lanes) { return pd_set_mapping(ctx, PD_MAP_SLICED, lanes); }

int pd_autotune(pd_ctx* ctx, int64_t trial_steps, int32_t* chosen)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        require_built(ctx);
        if (trial_steps < 1) fail(PD_EINVAL, "trial_steps must be >= 1");
        set_device(ctx);
        HostState S = snapshot(ctx);
        const int64_t step0 = ctx->step;
        const bool av = ctx->a_valid;
        struct Cand {
            int mapping, lanes, order;
        };
        std::vector<Cand> cands;
        const int orders[] = {PD_ORDER_NATURAL, PD_ORDER_MORTON};
        for (int o : orders) {
            if (!ctx->order_auto && o != ctx->order) continue;
            if (!fp32(ctx) && !ctx->has_osb)
                for (int L : {1, 4, 16, 64}) cands.push_back({PD_MAP_SLICED, L, o});
            for (int S : {1, 2, 4}) cands.push_back({PD_MAP_STAGED, S, o});
        }
        Cand best{ctx->mapping, ctx->lanes, ctx->order};
        double best_ms = std::numeric_limits<double>::infinity();
        for (const Cand& cd : cands) {
            ctx->mapping = cd.mapping;
            ctx->lanes = cd.lanes;
            ctx->order = cd.order;
            build_layout(ctx, &S);
            ctx->a_valid = av;
            for (int rep = 0; rep < 2; ++rep)  // first pass builds graphs and warms caches
                do_steps(ctx, trial_steps);
            float ms = 0.f;
            sync(ctx);
            hip_check(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1), "hipEventElapsedTime");
            if (ms < best_ms) {
                best_ms = ms;
                best = cd;
            }
            ctx->step = step0;
        }
        ctx->order = best.order;
        ctx->mapping = best.mapping;
        ctx->lanes = best.lanes;
        build_layout(ctx, &S);
        ctx->step = step0;
        const int64_t st = step0;
        upload(ctx->step_base, &st, sizeof st, 0, ctx->stream);
        sync(ctx);
        ctx->a_valid = av;
        reset_flags_after_state_change(ctx, av);
        if (chosen) *chosen = best.mapping == PD_MAP_STAGED ? -best.lanes : best.lanes;
    });
}

namespace {
std::atomic<int64_t> g_recordings{0};  // recording ids handed out in this process
}

int pd_adj_forward(pd_ctx* ctx, int64_t nsteps, int32_t ckpt_every, int64_t* recording)
{
    if (!ctx) return PD_EINVAL;
    if (recording) *recording = 0;
    return guarded(ctx, [&] {
        adjoint_checks(ctx);
        if (nsteps < 1) fail(PD_EINVAL, "nsteps must be >= 1");
        if (ckpt_every < 1) fail(PD_EINVAL, "ckpt_every must be >= 1");
        if (ctx->step + nsteps >= std::numeric_limits<int32_t>::max())
            fail(PD_ERANGE, "step counter would exceed 2^31 - 1");
        set_device(ctx);
        Inst& I = ctx->inst[0];
        check_symmetric(I);
        init_break_steps(ctx, I);
        const int64_t nn = ctx->nn;
        const size_t Rb = rec_bytes(nn), Vb = static_cast<size_t>(3 * nn) * sizeof(double);
        const int64_t C = (nsteps + ckpt_every - 1) / ckpt_every;
        // with a checkpoint at every level nothing is recomputed and v is not needed
        const size_t stride = Rb + (ckpt_every > 1 ? Vb : 0);
        const int64_t step0 = ctx->step;
        if (ckpt_every == 1) {
            // the whole trajectory: step k reads level k of the tape and writes level k+1
            // straight into it (every level first gets the positions, sentinel and spare
            // records); the last level then becomes the current state
            ctx->ck.alloc(static_cast<size_t>(nsteps + 1) * Rb);
            char* tape = ctx->ck.as<char>();
            for (int64_t k = 0; k <= nsteps; ++k)
                hip_check(hipMemcpyAsync(tape + static_cast<size_t>(k) * Rb, ctx->rec[ctx->cur].p, Rb,
                                         hipMemcpyDeviceToDevice, ctx->stream),
                          "trajectory init");
            for (int64_t k = 0; k < nsteps; ++k) {
                StepArgs A = step_args(ctx, ctx->cur, 1 - ctx->cur, k);
                A.rec_in = reinterpret_cast<const double*>(tape + static_cast<size_t>(k) * Rb);
                A.rec_out = reinterpret_cast<double*>(tape + static_cast<size_t>(k + 1) * Rb);
                launch_ec(ctx, A);
            }
            hip_check(launch_advance(ctx->step_base.as<int64_t>(), nsteps, ctx->stream), "advance launch");
            hip_check(hipMemcpyAsync(ctx->rec[ctx->cur].p, tape + static_cast<size_t>(nsteps) * Rb, Rb,
                                     hipMemcpyDeviceToDevice, ctx->stream),
                      "trajectory end");
            ctx->step += nsteps;
            ctx->tape_valid = true;
            ctx->tape_step0 = step0;
            ctx->tape_nsteps = nsteps;
            ctx->tape_every = 1;
            ctx->tape_id = ++g_recordings;
            if (recording) *recording = ctx->tape_id;
            return;
        }
        ctx->ck.alloc(static_cast<size_t>(C) * stride);
        for (int64_t c = 0; c < C; ++c) {
            char* dst = ctx->ck.as<char>() + static_cast<size_t>(c) * stride;
            hip_check(hipMemcpyAsync(dst, ctx->rec[ctx->cur].p, Rb, hipMemcpyDeviceToDevice, ctx->stream),
                      "checkpoint copy");
            if (ckpt_every > 1)
                hip_check(hipMemcpyAsync(dst + Rb, ctx->v.p, Vb, hipMemcpyDeviceToDevice, ctx->stream),
                          "checkpoint copy");
            do_steps(ctx, std::min<int64_t>(ckpt_every, nsteps - c * ckpt_every));
        }
        ctx->tape_valid = true;
        ctx->tape_step0 = step0;
        ctx->tape_nsteps = nsteps;
        ctx->tape_every = ckpt_every;
        ctx->tape_id = ++g_recordings;
        if (recording) *recording = ctx->tape_id;
    });
}

int pd_adj_backward(pd_ctx* ctx, int64_t recording, int64_t m, const int64_t* sensors, const double* dL_du,
                    double* grad_k, double* grad_A)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        adjoint_checks(ctx);
        if (!ctx->tape_valid) fail(PD_ESTATE, "no recorded forward run (pd_adj_forward) for the current problem");
        if (recording != 0 && recording != ctx->tape_id)
            fail(PD_ESTATE, "the recording asked for has been replaced by a later pd_adj_forward or discarded");
        if (m < 0 || (m > 0 && (!sensors || !dL_du))) fail(PD_EINVAL, "bad sensor arguments");
        if (!grad_k || !grad_A) fail(PD_EINVAL, "gradient outputs are NULL");
        const Inst& I = ctx->inst[0];
        std::vector<int64_t> dsens(static_cast<size_t>(m));
        for (int64_t p = 0; p < m; ++p) {
            if (sensors[p] < 0 || sensors[p] >= I.n) fail(PD_EINVAL, "sensor node id out of range");
            dsens[p] = I.node_off + I.iperm[sensors[p]];
        }
        for (int64_t q = 0; q < 3 * m; ++q)
            if (!std::isfinite(dL_du[q])) fail(PD_EINVAL, "dL_du must be finite");
        set_device(ctx);
        hipStream_t st = ctx->stream;
        const int64_t nn = ctx->nn, ns = ctx->ns, S = ctx->tape_every, T = ctx->tape_nsteps, step0 = ctx->tape_step0;
        // adjoint velocities: nn + 1 triples (the last one, the sentinel's, zero) and spare zero
        // entries for the staged kernel's fixed-size range windows
        const size_t Rb = rec_bytes(nn), Vb = static_cast<size_t>(3 * nn) * sizeof(double),
                     Nb = (static_cast<size_t>(3 * (nn + 1)) + kStageChunks) * sizeof(double);
        const int64_t Lmax = std::min(S, T);
        const size_t stride = Rb + (S > 1 ? Vb : 0);
        DevBuf traj, vwork, nu[2], lam, grad, gacc, base, sum, dsn, ddl;
        traj.alloc(static_cast<size_t>(Lmax) * Rb);  // levels 1 .. Lmax-1 of a segment (level 0: its checkpoint)
        vwork.alloc(Vb);
        nu[0].alloc(Nb);
        nu[1].alloc(Nb);
        lam.alloc(Vb);
        grad.alloc((static_cast<size_t>(ns) + kSpareRows * kWave) * sizeof(double));  // slot layout, spare rows
        gacc.alloc(static_cast<size_t>(nn) * sizeof(double));
        base.alloc(sizeof(int64_t));
        sum.alloc(sizeof(double));
        dsn.alloc(static_cast<size_t>(m) * sizeof(int64_t));
        ddl.alloc(static_cast<size_t>(3 * m) * sizeof(double));
        auto at = [](const DevBuf& b, size_t off) { return static_cast<char*>(b.p) + off; };
        // every level carries the positions, the sentinel and the spare records
        for (int64_t s = 1; s < Lmax; ++s)
            hip_check(hipMemcpyAsync(at(traj, s * Rb), ctx->rec[ctx->cur].p, Rb, hipMemcpyDeviceToDevice, st),
                      "trajectory init");
        for (DevBuf* b : {&nu[0], &nu[1], &lam, &grad, &gacc})
            hip_check(hipMemsetAsync(b->p, 0, b->bytes, st), "hipMemsetAsync");
        upload(dsn, dsens.data(), dsens.size() * sizeof(int64_t), 0, st);
        upload(ddl, dL_du, static_cast<size_t>(3 * m) * sizeof(double), 0, st);
        hip_check(launch_adj_seed(lam.as<double>(), nn, dsn.as<int64_t>(), ddl.as<double>(), m, st), "seed launch");
        hip_check(launch_adj_nu0(nu[0].as<double>(), lam.as<double>(), ctx->bc_id.as<int32_t>(), ctx->bc.as<BCRec>(),
                                 nn, ctx->dt, st),
                  "seed launch");

        AdjArgs a{};
        a.lam_u = lam.as<double>();
        a.grad = grad.as<double>();
        a.gacc = gacc.as<double>();
        a.bstep = ctx->bstep.as<int32_t>();
        a.col = ctx->col.as<int32_t>();
        a.ent = ctx->ent.as<uint16_t>();
        a.pieces = ctx->pieces.as<int2>();
        a.slice_piece = ctx->slice_piece.as<int32_t>();
        a.kslot = ctx->has_stiff ? ctx->kslot.as<double>() : nullptr;
        a.vol = ctx->has_vol ? ctx->vol.as<double>() : nullptr;
        a.na = ctx->has_knode ? ctx->na.as<double>() : nullptr;
        a.bhat = ctx->has_body ? ctx->bhat.as<double>() : nullptr;
        a.slice_ptr = ctx->slice_ptr.as<int64_t>();
        a.slice_T = ctx->slice_T.as<int32_t>();
        a.slice_inst = ctx->slice_inst.as<int32_t>();
        a.params = ctx->params.as<InstParams>();
        a.bc_id = ctx->bc_id.as<int32_t>();
        a.bc = ctx->bc.as<BCRec>();
        a.nn = nn;
        a.nslices = ctx->nslices;
        a.dt = ctx->dt;
        const bool staged = ctx->mapping == PD_MAP_STAGED;
        int nin = 0;
        const int64_t C = (T + S - 1) / S;
        for (int64_t c = C - 1; c >= 0; --c) {
            const int64_t s0 = step0 + c * S, len = std::min(S, T - c * S);
            const char* ck = ctx->ck.as<char>() + static_cast<size_t>(c) * stride;
            auto level = [&](int64_t s) {
                return reinterpret_cast<const double*>(s == 0 ? ck : at(traj, s * Rb));
            };
            if (len > 1) {
                // recompute levels 1 .. len-1 with the forward kernel from the checkpoint
                // (the reverse passes read levels 0 .. len-1)
                hip_check(launch_flags_at(ctx->bstep.as<int32_t>(), ctx->col.as<int32_t>(), ctx->ent.as<uint16_t>(),
                                          ns, s0, st),
                          "flags launch");
                hip_check(hipMemcpyAsync(vwork.p, ck + Rb, Vb, hipMemcpyDeviceToDevice, st), "checkpoint restore");
                hip_check(launch_set_i64(base.as<int64_t>(), s0, st), "base launch");
                for (int64_t s = 0; s + 1 < len; ++s) {
                    StepArgs A = step_args(ctx, ctx->cur, 1 - ctx->cur, s);
                    A.rec_in = level(s);
                    A.rec_out = reinterpret_cast<double*>(at(traj, (s + 1) * Rb));
                    A.v = vwork.as<double>();
                    A.step_base = base.as<int64_t>();  // breaks re-record the same passes
                    launch_ec(ctx, A);
                }
            }
            // reverse passes of the segment, last first
            for (int64_t s = len - 1; s >= 0; --s) {
                a.rec = level(s);
                a.nu_in = nu[nin].as<double>();
                a.nu_out = nu[1 - nin].as<double>();
                a.k = s0 + s;
                hip_check(launch_adjoint(a, staged, ctx->lanes, st), "adjoint launch");
                nin ^= 1;
            }
        }
        // leave the broken flags as the forward run left them
        hip_check(launch_flags_at(ctx->bstep.as<int32_t>(), ctx->col.as<int32_t>(), ctx->ent.as<uint16_t>(), ns,
                                  step0 + T, st),
                  "flags launch");
        hip_check(launch_sum(gacc.as<double>(), nn, sum.as<double>(), st), "sum launch");
        std::vector<double> g(static_cast<size_t>(I.n_dslots));
        double gA = 0.0;
        download(g.data(), grad, g.size() * sizeof(double), static_cast<size_t>(I.dslot_off) * sizeof(double), st);
        download(&gA, sum, sizeof gA, 0, st);
        sync(ctx);
        std::fill(grad_k, grad_k + I.nnz, 0.0);
        for (int64_t d = 0; d < I.n_dslots; ++d) {
            const int32_t b = I.dslot_user[d];
            if (b >= 0) grad_k[b] = g[d];
        }
        *grad_A = gA;
    });
}

int pd_get_break_steps(pd_ctx* ctx, int32_t inst, int32_t* out)
{
    if (!ctx) return PD_EINVAL;
    return guarded(ctx, [&] {
        const Inst& I = instance(ctx, inst);
        if (!out) fail(PD_EINVAL, "out is NULL");
        require_built(ctx);
        set_device(ctx);
        std::vector<int32_t> h(static_cast<size_t>(I.n_dslots));
        download(h.data(), ctx->bstep, h.size() * sizeof(int32_t), static_cast<size_t>(I.dslot_off) * sizeof(int32_t),
                 ctx->stream);
        sync(ctx);
        for (int64_t d = 0; d < I.n_dslots; ++d) {
            const int32_t b = I.dslot_user[d];
            if (b >= 0) out[b] = h[d];
        }
    });
}

int pd_get_info(const pd_ctx* ctx, pd_info* info)
{
    if (!ctx || !info) return PD_EINVAL;
    std::memset(info, 0, sizeof *info);
    if (!ctx->built) return PD_OK;
    int64_t n = 0, nnz = 0;
    for (auto& I : ctx->inst) {
        n += I.n;
        nnz += I.nnz;
    }
    info->n_nodes = n;
    info->n_slots = nnz;
    info->n_nodes_dev = ctx->nn;
    info->n_slots_dev = ctx->ns;
    info->n_instances = static_cast<int32_t>(ctx->inst.size());
    info->lanes_per_node = ctx->mapping == PD_MAP_STAGED ? 1 : ctx->lanes;
    info->waves_per_slice = ctx->mapping == PD_MAP_STAGED ? ctx->lanes : 1;
    info->mapping = ctx->mapping;
    info->order = ctx->order;
    info->precision = ctx->precision;
    info->scheme = ctx->scheme;
    // algorithmic bytes: 4 per slot (+8 with a stiffness field); per node x (24 B) read,
    // u read + write, v read + write, a read + write (velocity Verlet); the FP32 build also
    // reads and writes the f32 displacement copy (12 + 12 B)
    double per_node = 24.0 + 4.0 * 24.0 + (ctx->scheme == PD_VELOCITY_VERLET ? 2.0 * 24.0 : 0.0) +
                      (ctx->precision == PD_FP32 ? 24.0 : 0.0);
    per_node += ctx->has_knode ? 16.0 : 0.0;  // per-node stiffness factors (own and neighbour weight)
    per_node += ctx->corr_k ? 8.0 : 0.0;      // family volumes of the per-slot corrections
    info->model_bytes_per_step = static_cast<double>(nnz) * (4.0 + (ctx->has_stiff ? 8.0 : 0.0)) +
                                 static_cast<double>(n) * per_node;
    if (ctx->has_osb)  // two passes: the neighbour index twice; x and u read again, the node pair
                       // {theta/m, 1/m} written, then read, with 1/m read by the first pass
        info->model_bytes_per_step += static_cast<double>(nnz) * 4.0 + static_cast<double>(n) * (48.0 + 16.0 + 16.0 + 8.0);
    return PD_OK;
}

int pd_last_step_ms(pd_ctx* ctx, double* ms)
{
    if (!ctx || !ms) return PD_EINVAL;
    return guarded(ctx, [&] {
        if (!ctx->timed) fail(PD_ESTATE, "no pd_step has been timed yet");
        set_device(ctx);
        hip_check(hipEventSynchronize(ctx->ev1), "hipEventSynchronize");
        float f = 0.f;
        hip_check(hipEventElapsedTime(&f, ctx->ev0, ctx->ev1), "hipEventElapsedTime");
        *ms = f;
    });
}

}  // extern "C"
