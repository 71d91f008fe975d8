// pdmi_run.cpp -- stepping in stream order with hipGraph replay, force evaluation,
// damage, readouts into device memory and sums over node sets.
#include "pdmi_host.h"

namespace pdmi {
namespace host {

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
    A.slice_order = ctx->slice_order.p ? ctx->slice_order.as<int32_t>() : nullptr;
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

static void launch_steps(pd_ctx* ctx, int mode, int cur, int64_t count)
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
static void require_device_buffer(const pd_ctx* ctx, const void* p)
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

// Device indices of a host node list of one instance (validated).
std::vector<int64_t> device_nodes(const Inst& I, int64_t m, const int64_t* nodes)
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
void set_sum(pd_ctx* ctx, const std::vector<int64_t>& idx, const double* field, int64_t snode, int64_t scomp,
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

}  // namespace host
}  // namespace pdmi

