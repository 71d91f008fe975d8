// pdmi_api_state.cpp -- C ABI: stepping, readouts, state and checkpoints, the
// allocation-free readout, mapping and autotuning, and problem information.
#include "pdmi_host.h"

using namespace pdmi;
using namespace pdmi::host;

extern "C" {

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

