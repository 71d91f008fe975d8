// pdmi_api.cpp -- C ABI: contexts, families, material, boundary conditions, damage laws,
// corrections, loads and the integrator.
#include "pdmi_host.h"

using namespace pdmi;
using namespace pdmi::host;

namespace {
std::string g_create_error;  // message of the last failed pd_create
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

}  // extern "C"
