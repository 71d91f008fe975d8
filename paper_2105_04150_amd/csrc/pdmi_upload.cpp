// pdmi_upload.cpp -- instance parameters, boundary-condition, stiffness, volume, load
// and damage-law tables, the state and slot words, and readouts to the host.
#include "pdmi_host.h"

namespace pdmi {
namespace host {

static InstParams make_params(const Inst& I, int32_t law_off)
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

// Correction factors of one instance applied to a slot stiffness k (user CSR order b of
// row i): micromodulus profile, partial volume, surface correction, in that order.
struct CorrectionTable {
    std::vector<double> famvol;  // per node (surface correction)
    double v0 = 0.0;
};

static double partial_volume(const pd_corrections& c, double L)
{
    const double h = 0.5 * c.dx;
    if (L <= c.delta - h) return 1.0;
    if (L >= c.delta + h) return 0.0;
    return (c.delta + h - L) / c.dx;
}

static double ref_length(const Inst& I, int64_t i, int64_t j)
{
    const double a = I.x[3 * j] - I.x[3 * i], b = I.x[3 * j + 1] - I.x[3 * i + 1], c = I.x[3 * j + 2] - I.x[3 * i + 2];
    return std::sqrt((a * a + b * b) + c * c);
}

static CorrectionTable correction_table(const Inst& I)
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

static double corrected(const Inst& I, const CorrectionTable& T, int64_t i, int64_t j, double k)
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
static bool corrections_in_kernel(const pd_ctx* ctx)
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
static void upload_family_volumes(pd_ctx* ctx)
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

// Per-slot stiffness of every instance (instances without a field get their c), or only
// of instance `only` when the array already exists.
void upload_stiffness(pd_ctx* ctx, int32_t only)
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
static std::vector<uint8_t> nofail_slots(const Inst& I)
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
void upload_col(pd_ctx* ctx, Inst& I, const uint8_t* broken, bool keep_bsteps,
                const double* smax)
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

}  // namespace host
}  // namespace pdmi

