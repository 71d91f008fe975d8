// pdmi_api_adjoint.cpp -- C ABI: the recorded forward run and the reverse pass of
// the adjoint (Sec. 3.6).
#include "pdmi_host.h"

using namespace pdmi;
using namespace pdmi::host;

extern "C" {

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
                // staged: the step kernels' slice order (each XCD's share longest first)
                hip_check(staged ? launch_adjoint_ordered(a, ctx->slice_order.as<int32_t>(), true, ctx->lanes, st)
                                 : launch_adjoint(a, false, ctx->lanes, st),
                          "adjoint launch");
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

}  // extern "C"
