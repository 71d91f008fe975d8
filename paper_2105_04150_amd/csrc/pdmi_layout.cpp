// pdmi_layout.cpp -- family search, node renumbering and the device layout (sliced
// and staged) of new problems.
#include "pdmi_host.h"

namespace pdmi {
namespace host {

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
static double spacing_estimate(const Inst& I)
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

static uint64_t spread3(uint64_t v)
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
static void node_order(Inst& I, int order, double h)
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

// Processing order of the staged slices (context-wide indices).  xcd_remap hands each XCD
// a contiguous share of the dispatch positions; within every share the slices keep their
// device order but the longer ones (more slot rows, in buckets of 8) go first, so that the
// last workgroups of a launch are the short ones and the tail of the launch is short.
// Every slice writes only its own nodes, so results do not depend on the order.
static std::vector<int32_t> slice_dispatch_order(const std::vector<int32_t>& slice_piece,
                                                 const std::vector<int2>& pieces)
{
    const int64_t nsl = static_cast<int64_t>(slice_piece.size()) - 1;
    std::vector<int32_t> order(static_cast<size_t>(nsl)), rows(static_cast<size_t>(nsl), 0);
    for (int64_t s = 0; s < nsl; ++s) {
        order[s] = static_cast<int32_t>(s);
        for (int32_t q = slice_piece[s]; q < slice_piece[s + 1]; ++q) rows[s] += (pieces[q].y >> 8) & 0xff;
    }
    constexpr int64_t X = 8;  // XCDs, as xcd_remap splits the dispatch
    const int64_t m = nsl / X, r = nsl % X;
    int64_t b0 = 0;
    for (int64_t x = 0; x < X; ++x) {
        const int64_t len = m + (x < r ? 1 : 0);
        std::stable_sort(order.begin() + b0, order.begin() + b0 + len,
                         [&](int32_t a, int32_t b) { return rows[a] / 8 > rows[b] / 8; });
        b0 += len;
    }
    return order;
}

// Order of each row's slots on the device: by the bond offset rounded to the lattice
// spacing (z, then y, then x), so lanes of neighbouring nodes visit neighbours at the
// same relative position together.  On a natural-order lattice this is ascending j.
static std::vector<int32_t> slot_ranks(const Inst& I, double h)
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

// Staged layout of one instance (one lane per node, 64 nodes per slice): per slice, the
// sorted union of neighbour device indices is cut into ranges of consecutive nodes
// (at most kSegMax long); each lane's slots in a range, in ascending neighbour order,
// fill rows of pieces of at most kPieceRows rows.  Fills start (first slot of each slice),
// pieces, slice_piece, dslot_user and ent_idx; returns the slot count.
static int64_t build_staged(Inst& I, std::vector<int64_t>& start)
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
        const std::vector<int32_t> order = slice_dispatch_order(spc, pcs);
        ctx->slice_order.alloc(order.size() * sizeof(int32_t));
        upload(ctx->slice_order, order.data(), order.size() * sizeof(int32_t), 0, ctx->stream);
    } else {
        ctx->slice_order.release();
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
                 int order, const int64_t* user_row_ptr, const int32_t* user_col)
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

}  // namespace host
}  // namespace pdmi

