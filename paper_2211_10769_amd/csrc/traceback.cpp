// traceback.cpp -- the reconstruction phase: canonical CIGAR of the aligned
// rectangle in linear space.
//
// Definition reproduced (the full-matrix greedy walk): global Gotoh DP over
// A[1..p] x B[1..q] (G = H without zero clamp), walked back from (p, q) in
// state H preferring the diagonal, then F ('I'), then E ('D'), and inside a
// gap preferring to close it.  That walk only ever compares forward values
// of a node and its predecessors.
//
// Frontier-seeded divide and conquer, bottom half first.  A subproblem is
// rows (r_top, r_bot], columns [L, J], the true forward values on row r_top
// (H and the F it hands down) for those columns, and an end node (r_bot, J)
// in state H or F with its forward value V.  A split at mid row r:
//   * forward pass from the frontier to row r (strip kernel, global mode);
//   * backward pass from the end node up to row r+1 (the same kernel on the
//     reversed rows and columns; its values are the backward values);
//   * crossing scan: edges from row r into row r+1 with fwd + edge + bwd = V;
//     cmin = the leftmost frontier column such an edge uses.
// Bottom child: rows (r, r_bot], columns [cmin, J], frontier = the forward
// pass output there, same end.  Every node on an optimal path has a best
// path that crosses inside the crossing set, so the restricted DP gives the
// true forward value at every node the walk can visit, and non-optimal
// predecessors stay non-optimal: the walk is identical to the full-matrix
// one.  Top child: rows (r_top, r], columns [L, j*], the parent's frontier,
// ending at the node (r, j*) where the bottom child's walk leaves row r+1.
// When the crossing edge is unique that node is known at once and both
// halves are ready together; otherwise the top half waits for the walk.
//
// Subproblems are processed level by level: all ready splits in one batch of
// launches, all ready leaves in another, so the many small subproblems of
// the deep levels run side by side across the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <charconv>
#include <chrono>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "context.h"
#include "strips.h"
#include "tb_kernels.h"
#include "traceback.h"
#include "tune.h"

namespace swh {

namespace {

// Leaf budget inside the 64 KB of LDS one workgroup may take: 1 KB matrix,
// an 8-byte row buffer entry per column, one byte of tie flags per cell.
constexpr int64_t kLeafCells = 28672;
constexpr int64_t kLeafMaxWidth = 4096;
// Larger leaves keep their tie flags in global memory (one byte per cell):
// a subproblem of up to this many cells is solved by one wave at once rather
// than split further, which saves levels (each a host round trip) when many
// small subproblems are in flight; leaf launches are cut so that one launch's
// flags stay within kLeafFlagBytes.
constexpr int64_t kLeafCellsMax = (int64_t)1 << 19;
constexpr int64_t kLeafFlagBytes = (int64_t)8 << 30;


struct Node {
    int pair = 0;
    const uint8_t *A = nullptr;      // codes of the pair's rectangle rows (device)
    const uint8_t *bpad = nullptr;   // pad code, then the rectangle columns (device)
    int64_t r_top, r_bot, L, J;
    const Border *front;      // front[k] <-> column front_L + k, covers [L, J]
    int64_t front_L;
    int end_state;            // 0 = H, 1 = F
    int32_t V;
    int bottom = -1, top = -1, parent = -1;
    bool is_top_child = false;
    bool ready = false, leaf = false;
    bool exit_known = false;
    int64_t exit_col = -1;
    int exit_state = 0;
    int32_t exit_val = 0;
    int64_t ops_off = 0, nops = 0;   // leaf ops (backward) in the host op buffer
};

template <typename T>
swh_status upload(swh_ctx *ctx, DevBuf &buf, const std::vector<T> &v, hipStream_t st, const char *what)
{
    swh_status s = ensure(ctx, buf, v.size() * sizeof(T) + 16, what);
    if (s != SWH_OK) return s;
    hipError_t e = hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(ctx, e, what);
    return SWH_OK;
}

}  // namespace

swh_status traceback_batch(swh_ctx *ctx, const std::vector<TbInput> &in, const Scoring &sc, hipStream_t st,
                           std::vector<std::string> &cigars, TracebackStats &ts)
{
    const auto t0 = std::chrono::steady_clock::now();
    const uint8_t pad = (uint8_t)sc.asize;
    const int npairs = (int)in.size();
    cigars.assign((size_t)npairs, std::string());
    if (npairs == 0) return SWH_OK;
    Arena &arena = ctx->tb_arena;   // kept across calls, handed out afresh each time
    arena.reset();
    hipError_t e;
    swh_status s;

    // per pair: B with the pad code in front (bpad[j] = code of B_j, bpad[0] =
    // pad); per band the root of its subproblem tree: the top band starts from
    // the rectangle's top border G(0, j), F(1, j) = G(0, j) - o, every other
    // band from the single node where the path crosses into it
    std::vector<Node> nodes;
    nodes.reserve((size_t)npairs * 4);
    std::vector<std::vector<int>> roots((size_t)npairs);   // top band first
    std::vector<GatherDesc> gd0;
    std::vector<BorderInit> bi0;
    for (int k = 0; k < npairs; ++k) {
        const TbInput &x = in[k];
        uint8_t *bpad = (uint8_t *)arena.get((size_t)x.q + 2, ctx->held, ctx->opt.mem_cap);
        if (!bpad) return fail(ctx, SWH_E_NOMEM, "traceback arena");
        gd0.push_back(GatherDesc{x.B, bpad, 0, x.q, x.q + 1, 1, 1});
        std::vector<TbBand> bands = x.bands;
        if (bands.empty()) bands.push_back(TbBand{0, x.p, 0, x.q, false, 0, 0, 0, x.S});
        for (const TbBand &b : bands) {
            if (b.r_top < 0 || b.r_bot > x.p || b.r_top >= b.r_bot || b.L < 0 || b.J > x.q || b.L > b.J ||
                (!b.seeded && (b.r_top != 0 || b.L != 0))) {
                ts.inconsistent = true;
                return fail(ctx, SWH_E_DEVICE, "traceback: malformed band (internal error)");
            }
            const int64_t cnt = b.seeded ? b.J - b.L + 1 : x.q + 1;
            Border *front = (Border *)arena.get(sizeof(Border) * (size_t)cnt, ctx->held, ctx->opt.mem_cap);
            if (!front) return fail(ctx, SWH_E_NOMEM, "traceback arena");
            bi0.push_back(BorderInit{front, nullptr, cnt, cnt, b.seeded ? 3 : 1, b.seed_h, b.seed_f, 0});
            Node root;
            root.pair = k;
            root.A = x.A;
            root.bpad = bpad;
            root.r_top = b.r_top;
            root.r_bot = b.r_bot;
            root.L = b.L;
            root.J = b.J;
            root.front = front;
            root.front_L = b.seeded ? b.L : 0;
            root.end_state = b.end_state;
            root.V = b.V;
            root.ready = true;
            roots[k].push_back((int)nodes.size());
            nodes.push_back(root);
        }
    }
    if ((s = upload(ctx, ctx->tb_misc, gd0, st, "gather table")) != SWH_OK) return s;
    if ((e = launch_gather((const GatherDesc *)ctx->tb_misc.p, (int32_t)gd0.size(), pad, st)) != hipSuccess)
        return hip_fail(ctx, e, "gather launch");
    if ((s = upload(ctx, ctx->tb_leaf, bi0, st, "border table")) != SWH_OK) return s;
    if ((e = launch_border_init((const BorderInit *)ctx->tb_leaf.p, (int32_t)bi0.size(), sc.o, sc.e, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(ctx, e, "traceback setup");

    // the leaves' ops on the host: the context's pinned buffer, ops_used bytes in use
    size_t ops_used = 0;
    auto ops_room = [&](size_t more) -> bool {
        if (ops_used + more <= ctx->tb_ops_host_cap) return true;
        const size_t cap = std::max(ops_used + more, 2 * ctx->tb_ops_host_cap);
        char *p = nullptr;
        if (hipHostMalloc(reinterpret_cast<void **>(&p), cap, hipHostMallocDefault) != hipSuccess || !p) {
            (void)hipGetLastError();
            return false;
        }
        if (ops_used) std::memcpy(p, ctx->tb_ops_host, ops_used);
        if (ctx->tb_ops_host) hipHostFree(ctx->tb_ops_host);
        ctx->tb_ops_host = p;
        ctx->tb_ops_host_cap = cap;
        return true;
    };
    std::vector<int> ready((size_t)nodes.size());
    for (size_t k = 0; k < nodes.size(); ++k) ready[k] = (int)k;
    // the leaf-size option lowers it (tests use it to force deep recursion on small inputs)
    const int64_t leaf_cells =
        std::max<int64_t>(1, std::min<int64_t>(kLeafCellsMax, ctx->opt.tb_leaf > 0 ? ctx->opt.tb_leaf : kLeafCellsMax));

    // exit of node k is known: tell its parent chain and release a waiting top sibling
    auto propagate = [&](int k) {
        while (k >= 0) {
            Node &n = nodes[k];
            const int par = n.parent;
            if (par < 0) break;
            Node &pn = nodes[par];
            if (!n.is_top_child) {
                Node &tp = nodes[pn.top];
                if (!tp.ready && !tp.exit_known && tp.J < 0) {
                    tp.J = n.exit_col;
                    tp.end_state = n.exit_state;
                    tp.V = n.exit_val;
                    tp.ready = true;
                    ready.push_back(pn.top);
                }
                break;
            }
            // top child: its exit is its parent's exit
            pn.exit_known = true;
            pn.exit_col = n.exit_col;
            pn.exit_state = n.exit_state;
            pn.exit_val = n.exit_val;
            k = par;
        }
    };

    while (!ready.empty()) {
        if (cancelled(ctx)) return cancel_status(ctx);
        std::vector<int> cur;
        cur.swap(ready);
        std::vector<int> leaves, splits;
        for (int k : cur) {
            const Node &n = nodes[k];
            const int64_t rows = n.r_bot - n.r_top, w = n.J - n.L + 1;
            if (rows <= 1 || (rows * w <= leaf_cells && w <= kLeafMaxWidth))
                leaves.push_back(k);
            else
                splits.push_back(k);
        }

        // ---------------------------------------------------------------- splits
        if (!splits.empty()) {
            const int ns = (int)splits.size();
            // strip height from the rows of every pass of this level (forward
            // and backward halves together), but no taller than the mean pass
            // so that many short passes are not padded to tall strips
            int64_t allrows = 1;
            for (int k : splits) allrows += nodes[k].r_bot - nodes[k].r_top;
            StripShape shape = tuned_shape(ctx, allrows);
            const int64_t mean_pass = allrows / (2 * (int64_t)splits.size()) + 1;
            while (shape.R > 4 && 64 * shape.R > mean_pass && ctx->opt.rows == 0)
                shape.R = shape.R > 16 ? 16 : shape.R / 2;
            const int R = shape.R;
            std::vector<GatherDesc> gd;
            std::vector<BorderInit> bi;
            std::vector<StripProblem> fwdp, bwdp;
            std::vector<Border *> fwd_out(ns), bwd_out(ns);
            std::vector<int64_t> mid(ns);
            // sizes: codes scratch (temporary) and borders
            int64_t codes_bytes = 0, bwd_entries = 0;
            for (int i = 0; i < ns; ++i) {
                const Node &n = nodes[splits[i]];
                const int64_t w = n.J - n.L + 1;
                mid[i] = (n.r_top + n.r_bot) / 2;
                const int64_t P = mid[i] - n.r_top, Pb = n.r_bot - mid[i] - 1;
                codes_bytes += rows_padded(P, R) + rows_padded(std::max<int64_t>(Pb, 1), R) + 2 * cols_padded(w);
                bwd_entries += cols_padded(w);
            }
            if ((s = ensure(ctx, ctx->tb_codes_q, (size_t)codes_bytes + 256, "traceback codes")) != SWH_OK) return s;
            if ((s = ensure(ctx, ctx->tb_bwd, (size_t)bwd_entries * sizeof(Border) + 256, "backward borders")) !=
                SWH_OK)
                return s;
            uint8_t *cp = (uint8_t *)ctx->tb_codes_q.p;
            Border *bp = (Border *)ctx->tb_bwd.p;
            for (int i = 0; i < ns; ++i) {
                const Node &n = nodes[splits[i]];
                const int64_t w = n.J - n.L + 1, r = mid[i];
                const int64_t P = r - n.r_top, Pb = n.r_bot - r - 1;
                // forward pass rows A_{r_top+1}..A_r, columns L..J
                uint8_t *fq = cp; cp += rows_padded(P, R);
                uint8_t *ft = cp; cp += cols_padded(w);
                uint8_t *bq = cp; cp += rows_padded(std::max<int64_t>(Pb, 1), R);
                uint8_t *bt = cp; cp += cols_padded(w);
                gd.push_back(GatherDesc{n.A, fq, n.r_top, P, rows_padded(P, R), 1, 0});
                gd.push_back(GatherDesc{n.bpad, ft, n.L, w, cols_padded(w), 1, 0});
                // backward pass rows A_{r_bot}..A_{r+2}, columns J..L reversed, pad first
                gd.push_back(GatherDesc{n.A, bq, n.r_bot - 1, Pb, rows_padded(std::max<int64_t>(Pb, 1), R), -1, 0});
                gd.push_back(GatherDesc{n.bpad, bt, n.J, w - 1, cols_padded(w), -1, 1});
                Border *fo = (Border *)arena.get(sizeof(Border) * (size_t)cols_padded(w), ctx->held, ctx->opt.mem_cap);
                if (!fo) return fail(ctx, SWH_E_NOMEM, "traceback frontier arena");
                fwd_out[i] = fo;
                bwd_out[i] = bp;
                bi.push_back(BorderInit{fo, n.front + (n.L - n.front_L), w, cols_padded(w), 0, 0});
                bi.push_back(BorderInit{bp, nullptr, w, cols_padded(w), n.end_state == 0 ? 1 : 2, 0});
                bp += cols_padded(w);
                fwdp.push_back(StripProblem{fq, P, ft, w, fo});
                if (Pb > 0) bwdp.push_back(StripProblem{bq, Pb, bt, w, bwd_out[i]});
                ts.cells += (double)(P + std::max<int64_t>(Pb, 0)) * (double)w;
            }
            if ((s = upload(ctx, ctx->tb_misc, gd, st, "gather table")) != SWH_OK) return s;
            if ((e = launch_gather((const GatherDesc *)ctx->tb_misc.p, (int32_t)gd.size(), pad, st)) != hipSuccess)
                return hip_fail(ctx, e, "gather launch");
            if ((s = upload(ctx, ctx->tb_leaf, bi, st, "border table")) != SWH_OK) return s;
            if ((e = launch_border_init((const BorderInit *)ctx->tb_leaf.p, (int32_t)bi.size(), sc.o, sc.e, st)) !=
                hipSuccess)
                return hip_fail(ctx, e, "border init launch");
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(ctx, e, "traceback setup");
            // forward and backward passes are independent problems: one launch
            // for both keeps the strip chains' ramp and tail to one per level
            fwdp.insert(fwdp.end(), bwdp.begin(), bwdp.end());
            if ((s = run_strips(ctx, fwdp, sc, R, false, st, nullptr, nullptr, shape.waves)) != SWH_OK) return s;

            std::vector<CrossDesc> cd(ns);
            for (int i = 0; i < ns; ++i) {
                const Node &n = nodes[splits[i]];
                cd[i] = CrossDesc{fwd_out[i], bwd_out[i], n.bpad, n.A + mid[i], n.L, n.J, n.V, 0};
            }
            if ((s = upload(ctx, ctx->tb_misc, cd, st, "cross table")) != SWH_OK) return s;
            if ((s = ensure(ctx, ctx->tb_front, sizeof(CrossOut) * (size_t)ns, "cross results")) != SWH_OK) return s;
            if ((e = launch_cross((const CrossDesc *)ctx->tb_misc.p, ns, (const int8_t *)ctx->mat.p, sc.asize, sc.o,
                                  sc.e, (CrossOut *)ctx->tb_front.p, st)) != hipSuccess)
                return hip_fail(ctx, e, "cross launch");
            std::vector<CrossOut> co(ns);
            if ((e = hipMemcpyAsync(co.data(), ctx->tb_front.p, sizeof(CrossOut) * ns, hipMemcpyDeviceToHost, st)) !=
                    hipSuccess ||
                (e = hipStreamSynchronize(st)) != hipSuccess)
                return hip_fail(ctx, e, "cross results");

            for (int i = 0; i < ns; ++i) {
                const int k = splits[i];
                if (co[i].count <= 0 || co[i].cmin < nodes[k].L) {
                    ts.inconsistent = true;
                    return fail(ctx, SWH_E_DEVICE, "traceback: no optimal crossing found (internal error)");
                }
                Node bot;
                bot.pair = nodes[k].pair;
                bot.A = nodes[k].A;
                bot.bpad = nodes[k].bpad;
                bot.r_top = mid[i];
                bot.r_bot = nodes[k].r_bot;
                bot.L = co[i].cmin;
                bot.J = nodes[k].J;
                bot.front = fwd_out[i];
                bot.front_L = nodes[k].L;
                bot.end_state = nodes[k].end_state;
                bot.V = nodes[k].V;
                bot.parent = k;
                bot.is_top_child = false;
                bot.ready = true;
                Node top;
                top.pair = nodes[k].pair;
                top.A = nodes[k].A;
                top.bpad = nodes[k].bpad;
                top.r_top = nodes[k].r_top;
                top.r_bot = mid[i];
                top.L = nodes[k].L;
                top.J = -1;
                top.front = nodes[k].front;
                top.front_L = nodes[k].front_L;
                top.parent = k;
                top.is_top_child = true;
                if (co[i].count == 1) {
                    top.J = co[i].exit_col;
                    top.end_state = co[i].exit_state;
                    top.V = co[i].exit_val;
                    top.ready = true;
                }
                nodes.push_back(bot);
                nodes[k].bottom = (int)nodes.size() - 1;
                ready.push_back(nodes[k].bottom);
                nodes.push_back(top);
                nodes[k].top = (int)nodes.size() - 1;
                if (nodes.back().ready) ready.push_back(nodes[k].top);
                ++ts.splits;
            }
        }

        // ---------------------------------------------------------------- leaves
        for (size_t c0 = 0; c0 < leaves.size();) {
            // one launch: leaves whose global tie flags fit kLeafFlagBytes
            size_t c1 = c0;
            int64_t ops_total = 0, gflag_bytes = 0;
            size_t lds = 1024;
            while (c1 < leaves.size()) {
                const Node &n = nodes[leaves[c1]];
                const int64_t P = n.r_bot - n.r_top, w = n.J - n.L + 1;
                if (w > kLeafMaxWidth)
                    return fail(ctx, SWH_E_RANGE, "traceback: gap wider than " + std::to_string(kLeafMaxWidth) +
                                                      " columns in a subproblem of one row");
                const bool in_lds = P * w <= kLeafCells;
                const int64_t gb = in_lds ? 0 : (leaf_flag_bytes(P, w) + 255) / 256 * 256;
                if (c1 > c0 && gflag_bytes + gb > kLeafFlagBytes) break;
                gflag_bytes += gb;
                ops_total += P + w + 1;
                if (in_lds) lds = std::max(lds, (size_t)(1024 + 8 * w + P * w));
                ++c1;
            }
            // small leaves (flags in LDS) first, then the large ones
            std::stable_partition(leaves.begin() + c0, leaves.begin() + c1, [&](int k) {
                const Node &n = nodes[k];
                return (n.r_bot - n.r_top) * (n.J - n.L + 1) <= kLeafCells;
            });
            const int nl = (int)(c1 - c0);
            int nsmall = 0;
            int32_t max_w = 1;
            std::vector<LeafDesc> ld(nl);
            if ((s = ensure(ctx, ctx->tb_fwd, (size_t)ops_total + 256, "traceback ops")) != SWH_OK) return s;
            if (gflag_bytes && (s = ensure(ctx, ctx->tb_flags, (size_t)gflag_bytes, "traceback flags")) != SWH_OK)
                return s;
            uint8_t *gfl = (uint8_t *)ctx->tb_flags.p;
            char *op = (char *)ctx->tb_fwd.p;
            std::vector<int64_t> op_off(nl);
            int64_t off = 0;
            for (int i = 0; i < nl; ++i) {
                const Node &n = nodes[leaves[c0 + i]];
                const int64_t P = n.r_bot - n.r_top, w = n.J - n.L + 1;
                LeafDesc d;
                d.arows = n.A + n.r_top;
                d.bcols = n.bpad + n.L;
                d.front = n.front + (n.L - n.front_L);
                d.gflags = nullptr;
                if (P * w > kLeafCells) {
                    d.gflags = gfl;
                    gfl += (leaf_flag_bytes(P, w) + 255) / 256 * 256;
                    max_w = std::max<int32_t>(max_w, (int32_t)w);
                } else {
                    ++nsmall;
                }
                d.ops = op + off;
                d.P = (int32_t)P;
                d.w = (int32_t)w;
                d.end_state = n.end_state;
                d.ops_cap = (int32_t)(P + w + 1);
                d.V = n.V;
                d.pad_ = 0;
                op_off[i] = off;
                off += P + w + 1;
                ld[i] = d;
                ts.cells += (double)P * (double)w;
            }
            if ((s = upload(ctx, ctx->tb_misc, ld, st, "leaf table")) != SWH_OK) return s;
            if ((s = ensure(ctx, ctx->tb_front, sizeof(LeafOut) * (size_t)nl, "leaf results")) != SWH_OK) return s;
            const LeafDesc *ldd = (const LeafDesc *)ctx->tb_misc.p;
            LeafOut *lod = (LeafOut *)ctx->tb_front.p;
            if ((e = launch_leaf(ldd, nsmall, (const int8_t *)ctx->mat.p, sc.asize, sc.o, sc.e, lds, lod, st)) !=
                    hipSuccess ||
                (e = launch_leaf_big(ldd + nsmall, nl - nsmall, (const int8_t *)ctx->mat.p, sc.asize, sc.o, sc.e,
                                     max_w, lod + nsmall, st)) != hipSuccess)
                return hip_fail(ctx, e, "leaf launch");
            std::vector<LeafOut> lo(nl);
            const size_t base = ops_used;
            if (!ops_room((size_t)ops_total)) return fail(ctx, SWH_E_NOMEM, "pinned host memory for traceback ops");
            ops_used += (size_t)ops_total;
            if ((e = hipMemcpyAsync(lo.data(), ctx->tb_front.p, sizeof(LeafOut) * nl, hipMemcpyDeviceToHost, st)) !=
                    hipSuccess ||
                (e = hipMemcpyAsync(ctx->tb_ops_host + base, op, (size_t)ops_total, hipMemcpyDeviceToHost, st)) !=
                    hipSuccess ||
                (e = hipStreamSynchronize(st)) != hipSuccess)
                return hip_fail(ctx, e, "leaf results");
            for (int i = 0; i < nl; ++i) {
                Node &n = nodes[leaves[c0 + i]];
                if (lo[i].err) {
                    ts.inconsistent = true;
                    return fail(ctx, SWH_E_DEVICE, "traceback walk left its subproblem (internal error)");
                }
                n.leaf = true;
                n.ops_off = (int64_t)base + op_off[i];
                n.nops = lo[i].nops;
                n.exit_known = true;
                n.exit_col = n.L + lo[i].exit_col;
                n.exit_state = lo[i].exit_state;
                n.exit_val = lo[i].exit_val;
                ++ts.leaves;
            }
            for (int i = 0; i < nl; ++i) propagate(leaves[c0 + i]);
            c0 = c1;
        }
    }

    // every node must be resolved; assemble the ops, walking back from the end
    for (const Node &n : nodes)
        if (!n.leaf && (n.bottom < 0 || n.top < 0 || !nodes[n.top].ready)) {
            ts.inconsistent = true;
            return fail(ctx, SWH_E_DEVICE, "traceback left a subproblem unresolved (internal error)");
        }
    // the node where a band's walk leaves its top row
    auto band_exit = [&](int k) -> const Node & {
        while (!nodes[k].leaf) k = nodes[k].top;
        return nodes[k];
    };
    // checks first (serial, cheap): every seeded band leaves through its seed
    // node (column L, state H for a diagonal entry, F for a vertical one), and
    // the top band reaches row 0
    for (int pr = 0; pr < npairs; ++pr) {
        const std::vector<int> &rt = roots[(size_t)pr];
        for (size_t b = 1; b < rt.size(); ++b) {
            const Node &x = band_exit(rt[b]);
            const bool seed_f = in[pr].bands[b].seed_h == kNeg;
            if (x.exit_col != nodes[rt[b]].L || x.exit_state != (seed_f ? 1 : 0)) {
                ts.inconsistent = true;
                return fail(ctx, SWH_E_DEVICE, "traceback: band left through another node (internal error)");
            }
        }
        if (band_exit(rt[0]).exit_col < 0) {
            ts.inconsistent = true;
            return fail(ctx, SWH_E_DEVICE, "traceback: no exit on row 0 (internal error)");
        }
    }
    // then the CIGARs, pairs spread over host threads: the leaves' ops
    // (backward order) bottom band first, each subproblem's bottom half before
    // its top half, then run-length encoded in forward order
    auto assemble = [&](int pr) {
        std::string back;
        const std::vector<int> &rt = roots[(size_t)pr];
        for (size_t b = rt.size(); b-- > 0;) {
            std::vector<int> stack{rt[b]};
            while (!stack.empty()) {
                const int k = stack.back();
                stack.pop_back();
                const Node &n = nodes[k];
                if (n.leaf) {
                    back.append(ctx->tb_ops_host + n.ops_off, (size_t)n.nops);
                } else {
                    stack.push_back(n.top);
                    stack.push_back(n.bottom);
                }
            }
        }
        back.append((size_t)band_exit(rt[0]).exit_col, 'D');   // leading target residues against a gap
        std::string &cigar = cigars[(size_t)pr];
        char num[24];
        int64_t q = (int64_t)back.size() - 1;
        while (q >= 0) {
            const char opc = back[(size_t)q];
            const int64_t q0 = q;
            while (q >= 0 && back[(size_t)q] == opc) --q;
            const auto r = std::to_chars(num, num + sizeof(num), q0 - q);
            cigar.append(num, r.ptr);
            cigar += opc;
        }
    };
    const int nthreads = (int)std::min<int64_t>(npairs / 64 + 1, std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
    if (nthreads <= 1) {
        for (int pr = 0; pr < npairs; ++pr) assemble(pr);
    } else {
        std::atomic<int> next{0};
        std::vector<std::thread> pool;
        for (int t = 0; t < nthreads; ++t)
            pool.emplace_back([&] {
                for (int pr; (pr = next.fetch_add(16)) < npairs;)
                    for (int k = pr; k < std::min(pr + 16, npairs); ++k) assemble(k);
            });
        for (std::thread &t : pool) t.join();
    }
    ts.ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return SWH_OK;
}

swh_status traceback(swh_ctx *ctx, const uint8_t *A, int64_t p, const uint8_t *B, int64_t q, const Scoring &sc,
                     int32_t S, hipStream_t st, std::string &cigar, TracebackStats &ts)
{
    std::vector<std::string> out;
    swh_status s = traceback_batch(ctx, {TbInput{A, p, B, q, S}}, sc, st, out, ts);
    if (s == SWH_OK) cigar.swap(out[0]);
    return s;
}

}  // namespace swh
