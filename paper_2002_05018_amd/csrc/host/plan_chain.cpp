// The two sweeps over the factor of -K (steps 6-7, the lambda solve) as
// dependency-counted item lists, so that each sweep runs as one launch.
//
// The level-by-level schedule runs one diagonal launch and one update launch
// per elimination-tree level (294 levels per direction at 48^3, most of them
// small).  Here the same update tasks, in the same sequential order, become
// items of a work queue.  Every written vector tile (index into the K vector
// arrays; the x, y, v and accumulator arrays of one tile index are one
// resource) counts its completed writes.  An item waits until each tile it
// reads or writes has received all the writes that precede the item in the
// sequential order, and then adds one to the count of the tile it wrote.
// Writers of a tile therefore complete in the sequential order, and every
// read sees the writes the level-by-level schedule gives it.
//
// Diagonal solves: the solve of a one-tile unit needs its input tile (x going
// forward, the accumulator going back) complete, and its outputs are read
// only by later levels.  So it is carried by the item that writes its input
// tile last (no barrier separates levels here, so that item may belong to an
// earlier level than the launch schedule's fused update), and the solves
// whose input no update writes (the leaves going forward, the roots going
// back) form a list of their own that runs as one launch before the queue.
// Every product and sum is formed as in the level-by-level schedule, so both
// give the same bits.
//
// A later write of a tile that an earlier item read only as a source would
// need a wait for that reader; no such pair occurs (a tile is a source only
// after its diagonal solve, which follows its last write), and the builder
// rejects a plan where one would, or where a unit spans several tiles.
#include <algorithm>
#include <climits>
#include <stdexcept>
#include <string>

#include "plan.hpp"

namespace d3m {

namespace {

struct ChainBuilder {
    Plan &pl;
    std::string why;

    explicit ChainBuilder(Plan &p) : pl(p) {}

    i64 k_tile(int64_t e) const {
        if (e < 0) return -1;
        const int a = (int)(e >> ENC_SHIFT);
        if (a < V_KX || a > V_KACC) throw std::logic_error("solve chain: vector tile outside the K arrays");
        const i64 t = e & ENC_MASK;
        if (t < 0 || t >= pl.v_tiles_k) throw std::logic_error("solve chain: vector tile index out of range");
        return t;
    }

    // tile index of a one-tile diagonal solve (x, y, v and acc share it); -1
    // and a reason where the solve does not fit the item form
    i64 diag_tile(const VDiagTask &d) {
        if (d.t != 1) {
            why = "diagonal blocks of several tiles (whole-block pivot units)";
            return -1;
        }
        const i64 tx = k_tile(d.x), ty = k_tile(d.y), tv = k_tile(d.v), ta = k_tile(d.acc);
        if (tx != tv || (ty >= 0 && ty != tx) || (ta >= 0 && ta != tx)) {
            why = "a diagonal solve spans different tile indices";
            return -1;
        }
        return tx;
    }

    bool sweep(const std::vector<SolveStep> &steps, std::vector<ChainItem> &items, std::vector<ChainWait> &waits,
               std::vector<VDiagTask> &pre) {
        const i64 nt = pl.v_tiles_k;
        // the update tasks in order, and every diagonal solve of the sweep
        // (the launch schedule's unfused ones and those its updates carry)
        std::vector<i64> order, diags;
        for (const SolveStep &st : steps) {
            for (i64 i = st.dg0; i < st.dg0 + st.ndg; ++i) diags.push_back(i);
            for (i64 u = st.up0; u < st.up0 + st.nup; ++u) {
                if (st.up_mode == 1) {
                    why = "an update that overwrites its target";
                    return false;
                }
                order.push_back(u);
                if (pl.vfuse[u] >= 0) diags.push_back(pl.vfuse[u]);
            }
        }
        if ((i64)order.size() > INT32_MAX || (i64)pl.vdiag.size() > INT32_MAX)
            throw std::length_error("solve chain: task index beyond 32 bits");
        std::vector<i64> last(nt, -1);  // last item writing each tile
        for (size_t k = 0; k < order.size(); ++k) last[k_tile(pl.vupd[order[k]].out)] = (i64)k;
        std::vector<int64_t> carry(order.size(), -1);
        std::vector<char> has_diag(nt, 0);
        for (i64 d : diags) {
            const i64 t = diag_tile(pl.vdiag[d]);
            if (t < 0) return false;
            if (has_diag[t]) {
                why = "two diagonal solves on one tile in a sweep";
                return false;
            }
            has_diag[t] = 1;
            if (last[t] >= 0) carry[last[t]] = d;
            else pre.push_back(pl.vdiag[d]);
        }
        std::vector<int32_t> writes(nt, 0);  // item writes so far (sequential order)
        std::vector<char> read_open(nt, 0);  // read as a source since its last write
        std::vector<i64> reads;
        for (size_t k = 0; k < order.size(); ++k) {
            const VUpdTask &tk = pl.vupd[order[k]];
            const i64 w = k_tile(tk.out);
            reads.clear();
            reads.push_back(w);  // read-modify-write of the target
            for (int32_t p = tk.p0; p < tk.p0 + tk.np; ++p) reads.push_back(k_tile(pl.vpairs[p].src));
            std::sort(reads.begin(), reads.end());
            reads.erase(std::unique(reads.begin(), reads.end()), reads.end());
            if (waits.size() + reads.size() > (size_t)INT32_MAX)
                throw std::length_error("solve chain: wait list beyond 32 bits");
            ChainItem it{};
            it.idx = (int32_t)order[k];
            it.w0 = (int32_t)waits.size();
            for (i64 t : reads)
                if (writes[t] > 0) waits.push_back({(int32_t)t, writes[t]});
            it.nw = (int32_t)waits.size() - it.w0;
            it.sig = (int32_t)w;
            it.fz = (int32_t)carry[k];
            items.push_back(it);
            if (read_open[w] && why.empty())
                why = "a K vector tile is written after another item read it (tile " + std::to_string(w) + ")";
            for (i64 t : reads)
                if (t != w) read_open[t] = 1;
            ++writes[w];
        }
        return why.empty();
    }
};

}  // namespace

void build_solve_chain(Plan &pl) {
    for (int s = 0; s < 2; ++s) {
        pl.kc_items[s].clear();
        pl.kc_waits[s].clear();
        pl.kc_pre[s].clear();
    }
    pl.chain_ok = false;
    pl.chain_why.clear();
    if (pl.v_tiles_k <= 0 || pl.v_tiles_k > INT32_MAX) {
        pl.chain_why = "no K vector tiles";
        return;
    }
    ChainBuilder b(pl);
    if (!b.sweep(pl.k_fwd, pl.kc_items[0], pl.kc_waits[0], pl.kc_pre[0]) ||
        !b.sweep(pl.k_bwd, pl.kc_items[1], pl.kc_waits[1], pl.kc_pre[1])) {
        pl.chain_why = b.why.empty() ? "unsupported task" : b.why;
        for (int s = 0; s < 2; ++s) {
            pl.kc_items[s].clear();
            pl.kc_waits[s].clear();
            pl.kc_pre[s].clear();
        }
        return;
    }
    pl.chain_ok = true;
}

}  // namespace d3m
