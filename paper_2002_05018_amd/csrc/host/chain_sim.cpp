// Host simulation of the work-queue form of the two K solve sweeps.
//
// Independent of how the item lists were built, every item's accesses are
// read again from the task data (the update task's target, the sources of
// its products, the diagonal solve it carries) and the sequential order is
// taken from the level-by-level schedule (the update tasks of k_fwd / k_bwd,
// step after step).  Every diagonal solve of the sweep must run exactly once
// (before the queue or carried by the item that writes its input tile last),
// and a tile may be read as a source only after its solve.  Workers then
// take items (times column blocks) from one
// counter and wait on the write counts exactly as the kernel does, under
// pseudo-random interleavings of take / start / finish.  An item checks, when
// it starts and again when it finishes, that every tile it touches holds
// exactly the writes the sequential order gives it at that point (for its
// column block); finishing writes its tile and raises the tile's count.  A
// state in which no worker can move while items remain is a stalled queue.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <string>
#include <vector>

#include "race.hpp"

namespace d3m {

namespace {

struct Rng {
    uint64_t s;
    uint64_t next() {
        s ^= s << 13;
        s ^= s >> 7;
        s ^= s << 17;
        return s;
    }
};

struct ItemAccess {
    std::vector<int64_t> tiles;  // every tile the item reads or writes
    int64_t wtile = -1;
    std::vector<int32_t> expect;  // chain writes of each tile before the item, sequential order
};

void note(std::string &rep, int64_t &count, const std::string &msg) {
    if (count < 8) rep += msg + "\n";
    ++count;
}

int64_t simulate(const Plan &pl, int sw, int nyb, int workers, uint64_t seed, bool drop_wait, std::string &rep) {
    const std::vector<SolveStep> &steps = sw ? pl.k_bwd : pl.k_fwd;
    const std::vector<ChainItem> &items = pl.kc_items[sw];
    const std::vector<ChainWait> &waits = pl.kc_waits[sw];
    const int64_t nt = pl.v_tiles_k;
    int64_t bad = 0;
    const std::string tag = std::string(sw ? "backward" : "forward") + " sweep: ";
    // the sequential order: every step's update tasks, in order
    std::vector<int64_t> order;
    for (const SolveStep &st : steps)
        for (int64_t u = st.up0; u < st.up0 + st.nup; ++u) order.push_back(u);
    if (order.size() != items.size()) {
        note(rep, bad, tag + "item count differs from the update tasks of the sweep");
        return bad;
    }
    // the sweep's diagonal solves, by input tile (x forward, acc backward)
    const bool bwd = sw == 1;
    std::vector<int64_t> diag_of(nt, -1);
    auto add_diag = [&](const VDiagTask &d) {
        const int64_t t = (bwd ? d.acc : d.x) & ENC_MASK;
        if (t < 0 || t >= nt || diag_of[t] >= 0) {
            note(rep, bad, tag + "diagonal solve on a bad or repeated tile");
            return;
        }
        diag_of[t] = 1;
    };
    for (const SolveStep &st : steps) {
        for (int64_t i = st.dg0; i < st.dg0 + st.ndg; ++i) add_diag(pl.vdiag[i]);
        for (int64_t u = st.up0; u < st.up0 + st.nup; ++u)
            if (pl.vfuse[u] >= 0) add_diag(pl.vdiag[pl.vfuse[u]]);
    }
    if (bad) return bad;
    // where each solve runs: -1 before the queue, else its item
    std::vector<int64_t> solved_at(nt, INT64_MAX);
    std::vector<int64_t> last_write(nt, -1);
    for (size_t i = 0; i < items.size(); ++i) last_write[pl.vupd[order[i]].out & ENC_MASK] = (int64_t)i;
    auto run_diag = [&](const VDiagTask &d, int64_t where) {
        const int64_t t = (bwd ? d.acc : d.x) & ENC_MASK;
        if (t < 0 || t >= nt || diag_of[t] != 1 || solved_at[t] != INT64_MAX) {
            note(rep, bad, tag + "a diagonal solve that is not the sweep's, or runs twice");
            return (int64_t)-1;
        }
        solved_at[t] = where;
        if (where != last_write[t])
            note(rep, bad, tag + "the solve of tile " + std::to_string(t) + " is not run right after its last write");
        return t;
    };
    for (const VDiagTask &d : pl.kc_pre[sw]) run_diag(d, -1);
    for (size_t i = 0; i < items.size(); ++i)
        if (items[i].fz >= 0) {
            if (items[i].fz >= (int32_t)pl.vdiag.size()) {
                note(rep, bad, tag + "carried solve index out of range");
                return bad;
            }
            if (run_diag(pl.vdiag[items[i].fz], (int64_t)i) != (pl.vupd[order[i]].out & ENC_MASK))
                note(rep, bad, tag + "item " + std::to_string(i) + " carries the solve of another tile");
        }
    for (int64_t t = 0; t < nt; ++t)
        if (diag_of[t] == 1 && solved_at[t] == INT64_MAX) note(rep, bad, tag + "a diagonal solve never runs");
    if (bad) return bad;
    std::vector<ItemAccess> acc(items.size());
    std::vector<int32_t> seqw(nt, 0);
    for (size_t i = 0; i < items.size(); ++i) {
        if (items[i].idx != order[i]) {
            note(rep, bad, tag + "item " + std::to_string(i) + " is not the sweep's next update task");
            return bad;
        }
        const VUpdTask &tk = pl.vupd[order[i]];
        ItemAccess &a = acc[i];
        a.wtile = tk.out & ENC_MASK;
        a.tiles.push_back(a.wtile);
        for (int32_t p = tk.p0; p < tk.p0 + tk.np; ++p) {
            const int64_t t = pl.vpairs[p].src & ENC_MASK;
            if (t < 0 || t >= nt || solved_at[t] >= (int64_t)i)
                note(rep, bad, tag + "item " + std::to_string(i) + " reads tile " + std::to_string(t) +
                                   " before its diagonal solve");
            a.tiles.push_back(t);
        }
        if (items[i].fz >= 0) {
            const VDiagTask &d = pl.vdiag[items[i].fz];
            for (int64_t e : {d.x, d.y, d.v, d.acc})
                if (e >= 0) a.tiles.push_back(e & ENC_MASK);
        }
        std::sort(a.tiles.begin(), a.tiles.end());
        a.tiles.erase(std::unique(a.tiles.begin(), a.tiles.end()), a.tiles.end());
        for (int64_t t : a.tiles) {
            if (t < 0 || t >= nt) {
                note(rep, bad, tag + "tile index out of range");
                return bad;
            }
            a.expect.push_back(seqw[t]);
        }
        if (items[i].sig != a.wtile) note(rep, bad, tag + "item " + std::to_string(i) + " signals another tile");
        ++seqw[a.wtile];
    }
    if (bad) return bad;

    // concurrent execution
    const int64_t total = (int64_t)items.size() * nyb;
    std::vector<int32_t> ver((size_t)nt * nyb, 0);  // writes applied, per tile and column block
    std::vector<uint32_t> cnt(nt, 0);               // the kernel's counters (all column blocks)
    enum { IDLE, WAITING, RUNNING, DONE };
    struct Worker { int st = IDLE; int64_t it = -1; };
    std::vector<Worker> w(workers);
    int64_t head = 0, finished = 0;
    Rng rng{seed * 0x9E3779B97F4A7C15ull + 12345};
    auto check_view = [&](int64_t it, const char *when) {
        const int64_t k = it / nyb;
        const int cb = (int)(it % nyb);
        const ItemAccess &a = acc[k];
        for (size_t j = 0; j < a.tiles.size(); ++j)
            if (ver[(size_t)a.tiles[j] * nyb + cb] != a.expect[j]) {
                note(rep, bad, tag + "item " + std::to_string(k) + " (column block " + std::to_string(cb) + ") " +
                                   when + " with tile " + std::to_string(a.tiles[j]) + " at " +
                                   std::to_string(ver[(size_t)a.tiles[j] * nyb + cb]) + " writes, expected " +
                                   std::to_string(a.expect[j]));
                return;
            }
    };
    auto ready = [&](int64_t it) {
        const ChainItem &ci = items[it / nyb];
        for (int32_t q = drop_wait && ci.nw > 0 ? 1 : 0; q < ci.nw; ++q) {
            const ChainWait &cw = waits[ci.w0 + q];
            if (cw.tile < 0 || cw.tile >= nt) return false;
            if (cnt[cw.tile] < (uint32_t)cw.writes * (uint32_t)nyb) return false;
        }
        return true;
    };
    while (finished < total) {
        // one enabled action of a random worker, else of the next ones
        const int start = (int)(rng.next() % (uint64_t)workers);
        bool moved = false;
        for (int o = 0; o < workers && !moved; ++o) {
            Worker &x = w[(start + o) % workers];
            if (x.st == IDLE) {
                if (head < total) {
                    x.it = head++;
                    x.st = WAITING;
                    moved = true;
                }
            } else if (x.st == WAITING) {
                if (ready(x.it)) {
                    check_view(x.it, "starts");
                    x.st = RUNNING;
                    moved = true;
                }
            } else if (x.st == RUNNING) {
                // finishing is one of the choices only half the time, so
                // items overlap in varied ways
                if ((rng.next() & 1) || o + 1 == workers) {
                    check_view(x.it, "finishes");
                    const int64_t k = x.it / nyb;
                    const int cb = (int)(x.it % nyb);
                    ++ver[(size_t)acc[k].wtile * nyb + cb];
                    ++cnt[acc[k].wtile];
                    ++finished;
                    x.st = IDLE;
                    moved = true;
                }
            }
        }
        if (!moved) {
            // a running worker can always finish: only waiting ones remain
            bool any_running = false;
            for (auto &x : w) any_running |= x.st == RUNNING;
            if (any_running) continue;
            note(rep, bad, tag + "the queue stalls with " + std::to_string(total - finished) + " items left");
            break;
        }
        if (bad > 64) break;
    }
    return bad;
}

}  // namespace

int64_t check_solve_chain(const Plan &pl, bool drop_wait, std::string &report) {
    if (!pl.chain_ok) {
        report = "the plan has no work-queue form of the K sweeps: " + pl.chain_why;
        return -1;
    }
    int64_t bad = 0;
    uint64_t seed = 1;
    for (int sw = 0; sw < 2; ++sw)
        for (int nyb : {1, 2})
            for (int workers : {1, 7, 64, 512}) {
                bad += simulate(pl, sw, nyb, workers, seed++, drop_wait, report);
                if (bad > 64) return bad;
            }
    return bad;
}

}  // namespace d3m
