// Static race check of the factorisation schedule.
//
// Replays the launch sequence of the factor sweeps (the pivot, panel,
// scaling and update launches of every step, on the caller's stream and the
// side streams, with the event records and waits of the look-ahead and of
// the block-column tracking) without a GPU: every launch gets a vector
// clock over the streams, and every tile it reads or writes (decoded from
// the task lists: working tiles, panel products, factor tiles, TT tiles and
// the rows of the pivot data) is checked against the earlier accesses of
// that tile.  Two accesses race when at least one writes and neither launch
// is ordered before the other; inside one launch, two work-groups race when
// they write the same tile or one reads a tile another writes.
#include <algorithm>
#include <array>
#include <cstdint>
#include <string>
#include <unordered_map>

#include "plan.hpp"
#include "race.hpp"

namespace d3m {

namespace {

constexpr int kStreams = 3;  // 0 the caller's stream, 1 and 2 the side streams
using VC = std::array<int64_t, kStreams>;

struct Sim {
    VC stream[kStreams] = {};
    std::vector<VC> launch_vc;
    std::vector<int> launch_stream;
    std::vector<std::string> launch_what;
    struct Hist {
        int64_t write = -1;
        std::vector<int64_t> reads;
    };
    std::unordered_map<int64_t, Hist> tiles;
    int64_t races = 0;
    std::string report;

    bool before(int64_t a, int64_t b) const {  // launch a happens before launch b
        const int s = launch_stream[a];
        return launch_vc[a][s] <= launch_vc[b][s];
    }
    void note(const std::string &m) {
        ++races;
        if (report.size() < 4000) report += m + "\n";
    }
    VC record(int s) const { return stream[s]; }
    void wait(int s, const VC &e) {
        for (int q = 0; q < kStreams; ++q) stream[s][q] = std::max(stream[s][q], e[q]);
    }
    // one launch on stream s; acc: per task, the tiles it reads and writes
    void launch(int s, const std::string &what,
                const std::vector<std::pair<std::vector<int64_t>, std::vector<int64_t>>> &acc) {
        stream[s][s] += 1;
        const int64_t id = (int64_t)launch_vc.size();
        launch_vc.push_back(stream[s]);
        launch_stream.push_back(s);
        launch_what.push_back(what);
        // inside the launch: one writer per tile, no other task reading it
        std::unordered_map<int64_t, int64_t> writer;
        for (size_t t = 0; t < acc.size(); ++t)
            for (int64_t w : acc[t].second) {
                auto it = writer.find(w);
                if (it != writer.end() && it->second != (int64_t)t)
                    note(what + ": tile " + std::to_string(w) + " written by two work-groups");
                writer[w] = (int64_t)t;
            }
        for (size_t t = 0; t < acc.size(); ++t)
            for (int64_t r : acc[t].first) {
                auto it = writer.find(r);
                if (it != writer.end() && it->second != (int64_t)t)
                    note(what + ": tile " + std::to_string(r) + " read by one work-group, written by another");
            }
        // against earlier launches
        std::unordered_map<int64_t, char> mine;  // 1 read, 2 written
        for (const auto &a : acc) {
            for (int64_t r : a.first) mine[r] |= 1;
            for (int64_t w : a.second) mine[w] |= 2;
        }
        for (const auto &kv : mine) {
            Hist &h = tiles[kv.first];
            if (h.write >= 0 && !before(h.write, id))
                note(what + " vs " + launch_what[h.write] + ": tile " + std::to_string(kv.first) +
                     " written by the earlier launch, unordered");
            if (kv.second & 2) {
                for (int64_t r : h.reads)
                    if (r != id && !before(r, id))
                        note(what + " vs " + launch_what[r] + ": tile " + std::to_string(kv.first) +
                             " read by the earlier launch, unordered write");
                h.write = id;
                h.reads.clear();
            } else {
                h.reads.push_back(id);
            }
        }
    }
};

inline int64_t tile_id(int64_t e) {  // (array, tile) of an encoded tile offset
    const int64_t arr = e >> ENC_SHIFT, off = e & ENC_MASK;
    return (arr << 40) | (off / TILE_ELEMS);
}
inline int64_t drow_id(int64_t row) { return (int64_t(60) << 40) | (row / TILE); }

using Acc = std::vector<std::pair<std::vector<int64_t>, std::vector<int64_t>>>;

void add_pairs(const Plan &pl, int32_t p0, int32_t np, std::vector<int64_t> &rd) {
    for (int32_t q = p0; q < p0 + np; ++q) {
        rd.push_back(tile_id(pl.pairs[q].a));
        rd.push_back(tile_id(pl.pairs[q].b));
    }
}

Acc bk_access(const Plan &pl, int64_t b0, int64_t n) {
    Acc acc;
    for (int64_t x = b0; x < b0 + n; ++x) {
        const BkTask &t = pl.bk[x];
        std::vector<int64_t> rd, wr;
        const int nt = (t.n + TILE - 1) / TILE;
        const int64_t aa = t.a >> ENC_SHIFT, ao = t.a & ENC_MASK;
        const int64_t la = t.l >> ENC_SHIFT, lo = t.l & ENC_MASK;
        for (int c = 0; c < nt; ++c)
            for (int r = c; r < nt; ++r) {
                rd.push_back(tile_id(enc((int)aa, ao + (int64_t)c * t.ldt + (int64_t)r * TILE_ELEMS)));
                wr.push_back(tile_id(enc((int)la, lo + (int64_t)c * t.ldt + (int64_t)r * TILE_ELEMS)));
            }
        for (int c = 0; c < nt; ++c)
            for (int r = 0; r < nt; ++r) wr.push_back(tile_id(t.tt + (int64_t)(c * nt + r) * TILE_ELEMS));
        for (int r = 0; r < nt; ++r) wr.push_back(drow_id(t.drow + (int64_t)r * TILE));
        add_pairs(pl, t.p0, t.np, rd);
        acc.push_back({rd, wr});
    }
    return acc;
}

Acc gemm_access(const Plan &pl, int64_t g0, int64_t n, bool update) {
    Acc acc;
    for (int64_t x = g0; x < g0 + n; ++x) {
        const GemmTask &g = pl.gemm[x];
        std::vector<int64_t> rd, wr{tile_id(g.c)};
        add_pairs(pl, g.p0, g.np, rd);
        if (update) rd.push_back(tile_id(g.c));
        acc.push_back({rd, wr});
    }
    return acc;
}

Acc scale_access(const Plan &pl, int64_t s0, int64_t n) {
    Acc acc;
    for (int64_t x = s0; x < s0 + n; ++x) {
        const ScaleTask &t = pl.scale[x];
        std::vector<int64_t> rd{tile_id(t.x)}, wr{tile_id(t.w)};
        if (t.xprev >= 0) rd.push_back(tile_id(t.xprev));
        if (t.xnext >= 0) rd.push_back(tile_id(t.xnext));
        rd.push_back(drow_id(t.drow));
        if (t.ncols > 0) rd.push_back(drow_id(t.drow + t.ncols - 1));
        add_pairs(pl, t.q0, t.nq, rd);
        acc.push_back({rd, wr});
    }
    return acc;
}

Acc panel_scale_access(const Plan &pl, const FactorStep &st) {
    Acc acc = gemm_access(pl, st.pan0, st.npan, false);
    const Acc sc = scale_access(pl, st.sc0, st.nsc);
    for (size_t i = 0; i < acc.size() && i < sc.size(); ++i) {
        acc[i].first.insert(acc[i].first.end(), sc[i].first.begin(), sc[i].first.end());
        acc[i].second.insert(acc[i].second.end(), sc[i].second.begin(), sc[i].second.end());
    }
    return acc;
}

void panels(Sim &sim, const Plan &pl, const FactorStep &st, const std::string &tag) {
    if (st.nbk > 0) sim.launch(0, tag + " pivot", bk_access(pl, st.bk0, st.nbk));
    if (st.npan > 0 || st.nsc > 0) {
        if (st.fused_scale) {
            sim.launch(0, tag + " panel+scale", panel_scale_access(pl, st));
        } else {
            sim.launch(0, tag + " panel", gemm_access(pl, st.pan0, st.npan, false));
            sim.launch(0, tag + " scale", scale_access(pl, st.sc0, st.nsc));
        }
    }
}

// the look-ahead sweep (one side stream; a step's side updates waited for
// before the next step's critical updates)
void sweep_plain(Sim &sim, const Plan &pl, const std::vector<FactorStep> &steps, const ScheduleModel &m,
                 bool one_stream, const std::string &phase) {
    const int64_t min_split = one_stream ? INT64_MAX : (m.lookahead_tasks > 0 ? m.lookahead_tasks : 512);
    bool have_rest = false;
    VC rest_done{};
    for (size_t x = 0; x < steps.size(); ++x) {
        const FactorStep &st = steps[x];
        const std::string tag = phase + " step " + std::to_string(x);
        panels(sim, pl, st, tag);
        const bool split = st.nup - st.ncrit >= min_split;
        const int64_t ncrit = split ? st.ncrit : st.nup;
        const int64_t nrest = st.nup - ncrit;
        auto launch_rest = [&]() {
            sim.wait(1, sim.record(0));
            sim.launch(1, tag + " side updates", gemm_access(pl, st.up0 + ncrit, nrest, true));
        };
        const bool late = m.side_early == 0;
        if (nrest > 0 && !late) launch_rest();
        if (have_rest && st.wait_rest) {
            if (!m.drop_waits) sim.wait(0, rest_done);
            have_rest = false;
        }
        if (ncrit > 0) sim.launch(0, tag + " updates", gemm_access(pl, st.up0, ncrit, true));
        if (nrest > 0 && late) launch_rest();
        if (nrest > 0) {
            rest_done = sim.record(1);
            have_rest = true;
        }
    }
    if (have_rest && !m.drop_waits) sim.wait(0, rest_done);
}

// the K sweep with block-column tracking (two side streams)
void sweep_tracked(Sim &sim, const Plan &pl, const std::vector<FactorStep> &steps, const ScheduleModel &m) {
    const int64_t min_split = m.lookahead_tasks > 0 ? m.lookahead_tasks : 512;
    std::vector<VC> evs[2];
    std::vector<std::pair<int, int>> last(pl.k_units, {-1, -1});
    auto wait_cols = [&](const std::vector<int> &cols, int on) {
        int hi[2] = {-1, -1};
        for (int k : cols)
            if (last[k].first >= 0) hi[last[k].first] = std::max(hi[last[k].first], last[k].second);
        for (int q = 0; q < 2; ++q)
            if (hi[q] >= 0 && q + 1 != on && !m.drop_waits) sim.wait(on, evs[q][hi[q]]);
    };
    for (size_t x = 0; x < steps.size(); ++x) {
        const FactorStep &st = steps[x];
        const std::string tag = "K step " + std::to_string(x);
        wait_cols(st.cols_bk, 0);
        panels(sim, pl, st, tag);
        const int64_t nfar = st.nup - st.ncrit - st.nnear;
        const bool split = st.nup - st.ncrit >= min_split;
        bool have_ready = false;
        VC ready{};
        auto side_launch = [&](int q, int64_t off, int64_t n, const std::vector<int> &cols, const char *what) {
            if (!have_ready) {
                ready = sim.record(0);
                have_ready = true;
            }
            sim.wait(q + 1, ready);
            wait_cols(cols, q + 1);
            sim.launch(q + 1, tag + " " + what, gemm_access(pl, st.up0 + off, n, true));
            evs[q].push_back(sim.record(q + 1));
            for (int k : cols) last[k] = {q, (int)evs[q].size() - 1};
        };
        auto rest = [&]() {
            if (st.nnear > 0) side_launch(0, st.ncrit, st.nnear, st.cols_near, "near updates");
            if (nfar > 0) side_launch(1, st.ncrit + st.nnear, nfar, st.cols_far, "far updates");
        };
        const bool late = m.side_early == 0;
        if (split && !late) rest();
        const int64_t nmain = split ? st.ncrit : st.nup;
        if (nmain > 0) {
            wait_cols(st.cols_crit, 0);
            if (!split) {
                wait_cols(st.cols_near, 0);
                wait_cols(st.cols_far, 0);
            }
            sim.launch(0, tag + " updates", gemm_access(pl, st.up0, nmain, true));
        }
        if (split && late) rest();
    }
    for (int q = 0; q < 2; ++q)
        if (!evs[q].empty()) sim.wait(0, evs[q].back());
}

// step 5 in multifrontal form (one stream)
void sweep_multifrontal(Sim &sim, const Plan &pl) {
    for (size_t x = 0; x < pl.mf_steps.size(); ++x) {
        const FactorStep &st = pl.mf_steps[x];
        const std::string tag = "MF step " + std::to_string(x);
        if (st.nadd > 0) {
            Acc acc;
            for (int64_t a = st.add0; a < st.add0 + st.nadd; ++a) {
                const AddTask &t = pl.mf_add[a];
                std::vector<int64_t> rd, wr{tile_id(t.dst)};
                if (t.accumulate) rd.push_back(tile_id(t.dst));
                for (int32_t q = t.s0; q < t.s0 + t.ns; ++q) rd.push_back(tile_id(pl.mf_src[q]));
                acc.push_back({rd, wr});
            }
            sim.launch(0, tag + " extend-add", acc);
        }
        panels(sim, pl, st, tag);
        if (st.nup > 0) sim.launch(0, tag + " updates", gemm_access(pl, st.up0, st.nup, true));
    }
}

}  // namespace

int64_t check_factor_schedule(const Plan &pl, const ScheduleModel &m, std::string &report) {
    Sim sim;
    sweep_plain(sim, pl, pl.s1_steps, m, false, "S1");
    {
        // assembly of -K from the trailing subdomain blocks, on the caller's stream
        Acc acc;
        for (const AsmTask &t : pl.asmb) {
            std::vector<int64_t> rd, wr{tile_id(t.dst)};
            for (int c = 0; c < t.ncontrib; ++c) rd.push_back(((int64_t)ARR_M << 40) | t.mbase[c]);
            acc.push_back({rd, wr});
        }
        sim.launch(0, "assembly", acc);
    }
    if (pl.mf)
        sweep_multifrontal(sim, pl);
    else if (m.k_overlap && !pl.k_steps.empty() && pl.k_steps[0].track && !m.one_stream_k)
        sweep_tracked(sim, pl, pl.k_steps, m);
    else
        sweep_plain(sim, pl, pl.k_steps, m, m.one_stream_k, "K");
    report = sim.report;
    return sim.races;
}

}  // namespace d3m
