// Multifrontal form of step 5 (the block LDL^T of -K), the variant named
// after the seven steps of Section II.
//
// The right-looking schedule of build_plan applies the Schur updates of a
// unit straight to the block columns of its structure.  Here they go into
// the unit's update matrix instead:
//     U_j[i, k] = F_j[i, k] - X_ij W_kj^T      (i >= k in struct(j)),
// where the front F_j is block column j of -K (its own storage, as assembled
// by step 2) plus the update matrices of j's children added at their rows
// and columns (extend-add), and F_j[i, k] for i, k in struct(j) holds only
// the children's contributions.  The parent of j in the elimination tree is
// the first unit of struct(j); struct(c) minus the parent lies inside
// struct(parent), so every child's tile has a place in the parent's front.
// The pivot, panel and scaling launches and the factor storage (L-hat, TT,
// D) are the right-looking schedule's, so the solve is unchanged.
//
// Fronts are amalgamated along chains (supernodes): consecutive units of an
// elimination-tree chain, each the only child of the next, at most seg_max of
// them, share one front.  Inside the segment a unit updates the block columns
// of the later segment units in place (they are part of the front); its
// updates of rows and columns beyond the segment are applied by the
// segment's last unit, for all the segment's units at once, into the
// segment's update matrix U_s over struct(last unit).  Only a segment's first
// unit has children outside the segment, so the extend-adds of a front all
// happen at the first unit's step: into the block columns of the segment's
// units and into the initial U_s.  seg_max = 1 is the plain unit-by-unit
// multifrontal method.
//
// A step of the sweep (one elimination-tree level) is: extend-adds of the
// level's new fronts, the pivot launch, the panel launch, one update GEMM
// launch (in-segment columns and the update matrices of segments that end
// at this level).  An update matrix lives from its segment's first level to
// its parent's; the pool reuses the space of matrices already added in (first
// fit over slots, free from the level after their reader's, so on the one
// stream of the sweep every write to a reused slot comes after its last
// read).
#include <algorithm>
#include <map>

#include "plan.hpp"

namespace d3m {

namespace {

// first-fit allocator over tile slots of one pool
struct SlotPool {
    std::map<i64, i64> free_;  // start -> length
    i64 end = 0;
    i64 take(i64 n) {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                const i64 s = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[s + n] = len - n;
                return s;
            }
        // grow, absorbing a free run that ends at the pool's end
        if (!free_.empty()) {
            auto last = std::prev(free_.end());
            if (last->first + last->second == end) {
                const i64 s = last->first;
                free_.erase(last);
                end = s + n;
                return s;
            }
        }
        const i64 s = end;
        end += n;
        return s;
    }
    void give(i64 s, i64 n) {
        auto it = free_.emplace(s, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace

void build_multifrontal(Plan &pl, int seg_max) {
    const int nb = pl.k_units;
    const auto &S = pl.kstruct;
    auto E = [](int arr, i64 slot) { return enc(arr, slot * TILE_ELEMS); };
    auto trows = [](int n, int a) { return std::min(TILE, n - a * TILE); };
    seg_max = std::max(1, std::min(16, seg_max));

    // tree and levels
    std::vector<int> parent(nb, -1), level(nb, 0), nchild(nb, 0);
    for (int u = 0; u < nb; ++u)
        if (!S[u].empty()) {
            parent[u] = S[u][0];
            nchild[parent[u]]++;
        }
    int nlev = 0;
    for (int u = 0; u < nb; ++u) {
        if (parent[u] >= 0) level[parent[u]] = std::max(level[parent[u]], level[u] + 1);
        nlev = std::max(nlev, level[u] + 1);
    }
    if (nlev != (int)pl.k_steps.size()) throw Error{-1, "internal: multifrontal levels differ from the schedule's"};
    auto idx_in = [&](int j, int i) -> int {  // position of unit i in struct(j), -1 if absent
        auto it = std::lower_bound(S[j].begin(), S[j].end(), i);
        return (it != S[j].end() && *it == i) ? (int)(it - S[j].begin()) : -1;
    };
    for (int c = 0; c < nb; ++c)
        if (parent[c] >= 0)
            for (size_t x = 1; x < S[c].size(); ++x)
                if (idx_in(parent[c], S[c][x]) < 0)
                    throw Error{-1, "internal: a child's structure is not inside its parent's front"};
    auto kslot = [&](int j, int i, int a, int b) -> i64 {  // tile (a, b) of block (i, j) in column storage
        const i64 ro = i == j ? 0 : pl.krow_off[j][1 + idx_in(j, i)];
        return pl.kcol[j] + (i64)b * pl.kR[j] + ro + a;
    };

    // segments (units increase along a chain): first and last unit of each
    std::vector<int> seg_of(nb), seg_len(nb, 1);
    for (int u = 0; u < nb; ++u) seg_of[u] = u;
    for (int u = 0; u < nb; ++u) {
        const int p = parent[u];
        if (p >= 0 && nchild[p] == 1 && seg_len[seg_of[u]] < seg_max) {
            seg_of[p] = seg_of[u];
            seg_len[seg_of[u]]++;
        }
    }
    std::vector<int> seg_last(nb, -1);  // indexed by segment id (= its first unit)
    for (int u = 0; u < nb; ++u) seg_last[seg_of[u]] = u;
    auto in_seg = [&](int s, int k) { return seg_of[k] == s; };
    // update matrix of segment s: packed lower tile triangle over struct(last)
    std::vector<std::vector<int>> rpos(nb);
    std::vector<i64> rtiles(nb, 0);
    std::vector<std::vector<int>> seg_children(nb);  // child segments (by first unit) of segment s
    for (int s = 0; s < nb; ++s) {
        if (seg_of[s] != s) continue;
        const int l = seg_last[s];
        i64 r = 0;
        for (int i : S[l]) { rpos[s].push_back((int)r); r += pl.kt[i]; }
        rtiles[s] = r;
        if (parent[l] >= 0) {
            if (seg_of[parent[l]] != parent[l])
                throw Error{-1, "internal: a child segment attaches below its parent's first unit"};
            seg_children[parent[l]].push_back(s);
        }
    }
    auto useg = [&](int s, int i, int k, int a, int b) -> i64 {  // tile (a, b) of block (i, k) of U_s
        const int l = seg_last[s];
        const i64 r = rpos[s][idx_in(l, i)] + a, c = rpos[s][idx_in(l, k)] + b;
        return pl.mf_ubase[s] + tri_slot(r, c);
    };

    // pool slots of the update matrices: U_s lives from level(s) (its initial
    // value) to level(parent(last)) (read by the parent's extend-add)
    pl.mf_ubase.assign(nb, -1);
    std::vector<std::vector<int>> by_level(nlev);
    for (int j = 0; j < nb; ++j) by_level[level[j]].push_back(j);
    SlotPool pool;
    std::vector<int> pending_free;
    pl.ku_tiles_total = 0;
    for (int L = 0; L < nlev; ++L) {
        for (int c : pending_free) pool.give(pl.mf_ubase[c], rtiles[c] * (rtiles[c] + 1) / 2);
        pending_free.clear();
        for (int j : by_level[L])
            if (seg_of[j] == j && rtiles[j] > 0) {
                const i64 n = rtiles[j] * (rtiles[j] + 1) / 2;
                pl.mf_ubase[j] = pool.take(n);
                pl.ku_tiles_total += n;
            }
        for (int j : by_level[L])
            if (seg_of[j] == j)
                for (int c : seg_children[j]) pending_free.push_back(c);
    }
    pl.ku_tiles = pool.end;

    pl.mf_steps.clear();
    pl.mf_add.clear();
    pl.mf_src.clear();
    pl.mf_add_bytes = 0.0;
    const double tile_bytes = (double)TILE_ELEMS * 16.0;
    std::vector<int64_t> src;
    for (int L = 0; L < nlev; ++L) {
        const FactorStep &rl = pl.k_steps[L];
        const auto &J = by_level[L];
        FactorStep st;
        // ---- extend-adds: the new fronts (segments starting at this level)
        st.add0 = (i64)pl.mf_add.size();
        auto add_task = [&](int64_t dst, bool acc) {
            AddTask t{};
            t.dst = dst;
            t.s0 = (int32_t)pl.mf_src.size();
            t.ns = (int32_t)src.size();
            t.accumulate = acc ? 1 : 0;
            pl.mf_src.insert(pl.mf_src.end(), src.begin(), src.end());
            pl.mf_add.push_back(t);
            pl.mf_add_bytes += tile_bytes * (double)(src.size() + (acc ? 2 : 1));
        };
        for (int f : J) {
            if (seg_of[f] != f) continue;
            const int l = seg_last[f];
            const auto &kids = seg_children[f];
            // block columns of the segment's units: the children's blocks (i, k), k in the segment
            if (!kids.empty())
                for (int k = f; k <= l; ++k) {
                    if (!in_seg(f, k)) continue;
                    std::vector<int> rows{k};
                    rows.insert(rows.end(), S[k].begin(), S[k].end());
                    for (int i : rows)
                        for (int b = 0; b < pl.kt[k]; ++b)
                            for (int a = (i == k ? b : 0); a < pl.kt[i]; ++a) {
                                src.clear();
                                for (int c : kids) {
                                    const int lc = seg_last[c];
                                    if ((i == k || idx_in(lc, i) >= 0) && (k == f || idx_in(lc, k) >= 0))
                                        src.push_back(E(ARR_KU, useg(c, i, k, a, b)));
                                }
                                if (!src.empty()) add_task(E(ARR_K, kslot(k, i, a, b)), true);
                            }
                }
            // U_f starts as the children's contributions beyond the segment
            if (rtiles[f] > 0)
                for (size_t x = 0; x < S[l].size(); ++x)
                    for (size_t y = 0; y <= x; ++y) {
                        const int i = S[l][x], k = S[l][y];
                        for (int b = 0; b < pl.kt[k]; ++b)
                            for (int a = (x == y ? b : 0); a < pl.kt[i]; ++a) {
                                src.clear();
                                for (int c : kids) {
                                    const int lc = seg_last[c];
                                    if (idx_in(lc, i) >= 0 && idx_in(lc, k) >= 0)
                                        src.push_back(E(ARR_KU, useg(c, i, k, a, b)));
                                }
                                add_task(E(ARR_KU, useg(f, i, k, a, b)), false);
                            }
                    }
        }
        st.nadd = (i64)pl.mf_add.size() - st.add0;
        // ---- pivot and panel launches: the right-looking ones without the
        // fused pending updates (those arrive through the extend-adds and the
        // in-segment updates)
        st.bk0 = (i64)pl.bk.size();
        for (i64 t = rl.bk0; t < rl.bk0 + rl.nbk; ++t) {
            BkTask b = pl.bk[t];
            b.np = 0;
            b.p0 = 0;
            pl.bk.push_back(b);
        }
        st.nbk = rl.nbk;
        st.bk_maxn = rl.bk_maxn;
        st.pan0 = (i64)pl.gemm.size();
        for (i64 t = rl.pan0; t < rl.pan0 + rl.npan; ++t) pl.gemm.push_back(pl.gemm[t]);
        st.npan = rl.npan;
        st.sc0 = (i64)pl.scale.size();
        for (i64 t = rl.sc0; t < rl.sc0 + rl.nsc; ++t) {
            ScaleTask sc = pl.scale[t];
            sc.nq = 0;
            sc.q0 = 0;
            pl.scale.push_back(sc);
        }
        st.nsc = rl.nsc;
        st.fused_scale = rl.fused_scale;
        st.pan_flops = rl.pan_flops;
        // ---- updates, grouped by target tile (one work-group per target):
        // in place for block columns of the unit's own segment, into U_s for
        // the rest when the unit ends its segment (all the segment's units)
        st.up0 = (i64)pl.gemm.size();
        std::map<std::pair<int, int>, std::vector<int>> inseg;  // (i, k) -> units of this level
        std::vector<std::pair<int, std::vector<int>>> ends;     // segment -> its units
        for (int j : J) {
            const int s = seg_of[j];
            for (size_t x = 0; x < S[j].size(); ++x)
                for (size_t y = 0; y <= x; ++y) {
                    const int i = S[j][x], k = S[j][y];
                    if (in_seg(s, k)) inseg[{i, k}].push_back(j);
                }
            if (seg_last[s] == j) {
                std::vector<int> units;
                for (int u = s; u <= j; ++u)
                    if (in_seg(s, u)) units.push_back(u);
                ends.push_back({s, units});
            }
        }
        auto emit = [&](int64_t target, int i, int k, int a, int b, bool diag_blk, const std::vector<int> &units) {
            GemmTask g{target, (int32_t)pl.pairs.size(), 0};
            const int ra = trows(pl.unit_n[i], a), rb = trows(pl.unit_n[k], b);
            for (int u : units) {
                if (idx_in(u, i) < 0 || idx_in(u, k) < 0) continue;
                for (int c = 0; c < pl.kt[u]; ++c) {
                    pl.pairs.push_back({E(ARR_KX, kslot(u, i, a, c)), E(ARR_KL, kslot(u, k, b, c))});
                    ++g.np;
                    const int w = trows(pl.unit_n[u], c);
                    st.up_flops += 8.0 * w * ((diag_blk && a == b) ? ra * (ra + 1) / 2.0 : (double)ra * rb);
                }
            }
            if (g.np > 0) pl.gemm.push_back(g);
        };
        for (auto &kv : inseg) {
            const int i = kv.first.first, k = kv.first.second;
            for (int b = 0; b < pl.kt[k]; ++b)
                for (int a = (i == k ? b : 0); a < pl.kt[i]; ++a)
                    emit(E(ARR_K, kslot(k, i, a, b)), i, k, a, b, i == k, kv.second);
        }
        for (auto &se : ends) {
            const int s = se.first, l = seg_last[s];
            for (size_t x = 0; x < S[l].size(); ++x)
                for (size_t y = 0; y <= x; ++y) {
                    const int i = S[l][x], k = S[l][y];
                    for (int b = 0; b < pl.kt[k]; ++b)
                        for (int a = (x == y ? b : 0); a < pl.kt[i]; ++a)
                            emit(E(ARR_KU, useg(s, i, k, a, b)), i, k, a, b, x == y, se.second);
                }
        }
        st.nup = (i64)pl.gemm.size() - st.up0;
        st.ncrit = st.nup;
        st.crit_flops = st.up_flops;
        pl.mf_steps.push_back(st);
    }
    // every tile a multifrontal task touches lies inside its array
    auto inside = [&](int64_t e) {
        const int arr = (int)(e >> ENC_SHIFT);
        const i64 off = e & ENC_MASK;
        const i64 n = arr == ARR_KU ? pl.ku_tiles : (arr == ARR_K || arr == ARR_KX || arr == ARR_KL) ? pl.k_tiles : -1;
        return n >= 0 && off >= 0 && off % TILE_ELEMS == 0 && off / TILE_ELEMS < n;
    };
    for (const AddTask &t : pl.mf_add) {
        bool ok = inside(t.dst) && t.s0 >= 0 && t.ns >= 0 && (size_t)t.s0 + (size_t)t.ns <= pl.mf_src.size();
        for (int32_t x = 0; ok && x < t.ns; ++x) ok = inside(pl.mf_src[t.s0 + x]) && (pl.mf_src[t.s0 + x] >> ENC_SHIFT) == ARR_KU;
        if (!ok) throw Error{-1, "internal: an extend-add task leaves its arrays"};
    }
    for (const FactorStep &st : pl.mf_steps)
        for (i64 g = st.up0; g < st.up0 + st.nup; ++g) {
            const GemmTask &t = pl.gemm[g];
            bool ok = inside(t.c) && t.p0 >= 0 && (size_t)t.p0 + t.np <= pl.pairs.size();
            for (int32_t x = 0; ok && x < t.np; ++x)
                ok = inside(pl.pairs[t.p0 + x].a) && inside(pl.pairs[t.p0 + x].b);
            if (!ok) throw Error{-1, "internal: a multifrontal update task leaves its arrays"};
        }
    pl.mf = true;
}

}  // namespace d3m
