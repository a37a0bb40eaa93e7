// The decomposed system of Section II, eq. (1), built on the host:
// subdomain matrices A_d (FEM + ABC + Robin loss/gain), one set of Lagrange
// multipliers with signed maps D_d, and the blocks ("super-nodes") of K.
//
// Readings: on a triangle shared by subdomains p < q the multiplier is
// lambda = j_p - alpha e and the neighbour sees -lambda, so A_p gets
// +alpha T and A_q gets -alpha T ("loss or gain at the interfaces") while
// D_p = +1 and D_q = -1 on the shared edge; edges shared by m > 2 subdomains
// carry m - 1 multipliers along a spanning tree of the subdomain pairs that
// share a triangle containing the edge (Kruskal, lexicographic).  Edges of
// PEC triangles (tangential field zero) carry no multiplier, and their rows
// of A_d are the identity (every other entry of the row and column dropped),
// so the subdomain solves leave them at the zero load they are given.
#include <algorithm>
#include <array>
#include <functional>
#include <map>
#include <numeric>
#include <string>

#include "problem.hpp"

namespace d3m {

i64 Subdomain::row_of(i64 e) const {
    auto it = std::lower_bound(sorted.begin(), sorted.end(), e);
    if (it == sorted.end() || *it != e) return -1;
    return sorted_pos[it - sorted.begin()];
}

namespace {

struct Dsu {
    std::map<int, int> p;
    int find(int x) {
        auto it = p.find(x);
        if (it == p.end()) { p[x] = x; return x; }
        while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
        return x;
    }
    bool unite(int a, int b) {
        int ra = find(a), rb = find(b);
        if (ra == rb) return false;
        p[std::max(ra, rb)] = std::min(ra, rb);
        return true;
    }
};

}  // namespace

namespace {

// Nested-dissection order of the edge rows of one subdomain (interior and
// interface edges alike; the multiplier rows stay last), as groups in
// elimination order.  Two edges are neighbours when they share a
// tetrahedron of the subdomain (the pattern of A_d).  A region of more than
// `leaf` edges is cut at the median of its edge midpoints along its longest
// extent; the lower side's edges that neighbour the upper side form the
// separator, which follows both sides, so the two sides eliminate
// independently and fill stays inside fronts.  Each leaf and each separator
// is one group, by increasing global id.
std::vector<std::vector<i64>> nested_dissection(const Mesh &m, const std::vector<i32> &part, int d, const std::vector<i64> &edges,
                                   const std::vector<i64> &tets_of_d, int leaf) {
    const i64 n = (i64)edges.size();
    std::vector<i64> sorted(edges);
    std::sort(sorted.begin(), sorted.end());
    auto local = [&](i64 e) { return (i64)(std::lower_bound(sorted.begin(), sorted.end(), e) - sorted.begin()); };
    // neighbour lists (CSR) over local indices
    std::vector<std::vector<i64>> nb(n);
    for (i64 t : tets_of_d) {
        if (part[t] != d) continue;
        i64 le[6];
        for (int a = 0; a < 6; ++a) le[a] = local(m.tet_edges[6 * t + a]);
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b)
                if (a != b) nb[le[a]].push_back(le[b]);
    }
    for (auto &v : nb) {
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    std::vector<double> mid(3 * n);
    for (i64 i = 0; i < n; ++i) {
        const i64 e = sorted[i], a = m.edges[2 * e], b = m.edges[2 * e + 1];
        for (int c = 0; c < 3; ++c) mid[3 * i + c] = 0.5 * (m.xyz[3 * a + c] + m.xyz[3 * b + c]);
    }
    std::vector<std::vector<i64>> out;
    i64 placed = 0;
    std::vector<char> side(n, 0);  // 2: upper side of the current cut
    // regions are processed depth first: a region pushes (separator marker,
    // upper, lower) so that lower, upper and then the separator are emitted
    struct Item { std::vector<i64> r; bool emit; };
    std::vector<Item> work;
    {
        std::vector<i64> all(n);
        for (i64 i = 0; i < n; ++i) all[i] = i;
        work.push_back({all, false});
    }
    while (!work.empty()) {
        Item it = std::move(work.back());
        work.pop_back();
        std::vector<i64> &r = it.r;
        if (it.emit || (i64)r.size() <= leaf) {
            if (r.empty()) continue;
            std::sort(r.begin(), r.end());
            out.emplace_back();
            for (i64 i : r) out.back().push_back(sorted[i]);
            placed += (i64)r.size();
            continue;
        }
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (i64 i : r)
            for (int c = 0; c < 3; ++c) {
                lo[c] = std::min(lo[c], mid[3 * i + c]);
                hi[c] = std::max(hi[c], mid[3 * i + c]);
            }
        int ax = 0;
        for (int c = 1; c < 3; ++c)
            if (hi[c] - lo[c] > hi[ax] - lo[ax]) ax = c;
        std::vector<double> v;
        v.reserve(r.size());
        for (i64 i : r) v.push_back(mid[3 * i + ax]);
        std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
        const double cut = v[v.size() / 2];
        std::vector<i64> lower, upper, sep;
        for (i64 i : r) {
            const bool up = mid[3 * i + ax] >= cut;
            side[i] = up ? 2 : 1;
            (up ? upper : lower).push_back(i);
        }
        if (lower.empty() || upper.empty()) {
            for (i64 i : r) side[i] = 0;
            work.push_back({r, true});
            continue;
        }
        std::vector<i64> lower_in;
        for (i64 i : lower) {
            bool touches = false;
            for (i64 j : nb[i])
                if (side[j] == 2) { touches = true; break; }
            (touches ? sep : lower_in).push_back(i);
        }
        for (i64 i : r) side[i] = 0;
        work.push_back({sep, true});
        work.push_back({upper, false});
        work.push_back({lower_in, false});
    }
    if (placed != n) throw Error{-1, "internal: nested dissection lost edges"};
    return out;
}

}  // namespace

void build_decomposition(Decomp &dc, const Mesh &m, const i32 *part, double k,
                         cplx alpha, const double *eps, int s1_order) {
    if (!(k > 0.0)) throw Error{-1, "k must be positive"};
    dc.part.assign(part, part + m.nt);
    int N = 0;
    for (i64 t = 0; t < m.nt; ++t) {
        if (part[t] < 0) throw Error{-1, "negative partition id"};
        N = std::max(N, part[t] + 1);
    }
    std::vector<i64> cnt(N, 0);
    for (i64 t = 0; t < m.nt; ++t) cnt[part[t]]++;
    for (int d = 0; d < N; ++d)
        if (cnt[d] == 0) throw Error{-1, "empty subdomain " + std::to_string(d)};
    dc.N = N;

    // Sub(e)
    std::vector<std::pair<i64, i32>> es;
    es.reserve(6 * m.nt);
    for (i64 t = 0; t < m.nt; ++t)
        for (int a = 0; a < 6; ++a) es.push_back({m.tet_edges[6 * t + a], part[t]});
    std::sort(es.begin(), es.end());
    es.erase(std::unique(es.begin(), es.end()), es.end());
    dc.sub_ptr.assign(m.ne + 1, 0);
    dc.sub_list.resize(es.size());
    for (size_t i = 0; i < es.size(); ++i) {
        dc.sub_ptr[es[i].first + 1]++;
        dc.sub_list[i] = es[i].second;
    }
    for (i64 e = 0; e < m.ne; ++e) dc.sub_ptr[e + 1] += dc.sub_ptr[e];
    dc.owner.resize(m.ne);
    for (i64 e = 0; e < m.ne; ++e) dc.owner[e] = (i32)dc.sub_list[dc.sub_ptr[e]];

    // faces: boundary (one tetrahedron) and interface (two, different parts)
    dc.bface.clear(); dc.iface.clear(); dc.iface_p.clear(); dc.iface_q.clear();
    for (i64 f = 0; f < m.nf; ++f) {
        i64 t0 = m.face_tet[2 * f], t1 = m.face_tet[2 * f + 1];
        if (t1 < 0) { dc.bface.push_back(f); continue; }
        i32 a = part[t0], b = part[t1];
        if (a != b) {
            dc.iface.push_back(f);
            dc.iface_p.push_back(std::min(a, b));
            dc.iface_q.push_back(std::max(a, b));
        }
    }

    // subdomain rows: [interior | interface], each sorted by global id
    // (s1_order 0), or all edge rows in nested-dissection order (1)
    dc.sub.assign(N, Subdomain());
    {
        std::vector<std::vector<i64>> edges_of(N), tets_of(N);
        for (i64 e = 0; e < m.ne; ++e)
            for (i64 s = dc.sub_ptr[e]; s < dc.sub_ptr[e + 1]; ++s) edges_of[dc.sub_list[s]].push_back(e);
        if (s1_order == 2) {
            std::vector<i64> sz(N);
            for (int d = 0; d < N; ++d) sz[d] = (i64)edges_of[d].size();
            std::nth_element(sz.begin(), sz.begin() + N / 2, sz.end());
            s1_order = sz[N / 2] >= kNdAutoRows ? 1 : 0;
        }
        dc.s1_order = s1_order;
        if (s1_order == 1)
            for (i64 t = 0; t < m.nt; ++t) tets_of[part[t]].push_back(t);
        for (int d = 0; d < N; ++d) {
            Subdomain &S = dc.sub[d];
            std::vector<i64> I, B;
            for (i64 e : edges_of[d]) (dc.sub_ptr[e + 1] - dc.sub_ptr[e] == 1 ? I : B).push_back(e);
            S.nI = (i64)I.size();
            S.edges = I;
            S.edges.insert(S.edges.end(), B.begin(), B.end());
            if (s1_order == 1) {
                // every group starts a tile: rows of different groups never
                // share a tile, so the tile pattern keeps the dissection's
                // fill (padding rows: -1, identity, no load)
                S.edges.clear();
                for (const auto &g : nested_dissection(m, dc.part, d, edges_of[d], tets_of[d], kNdLeaf)) {
                    S.edges.insert(S.edges.end(), g.begin(), g.end());
                    while (S.edges.size() % TILE) S.edges.push_back(-1);
                }
            }
            S.n = (i64)S.edges.size();
            S.sorted = edges_of[d];  // already increasing
            S.sorted_pos.resize(S.sorted.size());
            for (i64 r = 0; r < S.n; ++r) {
                if (S.edges[r] < 0) continue;
                auto it = std::lower_bound(S.sorted.begin(), S.sorted.end(), S.edges[r]);
                S.sorted_pos[it - S.sorted.begin()] = (i32)r;
            }
        }
    }

    // Lagrange multipliers: spanning trees over interface-triangle pairs
    {
        std::vector<std::array<i64, 3>> cand;  // (e, p, q)
        for (size_t i = 0; i < dc.iface.size(); ++i)
            for (int a = 0; a < 3; ++a)
                cand.push_back({m.face_edges[3 * dc.iface[i] + a], dc.iface_p[i], dc.iface_q[i]});
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        std::vector<std::array<i64, 3>> lms;  // (p, q, e)
        size_t c = 0;
        for (i64 e = 0; e < m.ne; ++e) {
            i64 mult = dc.sub_ptr[e + 1] - dc.sub_ptr[e];
            size_t c0 = c;
            while (c < cand.size() && cand[c][0] == e) ++c;
            if (mult < 2 || (!m.pec.empty() && m.pec[e])) continue;
            Dsu dsu;
            i64 chosen = 0;
            for (size_t i = c0; i < c; ++i)  // candidates sorted by (p, q)
                if (dsu.unite((int)cand[i][1], (int)cand[i][2])) {
                    lms.push_back({cand[i][1], cand[i][2], e});
                    ++chosen;
                }
            if (chosen != mult - 1)
                throw Error{-1, "edge " + std::to_string(e) +
                                    ": its subdomains are not connected through shared triangles"};
        }
        std::sort(lms.begin(), lms.end());
        dc.n_lm = (i64)lms.size();
        dc.lm_p.resize(dc.n_lm); dc.lm_q.resize(dc.n_lm); dc.lm_e.resize(dc.n_lm);
        dc.blk_p.clear(); dc.blk_q.clear(); dc.blk_start.clear();
        for (i64 l = 0; l < dc.n_lm; ++l) {
            dc.lm_p[l] = lms[l][0]; dc.lm_q[l] = lms[l][1]; dc.lm_e[l] = lms[l][2];
            if (l == 0 || lms[l][0] != lms[l - 1][0] || lms[l][1] != lms[l - 1][1]) {
                dc.blk_p.push_back((i32)lms[l][0]);
                dc.blk_q.push_back((i32)lms[l][1]);
                dc.blk_start.push_back(l);
            }
        }
        dc.blk_start.push_back(dc.n_lm);
        dc.nblk = (int)dc.blk_p.size();
    }
    // blocks touching each subdomain and their LM-region offsets
    for (int b = 0; b < dc.nblk; ++b) {
        dc.sub[dc.blk_p[b]].blocks.push_back(b);
        dc.sub[dc.blk_q[b]].blocks.push_back(b);
    }
    for (int d = 0; d < N; ++d) {
        Subdomain &S = dc.sub[d];
        S.block_off.clear();
        i64 off = 0;
        for (int b : S.blocks) {
            S.block_off.push_back(off);
            off += dc.blk_start[b + 1] - dc.blk_start[b];
        }
        S.m = off;
    }

    // A_d pattern (lower triangle in row order) and values
    for (int d = 0; d < N; ++d) {
        Subdomain &S = dc.sub[d];
        S.contrib_slot.clear(); S.contrib_tet.clear(); S.contrib_a.clear(); S.contrib_b.clear();
    }
    // collect keyed contributions: (row, col) -> value parts
    std::vector<std::vector<std::array<i64, 4>>> tetc(N);   // (row, col, tet, a*6+b)
    std::vector<std::vector<std::pair<std::array<i64, 2>, cplx>>> statc(N);
    auto is_pec = [&](i64 e) { return !m.pec.empty() && m.pec[e] != 0; };
    for (i64 t = 0; t < m.nt; ++t) {
        Subdomain &S = dc.sub[part[t]];
        i64 r[6];
        bool z[6];
        for (int a = 0; a < 6; ++a) {
            r[a] = S.row_of(m.tet_edges[6 * t + a]);
            z[a] = is_pec(m.tet_edges[6 * t + a]);
        }
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b)
                if (r[a] >= r[b] && !z[a] && !z[b]) tetc[part[t]].push_back({r[a], r[b], t, a * 6 + b});
    }
    auto add_face = [&](int d, i64 f, cplx scale) {
        Subdomain &S = dc.sub[d];
        double T[9];
        tri_tangential_mass(m, f, T);
        i64 r[3];
        bool z[3];
        for (int a = 0; a < 3; ++a) {
            r[a] = S.row_of(m.face_edges[3 * f + a]);
            z[a] = is_pec(m.face_edges[3 * f + a]);
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                if (r[a] >= r[b] && !z[a] && !z[b]) statc[d].push_back({{r[a], r[b]}, scale * T[3 * a + b]});
    };
    for (int d = 0; d < N; ++d)
        for (i64 r = 0; r < dc.sub[d].n; ++r)
            if (dc.sub[d].edges[r] < 0 || is_pec(dc.sub[d].edges[r])) statc[d].push_back({{r, r}, cplx(1.0, 0.0)});
    const cplx jk(0.0, k);
    for (i64 f : dc.bface) add_face(part[m.face_tet[2 * f]], f, jk);
    for (size_t i = 0; i < dc.iface.size(); ++i) {
        add_face(dc.iface_p[i], dc.iface[i], alpha);
        add_face(dc.iface_q[i], dc.iface[i], -alpha);
    }
    for (int d = 0; d < N; ++d) {
        Subdomain &S = dc.sub[d];
        std::vector<std::array<i64, 2>> keys;
        keys.reserve(tetc[d].size() + statc[d].size());
        for (auto &x : tetc[d]) keys.push_back({x[0], x[1]});
        for (auto &x : statc[d]) keys.push_back(x.first);
        std::sort(keys.begin(), keys.end());
        keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
        S.a_row.resize(keys.size()); S.a_col.resize(keys.size());
        for (size_t i = 0; i < keys.size(); ++i) { S.a_row[i] = keys[i][0]; S.a_col[i] = keys[i][1]; }
        auto slot = [&](const std::array<i64, 2> &key) {
            return (i64)(std::lower_bound(keys.begin(), keys.end(), key) - keys.begin());
        };
        S.a_static.assign(keys.size(), 0.0);
        for (auto &x : statc[d]) S.a_static[slot(x.first)] += x.second;
        for (auto &x : tetc[d]) {
            S.contrib_slot.push_back(slot({x[0], x[1]}));
            S.contrib_tet.push_back(x[2]);
            S.contrib_a.push_back((int8_t)(x[3] / 6));
            S.contrib_b.push_back((int8_t)(x[3] % 6));
        }
    }
    reassemble_values(dc, m, k, eps);
}

void reassemble_values(Decomp &dc, const Mesh &m, double k, const double *eps) {
    std::vector<double> Kc(36 * m.nt), M(36 * m.nt);
    for (i64 t = 0; t < m.nt; ++t) tet_curl_mass(m, t, &Kc[36 * t], &M[36 * t]);
    for (int d = 0; d < dc.N; ++d) {
        Subdomain &S = dc.sub[d];
        S.a_val = S.a_static;
        for (size_t c = 0; c < S.contrib_slot.size(); ++c) {
            i64 t = S.contrib_tet[c];
            int ab = S.contrib_a[c] * 6 + S.contrib_b[c];
            S.a_val[S.contrib_slot[c]] += Kc[36 * t + ab] - k * k * eps[t] * M[36 * t + ab];
        }
    }
}

// ------------------------------------------------------------------------
// Steps 3-4: geometric nested dissection of the clique graph of K (blocks
// adjacent when they share a subdomain) on subdomain centroids, then block
// symbolic elimination and elimination-tree levels.  sub_group (empty or one
// entry per subdomain) splits the subdomains into independent problems whose
// blocks never meet: each group is dissected on its own, one after another,
// so the elimination tree is a forest with one tree per problem.
void order_blocks(BlockOrder &bo, const Decomp &dc, const Mesh &m, const std::vector<int> &sub_group) {
    int N = dc.N, nb = dc.nblk;
    std::vector<double> cen(3 * N, 0.0);
    std::vector<i64> cnt(N, 0);
    for (i64 t = 0; t < m.nt; ++t) {
        int d = dc.part[t];
        for (int a = 0; a < 4; ++a)
            for (int x = 0; x < 3; ++x) cen[3 * d + x] += m.xyz[3 * m.tets[4 * t + a] + x] * 0.25;
        cnt[d]++;
    }
    for (int d = 0; d < N; ++d)
        for (int x = 0; x < 3; ++x) cen[3 * d + x] /= (double)cnt[d];

    std::vector<std::vector<int>> blocks_of(N);
    for (int b = 0; b < nb; ++b) {
        blocks_of[dc.blk_p[b]].push_back(b);
        blocks_of[dc.blk_q[b]].push_back(b);
    }
    bo.order.clear();
    std::vector<char> side(N, 0);
    // recursive bisection of a set of subdomains
    std::function<void(std::vector<int>)> rec = [&](std::vector<int> set) {
        if (set.size() <= 1) return;
        int best_ax = -1;
        std::vector<double> vals;
        double best_ext = -1.0;
        for (int ax = 0; ax < 3; ++ax) {
            double lo = 1e300, hi = -1e300;
            for (int d : set) { lo = std::min(lo, cen[3 * d + ax]); hi = std::max(hi, cen[3 * d + ax]); }
            if (hi - lo > best_ext + 1e-12) { best_ext = hi - lo; best_ax = ax; }
        }
        std::vector<int> left, right;
        if (best_ext <= 1e-12) {
            std::vector<int> s = set;
            std::sort(s.begin(), s.end());
            left.assign(s.begin(), s.begin() + s.size() / 2);
            right.assign(s.begin() + s.size() / 2, s.end());
        } else {
            for (int d : set) vals.push_back(cen[3 * d + best_ax]);
            std::sort(vals.begin(), vals.end());
            std::vector<double> distinct;
            for (double v : vals)
                if (distinct.empty() || v - distinct.back() > 1e-9) distinct.push_back(v);
            double cut = distinct[distinct.size() / 2 - 1] + 1e-9;  // first floor(n/2) values left
            for (int d : set) (cen[3 * d + best_ax] <= cut ? left : right).push_back(d);
        }
        rec(left);
        rec(right);
        for (int d : left) side[d] = 1;
        for (int d : right) side[d] = 2;
        std::vector<int> sep;
        for (int d : left)
            for (int b : blocks_of[d]) {
                int other = dc.blk_p[b] == d ? dc.blk_q[b] : dc.blk_p[b];
                if (side[other] == 2) sep.push_back(b);
            }
        for (int d : set) side[d] = 0;
        std::sort(sep.begin(), sep.end());
        sep.erase(std::unique(sep.begin(), sep.end()), sep.end());
        for (int b : sep) bo.order.push_back(b);
    };
    if (sub_group.empty()) {
        std::vector<int> all(N);
        std::iota(all.begin(), all.end(), 0);
        rec(all);
    } else {
        if ((int)sub_group.size() != N) throw Error{-1, "internal: subdomain groups do not match the partition"};
        const int ng = *std::max_element(sub_group.begin(), sub_group.end()) + 1;
        std::vector<std::vector<int>> groups(ng);
        for (int d = 0; d < N; ++d) groups[sub_group[d]].push_back(d);
        for (auto &g : groups) rec(g);
    }
    if ((int)bo.order.size() != nb) throw Error{-1, "ordering did not cover every block"};
    bo.pos.assign(nb, -1);
    for (int j = 0; j < nb; ++j) bo.pos[bo.order[j]] = j;

    // block symbolic factorisation: struct(j) = later neighbours of j plus the
    // structs of its elimination-tree children (minus j itself)
    std::vector<std::vector<i32>> adj(nb);
    for (int d = 0; d < N; ++d)
        for (int a : blocks_of[d])
            for (int b : blocks_of[d])
                if (a != b) adj[bo.pos[a]].push_back(bo.pos[b]);
    bo.strct.assign(nb, {});
    std::vector<std::vector<i32>> pending(nb);
    std::vector<int> parent(nb, -1);
    for (int j = 0; j < nb; ++j) {
        std::vector<i32> s;
        for (i32 x : adj[j]) if (x > j) s.push_back(x);
        for (i32 x : pending[j]) if (x > j) s.push_back(x);
        std::sort(s.begin(), s.end());
        s.erase(std::unique(s.begin(), s.end()), s.end());
        bo.strct[j] = s;
        std::vector<i32>().swap(pending[j]);
        if (!s.empty()) {
            parent[j] = s[0];
            pending[s[0]].insert(pending[s[0]].end(), s.begin() + 1, s.end());
        }
    }
    bo.level.assign(nb, 0);
    for (int j = 0; j < nb; ++j)
        if (parent[j] >= 0) bo.level[parent[j]] = std::max(bo.level[parent[j]], bo.level[j] + 1);
    bo.n_levels = 0;
    for (int j = 0; j < nb; ++j) bo.n_levels = std::max(bo.n_levels, bo.level[j] + 1);
}

}  // namespace d3m
