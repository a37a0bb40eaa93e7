// Tile layouts and batched launch schedules.
//
// Step 1 (dense domain matrices) is carried out as a partial block LDL^T of
// the augmented subdomain matrix M_d = [A_d D_d; D_d^T 0] (rows: interior
// edges, interface edges, then the multipliers touching d): eliminating the
// n_d edge rows leaves -D_d^T A_d^{-1} D_d = -K_D^(d) in the trailing block.
// Step 2 sums those trailing blocks into -K; step 5 factors -K block by block
// (Algorithm 1).  Solving the saddle system with these factors is steps 6-7:
// forward over the edge rows of every M_d gives -g on the multiplier rows,
// the -K solve gives lambda, and the backward sweep over the edge rows gives
// E_d = A_d^{-1}(f_d - D_d lambda).
#include <algorithm>
#include <map>
#include <unordered_set>

#include "plan.hpp"

namespace d3m {

namespace {
inline int ceil_div(i64 a, i64 b) { return (int)((a + b - 1) / b); }
inline int tile_rows(i64 total, int t) { return (int)std::min<i64>(TILE, total - (i64)t * TILE); }

}  // namespace

void build_plan(Plan &pl, const Decomp &dc, const BlockOrder &bo, int unit_max, int s1_block, int k_block,
                bool k_fuse, bool s1_tree) {
    const int S1_BLOCK = std::max(1, std::min(16, s1_block > 0 ? s1_block : 2));
    const int K_BLOCK = std::max(1, std::min(16, k_block > 0 ? k_block : 2));
    const int N = dc.N;
    pl = Plan();

    // ------------------------------------------------------------ layouts --
    pl.TE.resize(N); pl.TL.resize(N); pl.T.resize(N); pl.fb.resize(N);
    pl.tt_s1.resize(N); pl.drow_s1.resize(N);
    i64 slot = 0, tt = 0, drow = 0;
    int maxTE = 0;
    for (int d = 0; d < N; ++d) {
        const Subdomain &S = dc.sub[d];
        pl.TE[d] = ceil_div(S.n, TILE);
        pl.TL[d] = ceil_div(S.m, TILE);
        pl.T[d] = pl.TE[d] + pl.TL[d];
        pl.fb[d] = (int)(S.nI / TILE);
        pl.tt_s1[d] = tt;
        tt += pl.TE[d];
        pl.drow_s1[d] = drow;
        drow += (i64)pl.TE[d] * TILE;
        maxTE = std::max(maxTE, pl.TE[d]);
    }

    // Units of the LM Schur complement: the blocks in elimination order, each
    // split into ceil(n / unit_max) nearly equal consecutive pieces when
    // unit_max > 0 (the pivot search of step 5 is then restricted to a
    // piece).  unit_max <= 0 keeps whole blocks.
    std::vector<int> ublk, uoff, nsz, ufirst(dc.nblk + 1, 0);
    for (int j = 0; j < (int)bo.order.size(); ++j) {
        const int b = bo.order[j];
        const int n = (int)(dc.blk_start[b + 1] - dc.blk_start[b]);
        const int pieces = unit_max > 0 ? std::max(1, (n + unit_max - 1) / unit_max) : 1;
        ufirst[j] = (int)ublk.size();
        int o = 0;
        for (int c = 0; c < pieces; ++c) {
            const int sz = n / pieces + (c < n % pieces ? 1 : 0);
            ublk.push_back(b);
            uoff.push_back(o);
            nsz.push_back(sz);
            o += sz;
        }
    }
    ufirst[bo.order.size()] = (int)ublk.size();
    const int nb = (int)ublk.size();
    std::vector<std::vector<int>> ustruct(nb);
    std::vector<int> ulevel(nb, 0), upos_block(nb);
    for (int j = 0; j < (int)bo.order.size(); ++j)
        for (int u = ufirst[j]; u < ufirst[j + 1]; ++u) {
            upos_block[u] = j;
            for (int v = u + 1; v < ufirst[j + 1]; ++v) ustruct[u].push_back(v);
            for (int i : bo.strct[j])
                for (int v = ufirst[i]; v < ufirst[i + 1]; ++v) ustruct[u].push_back(v);
            for (size_t x = 0; x < ustruct[u].size(); ++x)
                if (ustruct[u][x] <= u || (x && ustruct[u][x] <= ustruct[u][x - 1]))
                    throw Error{-1, "internal: unit structure not increasing"};
        }
    int nlev = 0;
    for (int u = 0; u < nb; ++u) {
        if (!ustruct[u].empty()) ulevel[ustruct[u][0]] = std::max(ulevel[ustruct[u][0]], ulevel[u] + 1);
        nlev = std::max(nlev, ulevel[u] + 1);
    }
    pl.k_units = nb;
    pl.k_levels = nlev;
    pl.unit_block = ublk;
    pl.unit_off = uoff;
    pl.unit_n = nsz;
    pl.kstruct = ustruct;
    pl.kt.resize(nb); pl.kcol.resize(nb); pl.kR.resize(nb); pl.krow_off.resize(nb);
    pl.tt_k.resize(nb); pl.drow_k.resize(nb);
    for (int j = 0; j < nb; ++j) pl.kt[j] = ceil_div(nsz[j], TILE);
    slot = 0;
    for (int j = 0; j < nb; ++j) {
        std::vector<int> &ro = pl.krow_off[j];
        ro.clear();
        int r = pl.kt[j];
        ro.push_back(0);
        for (int i : ustruct[j]) { ro.push_back(r); r += pl.kt[i]; }
        pl.kR[j] = r;
        pl.kcol[j] = slot;
        slot += (i64)r * pl.kt[j];
        pl.tt_k[j] = tt;
        tt += (i64)pl.kt[j] * pl.kt[j];
        pl.drow_k[j] = drow;
        drow += (i64)pl.kt[j] * TILE;
    }
    pl.k_tiles = slot;
    pl.tt_tiles = tt;
    pl.d_rows = drow;

    auto mrows = [&](int d, int a) {
        const Subdomain &S = dc.sub[d];
        return a < pl.TE[d] ? tile_rows(S.n, a) : tile_rows(S.m, a - pl.TE[d]);
    };
    // row-tile offset of block i inside the panel of block column j
    auto rowoff = [&](int j, int i) -> int {
        if (i == j) return 0;
        const auto &s = ustruct[j];
        auto it = std::lower_bound(s.begin(), s.end(), i);
        if (it == s.end() || *it != i) throw Error{-1, "internal: block not in struct"};
        return pl.krow_off[j][1 + (it - s.begin())];
    };
    auto kslot = [&](int j, int i, int a, int b) {  // block (i, j), tile (a, b)
        return pl.kcol[j] + (i64)b * pl.kR[j] + rowoff(j, i) + a;
    };
    auto E = [](int arr, i64 slot_) { return enc(arr, slot_ * TILE_ELEMS); };

    // ----------------------------- tile pattern of M_d after elimination --
    // nz[d][a][b] (b <= a): tile (a, b) of M_d is structurally nonzero after
    // the first TE[d] tile columns are eliminated.  Interchanges stay inside
    // a diagonal tile, so the tile pattern does not depend on the pivots.
    // Edges are numbered lexicographically from the mesh, so A_d is banded and
    // the multiplier rows meet only interface edges: most tiles stay zero and
    // are never touched (no panel, update or solve work on them).
    std::vector<std::vector<std::vector<char>>> nz(N);
    for (int d = 0; d < N; ++d) {
        const Subdomain &S = dc.sub[d];
        const int T = pl.T[d];
        auto &P = nz[d];
        P.assign(T, std::vector<char>(T, 0));
        for (int a = 0; a < T; ++a) P[a][a] = 1;
        for (size_t x = 0; x < S.a_row.size(); ++x) P[S.a_row[x] / TILE][S.a_col[x] / TILE] = 1;
        for (size_t ob = 0; ob < S.blocks.size(); ++ob) {
            const int Pb = S.blocks[ob];
            for (i64 l = dc.blk_start[Pb]; l < dc.blk_start[Pb + 1]; ++l) {
                const i64 r = (i64)pl.TE[d] * TILE + S.block_off[ob] + (l - dc.blk_start[Pb]);
                P[r / TILE][S.row_of(dc.lm_e[l]) / TILE] = 1;
            }
        }
        for (int j = 0; j < pl.TE[d]; ++j)
            for (int x = j + 1; x < T; ++x) {
                if (!P[x][j]) continue;
                for (int y = j + 1; y <= x; ++y)
                    if (P[y][j]) P[x][y] = 1;
            }
    }
    pl.s1_tiles = 0;
    for (int d = 0; d < N; ++d)
        for (int a = 0; a < pl.T[d]; ++a)
            for (int b = 0; b <= a && b < pl.TE[d]; ++b) pl.s1_tiles += nz[d][a][b];

    // ARR_M holds, per subdomain, only the structurally nonzero tiles of the
    // eliminated tile columns (column by column), then the whole trailing
    // multiplier triangle (tile (TE, TE) onwards, packed lower triangle),
    // which the assembly of -K reads at arbitrary row offsets.
    pl.m_cslot.assign(N, {});
    pl.m_tbase.assign(N, 0);
    slot = 0;
    for (int d = 0; d < N; ++d) {
        const int T = pl.T[d], TEd = pl.TE[d];
        auto &cs = pl.m_cslot[d];
        cs.assign((size_t)T * TEd, -1);
        for (int b = 0; b < TEd; ++b)
            for (int a = b; a < T; ++a)
                if (nz[d][a][b]) cs[(size_t)a * TEd + b] = slot++;
        pl.m_tbase[d] = slot;
        slot += tri_slot(pl.TL[d], 0);
    }
    pl.m_tiles = slot;
    auto mslot = [&](int d, int a, int b) -> i64 {
        const int TEd = pl.TE[d];
        if (b >= TEd) return pl.m_tbase[d] + tri_slot(a - TEd, b - TEd);
        const i64 x = pl.m_cslot[d][(size_t)a * TEd + b];
        if (x < 0) throw Error{-1, "internal: a zero tile of a subdomain matrix is addressed"};
        return x;
    };

    // --------------------------------------------- step 1 (subdomain) plan --
    // levels of the tile elimination tree of every M_d (parent of tile
    // column j: the first eliminated row tile below it that is structurally
    // nonzero); used with s1_tree
    std::vector<std::vector<int>> lev(N);
    int nl = 0;
    if (s1_tree)
        for (int d = 0; d < N; ++d) {
            lev[d].assign(pl.TE[d], 0);
            for (int j = 0; j < pl.TE[d]; ++j) {
                int par = -1;
                for (int a = j + 1; a < pl.TE[d] && par < 0; ++a)
                    if (nz[d][a][j]) par = a;
                if (par >= 0) lev[d][par] = std::max(lev[d][par], lev[d][j] + 1);
                nl = std::max(nl, lev[d][j] + 1);
            }
        }
    if (s1_tree) {
        // Steps by level of the tile elimination trees: the columns of one
        // level are independent (none lies in another's structure), so they
        // factor in one step, and each target tile gathers the pairs of all
        // of its step's columns in one task.  With a nested-dissection row
        // order the subtrees of the dissection run side by side; targets in
        // columns of the next level go first (the next step's pivots need
        // them), the rest may run on the look-ahead stream.
        for (int L = 0; L < nl; ++L) {
            FactorStep st;
            st.bk0 = (i64)pl.bk.size();
            for (int d = 0; d < N; ++d)
                for (int j = 0; j < pl.TE[d]; ++j) {
                    if (lev[d][j] != L) continue;
                    BkTask t{};
                    t.a = t.l = E(ARR_M, mslot(d, j, j));
                    t.tt = E(ARR_TT, pl.tt_s1[d] + j);
                    t.drow = pl.drow_s1[d] + (i64)j * TILE;
                    t.n = mrows(d, j);
                    t.ldt = 0;
                    t.status = (int)pl.bk.size();
                    pl.bk.push_back(t);
                    st.bk_maxn = std::max(st.bk_maxn, t.n);
                    pl.flops_s1 += 8.0 * t.n * (double)t.n * t.n / 6.0;
                }
            st.nbk = (i64)pl.bk.size() - st.bk0;
            st.pan0 = (i64)pl.gemm.size();
            st.sc0 = (i64)pl.scale.size();
            for (int d = 0; d < N; ++d)
                for (int j = 0; j < pl.TE[d]; ++j) {
                    if (lev[d][j] != L) continue;
                    const int w = mrows(d, j);
                    for (int a = j + 1; a < pl.T[d]; ++a) {
                        if (!nz[d][a][j]) continue;
                        pl.gemm.push_back({E(ARR_MX, mslot(d, a, j)), (int32_t)pl.pairs.size(), 1});
                        pl.pairs.push_back({E(ARR_M, mslot(d, a, j)), E(ARR_TT, pl.tt_s1[d] + j)});
                        ScaleTask sc{};
                        sc.x = E(ARR_MX, mslot(d, a, j));
                        sc.w = E(ARR_M, mslot(d, a, j));
                        sc.xprev = sc.xnext = -1;
                        sc.drow = pl.drow_s1[d] + (i64)j * TILE;
                        sc.ncols = w;
                        pl.scale.push_back(sc);
                        const double pf = 8.0 * mrows(d, a) * (double)w * w / 2.0;
                        st.pan_flops += pf;
                        pl.flops_s1 += pf;
                    }
                }
            st.npan = (i64)pl.gemm.size() - st.pan0;
            st.nsc = (i64)pl.scale.size() - st.sc0;
            st.fused_scale = st.npan == st.nsc;
            st.up0 = (i64)pl.gemm.size();
            for (int pass = 0; pass < 2; ++pass) {
                for (int d = 0; d < N; ++d) {
                    std::vector<int> cols;
                    for (int j = 0; j < pl.TE[d]; ++j)
                        if (lev[d][j] == L) cols.push_back(j);
                    if (cols.empty()) continue;
                    for (int b = cols.front() + 1; b < pl.T[d]; ++b) {
                        const bool crit = b < pl.TE[d] && lev[d][b] == L + 1;
                        if (crit != (pass == 0)) continue;
                        for (int a = b; a < pl.T[d]; ++a) {
                            GemmTask g{E(ARR_M, 0), (int32_t)pl.pairs.size(), 0};
                            const int ra = mrows(d, a), rb = mrows(d, b);
                            for (int j : cols) {
                                if (j >= b || !nz[d][a][j] || !nz[d][b][j]) continue;
                                pl.pairs.push_back({E(ARR_MX, mslot(d, a, j)), E(ARR_M, mslot(d, b, j))});
                                ++g.np;
                                const double f = 8.0 * mrows(d, j) * (a == b ? ra * (ra + 1) / 2.0 : (double)ra * rb);
                                st.up_flops += f;
                                if (pass == 0) st.crit_flops += f;
                            }
                            if (g.np == 0) continue;
                            g.c = E(ARR_M, mslot(d, a, b));
                            pl.gemm.push_back(g);
                        }
                    }
                }
                if (pass == 0) st.ncrit = (i64)pl.gemm.size() - st.up0;
            }
            st.nup = (i64)pl.gemm.size() - st.up0;
            pl.flops_s1 += st.up_flops;
            pl.flops_update += st.up_flops;
            pl.s1_steps.push_back(st);
        }
    }
    for (int j = 0; j < maxTE && !s1_tree; ++j) {
        FactorStep st;
        st.bk0 = (i64)pl.bk.size();
        for (int d = 0; d < N; ++d) {
            if (j >= pl.TE[d]) continue;
            BkTask t{};
            t.a = t.l = E(ARR_M, mslot(d, j, j));
            t.tt = E(ARR_TT, pl.tt_s1[d] + j);
            t.drow = pl.drow_s1[d] + (i64)j * TILE;
            t.n = mrows(d, j);
            t.ldt = 0;
            t.status = (int)pl.bk.size();
            pl.bk.push_back(t);
            st.bk_maxn = std::max(st.bk_maxn, t.n);
            pl.flops_s1 += 8.0 * t.n * (double)t.n * t.n / 6.0;
        }
        st.nbk = (i64)pl.bk.size() - st.bk0;
        // panels: X = M(a, j) P L^-T for every nonzero row tile below j
        st.pan0 = (i64)pl.gemm.size();
        st.sc0 = (i64)pl.scale.size();
        for (int d = 0; d < N; ++d) {
            if (j >= pl.TE[d]) continue;
            int w = mrows(d, j);
            for (int a = j + 1; a < pl.T[d]; ++a) {
                if (!nz[d][a][j]) continue;
                pl.gemm.push_back({E(ARR_MX, mslot(d, a, j)), (int32_t)pl.pairs.size(), 1});
                pl.pairs.push_back({E(ARR_M, mslot(d, a, j)), E(ARR_TT, pl.tt_s1[d] + j)});
                ScaleTask s{};
                s.x = E(ARR_MX, mslot(d, a, j));
                s.w = E(ARR_M, mslot(d, a, j));
                s.xprev = s.xnext = -1;
                s.drow = pl.drow_s1[d] + (i64)j * TILE;
                s.ncols = w;
                pl.scale.push_back(s);
                double pf = 8.0 * mrows(d, a) * (double)w * w / 2.0;
                st.pan_flops += pf;
                pl.flops_s1 += pf;
            }
        }
        st.npan = (i64)pl.gemm.size() - st.pan0;
        st.nsc = (i64)pl.scale.size() - st.sc0;
        st.fused_scale = st.npan == st.nsc;
        for (i64 x = st.sc0; x < st.sc0 + st.nsc && st.fused_scale; ++x)
            st.fused_scale = pl.scale[x].xprev < 0 && pl.scale[x].xnext < 0 &&
                             pl.scale[x].x == pl.gemm[st.pan0 + (x - st.sc0)].c;
        // Trailing updates M(a, b) -= sum_j' X(a, j') L-hat(b, j')^T, blocked
        // by S1_BLOCK tile columns [j0, jend): an inner step updates only the
        // remaining columns of its block (one pair per target), the last step
        // of a block updates every column beyond it with the pairs of all
        // the block's columns at once (the target tile is read and written
        // once per block).  Targets in the next block's columns come first.
        const int j0 = (j / S1_BLOCK) * S1_BLOCK, jend = std::min(j0 + S1_BLOCK, maxTE);
        st.up0 = (i64)pl.gemm.size();
        if (j + 1 < jend) {
            for (int d = 0; d < N; ++d) {
                if (j >= pl.TE[d]) continue;
                const int w = mrows(d, j);
                for (int b = j + 1; b < std::min(jend, pl.T[d]); ++b) {
                    if (!nz[d][b][j]) continue;
                    for (int a = b; a < pl.T[d]; ++a) {
                        if (!nz[d][a][j]) continue;
                        pl.gemm.push_back({E(ARR_M, mslot(d, a, b)), (int32_t)pl.pairs.size(), 1});
                        pl.pairs.push_back({E(ARR_MX, mslot(d, a, j)), E(ARR_M, mslot(d, b, j))});
                        int ra = mrows(d, a), rb = mrows(d, b);
                        st.up_flops += 8.0 * w * (a == b ? ra * (ra + 1) / 2.0 : (double)ra * rb);
                    }
                }
            }
            st.ncrit = (i64)pl.gemm.size() - st.up0;
            st.crit_flops = st.up_flops;
            st.wait_rest = false;
        } else {
            for (int pass = 0; pass < 2; ++pass) {
                for (int d = 0; d < N; ++d) {
                    const int jlast = std::min(jend, pl.TE[d]);
                    if (j0 >= jlast) continue;
                    for (int b = jend; b < pl.T[d]; ++b) {
                        if ((b < jend + S1_BLOCK) != (pass == 0)) continue;
                        for (int a = b; a < pl.T[d]; ++a) {
                            if (b < pl.TE[d] && !nz[d][a][b]) continue;  // no pair reaches a zero tile
                            GemmTask g{E(ARR_M, mslot(d, a, b)), (int32_t)pl.pairs.size(), 0};
                            const int ra = mrows(d, a), rb = mrows(d, b);
                            for (int jj = j0; jj < jlast; ++jj) {
                                if (!nz[d][a][jj] || !nz[d][b][jj]) continue;
                                pl.pairs.push_back({E(ARR_MX, mslot(d, a, jj)), E(ARR_M, mslot(d, b, jj))});
                                ++g.np;
                                const double f = 8.0 * mrows(d, jj) * (a == b ? ra * (ra + 1) / 2.0 : (double)ra * rb);
                                st.up_flops += f;
                                if (pass == 0) st.crit_flops += f;
                            }
                            if (g.np > 0) pl.gemm.push_back(g);
                        }
                    }
                }
                if (pass == 0) st.ncrit = (i64)pl.gemm.size() - st.up0;
            }
        }
        st.nup = (i64)pl.gemm.size() - st.up0;
        pl.flops_s1 += st.up_flops;
        pl.flops_update += st.up_flops;
        pl.s1_steps.push_back(st);
    }

    // --------------------------------------------- step 2 (assembly) plan --
    // -K(i, j) = sum over subdomains d holding both blocks of the trailing
    // block of M_d at the rows of block i and the columns of block j
    for (int j = 0; j < nb; ++j) {
        int Q = ublk[j];
        std::vector<int> rows_blocks{j};
        rows_blocks.insert(rows_blocks.end(), ustruct[j].begin(), ustruct[j].end());
        for (int i : rows_blocks) {
            int P = ublk[i];
            std::vector<int> common;
            for (int dP : {dc.blk_p[P], dc.blk_q[P]})
                for (int dQ : {dc.blk_p[Q], dc.blk_q[Q]})
                    if (dP == dQ && std::find(common.begin(), common.end(), dP) == common.end())
                        common.push_back(dP);
            for (int b = 0; b < pl.kt[j]; ++b)
                for (int a = (i == j ? b : 0); a < pl.kt[i]; ++a) {
                    AsmTask t{};
                    t.dst = E(ARR_K, kslot(j, i, a, b));
                    t.nrow = tile_rows(nsz[i], a);
                    t.ncol = tile_rows(nsz[j], b);
                    t.ncontrib = (int)common.size();
                    for (size_t c = 0; c < common.size(); ++c) {
                        int d = common[c];
                        const Subdomain &S = dc.sub[d];
                        auto oP = std::lower_bound(S.blocks.begin(), S.blocks.end(), P) - S.blocks.begin();
                        auto oQ = std::lower_bound(S.blocks.begin(), S.blocks.end(), Q) - S.blocks.begin();
                        t.mbase[c] = pl.m_tbase[d];
                        t.row0[c] = (int32_t)(S.block_off[oP] + uoff[i] + (i64)a * TILE);
                        t.col0[c] = (int32_t)(S.block_off[oQ] + uoff[j] + (i64)b * TILE);
                    }
                    pl.asmb.push_back(t);
                }
        }
    }

    // ------------------------------------- step 5 (block LDL^T of -K) plan --
    std::vector<std::vector<int>> by_level(nlev);
    for (int j = 0; j < nb; ++j) by_level[ulevel[j]].push_back(j);
    // Chain blocking of the trailing updates (the tree analogue of S1_BLOCK):
    // consecutive units of an elimination-tree chain (each the only child of
    // the next), at most K_BLOCK long, form a segment.  A unit updates the
    // columns of the later units of its segment at once (the next one needs
    // them); its updates of every column beyond the segment are delayed to
    // the step of the segment's last unit, which applies the pairs of all the
    // segment's units together (one read-modify-write of each target per
    // segment).  Every column k beyond the segment belongs to an ancestor of
    // the segment's last unit, so its updates still land before its step.
    std::vector<int> nchild(nb, 0), seg_last(nb), seg_len(nb, 1), seg_of(nb);
    for (int j = 0; j < nb; ++j)
        if (!ustruct[j].empty()) nchild[ustruct[j][0]]++;
    for (int j = 0; j < nb; ++j) seg_of[j] = j;
    for (int j = 0; j < nb; ++j) {
        if (ustruct[j].empty()) continue;
        const int p = ustruct[j][0];
        if (nchild[p] == 1 && seg_len[seg_of[j]] < K_BLOCK) {
            seg_of[p] = seg_of[j];
            seg_len[seg_of[j]]++;
        }
    }
    for (int j = 0; j < nb; ++j) seg_last[seg_of[j]] = j;  // units of a segment increase along the chain
    std::vector<std::vector<int>> delayed(nb);  // per segment end: units whose updates it applies
    // With one-tile units, the updates of the next level's columns (the
    // critical ones) are not launched on their own: the pivot launch of the
    // next level applies the pairs of its diagonal tile before factoring it,
    // and its panel launch those of each panel tile before the product.
    const bool fuse_next = k_fuse && unit_max > 0 && unit_max <= TILE;
    std::map<std::pair<int, int>, std::vector<GemmPair>> pending;  // (unit k, row unit i) -> pairs
    const int LDS_MAX_N = 136;
    for (int L = 0; L < nlev; ++L) {
        const auto &J = by_level[L];
        FactorStep st;
        st.bk0 = (i64)pl.bk.size();
        for (int j : J) {
            BkTask t{};
            t.a = E(ARR_K, pl.kcol[j]);
            t.l = E(ARR_KL, pl.kcol[j]);
            t.tt = E(ARR_TT, pl.tt_k[j]);
            t.drow = pl.drow_k[j];
            t.n = nsz[j];
            t.ldt = (int32_t)((i64)pl.kR[j] * TILE_ELEMS);
            t.status = (int)pl.bk.size();
            auto pd = pending.find({j, j});
            if (pd != pending.end()) {
                t.p0 = (int32_t)pl.pairs.size();
                t.np = (int32_t)pd->second.size();
                pl.pairs.insert(pl.pairs.end(), pd->second.begin(), pd->second.end());
            }
            pl.bk.push_back(t);
            st.bk_maxn = std::max(st.bk_maxn, t.n);
            pl.flops_s3 += 8.0 * (double)t.n * t.n * t.n / 6.0;
        }
        st.nbk = (i64)pl.bk.size() - st.bk0;
        if (st.bk_maxn > LDS_MAX_N)
            pl.bk_scratch_elems = std::max<i64>(pl.bk_scratch_elems,
                                                st.nbk * ((i64)st.bk_maxn * (st.bk_maxn + 1) / 2));
        st.pan0 = (i64)pl.gemm.size();
        st.sc0 = (i64)pl.scale.size();
        for (int j : J) {
            int tj = pl.kt[j];
            for (int i : ustruct[j])
                for (int a = 0; a < pl.kt[i]; ++a)
                    for (int b = 0; b < tj; ++b) {
                        pl.gemm.push_back({E(ARR_KX, kslot(j, i, a, b)), (int32_t)pl.pairs.size(), tj});
                        for (int c = 0; c < tj; ++c)
                            pl.pairs.push_back({E(ARR_K, kslot(j, i, a, c)),
                                                E(ARR_TT, pl.tt_k[j] + (i64)c * tj + b)});
                        ScaleTask s{};
                        s.x = E(ARR_KX, kslot(j, i, a, b));
                        s.w = E(ARR_KL, kslot(j, i, a, b));
                        s.xprev = b > 0 ? E(ARR_KX, kslot(j, i, a, b - 1)) : -1;
                        s.xnext = b + 1 < tj ? E(ARR_KX, kslot(j, i, a, b + 1)) : -1;
                        s.drow = pl.drow_k[j] + (i64)b * TILE;
                        s.ncols = tile_rows(nsz[j], b);
                        auto pd = pending.find({j, i});
                        if (pd != pending.end()) {
                            s.q0 = (int32_t)pl.pairs.size();
                            s.nq = (int32_t)pd->second.size();
                            pl.pairs.insert(pl.pairs.end(), pd->second.begin(), pd->second.end());
                        }
                        pl.scale.push_back(s);
                    }
            double pf = 0.0;
            for (int i : ustruct[j]) pf += 8.0 * nsz[i] * (double)nsz[j] * nsz[j] / 2.0;
            st.pan_flops += pf;
            pl.flops_s3 += pf;
        }
        st.npan = (i64)pl.gemm.size() - st.pan0;
        st.nsc = (i64)pl.scale.size() - st.sc0;
        st.fused_scale = st.npan == st.nsc;
        for (i64 x = st.sc0; x < st.sc0 + st.nsc && st.fused_scale; ++x)
            st.fused_scale = pl.scale[x].xprev < 0 && pl.scale[x].xnext < 0 &&
                             pl.scale[x].x == pl.gemm[st.pan0 + (x - st.sc0)].c;
        // updates grouped by target block so that every target tile is
        // written by exactly one work-group (deterministic, atomic-free)
        std::map<std::pair<int, int>, std::vector<int>> targets;
        for (int j : J) {
            const int f = seg_last[seg_of[j]];
            for (size_t x = 0; x < ustruct[j].size(); ++x)
                for (size_t y = 0; y <= x; ++y) {
                    const int k = ustruct[j][y];
                    if (f == j || k <= f) targets[{ustruct[j][x], k}].push_back(j);
                }
            if (f != j) delayed[f].push_back(j);
        }
        for (int f : J)
            for (int j : delayed[f])  // columns beyond the segment, from its earlier units
                for (size_t x = 0; x < ustruct[j].size(); ++x)
                    for (size_t y = 0; y <= x; ++y)
                        if (ustruct[j][y] > f) targets[{ustruct[j][x], ustruct[j][y]}].push_back(j);
        for (auto &kv : targets) std::sort(kv.second.begin(), kv.second.end());
        // targets in block columns of the next level first (critical), then
        // those of the next few levels (near: the next chain segment needs
        // them soon), then the rest (far); each group is one launch, and the
        // columns each launch writes are recorded for the dependency waits
        st.up0 = (i64)pl.gemm.size();
        st.track = true;
        st.cols_bk.assign(J.begin(), J.end());
        auto group = [&](int k) { return ulevel[k] == L + 1 ? 0 : (ulevel[k] <= L + 1 + K_BLOCK ? 1 : 2); };
        for (int pass = 0; pass < 3; ++pass) {
            std::vector<int> &cols = pass == 0 ? st.cols_crit : (pass == 1 ? st.cols_near : st.cols_far);
            for (auto &kv : targets) {
                int i = kv.first.first, k = kv.first.second;
                if (group(k) != pass) continue;
                if (cols.empty() || cols.back() != k) cols.push_back(k);
                if (pass == 0 && fuse_next) {  // applied by the next level's pivot and panel launches
                    auto &pd = pending[{k, i}];
                    const int ra = tile_rows(nsz[i], 0), rb = tile_rows(nsz[k], 0);
                    for (int j : kv.second) {
                        pd.push_back({E(ARR_KX, kslot(j, i, 0, 0)), E(ARR_KL, kslot(j, k, 0, 0))});
                        const double f = 8.0 * tile_rows(nsz[j], 0) * (i == k ? ra * (ra + 1) / 2.0 : (double)ra * rb);
                        pl.flops_s3 += f;
                    }
                    continue;
                }
                for (int b = 0; b < pl.kt[k]; ++b)
                    for (int a = (i == k ? b : 0); a < pl.kt[i]; ++a) {
                        GemmTask g{E(ARR_K, kslot(k, i, a, b)), (int32_t)pl.pairs.size(), 0};
                        int ra = tile_rows(nsz[i], a), rb = tile_rows(nsz[k], b);
                        for (int j : kv.second)
                            for (int c = 0; c < pl.kt[j]; ++c) {
                                pl.pairs.push_back({E(ARR_KX, kslot(j, i, a, c)), E(ARR_KL, kslot(j, k, b, c))});
                                ++g.np;
                                int w = tile_rows(nsz[j], c);
                                double f = 8.0 * w * ((i == k && a == b) ? ra * (ra + 1) / 2.0 : (double)ra * rb);
                                st.up_flops += f;
                                if (pass == 0) st.crit_flops += f;
                                if (pass == 1) st.near_flops += f;
                            }
                        pl.gemm.push_back(g);
                    }
            }
            if (pass == 0) st.ncrit = (i64)pl.gemm.size() - st.up0;
            if (pass == 1) st.nnear = (i64)pl.gemm.size() - st.up0 - st.ncrit;
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        }
        st.nup = (i64)pl.gemm.size() - st.up0;
        pl.flops_s3 += st.up_flops;
        pl.flops_update += st.up_flops;
        pl.k_steps.push_back(st);
    }
    pl.n_status = (int)pl.bk.size();

    // ------------------------------------------------ scatter of A_d, D_d --
    pl.coo_off.clear();
    for (int d = 0; d < N; ++d) {
        const Subdomain &S = dc.sub[d];
        for (size_t x = 0; x < S.a_row.size(); ++x) {
            i64 r = S.a_row[x], c = S.a_col[x];
            pl.coo_off.push_back(mslot(d, (int)(r / TILE), (int)(c / TILE)) * TILE_ELEMS + (c % TILE) * TILE + r % TILE);
        }
    }
    pl.n_coo_a = (i64)pl.coo_off.size();
    for (int d = 0; d < N; ++d) {
        const Subdomain &S = dc.sub[d];
        for (size_t ob = 0; ob < S.blocks.size(); ++ob) {
            int P = S.blocks[ob];
            for (i64 l = dc.blk_start[P]; l < dc.blk_start[P + 1]; ++l) {
                i64 r = (i64)pl.TE[d] * TILE + S.block_off[ob] + (l - dc.blk_start[P]);
                i64 c = S.row_of(dc.lm_e[l]);
                pl.coo_off.push_back(mslot(d, (int)(r / TILE), (int)(c / TILE)) * TILE_ELEMS + (c % TILE) * TILE + r % TILE);
            }
        }
    }

    // ------------------------------------------------------ solve plan ----
    pl.vs1.resize(N);
    i64 v = 0;
    for (int d = 0; d < N; ++d) { pl.vs1[d] = v; v += pl.T[d]; }
    pl.v_tiles_s1 = v;
    pl.vk.resize(nb);
    v = 0;
    for (int j = 0; j < nb; ++j) { pl.vk[j] = v; v += pl.kt[j]; }
    pl.v_tiles_k = v;
    auto V = [](int arr, i64 tile) { return enc(arr, tile); };

    pl.split_map.assign(pl.v_tiles_s1 * TILE, -1);
    for (int d = 0; d < N; ++d) {
        const Subdomain &S = dc.sub[d];
        for (i64 r = 0; r < S.n; ++r) {
            i64 e = S.edges[r];
            if (e >= 0 && dc.owner[e] == d) pl.split_map[pl.vs1[d] * TILE + r] = e;
        }
    }
    pl.collect_map.assign(dc.owner.size(), -1);
    for (size_t e = 0; e < dc.owner.size(); ++e) {
        int d = dc.owner[e];
        pl.collect_map[e] = pl.vs1[d] * TILE + dc.sub[d].row_of((i64)e);
    }
    pl.copy_map.assign(pl.v_tiles_s1 * TILE, -1);
    for (int d = 0; d < N; ++d) {
        const Subdomain &S = dc.sub[d];
        for (i64 r = 0; r < S.n; ++r) {
            const i64 e = S.edges[r];
            if (e >= 0 && dc.owner[e] != d) pl.copy_map[pl.vs1[d] * TILE + r] = pl.collect_map[e];
        }
    }
    // multiplier rows: K vector row <-> the two subdomain copies
    std::vector<i64> &kvrow_of_lm = pl.lm_vrow;
    kvrow_of_lm.assign(dc.n_lm, -1);
    for (int j = 0; j < nb; ++j) {
        int P = ublk[j];
        for (int o = 0; o < nsz[j]; ++o)
            kvrow_of_lm[dc.blk_start[P] + uoff[j] + o] = pl.vk[j] * TILE + o;
    }
    std::vector<int64_t> &hmap = pl.h_map;
    hmap.assign(pl.v_tiles_k * TILE * 2, -1);
    std::vector<int64_t> &lmap = pl.lam_map;
    lmap.assign(pl.v_tiles_s1 * TILE, -1);
    for (int d = 0; d < N; ++d) {
        const Subdomain &S = dc.sub[d];
        for (size_t ob = 0; ob < S.blocks.size(); ++ob) {
            int P = S.blocks[ob];
            for (i64 l = dc.blk_start[P]; l < dc.blk_start[P + 1]; ++l) {
                i64 srow = pl.vs1[d] * TILE + (i64)pl.TE[d] * TILE + S.block_off[ob] + (l - dc.blk_start[P]);
                i64 kr = kvrow_of_lm[l];
                int slotc = hmap[2 * kr] < 0 ? 0 : 1;
                hmap[2 * kr + slotc] = srow;
                lmap[srow] = kr;
            }
        }
    }

    // S1 forward
    // (s1_tree: by levels of the tile elimination trees, as the
    // factorisation: a level's diagonal solves, then every row tile below
    // its columns receives their products in one task)
    for (int L = 0; L < nl && s1_tree; ++L) {
        SolveStep st;
        st.dg0 = (i64)pl.vdiag.size();
        for (int d = 0; d < N; ++d)
            for (int j = 0; j < pl.TE[d]; ++j) {
                if (lev[d][j] != L) continue;
                VDiagTask t{};
                t.tt = E(ARR_TT, pl.tt_s1[d] + j);
                t.x = V(V_X, pl.vs1[d] + j); t.y = V(V_Y, pl.vs1[d] + j); t.v = V(V_V, pl.vs1[d] + j);
                t.acc = -1;
                t.drow = pl.drow_s1[d] + (i64)j * TILE;
                t.t = 1; t.n = mrows(d, j);
                pl.vdiag.push_back(t);
            }
        st.ndg = (i64)pl.vdiag.size() - st.dg0;
        st.up0 = (i64)pl.vupd.size();
        st.up_mode = 0;
        for (int d = 0; d < N; ++d) {
            std::vector<int> cols;
            for (int j = 0; j < pl.TE[d]; ++j)
                if (lev[d][j] == L) cols.push_back(j);
            if (cols.empty()) continue;
            for (int a = cols.front() + 1; a < pl.T[d]; ++a) {
                const int32_t p0 = (int32_t)pl.vpairs.size();
                for (int j : cols)
                    if (j < a && nz[d][a][j]) pl.vpairs.push_back({E(ARR_M, mslot(d, a, j)), V(V_Y, pl.vs1[d] + j)});
                const int32_t np = (int32_t)pl.vpairs.size() - p0;
                if (np > 0) pl.vupd.push_back({V(V_X, pl.vs1[d] + a), p0, np});
            }
        }
        st.nup = (i64)pl.vupd.size() - st.up0;
        pl.s1_fwd.push_back(st);
    }
    for (int j = 0; j < maxTE && !s1_tree; ++j) {
        SolveStep st;
        st.dg0 = (i64)pl.vdiag.size();
        for (int d = 0; d < N; ++d) {
            if (j >= pl.TE[d]) continue;
            VDiagTask t{};
            t.tt = E(ARR_TT, pl.tt_s1[d] + j);
            t.x = V(V_X, pl.vs1[d] + j); t.y = V(V_Y, pl.vs1[d] + j); t.v = V(V_V, pl.vs1[d] + j);
            t.acc = -1;
            t.drow = pl.drow_s1[d] + (i64)j * TILE;
            t.t = 1; t.n = mrows(d, j);
            pl.vdiag.push_back(t);
        }
        st.ndg = (i64)pl.vdiag.size() - st.dg0;
        st.up0 = (i64)pl.vupd.size();
        st.up_mode = 0;
        // Tile columns are taken S1_BLOCK at a time, as in the factorisation:
        // rows inside the column's block get its product at once (they are
        // solved next), rows beyond it receive the products of all the
        // block's columns in one task at the block's last column (one
        // read-modify-write of the target instead of one per column).
        for (int d = 0; d < N; ++d) {
            if (j >= pl.TE[d]) continue;
            const int j0 = j / S1_BLOCK * S1_BLOCK, je = std::min(j0 + S1_BLOCK, pl.TE[d]) - 1;
            for (int a = j + 1; a <= je; ++a) {
                if (!nz[d][a][j]) continue;
                pl.vupd.push_back({V(V_X, pl.vs1[d] + a), (int32_t)pl.vpairs.size(), 1});
                pl.vpairs.push_back({E(ARR_M, mslot(d, a, j)), V(V_Y, pl.vs1[d] + j)});
            }
            if (j != je) continue;
            for (int a = je + 1; a < pl.T[d]; ++a) {
                const int32_t p0 = (int32_t)pl.vpairs.size();
                for (int c = j0; c <= je; ++c)
                    if (nz[d][a][c]) pl.vpairs.push_back({E(ARR_M, mslot(d, a, c)), V(V_Y, pl.vs1[d] + c)});
                const int32_t np = (int32_t)pl.vpairs.size() - p0;
                if (np > 0) pl.vupd.push_back({V(V_X, pl.vs1[d] + a), p0, np});
            }
        }
        st.nup = (i64)pl.vupd.size() - st.up0;
        pl.s1_fwd.push_back(st);
    }
    // K forward / backward
    for (int L = 0; L < nlev; ++L) {
        SolveStep st;
        st.dg0 = (i64)pl.vdiag.size();
        for (int j : by_level[L]) {
            VDiagTask t{};
            t.tt = E(ARR_TT, pl.tt_k[j]);
            t.x = V(V_KX, pl.vk[j]); t.y = V(V_KY, pl.vk[j]); t.v = V(V_KV, pl.vk[j]);
            t.acc = -1;
            t.drow = pl.drow_k[j];
            t.t = pl.kt[j]; t.n = nsz[j];
            st.dg_maxt = std::max(st.dg_maxt, (int)t.t);
            pl.vdiag.push_back(t);
        }
        st.ndg = (i64)pl.vdiag.size() - st.dg0;
        std::map<int, std::vector<int>> targets;
        for (int j : by_level[L])
            for (int i : ustruct[j]) targets[i].push_back(j);
        st.up0 = (i64)pl.vupd.size();
        st.up_mode = 0;
        for (auto &kv : targets) {
            int i = kv.first;
            for (int a = 0; a < pl.kt[i]; ++a) {
                VUpdTask u{V(V_KX, pl.vk[i] + a), (int32_t)pl.vpairs.size(), 0};
                for (int j : kv.second)
                    for (int c = 0; c < pl.kt[j]; ++c) {
                        pl.vpairs.push_back({E(ARR_KL, kslot(j, i, a, c)), V(V_KY, pl.vk[j] + c)});
                        ++u.np;
                    }
                pl.vupd.push_back(u);
            }
        }
        st.nup = (i64)pl.vupd.size() - st.up0;
        pl.k_fwd.push_back(st);
    }
    // backward over K, right-looking: after the diagonal solves of a level,
    // its multipliers are pushed into the accumulators of every descendant
    // that holds them in its struct, grouped by target (deterministic)
    std::vector<std::map<int, std::vector<int>>> push(nlev);
    for (int c = 0; c < nb; ++c)
        for (int i : ustruct[c]) push[ulevel[i]][c].push_back(i);
    for (int L = nlev - 1; L >= 0; --L) {
        SolveStep st;
        st.dg0 = (i64)pl.vdiag.size();
        for (int j : by_level[L]) {
            VDiagTask t{};
            t.tt = E(ARR_TT, pl.tt_k[j]);
            t.x = V(V_KX, pl.vk[j]); t.y = -1; t.v = V(V_KV, pl.vk[j]);
            t.acc = V(V_KACC, pl.vk[j]);
            t.drow = pl.drow_k[j];
            t.t = pl.kt[j]; t.n = nsz[j];
            st.dg_maxt = std::max(st.dg_maxt, (int)t.t);
            pl.vdiag.push_back(t);
        }
        st.ndg = (i64)pl.vdiag.size() - st.dg0;
        st.up0 = (i64)pl.vupd.size();
        st.up_mode = 2;
        for (auto &kv : push[L]) {
            const int c = kv.first;
            for (int b = 0; b < pl.kt[c]; ++b) {
                VUpdTask u{V(V_KACC, pl.vk[c] + b), (int32_t)pl.vpairs.size(), 0};
                for (int i : kv.second)
                    for (int a = 0; a < pl.kt[i]; ++a) {
                        pl.vpairs.push_back({E(ARR_KL, kslot(c, i, a, b)), V(V_KX, pl.vk[i] + a)});
                        ++u.np;
                    }
                pl.vupd.push_back(u);
            }
        }
        st.nup = (i64)pl.vupd.size() - st.up0;
        pl.k_bwd.push_back(st);
    }
    // S1 backward: first the multiplier rows' contribution, then tile columns
    {
        SolveStep st;
        st.ndg = 0;
        st.up_first = true;
        st.up0 = (i64)pl.vupd.size();
        st.up_mode = 1;
        for (int d = 0; d < N; ++d)
            for (int c = 0; c < pl.TE[d]; ++c) {
                VUpdTask u{V(V_ACC, pl.vs1[d] + c), (int32_t)pl.vpairs.size(), 0};
                for (int a = pl.TE[d]; a < pl.T[d]; ++a) {
                    if (!nz[d][a][c]) continue;
                    pl.vpairs.push_back({E(ARR_M, mslot(d, a, c)), V(V_X, pl.vs1[d] + a)});
                    ++u.np;
                }
                pl.vupd.push_back(u);
            }
        st.nup = (i64)pl.vupd.size() - st.up0;
        pl.s1_bwd.push_back(st);
    }
    // (s1_tree: by levels from the top, a level's diagonal solves, then each
    // accumulator below its columns receives their products in one task)
    for (int L = nl - 1; L >= 0 && s1_tree; --L) {
        SolveStep st;
        st.dg0 = (i64)pl.vdiag.size();
        for (int d = 0; d < N; ++d)
            for (int j = 0; j < pl.TE[d]; ++j) {
                if (lev[d][j] != L) continue;
                VDiagTask t{};
                t.tt = E(ARR_TT, pl.tt_s1[d] + j);
                t.x = V(V_X, pl.vs1[d] + j); t.y = -1; t.v = V(V_V, pl.vs1[d] + j);
                t.acc = V(V_ACC, pl.vs1[d] + j);
                t.drow = pl.drow_s1[d] + (i64)j * TILE;
                t.t = 1; t.n = mrows(d, j);
                pl.vdiag.push_back(t);
            }
        st.ndg = (i64)pl.vdiag.size() - st.dg0;
        st.up0 = (i64)pl.vupd.size();
        st.up_mode = 2;
        for (int d = 0; d < N; ++d) {
            std::vector<int> cols;
            for (int j = 0; j < pl.TE[d]; ++j)
                if (lev[d][j] == L) cols.push_back(j);
            if (cols.empty()) continue;
            for (int c = 0; c < cols.back(); ++c) {
                const int32_t p0 = (int32_t)pl.vpairs.size();
                for (int j : cols)
                    if (c < j && nz[d][j][c]) pl.vpairs.push_back({E(ARR_M, mslot(d, j, c)), V(V_X, pl.vs1[d] + j)});
                const int32_t np = (int32_t)pl.vpairs.size() - p0;
                if (np > 0) pl.vupd.push_back({V(V_ACC, pl.vs1[d] + c), p0, np});
            }
        }
        st.nup = (i64)pl.vupd.size() - st.up0;
        pl.s1_bwd.push_back(st);
    }
    for (int j = maxTE - 1; j >= 0 && !s1_tree; --j) {
        SolveStep st;
        st.dg0 = (i64)pl.vdiag.size();
        for (int d = 0; d < N; ++d) {
            if (j >= pl.TE[d]) continue;
            VDiagTask t{};
            t.tt = E(ARR_TT, pl.tt_s1[d] + j);
            t.x = V(V_X, pl.vs1[d] + j); t.y = -1; t.v = V(V_V, pl.vs1[d] + j);
            t.acc = V(V_ACC, pl.vs1[d] + j);
            t.drow = pl.drow_s1[d] + (i64)j * TILE;
            t.t = 1; t.n = mrows(d, j);
            pl.vdiag.push_back(t);
        }
        st.ndg = (i64)pl.vdiag.size() - st.dg0;
        st.up0 = (i64)pl.vupd.size();
        st.up_mode = 2;
        for (int d = 0; d < N; ++d) {
            if (j >= pl.TE[d]) continue;
            for (int c = 0; c < j; ++c) {
                if (!nz[d][j][c]) continue;
                pl.vupd.push_back({V(V_ACC, pl.vs1[d] + c), (int32_t)pl.vpairs.size(), 1});
                pl.vpairs.push_back({E(ARR_M, mslot(d, j, c)), V(V_X, pl.vs1[d] + j)});
            }
        }
        st.nup = (i64)pl.vupd.size() - st.up0;
        pl.s1_bwd.push_back(st);
    }

    // ------------------------------------------- fused update + diagonal --
    // An update task of step s whose target is the input of a one-tile
    // diagonal solve of step s + 1 is the last update that input receives
    // (forward sweeps update blocks of later steps only from earlier ones,
    // backward sweeps push into blocks of the next step from this one at the
    // latest), so the task goes on with that solve.  The next step keeps only
    // the diagonal solves not so fused, moved to the front of its range.
    pl.vfuse.assign(pl.vupd.size(), -1);
    auto fuse_sweep = [&](std::vector<SolveStep> &steps, bool bwd) {
        for (size_t q = 0; q + 1 < steps.size(); ++q) {
            SolveStep &cur = steps[q], &nxt = steps[q + 1];
            if (nxt.dg_maxt > 1 || nxt.ndg == 0 || cur.nup == 0) continue;
            std::map<i64, i64> key2diag;
            for (i64 i = nxt.dg0; i < nxt.dg0 + nxt.ndg; ++i) key2diag[bwd ? pl.vdiag[i].acc : pl.vdiag[i].x] = i;
            std::vector<i64> fused_by(nxt.ndg, -1);  // update task fusing diag i
            for (i64 u = cur.up0; u < cur.up0 + cur.nup; ++u) {
                auto it = key2diag.find(pl.vupd[u].out);
                if (it == key2diag.end() || fused_by[it->second - nxt.dg0] >= 0) continue;
                fused_by[it->second - nxt.dg0] = u;
            }
            std::vector<VDiagTask> keep, moved;
            std::vector<i64> moved_by;
            for (i64 i = 0; i < nxt.ndg; ++i) {
                if (fused_by[i] < 0) keep.push_back(pl.vdiag[nxt.dg0 + i]);
                else { moved.push_back(pl.vdiag[nxt.dg0 + i]); moved_by.push_back(fused_by[i]); }
            }
            i64 at = nxt.dg0;
            for (auto &t : keep) pl.vdiag[at++] = t;
            for (size_t m = 0; m < moved.size(); ++m) {
                pl.vfuse[moved_by[m]] = at;
                pl.vdiag[at++] = moved[m];
            }
            nxt.ndg = (i64)keep.size();
        }
    };
    fuse_sweep(pl.s1_fwd, false);
    fuse_sweep(pl.k_fwd, false);
    fuse_sweep(pl.k_bwd, true);
    fuse_sweep(pl.s1_bwd, true);

    // -------------------- S1 sweeps as one ordered task list per subdomain --
    // (tuning solve_seq) Left-looking: each target tile of a subdomain is
    // written by one task that gathers every product it needs, so one
    // work-group can run a subdomain's whole sweep in order with no
    // read-modify-write of partial sums.  Forward: x_j -= sum_{c<j} L(j,c) y_c
    // fused with y_j = TT_j x_j, v_j = D_j^{-1} y_j, for the tile columns in
    // order, then the multiplier rows a: x_a -= sum_c L(a,c) y_c.  Backward:
    // for j from the last column down, acc_j = sum_{a>j} L(a,j)^T x_a fused
    // with x_j = TT_j^T (v_j - acc_j) (x_a of the multiplier rows is lambda).
    pl.sq_fwd_off.assign(N + 1, 0);
    pl.sq_bwd_off.assign(N + 1, 0);
    auto s1_diag = [&](int d, int j, bool bwd) {
        VDiagTask t{};
        t.tt = E(ARR_TT, pl.tt_s1[d] + j);
        t.x = V(V_X, pl.vs1[d] + j);
        t.y = bwd ? -1 : V(V_Y, pl.vs1[d] + j);
        t.v = V(V_V, pl.vs1[d] + j);
        t.acc = bwd ? V(V_ACC, pl.vs1[d] + j) : -1;
        t.drow = pl.drow_s1[d] + (i64)j * TILE;
        t.t = 1;
        t.n = mrows(d, j);
        pl.vdiag.push_back(t);
        return (i64)pl.vdiag.size() - 1;
    };
    for (int d = 0; d < N; ++d) {
        pl.sq_fwd_off[d] = (i64)pl.vupd.size();
        for (int a = 0; a < pl.T[d]; ++a) {
            VUpdTask u{V(V_X, pl.vs1[d] + a), (int32_t)pl.vpairs.size(), 0};
            for (int c = 0; c < std::min(a, pl.TE[d]); ++c)
                if (nz[d][a][c]) {
                    pl.vpairs.push_back({E(ARR_M, mslot(d, a, c)), V(V_Y, pl.vs1[d] + c)});
                    ++u.np;
                }
            pl.vupd.push_back(u);
            pl.vfuse.push_back(a < pl.TE[d] ? s1_diag(d, a, false) : -1);
        }
    }
    pl.sq_fwd_off[N] = (i64)pl.vupd.size();
    for (int d = 0; d < N; ++d) {
        pl.sq_bwd_off[d] = (i64)pl.vupd.size();
        for (int j = pl.TE[d] - 1; j >= 0; --j) {
            VUpdTask u{V(V_ACC, pl.vs1[d] + j), (int32_t)pl.vpairs.size(), 0};
            for (int a = j + 1; a < pl.T[d]; ++a)
                if (nz[d][a][j]) {
                    pl.vpairs.push_back({E(ARR_M, mslot(d, a, j)), V(V_X, pl.vs1[d] + a)});
                    ++u.np;
                }
            pl.vupd.push_back(u);
            pl.vfuse.push_back(s1_diag(d, j, true));
        }
    }
    pl.sq_bwd_off[N] = (i64)pl.vupd.size();
    if (pl.vfuse.size() != pl.vupd.size()) throw Error{-1, "internal: fused-solve index list out of step"};
    for (VUpdTask &u : pl.vupd)
        if (u.np > 0) { u.l0 = pl.vpairs[u.p0].l; u.src0 = pl.vpairs[u.p0].src; }

    // ------------------------------------------------ algorithmic counts --
    i64 ent = 0;
    for (int d = 0; d < N; ++d)  // stored factor tiles of step 1 (diagonal ones are half)
        for (int a = 0; a < pl.T[d]; ++a)
            for (int b = 0; b <= a && b < pl.TE[d]; ++b)
                if (nz[d][a][b]) ent += (a == b) ? (i64)mrows(d, a) * (mrows(d, a) - 1) / 2 : (i64)mrows(d, a) * mrows(d, b);
    for (int j = 0; j < nb; ++j) {
        ent += (i64)nsz[j] * (nsz[j] - 1) / 2;
        for (int i : ustruct[j]) ent += (i64)nsz[i] * nsz[j];
    }
    pl.factor_entries = ent;
    pl.solve_bytes = 2.0 * 16.0 * (double)ent;
    // off-diagonal factor tiles (L-hat = X D^{-1}) for the growth monitor
    pl.lhat_s1.clear();
    pl.lhat_k.clear();
    for (int d = 0; d < N; ++d)
        for (int j = 0; j < pl.TE[d]; ++j)
            for (int a = j + 1; a < pl.T[d]; ++a)
                if (nz[d][a][j])
                    pl.lhat_s1.push_back({E(ARR_M, mslot(d, a, j)), (int32_t)mrows(d, a), (int32_t)mrows(d, j)});
    for (int j = 0; j < nb; ++j)
        for (int i : ustruct[j])
            for (int a = 0; a < pl.kt[i]; ++a)
                for (int b = 0; b < pl.kt[j]; ++b)
                    pl.lhat_k.push_back({E(ARR_KL, kslot(j, i, a, b)), (int32_t)tile_rows(nsz[i], a),
                                         (int32_t)tile_rows(nsz[j], b)});
    // every pair of an update task is one full 64x64x64 complex tile product
    // (8 flops per complex multiply-add), whatever the rows actually used
    pl.mfma_flops_update = 0.0;
    pl.update_min_tiles = 0;
    for (const auto *steps : {&pl.s1_steps, &pl.k_steps})
        for (const FactorStep &st : *steps) {
            // least HBM traffic of a step's updates: every distinct operand
            // tile read once, every target tile read and written once
            std::unordered_set<i64> ops;
            for (i64 g = st.up0; g < st.up0 + st.nup; ++g) {
                pl.mfma_flops_update += 8.0 * TILE * (double)TILE * TILE * pl.gemm[g].np;
                for (int32_t q = pl.gemm[g].p0; q < pl.gemm[g].p0 + pl.gemm[g].np; ++q) {
                    ops.insert(pl.pairs[q].a);
                    ops.insert(pl.pairs[q].b);
                }
            }
            pl.update_min_tiles += (i64)ops.size() + 2 * st.nup;
        }
    // vector blocks (64 rows x nrhs) the solve's update launches must move at
    // least: each distinct source block of a sweep step read once, each
    // target read and written once
    pl.solve_min_vblocks = 0;
    for (const auto *steps : {&pl.s1_fwd, &pl.k_fwd, &pl.k_bwd, &pl.s1_bwd})
        for (const SolveStep &st : *steps) {
            std::unordered_set<i64> src;
            for (i64 u = st.up0; u < st.up0 + st.nup; ++u)
                for (int32_t q = pl.vupd[u].p0; q < pl.vupd[u].p0 + pl.vupd[u].np; ++q) src.insert(pl.vpairs[q].src);
            pl.solve_min_vblocks += (i64)src.size() + 2 * st.nup;
        }
}

}  // namespace d3m
