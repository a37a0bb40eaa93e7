// Tile layouts and launch schedules of the factor and solve phases.
#pragma once

#include <string>
#include <vector>

#include "../tasks.hpp"
#include "problem.hpp"

namespace d3m {

// One batched step of the factorisation: a Bunch-Kaufman launch over the
// diagonal blocks of the step, a panel GEMM launch (X = M P L^-T), a scaling
// launch (L-hat = X D^-1) and a trailing-update GEMM launch.
struct FactorStep {
    i64 bk0 = 0, nbk = 0;
    int bk_maxn = 0;
    i64 pan0 = 0, npan = 0;
    i64 sc0 = 0, nsc = 0;
    bool fused_scale = false;  // panel task i and scale task i are the same single-tile block
    i64 up0 = 0, nup = 0;
    i64 ncrit = 0;           // the first ncrit update tasks target the next step's block columns
    bool wait_rest = true;   // updates may touch tiles of the previous side-stream updates
    double up_flops = 0.0;   // algorithmic flops of the update GEMMs
    double crit_flops = 0.0; // ... of which in the first ncrit tasks
    double pan_flops = 0.0;  // algorithmic flops of the panels (triangular solves)
    // K phase: the update tasks after the ncrit critical ones are split into
    // nnear tasks whose block columns belong to the next few levels and the
    // far rest; the block columns (units) each launch touches drive the waits
    // between the streams (a launch waits only for earlier launches that
    // wrote its columns)
    bool track = false;
    i64 add0 = 0, nadd = 0;  // multifrontal form: extend-add tasks run before the pivot launch
    i64 nnear = 0;
    double near_flops = 0.0;
    std::vector<int> cols_bk, cols_crit, cols_near, cols_far;
};

// One sweep step of the solve: a diagonal launch and an update launch.
struct SolveStep {
    i64 dg0 = 0, ndg = 0;
    int dg_maxt = 1;  // largest number of tiles of a diagonal block in this step
    i64 up0 = 0, nup = 0;
    int up_mode = 0;  // 0: out -= sum L y   1: out = sum L^T x   2: out += sum L^T x
    bool up_first = false;  // run the update launch before the diagonal launch
};

struct Plan {
    // ---- subdomain matrices M_d = [A_d D_d; D_d^T 0] --------------------
    std::vector<int> TE, TL, T, fb;    // E tiles, LM tiles, total, first tile column holding interface rows
    std::vector<std::vector<i64>> m_cslot;  // per subdomain: slot of tile (a, b < TE) at a * TE + b, -1 if zero
    std::vector<i64> m_tbase;          // slot of the trailing tile (TE, TE); the trailing triangle is packed
    i64 m_tiles = 0;
    i64 s1_tiles = 0;                  // structurally nonzero tiles in the eliminated columns
    // ---- LM Schur complement (-K), elimination-position order -----------
    // Units are the blocks of K in elimination order, or pieces of them
    // (consecutive rows of one block) when the pivot scope is restricted.
    int k_units = 0, k_levels = 0;
    std::vector<int> unit_block, unit_off, unit_n;
    std::vector<std::vector<int>> kstruct;  // struct of every unit (unit indices)
    std::vector<int> kt;               // tiles per block
    std::vector<i64> kcol;             // slot of the panel's tile (0,0) for each block column
    std::vector<int> kR;               // row tiles of each block-column panel
    std::vector<std::vector<int>> krow_off;  // per block column j: row-tile offset of block struct(j)[i]
    i64 k_tiles = 0;
    // ---- TT tiles and D rows ---------------------------------------------
    std::vector<i64> tt_s1, tt_k;      // TT tile slot per subdomain (then +j) / per block
    i64 tt_tiles = 0;
    std::vector<i64> drow_s1, drow_k;  // first D row per subdomain / per block
    i64 d_rows = 0;
    int n_status = 0;
    // ---- factor schedule ------------------------------------------------
    std::vector<BkTask> bk;
    std::vector<GemmTask> gemm;
    std::vector<GemmPair> pairs;
    std::vector<ScaleTask> scale;
    std::vector<AsmTask> asmb;
    std::vector<FactorStep> s1_steps, k_steps;
    std::vector<int64_t> coo_off;      // ARR_M element of each A_d / D_d entry
    i64 n_coo_a = 0;                   // leading entries that are A_d values
    i64 bk_scratch_elems = 0;          // per-launch global scratch for big blocks
    // ---- solve schedule ---------------------------------------------------
    std::vector<i64> vs1;              // first vector tile of each subdomain
    std::vector<i64> vk;               // first vector tile of each block (position)
    i64 v_tiles_s1 = 0, v_tiles_k = 0;
    std::vector<int64_t> split_map;    // per S1 vector row: global edge if owner, else -1
    std::vector<int64_t> collect_map;  // per global edge: S1 vector row of its owner copy
    std::vector<int64_t> copy_map;     // per S1 vector row of a non-owner copy of an edge: the owner
                                       // copy's row, else -1
    std::vector<VDiagTask> vdiag;
    std::vector<VUpdTask> vupd;
    std::vector<VUpdPair> vpairs;
    std::vector<int64_t> vfuse;  // per update task: diagonal solve it completes (index into vdiag) or -1
    std::vector<SolveStep> s1_fwd, k_fwd, k_bwd, s1_bwd;
    // the S1 sweeps as ordered per-subdomain task lists (left-looking, each
    // target written once): subdomain d's forward tasks are vupd
    // [sq_fwd_off[d], sq_fwd_off[d+1]) in mode 0, its backward tasks
    // [sq_bwd_off[d], sq_bwd_off[d+1]) in mode 1, diagonal solves fused (vfuse)
    std::vector<i64> sq_fwd_off, sq_bwd_off;
    std::vector<int64_t> h_map;        // per K vector row: the two subdomain vector rows (-1: padding)
    std::vector<int64_t> lam_map;      // per S1 vector row: K vector row of a multiplier row, else -1
    std::vector<int64_t> lm_vrow;      // per global multiplier: its K vector row
    // ---- multifrontal form of step 5 (built on request) --------------------
    // Same units, pivot, panel and factor storage as the right-looking
    // schedule; the Schur updates beyond a front (a chain segment of units)
    // go to its update matrix (a packed lower tile triangle over the tile
    // rows of the last unit's struct, in the ARR_KU pool, indexed by the
    // segment's first unit), which the parent's step adds into its front.
    bool mf = false;
    std::vector<FactorStep> mf_steps;
    std::vector<AddTask> mf_add;
    std::vector<int64_t> mf_src;
    std::vector<i64> mf_ubase;         // pool slot of U_s by first unit s (-1: none)
    i64 ku_tiles = 0;                  // tiles of the update-matrix pool
    i64 ku_tiles_total = 0;            // ... without reuse (sum over units)
    double mf_add_bytes = 0.0;         // complex128 bytes moved by the extend-adds of one factorisation
    // ---- the two sweeps over the factor of -K as work-queue item lists ------
    // (one launch per sweep; built by build_solve_chain, index 0 forward, 1
    // backward).  chain_ok is false, with the reason in chain_why, where the
    // sweeps hold tasks the item form does not cover (diagonal blocks of
    // several tiles).
    bool chain_ok = false;
    std::string chain_why;
    std::vector<ChainItem> kc_items[2];
    std::vector<ChainWait> kc_waits[2];
    std::vector<VDiagTask> kc_pre[2];  // diagonal solves no update precedes: one launch before the queue
    // ---- algorithmic counts -----------------------------------------------
    double flops_s1 = 0.0, flops_s3 = 0.0, flops_update = 0.0;
    double mfma_flops_update = 0.0;    // update-GEMM work as executed on full 64x64x64 tile
                                       // products (padding and upper halves of diagonal tiles)
    std::vector<FactorTile> lhat_s1, lhat_k;  // off-diagonal factor tiles of step 1 / of -K
    i64 update_min_tiles = 0;          // least tile reads + writes of the update GEMMs, summed over steps
    i64 solve_min_vblocks = 0;         // least vector-block reads + writes of the solve updates
    double solve_bytes = 0.0;          // complex128 factor bytes read per solve
    i64 factor_entries = 0;
};

// s1_tree: step 1 by levels of each subdomain's tile elimination tree (for
// nested-dissection row orders) instead of one tile column per step
void build_plan(Plan &pl, const Decomp &dc, const BlockOrder &bo, int unit_max, int s1_block, int k_block,
                bool k_fuse, bool s1_tree = false);

// Builds the work-queue form of the two K sweeps of the solve from the
// level-by-level schedule (k_fwd, k_bwd, vdiag, vupd, vfuse of build_plan).
void build_solve_chain(Plan &pl);

// Adds the multifrontal schedule of step 5 to a plan made by build_plan;
// fronts are amalgamated along elimination-tree chains of at most seg_max
// units (1: one front per unit).
void build_multifrontal(Plan &pl, int seg_max);

}  // namespace d3m
