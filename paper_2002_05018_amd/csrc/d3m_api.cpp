// C ABI of the D3M library: handle life cycle, device memory, and the
// orchestration of the factor (recipe steps 1, 2, 5) and solve (steps 6-7)
// launch schedules built by the planner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <string>
#include <vector>

#include "../../include/d3m.h"
#include "host/plan.hpp"
#include "host/problem.hpp"
#include "host/race.hpp"
#include "kernels/launch.hpp"
#include "noalloc.hpp"

using namespace d3m;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            return fail(e_ == hipErrorOutOfMemory ? D3M_ENOMEM : D3M_EHIP,                            \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                           \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

enum KernelId { KID_UPDATE = 0, KID_PANEL = 1, KID_BK = 2, KID_ASM = 3, KID_SOLVE = 4, KID_RESID = 5, KID_COUNT = 6 };

}  // namespace

struct d3m_problem {
    Mesh mesh;
    Decomp dc;
    BlockOrder bo;
    Plan pl;
    double k = 0.0;
    cplx alpha;
    std::vector<double> eps;
    d3m_options opt{};
    int factored = 0;  // 0 none, 1 fp64, 2 fp32
    bool device_ready = false;
    // independent problems held by the handle (one for d3m_setup): edges and
    // tetrahedra of problem p are [off[p], off[p + 1]) of the global numbering
    int n_problems = 1;
    std::vector<int64_t> prob_edge_off, prob_tet_off;
    std::vector<int> sub_prob;      // problem of every subdomain
    std::vector<int32_t> eprob;     // problem of every edge
    int32_t *d_eprob = nullptr;
    // device: task lists and maps
    std::vector<DevBuf> bufs;
    BkTask *d_bk = nullptr;
    GemmTask *d_gemm = nullptr;
    GemmPair *d_pairs = nullptr;
    ScaleTask *d_scale = nullptr;
    AsmTask *d_asm = nullptr;
    VDiagTask *d_vdiag = nullptr;
    VUpdTask *d_vupd = nullptr;
    VUpdPair *d_vpairs = nullptr;
    int64_t *d_vfuse = nullptr;
    int64_t *d_coo_off = nullptr;
    double2 *d_coo_val = nullptr;
    int64_t *d_split = nullptr, *d_collect = nullptr, *d_hmap = nullptr, *d_lmap = nullptr;
    int64_t *d_copymap = nullptr;
    int64_t *d_sq_fwd = nullptr, *d_sq_bwd = nullptr;
    AddTask *d_mfadd = nullptr;
    int64_t *d_mfsrc = nullptr;
    // the two K sweeps of the solve as work queues (tuning solve_chain):
    // item and wait lists, and d_chain = [queue heads of both sweeps, the
    // sticky timeout flag, unused, write counts of the forward sweep's K
    // vector tiles, then of the backward sweep's]
    ChainItem *d_kc_items[2] = {nullptr, nullptr};
    ChainWait *d_kc_waits[2] = {nullptr, nullptr};
    VDiagTask *d_kc_pre[2] = {nullptr, nullptr};
    unsigned *d_chain = nullptr;
    uint64_t chain_spin_ticks = 0;  // bound of one dependency wait (wall-clock ticks, 2 s)
    int chain_clock_khz = 100000;   // rate of the device's wall clock
    unsigned long long *d_disc = nullptr;
    FactorTile *d_lhat_s1 = nullptr, *d_lhat_k = nullptr;
    unsigned long long *d_growth = nullptr;
    int pivot_fallbacks = 0;  // factorisations redone with whole-block pivot scope
    int *d_status = nullptr;
    DArrays D{};
    double2 *d_bkscratch = nullptr;
    // global FEM matrix for refinement residuals
    int64_t *d_rowptr = nullptr;
    int32_t *d_col = nullptr;
    double2 *d_sval = nullptr;
    // adjoint data
    int64_t *d_tet_edges = nullptr;
    double *d_mass = nullptr;
    // precision-dependent matrices and vectors
    DevBuf arr[2][ARR_COUNT];
    DevBuf vec[2][VARR_COUNT];
    int vec_nrhs[2] = {0, 0};
    DevBuf stage_f, stage_E, stage_r, stage_w, stage_g;
    DevBuf stage_rc, stage_ec;  // refinement: residual and field rows of the right-hand sides still refined
    DevBuf stage_et;  // the field transposed (right-hand sides of an edge contiguous) for the residual
    DevBuf norms;
    double2 *d_unused = nullptr;
    // profiling
    double kstat_ms[KID_COUNT] = {0};
    int64_t kstat_n[KID_COUNT] = {0};
    double kstat_flops[KID_COUNT] = {0};
    std::vector<hipEvent_t> ev_pool;
    // second stream for the updates that the next elimination step does not
    // need (look-ahead), and ordering events between the two streams
    hipStream_t side = nullptr;
    hipStream_t side2 = nullptr;  // far updates of the K phase (near ones go on side)
    std::vector<hipEvent_t> dep_pool;  // events of the K phase's dependency waits
    std::vector<hipEvent_t> sync_pool;
    size_t sync_next = 0;
    hipEvent_t sync_event() {
        hipEvent_t e = sync_pool[sync_next];
        sync_next = (sync_next + 1) % sync_pool.size();
        return e;
    }
    struct Rec { int kid; hipEvent_t a, b; double flops; };
    std::vector<Rec> recs;
    size_t ev_next = 0;
    // HIP graphs (opt.use_graph): the factor launch sequence per precision
    // and the solve passes per (precision, buffers, nrhs, accumulate), each
    // captured once on gstream and replayed there, ordered after the work
    // already queued on the caller's stream and before its later work
    struct Graph { hipGraph_t g = nullptr; hipGraphExec_t x = nullptr; };
    struct SolveGraph { int pr; const void *f; void *E; int nrhs; bool acc; Graph gr; };
    Graph fgraph[2];
    std::vector<SolveGraph> sgraphs;
    hipStream_t gstream = nullptr;
    hipEvent_t g_in = nullptr, g_out = nullptr;
    bool capturing = false;
    bool quiet = false;  // no profiling events (the allocation-free solve)
    static void destroy_graph(Graph &g) {
        if (g.x) (void)hipGraphExecDestroy(g.x);
        if (g.g) (void)hipGraphDestroy(g.g);
        g = Graph{};
    }
    void drop_solve_graphs() {
        for (auto &sg : sgraphs) destroy_graph(sg.gr);
        sgraphs.clear();
    }
    void drop_graphs() {
        destroy_graph(fgraph[0]);
        destroy_graph(fgraph[1]);
        drop_solve_graphs();
    }
    // launch-shape choices (d3m_set_tuning)
    d3m_tuning tune{};

    ~d3m_problem() {
        drop_graphs();
        for (auto &b : bufs) if (b.p) (void)hipFree(b.p);
        for (int pr = 0; pr < 2; ++pr) {
            for (auto &b : arr[pr]) if (b.p) (void)hipFree(b.p);
            for (auto &b : vec[pr]) if (b.p) (void)hipFree(b.p);
        }
        for (DevBuf *b : {&stage_f, &stage_E, &stage_r, &stage_w, &stage_g, &stage_rc, &stage_ec, &stage_et, &norms})
            if (b->p) (void)hipFree(b->p);
        for (auto e : ev_pool) (void)hipEventDestroy(e);
        for (auto e : sync_pool) (void)hipEventDestroy(e);
        for (auto e : dep_pool) (void)hipEventDestroy(e);
        if (side) (void)hipStreamDestroy(side);
        if (side2) (void)hipStreamDestroy(side2);
        if (gstream) (void)hipStreamDestroy(gstream);
        if (g_in) (void)hipEventDestroy(g_in);
        if (g_out) (void)hipEventDestroy(g_out);
    }

    template <typename P>
    int upload(P *&dst, const void *src, size_t bytes) {
        DevBuf b;
        b.bytes = std::max<size_t>(bytes, 16);
        HIPCHK(hipMalloc(&b.p, b.bytes));
        bufs.push_back(b);
        if (bytes) HIPCHK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
        dst = reinterpret_cast<P *>(b.p);
        return D3M_OK;
    }
    // replaces a buffer made by upload() (same owner list)
    template <typename P>
    int reupload(P *&dst, const void *src, size_t bytes) {
        for (size_t i = 0; i < bufs.size(); ++i)
            if (bufs[i].p == (void *)dst) {
                (void)hipFree(bufs[i].p);
                bufs.erase(bufs.begin() + (long)i);
                break;
            }
        dst = nullptr;
        return upload(dst, src, bytes);
    }
    template <typename P>
    int zeros(P *&dst, size_t bytes) {
        DevBuf b;
        b.bytes = std::max<size_t>(bytes, 16);
        HIPCHK(hipMalloc(&b.p, b.bytes));
        HIPCHK(hipMemset(b.p, 0, b.bytes));
        bufs.push_back(b);
        dst = reinterpret_cast<P *>(b.p);
        return D3M_OK;
    }
    int ensure(DevBuf &b, size_t bytes) {
        if (b.bytes >= bytes && b.p) return D3M_OK;
        if (b.p) { (void)hipFree(b.p); b.p = nullptr; b.bytes = 0; }
        HIPCHK(hipMalloc(&b.p, std::max<size_t>(bytes, 16)));
        b.bytes = std::max<size_t>(bytes, 16);
        return D3M_OK;
    }

    // ---- profiling helpers
    // opt.profile: 0 off, 1 the update GEMMs only, 2 every kernel group
    bool prof_wanted(int kid) const {
        if (capturing || quiet) return false;  // graphs carry no timing events
        return opt.profile >= 2 || (opt.profile == 1 && kid == KID_UPDATE);
    }
    void prof_begin(int kid, hipEvent_t &a, hipStream_t s) {
        a = nullptr;
        if (!prof_wanted(kid)) return;
        if (ev_next + 2 > ev_pool.size()) {
            for (int i = 0; i < 256; ++i) { hipEvent_t e; if (hipEventCreate(&e) == hipSuccess) ev_pool.push_back(e); }
        }
        a = ev_pool[ev_next++];
        (void)hipEventRecord(a, s);
    }
    void prof_end(int kid, hipEvent_t a, double flops, hipStream_t s) {
        if (!a) return;
        hipEvent_t b = ev_pool[ev_next++];
        (void)hipEventRecord(b, s);
        recs.push_back({kid, a, b, flops});
    }
    void prof_collect() {
        for (auto &r : recs) {
            float ms = 0.f;
            (void)hipEventSynchronize(r.b);
            (void)hipEventElapsedTime(&ms, r.a, r.b);
            kstat_ms[r.kid] += ms;
            kstat_n[r.kid] += 1;
            kstat_flops[r.kid] += r.flops;
        }
        recs.clear();
        ev_next = 0;
    }
};

namespace {

void build_global_csr(const Mesh &m, const Decomp &dc, double k, const double *eps, std::vector<int64_t> &rowptr,
                      std::vector<int32_t> &col, std::vector<double2> &val) {
    // rows and columns of PEC edges are left out (no unknowns; the residual
    // kernel skips their rows)
    std::vector<std::vector<std::pair<int64_t, cplx>>> rows(m.ne);
    auto keep = [&](i64 e) { return m.pec.empty() || !m.pec[e]; };
    double Kc[36], M[36], T[9];
    for (i64 t = 0; t < m.nt; ++t) {
        tet_curl_mass(m, t, Kc, M);
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b)
                if (keep(m.tet_edges[6 * t + a]) && keep(m.tet_edges[6 * t + b]))
                    rows[m.tet_edges[6 * t + a]].push_back(
                        {m.tet_edges[6 * t + b], cplx(Kc[6 * a + b] - k * k * eps[t] * M[6 * a + b], 0.0)});
    }
    for (i64 f : dc.bface) {
        tri_tangential_mass(m, f, T);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                if (keep(m.face_edges[3 * f + a]) && keep(m.face_edges[3 * f + b]))
                    rows[m.face_edges[3 * f + a]].push_back({m.face_edges[3 * f + b], cplx(0.0, k * T[3 * a + b])});
    }
    rowptr.assign(m.ne + 1, 0);
    col.clear();
    val.clear();
    for (i64 r = 0; r < m.ne; ++r) {
        auto &v = rows[r];
        std::sort(v.begin(), v.end(), [](auto &x, auto &y) { return x.first < y.first; });
        for (size_t i = 0; i < v.size();) {
            size_t j = i;
            cplx s = 0.0;
            while (j < v.size() && v[j].first == v[i].first) s += v[j++].second;
            col.push_back((int32_t)v[i].first);
            val.push_back(make_double2(s.real(), s.imag()));
            i = j;
        }
        rowptr[r + 1] = (int64_t)col.size();
        std::vector<std::pair<int64_t, cplx>>().swap(v);
    }
}

// task lists and maps of the plan (again after a re-plan: replace = true)
int upload_schedules(d3m_problem *h, bool replace) {
    const Plan &pl = h->pl;
    int rc;
#define UPS(dst, vec)                                                                                          \
    if ((rc = replace ? h->reupload(dst, vec.data(), vec.size() * sizeof(vec[0]))                              \
                      : h->upload(dst, vec.data(), vec.size() * sizeof(vec[0]))) != D3M_OK)                   \
    return rc
    UPS(h->d_bk, pl.bk);
    UPS(h->d_gemm, pl.gemm);
    UPS(h->d_pairs, pl.pairs);
    UPS(h->d_scale, pl.scale);
    UPS(h->d_asm, pl.asmb);
    UPS(h->d_vdiag, pl.vdiag);
    UPS(h->d_vupd, pl.vupd);
    UPS(h->d_vpairs, pl.vpairs);
    UPS(h->d_vfuse, pl.vfuse);
    UPS(h->d_coo_off, pl.coo_off);
    UPS(h->d_split, pl.split_map);
    UPS(h->d_collect, pl.collect_map);
    UPS(h->d_copymap, pl.copy_map);
    UPS(h->d_sq_fwd, pl.sq_fwd_off);
    UPS(h->d_sq_bwd, pl.sq_bwd_off);
    UPS(h->d_lhat_s1, pl.lhat_s1);
    UPS(h->d_lhat_k, pl.lhat_k);
    UPS(h->d_hmap, pl.h_map);
    UPS(h->d_lmap, pl.lam_map);
    UPS(h->d_mfadd, pl.mf_add);
    UPS(h->d_mfsrc, pl.mf_src);
    UPS(h->d_kc_items[0], pl.kc_items[0]);
    UPS(h->d_kc_items[1], pl.kc_items[1]);
    UPS(h->d_kc_waits[0], pl.kc_waits[0]);
    UPS(h->d_kc_waits[1], pl.kc_waits[1]);
    UPS(h->d_kc_pre[0], pl.kc_pre[0]);
    UPS(h->d_kc_pre[1], pl.kc_pre[1]);
    {
        // queue heads, timeout flag, unused word, write counts of both sweeps
        const std::vector<unsigned> zero(4 + 2 * (size_t)std::max<i64>(pl.v_tiles_k, 1), 0u);
        UPS(h->d_chain, zero);
    }
#undef UPS
    return D3M_OK;
}

int setup_device(d3m_problem *h) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(D3M_ENODEV, "no HIP device");
    if (h->opt.device < 0 || h->opt.device >= ndev) return fail(D3M_ENODEV, "device ordinal out of range");
    HIPCHK(hipSetDevice(h->opt.device));
    // default priority (the same as the caller's streams)
    HIPCHK(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&h->side2, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&h->g_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h->g_out, hipEventDisableTiming));
    h->sync_pool.resize(512);
    for (auto &e : h->sync_pool) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    Plan &pl = h->pl;
    int rc;
    if ((rc = upload_schedules(h, false)) != D3M_OK) return rc;
#define UP(dst, vec) if ((rc = h->upload(dst, vec.data(), vec.size() * sizeof(vec[0]))) != D3M_OK) return rc
    {
        // the device copy marks PEC edges with -1: the residual and norm
        // kernels leave those rows out
        std::vector<int32_t> ep = h->eprob;
        if (!h->mesh.pec.empty())
            for (int64_t e = 0; e < h->mesh.ne; ++e)
                if (h->mesh.pec[e]) ep[e] = -1;
        UP(h->d_eprob, ep);
    }
    if ((rc = h->zeros(h->d_status, sizeof(int) * (pl.n_status + 1))) != D3M_OK) return rc;
    {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->opt.device) != hipSuccess || khz <= 0)
            khz = 100000;
        h->chain_clock_khz = khz;
        h->chain_spin_ticks = (uint64_t)khz * 1000ull * 2ull;
    }
    size_t dr = (size_t)std::max<i64>(pl.d_rows, 1);
    if ((rc = h->zeros(h->D.d, dr * sizeof(double2))) != D3M_OK) return rc;
    if ((rc = h->zeros(h->D.doff, dr * sizeof(double2))) != D3M_OK) return rc;
    if ((rc = h->zeros(h->D.dinv, dr * sizeof(double2))) != D3M_OK) return rc;
    if ((rc = h->zeros(h->D.dinvoff, dr * sizeof(double2))) != D3M_OK) return rc;
    if ((rc = h->zeros(h->D.piv, dr * sizeof(int))) != D3M_OK) return rc;
    if ((rc = h->zeros(h->D.perm, dr * sizeof(int))) != D3M_OK) return rc;
    if (pl.bk_scratch_elems > 0)
        if ((rc = h->zeros(h->d_bkscratch, (size_t)pl.bk_scratch_elems * sizeof(double2))) != D3M_OK) return rc;
    // values of the scatter (A_d entries then the +-1 of D_d)
    {
        std::vector<double2> v;
        v.reserve(pl.coo_off.size());
        for (int d = 0; d < h->dc.N; ++d)
            for (auto &x : h->dc.sub[d].a_val) v.push_back(make_double2(x.real(), x.imag()));
        for (int d = 0; d < h->dc.N; ++d) {
            const Subdomain &S = h->dc.sub[d];
            for (int P : S.blocks)
                for (i64 l = h->dc.blk_start[P]; l < h->dc.blk_start[P + 1]; ++l)
                    v.push_back(make_double2(h->dc.lm_p[l] == d ? 1.0 : -1.0, 0.0));
        }
        UP(h->d_coo_val, v);
    }
    {
        std::vector<int64_t> rp;
        std::vector<int32_t> col;
        std::vector<double2> val;
        build_global_csr(h->mesh, h->dc, h->k, h->eps.data(), rp, col, val);
        UP(h->d_rowptr, rp);
        UP(h->d_col, col);
        UP(h->d_sval, val);
    }
    {
        UP(h->d_tet_edges, h->mesh.tet_edges);
        std::vector<double> mass(36 * h->mesh.nt);
        double Kc[36];
        for (i64 t = 0; t < h->mesh.nt; ++t) tet_curl_mass(h->mesh, t, Kc, &mass[36 * t]);
        UP(h->d_mass, mass);
    }
#undef UP
    HIPCHK(hipDeviceSynchronize());
    h->device_ready = true;
    return D3M_OK;
}

template <typename T>
int ensure_arrays(d3m_problem *h) {
    const int pr = std::is_same<T, double>::value ? 0 : 1;
    const size_t es = sizeof(T) * 2;
    const Plan &pl = h->pl;
    const i64 tiles[ARR_COUNT] = {pl.m_tiles, pl.m_tiles, pl.k_tiles, pl.k_tiles,
                                  pl.k_tiles, pl.tt_tiles, pl.mf ? pl.ku_tiles : 0};
    for (int a = 0; a < ARR_COUNT; ++a) {
        int rc = h->ensure(h->arr[pr][a], (size_t)tiles[a] * TILE_ELEMS * es);
        if (rc != D3M_OK) return rc;
    }
    return D3M_OK;
}

template <typename T>
Bases bases_of(d3m_problem *h) {
    const int pr = std::is_same<T, double>::value ? 0 : 1;
    Bases b;
    for (int a = 0; a < ARR_COUNT; ++a) b.p[a] = h->arr[pr][a].p;
    return b;
}

template <typename T>
int ensure_vectors(d3m_problem *h, int nrhs) {
    const int pr = std::is_same<T, double>::value ? 0 : 1;
    if (h->vec_nrhs[pr] >= nrhs) return D3M_OK;
    h->drop_solve_graphs();  // they hold the old vector addresses
    const size_t es = sizeof(T) * 2;
    const Plan &pl = h->pl;
    for (int v = 0; v < VARR_COUNT; ++v) {
        i64 tiles = v < V_KX ? pl.v_tiles_s1 : pl.v_tiles_k;
        int rc = h->ensure(h->vec[pr][v], (size_t)std::max<i64>(tiles, 1) * 64 * nrhs * es);
        if (rc != D3M_OK) return rc;
    }
    h->vec_nrhs[pr] = nrhs;
    return D3M_OK;
}

template <typename T>
VBases vbases_of(d3m_problem *h) {
    const int pr = std::is_same<T, double>::value ? 0 : 1;
    VBases b;
    for (int v = 0; v < VARR_COUNT; ++v) b.p[v] = h->vec[pr][v].p;
    return b;
}

// One elimination sweep (subdomain tiles or levels of K) with a look-ahead
// of one step: the update tasks of step j that target the block columns of
// step j + 1 (the first ncrit) run on the caller's stream right after the
// panels; the others run on the side stream, overlapping the factorisation
// of step j + 1.  Two launches never write the same tile at once: the
// next-column updates of step j wait for the side-stream updates of step
// j - 1 (which also reach those columns), and a side-stream launch starts
// only after the panels it reads are scaled.
constexpr i64 kLookaheadMinTasks = 512;  // default of d3m_tuning.lookahead_tasks

// The K phase with dependency tracking by block column (unit): a step's
// pivot and panel launches and its critical updates run on s; its near
// updates (columns of the next few levels) on the side stream and its far
// updates on a second side stream, each after the step's panels.  Every
// launch waits only for the side launches that last wrote one of its
// columns (a side stream runs in order, so the latest writer on it covers
// the earlier ones), so the far updates of a chain segment overlap the pivot
// chain of the next segment instead of stalling it.  Launches that write a
// tile in the same order as before, so results are bitwise unchanged.
template <typename T>
int run_factor_sweep_tracked(d3m_problem *h, const std::vector<FactorStep> &steps, const Bases &b, hipStream_t s) {
    hipStream_t ss[2] = {h->side, h->side2};
    const i64 min_split = h->tune.lookahead_tasks > 0 ? h->tune.lookahead_tasks : kLookaheadMinTasks;
    // a step records at most three events (panels done, near done, far done);
    // none is reused within the sweep
    const size_t need = 3 * steps.size() + 4;
    while (h->dep_pool.size() < need) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        h->dep_pool.push_back(e);
    }
    size_t next_ev = 0;
    auto take_event = [&]() { return next_ev < h->dep_pool.size() ? h->dep_pool[next_ev++] : nullptr; };
    std::vector<hipEvent_t> evs[2];                  // events recorded on each side stream, in order
    std::vector<std::pair<int, int>> last(h->pl.k_units, {-1, -1});  // (side stream, event index) of the last writer
    auto wait_cols = [&](const std::vector<int> &cols, hipStream_t on) -> int {
        int hi[2] = {-1, -1};
        for (int k : cols)
            if (last[k].first >= 0) hi[last[k].first] = std::max(hi[last[k].first], last[k].second);
        for (int q = 0; q < 2; ++q)
            if (hi[q] >= 0 && ss[q] != on) HIPCHK(hipStreamWaitEvent(on, evs[q][hi[q]], 0));
        return D3M_OK;
    };
    int rc;
    for (const auto &st : steps) {
        hipEvent_t ev{};
        if ((rc = wait_cols(st.cols_bk, s)) != D3M_OK) return rc;
        if (st.nbk > 0) {
            h->prof_begin(KID_BK, ev, s);
            HIPCHK(launch_bk<T>(h->d_bk + st.bk0, st.nbk, st.bk_maxn, h->d_pairs, b, h->D, h->d_status,
                                h->d_bkscratch, s));
            h->prof_end(KID_BK, ev, 0.0, s);
        }
        if (st.npan > 0 || st.nsc > 0) {
            h->prof_begin(KID_PANEL, ev, s);
            if (st.fused_scale) {
                HIPCHK(launch_panel_scale<T>(h->d_gemm + st.pan0, h->d_scale + st.sc0, st.npan, h->d_pairs, b, h->D,
                                             h->tune.panel_rows == 16 ? 16 : 64, s));
            } else {
                HIPCHK(launch_gemm<T>(h->d_gemm + st.pan0, st.npan, h->d_pairs, b, 0, s));
                HIPCHK(launch_scale<T>(h->d_scale + st.sc0, st.nsc, b, h->D, s));
            }
            h->prof_end(KID_PANEL, ev, st.pan_flops, s);
        }
        const i64 nfar = st.nup - st.ncrit - st.nnear;
        // small off-critical groups stay on s (a cross-stream hand-off costs
        // more than the overlap gains)
        const bool split = st.nup - st.ncrit >= min_split;
        hipEvent_t ready = nullptr;
        auto side_launch = [&](int q, i64 off, i64 n, const std::vector<int> &cols, double fl) -> int {
            if (!ready) {
                if (!(ready = take_event())) return fail(D3M_EHIP, "internal: dependency event pool exhausted");
                HIPCHK(hipEventRecord(ready, s));
            }
            HIPCHK(hipStreamWaitEvent(ss[q], ready, 0));
            int r = wait_cols(cols, ss[q]);
            if (r != D3M_OK) return r;
            hipEvent_t e2{};
            h->prof_begin(KID_UPDATE, e2, ss[q]);
            HIPCHK(launch_gemm<T>(h->d_gemm + st.up0 + off, n, h->d_pairs, b, 1, ss[q]));
            h->prof_end(KID_UPDATE, e2, fl, ss[q]);
            hipEvent_t done = take_event();
            if (!done) return fail(D3M_EHIP, "internal: dependency event pool exhausted");
            HIPCHK(hipEventRecord(done, ss[q]));
            evs[q].push_back(done);
            for (int k : cols) last[k] = {q, (int)evs[q].size() - 1};
            return D3M_OK;
        };
        auto rest = [&]() -> int {
            if (st.nnear > 0 && (rc = side_launch(0, st.ncrit, st.nnear, st.cols_near, st.near_flops)) != D3M_OK)
                return rc;
            if (nfar > 0 && (rc = side_launch(1, st.ncrit + st.nnear, nfar, st.cols_far,
                                              st.up_flops - st.crit_flops - st.near_flops)) != D3M_OK)
                return rc;
            return D3M_OK;
        };
        const bool late = h->tune.side_early == 0;
        if (split && !late && (rc = rest()) != D3M_OK) return rc;
        const i64 nmain = split ? st.ncrit : st.nup;
        if (nmain > 0) {
            if ((rc = wait_cols(st.cols_crit, s)) != D3M_OK) return rc;
            if (!split) {
                if ((rc = wait_cols(st.cols_near, s)) != D3M_OK) return rc;
                if ((rc = wait_cols(st.cols_far, s)) != D3M_OK) return rc;
            }
            h->prof_begin(KID_UPDATE, ev, s);
            HIPCHK(launch_gemm<T>(h->d_gemm + st.up0, nmain, h->d_pairs, b, 1, s));
            h->prof_end(KID_UPDATE, ev, split ? st.crit_flops : st.up_flops, s);
        }
        if (split && late && (rc = rest()) != D3M_OK) return rc;
    }
    for (int q = 0; q < 2; ++q)
        if (!evs[q].empty()) HIPCHK(hipStreamWaitEvent(s, evs[q].back(), 0));
    return D3M_OK;
}

template <typename T>
int run_factor_sweep(d3m_problem *h, const std::vector<FactorStep> &steps, const Bases &b, hipStream_t s) {
    // Whole-block pivot units (pivot_scope 1, blocks of more than one tile)
    // run the K phase on one stream: with the look-ahead side stream their
    // factor came out wrong at 48^3 hexes in 512 subdomains (and one run
    // faulted), while the same schedule on one stream, and every one-tile
    // unit schedule, is correct; the cause is not found, so that combination
    // is not launched.
    const bool one_stream = h->opt.pivot_scope == 1 && !steps.empty() && steps[0].track;
    if (h->tune.k_overlap && !one_stream && !steps.empty() && steps[0].track)
        return run_factor_sweep_tracked<T>(h, steps, b, s);
    hipStream_t s2 = h->side;
    hipEvent_t rest_done = nullptr;
    const i64 min_split = one_stream ? std::numeric_limits<i64>::max()
                                     : (h->tune.lookahead_tasks > 0 ? h->tune.lookahead_tasks : kLookaheadMinTasks);
    for (const auto &st : steps) {
        hipEvent_t ev{};
        if (st.nbk > 0) {
            h->prof_begin(KID_BK, ev, s);
            HIPCHK(launch_bk<T>(h->d_bk + st.bk0, st.nbk, st.bk_maxn, h->d_pairs, b, h->D, h->d_status,
                                h->d_bkscratch, s));
            h->prof_end(KID_BK, ev, 0.0, s);
        }
        if (st.npan > 0 || st.nsc > 0) {
            h->prof_begin(KID_PANEL, ev, s);
            if (st.fused_scale) {
                HIPCHK(launch_panel_scale<T>(h->d_gemm + st.pan0, h->d_scale + st.sc0, st.npan, h->d_pairs, b, h->D,
                                             h->tune.panel_rows == 16 ? 16 : 64, s));
            } else {
                HIPCHK(launch_gemm<T>(h->d_gemm + st.pan0, st.npan, h->d_pairs, b, 0, s));
                HIPCHK(launch_scale<T>(h->d_scale + st.sc0, st.nsc, b, h->D, s));
            }
            h->prof_end(KID_PANEL, ev, st.pan_flops, s);
        }
        // small updates stay on one stream: a cross-stream hand-off costs
        // more than the overlap gains when the side launch is short
        const bool split = st.nup - st.ncrit >= min_split;
        const i64 ncrit = split ? st.ncrit : st.nup;
        const double crit_flops = split ? st.crit_flops : st.up_flops;
        const i64 nrest = st.nup - ncrit;
        // side launch: after the critical updates, so that the next pivot
        // launch is dispatched before the side work fills the machine (a
        // pivot work-group sharing compute units with update waves runs its
        // sequential steps 2-3x slower), or (side_early) right after the
        // panels it reads
        auto launch_rest = [&]() -> int {
            hipEvent_t ready = h->sync_event();
            HIPCHK(hipEventRecord(ready, s));
            HIPCHK(hipStreamWaitEvent(s2, ready, 0));
            hipEvent_t e2{};
            h->prof_begin(KID_UPDATE, e2, s2);
            HIPCHK(launch_gemm<T>(h->d_gemm + st.up0 + ncrit, nrest, h->d_pairs, b, 1, s2));
            h->prof_end(KID_UPDATE, e2, st.up_flops - crit_flops, s2);
            return D3M_OK;
        };
        const bool late = h->tune.side_early == 0;
        int rc;
        if (nrest > 0 && !late && (rc = launch_rest()) != D3M_OK) return rc;
        if (rest_done && st.wait_rest) {
            HIPCHK(hipStreamWaitEvent(s, rest_done, 0));
            rest_done = nullptr;
        }
        if (ncrit > 0) {  // timed only when launched, so averages are per launch
            h->prof_begin(KID_UPDATE, ev, s);
            HIPCHK(launch_gemm<T>(h->d_gemm + st.up0, ncrit, h->d_pairs, b, 1, s));
            h->prof_end(KID_UPDATE, ev, crit_flops, s);
        }
        if (nrest > 0 && late && (rc = launch_rest()) != D3M_OK) return rc;
        if (nrest > 0) {  // (a step with side updates always waited above, so nothing is lost)
            rest_done = h->sync_event();
            HIPCHK(hipEventRecord(rest_done, s2));
        }
    }
    if (rest_done) HIPCHK(hipStreamWaitEvent(s, rest_done, 0));
    return D3M_OK;
}

// Step 5 in multifrontal form, one elimination-tree level per step on s:
// the extend-adds of the level's fronts, the pivot and panel launches, then
// the update GEMMs into the level's update matrices.
template <typename T>
int run_multifrontal_sweep(d3m_problem *h, const Bases &b, hipStream_t s) {
    for (const auto &st : h->pl.mf_steps) {
        hipEvent_t ev{};
        if (st.nadd > 0) {
            h->prof_begin(KID_ASM, ev, s);
            HIPCHK(launch_extend_add<T>(h->d_mfadd + st.add0, st.nadd, h->d_mfsrc, b, s));
            h->prof_end(KID_ASM, ev, 0.0, s);
        }
        if (st.nbk > 0) {
            h->prof_begin(KID_BK, ev, s);
            HIPCHK(launch_bk<T>(h->d_bk + st.bk0, st.nbk, st.bk_maxn, h->d_pairs, b, h->D, h->d_status,
                                h->d_bkscratch, s));
            h->prof_end(KID_BK, ev, 0.0, s);
        }
        if (st.npan > 0 || st.nsc > 0) {
            h->prof_begin(KID_PANEL, ev, s);
            if (st.fused_scale) {
                HIPCHK(launch_panel_scale<T>(h->d_gemm + st.pan0, h->d_scale + st.sc0, st.npan, h->d_pairs, b, h->D,
                                             h->tune.panel_rows == 16 ? 16 : 64, s));
            } else {
                HIPCHK(launch_gemm<T>(h->d_gemm + st.pan0, st.npan, h->d_pairs, b, 0, s));
                HIPCHK(launch_scale<T>(h->d_scale + st.sc0, st.nsc, b, h->D, s));
            }
            h->prof_end(KID_PANEL, ev, st.pan_flops, s);
        }
        if (st.nup > 0) {
            h->prof_begin(KID_UPDATE, ev, s);
            HIPCHK(launch_gemm<T>(h->d_gemm + st.up0, st.nup, h->d_pairs, b, 1, s));
            h->prof_end(KID_UPDATE, ev, st.up_flops, s);
        }
    }
    return D3M_OK;
}

// Captures the launches body(gstream) makes into g (nothing runs).
template <typename F>
int capture_graph(d3m_problem *h, d3m_problem::Graph &g, F &&body) {
    HIPCHK(hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal));
    h->capturing = true;
    const int rc = body(h->gstream);
    h->capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(h->gstream, &graph);
    if (rc != D3M_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(D3M_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    const hipError_t ei = hipGraphInstantiate(&x, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(D3M_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    g.g = graph;
    g.x = x;
    return D3M_OK;
}

// Replays g on gstream after the work queued on s; later work on s waits for it.
int replay_graph(d3m_problem *h, const d3m_problem::Graph &g, hipStream_t s) {
    HIPCHK(hipEventRecord(h->g_in, s));
    HIPCHK(hipStreamWaitEvent(h->gstream, h->g_in, 0));
    HIPCHK(hipGraphLaunch(g.x, h->gstream));
    HIPCHK(hipEventRecord(h->g_out, h->gstream));
    HIPCHK(hipStreamWaitEvent(s, h->g_out, 0));
    return D3M_OK;
}

// every launch of the factorisation (recipe steps 1, 2, 5), in order, on s
template <typename T>
int factor_launch(d3m_problem *h, hipStream_t s) {
    const Plan &pl = h->pl;
    Bases b = bases_of<T>(h);
    int rc;
    hipEvent_t ev{};
    h->prof_begin(KID_ASM, ev, s);
    HIPCHK(launch_fill_zero<T>(b.p[ARR_M], pl.m_tiles * TILE_ELEMS, s));
    HIPCHK(launch_coo_scatter<T>(b.p[ARR_M], h->d_coo_off, h->d_coo_val, (int64_t)pl.coo_off.size(), s));
    HIPCHK(launch_zero_i32(h->d_status, pl.n_status + 1, s));
    h->prof_end(KID_ASM, ev, 0.0, s);
    if ((rc = run_factor_sweep<T>(h, pl.s1_steps, b, s)) != D3M_OK) return rc;
    h->prof_begin(KID_ASM, ev, s);
    HIPCHK(launch_asm<T>(h->d_asm, (int64_t)pl.asmb.size(), b, s));
    h->prof_end(KID_ASM, ev, 0.0, s);
    if (pl.mf) return run_multifrontal_sweep<T>(h, b, s);
    return run_factor_sweep<T>(h, pl.k_steps, b, s);
}

template <typename T>
int factor_impl(d3m_problem *h, hipStream_t s) {
    int rc = ensure_arrays<T>(h);
    if (rc != D3M_OK) return rc;
    const Plan &pl = h->pl;
    const int pr = std::is_same<T, double>::value ? 0 : 1;
    if (h->opt.use_graph) {
        if (!h->fgraph[pr].x &&
            (rc = capture_graph(h, h->fgraph[pr], [&](hipStream_t gs) { return factor_launch<T>(h, gs); })) != D3M_OK)
            return rc;
        if ((rc = replay_graph(h, h->fgraph[pr], s)) != D3M_OK) return rc;
    } else if ((rc = factor_launch<T>(h, s)) != D3M_OK) {
        return rc;
    }
    std::vector<int> status(pl.n_status + 1, 0);
    HIPCHK(hipMemcpyAsync(status.data(), h->d_status, sizeof(int) * status.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    h->prof_collect();
    for (int i = 0; i < pl.n_status; ++i)
        if (status[i] != 0) {
            const BkTask &t = pl.bk[i];
            std::string where;
            const i64 first_k = pl.k_steps.empty() ? (i64)pl.bk.size() : pl.k_steps[0].bk0;
            if (i < first_k) {
                where = "subdomain diagonal tile (task " + std::to_string(i) + ")";
            } else {
                int pos = -1;
                for (size_t j = 0; j < pl.drow_k.size(); ++j) if (pl.drow_k[j] == t.drow) pos = (int)j;
                where = "unit " + std::to_string(pos) + " of block " +
                        std::to_string(pos >= 0 ? pl.unit_block[pos] : -1) + " (rows from " +
                        std::to_string(pos >= 0 ? pl.unit_off[pos] : -1) + ")";
            }
            return fail(D3M_ESINGULAR, "singular pivot block: " + where + ", column " + std::to_string(status[i] - 1));
        }
    return D3M_OK;
}

template <typename T>
int solve_step(d3m_problem *h, const SolveStep &st, const Bases &b, const VBases &vb, bool bwd, int nrhs,
               hipStream_t s) {
    // steps with few update tasks take 16 right-hand sides per work-group
    // (twice the work-groups, half the MFMA chain each)
    const int cols = st.nup < h->tune.solve_narrow ? 16 : h->tune.solve_cols;
    if (st.up_first)
        HIPCHK(launch_vupd<T>(h->d_vupd + st.up0, h->d_vfuse + st.up0, st.nup, h->d_vpairs, h->d_vdiag, st.up_mode, b,
                              vb, h->D, nrhs, cols, s));
    HIPCHK(launch_vdiag<T>(h->d_vdiag + st.dg0, st.ndg, st.dg_maxt, bwd, b, vb, h->D, nrhs, cols, s));
    if (!st.up_first)
        HIPCHK(launch_vupd<T>(h->d_vupd + st.up0, h->d_vfuse + st.up0, st.nup, h->d_vpairs, h->d_vdiag, st.up_mode, b,
                              vb, h->D, nrhs, cols, s));
    return D3M_OK;
}

// E (=|+=) S^{-1} f through the factors of precision T; f and E on the
// device; every launch of recipe steps 6-7, in order, on s
template <typename T>
int solve_launch_vb(d3m_problem *h, const VBases &vb, const double2 *f, double2 *E, int nrhs, bool accumulate,
                    hipStream_t s) {
    int rc;
    const Plan &pl = h->pl;
    Bases b = bases_of<T>(h);
    hipEvent_t ev{};
    h->prof_begin(KID_SOLVE, ev, s);
    HIPCHK(launch_vsplit<T>(vb.p[V_X], f, h->d_split, pl.v_tiles_s1 * 64, nrhs, h->mesh.ne, s));
    if (h->tune.solve_seq)
        HIPCHK(launch_vseq<T>(h->d_vupd, h->d_vfuse, h->d_sq_fwd, h->dc.N, h->d_vpairs, h->d_vdiag, false, b, vb, h->D,
                              nrhs, h->tune.solve_cols, s));
    else
        for (const auto &st : pl.s1_fwd) if ((rc = solve_step<T>(h, st, b, vb, false, nrhs, s))) return rc;
    HIPCHK(launch_vgather_h<T>(vb.p[V_KX], vb.p[V_X], h->d_hmap, pl.v_tiles_k * 64, nrhs, s));
    if (h->tune.solve_chain && pl.chain_ok) {
        // each K sweep: the diagonal solves no update precedes, then one
        // work-queue launch over all its update tasks in the level-by-level
        // order (each carrying the solve of the tile it writes last)
        unsigned *head = h->d_chain, *err = h->d_chain + 2, *cnt = h->d_chain + 4;
        const int cols = h->tune.solve_cols;
        HIPCHK(launch_vchain_reset(head, cnt, 2 * pl.v_tiles_k, s));
        for (int sw = 0; sw < 2; ++sw) {
            const bool bwd = sw == 1;
            if (bwd) HIPCHK(launch_fill_zero<T>(vb.p[V_KACC], pl.v_tiles_k * 64 * nrhs, s));
            HIPCHK(launch_vdiag<T>(h->d_kc_pre[sw], (int64_t)pl.kc_pre[sw].size(), 1, bwd, b, vb, h->D, nrhs, cols, s));
            HIPCHK(launch_vchain<T>(h->d_kc_items[sw], (int64_t)pl.kc_items[sw].size(), h->d_kc_waits[sw], h->d_vupd,
                                    h->d_vpairs, h->d_vdiag, bwd, b, vb, h->D, nrhs, cols, head + sw, err,
                                    cnt + sw * pl.v_tiles_k, h->chain_spin_ticks, s));
        }
    } else {
        for (const auto &st : pl.k_fwd) if ((rc = solve_step<T>(h, st, b, vb, false, nrhs, s))) return rc;
        HIPCHK(launch_fill_zero<T>(vb.p[V_KACC], pl.v_tiles_k * 64 * nrhs, s));
        for (const auto &st : pl.k_bwd) if ((rc = solve_step<T>(h, st, b, vb, true, nrhs, s))) return rc;
    }
    HIPCHK(launch_vscatter_lam<T>(vb.p[V_X], vb.p[V_KX], h->d_lmap, pl.v_tiles_s1 * 64, nrhs, s));
    if (h->tune.solve_seq)
        HIPCHK(launch_vseq<T>(h->d_vupd, h->d_vfuse, h->d_sq_bwd, h->dc.N, h->d_vpairs, h->d_vdiag, true, b, vb, h->D,
                              nrhs, h->tune.solve_cols, s));
    else
        for (const auto &st : pl.s1_bwd) if ((rc = solve_step<T>(h, st, b, vb, true, nrhs, s))) return rc;
    HIPCHK(launch_vcollect<T>(E, vb.p[V_X], h->d_collect, h->mesh.ne, nrhs, accumulate, s));
    h->prof_end(KID_SOLVE, ev, 0.0, s);
    return D3M_OK;
}

template <typename T>
int solve_launch(d3m_problem *h, const double2 *f, double2 *E, int nrhs, bool accumulate, hipStream_t s) {
    return solve_launch_vb<T>(h, vbases_of<T>(h), f, E, nrhs, accumulate, s);
}

// bytes of solve vector array v (precision T) for nrhs right-hand sides,
// rounded up to 256
template <typename T>
size_t vec_bytes(const d3m_problem *h, int v, int nrhs) {
    const i64 tiles = v < V_KX ? h->pl.v_tiles_s1 : h->pl.v_tiles_k;
    const size_t b = (size_t)std::max<i64>(tiles, 1) * 64 * nrhs * sizeof(T) * 2;
    return (b + 255) & ~(size_t)255;
}

template <typename T>
int solve_pass(d3m_problem *h, const double2 *f, double2 *E, int nrhs, bool accumulate, hipStream_t s) {
    int rc = ensure_vectors<T>(h, nrhs);
    if (rc != D3M_OK) return rc;
    if (!h->opt.use_graph) return solve_launch<T>(h, f, E, nrhs, accumulate, s);
    const int pr = std::is_same<T, double>::value ? 0 : 1;
    d3m_problem::Graph *g = nullptr;
    for (auto &sg : h->sgraphs)
        if (sg.pr == pr && sg.f == f && sg.E == E && sg.nrhs == nrhs && sg.acc == accumulate) g = &sg.gr;
    if (!g) {
        constexpr size_t kMaxSolveGraphs = 8;
        if (h->sgraphs.size() >= kMaxSolveGraphs) {
            d3m_problem::destroy_graph(h->sgraphs.front().gr);
            h->sgraphs.erase(h->sgraphs.begin());
        }
        h->sgraphs.push_back({pr, f, E, nrhs, accumulate, {}});
        g = &h->sgraphs.back().gr;
        rc = capture_graph(h, *g, [&](hipStream_t gs) { return solve_launch<T>(h, f, E, nrhs, accumulate, gs); });
        if (rc != D3M_OK) {
            h->sgraphs.pop_back();
            return rc;
        }
    }
    return replay_graph(h, *g, s);
}

bool is_device_ptr(const void *p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) { (void)hipGetLastError(); return false; }
    return a.type == hipMemoryTypeDevice;
}

// per-column infinity norms gathered in h->norms, copied to the host
int fetch_norms(d3m_problem *h, int nrhs, std::vector<double> &out, hipStream_t s) {
    std::vector<unsigned long long> bits(nrhs);
    HIPCHK(hipMemcpyAsync(bits.data(), h->norms.p, sizeof(unsigned long long) * nrhs, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    out.resize(nrhs);
    for (int c = 0; c < nrhs; ++c) std::memcpy(&out[c], &bits[c], sizeof(double));
    return D3M_OK;
}

// per problem and right-hand side: max_e |v[c][e]| over the problem's edges
int norms_inf(d3m_problem *h, const double2 *v, int nrhs, std::vector<double> &out, hipStream_t s) {
    const size_t n = (size_t)h->n_problems * nrhs;
    int rc = h->ensure(h->norms, sizeof(unsigned long long) * n);
    if (rc) return rc;
    HIPCHK(hipMemsetAsync(h->norms.p, 0, sizeof(unsigned long long) * n, s));
    HIPCHK(launch_rownorm_max((unsigned long long *)h->norms.p, v, h->d_eprob, h->mesh.ne, nrhs, s));
    return fetch_norms(h, (int)n, out, s);
}

// r = f - S E into h->stage_r (FP64) and, per problem and right-hand side,
// the infinity norm of r
int residual_inf(d3m_problem *h, const double2 *f, const double2 *E, int nrhs, std::vector<double> &out,
                 hipStream_t s) {
    const size_t n = (size_t)h->n_problems * nrhs;
    int rc = h->ensure(h->norms, sizeof(unsigned long long) * n);
    if (rc) return rc;
    if ((rc = h->ensure(h->stage_et, sizeof(double2) * (size_t)nrhs * h->mesh.ne))) return rc;
    HIPCHK(hipMemsetAsync(h->norms.p, 0, sizeof(unsigned long long) * n, s));
    hipEvent_t ev{};
    h->prof_begin(KID_RESID, ev, s);
    HIPCHK(launch_residual((double2 *)h->stage_r.p, f, E, (double2 *)h->stage_et.p, h->d_rowptr, h->d_col, h->d_sval,
                           h->d_eprob, h->mesh.ne, nrhs, (unsigned long long *)h->norms.p, s));
    h->prof_end(KID_RESID, ev, 0.0, s);
    return fetch_norms(h, (int)n, out, s);
}

// max over problems and right-hand sides of ||r||_inf / ||f||_inf (NaN if any
// norm is NaN, so that a non-finite solution never counts as converged)
double relative_residual(const std::vector<double> &rn, const std::vector<double> &fn) {
    double res = 0.0;
    for (size_t i = 0; i < rn.size(); ++i) {
        const double q = fn[i] > 0 ? rn[i] / fn[i] : rn[i];
        if (q != q) return q;
        res = std::max(res, q);
    }
    return res;
}

// largest |difference| between subdomain copies of a shared edge in the
// subdomain vectors of the last solve pass of precision T (the continuity
// D^T E = 0 of eq. (1) holds up to the rounding of lambda)
template <typename T>
int copy_discrepancy(d3m_problem *h, int nrhs, double &out, hipStream_t s) {
    if (!h->d_disc) {
        int rc = h->zeros(h->d_disc, sizeof(unsigned long long));
        if (rc != D3M_OK) return rc;
    }
    HIPCHK(hipMemsetAsync(h->d_disc, 0, sizeof(unsigned long long), s));
    VBases vb = vbases_of<T>(h);
    HIPCHK(launch_copy_disc<T>(h->d_disc, vb.p[V_X], h->d_copymap, h->pl.v_tiles_s1 * 64, nrhs, s));
    unsigned long long bits = 0;
    HIPCHK(hipMemcpyAsync(&bits, h->d_disc, sizeof(bits), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::memcpy(&out, &bits, sizeof(double));
    return D3M_OK;
}

// the work-queue K sweeps bound every dependency wait; a wait that ran out
// leaves the flag set (and the solution wrong): report it once, then clear it
int chain_check(d3m_problem *h, hipStream_t s) {
    if (!h->d_chain) return D3M_OK;
    unsigned flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, h->d_chain + 2, sizeof(flag), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (flag == 0) return D3M_OK;
    const unsigned zero = 0;
    HIPCHK(hipMemcpyAsync(h->d_chain + 2, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return fail(D3M_EHIP, "a dependency wait of the work-queue K solve sweep timed out (solution invalid)");
}

// full solve on device buffers (both precisions); optional diagnostics
int solve_device(d3m_problem *h, const double2 *f, double2 *E, int nrhs, d3m_solve_info *info, hipStream_t s) {
    const size_t vbytes = sizeof(double2) * (size_t)nrhs * h->mesh.ne;
    int rc;
    if (h->factored == 1) {
        if ((rc = solve_pass<double>(h, f, E, nrhs, false, s))) return rc;
        if (info) {
            if ((rc = h->ensure(h->stage_r, vbytes))) return rc;
            std::vector<double> rn, fn;
            if ((rc = residual_inf(h, f, E, nrhs, rn, s))) return rc;
            if ((rc = norms_inf(h, f, nrhs, fn, s))) return rc;
            const double res = relative_residual(rn, fn);
            info->iterations = 0;
            info->converged = res == res ? 1 : 0;  // a NaN residual passes no test
            info->residual = res;
            if ((rc = copy_discrepancy<double>(h, nrhs, info->copy_discrepancy, s))) return rc;
        }
        HIPCHK(hipStreamSynchronize(s));
        h->prof_collect();
        return chain_check(h, s);
    }
    // FP32 factors with FP64 iterative refinement on S E = f
    if ((rc = h->ensure(h->stage_r, vbytes))) return rc;
    std::vector<double> fn, rn;
    if ((rc = norms_inf(h, f, nrhs, fn, s))) return rc;
    if ((rc = solve_pass<float>(h, f, E, nrhs, false, s))) return rc;
    // E is the sum of the passes' fields, so the sum of their copy
    // discrepancies bounds that of E
    double disc = 0.0, d1 = 0.0;
    if (info && (rc = copy_discrepancy<float>(h, nrhs, disc, s))) return rc;
    int it = 0;
    double res = 0.0;
    bool ok = false;
    const int64_t ne = h->mesh.ne;
    const size_t row = sizeof(double2) * (size_t)ne;
    for (;;) {
        if ((rc = residual_inf(h, f, E, nrhs, rn, s))) return rc;
        res = relative_residual(rn, fn);
        if (res <= h->opt.ir_tol) { ok = true; break; }
        if (it >= h->opt.ir_max_iter) break;
        // right-hand sides still above the tolerance in some problem (a NaN
        // residual counts as not converged); the others keep their field
        std::vector<int> todo;
        for (int c = 0; c < nrhs; ++c) {
            bool done = true;
            for (int p = 0; p < h->n_problems; ++p) {
                const size_t i = (size_t)p * nrhs + c;
                const double q = fn[i] > 0 ? rn[i] / fn[i] : rn[i];
                if (!(q <= h->opt.ir_tol)) done = false;
            }
            if (!done) todo.push_back(c);
        }
        const int m = (int)todo.size();
        if (m == nrhs) {
            if ((rc = solve_pass<float>(h, (double2 *)h->stage_r.p, E, nrhs, true, s))) return rc;
        } else {
            // one correction solve over those right-hand sides only: their
            // residual and field rows gathered, corrected, written back
            if ((rc = h->ensure(h->stage_rc, row * m)) || (rc = h->ensure(h->stage_ec, row * m))) return rc;
            double2 *rcm = (double2 *)h->stage_rc.p, *ecm = (double2 *)h->stage_ec.p;
            for (int i = 0; i < m; ++i) {
                HIPCHK(hipMemcpyAsync(rcm + (size_t)i * ne, (double2 *)h->stage_r.p + (size_t)todo[i] * ne, row,
                                      hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemcpyAsync(ecm + (size_t)i * ne, E + (size_t)todo[i] * ne, row, hipMemcpyDeviceToDevice, s));
            }
            if ((rc = solve_pass<float>(h, rcm, ecm, m, true, s))) return rc;
            for (int i = 0; i < m; ++i)
                HIPCHK(hipMemcpyAsync(E + (size_t)todo[i] * ne, ecm + (size_t)i * ne, row, hipMemcpyDeviceToDevice, s));
        }
        if (info) {
            if ((rc = copy_discrepancy<float>(h, m, d1, s))) return rc;
            disc += d1;
        }
        ++it;
    }
    HIPCHK(hipStreamSynchronize(s));
    h->prof_collect();
    if ((rc = chain_check(h, s)) != D3M_OK) return rc;
    if (info) {
        info->iterations = it;
        info->converged = ok ? 1 : 0;
        info->residual = res;
        info->copy_discrepancy = disc;
    }
    if (!ok) {
        char msg[96];
        std::snprintf(msg, sizeof(msg), "iterative refinement stopped at relative residual %.3e after %d steps", res,
                      it);
        return fail(D3M_ENOCONV, msg);
    }
    return D3M_OK;
}

}  // namespace

namespace d3m {

int set_error(int code, const char *msg) { return fail(code, msg); }

int handle_device(const d3m_problem *h) { return h->opt.device; }

int solve_scratch_bytes(const d3m_problem *h, int nrhs, size_t *bytes) {
    if (!h->device_ready) return fail(D3M_ESTATE, "handle was set up host-only");
    if (h->factored != 1) return fail(D3M_ESTATE, "the allocation-free solve needs FP64 factors (d3m_factor D3M_FP64)");
    size_t need = 0;
    for (int v = 0; v < VARR_COUNT; ++v) need += vec_bytes<double>(h, v, nrhs);
    *bytes = need;
    return D3M_OK;
}

int solve_into_scratch(d3m_problem *h, const double2 *f, double2 *E, int nrhs, void *scratch, size_t bytes,
                       hipStream_t s) {
    size_t need = 0;
    int rc = solve_scratch_bytes(h, nrhs, &need);
    if (rc != D3M_OK) return rc;
    if (need > bytes) return fail(D3M_EINVAL, "scratch too small");
    VBases vb;
    char *p = static_cast<char *>(scratch);
    for (int v = 0; v < VARR_COUNT; ++v) {
        vb.p[v] = p;
        p += vec_bytes<double>(h, v, nrhs);
    }
    h->quiet = true;
    rc = solve_launch_vb<double>(h, vb, f, E, nrhs, false, s);
    h->quiet = false;
    return rc;
}

}  // namespace d3m

namespace {

// max |L-hat| over the off-diagonal factor tiles of step 1 and of -K of the
// factors of precision T (one pass over those tiles; synchronous on s)
template <typename T>
int factor_growth(d3m_problem *h, double &s1, double &k, hipStream_t s) {
    if (!h->d_growth) {
        int rc = h->zeros(h->d_growth, 2 * sizeof(unsigned long long));
        if (rc != D3M_OK) return rc;
    }
    HIPCHK(hipMemsetAsync(h->d_growth, 0, 2 * sizeof(unsigned long long), s));
    Bases b = bases_of<T>(h);
    HIPCHK(launch_growth<T>(h->d_lhat_s1, (int64_t)h->pl.lhat_s1.size(), b, h->d_growth, s));
    HIPCHK(launch_growth<T>(h->d_lhat_k, (int64_t)h->pl.lhat_k.size(), b, h->d_growth + 1, s));
    unsigned long long bits[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(bits, h->d_growth, sizeof(bits), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::memcpy(&s1, &bits[0], sizeof(double));
    std::memcpy(&k, &bits[1], sizeof(double));
    return D3M_OK;
}

// The plan of a handle: build_plan, then the multifrontal schedule of step 5
// when the handle's options ask for it.
void make_plan(Plan &pl, const d3m_problem *h, int scope, int s1_block, int k_block, bool k_fuse) {
    build_plan(pl, h->dc, h->bo, scope == 1 ? 0 : TILE, s1_block, k_block, k_fuse, h->dc.s1_order == 1);
    build_solve_chain(pl);
    if (h->opt.k_multifrontal) build_multifrontal(pl, k_block > 0 ? k_block : 2);
    // loads on PEC edges are ignored: their subdomain rows start from zero
    if (h->mesh.n_pec > 0)
        for (auto &e : pl.split_map)
            if (e >= 0 && h->mesh.pec[e]) e = -1;
}

// Re-plans the handle for another pivot scope of step 5 (0: pieces of at most
// 64 rows, 1: whole blocks as in Algorithm 1).  The units, and with them the
// schedules, the pivot data of K and its storage, change; the factors are
// dropped.
int replan_scope(d3m_problem *h, int scope) {
    Plan np;
    try {
        make_plan(np, h, scope, h->tune.s1_block, h->tune.k_block, h->tune.k_fuse != 0);
    } catch (const Error &e) {
        return fail(D3M_EINVAL, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(D3M_ENOMEM, "host allocation failed in re-planning");
    }
    h->drop_graphs();
    const i64 old_status = h->pl.n_status, old_rows = h->pl.d_rows, old_scr = h->pl.bk_scratch_elems;
    h->pl = std::move(np);
    h->opt.pivot_scope = scope;
    h->factored = 0;
    h->vec_nrhs[0] = h->vec_nrhs[1] = 0;  // vector layouts are sized again on the next solve
    if (!h->device_ready) return D3M_OK;
    int rc;
    if ((rc = upload_schedules(h, true)) != D3M_OK) return rc;
    const Plan &pl = h->pl;
    if (pl.n_status > old_status && (rc = h->zeros(h->d_status, sizeof(int) * (pl.n_status + 1))) != D3M_OK)
        return rc;
    if (pl.d_rows > old_rows) {
        const size_t dr = (size_t)pl.d_rows;
        if ((rc = h->zeros(h->D.d, dr * sizeof(double2))) != D3M_OK) return rc;
        if ((rc = h->zeros(h->D.doff, dr * sizeof(double2))) != D3M_OK) return rc;
        if ((rc = h->zeros(h->D.dinv, dr * sizeof(double2))) != D3M_OK) return rc;
        if ((rc = h->zeros(h->D.dinvoff, dr * sizeof(double2))) != D3M_OK) return rc;
        if ((rc = h->zeros(h->D.piv, dr * sizeof(int))) != D3M_OK) return rc;
        if ((rc = h->zeros(h->D.perm, dr * sizeof(int))) != D3M_OK) return rc;
    }
    if (pl.bk_scratch_elems > old_scr &&
        (rc = h->zeros(h->d_bkscratch, (size_t)pl.bk_scratch_elems * sizeof(double2))) != D3M_OK)
        return rc;
    return D3M_OK;
}

// Host setup of a handle (mesh, decomposition, ordering, plan), then the
// device upload.  sub_group: problem of every subdomain (empty: one problem).
int setup_common(std::unique_ptr<d3m_problem> &h, int64_t nv, const double *xyz, int64_t nt, const int64_t *tets,
                 int64_t npec, const int64_t *pec, const int32_t *part, const double *eps_r, double k,
                 d3m_c128 alpha, const d3m_options *opt, std::vector<int> sub_group) {
    if (opt) h->opt = *opt; else d3m_default_options(&h->opt);
    if (h->opt.quad_points <= 0) h->opt.quad_points = 12;
    if (h->opt.ir_max_iter <= 0 && !opt) h->opt.ir_max_iter = 10;
    if (!(h->opt.ir_tol > 0)) h->opt.ir_tol = 1e-10;
    if (h->opt.pivot_scope != 0 && h->opt.pivot_scope != 1) return fail(D3M_EINVAL, "pivot_scope must be 0 or 1");
    if (h->opt.k_multifrontal != 0 && h->opt.k_multifrontal != 1)
        return fail(D3M_EINVAL, "k_multifrontal must be 0 or 1");
    if (h->opt.s1_order < 0 || h->opt.s1_order > 2) return fail(D3M_EINVAL, "s1_order must be 0, 1 or 2");
    try {
        build_mesh(h->mesh, nv, xyz, nt, tets);
        mark_pec(h->mesh, npec, pec);
        h->k = k;
        h->alpha = cplx(alpha.re, alpha.im);
        h->eps.assign(eps_r, eps_r + nt);
        build_decomposition(h->dc, h->mesh, part, k, h->alpha, eps_r, h->opt.s1_order);
        if (!sub_group.empty() && (int)sub_group.size() != h->dc.N)
            throw Error{-1, "a problem of the batch has an empty subdomain"};
        order_blocks(h->bo, h->dc, h->mesh, sub_group);
        make_plan(h->pl, h.get(), h->opt.pivot_scope, h->opt.s1_block, 0, false);
    } catch (const Error &e) {
        return fail(D3M_EINVAL, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(D3M_ENOMEM, "host allocation failed in setup");
    }
    h->tune.s1_block = h->opt.s1_block;
    h->sub_prob = sub_group.empty() ? std::vector<int>(h->dc.N, 0) : sub_group;
    if (h->prob_edge_off.empty()) h->prob_edge_off = {0, h->mesh.ne};
    if (h->prob_tet_off.empty()) h->prob_tet_off = {0, h->mesh.nt};
    h->eprob.assign(h->mesh.ne, 0);
    for (int p = 0; p < h->n_problems; ++p)
        for (int64_t e = h->prob_edge_off[p]; e < h->prob_edge_off[p + 1]; ++e) h->eprob[e] = p;
    if (!h->opt.host_only) {
        int rc = setup_device(h.get());
        if (rc != D3M_OK) return rc;
    }
    return D3M_OK;
}

}  // namespace

namespace {
// plane-wave loads of every boundary face; the face's problem p takes the
// direction and polarisation at dirs + 3 * (p * pstride + c)
void planewave_loads(d3m_problem *h, const double *dirs, const double *pols, int32_t nrhs, int32_t pstride,
                     d3m_c128 *f) {
    std::vector<double> qs, qt, qw;
    triangle_rule(h->opt.quad_points, qs, qt, qw);
    const int64_t ne = h->mesh.ne;
    std::memset(f, 0, sizeof(d3m_c128) * (size_t)nrhs * ne);
    for (int c = 0; c < nrhs; ++c) {
        for (i64 fi : h->dc.bface) {
            const int p = h->eprob[h->mesh.face_edges[3 * fi]];
            const size_t o = 3 * ((size_t)p * pstride + c);
            cplx out[3];
            face_planewave_load(h->mesh, fi, h->k, dirs + o, pols + o, qs, qt, qw, out);
            for (int a = 0; a < 3; ++a) {
                d3m_c128 &x = f[(size_t)c * ne + h->mesh.face_edges[3 * fi + a]];
                x.re += out[a].real();
                x.im += out[a].imag();
            }
        }
        if (h->mesh.n_pec > 0)
            for (int64_t e = 0; e < ne; ++e)
                if (h->mesh.pec[e]) f[(size_t)c * ne + e] = d3m_c128{0.0, 0.0};
    }
}

// the tetrahedron holding point r (largest smallest barycentric coordinate,
// the first one that holds it) and its barycentric coordinates; -1 outside
i64 locate_point(const Mesh &m, const double *r, double bl[4]) {
    i64 best = -1;
    double bestmin = -1e300;
    for (i64 t = 0; t < m.nt; ++t) {
        const double *x0 = &m.xyz[3 * m.tets[4 * t]];
        const double *g = &m.grads[12 * t];
        double l[4];
        const double d[3] = {r[0] - x0[0], r[1] - x0[1], r[2] - x0[2]};
        for (int a = 1; a < 4; ++a) l[a] = g[3 * a] * d[0] + g[3 * a + 1] * d[1] + g[3 * a + 2] * d[2];
        l[0] = 1.0 - l[1] - l[2] - l[3];
        const double mn = std::min(std::min(l[0], l[1]), std::min(l[2], l[3]));
        if (mn > bestmin) { bestmin = mn; best = t; std::memcpy(bl, l, sizeof(l)); }
        if (mn >= 0) break;
    }
    return (best < 0 || bestmin < -1e-12) ? -1 : best;
}
}  // namespace

// =========================================================== C ABI ======
extern "C" {

const char *d3m_last_error(void) { return g_err.c_str(); }

int d3m_set_profile(d3m_handle h, int level) {
    if (!h) return fail(D3M_EINVAL, "null handle");
    if (level < 0 || level > 2) return fail(D3M_EINVAL, "profile level must be 0, 1 or 2");
    h->opt.profile = level;
    return D3M_OK;
}

int d3m_set_graphs(d3m_handle h, int use_graph) {
    if (!h) return fail(D3M_EINVAL, "null handle");
    if (use_graph != 0 && use_graph != 1) return fail(D3M_EINVAL, "use_graph must be 0 or 1");
    if (!use_graph) h->drop_graphs();
    h->opt.use_graph = use_graph;
    return D3M_OK;
}

int d3m_get_tuning(d3m_handle h, d3m_tuning *t) {
    if (!h || !t) return fail(D3M_EINVAL, "null argument");
    *t = h->tune;
    return D3M_OK;
}

int d3m_set_tuning(d3m_handle h, const d3m_tuning *t) {
    if (!h || !t) return fail(D3M_EINVAL, "null argument");
    if (t->s1_block < 0 || t->s1_block > 16) return fail(D3M_EINVAL, "s1_block must be in [0, 16]");
    if (t->solve_cols != 0 && t->solve_cols != 16 && t->solve_cols != 32)
        return fail(D3M_EINVAL, "solve_cols must be 0, 16 or 32");
    if (t->lookahead_tasks < 0) return fail(D3M_EINVAL, "lookahead_tasks must be >= 0");
    if (t->k_block < 0 || t->k_block > 16) return fail(D3M_EINVAL, "k_block must be in [0, 16]");
    if (t->side_early != 0 && t->side_early != 1) return fail(D3M_EINVAL, "side_early must be 0 or 1");
    if (t->k_fuse != 0 && t->k_fuse != 1) return fail(D3M_EINVAL, "k_fuse must be 0 or 1");
    if (t->panel_rows != 0 && t->panel_rows != 16 && t->panel_rows != 64)
        return fail(D3M_EINVAL, "panel_rows must be 0, 16 or 64");
    if (t->solve_seq != 0 && t->solve_seq != 1) return fail(D3M_EINVAL, "solve_seq must be 0 or 1");
    if (t->solve_narrow < 0) return fail(D3M_EINVAL, "solve_narrow must be >= 0");
    if (t->k_overlap != 0 && t->k_overlap != 1) return fail(D3M_EINVAL, "k_overlap must be 0 or 1");
    if (t->solve_chain != 0 && t->solve_chain != 1) return fail(D3M_EINVAL, "solve_chain must be 0 or 1");
    if (t->reserved[0] != 0) return fail(D3M_EINVAL, "reserved tuning fields must be 0");
    const int old_s1 = h->tune.s1_block, old_k = h->tune.k_block, old_f = h->tune.k_fuse;
    h->drop_graphs();
    h->tune = *t;
    if (t->s1_block != old_s1 || t->k_block != old_k || t->k_fuse != old_f) {
        // the tile layout does not depend on the blocking: only the schedules
        // change (and the size of the multifrontal update-matrix pool, which
        // the next factorisation allocates)
        Plan np;
        try {
            make_plan(np, h, h->opt.pivot_scope, t->s1_block, t->k_block, t->k_fuse != 0);
        } catch (const Error &e) {
            return fail(D3M_EINVAL, e.msg);
        } catch (const std::bad_alloc &) {
            return fail(D3M_ENOMEM, "host allocation failed in re-planning");
        }
        const Plan &op = h->pl;
        if (np.m_tiles != op.m_tiles || np.k_tiles != op.k_tiles || np.tt_tiles != op.tt_tiles ||
            np.d_rows != op.d_rows || np.n_status != op.n_status || np.bk_scratch_elems != op.bk_scratch_elems)
            return fail(D3M_EINVAL, "internal: re-planning changed the storage layout");
        h->pl = std::move(np);
        h->opt.s1_block = t->s1_block;
        h->factored = 0;
        if (h->device_ready) return upload_schedules(h, true);
    }
    return D3M_OK;
}

void d3m_default_options(d3m_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->quad_points = 12;
    o->ir_max_iter = 10;
    o->ir_tol = 1e-10;
    o->pivot_fallback = 1;
}


int d3m_setup(const d3m_mesh *mesh, const int32_t *part, const double *eps_r, double k, d3m_c128 alpha,
              const d3m_options *opt, d3m_handle *out) {
    if (!out) return fail(D3M_EINVAL, "null output handle");
    *out = nullptr;
    if (!mesh || !mesh->xyz || !mesh->tets || !part || !eps_r) return fail(D3M_EINVAL, "null argument");
    if (mesh->n_pec_faces < 0 || (mesh->n_pec_faces > 0 && !mesh->pec_faces))
        return fail(D3M_EINVAL, "n_pec_faces > 0 needs pec_faces");
    std::unique_ptr<d3m_problem> h(new d3m_problem());
    int rc = setup_common(h, mesh->n_vertices, mesh->xyz, mesh->n_tets, mesh->tets, mesh->n_pec_faces,
                          mesh->pec_faces, part, eps_r, k, alpha, opt, {});
    if (rc != D3M_OK) return rc;
    *out = h.release();
    return D3M_OK;
}

int d3m_setup_batch(const d3m_batch_item *items, int32_t count, double k, d3m_c128 alpha, const d3m_options *opt,
                    d3m_handle *out) {
    if (!out) return fail(D3M_EINVAL, "null output handle");
    *out = nullptr;
    if (!items || count < 1) return fail(D3M_EINVAL, "a batch needs at least one problem");
    std::unique_ptr<d3m_problem> h(new d3m_problem());
    // disjoint union: vertex, tetrahedron and subdomain ids of problem p are
    // shifted past those of problems 0 .. p-1
    int64_t nv = 0, nt = 0;
    for (int p = 0; p < count; ++p) {
        const d3m_batch_item &it = items[p];
        if (!it.mesh.xyz || !it.mesh.tets || !it.part || !it.eps_r) return fail(D3M_EINVAL, "null argument in batch");
        if (it.mesh.n_vertices <= 0 || it.mesh.n_tets <= 0) return fail(D3M_EINVAL, "empty mesh in batch");
        nv += it.mesh.n_vertices;
        nt += it.mesh.n_tets;
    }
    std::vector<double> xyz;
    std::vector<int64_t> tets;
    std::vector<int32_t> part;
    std::vector<double> eps;
    std::vector<int64_t> pec;
    std::vector<int> sub_group;
    std::vector<int64_t> vert_off{0};
    try {
        xyz.reserve(3 * nv); tets.reserve(4 * nt); part.reserve(nt); eps.reserve(nt);
        h->prob_tet_off.assign(1, 0);
        int32_t sub0 = 0;
        for (int p = 0; p < count; ++p) {
            const d3m_batch_item &it = items[p];
            const int64_t v0 = vert_off.back();
            xyz.insert(xyz.end(), it.mesh.xyz, it.mesh.xyz + 3 * it.mesh.n_vertices);
            for (int64_t x = 0; x < 4 * it.mesh.n_tets; ++x) {
                const int64_t v = it.mesh.tets[x];
                if (v < 0 || v >= it.mesh.n_vertices) return fail(D3M_EINVAL, "tetrahedron vertex id out of range");
                tets.push_back(v + v0);
            }
            int32_t np = 0;
            for (int64_t t = 0; t < it.mesh.n_tets; ++t) {
                if (it.part[t] < 0) return fail(D3M_EINVAL, "negative subdomain id");
                np = std::max(np, it.part[t] + 1);
                part.push_back(it.part[t] + sub0);
            }
            eps.insert(eps.end(), it.eps_r, it.eps_r + it.mesh.n_tets);
            if (it.mesh.n_pec_faces < 0 || (it.mesh.n_pec_faces > 0 && !it.mesh.pec_faces))
                return fail(D3M_EINVAL, "n_pec_faces > 0 needs pec_faces");
            for (int64_t x = 0; x < 3 * it.mesh.n_pec_faces; ++x) {
                const int64_t v = it.mesh.pec_faces[x];
                if (v < 0 || v >= it.mesh.n_vertices) return fail(D3M_EINVAL, "PEC vertex id out of range");
                pec.push_back(v + v0);
            }
            for (int32_t d = 0; d < np; ++d) sub_group.push_back(p);
            sub0 += np;
            vert_off.push_back(v0 + it.mesh.n_vertices);
            h->prob_tet_off.push_back(h->prob_tet_off.back() + it.mesh.n_tets);
        }
    } catch (const std::bad_alloc &) {
        return fail(D3M_ENOMEM, "host allocation failed in batch setup");
    }
    h->n_problems = count;
    // edges are numbered by (lower vertex, higher vertex), so the edges of a
    // problem form one contiguous range, in problem order
    {
        Mesh probe;
        try {
            build_mesh(probe, nv, xyz.data(), nt, tets.data());
        } catch (const Error &e) {
            return fail(D3M_EINVAL, e.msg);
        }
        h->prob_edge_off.assign(count + 1, probe.ne);
        int p = 0;
        h->prob_edge_off[0] = 0;
        for (int64_t e = 0; e < probe.ne; ++e) {
            while (probe.edges[2 * e] >= vert_off[p + 1]) h->prob_edge_off[++p] = e;
        }
        for (int q = p + 1; q <= count; ++q) h->prob_edge_off[q] = probe.ne;
    }
    int rc = setup_common(h, nv, xyz.data(), nt, tets.data(), (int64_t)pec.size() / 3, pec.data(), part.data(),
                          eps.data(), k, alpha, opt, sub_group);
    if (rc != D3M_OK) return rc;
    *out = h.release();
    return D3M_OK;
}

int d3m_batch_layout(d3m_handle h, int32_t *count, int64_t *edge_off, int64_t *tet_off) {
    if (!h) return fail(D3M_EINVAL, "null handle");
    if (count) *count = h->n_problems;
    if (edge_off) std::copy(h->prob_edge_off.begin(), h->prob_edge_off.end(), edge_off);
    if (tet_off) std::copy(h->prob_tet_off.begin(), h->prob_tet_off.end(), tet_off);
    return D3M_OK;
}

int d3m_update_eps(d3m_handle h, const double *eps_r) {
    if (!h || !eps_r) return fail(D3M_EINVAL, "null argument");
    h->eps.assign(eps_r, eps_r + h->mesh.nt);
    reassemble_values(h->dc, h->mesh, h->k, eps_r);
    h->factored = 0;
    if (h->device_ready) {
        std::vector<double2> v;
        for (int d = 0; d < h->dc.N; ++d)
            for (auto &x : h->dc.sub[d].a_val) v.push_back(make_double2(x.real(), x.imag()));
        HIPCHK(hipMemcpy(h->d_coo_val, v.data(), v.size() * sizeof(double2), hipMemcpyHostToDevice));
        std::vector<int64_t> rp;
        std::vector<int32_t> col;
        std::vector<double2> val;
        build_global_csr(h->mesh, h->dc, h->k, eps_r, rp, col, val);
        HIPCHK(hipMemcpy(h->d_sval, val.data(), val.size() * sizeof(double2), hipMemcpyHostToDevice));
    }
    return D3M_OK;
}

int d3m_factor(d3m_handle h, int precision, void *stream) {
    if (!h) return fail(D3M_EINVAL, "null handle");
    if (!h->device_ready) return fail(D3M_ESTATE, "handle was set up host-only");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipSetDevice(h->opt.device));
    int rc;
    h->factored = 0;
    if (precision != D3M_FP64 && precision != D3M_FP32_IR) return fail(D3M_EINVAL, "unknown precision");
    auto run = [&]() { return precision == D3M_FP64 ? factor_impl<double>(h, s) : factor_impl<float>(h, s); };
    rc = run();
    if (h->opt.pivot_scope == 0 && h->opt.pivot_fallback) {
        // a piece of a block singular, or its multipliers grown past the
        // limit: factor again with the pivot search over whole blocks
        bool redo = rc == D3M_ESINGULAR;
        if (rc == D3M_OK && h->opt.growth_limit_log10 != 0) {
            double g1 = 0.0, gk = 0.0;
            const int rg = precision == D3M_FP64 ? factor_growth<double>(h, g1, gk, s)
                                                 : factor_growth<float>(h, g1, gk, s);
            if (rg != D3M_OK) return rg;
            redo = !(gk <= std::pow(10.0, h->opt.growth_limit_log10));
        }
        if (redo) {
            if ((rc = replan_scope(h, 1)) != D3M_OK) return rc;
            ++h->pivot_fallbacks;
            rc = run();
        }
    }
    if (rc == D3M_OK) h->factored = precision == D3M_FP64 ? 1 : 2;
    return rc;
}

int d3m_factor_growth(d3m_handle h, double *lhat_subdomains, double *lhat_k) {
    if (!h) return fail(D3M_EINVAL, "null handle");
    if (!h->factored) return fail(D3M_ESTATE, "growth before factor");
    HIPCHK(hipSetDevice(h->opt.device));
    double g1 = 0.0, gk = 0.0;
    const int rc = h->factored == 1 ? factor_growth<double>(h, g1, gk, nullptr) : factor_growth<float>(h, g1, gk, nullptr);
    if (rc != D3M_OK) return rc;
    if (lhat_subdomains) *lhat_subdomains = g1;
    if (lhat_k) *lhat_k = gk;
    return D3M_OK;
}

int d3m_solve(d3m_handle h, const d3m_c128 *rhs, int32_t nrhs, d3m_c128 *E, d3m_solve_info *info, void *stream) {
    if (!h || !rhs || !E) return fail(D3M_EINVAL, "null argument");
    if (nrhs < 1) return fail(D3M_EINVAL, "nrhs must be >= 1");
    if (!h->factored) return fail(D3M_ESTATE, "solve before factor");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipSetDevice(h->opt.device));
    const size_t bytes = sizeof(double2) * (size_t)nrhs * h->mesh.ne;
    const double2 *f = reinterpret_cast<const double2 *>(rhs);
    double2 *e = reinterpret_cast<double2 *>(E);
    bool fdev = is_device_ptr(rhs), edev = is_device_ptr(E);
    int rc;
    if (!fdev) {
        if ((rc = h->ensure(h->stage_f, bytes))) return rc;
        HIPCHK(hipMemcpyAsync(h->stage_f.p, rhs, bytes, hipMemcpyHostToDevice, s));
        f = (const double2 *)h->stage_f.p;
    }
    if (!edev) {
        if ((rc = h->ensure(h->stage_E, bytes))) return rc;
        e = (double2 *)h->stage_E.p;
    }
    rc = solve_device(h, f, e, nrhs, info, s);
    if (!edev && (rc == D3M_OK || rc == D3M_ENOCONV)) {
        HIPCHK(hipMemcpyAsync(E, e, bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    return rc;
}

int d3m_adjoint(d3m_handle h, const d3m_c128 *grad_E, const d3m_c128 *E, int32_t nrhs, double *grad_eps,
                d3m_c128 *w_out, void *stream) {
    if (!h || !grad_E || !E || !grad_eps) return fail(D3M_EINVAL, "null argument");
    if (nrhs < 1) return fail(D3M_EINVAL, "nrhs must be >= 1");
    if (!h->factored) return fail(D3M_ESTATE, "adjoint before factor");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipSetDevice(h->opt.device));
    const int64_t ne = h->mesh.ne;
    const size_t bytes = sizeof(double2) * (size_t)nrhs * ne;
    int rc;
    const double2 *g = reinterpret_cast<const double2 *>(grad_E);
    const double2 *ef = reinterpret_cast<const double2 *>(E);
    if (!is_device_ptr(grad_E)) {
        if ((rc = h->ensure(h->stage_f, bytes))) return rc;
        HIPCHK(hipMemcpyAsync(h->stage_f.p, grad_E, bytes, hipMemcpyHostToDevice, s));
        g = (const double2 *)h->stage_f.p;
    }
    if (!is_device_ptr(E)) {
        if ((rc = h->ensure(h->stage_E, bytes))) return rc;
        HIPCHK(hipMemcpyAsync(h->stage_E.p, E, bytes, hipMemcpyHostToDevice, s));
        ef = (const double2 *)h->stage_E.p;
    }
    if ((rc = h->ensure(h->stage_g, bytes))) return rc;
    if ((rc = h->ensure(h->stage_w, bytes))) return rc;
    HIPCHK(launch_conj((double2 *)h->stage_g.p, g, (int64_t)nrhs * ne, s));
    rc = solve_device(h, (double2 *)h->stage_g.p, (double2 *)h->stage_w.p, nrhs, nullptr, s);
    if (rc != D3M_OK) return rc;
    bool gdev = is_device_ptr(grad_eps);
    double *gout = grad_eps;
    DevBuf tmp;
    if (!gdev) {
        if ((rc = h->ensure(h->stage_r, sizeof(double) * h->mesh.nt))) return rc;
        gout = (double *)h->stage_r.p;
    }
    HIPCHK(launch_adjoint_grad(gout, (double2 *)h->stage_w.p, ef, h->d_tet_edges, h->d_mass, h->k * h->k,
                               h->mesh.nt, ne, nrhs, s));
    if (!gdev) HIPCHK(hipMemcpyAsync(grad_eps, gout, sizeof(double) * h->mesh.nt, hipMemcpyDeviceToHost, s));
    if (w_out) HIPCHK(hipMemcpyAsync(w_out, h->stage_w.p, bytes, hipMemcpyDefault, s));
    HIPCHK(hipStreamSynchronize(s));
    return D3M_OK;
}


int d3m_rhs_planewave(d3m_handle h, const double *dirs, const double *pols, int32_t nrhs, d3m_c128 *f) {
    if (!h || !dirs || !pols || !f) return fail(D3M_EINVAL, "null argument");
    if (nrhs < 1) return fail(D3M_EINVAL, "nrhs must be >= 1");
    planewave_loads(h, dirs, pols, nrhs, 0, f);
    return D3M_OK;
}

int d3m_rhs_planewave_batch(d3m_handle h, const double *dirs, const double *pols, int32_t nrhs, d3m_c128 *f) {
    if (!h || !dirs || !pols || !f) return fail(D3M_EINVAL, "null argument");
    if (nrhs < 1) return fail(D3M_EINVAL, "nrhs must be >= 1");
    planewave_loads(h, dirs, pols, nrhs, nrhs, f);
    return D3M_OK;
}

int d3m_rhs_dipole(d3m_handle h, const double *pos, const d3m_c128 *moment, int32_t nrhs, d3m_c128 *f) {
    if (!h || !pos || !moment || !f) return fail(D3M_EINVAL, "null argument");
    if (nrhs < 1) return fail(D3M_EINVAL, "nrhs must be >= 1");
    if (h->n_problems != 1) return fail(D3M_EINVAL, "dipole loads need a single-problem handle");
    const Mesh &m = h->mesh;
    static const int te[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    const int64_t ne = m.ne;
    std::memset(f, 0, sizeof(d3m_c128) * (size_t)nrhs * ne);
    const cplx scale = cplx(0.0, -h->k * D3M_ETA0);
    for (int c = 0; c < nrhs; ++c) {
        double bl[4];
        const i64 t = locate_point(m, pos + 3 * c, bl);
        if (t < 0) return fail(D3M_EINVAL, "dipole " + std::to_string(c) + " outside the mesh");
        const double *g = &m.grads[12 * t];
        const d3m_c128 *mo = moment + 3 * c;
        for (int a = 0; a < 6; ++a) {
            const int i = te[a][0], j = te[a][1];
            const i64 e = m.tet_edges[6 * t + a];
            if (!m.pec.empty() && m.pec[e]) continue;
            cplx dot = 0.0;
            for (int x = 0; x < 3; ++x)
                dot += cplx(mo[x].re, mo[x].im) * (bl[i] * g[3 * j + x] - bl[j] * g[3 * i + x]);
            const cplx v = scale * dot;
            f[(size_t)c * ne + e].re += v.real();
            f[(size_t)c * ne + e].im += v.imag();
        }
    }
    return D3M_OK;
}

int64_t d3m_debug_check_schedule(d3m_handle h, int32_t flags, char *report, int64_t report_bytes) {
    if (!h) return fail(D3M_EINVAL, "null handle");
    if (flags < 0 || flags > 15) return fail(D3M_EINVAL, "flags must be in [0, 15]");
    if (flags & 4) {
        std::string rep;
        int64_t bad = 0;
        try {
            bad = check_solve_chain(h->pl, (flags & 8) != 0, rep);
        } catch (const std::bad_alloc &) {
            return fail(D3M_ENOMEM, "host allocation failed in the queue simulation");
        }
        if (bad < 0) return fail(D3M_EINVAL, rep);
        if (report && report_bytes > 0) {
            const size_t n = std::min<size_t>(rep.size(), (size_t)report_bytes - 1);
            std::memcpy(report, rep.data(), n);
            report[n] = 0;
        }
        return bad;
    }
    const bool force_side = (flags & 1) != 0;
    ScheduleModel m;
    m.lookahead_tasks = h->tune.lookahead_tasks;
    m.side_early = h->tune.side_early;
    m.k_overlap = h->tune.k_overlap;
    // the streams the factorisation takes: whole-block units run the K phase
    // on one stream (run_factor_sweep) unless force_side asks for the
    // side-stream schedule anyway
    m.one_stream_k = h->opt.pivot_scope == 1 && !force_side;
    m.drop_waits = (flags & 2) != 0;
    std::string rep;
    int64_t races = 0;
    try {
        races = check_factor_schedule(h->pl, m, rep);
    } catch (const std::bad_alloc &) {
        return fail(D3M_ENOMEM, "host allocation failed in the schedule check");
    }
    if (report && report_bytes > 0) {
        const size_t n = std::min<size_t>(rep.size(), (size_t)report_bytes - 1);
        std::memcpy(report, rep.data(), n);
        report[n] = 0;
    }
    return races;
}

int d3m_debug_chain_wait_limit(d3m_handle h, double seconds) {
    if (!h) return fail(D3M_EINVAL, "null handle");
    if (!(seconds >= 0.0 && seconds <= 60.0)) return fail(D3M_EINVAL, "seconds must be in [0, 60]");
    if (!h->device_ready) return fail(D3M_ESTATE, "handle was set up host-only");
    h->chain_spin_ticks = (uint64_t)(seconds * 1000.0 * (double)h->chain_clock_khz);
    h->drop_solve_graphs();  // captured launches hold the old bound
    return D3M_OK;
}

int d3m_probe(d3m_handle h, const double *pts, int32_t n, int64_t *edges, double *coef) {
    if (!h || !pts || !edges || !coef) return fail(D3M_EINVAL, "null argument");
    if (h->n_problems != 1) return fail(D3M_EINVAL, "probe needs a single-problem handle");
    const Mesh &m = h->mesh;
    static const int te[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    for (int p = 0; p < n; ++p) {
        double bl[4] = {0, 0, 0, 0};
        const i64 best = locate_point(m, pts + 3 * p, bl);
        if (best < 0) return fail(D3M_EINVAL, "probe point outside the mesh");
        const double *g = &m.grads[12 * best];
        for (int a = 0; a < 6; ++a) {
            int i = te[a][0], j = te[a][1];
            edges[6 * p + a] = m.tet_edges[6 * best + a];
            for (int x = 0; x < 3; ++x) coef[18 * p + 3 * a + x] = bl[i] * g[3 * j + x] - bl[j] * g[3 * i + x];
        }
    }
    return D3M_OK;
}

int d3m_query(d3m_handle h, d3m_info *info) {
    if (!h || !info) return fail(D3M_EINVAL, "null argument");
    std::memset(info, 0, sizeof(*info));
    info->n_edges = h->mesh.ne;
    info->n_tets = h->mesh.nt;
    info->n_subdomains = h->dc.N;
    info->n_blocks = h->dc.nblk;
    info->n_lm = h->dc.n_lm;
    int mb = 0;
    for (int b = 0; b < h->dc.nblk; ++b) mb = std::max<int>(mb, (int)(h->dc.blk_start[b + 1] - h->dc.blk_start[b]));
    info->max_block = mb;
    info->n_levels = h->bo.n_levels;
    info->factor_bytes = (int64_t)h->pl.factor_entries * 16;
    int64_t dev = 0;
    for (auto &b : h->bufs) dev += (int64_t)b.bytes;
    for (int pr = 0; pr < 2; ++pr) {
        for (auto &b : h->arr[pr]) dev += (int64_t)b.bytes;
        for (auto &b : h->vec[pr]) dev += (int64_t)b.bytes;
    }
    info->device_bytes = dev;
    info->flops_domain = h->pl.flops_s1;
    info->flops_block_ldlt = h->pl.flops_s3;
    info->flops_update_gemm = h->pl.flops_update;
    info->solve_bytes = h->pl.solve_bytes;
    info->factored = h->factored;
    info->n_units = h->pl.k_units;
    info->n_unit_levels = h->pl.k_levels;
    info->n_problems = h->n_problems;
    info->array_bytes = (2 * h->pl.m_tiles + 3 * h->pl.k_tiles + h->pl.tt_tiles) * (int64_t)TILE_ELEMS * 16;
    info->mfma_flops_update = h->pl.mfma_flops_update;
    info->bytes_update_gemm = (double)h->pl.update_min_tiles * TILE_ELEMS * 16.0;
    info->pivot_scope = h->opt.pivot_scope;
    info->pivot_fallbacks = h->pivot_fallbacks;
    info->solve_vector_bytes = (double)h->pl.solve_min_vblocks * TILE * 16.0;
    info->k_multifrontal = h->pl.mf ? 1 : 0;
    info->s1_order = h->dc.s1_order;
    if (h->pl.mf) {
        info->mf_pool_bytes = (double)h->pl.ku_tiles * TILE_ELEMS * 16.0;
        info->mf_update_bytes = (double)h->pl.ku_tiles_total * TILE_ELEMS * 16.0;
        info->mf_extend_add_bytes = h->pl.mf_add_bytes;
        info->array_bytes += h->pl.ku_tiles * (int64_t)TILE_ELEMS * 16;
    }
    return D3M_OK;
}

void d3m_destroy(d3m_handle h) { delete h; }

int d3m_kernel_stats(d3m_handle h, int kernel, int reset, int64_t *launches, double *total_ms, double *flops) {
    if (!h) return fail(D3M_EINVAL, "null handle");
    if (kernel < 0 || kernel >= KID_COUNT) return fail(D3M_EINVAL, "unknown kernel id");
    if (launches) *launches = h->kstat_n[kernel];
    if (total_ms) *total_ms = h->kstat_ms[kernel];
    if (flops) *flops = h->kstat_flops[kernel];
    if (reset) { h->kstat_n[kernel] = 0; h->kstat_ms[kernel] = 0; h->kstat_flops[kernel] = 0; }
    return D3M_OK;
}

int64_t d3m_debug_export(d3m_handle h, int what, int64_t index, void *buf, int64_t bytes) {
    if (!h) return fail(D3M_EINVAL, "null handle");
    std::vector<char> out;
    auto put = [&](const void *p, size_t n) {
        const char *c = (const char *)p;
        out.insert(out.end(), c, c + n);
    };
    const Decomp &dc = h->dc;
    switch (what) {
    case D3M_EXPORT_EDGES: put(h->mesh.edges.data(), h->mesh.edges.size() * 8); break;
    case D3M_EXPORT_SUB_EDGES:
    case D3M_EXPORT_SUB_NI:
    case D3M_EXPORT_A_COO: {
        if (index < 0 || index >= dc.N) return fail(D3M_EINVAL, "subdomain index out of range");
        const Subdomain &S = dc.sub[index];
        if (what == D3M_EXPORT_SUB_EDGES) put(S.edges.data(), S.edges.size() * 8);
        else if (what == D3M_EXPORT_SUB_NI) put(&S.nI, 8);
        else
            for (size_t x = 0; x < S.a_row.size(); ++x) {
                double re = S.a_val[x].real(), im = S.a_val[x].imag();
                put(&S.a_row[x], 8); put(&S.a_col[x], 8); put(&re, 8); put(&im, 8);
            }
        break;
    }
    case D3M_EXPORT_LMS:
        for (i64 l = 0; l < dc.n_lm; ++l) { put(&dc.lm_p[l], 8); put(&dc.lm_q[l], 8); put(&dc.lm_e[l], 8); }
        break;
    case D3M_EXPORT_ORDER: put(h->bo.order.data(), h->bo.order.size() * 4); break;
    case D3M_EXPORT_STRUCT: {
        std::vector<int32_t> off{0}, lst;
        for (auto &s : h->bo.strct) { lst.insert(lst.end(), s.begin(), s.end()); off.push_back((int32_t)lst.size()); }
        put(off.data(), off.size() * 4);
        put(lst.data(), lst.size() * 4);
        break;
    }
    case D3M_EXPORT_KD: {
        if (h->factored != 1) return fail(D3M_ESTATE, "K_D export needs an FP64 factorisation");
        if (index < 0 || index >= dc.N) return fail(D3M_EINVAL, "subdomain index out of range");
        const Subdomain &S = dc.sub[index];
        const Plan &pl = h->pl;
        const i64 m = S.m;
        std::vector<double2> tiles((size_t)tri_slot(pl.TL[index], 0) * TILE_ELEMS);
        if (hipMemcpy(tiles.data(), (double2 *)h->arr[0][ARR_M].p + pl.m_tbase[index] * TILE_ELEMS,
                      tiles.size() * sizeof(double2), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(D3M_EHIP, "copy of the subdomain tiles failed");
        for (i64 r = 0; r < m; ++r)
            for (i64 c = 0; c < m; ++c) {
                i64 R = std::max(r, c), C = std::min(r, c);  // inside the trailing triangle
                double2 v = tiles[tri_slot(R / TILE, C / TILE) * TILE_ELEMS + (C % TILE) * TILE + R % TILE];
                double2 kd = make_double2(-v.x, -v.y);  // trailing block = -K_D
                put(&kd, sizeof(kd));
            }
        break;
    }
    case D3M_EXPORT_KFACTOR: {
        if (!h->factored) return fail(D3M_ESTATE, "not factored");
        const Plan &pl = h->pl;
        const i64 n = dc.n_lm;
        if (n > 20000) return fail(D3M_EINVAL, "factor export is for small problems");
        const int pr = h->factored == 1 ? 0 : 1;
        const size_t es = pr == 0 ? 16 : 8;
        std::vector<char> raw(pl.k_tiles * TILE_ELEMS * es);
        if (hipMemcpy(raw.data(), h->arr[pr][ARR_KL].p, raw.size(), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(D3M_EHIP, "copy of the K factor failed");
        auto tile_val = [&](i64 slot, int r, int c) -> double2 {
            size_t idx = (size_t)slot * TILE_ELEMS + (size_t)c * TILE + r;
            if (pr == 0) return ((double2 *)raw.data())[idx];
            float2 v = ((float2 *)raw.data())[idx];
            return make_double2(v.x, v.y);
        };
        std::vector<int> perm(pl.d_rows), piv(pl.d_rows);
        std::vector<double2> dd(pl.d_rows), doff(pl.d_rows);
        if (hipMemcpy(perm.data(), h->D.perm, pl.d_rows * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(dd.data(), h->D.d, pl.d_rows * 16, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(doff.data(), h->D.doff, pl.d_rows * 16, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(piv.data(), h->D.piv, pl.d_rows * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(D3M_EHIP, "copy of the pivot data failed");
        const int nu = pl.k_units;
        std::vector<i64> off(nu + 1, 0);
        for (int j = 0; j < nu; ++j) off[j + 1] = off[j] + pl.unit_n[j];
        int32_t nu32 = nu;
        put(&nu32, 4);
        put(pl.unit_n.data(), (size_t)nu * 4);
        std::vector<int32_t> pv(n);
        std::vector<double2> d0(n), d1(n);
        for (int j = 0; j < nu; ++j)
            for (int r = 0; r < pl.unit_n[j]; ++r) {
                pv[off[j] + r] = perm[pl.drow_k[j] + r];
                d0[off[j] + r] = dd[pl.drow_k[j] + r];
                d1[off[j] + r] = piv[pl.drow_k[j] + r] == 1 ? doff[pl.drow_k[j] + r] : make_double2(0, 0);
            }
        put(pv.data(), n * 4);
        put(d0.data(), n * 16);
        put(d1.data(), n * 16);
        std::vector<double2> L((size_t)n * n, make_double2(0, 0));
        for (int j = 0; j < nu; ++j) {
            // rows of panel j: unit j, then the units of its struct
            const std::vector<int> &ro = pl.krow_off[j];
            for (size_t ii = 0; ii < ro.size(); ++ii) {
                int i = ii == 0 ? j : pl.kstruct[j][ii - 1];
                for (int r = 0; r < pl.unit_n[i]; ++r)
                    for (int c = 0; c < pl.unit_n[j]; ++c) {
                        if (i == j && r < c) continue;
                        i64 slot = pl.kcol[j] + (i64)(c / TILE) * pl.kR[j] + ro[ii] + r / TILE;
                        L[(size_t)(off[i] + r) * n + off[j] + c] = tile_val(slot, r % TILE, c % TILE);
                    }
            }
        }
        put(L.data(), L.size() * 16);
        break;
    }
    case D3M_EXPORT_LAMBDA: {
        if (h->factored != 1) return fail(D3M_ESTATE, "multiplier export needs an FP64 solve");
        int nrhs = (int)index;
        if (nrhs < 1 || nrhs > h->vec_nrhs[0]) return fail(D3M_EINVAL, "index must be the nrhs of the last solve");
        const Plan &pl = h->pl;
        std::vector<double2> xk((size_t)pl.v_tiles_k * 64 * nrhs);
        if (hipMemcpy(xk.data(), h->vec[0][V_KX].p, xk.size() * 16, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(D3M_EHIP, "copy of the multipliers failed");
        for (int c = 0; c < nrhs; ++c)
            for (i64 l = 0; l < dc.n_lm; ++l) {
                i64 R = pl.lm_vrow[l];
                put(&xk[(size_t)(R / 64) * 64 * nrhs + (size_t)c * 64 + R % 64], 16);
            }
        break;
    }
    default: return fail(D3M_EINVAL, "unknown export selector");
    }
    if (buf) {
        if (bytes < (int64_t)out.size()) return fail(D3M_EINVAL, "export buffer too small");
        std::memcpy(buf, out.data(), out.size());
    }
    return (int64_t)out.size();
}

// Test hook: the Bunch-Kaufman kernels of the factorisation on caller blocks.
int d3m_debug_bk(const d3m_c128 *a, int32_t n, int32_t count, int precision, int variant, int device,
                 d3m_bk_out *out) {
    if (!a || !out || n < 1 || n > 1024 || count < 1) return fail(D3M_EINVAL, "bad block arguments");
    if (precision != D3M_FP64 && precision != D3M_FP32_IR) return fail(D3M_EINVAL, "unknown precision");
    if (variant < 0 || variant > 2) return fail(D3M_EINVAL, "variant must be 0, 1 or 2");
    if (variant == 1 && bk_lds_bytes(n, ((n + 63) / 64) * 64, true) > 160 * 1024 - 256)
        return fail(D3M_EINVAL, "block too large for the LDS variant");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= device || device < 0)
        return fail(D3M_ENODEV, "no such HIP device");
    HIPCHK(hipSetDevice(device));
    const bool f32 = precision == D3M_FP32_IR;
    const size_t es = f32 ? 8 : 16;
    const int t = (n + TILE - 1) / TILE;
    const size_t blk = (size_t)t * t * TILE_ELEMS;  // tile elements per block
    const size_t ne = blk * count;
    // host staging in the kernels' tile layout: tile (b, c) of block q at
    // q*blk + (c*t + b)*4096, column-major inside a tile
    std::vector<double2> A(ne, make_double2(0, 0));
    for (int q = 0; q < count; ++q)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j <= i; ++j) {
                const d3m_c128 v = a[((size_t)q * n + i) * n + j];
                A[q * blk + ((size_t)(j / TILE) * t + i / TILE) * TILE_ELEMS + (j % TILE) * TILE + i % TILE] =
                    make_double2(v.re, v.im);
            }
    std::vector<float2> Af;
    if (f32) {
        Af.resize(ne);
        for (size_t e = 0; e < ne; ++e) Af[e] = make_float2((float)A[e].x, (float)A[e].y);
    }
    std::vector<BkTask> tasks(count);
    for (int q = 0; q < count; ++q) {
        BkTask &k = tasks[q];
        std::memset(&k, 0, sizeof(k));
        k.a = enc(ARR_M, (int64_t)(q * blk));
        k.l = enc(ARR_KL, (int64_t)(q * blk));
        k.tt = enc(ARR_TT, (int64_t)(q * blk));
        k.drow = (int64_t)q * n;
        k.n = n;
        k.ldt = (int32_t)((size_t)t * TILE_ELEMS);
        k.status = q;
    }
    struct Mem {
        std::vector<void *> ps;
        ~Mem() { for (void *p : ps) (void)hipFree(p); }
        hipError_t get(void **p, size_t bytes) {
            hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
            if (e == hipSuccess) ps.push_back(*p);
            return e;
        }
    } mem;
    void *dA, *dL, *dT, *dtask, *dstat, *dscr = nullptr;
    void *dd[4], *dpiv, *dperm;
    HIPCHK(mem.get(&dA, ne * es));
    HIPCHK(mem.get(&dL, ne * es));
    HIPCHK(mem.get(&dT, ne * es));
    HIPCHK(mem.get(&dtask, sizeof(BkTask) * count));
    HIPCHK(mem.get(&dstat, sizeof(int) * count));
    for (int x = 0; x < 4; ++x) HIPCHK(mem.get(&dd[x], sizeof(double2) * n * count));
    HIPCHK(mem.get(&dpiv, sizeof(int) * n * count));
    HIPCHK(mem.get(&dperm, sizeof(int) * n * count));
    if (n > 64 || variant != 0) HIPCHK(mem.get(&dscr, sizeof(double2) * ((size_t)n * (n + 1) / 2) * count));
    HIPCHK(hipMemcpy(dA, f32 ? (const void *)Af.data() : (const void *)A.data(), ne * es, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(dL, 0, ne * es));
    HIPCHK(hipMemset(dT, 0, ne * es));
    HIPCHK(hipMemset(dstat, 0, sizeof(int) * count));
    HIPCHK(hipMemcpy(dtask, tasks.data(), sizeof(BkTask) * count, hipMemcpyHostToDevice));
    Bases b{};
    b.p[ARR_M] = dA;
    b.p[ARR_KL] = dL;
    b.p[ARR_TT] = dT;
    DArrays D{(double2 *)dd[0], (double2 *)dd[1], (double2 *)dd[2], (double2 *)dd[3], (int *)dpiv, (int *)dperm};
    if (f32) HIPCHK(launch_bk<float>((const BkTask *)dtask, count, n, nullptr, b, D, (int *)dstat,
                                     (double2 *)dscr, nullptr, variant));
    else HIPCHK(launch_bk<double>((const BkTask *)dtask, count, n, nullptr, b, D, (int *)dstat,
                                  (double2 *)dscr, nullptr, variant));
    HIPCHK(hipDeviceSynchronize());
    std::vector<int> st(count);
    HIPCHK(hipMemcpy(st.data(), dstat, sizeof(int) * count, hipMemcpyDeviceToHost));
    auto tile_val = [&](const std::vector<double2> &src, const std::vector<float2> &srcf, int q, int i, int j) {
        const size_t e = q * blk + ((size_t)(j / TILE) * t + i / TILE) * TILE_ELEMS + (j % TILE) * TILE + i % TILE;
        return f32 ? d3m_c128{srcf[e].x, srcf[e].y} : d3m_c128{src[e].x, src[e].y};
    };
    if (out->L || out->tt) {
        std::vector<double2> h(f32 ? 0 : ne);
        std::vector<float2> hf(f32 ? ne : 0);
        for (int which = 0; which < 2; ++which) {
            d3m_c128 *dst = which == 0 ? out->L : out->tt;
            if (!dst) continue;
            HIPCHK(hipMemcpy(f32 ? (void *)hf.data() : (void *)h.data(), which == 0 ? dL : dT, ne * es,
                             hipMemcpyDeviceToHost));
            for (int q = 0; q < count; ++q)
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j)
                        dst[((size_t)q * n + i) * n + j] = (which == 0 && j > i) ? d3m_c128{0, 0} : tile_val(h, hf, q, i, j);
        }
    }
    d3m_c128 *douts[4] = {out->d, out->doff, out->dinv, out->dinvoff};
    for (int x = 0; x < 4; ++x)
        if (douts[x]) HIPCHK(hipMemcpy(douts[x], dd[x], sizeof(double2) * n * count, hipMemcpyDeviceToHost));
    if (out->kind) HIPCHK(hipMemcpy(out->kind, dpiv, sizeof(int) * n * count, hipMemcpyDeviceToHost));
    if (out->perm) HIPCHK(hipMemcpy(out->perm, dperm, sizeof(int) * n * count, hipMemcpyDeviceToHost));
    if (out->singular) std::memcpy(out->singular, st.data(), sizeof(int) * count);
    for (int q = 0; q < count; ++q)
        if (st[q] != 0)
            return fail(D3M_ESINGULAR, "singular pivot block: block " + std::to_string(q) + ", column " +
                                           std::to_string(st[q] - 1));
    return D3M_OK;
}

}  // extern "C"
