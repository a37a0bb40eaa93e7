/*
 * d3m.h -- C ABI of the MI355X D3M factor/solve library (libd3m.so).
 *
 * Method: Moshfegh & Vouvakis, "Direct Domain Decomposition Method (D3M) for
 * Finite Element Electromagnetic Computations" (ICEAA 2016).  The library
 * discretises the decomposed boundary-value problem of Section II with
 * lowest-order Nedelec (Whitney) edge elements and a first-order absorbing
 * boundary, couples box subdomains by one set of Robin-type Lagrange
 * multipliers (eq. (1)), and solves the saddle system by
 *   step 1  dense domain matrices K_D^(d) = D_d^T A_d^{-1} D_d,
 *   step 2  assembly of the block-wise sparse reduced matrix K,
 *   steps 3-4 nested-dissection ordering and block symbolic factorisation,
 *   step 5  block LDL^T of K with Bunch-Kaufman pivoting restricted to each
 *           diagonal block (Algorithm 1),
 *   steps 6-7 forward/diagonal/backward substitution and recovery of E.
 * Steps 1, 2, 5, 6 and 7 run on the GPU; steps 3-4 and the FEM assembly run
 * on the host inside d3m_setup.
 *
 * Conventions
 *   - Complex numbers are interleaved (re, im) pairs of doubles, the layout
 *     of C99 double _Complex and of a torch.complex128 tensor.
 *   - All matrices are complex symmetric (A^T = A, never conjugated).
 *   - Time convention e^{+j omega t}; incident plane wave p exp(-jk d.r).
 *   - Every function returns D3M_OK (0) or a negative status; the message of
 *     the last failure on the calling thread is d3m_last_error().
 *   - Functions taking a `stream` accept a hipStream_t (NULL = default
 *     stream).  They enqueue their GPU work on that stream and return after
 *     it has completed unless stated otherwise.
 *   - Buffers passed to d3m_solve / d3m_adjoint may live in host memory or in
 *     device memory of the current device; the library inspects the pointer
 *     (hipPointerGetAttributes).  Caller keeps ownership of all buffers.
 */
#ifndef D3M_H
#define D3M_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define D3M_OK          0
#define D3M_EINVAL     -1  /* invalid argument, mesh or partition            */
#define D3M_ESINGULAR  -2  /* a restricted pivot block has a zero column     */
#define D3M_ENOMEM     -3  /* device or host allocation failed               */
#define D3M_EHIP       -4  /* a HIP runtime call failed                      */
#define D3M_ESTATE     -5  /* call out of order (e.g. solve before factor)   */
#define D3M_ENOCONV    -6  /* iterative refinement missed its tolerance      */
#define D3M_ENODEV     -7  /* no usable HIP device                           */

/* ---- factorisation precisions ------------------------------------------ */
#define D3M_FP64       0   /* complex128 everywhere                          */
#define D3M_FP32_IR    1   /* complex64 factor and sweeps (Bunch-Kaufman
                              pivot choice, 2x2 inverses and D in FP64) plus
                              FP64 iterative refinement on the global system */

typedef struct { double re, im; } d3m_c128;

typedef struct d3m_problem *d3m_handle;

/* Tetrahedral mesh.  xyz: [n_vertices][3] row-major; tets: [n_tets][4],
 * 0-based vertex ids (any vertex order; the library sorts each tetrahedron so
 * every local edge points from the lower to the higher global vertex id).
 * pec_faces: [n_pec_faces][3] vertex ids of mesh triangles on perfectly
 * conducting surfaces (n x E = 0, the PEC scatterers of Section III), or
 * NULL with n_pec_faces = 0.  Every edge of such a triangle has a zero
 * tangential field: it is no unknown of any subdomain system and carries no
 * multiplier; E is 0 there and loads on it are ignored.  A triple that is not
 * a face of the mesh is refused (D3M_EINVAL). */
typedef struct {
    int64_t n_vertices;
    const double *xyz;
    int64_t n_tets;
    const int64_t *tets;
    int64_t n_pec_faces;
    const int64_t *pec_faces;
} d3m_mesh;

/* Free-space wave impedance (ohm) of the impressed-current term -jk eta J_imp
 * of the BVP (Section II, first line). */
#define D3M_ETA0 376.730313668

typedef struct {
    int32_t host_only;    /* 1: d3m_setup stops before any HIP call; only the
                             host products (d3m_debug_export) are available  */
    int32_t quad_points;  /* Gauss points per direction of the collapsed
                             triangle rule for the plane-wave load (default 12) */
    int32_t ir_max_iter;  /* FP32_IR: maximum refinement steps (default 10)  */
    int32_t profile;      /* timing with HIP events for d3m_kernel_stats:
                             0 off, 1 the update GEMM launches only, 2 every
                             kernel group (each timed launch adds a little
                             overhead; 2 adds about a tenth on 24^3 hexes
                             in 64 subdomains)                              */
    double ir_tol;        /* FP32_IR: stop when max over right-hand sides of
                             ||f - S E||_inf / ||f||_inf <= ir_tol (1e-10)   */
    int32_t use_graph;    /* 1: d3m_factor captures its launch sequence into a
                             HIP graph on first use (per precision) and
                             replays it; d3m_solve does the same per
                             (precision, rhs and E buffers, nrhs), keeping at
                             most 8 solve graphs.  Graphs run on a stream of
                             the handle, ordered after the work already on
                             the caller's stream and before its later work.
                             Profiling events are not recorded in graphs.   */
    int32_t device;       /* HIP device ordinal (default 0)                   */
    int32_t pivot_scope;  /* Bunch-Kaufman pivot search of step 5 restricted
                             to: 0 (default) consecutive pieces of at most 64
                             rows of each block of K; 1 whole blocks, as in
                             Algorithm 1 (slower: the search is sequential)  */
    int32_t s1_block;     /* tile columns of a subdomain matrix whose Schur
                             updates beyond them are applied together (one
                             read-modify-write of each target per block);
                             0 selects the default 2, at most 16            */
    int32_t pivot_fallback; /* 1 (default): with pivot_scope 0, a factorisation
                             that finds a piece of a block singular (or whose
                             multipliers exceed growth_limit_log10) is redone
                             with the whole-block scope of Algorithm 1, which
                             the handle keeps from then on; 0: report the
                             error instead                                   */
    int32_t growth_limit_log10; /* 0 (default): no growth check; otherwise,
                             with pivot_scope 0 and pivot_fallback, every
                             factorisation measures max |L-hat_ij| over the
                             factor of -K (one pass over its off-diagonal
                             tiles) and falls back to the whole-block scope
                             when it exceeds 10^growth_limit_log10          */
    int32_t k_multifrontal; /* 0 (default): step 5 right-looking, every unit's
                             Schur updates applied in place to the block
                             columns of its structure; 1: its multifrontal
                             form (the variant named after the seven steps of
                             Section II): a unit's updates go to its update
                             matrix, which its parent's front adds in
                             (extend-add).  Same factors up to the order of
                             rounding; needs an extra pool of update
                             matrices (d3m_info.mf_pool_bytes)               */
    int32_t s1_order;     /* row order of the edge part of each subdomain
                             matrix M_d in step 1: 0 (default) interior then
                             interface edges, each by global id (A_d
                             banded); 1 nested dissection of all its edge
                             rows (geometric bisection, separators after
                             both sides; step 1 and its solve sweeps run by
                             levels of the dissection tree); 2 the
                             dissection when the median subdomain has at
                             least 4,000 edge rows (about 8^3 hexes), the
                             banded order otherwise.  The multiplier rows
                             come last either way; the tile pattern
                             follows the fill of the order taken
                             (d3m_info.s1_order)                             */
    int32_t reserved[2];
} d3m_options;

typedef struct {
    int64_t n_edges;          /* global unknowns (edges)                     */
    int64_t n_tets;
    int32_t n_subdomains;     /* N                                           */
    int32_t n_blocks;         /* l: blocks (subdomain pairs) of K            */
    int64_t n_lm;             /* Lagrange multipliers = order of K           */
    int32_t max_block;        /* largest block order                         */
    int32_t n_levels;         /* elimination-tree levels of the block graph  */
    int64_t factor_bytes;     /* device bytes held for the factors           */
    int64_t device_bytes;     /* all device bytes held by the handle         */
    double flops_domain;      /* algorithmic flops of step 1 (complex
                                 multiply-add = 8 flops)                     */
    double flops_block_ldlt;  /* algorithmic flops of step 5                 */
    double flops_update_gemm; /* algorithmic flops of all Schur-update GEMMs */
    double solve_bytes;       /* algorithmic factor bytes read by one solve
                                 (complex128), excluding vector traffic      */
    int32_t factored;         /* 0 none, else D3M_FP64 + 1 or D3M_FP32_IR + 1 */
    int32_t n_units;          /* pivot units of K (blocks or pieces of blocks) */
    int32_t n_unit_levels;    /* elimination-tree levels over the units       */
    int32_t n_problems;       /* independent problems held (1 unless batched) */
    int64_t array_bytes;      /* device bytes of the factor arrays of one
                                 precision (complex128; half for FP32_IR)     */
    double mfma_flops_update; /* the update GEMMs' work as executed: full
                                 64x64x64 tile products, counted like
                                 flops_update_gemm (flops_update_gemm divided
                                 by this is the share of MFMA work that is not
                                 tile padding or upper halves of diagonal
                                 tiles)                                       */
    double bytes_update_gemm; /* least HBM bytes of all update GEMMs of one
                                 factorisation (complex128; half for FP32):
                                 per elimination step every distinct operand
                                 tile read once and every target tile read and
                                 written once                                 */
    double solve_vector_bytes;/* least vector bytes moved by the update
                                 launches of one solve, per right-hand side
                                 (complex128): per sweep step each distinct
                                 source block read once, each target read and
                                 written once; factor bytes are solve_bytes   */
    int32_t pivot_scope;      /* pivot scope of step 5 in effect (0 pieces of
                                 at most 64 rows, 1 whole blocks)             */
    int32_t pivot_fallbacks;  /* factorisations redone with the whole-block
                                 scope (options.pivot_fallback)               */
    int32_t k_multifrontal;   /* 1 when step 5 runs in multifrontal form      */
    int32_t s1_order;         /* row order the subdomain matrices got: 0
                                 banded, 1 nested dissection (options.s1_order
                                 2 resolved)                                  */
    double mf_pool_bytes;     /* device bytes of the update-matrix pool of one
                                 precision (complex128; half for FP32_IR), 0
                                 in the right-looking form                    */
    double mf_update_bytes;   /* bytes of all update matrices of one
                                 factorisation without reuse (complex128)     */
    double mf_extend_add_bytes; /* bytes the extend-adds of one factorisation
                                 read and write (complex128)                  */
} d3m_info;

typedef struct {
    int32_t iterations;       /* refinement steps taken (0 for FP64)         */
    int32_t converged;        /* 1 when the residual test passed             */
    double residual;          /* final max_rhs ||f - S E||_inf / ||f||_inf
                                 (FP64 evaluation; computed for both modes)   */
    double copy_discrepancy;  /* max over shared edges e, right-hand sides and
                                 pairs of subdomain copies of |E_d[e] - E_d'[e]|
                                 (the recovered subdomain fields of step 7; the
                                 continuity D^T E = 0 of eq. (1) holds up to
                                 the rounding of lambda).  FP32_IR: the sum of
                                 this figure over the solve passes, a bound
                                 for the refined field                       */
} d3m_solve_info;

/* Fill `opt` with the defaults listed above. */
void d3m_default_options(d3m_options *opt);

/* Build the decomposed FEM system (Section II: the BVP, eq. (1); recipe
 * steps 3-4) on the host and upload it to the device.
 *   mesh   tetrahedral mesh (copied).
 *   part   [n_tets] subdomain of each tetrahedron, ids dense in [0, N).
 *   eps_r  [n_tets] real relative permittivity (mu_r = 1).
 *   k      free-space wavenumber, > 0.
 *   alpha  Robin coefficient of the transmission condition (e.g. -jk).
 *   opt    options (NULL = defaults).
 * On success *out receives a handle that owns all device memory.
 * Errors: D3M_EINVAL (degenerate tetrahedron, non-manifold mesh, partition id
 * out of range, empty subdomain, k <= 0, an edge whose subdomains are not
 * connected through shared triangles), D3M_ENOMEM, D3M_ENODEV, D3M_EHIP. */
int d3m_setup(const d3m_mesh *mesh, const int32_t *part, const double *eps_r,
              double k, d3m_c128 alpha, const d3m_options *opt, d3m_handle *out);

/* One problem of a batch: its mesh, partition (ids dense in [0, N_p)) and
 * eps_r, with the same meaning as the arguments of d3m_setup. */
typedef struct {
    d3m_mesh mesh;
    const int32_t *part;
    const double *eps_r;
} d3m_batch_item;

/* Batch of `count` independent problems at one wavenumber k and Robin
 * coefficient alpha (Section II applied to each problem; the problems share
 * no unknowns, so their systems do not couple).  The handle holds their
 * disjoint union: every phase runs over the subdomains of all problems at
 * once (uneven subdomain sizes included) and the block elimination tree of
 * K is a forest with one nested-dissection tree per problem.  Edges and
 * tetrahedra of problem p are the contiguous ranges [edge_off[p],
 * edge_off[p+1]) and [tet_off[p], tet_off[p+1]) of the handle's numbering
 * (d3m_batch_layout), in each problem's own order, so a right-hand side or
 * solution of the batch is [nrhs][sum of n_edges] with problem p's columns
 * in its range.  The refinement tolerance of FP32_IR holds for every problem
 * and right-hand side separately.  Errors as for d3m_setup. */
int d3m_setup_batch(const d3m_batch_item *items, int32_t count, double k,
                    d3m_c128 alpha, const d3m_options *opt, d3m_handle *out);

/* Number of problems and the offsets above ([count + 1] each; any output
 * pointer may be NULL).  A handle from d3m_setup holds one problem. */
int d3m_batch_layout(d3m_handle h, int32_t *count, int64_t *edge_off,
                     int64_t *tet_off);

/* Replace eps_r ([n_tets], copied), reassemble the subdomain matrices and
 * invalidate the factors.  Errors: D3M_EINVAL, D3M_EHIP. */
int d3m_update_eps(d3m_handle h, const double *eps_r);

/* Recipe steps 1, 2 and 5 on the device (Algorithm 1): dense interior
 * elimination of every subdomain into its domain matrix, assembly of K, block
 * LDL^T of K with Bunch-Kaufman pivoting restricted to each diagonal block.
 * precision: D3M_FP64 or D3M_FP32_IR.  Returns after the stream completes.
 * With pivot_scope 0 and options.pivot_fallback set, a singular piece (or
 * multipliers beyond options.growth_limit_log10) makes the call re-plan the
 * handle for whole-block pivoting and factor again (d3m_info.pivot_scope,
 * .pivot_fallbacks).
 * Errors: D3M_ESINGULAR (a pivot block is singular; d3m_last_error names the
 * block and column; there are no delayed pivots), D3M_ENOMEM, D3M_EHIP. */
int d3m_factor(d3m_handle h, int precision, void *stream);

/* Growth monitor of the last factorisation: the largest |entry| of the
 * off-diagonal factor blocks L-hat_ij = X_ij D_jj^{-1} (Algorithm 1; their
 * size is bounded by no pivoting, since pivots are searched only inside a
 * diagonal block and none is delayed), over the tile columns of step 1
 * (lhat_subdomains) and over the units of -K (lhat_k).  One pass over those
 * tiles on the default stream; synchronous.  NULL outputs are skipped.
 * Errors: D3M_ESTATE (not factored), D3M_EHIP. */
int d3m_factor_growth(d3m_handle h, double *lhat_subdomains, double *lhat_k);

/* Recipe steps 6-7: E = S^{-1} f for nrhs right-hand sides.
 *   rhs  [nrhs][n_edges] complex128 (global load f, row per right-hand side).
 *   E    [nrhs][n_edges] complex128 output.
 *   info optional diagnostics (NULL allowed).
 * FP32_IR handles refine in FP64 on the global system until ir_tol: each
 * step computes r = f - S E in FP64 and adds the FP32 solution of S d = r,
 * over the right-hand sides whose relative residual is still above ir_tol
 * (in some problem of a batch); the others keep their field.
 * Errors: D3M_ESTATE (not factored), D3M_EINVAL (nrhs < 1), D3M_ENOCONV
 * (refinement missed ir_tol; E holds the best iterate), D3M_EHIP. */
int d3m_solve(d3m_handle h, const d3m_c128 *rhs, int32_t nrhs, d3m_c128 *E,
              d3m_solve_info *info, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid hipMalloc): the FP64 solve
 * of d3m_solve (steps 6-7) with its working vectors in a fixed device array
 * of D3M_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs
 * on until the process ends.  Only kernel launches are enqueued on `stream`
 * (no allocation, no memset, no host synchronisation); the call returns
 * without waiting for them.
 *   rhs, E  [nrhs][n_edges] complex128 device buffers (caller-owned).
 * The handle must hold FP64 factors.  The scratch of one GPU is shared by all
 * handles and calls on it: calls whose kernels overlap on one GPU (other
 * streams, other host threads) race and must be serialised by the caller.
 * Errors: D3M_EINVAL (null or host buffers, nrhs < 1, or a scratch need above
 * D3M_NOALLOC_SCRATCH_BYTES: the message gives the need), D3M_ESTATE (not
 * factored in FP64, host-only handle), D3M_EHIP. */
#define D3M_NOALLOC_SCRATCH_BYTES (64ull << 20)
int d3m_solve_noalloc(d3m_handle h, const d3m_c128 *rhs, int32_t nrhs, d3m_c128 *E,
                      void *stream);

/* Adjoint of E = S(eps_r)^{-1} f with respect to eps_r, reusing the factors
 * (S is complex symmetric, so S^{-T} = S^{-1}):
 *   w = S^{-1} conj(grad_E),  grad_eps[t] = k^2 Re sum_rhs w_t^T M_t E_t,
 * with M_t the unit-eps_r mass matrix of tetrahedron t.
 *   grad_E [nrhs][n_edges] dL/dRe E + j dL/dIm E (PyTorch's convention).
 *   E      [nrhs][n_edges] the forward solution.
 *   grad_eps [n_tets] real output (overwritten).  w_out optional [nrhs][n_edges].
 * Errors as for d3m_solve. */
int d3m_adjoint(d3m_handle h, const d3m_c128 *grad_E, const d3m_c128 *E,
                int32_t nrhs, double *grad_eps, d3m_c128 *w_out, void *stream);

/* Plane-wave load of the absorbing boundary (second line of the BVP):
 * f = -oint N . (n x curl E_inc - jk E_inc,t) dS with E_inc = p exp(-jk d.r).
 *   dirs, pols [nrhs][3] unit propagation directions and polarisations.
 *   f [nrhs][n_edges] host output.  Works on host-only handles. */
int d3m_rhs_planewave(d3m_handle h, const double *dirs, const double *pols,
                      int32_t nrhs, d3m_c128 *f);

/* d3m_rhs_planewave with its own waves per problem of a batch:
 *   dirs, pols [count][nrhs][3]; f [nrhs][n_edges] host output. */
int d3m_rhs_planewave_batch(d3m_handle h, const double *dirs,
                            const double *pols, int32_t nrhs, d3m_c128 *f);

/* Loads of point dipoles (the impressed current J_imp of the BVP in Section
 * II, first line), one per right-hand side: J_imp = m_c delta(r - r_c) with
 * position pos[c] ([nrhs][3]) and complex current moment m_c = moment[c]
 * ([nrhs][3], I l in A m), giving f[c][e] = -jk eta0 m_c . N_e(r_c) (N_e the
 * Whitney function of edge e in the tetrahedron holding r_c; zero on PEC
 * edges).  f: host buffer [nrhs][n_edges], overwritten.  Single-problem
 * handles only; D3M_EINVAL for a point outside the mesh. */
int d3m_rhs_dipole(d3m_handle h, const double *pos, const d3m_c128 *moment, int32_t nrhs, d3m_c128 *f);

/* Static race check of the factorisation schedule of the handle's plan and
 * tuning (no GPU needed: host_only handles work): the launches of one
 * factorisation are replayed with their streams, event records and waits,
 * and every tile each work-group reads or writes (working, panel, factor
 * and TT tiles, pivot-data rows) is checked against the other accesses that
 * are not ordered before or after it.  Returns the number of conflicting
 * pairs found (0: race-free) or a negative error; a description of the
 * first ones is copied to report (NUL-terminated, at most report_bytes,
 * NULL allowed).  flags: bit 0 models the side-stream schedule for
 * whole-block pivot units too (which the library does not launch); bit 1
 * leaves out every stream wait for earlier side-stream updates (a planted
 * mistake, so tests can see the check report it).  Bit 2 checks the
 * work-queue form of the two K solve sweeps instead (d3m_tuning.solve_chain):
 * a host simulation in which workers take the items from one counter and
 * wait on the tiles' write counts as the kernel does, under pseudo-random
 * interleavings; it counts every item that would see a tile with other
 * writes than the level-by-level order gives it, and a stalled queue
 * (D3M_EINVAL where the plan has no such form); bit 3 then leaves out each
 * item's first wait (planted mistake).  For the race detection of the
 * factor schedules and the queue (tests), not the paper. */
int64_t d3m_debug_check_schedule(d3m_handle h, int32_t flags, char *report, int64_t report_bytes);

/* Bound of one dependency wait of the work-queue K solve sweeps
 * (d3m_tuning.solve_chain), in seconds of the device's wall clock (default 2;
 * 0 makes every wait that is not met at once run out, so a test can see the
 * solve fail with D3M_EHIP while every kernel still ends normally).
 * Errors: D3M_EINVAL (seconds outside [0, 60]), D3M_ESTATE (host-only
 * handle).  For tests of the failure path, not the paper. */
int d3m_debug_chain_wait_limit(d3m_handle h, double seconds);

/* Whitney field evaluation at points: for point m, E(r_m) = sum_a c[m][a][:] *
 * u[edge[m][a]] over the six edges of the tetrahedron containing r_m.
 *   pts [n][3]; edges [n][6] (int64) and coef [n][6][3] (double) host outputs.
 * Errors: D3M_EINVAL when a point lies outside the mesh or the handle holds
 * a batch. */
int d3m_probe(d3m_handle h, const double *pts, int32_t n, int64_t *edges,
              double *coef);

int d3m_query(d3m_handle h, d3m_info *info);
void d3m_destroy(d3m_handle h);
const char *d3m_last_error(void);

/* Switch opt.use_graph for later calls (0 drops the captured graphs).
 * Errors: D3M_EINVAL. */
int d3m_set_graphs(d3m_handle h, int use_graph);

/* Launch-shape choices of the schedules; paper_2002_05018_amd.autotune picks
 * them by timing.  Zero selects the default. */
typedef struct {
    int32_t s1_block;        /* tile columns of a subdomain matrix whose Schur
                                updates beyond them are applied together
                                (d3m_options.s1_block; default 2, at most 16) */
    int32_t solve_cols;      /* right-hand sides per work-group of the solve
                                sweeps: 16 or 32 (default 32)                 */
    int32_t lookahead_tasks; /* an elimination step whose updates off the
                                next step's columns number at least this many
                                tasks runs them on a second stream (512)     */
    int32_t k_block;         /* longest chain of pivot units of K (each the
                                only child of the next in the elimination
                                tree) whose updates beyond the chain are
                                applied together (default 2, at most 16)     */
    int32_t side_early;      /* 1: a step's second-stream updates start as
                                soon as its panels are done; 0 (default):
                                after its critical updates, so that the next
                                pivot launch finds free compute units        */
    int32_t k_fuse;          /* 1: the updates of the next level's columns of
                                K are applied by that level's pivot and panel
                                launches (one launch fewer per level) instead
                                of a separate update launch; default 0       */
    int32_t panel_rows;      /* rows of a panel tile per work-group: 64
                                (default) or 16 (four work-groups per tile,
                                so a short block column's panel products
                                run on four times as many compute units)    */
    int32_t solve_seq;       /* 1: each subdomain sweep of the solve (steps 6
                                and 7 over the factors of step 1) is one
                                launch in which a work-group runs one
                                subdomain's tile columns in order, every
                                target gathering all its products at once;
                                0 (default): one launch per tile column over
                                all subdomains                               */
    int32_t solve_narrow;    /* sweep steps with fewer update tasks than this
                                take 16 right-hand sides per work-group
                                whatever solve_cols says (more, shorter
                                work-groups where a step is latency-bound);
                                0 (default): never                           */
    int32_t k_overlap;       /* 1: the block-LDL^T updates of K off the next
                                level's columns go to two side streams (the
                                next few levels' columns, the rest), and every
                                launch waits only for the launches that wrote
                                its block columns, so the bulk updates of a
                                chain segment overlap the next segment's pivot
                                chain; 0 (default): one side stream, each step
                                waiting for the previous step's side updates */
    int32_t solve_chain;     /* 1: each of the two solve sweeps over the
                                factor of -K runs as one launch whose
                                work-groups take the update tasks in the
                                level-by-level order from a work queue, each
                                waiting (bounded, 2 s) only for the writes of
                                the vector tiles it reads; same results bit
                                for bit.  A wait that runs out fails the
                                solve with D3M_EHIP (d3m_solve_noalloc: the
                                next d3m_solve or d3m_adjoint on the handle
                                reports it).  Ignored where the plan holds
                                diagonal blocks of several tiles (whole-block
                                pivot units); 0 (default): one launch per
                                level and phase                              */
    int32_t reserved[1];
} d3m_tuning;

/* Read / replace the tuning.  A new s1_block, k_block or k_fuse rebuilds the factor schedule
 * (the storage layout is unchanged) and invalidates the factors; any change
 * drops captured graphs.  Errors: D3M_EINVAL (value out of range). */
int d3m_get_tuning(d3m_handle h, d3m_tuning *t);
int d3m_set_tuning(d3m_handle h, const d3m_tuning *t);

/* Change the profiling level of opt.profile (0, 1 or 2) for later calls.
 * Returns D3M_EINVAL for another level or a null handle. */
int d3m_set_profile(d3m_handle h, int level);

/* Per-kernel timings recorded while opt.profile > 0 (reset by this call when
 * reset != 0).  kernel: 0 update GEMM, 1 panel GEMM, 2 Bunch-Kaufman block,
 * 3 scatter/assembly, 4 solve sweeps, 5 refinement residual.  Outputs: number
 * of launches, summed launch milliseconds and algorithmic flops. */
int d3m_kernel_stats(d3m_handle h, int kernel, int reset, int64_t *launches,
                     double *total_ms, double *flops);

/* ---- host-side products for parity tests --------------------------------
 * d3m_debug_export copies one product into a caller-provided host buffer of
 * `bytes` bytes and returns the number of bytes needed (call with buf = NULL
 * to size it), or a negative status.  `index` selects a subdomain where
 * relevant.
 *   D3M_EXPORT_EDGES     int64 [n_edges][2] global edges (lo, hi)
 *   D3M_EXPORT_SUB_EDGES int64 [n_d] global edge of each row of subdomain
 *                        `index` in its elimination order ([interior |
 *                        interface], or the nested-dissection order with
 *                        -1 on the padding rows that start each group at
 *                        a tile boundary)
 *   D3M_EXPORT_SUB_NI    int64 [1] interior edge count of subdomain `index`
 *   D3M_EXPORT_A_COO     {int64 row, int64 col, double re, double im}[nnz]
 *                        lower triangle of A_d in the subdomain's order
 *   D3M_EXPORT_LMS       int64 [n_lm][3] (p, q, edge) in global LM order
 *   D3M_EXPORT_ORDER     int32 [n_blocks] block (canonical id) eliminated at
 *                        each position
 *   D3M_EXPORT_STRUCT    int32 CSR of struct(j) by position: [l+1] offsets
 *                        followed by the position lists
 *   D3M_EXPORT_KD        complex128 [m][m] domain matrix K_D^(index) in
 *                        global-LM order (after d3m_factor, FP64 only)
 *   D3M_EXPORT_KFACTOR   the factor of -K over the pivot units in
 *                        elimination order (units are consecutive rows of
 *                        the blocks in D3M_EXPORT_ORDER): int32 n_units,
 *                        int32 [n_units] unit sizes, int32 [n_lm] perm
 *                        within the unit, complex128 [n_lm] D diagonal,
 *                        complex128 [n_lm] D sub-diagonal (first row of a
 *                        2x2 pivot), then complex128 [n_lm][n_lm] row-major
 *                        unit lower L whose diagonal unit blocks are L_jj and
 *                        whose off-diagonal unit blocks are L-hat_ij (rows in
 *                        the unit's original order); small problems only
 *   D3M_EXPORT_LAMBDA    complex128 [nrhs][n_lm] multipliers of the last
 *                        solve in global LM order                           */
#define D3M_EXPORT_EDGES      1
#define D3M_EXPORT_SUB_EDGES  2
#define D3M_EXPORT_SUB_NI     3
#define D3M_EXPORT_A_COO      4
#define D3M_EXPORT_LMS        5
#define D3M_EXPORT_ORDER      6
#define D3M_EXPORT_STRUCT     7
#define D3M_EXPORT_KD         8
#define D3M_EXPORT_KFACTOR    9
#define D3M_EXPORT_LAMBDA    10
int64_t d3m_debug_export(d3m_handle h, int what, int64_t index, void *buf,
                         int64_t bytes);

/* ---- test hook: the Bunch-Kaufman kernels on caller blocks ---------------
 * Runs the kernels that factor the diagonal blocks of step 5 (the first line
 * of Algorithm 1: P^T K_jj P = L D L^T with Bunch-Kaufman 1x1/2x2 pivoting
 * restricted to the block, no delayed pivots) and the diagonal tiles of
 * step 1 on `count` independent blocks of order n, so that their pivot
 * decisions and outputs can be compared with a reference one by one.
 *   a         [count][n][n] host, row-major complex symmetric blocks (only
 *             the lower triangle is read)
 *   n         1..1024
 *   precision D3M_FP64 (blocks stored in complex128) or D3M_FP32_IR (stored
 *             in complex64: the input is rounded to it; the pivot search, D
 *             and D^{-1} stay FP64 as in the factorisation)
 *   variant   0 the kernel d3m_factor uses for this order (register kernel
 *             for n <= 64, else the general kernel with the block in LDS if
 *             it fits, else in global memory); 1 the general kernel with the
 *             block in LDS (D3M_EINVAL if it does not fit); 2 the general
 *             kernel with the block in global memory
 *   device    HIP device ordinal
 * Outputs (host arrays owned by the caller; any pointer may be NULL):
 *   L        [count][n][n] row-major unit lower L of P^T A P (upper zero)
 *   d, doff  [count][n] diagonal of D and the off-diagonal of each 2x2 pivot
 *            (stored on both of its rows; 0 for 1x1 pivots)
 *   dinv, dinvoff [count][n] the same for D^{-1}
 *   kind     [count][n] 0: 1x1 pivot, 1: first row of a 2x2, -1: second row
 *   perm     [count][n] (P^T A P)[i][j] = A[perm[i]][perm[j]]
 *   tt       [count][n][n] row-major L^{-1} P^T (what the sweeps apply)
 *   singular [count] 0, or 1 + the column at which no pivot was found
 * Returns D3M_ESINGULAR (naming the first singular block and column) when a
 * block has a zero column; the outputs of the other blocks are still
 * written.  Allocates and frees its own device memory.  Errors: D3M_EINVAL,
 * D3M_ENODEV, D3M_ENOMEM, D3M_EHIP. */
typedef struct {
    d3m_c128 *L;
    d3m_c128 *d, *doff;
    d3m_c128 *dinv, *dinvoff;
    int32_t *kind;
    int32_t *perm;
    d3m_c128 *tt;
    int32_t *singular;
} d3m_bk_out;
int d3m_debug_bk(const d3m_c128 *a, int32_t n, int32_t count, int precision,
                 int variant, int device, d3m_bk_out *out);

#ifdef __cplusplus
}
#endif
#endif /* D3M_H */
