// Host-side launchers of the HIP kernels (declarations).
#pragma once

#include <hip/hip_runtime.h>

#include "../tasks.hpp"

namespace d3m {

// Pivot data of every diagonal block, FP64 for both precisions, indexed by
// the "D row" of the block (see the planner).
struct DArrays {
    double2 *d, *doff;      // D diagonal and 2x2 off-diagonal
    double2 *dinv, *dinvoff;
    int *piv;               // 0: 1x1, 1: first row of a 2x2, -1: second row
    int *perm;              // block-local permutation
};

struct VBases {
    void *p[VARR_COUNT];
};

template <typename T> hipError_t launch_fill_zero(void *p, int64_t n, hipStream_t s);
hipError_t launch_zero_i32(int *p, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_coo_scatter(void *M, const int64_t *off, const double2 *val, int64_t n, hipStream_t s);
// variant: 0 as the factorisation runs it (register kernel for blocks of at
// most 64 rows, else the general kernel with the block in LDS when it fits,
// else in `scratch`); 1 the general kernel with the block in LDS; 2 the
// general kernel with the block in global scratch (tests of every kernel)
template <typename T>
hipError_t launch_bk(const BkTask *tasks, int64_t ntask, int maxn, const GemmPair *pairs, const Bases &b,
                     const DArrays &D, int *status,
                     double2 *scratch, hipStream_t s, int variant = 0);
size_t bk_lds_bytes(int n, int nthr, bool lds);
template <typename T>
hipError_t launch_gemm(const GemmTask *tasks, int64_t ntask, const GemmPair *pairs, const Bases &b, int mode,
                       hipStream_t s);
template <typename T>
hipError_t launch_scale(const ScaleTask *tasks, int64_t ntask, const Bases &b, const DArrays &D, hipStream_t s);
template <typename T>
hipError_t launch_panel_scale(const GemmTask *tasks, const ScaleTask *stasks, int64_t ntask, const GemmPair *pairs,
                              const Bases &b, const DArrays &D, int rows, hipStream_t s);
template <typename T> hipError_t launch_asm(const AsmTask *tasks, int64_t ntask, const Bases &b, hipStream_t s);
// multifrontal extend-adds: one work-group per destination tile
template <typename T>
hipError_t launch_extend_add(const AddTask *tasks, int64_t ntask, const int64_t *srcs, const Bases &b,
                             hipStream_t s);
// max |entry| over the valid part of the given factor tiles, folded into
// *gmax (bit pattern of a non-negative double; zeroed by the caller)
template <typename T>
hipError_t launch_growth(const FactorTile *tiles, int64_t ntile, const Bases &b, unsigned long long *gmax,
                         hipStream_t s);

// solve sweeps
template <typename T>
hipError_t launch_vsplit(void *X, const double2 *f, const int64_t *map, int64_t nrows, int nrhs, int64_t ne,
                         hipStream_t s);
// cols: right-hand sides per work-group (16 or 32; 0 = 32)
template <typename T>
hipError_t launch_vdiag(const VDiagTask *tasks, int64_t ntask, int maxt, bool bwd, const Bases &b, const VBases &vb,
                        const DArrays &D, int nrhs, int cols, hipStream_t s);
template <typename T>
hipError_t launch_vupd(const VUpdTask *tasks, const int64_t *fuse, int64_t ntask, const VUpdPair *pairs,
                       const VDiagTask *vdiag, int mode, const Bases &b, const VBases &vb, const DArrays &D, int nrhs,
                       int cols, hipStream_t s);
// a whole S1 sweep, one work-group per subdomain (and column block) running
// its ordered task list [off[d], off[d + 1]) (forward: mode 0, backward: mode 1)
template <typename T>
hipError_t launch_vseq(const VUpdTask *tasks, const int64_t *fuse, const int64_t *off, int nsub,
                       const VUpdPair *pairs, const VDiagTask *vdiag, bool bwd, const Bases &b, const VBases &vb,
                       const DArrays &D, int nrhs, int cols, hipStream_t s);
// a whole sweep over the factor of -K in one launch, from the work-queue item
// list of build_solve_chain (forward: update mode 0, backward: mode 2; the
// list's pre-launched diagonal solves must be complete).
// head: the sweep's queue counter, err: the sticky timeout flag, cnt: one
// write counter per K vector tile; head and cnt zeroed by launch_vchain_reset
// before the sweep.  spin_ticks bounds every dependency wait (wall-clock
// ticks).
template <typename T>
hipError_t launch_vchain(const ChainItem *items, int64_t nitem, const ChainWait *waits, const VUpdTask *tasks,
                         const VUpdPair *pairs, const VDiagTask *vdiag, bool bwd, const Bases &b,
                         const VBases &vb, const DArrays &D, int nrhs, int cols, unsigned *head, unsigned *err,
                         unsigned *cnt, uint64_t spin_ticks, hipStream_t s);
// head[0..1] = 0 and cnt[0..n) = 0 (a kernel, so graphs may hold it)
hipError_t launch_vchain_reset(unsigned *head, unsigned *cnt, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_vgather_h(void *XK, const void *X, const int64_t *hmap, int64_t nrows_k, int nrhs, hipStream_t s);
template <typename T>
hipError_t launch_vscatter_lam(void *X, const void *XK, const int64_t *lmap, int64_t nrows_s1, int nrhs,
                               hipStream_t s);
template <typename T>
hipError_t launch_vcollect(double2 *E, const void *X, const int64_t *cmap, int64_t ne, int nrhs, bool accumulate,
                           hipStream_t s);

// largest |difference| between a non-owner subdomain copy of a shared edge
// (row r of the subdomain vectors X, cmap[r] = its owner's row, else -1) and
// the owner copy, over all right-hand sides, folded into *dmax (bit pattern of
// a non-negative double; zeroed by the caller)
template <typename T>
hipError_t launch_copy_disc(unsigned long long *dmax, const void *X, const int64_t *cmap, int64_t nrows, int nrhs,
                            hipStream_t s);

// refinement and adjoint
// r = f - S E; the largest |r| over the rows of each problem (eprob: problem
// of every row) and right-hand side is folded into nmax[p * nrhs + c]
// (zeroed by the caller)
hipError_t launch_residual(double2 *r, const double2 *f, const double2 *E, double2 *Et, const int64_t *rowptr,
                           const int32_t *col, const double2 *val, const int32_t *eprob, int64_t ne, int nrhs,
                           unsigned long long *nmax, hipStream_t s);
hipError_t launch_rownorm_max(unsigned long long *nmax, const double2 *v, const int32_t *eprob, int64_t ne, int nrhs,
                              hipStream_t s);
hipError_t launch_conj(double2 *out, const double2 *in, int64_t n, hipStream_t s);
hipError_t launch_adjoint_grad(double *grad, const double2 *w, const double2 *E, const int64_t *tet_edges,
                               const double *mass, double k2, int64_t nt, int64_t ne, int nrhs, hipStream_t s);

}  // namespace d3m
