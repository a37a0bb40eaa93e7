// Factor-phase kernels: initialisation of the subdomain matrices, the
// Bunch-Kaufman factorisation of diagonal blocks (pivoting restricted to the
// block, reference [bunch1977] of the paper), the complex Schur-update GEMM on
// MFMA, the L-hat = X D^{-1} scaling and the assembly of -K.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace d3m {

// ------------------------------------------------------------ utilities --
template <typename T2>
__global__ void fill_zero_kernel(T2 *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = T2{0, 0};
}

template <typename T2>
__global__ void coo_scatter_kernel(T2 *M, const int64_t *off, const double2 *val, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) M[off[i]] = from_d2<T2>(val[i]);
}

// ----------------------------------------------------- Bunch-Kaufman ----
// One work-group per diagonal block; thread i owns row i (blockDim >= n).
// The block is copied into packed lower column-major storage (LDS when it
// fits, otherwise a per-block global scratch) and factored in FP64 for both
// precisions:  P^T A P = L D L^T with 1x1 and 2x2 pivots.  Pivot choice:
//   lam1 = max_{i>k} |a_ik| (row r, lowest index on ties), |z| = |Re|+|Im|;
//   |a_kk| >= alpha lam1                     -> 1x1 at k
//   sigma = max_{i>=k, i!=r} |a_ir|:
//   |a_kk| sigma >= alpha lam1^2              -> 1x1 at k
//   |a_rr| >= alpha sigma                     -> swap k<->r, 1x1
//   otherwise                                 -> swap k+1<->r, 2x2
// with alpha = (1 + sqrt 17)/8.  A zero column (lam1 = a_kk = 0) is reported
// in status[] as column+1; there are no delayed pivots.
// Outputs: unit lower L (same tile layout as the input), perm, D, D^{-1}
// (1x1 reciprocals; 2x2 inverses [[c,-b],[-b,a]]/(ac-b^2)), the pivot kind
// and TT = L^{-1} P^T.
constexpr double kAlphaBK = 0.64038820320220756872767623199676;  // (1+sqrt(17))/8

__device__ __forceinline__ int64_t pk(int i, int j, int n) {  // packed lower, i >= j
    return (int64_t)j * n - (int64_t)j * (j - 1) / 2 + (i - j);
}
__device__ __forceinline__ int64_t pks(int i, int j, int n) { return i >= j ? pk(i, j, n) : pk(j, i, n); }
__device__ __forceinline__ int64_t tile_elem(int i, int j, int ldt) {
    return (int64_t)(i >> 6) * TILE_ELEMS_D + (int64_t)(j >> 6) * ldt + (j & 63) * 64 + (i & 63);
}

__device__ void block_argmax(double v, int i, double *rv, int *ri, double &ov, int &oi) {
    for (int off = 32; off >= 1; off >>= 1) {
        double v2 = __shfl_xor(v, off);
        int i2 = __shfl_xor(i, off);
        if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
    }
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { rv[w] = v; ri[w] = i; }
    __syncthreads();
    v = rv[0]; i = ri[0];
    int nw = blockDim.x >> 6;
    for (int x = 1; x < nw; ++x)
        if (rv[x] > v || (rv[x] == v && ri[x] < i)) { v = rv[x]; i = ri[x]; }
    __syncthreads();
    ov = v; oi = i;
}

template <typename T2, bool LDS>
__global__ void bk_kernel(const BkTask *tasks, Bases bases, DArrays D, int *status,
                          double2 *scratch, int64_t scratch_stride) {
    extern __shared__ double2 smem[];
    const BkTask tk = tasks[blockIdx.x];
    const int n = tk.n, tid = threadIdx.x, nthr = blockDim.x;
    double2 *A = LDS ? smem : scratch + (int64_t)blockIdx.x * scratch_stride;
    int64_t aoff = LDS ? (int64_t)n * (n + 1) / 2 : 0;
    double2 *xv0 = smem + aoff;
    double2 *xv1 = xv0 + nthr;
    double *rv = reinterpret_cast<double *>(xv1 + nthr);
    int *ri = reinterpret_cast<int *>(rv + 16);
    int *sperm = ri + 16;

    const T2 *src = enc_ptr<T2>(bases, tk.a);
    for (int j = 0; j < n; ++j)
        for (int i = j + tid; i < n; i += nthr) A[pk(i, j, n)] = to_d2(src[tile_elem(i, j, tk.ldt)]);
    for (int i = tid; i < n; i += nthr) sperm[i] = i;
    __syncthreads();

    const int64_t dr = tk.drow;
    int k = 0;
    bool singular = false;
    while (k < n) {
        double v = -1.0;
        if (tid > k && tid < n) v = cabs1(A[pk(tid, k, n)]);
        double lam1;
        int r;
        block_argmax(v, tid, rv, ri, lam1, r);
        if (lam1 < 0.0) { lam1 = 0.0; r = k; }  // no rows below k (NaN keeps its row)
        if (r < k || r >= n) r = k;
        const double akk = cabs1(A[pk(k, k, n)]);
        int size = 1, p = k;
        if (!(fmax(akk, lam1) > 0.0)) {
            singular = true;
        } else if (akk >= kAlphaBK * lam1) {
            size = 1; p = k;
        } else {
            double v2 = -1.0;
            if (tid >= k && tid < n && tid != r) v2 = cabs1(A[pks(tid, r, n)]);
            double sigma;
            int dummy;
            block_argmax(v2, tid, rv, ri, sigma, dummy);
            if (akk * sigma >= kAlphaBK * lam1 * lam1) { size = 1; p = k; }
            else if (cabs1(A[pk(r, r, n)]) >= kAlphaBK * sigma) { size = 1; p = r; }
            else { size = 2; p = r; }
        }
        if (singular) break;
        const int kk = k + size - 1;
        if (p != kk) {
            if (tid < n && tid != kk && tid != p) {
                int64_t a1 = pks(kk, tid, n), a2 = pks(p, tid, n);
                double2 t = A[a1]; A[a1] = A[a2]; A[a2] = t;
            }
            if (tid == 0) {
                int64_t a1 = pk(kk, kk, n), a2 = pk(p, p, n);
                double2 t = A[a1]; A[a1] = A[a2]; A[a2] = t;
                int s = sperm[kk]; sperm[kk] = sperm[p]; sperm[p] = s;
            }
        }
        __syncthreads();
        if (size == 1) {
            const double2 d = A[pk(k, k, n)];
            const double2 di = crecip(d);
            double2 l = make_double2(0.0, 0.0);
            if (tid > k && tid < n) {
                double2 x = A[pk(tid, k, n)];
                l = cmul(x, di);
                xv0[tid] = x;
            }
            __syncthreads();
            if (tid > k && tid < n) {
                for (int j = k + 1; j <= tid; ++j) {
                    int64_t a = pk(tid, j, n);
                    A[a] = cfms(A[a], l, xv0[j]);
                }
                A[pk(tid, k, n)] = l;
            }
            if (tid == 0) {
                D.d[dr + k] = d; D.doff[dr + k] = make_double2(0, 0);
                D.dinv[dr + k] = di; D.dinvoff[dr + k] = make_double2(0, 0);
                D.piv[dr + k] = 0;
            }
        } else {
            const double2 a = A[pk(k, k, n)], b = A[pk(k + 1, k, n)], c = A[pk(k + 1, k + 1, n)];
            const double2 idet = crecip(csub(cmul(a, c), cmul(b, b)));
            const double2 e11 = cmul(c, idet), e22 = cmul(a, idet);
            const double2 e12 = make_double2(-(b.x * idet.x - b.y * idet.y), -(b.x * idet.y + b.y * idet.x));
            double2 l0 = make_double2(0, 0), l1 = make_double2(0, 0);
            if (tid > k + 1 && tid < n) {
                double2 x0 = A[pk(tid, k, n)], x1 = A[pk(tid, k + 1, n)];
                l0 = cadd(cmul(x0, e11), cmul(x1, e12));
                l1 = cadd(cmul(x0, e12), cmul(x1, e22));
                xv0[tid] = x0;
                xv1[tid] = x1;
            }
            __syncthreads();
            if (tid > k + 1 && tid < n) {
                for (int j = k + 2; j <= tid; ++j) {
                    int64_t aa = pk(tid, j, n);
                    A[aa] = cfms(cfms(A[aa], l0, xv0[j]), l1, xv1[j]);
                }
                A[pk(tid, k, n)] = l0;
                A[pk(tid, k + 1, n)] = l1;
            }
            if (tid == 0) {
                D.d[dr + k] = a; D.d[dr + k + 1] = c;
                D.doff[dr + k] = b; D.doff[dr + k + 1] = b;
                D.dinv[dr + k] = e11; D.dinv[dr + k + 1] = e22;
                D.dinvoff[dr + k] = e12; D.dinvoff[dr + k + 1] = e12;
                D.piv[dr + k] = 1; D.piv[dr + k + 1] = -1;
                A[pk(k + 1, k, n)] = make_double2(0, 0);
            }
        }
        __syncthreads();
        k += size;
    }
    if (singular) {
        if (tid == 0) status[tk.status] = k + 1;
        return;
    }
    // unit lower L to the output tiles, perm to the D arrays
    T2 *lout = enc_ptr<T2>(bases, tk.l);
    for (int j = 0; j < n; ++j)
        for (int i = j + tid; i < n; i += nthr)
            lout[tile_elem(i, j, tk.ldt)] = from_d2<T2>(i == j ? make_double2(1.0, 0.0) : A[pk(i, j, n)]);
    for (int i = tid; i < n; i += nthr) D.perm[dr + i] = sperm[i];
    __syncthreads();
    // Z = L^{-1} in place, one row at a time:
    //   Z(r,c) = -L(r,c) - sum_{c<t<r} L(r,t) Z(t,c)
    for (int r = 1; r < n; ++r) {
        if (tid < r) xv0[tid] = A[pk(r, tid, n)];
        __syncthreads();
        if (tid < r) {
            double2 acc = make_double2(-xv0[tid].x, -xv0[tid].y);
            for (int t = tid + 1; t < r; ++t) acc = cfms(acc, xv0[t], A[pk(t, tid, n)]);
            A[pk(r, tid, n)] = acc;
        }
        __syncthreads();
    }
    // TT = Z P^T: TT[b][perm[a]] = Z[b][a]; tile (bt, ct) at tt + (ct*t + bt)*4096
    T2 *tt = enc_ptr<T2>(bases, tk.tt);
    const int t = (n + 63) >> 6;
    for (int64_t e = tid; e < (int64_t)t * t * TILE_ELEMS_D; e += nthr) tt[e] = T2{0, 0};
    __syncthreads();
    for (int a = 0; a < n; ++a) {
        const int col = sperm[a];
        const int b = tid;
        if (b >= a && b < n) {
            double2 val = b == a ? make_double2(1.0, 0.0) : A[pk(b, a, n)];
            tt[((int64_t)(col >> 6) * t + (b >> 6)) * TILE_ELEMS_D + (col & 63) * 64 + (b & 63)] = from_d2<T2>(val);
        }
    }
}

// ------------------------------------- Bunch-Kaufman, register variant --
// Same pivoting rule and outputs as bk_kernel, for blocks of order <= NM.
// The whole block is held as a full symmetric square in registers: thread
// (pr, qc) owns rows pr + TR*a and columns qc + TC*b.  Each pivot step
// broadcasts the pivot column and the rows being interchanged through small
// LDS vectors, so a step costs two or three work-group barriers and no
// serial per-thread loops.  L^{-1} is accumulated alongside the elimination
// (Z <- (I - l_k e_k^T) Z, with the row interchanges applied to Z as they are
// to L) in owner-exclusive LDS storage, giving TT = L^{-1} P^T at the end.
// wave-uniform values kept in scalar registers
__device__ __forceinline__ double uni(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double2 uni2(double2 z) { return make_double2(uni(z.x), uni(z.y)); }

// Wave-wide maximum of a double with DPP row shifts and row broadcasts
// (no LDS traffic); every lane receives the result.
__device__ __forceinline__ double dpp_max_step(double v, int ctrl, int row_mask) {
    const long long b = __double_as_longlong(v);
    const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
    int lo2, hi2;
    switch (ctrl) {
    case 0x111: lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x111, 0xf, 0xf, false);
                hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x111, 0xf, 0xf, false); break;
    case 0x112: lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x112, 0xf, 0xf, false);
                hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x112, 0xf, 0xf, false); break;
    case 0x114: lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x114, 0xf, 0xf, false);
                hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x114, 0xf, 0xf, false); break;
    case 0x118: lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x118, 0xf, 0xf, false);
                hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x118, 0xf, 0xf, false); break;
    case 0x142: lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x142, 0xa, 0xf, false);
                hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x142, 0xa, 0xf, false); break;
    default:    lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x143, 0xc, 0xf, false);
                hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x143, 0xc, 0xf, false); break;
    }
    (void)row_mask;
    return fmax(v, __longlong_as_double(((long long)hi2 << 32) | (unsigned int)lo2));
}
__device__ __forceinline__ double wave_max(double v) {
    v = dpp_max_step(v, 0x111, 0xf);  // row_shr:1
    v = dpp_max_step(v, 0x112, 0xf);  // row_shr:2
    v = dpp_max_step(v, 0x114, 0xf);  // row_shr:4
    v = dpp_max_step(v, 0x118, 0xf);  // row_shr:8
    v = dpp_max_step(v, 0x142, 0xa);  // row_bcast:15
    v = dpp_max_step(v, 0x143, 0xc);  // row_bcast:31
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Arg-max of |col[i]| = |Re|+|Im| over lo <= i < hi, i != skip (64 rows, one
// per lane), computed by every wave on its own: wave maximum, then the lowest
// row holding it (ballot).  Returns value -1 when the range is empty.
__device__ __forceinline__ void wave_argmax_col(const double2 *col, int lo, int hi, int skip, double &mv, int &mi) {
    const int i = threadIdx.x & 63;
    const bool act = i >= lo && i < hi && i != skip;
    const double v = act ? cabs1(col[i]) : -1.0;
    const double m = wave_max(v);
    const unsigned long long b = __ballot(act && v == m);
    mv = m;
    mi = b ? (__ffsll((long long)b) - 1) : -1;
}

// c ? x : y on the components (a conditional on the vector class itself
// selects between addresses and forces its operands into private memory)
__device__ __forceinline__ double2 sel2(bool c, double2 x, double2 y) {
    return make_double2(c ? x.x : y.x, c ? x.y : y.y);
}
// v if keep, else +0 (bitwise, so that no select of the register array is
// turned into an indexed private-memory access)
__device__ __forceinline__ double2 keep_or_zero(double2 v, bool keep) {
    const long long m = -(long long)keep;
    return make_double2(__longlong_as_double(__double_as_longlong(v.x) & m),
                        __longlong_as_double(__double_as_longlong(v.y) & m));
}

// Bunch-Kaufman on a block of order <= 64 (same pivoting rule and outputs as
// bk_kernel) with implicit interchanges.  The block stays in its stored
// (physical) order: lane r of wave w (NW waves) holds, for the columns
// s = w + NW b, A(r, s) and Z(s, r), Z = L^{-1} in physical order (TT(b, c)
// = Z(perm b, c)).  An interchange only updates the permutation (held by
// every wave, one entry per lane) and the mask of rows not yet eliminated.
//
// Each step is one work-group barrier.  Before it, the wave owning the next
// natural pivot column p (logical position k) publishes through LDS the
// column of A, with p and the eliminated rows zeroed, row p of Z, and the
// start of the pivot test it computes itself: the largest remaining
// off-diagonal magnitude, its row, and 1/A(p, p).  So the search is done
// while the other waves still update, and after the barrier every wave reads
// all operands of the common step (a 1x1 pivot that needs no interchange) in
// one round of loads.  When the test needs column r, its owner publishes it
// and a second barrier follows.  The update touches only the remaining
// columns s:
//   A(r, s) -= l(r) x(s),   Z(s, r) -= w(r) x(s),
// with l = X(r, :) E^{-1} (zero on eliminated rows: masked column) and
// w = Z(piv, r) E^{-1} (zero on remaining rows).  The pivot column of a 1x1
// step keeps A(r, p), and L = A(r, p) / d is formed at the end; a 2x2 step
// stores its multipliers directly.  Equal magnitudes in the pivot search go
// to the lowest stored row.
struct BkHead {
    double2 dg, inv;  // pivot A(p, p) and its reciprocal
    double lam;       // largest remaining off-diagonal magnitude in column p
    int r;            // its row (lowest on ties), or p when there is none
    int pad;
};

// sum_p A_p B_p^T of one task for a wave's MS x QS sub-tiles of 16 x 16 at
// rows wr, columns wc (defined with the GEMM kernels)
template <typename T, int MS, int QS>
__device__ __forceinline__ void gemm_sub_acc(const GemmTask &tk, const GemmPair *pairs, const Bases &bases, int wr,
                                             int wc, typename Mfma<T>::acc (&re)[MS][QS],
                                             typename Mfma<T>::acc (&im)[MS][QS]);

template <typename T2, int NW>
__global__ __launch_bounds__(64 * NW) void bk64_kernel(const BkTask *tasks, const GemmPair *pairs, Bases bases,
                                                       DArrays D, int *status) {
    constexpr int NM = 64, RB = NM / NW, SLD = NM + 1;
    typedef double Regs __attribute__((ext_vector_type(2 * RB)));
    __shared__ double2 colA[2][NM], zcA[2][NM], colB[2][NM], zcB[2][NM];
    __shared__ BkHead head[2];
    __shared__ double2 dgB[2];
    __shared__ double2 sd[NM], sdoff[NM], sdinv[NM], sdinvoff[NM];  // D outputs, flushed at the end
    __shared__ int spiv[NM];
    __shared__ double2 stage[NM * SLD];  // TT staged for coalesced stores

    const BkTask tk = tasks[blockIdx.x];
    const int n = tk.n, t = threadIdx.x;
    const int lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
    const double2 zero = make_double2(0, 0);
    // A(lane, s) and Z(s, lane) for s = w + NW b, as (re, im) pairs; a vector so
    // that a column picked by a wave-uniform b is a register-indexed move
    Regs av, zv;
    {
        const T2 *src = enc_ptr<T2>(bases, tk.a);
#pragma unroll
        for (int bb = 0; bb < RB; ++bb) {
            const int i = lane, j = w + NW * bb;
            double2 v = zero;
            if (i < n && j < n) v = to_d2(src[tile_elem(i > j ? i : j, i > j ? j : i, tk.ldt)]);
            av[2 * bb] = v.x;
            av[2 * bb + 1] = v.y;
            zv[2 * bb] = i == j ? 1.0 : 0.0;
            zv[2 * bb + 1] = 0.0;
        }
    }
    if (tk.np > 0) {
        // pending updates of the block, A -= sum_p X_p W_p^T (the previous
        // step's updates of this column): the eight waves form U on MFMA
        // (the update GEMM's tile product), U goes through LDS, and every
        // thread takes U(i, s) for i >= s and U(s, i) above the diagonal, so
        // that both triangles carry the lower one's rounding (U is symmetric:
        // W = X D^{-1})
        using T = typename T2S<T2>::type;
        using M = Mfma<T>;
        {
            // wave w forms the 32 x 16 block at rows 32 (w / 4), columns 16 (w % 4)
            typename M::acc ure[2][1], uim[2][1];
            const GemmTask ut{0, tk.p0, tk.np};
            const int wr = (w >> 2) * 32, wc = (w & 3) * 16, li = lane & 15, lk = lane >> 4;
            gemm_sub_acc<T, 2, 1>(ut, pairs, bases, wr, wc, ure, uim);
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    stage[(wc + M::out_row(lk, r)) * SLD + wr + 16 * m + li] = make_double2(ure[m][0][r], uim[m][0][r]);
        }
        __syncthreads();
#pragma unroll
        for (int bb = 0; bb < RB; ++bb) {
            const int j = w + NW * bb;
            const double2 u = lane >= j ? stage[j * SLD + lane] : stage[lane * SLD + j];
            av[2 * bb] -= u.x;
            av[2 * bb + 1] -= u.y;
        }
        __syncthreads();  // stage is written again at the end
    }
    int vperm = lane, vinv = lane;  // perm[lane] and its inverse
    unsigned long long active = n >= 64 ? ~0ull : ((1ull << n) - 1ull);

    // publish column p (owner wave) into buffer bf with the start of its test
    auto publish = [&](int p, int bf, unsigned long long act) {
        const int b = p / NW;
        const double2 x = make_double2(av[2 * b], av[2 * b + 1]);
        const bool keep = ((act >> lane) & 1ull) && lane != p;
        colA[bf][lane] = keep_or_zero(x, keep);
        zcA[bf][lane] = make_double2(zv[2 * b], zv[2 * b + 1]);
        const double lv = keep ? cabs1(x) : -1.0;
        const double lam = fmax(wave_max(lv), 0.0);
        const unsigned long long cand = __ballot(keep && lv == lam);
        const int r = cand ? __ffsll((long long)cand) - 1 : p;
        if (lane == p) {
            head[bf].dg = x;
            head[bf].inv = crecip(x);
            head[bf].lam = lam;
            head[bf].r = r;
        }
    };
    if (n > 0 && w == 0) publish(0, 0, active);

    int k = 0, step = 0;
    bool singular = false;
    while (k < n) {
        const int buf = step & 1;
        const int pk = __builtin_amdgcn_readfirstlane(__builtin_amdgcn_readlane(vperm, k));
        __syncthreads();
        // ---- operands of the common step, in one round of loads
        const double2 dA = uni2(head[buf].dg);
        double2 e11 = uni2(head[buf].inv);
        const double lam1 = uni(head[buf].lam);
        const int r = __builtin_amdgcn_readfirstlane(head[buf].r);
        const double2 xl = colA[buf][lane], zl = zcA[buf][lane];
        double2 xs[RB];
#pragma unroll
        for (int bb = 0; bb < RB; ++bb) xs[bb] = colA[buf][w + NW * bb];
        const double akk = cabs1(dA);
        int size = 1, p0 = pk, p1 = pk;
        double2 dB = zero;
        if (!(fmax(akk, lam1) > 0.0)) {
            singular = true;
        } else if (!(akk >= kAlphaBK * lam1) && r != pk) {
            // ---- publish column r of A (remaining rows other than r) and row r of Z
            if (w == r % NW) {
                const int b = r / NW;
                const double2 v = make_double2(av[2 * b], av[2 * b + 1]);
                colB[buf][lane] = keep_or_zero(v, ((active >> lane) & 1ull) && lane != r);
                zcB[buf][lane] = make_double2(zv[2 * b], zv[2 * b + 1]);
                if (lane == r) dgB[buf] = v;
            }
            __syncthreads();
            const bool sact = ((active >> lane) & 1ull) && lane != r;
            const double sv = sact ? cabs1(colB[buf][lane]) : -1.0;
            const double sigma = fmax(wave_max(sv), 0.0);
            dB = uni2(dgB[buf]);
            const double arr = cabs1(dB);
            if (akk * sigma >= kAlphaBK * lam1 * lam1) { size = 1; p0 = pk; }
            else if (arr >= kAlphaBK * sigma) { size = 1; p0 = r; }
            else { size = 2; p0 = pk; p1 = r; }
        }
        if (singular) break;
        if (size == 1) p1 = p0;
        // ---- interchange: logical position q (k for a 1x1 pivot, k+1 for a
        // 2x2 one) receives row r
        if (p0 != pk || size == 2) {
            const int q = k + size - 1;
            const int posr = __builtin_amdgcn_readlane(vinv, r);
            const int atq = __builtin_amdgcn_readlane(vperm, q);
            if (lane == q) vperm = r;
            if (lane == posr) vperm = atq;
            if (lane == r) vinv = q;
            if (lane == atq) vinv = posr;
        }
        const unsigned long long rest = active & ~((1ull << p0) | (1ull << p1));
        const int pnext = k + size < n ? __builtin_amdgcn_readfirstlane(__builtin_amdgcn_readlane(vperm, k + size)) : -1;
        // ---- pivot block E = [[ea, eb], [eb, ec]] and its inverse; per row the
        // coefficients l_u, w_u of each pivot column u
        double2 ea, eb = zero, ec = zero, e12 = zero, e22 = zero, l0, l1 = zero, w0, w1 = zero;
        if (size == 1 && p0 == pk) {
            ea = dA;
            l0 = cmul(xl, e11);
            w0 = cmul(zl, e11);
        } else if (size == 1) {
            ea = dB;
            e11 = uni2(crecip(dB));
            l0 = cmul(colB[buf][lane], e11);
            w0 = cmul(zcB[buf][lane], e11);
#pragma unroll
            for (int bb = 0; bb < RB; ++bb) xs[bb] = colB[buf][w + NW * bb];
        } else {
            ea = dA;
            ec = dB;
            eb = uni2(colA[buf][p1]);
            const double2 idet = crecip(csub(cmul(ea, ec), cmul(eb, eb)));
            e11 = uni2(cmul(ec, idet));
            e22 = uni2(cmul(ea, idet));
            e12 = uni2(make_double2(-(eb.x * idet.x - eb.y * idet.y), -(eb.x * idet.y + eb.y * idet.x)));
            const bool rin = (rest >> lane) & 1ull;
            const double2 u1 = colB[buf][lane], z1 = zcB[buf][lane];
            l0 = keep_or_zero(cadd(cmul(xl, e11), cmul(u1, e12)), rin);
            l1 = keep_or_zero(cadd(cmul(xl, e12), cmul(u1, e22)), rin);
            w0 = cadd(cmul(zl, e11), cmul(z1, e12));
            w1 = cadd(cmul(zl, e12), cmul(z1, e22));
        }
        // ---- rank-1 update per pivot column, remaining columns only
#pragma unroll
        for (int bb = 0; bb < RB; ++bb) {
            if ((rest >> (w + NW * bb)) & 1ull) {
                const double2 v = cfma_neg(make_double2(av[2 * bb], av[2 * bb + 1]), l0, xs[bb]);
                const double2 y = cfma_neg(make_double2(zv[2 * bb], zv[2 * bb + 1]), w0, xs[bb]);
                av[2 * bb] = v.x; av[2 * bb + 1] = v.y;
                zv[2 * bb] = y.x; zv[2 * bb + 1] = y.y;
            }
        }
        if (size == 2) {
#pragma unroll
            for (int bb = 0; bb < RB; ++bb) {
                const int sc = w + NW * bb;
                const double2 x1 = colB[buf][sc];
                if ((rest >> sc) & 1ull) {
                    const double2 v = cfma_neg(make_double2(av[2 * bb], av[2 * bb + 1]), l1, x1);
                    const double2 y = cfma_neg(make_double2(zv[2 * bb], zv[2 * bb + 1]), w1, x1);
                    av[2 * bb] = v.x; av[2 * bb + 1] = v.y;
                    zv[2 * bb] = y.x; zv[2 * bb + 1] = y.y;
                }
            }
            // a 2x2 step stores its multipliers; L(k+1, k) = 0
            const bool rin = (rest >> lane) & 1ull;
            if (w == p0 % NW) {
                const int b = p0 / NW;
                const double2 v = sel2(rin, l0, sel2(lane == p1, zero, make_double2(av[2 * b], av[2 * b + 1])));
                av[2 * b] = v.x; av[2 * b + 1] = v.y;
            }
            if (w == p1 % NW) {
                const int b = p1 / NW;
                const double2 v = sel2(rin, l1, make_double2(av[2 * b], av[2 * b + 1]));
                av[2 * b] = v.x; av[2 * b + 1] = v.y;
            }
        }
        // ---- the next pivot column's owner publishes it and starts its test
        if (pnext >= 0 && w == pnext % NW) publish(pnext, buf ^ 1, rest);
        if (t == 0) {
            sd[k] = ea; sdoff[k] = eb; sdinv[k] = e11; sdinvoff[k] = e12; spiv[k] = size == 2 ? 1 : 0;
            if (size == 2) { sd[k + 1] = ec; sdoff[k + 1] = eb; sdinv[k + 1] = e22; sdinvoff[k + 1] = e12; spiv[k + 1] = -1; }
        }
        active = rest;
        k += size;
        ++step;
    }
    if (singular) {
        if (t == 0) status[tk.status] = k + 1;
        return;
    }
    __syncthreads();
    const int64_t dr = tk.drow;
    if (t < n) {
        D.d[dr + t] = sd[t]; D.doff[dr + t] = sdoff[t];
        D.dinv[dr + t] = sdinv[t]; D.dinvoff[dr + t] = sdinvoff[t];
        D.piv[dr + t] = spiv[t];
        D.perm[dr + t] = vperm;
    }
    // ---- outputs: unit lower L(a, b) = A(perm a, perm b) (times 1/d for a
    // 1x1 pivot column); TT(inv s, c) = Z(s, c), zero outside the n x n corner
    T2 *lout = enc_ptr<T2>(bases, tk.l);
    T2 *tt = enc_ptr<T2>(bases, tk.tt);
    const int la = vinv;
#pragma unroll
    for (int bb = 0; bb < RB; ++bb) {
        const int sc = w + NW * bb;
        const int lb = __builtin_amdgcn_readlane(vinv, sc);
        const bool in = lane < n && sc < n;
        if (in && la >= lb) {
            double2 v = make_double2(av[2 * bb], av[2 * bb + 1]);
            if (spiv[lb] == 0) v = cmul(v, sdinv[lb]);
            lout[tile_elem(la, lb, tk.ldt)] = from_d2<T2>(sel2(la == lb, make_double2(1.0, 0.0), v));
        }
        stage[lane * SLD + lb] = sel2(in, make_double2(zv[2 * bb], zv[2 * bb + 1]), zero);
    }
    __syncthreads();
    for (int e = t; e < NM * NM; e += 64 * NW) tt[e] = from_d2<T2>(stage[(e >> 6) * SLD + (e & 63)]);
}

// ------------------------------------------------- complex GEMM (MFMA) --
// C (=|-=) sum_p A_p B_p^T for 64x64 complex tiles on real MFMAs (three per
// complex product), 256 threads: wave w owns the 32x32 quadrant
// (rows 32*(w>>1), cols 32*(w&1)).  The MFMA's first operand is taken from B
// and its second from A so that the accumulator holds C^T, whose per-lane
// layout maps to contiguous runs of column-major C.

// One k-step (4 inner indices) of the complex products of a wave's MS x QS
// sub-tiles of 16 x 16, with three real products per complex one
// (P1 = Re w Re x, P2 = Im w Im x, P3 = (Re w + Im w)(Re x + Im x);
// Re = P1 - P2, Im = P3 - P1 - P2, combined by cmma_finish): a quarter fewer
// MFMAs than four products.  Its rounding (cancellation in Im when Im is small
// next to the operands) stays at the working precision's level; in FP32 it
// costs the refinement one more correction at 48^3 hexes, which the faster
// factorisation more than pays for.
template <typename T, int MS, int QS>
__device__ __forceinline__ void cmma_step(const typename C2T<T>::type (&wq)[QS], const typename C2T<T>::type (&xm)[MS],
                                          typename Mfma<T>::acc (&re)[MS][QS], typename Mfma<T>::acc (&im)[MS][QS],
                                          typename Mfma<T>::acc (&p3)[MS][QS]) {
    using M = Mfma<T>;
    T ws[QS], xsum[MS];
#pragma unroll
    for (int q = 0; q < QS; ++q) ws[q] = wq[q].x + wq[q].y;
#pragma unroll
    for (int m = 0; m < MS; ++m) xsum[m] = xm[m].x + xm[m].y;
#pragma unroll
    for (int m = 0; m < MS; ++m)
#pragma unroll
        for (int q = 0; q < QS; ++q) {
            re[m][q] = M::mma(wq[q].x, xm[m].x, re[m][q]);
            im[m][q] = M::mma(wq[q].y, xm[m].y, im[m][q]);
            p3[m][q] = M::mma(ws[q], xsum[m], p3[m][q]);
        }
}
template <typename T, int MS, int QS>
__device__ __forceinline__ void cmma_finish(typename Mfma<T>::acc (&re)[MS][QS], typename Mfma<T>::acc (&im)[MS][QS],
                                            const typename Mfma<T>::acc (&p3)[MS][QS]) {
#pragma unroll
    for (int m = 0; m < MS; ++m)
#pragma unroll
        for (int q = 0; q < QS; ++q) {
            const typename Mfma<T>::acc r = re[m][q] - im[m][q];
            im[m][q] = p3[m][q] - re[m][q] - im[m][q];
            re[m][q] = r;
        }
}

// Accumulates sum_p A_p B_p^T of one task for the output rows wr + 16 m + i
// (m < MS) and columns wc + 16 q + i (q < QS), i < 16, of the calling wave
// (C^T layout, see above).
template <typename T, int MS, int QS>
__device__ __forceinline__ void gemm_sub_acc(const GemmTask &tk, const GemmPair *pairs, const Bases &bases, int wr,
                                             int wc, typename Mfma<T>::acc (&re)[MS][QS],
                                             typename Mfma<T>::acc (&im)[MS][QS]) {
    using T2 = typename C2T<T>::type;
    using acc_t = typename Mfma<T>::acc;
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    acc_t p3[MS][QS];
#pragma unroll
    for (int m = 0; m < MS; ++m)
#pragma unroll
        for (int q = 0; q < QS; ++q) re[m][q] = im[m][q] = p3[m][q] = acc_t{0, 0, 0, 0};
    // operands of k-step s + 2 are loaded while k-step s runs
    constexpr int PF = 2;
    for (int p = 0; p < tk.np; ++p) {
        const GemmPair pr = pairs[tk.p0 + p];
        const T2 *A = enc_ptr<T2>(bases, pr.a);
        const T2 *B = enc_ptr<T2>(bases, pr.b);
        T2 w[PF][QS], x[PF][MS];
#pragma unroll
        for (int s = 0; s < PF; ++s) {
            const int kcol = (4 * s + lk) * 64;
#pragma unroll
            for (int q = 0; q < QS; ++q) w[s][q] = B[kcol + wc + 16 * q + li];
#pragma unroll
            for (int m = 0; m < MS; ++m) x[s][m] = A[kcol + wr + 16 * m + li];
        }
#pragma unroll
        for (int k0 = 0; k0 < 64; k0 += 4) {
            const int s = (k0 / 4) % PF;
            T2 wq[QS], xm[MS];
#pragma unroll
            for (int q = 0; q < QS; ++q) wq[q] = w[s][q];
#pragma unroll
            for (int m = 0; m < MS; ++m) xm[m] = x[s][m];
            if (k0 + 4 * PF < 64) {
                const int kcol = (k0 + 4 * PF + lk) * 64;
#pragma unroll
                for (int q = 0; q < QS; ++q) w[s][q] = B[kcol + wc + 16 * q + li];
#pragma unroll
                for (int m = 0; m < MS; ++m) x[s][m] = A[kcol + wr + 16 * m + li];
            }
            cmma_step<T, MS, QS>(wq, xm, re, im, p3);
        }
    }
    cmma_finish<T, MS, QS>(re, im, p3);
}

// The same for the wave's 32x32 quadrant of a 256-thread work-group: wave w
// owns rows 32 (w >> 1) and columns 32 (w & 1) onwards.
template <typename T>
__device__ __forceinline__ void gemm_task_acc(const GemmTask &tk, const GemmPair *pairs, const Bases &bases,
                                              typename Mfma<T>::acc (&re)[2][2], typename Mfma<T>::acc (&im)[2][2]) {
    const int wave = (threadIdx.x >> 6) & 3;
    gemm_sub_acc<T, 2, 2>(tk, pairs, bases, (wave >> 1) * 32, (wave & 1) * 32, re, im);
}

// One product A B^T with A staged in LDS (column-major, column stride lda,
// rows wr + 16 m + i of the calling wave), B from memory; same operand
// mapping and accumulator layout as gemm_sub_acc.
template <typename T, int MS, int QS>
__device__ __forceinline__ void gemm_lds_sub(const typename C2T<T>::type *alds, int lda,
                                             const typename C2T<T>::type *B, int wr, int wc,
                                             typename Mfma<T>::acc (&re)[MS][QS], typename Mfma<T>::acc (&im)[MS][QS]) {
    using T2 = typename C2T<T>::type;
    using acc_t = typename Mfma<T>::acc;
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    acc_t p3[MS][QS];
#pragma unroll
    for (int m = 0; m < MS; ++m)
#pragma unroll
        for (int q = 0; q < QS; ++q) re[m][q] = im[m][q] = p3[m][q] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < 64; k0 += 4) {
        const int k = k0 + lk;
        T2 wq[QS], xm[MS];
#pragma unroll
        for (int q = 0; q < QS; ++q) wq[q] = B[k * 64 + wc + 16 * q + li];
#pragma unroll
        for (int m = 0; m < MS; ++m) xm[m] = alds[k * lda + wr + 16 * m + li];
        cmma_step<T, MS, QS>(wq, xm, re, im, p3);
    }
    cmma_finish<T, MS, QS>(re, im, p3);
}

// Three work-groups per compute unit: room for the three FP64 accumulator sets
// of a quadrant without spills.
template <typename T, int MODE>
__global__ __launch_bounds__(256, 3) void gemm_nt_kernel(const GemmTask *tasks, int64_t ntask, const GemmPair *pairs,
                                                      Bases bases) {
    using T2 = typename C2T<T>::type;
    using M = Mfma<T>;
    using acc_t = typename M::acc;
    const int64_t task = xcd_task(ntask);
    if (task >= ntask) return;
    const GemmTask tk = tasks[task];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    T2 *C = enc_ptr<T2>(bases, tk.c);
    // the target tile of an update is loaded first, so its latency overlaps the products
    // (FP64 keeps its three accumulator sets in registers instead and reads the
    // target after the products)
    constexpr bool kPreC = MODE == 1 && !std::is_same<T, double>::value;
    T2 cpre[2][2][4];
    if (kPreC) {
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) cpre[m][q][r] = C[(wc + 16 * q + M::out_row(lk, r)) * 64 + wr + 16 * m + li];
    }
    acc_t re[2][2], im[2][2];
    gemm_task_acc<T>(tk, pairs, bases, re, im);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wr + 16 * m + li;
                const int col = wc + 16 * q + M::out_row(lk, r);
                T2 *c = C + col * 64 + row;
                if (MODE == 0) {
                    *c = T2{re[m][q][r], im[m][q][r]};
                } else {
                    const T2 old = kPreC ? cpre[m][q][r] : *c;
                    *c = T2{old.x - re[m][q][r], old.y - im[m][q][r]};
                }
            }
}

// Panel of one tile with its scaling fused: X = sum_p A_p B_p^T (stored) and
// L-hat = X D^{-1} over the tile's own columns (1x1 and 2x2 pivots of a
// block of one tile never reach a neighbouring tile).  Task i of the panel
// list and task i of the scale list describe the same tile.
// (its LDS tile allows two work-groups per compute unit; the bound lets the
// FP64 accumulators of the three-product form stay in registers)
template <typename T>
__global__ __launch_bounds__(256, 2) void panel_scale_kernel(const GemmTask *tasks, const ScaleTask *stasks,
                                                          int64_t ntask, const GemmPair *pairs, Bases bases,
                                                          DArrays D) {
    using T2 = typename C2T<T>::type;
    using M = Mfma<T>;
    using acc_t = typename M::acc;
    __shared__ T2 xs[64 * 65];
    const int64_t task = xcd_task(ntask);
    if (task >= ntask) return;
    const GemmTask tk = tasks[task];
    const ScaleTask sk = stasks[task];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    acc_t re[2][2], im[2][2];
    if (sk.nq == 0) {
        gemm_task_acc<T>(tk, pairs, bases, re, im);
    } else {
        // pending updates of the input tile first: A' = A - sum X W^T, staged
        // in LDS, then X = A' TT^T with A' read from there
        const GemmTask ut{0, sk.q0, sk.nq};
        gemm_task_acc<T>(ut, pairs, bases, re, im);
        const GemmPair pr = pairs[tk.p0];
        const T2 *A = enc_ptr<T2>(bases, pr.a);
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wr + 16 * m + li;
                    const int col = wc + 16 * q + M::out_row(lk, r);
                    const T2 a = A[col * 64 + row];
                    xs[col * 65 + row] = T2{a.x - re[m][q][r], a.y - im[m][q][r]};
                }
        __syncthreads();
        gemm_lds_sub<T, 2, 2>(xs, 65, enc_ptr<T2>(bases, pr.b), wr, wc, re, im);
        __syncthreads();  // xs is rewritten below
    }
    T2 *C = enc_ptr<T2>(bases, tk.c);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wr + 16 * m + li;
                const int col = wc + 16 * q + M::out_row(lk, r);
                const T2 v = T2{re[m][q][r], im[m][q][r]};
                C[col * 64 + row] = v;
                xs[col * 65 + row] = v;
            }
    __syncthreads();
    T2 *W = enc_ptr<T2>(bases, sk.w);
    for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
        const int r = e & 63, c = e >> 6;
        double2 out = make_double2(0, 0);
        if (c < sk.ncols) {
            const int64_t row = sk.drow + c;
            const int pv = D.piv[row];
            out = cmul(to_d2(xs[c * 65 + r]), D.dinv[row]);
            if (pv != 0) out = cadd(out, cmul(to_d2(xs[(c + pv) * 65 + r]), D.dinvoff[row]));
        }
        W[e] = from_d2<T2>(out);
    }
}

// The same panel in four row strips of 16, one work-group each: the four
// waves own 16 columns of the strip, so a tile's products are spread over
// four compute units (the panels of a short block column are on the
// critical path of the factorisation, one tile product per work-group
// taking ~5 us at the MFMA peak of one compute unit).  Strips of a tile are
// neighbours in the task order, so they run on one XCD and share W and TT
// through its L2.
template <typename T>
__global__ __launch_bounds__(256) void panel_scale16_kernel(const GemmTask *tasks, const ScaleTask *stasks,
                                                            int64_t ntask, const GemmPair *pairs, Bases bases,
                                                            DArrays D) {
    using T2 = typename C2T<T>::type;
    using M = Mfma<T>;
    using acc_t = typename M::acc;
    constexpr int LD = 17;
    __shared__ T2 xs[64 * LD];  // the strip, column-major: xs[col * LD + row - wr]
    const int64_t idx = xcd_task(4 * ntask);
    if (idx >= 4 * ntask) return;
    const int64_t task = idx >> 2;
    const GemmTask tk = tasks[task];
    const ScaleTask sk = stasks[task];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = 16 * (int)(idx & 3), wc = 16 * wave;
    const int li = lane & 15, lk = lane >> 4;
    acc_t re[1][1], im[1][1];
    if (sk.nq == 0) {
        gemm_sub_acc<T, 1, 1>(tk, pairs, bases, wr, wc, re, im);
    } else {
        const GemmTask ut{0, sk.q0, sk.nq};
        gemm_sub_acc<T, 1, 1>(ut, pairs, bases, wr, wc, re, im);
        const GemmPair pr = pairs[tk.p0];
        const T2 *A = enc_ptr<T2>(bases, pr.a);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int col = wc + M::out_row(lk, r);
            const T2 a = A[col * 64 + wr + li];
            xs[col * LD + li] = T2{a.x - re[0][0][r], a.y - im[0][0][r]};
        }
        __syncthreads();
        gemm_lds_sub<T, 1, 1>(xs, LD, enc_ptr<T2>(bases, pr.b), 0, wc, re, im);
        __syncthreads();  // xs is rewritten below
    }
    T2 *C = enc_ptr<T2>(bases, tk.c);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int col = wc + M::out_row(lk, r);
        const T2 v = T2{re[0][0][r], im[0][0][r]};
        C[col * 64 + wr + li] = v;
        xs[col * LD + li] = v;
    }
    __syncthreads();
    T2 *W = enc_ptr<T2>(bases, sk.w);
    for (int e = threadIdx.x; e < 16 * 64; e += blockDim.x) {
        const int rl = e & 15, c = e >> 4;
        double2 out = make_double2(0, 0);
        if (c < sk.ncols) {
            const int64_t row = sk.drow + c;
            const int pv = D.piv[row];
            out = cmul(to_d2(xs[c * LD + rl]), D.dinv[row]);
            if (pv != 0) out = cadd(out, cmul(to_d2(xs[(c + pv) * LD + rl]), D.dinvoff[row]));
        }
        W[c * 64 + wr + rl] = from_d2<T2>(out);
    }
}

// ------------------------------------------------- L-hat = X D^{-1} -----
template <typename T2>
__global__ void scale_kernel(const ScaleTask *tasks, Bases bases, DArrays D) {
    const ScaleTask tk = tasks[blockIdx.x];
    const T2 *X = enc_ptr<T2>(bases, tk.x);
    const T2 *Xp = tk.xprev >= 0 ? enc_ptr<T2>(bases, tk.xprev) : nullptr;
    const T2 *Xn = tk.xnext >= 0 ? enc_ptr<T2>(bases, tk.xnext) : nullptr;
    T2 *W = enc_ptr<T2>(bases, tk.w);
    for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
        const int r = e & 63, c = e >> 6;
        double2 out = make_double2(0, 0);
        if (c < tk.ncols) {
            const int64_t row = tk.drow + c;
            const int pv = D.piv[row];
            out = cmul(to_d2(X[e]), D.dinv[row]);
            if (pv == 1) {
                double2 xp = c + 1 < 64 ? to_d2(X[e + 64]) : (Xn ? to_d2(Xn[r]) : make_double2(0, 0));
                out = cadd(out, cmul(xp, D.dinvoff[row]));
            } else if (pv == -1) {
                double2 xp = c >= 1 ? to_d2(X[e - 64]) : (Xp ? to_d2(Xp[63 * 64 + r]) : make_double2(0, 0));
                out = cadd(out, cmul(xp, D.dinvoff[row]));
            }
        }
        W[e] = from_d2<T2>(out);
    }
}

// ---------------------------------------------- assembly of -K (step 2) --
template <typename T2>
__global__ void asm_kernel(const AsmTask *tasks, Bases bases) {
    const AsmTask tk = tasks[blockIdx.x];
    T2 *dst = enc_ptr<T2>(bases, tk.dst);
    const T2 *M = reinterpret_cast<const T2 *>(bases.p[ARR_M]);
    for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
        const int r = e & 63, c = e >> 6;
        double2 acc = make_double2(0, 0);
        if (r < tk.nrow && c < tk.ncol) {
            for (int q = 0; q < tk.ncontrib; ++q) {
                int R = tk.row0[q] + r, C = tk.col0[q] + c;
                if (R < C) { int t = R; R = C; C = t; }
                int64_t slot = tk.mbase[q] + (int64_t)(R >> 6) * ((R >> 6) + 1) / 2 + (C >> 6);
                acc = cadd(acc, to_d2(M[slot * TILE_ELEMS_D + (C & 63) * 64 + (R & 63)]));
            }
        }
        dst[e] = from_d2<T2>(acc);
    }
}

// Extend-add of the multifrontal form: one work-group per destination tile,
// dst (= or +=) the sum of its source tiles (whole 64 x 64 tiles; the sum is
// formed in FP64 and rounded once).  Each thread handles 16 consecutive
// complex entries of a tile; the source list of the task is read into a
// register of each lane first.
template <typename T2>
__global__ __launch_bounds__(256) void extend_add_kernel(const AddTask *tasks, const int64_t *srcs, Bases bases) {
    const AddTask tk = tasks[blockIdx.x];
    T2 *dst = enc_ptr<T2>(bases, tk.dst);
    double2 acc[16];
    const int e0 = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = tk.accumulate ? to_d2(dst[e0 + 256 * q]) : make_double2(0.0, 0.0);
    for (int x = 0; x < tk.ns; ++x) {
        const T2 *src = enc_ptr<T2>(bases, srcs[tk.s0 + x]);
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = cadd(acc[q], to_d2(src[e0 + 256 * q]));
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) dst[e0 + 256 * q] = from_d2<T2>(acc[q]);
}

// ------------------------------------------------------------ launchers --
namespace {
inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g < 65535 * 64 ? (g > 0 ? g : 1) : 65535 * 64);
}
}  // namespace

// ------------------------------------------------- growth monitor -------
// max |L-hat| over the valid entries of factor tiles (one work-group of 256
// per tile, 16 entries per thread), folded into *gmax as the bit pattern of a
// non-negative double (NaN compares above every number and is kept).
template <typename T2>
__global__ __launch_bounds__(256) void growth_kernel(const FactorTile *tiles, Bases bases, unsigned long long *gmax) {
    __shared__ double red[4];
    const FactorTile ft = tiles[blockIdx.x];
    const T2 *p = enc_ptr<T2>(bases, ft.tile);
    double m = 0.0;
    for (int e = threadIdx.x; e < TILE_ELEMS_D; e += 256) {
        const int r = e & 63, c = e >> 6;
        if (r < ft.rows && c < ft.cols) {
            const double2 z = to_d2(p[e]);
            const double a = sqrt(z.x * z.x + z.y * z.y);
            m = (a > m || a != a) ? a : m;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(m, off);
        m = (o > m || o != o) ? o : m;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) m = (red[w] > m || red[w] != red[w]) ? red[w] : m;
        atomicMax(gmax, (unsigned long long)__double_as_longlong(m));
    }
}

template <typename T>
hipError_t launch_growth(const FactorTile *tiles, int64_t ntile, const Bases &b, unsigned long long *gmax,
                         hipStream_t s) {
    using T2 = typename C2T<T>::type;
    for (int64_t t0 = 0; t0 < ntile; t0 += (1 << 30)) {
        const int64_t n = std::min<int64_t>(ntile - t0, 1 << 30);
        hipLaunchKernelGGL((growth_kernel<T2>), dim3((unsigned)n), dim3(256), 0, s, tiles + t0, b, gmax);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_zero(void *p, int64_t n, hipStream_t s) {
    using T2 = typename C2T<T>::type;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero_kernel<T2>, dim3(grid_for(n, 256)), dim3(256), 0, s, (T2 *)p, n);
    return hipGetLastError();
}

__global__ void zero_i32_kernel(int *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
// (a kernel, not a memset, so that it can sit in a captured graph)
hipError_t launch_zero_i32(int *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coo_scatter(void *M, const int64_t *off, const double2 *val, int64_t n, hipStream_t s) {
    using T2 = typename C2T<T>::type;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(coo_scatter_kernel<T2>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (T2 *)M, off, val, n);
    return hipGetLastError();
}

size_t bk_lds_bytes(int n, int nthr, bool lds) {
    size_t a = lds ? (size_t)n * (n + 1) / 2 : 0;
    return (a + 2 * (size_t)nthr) * sizeof(double2) + 16 * sizeof(double) + 16 * sizeof(int) + (size_t)nthr * sizeof(int);
}

#ifndef BK64_NW
#define BK64_NW 8  // 8 waves: 8 elements of A and of Z per thread
#endif
template <typename T>
hipError_t launch_bk(const BkTask *tasks, int64_t ntask, int maxn, const GemmPair *pairs, const Bases &b,
                     const DArrays &D, int *status,
                     double2 *scratch, hipStream_t s, int variant) {
    using T2 = typename C2T<T>::type;
    if (ntask <= 0) return hipSuccess;
    if (maxn <= 64 && variant == 0) {
        hipLaunchKernelGGL((bk64_kernel<T2, BK64_NW>), dim3((unsigned)ntask), dim3(64 * BK64_NW), 0, s,
                           tasks, pairs, b, D, status);
        return hipGetLastError();
    }
    int nthr = ((maxn + 63) / 64) * 64;
    if (nthr > 1024) return hipErrorInvalidValue;
    const bool fits = bk_lds_bytes(maxn, nthr, true) <= 160 * 1024 - 256;
    if (variant == 1 && !fits) return hipErrorInvalidValue;
    bool lds = variant == 2 ? false : fits;
    size_t shm = bk_lds_bytes(maxn, nthr, lds);
    if (lds) {
        hipFuncSetAttribute((const void *)bk_kernel<T2, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        hipLaunchKernelGGL((bk_kernel<T2, true>), dim3((unsigned)ntask), dim3(nthr), shm, s, tasks, b, D, status,
                           scratch, (int64_t)0);
    } else {
        if (!scratch) return hipErrorInvalidValue;
        hipFuncSetAttribute((const void *)bk_kernel<T2, false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        hipLaunchKernelGGL((bk_kernel<T2, false>), dim3((unsigned)ntask), dim3(nthr), shm, s, tasks, b, D, status,
                           scratch, (int64_t)maxn * (maxn + 1) / 2);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm(const GemmTask *tasks, int64_t ntask, const GemmPair *pairs, const Bases &b, int mode,
                       hipStream_t s) {
    if (ntask <= 0) return hipSuccess;
    const unsigned groups = (unsigned)(((ntask + kXcds - 1) / kXcds) * kXcds);
    if (mode == 0)
        hipLaunchKernelGGL((gemm_nt_kernel<T, 0>), dim3(groups), dim3(256), 0, s, tasks, ntask, pairs, b);
    else
        hipLaunchKernelGGL((gemm_nt_kernel<T, 1>), dim3(groups), dim3(256), 0, s, tasks, ntask, pairs, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_panel_scale(const GemmTask *tasks, const ScaleTask *stasks, int64_t ntask, const GemmPair *pairs,
                              const Bases &b, const DArrays &D, int rows, hipStream_t s) {
    if (ntask <= 0) return hipSuccess;
    if (rows == 16) {
        const unsigned groups = (unsigned)(((4 * ntask + kXcds - 1) / kXcds) * kXcds);
        hipLaunchKernelGGL((panel_scale16_kernel<T>), dim3(groups), dim3(256), 0, s, tasks, stasks, ntask, pairs, b,
                           D);
        return hipGetLastError();
    }
    if (rows != 64) return hipErrorInvalidValue;
    const unsigned groups = (unsigned)(((ntask + kXcds - 1) / kXcds) * kXcds);
    hipLaunchKernelGGL((panel_scale_kernel<T>), dim3(groups), dim3(256), 0, s, tasks, stasks, ntask, pairs, b, D);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale(const ScaleTask *tasks, int64_t ntask, const Bases &b, const DArrays &D, hipStream_t s) {
    using T2 = typename C2T<T>::type;
    if (ntask <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_kernel<T2>, dim3((unsigned)ntask), dim3(256), 0, s, tasks, b, D);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_extend_add(const AddTask *tasks, int64_t ntask, const int64_t *srcs, const Bases &b,
                             hipStream_t s) {
    using T2 = typename C2T<T>::type;
    if (ntask <= 0) return hipSuccess;
    if (ntask > 0x7fffffffll) return hipErrorInvalidValue;
    hipLaunchKernelGGL(extend_add_kernel<T2>, dim3((unsigned)ntask), dim3(256), 0, s, tasks, srcs, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_asm(const AsmTask *tasks, int64_t ntask, const Bases &b, hipStream_t s) {
    using T2 = typename C2T<T>::type;
    if (ntask <= 0) return hipSuccess;
    hipLaunchKernelGGL(asm_kernel<T2>, dim3((unsigned)ntask), dim3(256), 0, s, tasks, b);
    return hipGetLastError();
}

#define D3M_INST(T)                                                                                          \
    template hipError_t launch_fill_zero<T>(void *, int64_t, hipStream_t);                                     \
    template hipError_t launch_coo_scatter<T>(void *, const int64_t *, const double2 *, int64_t, hipStream_t); \
    template hipError_t launch_bk<T>(const BkTask *, int64_t, int, const GemmPair *, const Bases &,            \
                                     const DArrays &, int *,                                                  \
                                     double2 *, hipStream_t, int);                                            \
    template hipError_t launch_gemm<T>(const GemmTask *, int64_t, const GemmPair *, const Bases &, int,        \
                                       hipStream_t);                                                          \
    template hipError_t launch_panel_scale<T>(const GemmTask *, const ScaleTask *, int64_t, const GemmPair *,   \
                                              const Bases &, const DArrays &, int, hipStream_t);              \
    template hipError_t launch_scale<T>(const ScaleTask *, int64_t, const Bases &, const DArrays &,            \
                                        hipStream_t);                                                         \
    template hipError_t launch_extend_add<T>(const AddTask *, int64_t, const int64_t *, const Bases &,          \
                                             hipStream_t);                                                    \
    template hipError_t launch_asm<T>(const AsmTask *, int64_t, const Bases &, hipStream_t);                    \
    template hipError_t launch_growth<T>(const FactorTile *, int64_t, const Bases &, unsigned long long *,       \
                                         hipStream_t);
D3M_INST(double)
D3M_INST(float)
#undef D3M_INST

}  // namespace d3m
