// Factor-phase kernels: initialisation of the subdomain matrices, the
// Bunch-Kaufman factorisation of diagonal blocks (pivoting restricted to the
// block, reference [bunch1977] of the paper), the complex Schur-update GEMM on
// MFMA, the L-hat = X D^{-1} scaling and the assembly of -K.
#include <climits>

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

// Bunch-Kaufman on a block of order <= 64 (same pivoting rule and outputs as
// bk_kernel).  The block is a full symmetric square in registers: thread
// (pr, qc) of a TR x TC grid owns rows pr + TR a and columns qc + TC b.  So is
// Z = L^{-1}, accumulated alongside the elimination (Z <- (I - l_k e_k^T) Z,
// with the row interchanges applied to Z as to L).  Each pivot step
// publishes the pivot column (and column r, and the rows that move) through
// small LDS vectors; every wave reduces them itself with DPP, so a step costs
// two or three work-group barriers.
template <typename T2, int TR, int TC>
__global__ __launch_bounds__(TR * TC) void bk64_kernel(const BkTask *tasks, Bases bases, DArrays D, int *status) {
    constexpr int NM = 64, NT = TR * TC, RA = NM / TR, RB = NM / TC;
    __shared__ double2 colk[NM], colr[NM], rkk[NM], rp[NM], zk[NM], zkk[NM], zp[NM];
    __shared__ double2 sd[NM], sdoff[NM], sdinv[NM], sdinvoff[NM];  // D outputs, flushed at the end
    __shared__ int sperm[NM], spiv[NM];

    const BkTask tk = tasks[blockIdx.x];
    const int n = tk.n, t = threadIdx.x, pr = t % TR, qc = t / TR;
    double2 a[RA][RB], z[RA][RB];
    {
        const T2 *src = enc_ptr<T2>(bases, tk.a);
#pragma unroll
        for (int aa = 0; aa < RA; ++aa)
#pragma unroll
            for (int bb = 0; bb < RB; ++bb) {
                const int i = pr + TR * aa, j = qc + TC * bb;
                a[aa][bb] = make_double2(0, 0);
                if (i < n && j < n) a[aa][bb] = to_d2(src[tile_elem(i > j ? i : j, i > j ? j : i, tk.ldt)]);
                z[aa][bb] = make_double2(i == j ? 1.0 : 0.0, 0.0);
            }
    }
    if (t < NM) sperm[t] = t;
    __syncthreads();

    int k = 0;
    bool singular = false;
    while (k < n) {
        const int qk = k % TC, bk = k / TC;
        if (qc == qk) {
#pragma unroll
            for (int bb = 0; bb < RB; ++bb)
                if (bb == bk) {
#pragma unroll
                    for (int aa = 0; aa < RA; ++aa) colk[pr + TR * aa] = a[aa][bb];
                }
        }
        __syncthreads();
        double lam1;
        int r;
        wave_argmax_col(colk, k + 1, n, -1, lam1, r);
        if (lam1 < 0.0 || r < 0) { lam1 = 0.0; r = k; }
        const double akk = cabs1(colk[k]);
        int size = 1, p = k;
        if (!(fmax(akk, lam1) > 0.0)) {
            singular = true;
        } else if (!(akk >= kAlphaBK * lam1) && r > k) {
            const int qr = r % TC, br = r / TC;
            if (qc == qr) {
#pragma unroll
                for (int bb = 0; bb < RB; ++bb)
                    if (bb == br) {
#pragma unroll
                        for (int aa = 0; aa < RA; ++aa) colr[pr + TR * aa] = a[aa][bb];
                    }
            }
            __syncthreads();
            double sigma;
            int dummy;
            wave_argmax_col(colr, k, n, r, sigma, dummy);
            const double arr = cabs1(colr[r]);
            if (akk * sigma >= kAlphaBK * lam1 * lam1) { size = 1; p = k; }
            else if (arr >= kAlphaBK * sigma) { size = 1; p = r; }
            else { size = 2; p = r; }
        }
        if (singular) break;
        const int kk = k + size - 1;
        const bool swap = p != kk;
        // ---- publish the rows that move (rows kk, p of A and Z; row k of Z)
        if (swap && pr == kk % TR) {
            const int ak = kk / TR;
#pragma unroll
            for (int aa = 0; aa < RA; ++aa)
                if (aa == ak) {
#pragma unroll
                    for (int bb = 0; bb < RB; ++bb) { rkk[qc + TC * bb] = a[aa][bb]; zkk[qc + TC * bb] = z[aa][bb]; }
                }
        }
        if ((swap || size == 2) && pr == p % TR) {
            const int ap = p / TR;
#pragma unroll
            for (int aa = 0; aa < RA; ++aa)
                if (aa == ap) {
#pragma unroll
                    for (int bb = 0; bb < RB; ++bb) { rp[qc + TC * bb] = a[aa][bb]; zp[qc + TC * bb] = z[aa][bb]; }
                }
        }
        if ((size == 2 || !swap) && pr == k % TR) {
            const int ak = k / TR;
#pragma unroll
            for (int aa = 0; aa < RA; ++aa)
                if (aa == ak) {
#pragma unroll
                    for (int bb = 0; bb < RB; ++bb) zk[qc + TC * bb] = z[aa][bb];
                }
        }
        __syncthreads();
        auto pi = [&](int x) { return !swap ? x : (x == kk ? p : (x == p ? kk : x)); };
        // ---- symmetric interchange kk <-> p (rows of A, L and Z; columns of A)
        if (swap) {
#pragma unroll
            for (int aa = 0; aa < RA; ++aa) {
                const int i = pr + TR * aa;
                if (i == kk || i == p) {
                    const double2 *src = (i == kk) ? rp : rkk;
                    const double2 *zsrc = (i == kk) ? zp : zkk;
#pragma unroll
                    for (int bb = 0; bb < RB; ++bb) {
                        const int j = qc + TC * bb;
                        a[aa][bb] = src[pi(j)];
                        if (j < k) z[aa][bb] = zsrc[j];
                    }
                }
            }
#pragma unroll
            for (int bb = 0; bb < RB; ++bb) {
                const int j = qc + TC * bb;
                if (j == kk || j == p) {
                    const double2 *src = (j == kk) ? rp : rkk;
#pragma unroll
                    for (int aa = 0; aa < RA; ++aa) {
                        const int i = pr + TR * aa;
                        if (i != kk && i != p) a[aa][bb] = src[i];
                    }
                }
            }
            if (t == 0) { int sw = sperm[kk]; sperm[kk] = sperm[p]; sperm[p] = sw; }
        }
        // ---- pivot block and multipliers.  New column k: c0[pi(.)] with
        // c0 = row p for a 1x1 pivot with interchange, else column k; new
        // column k+1 (2x2): row p [pi(.)].
        const bool two = size == 2;
        const double2 *c0 = (!two && swap) ? rp : colk;
        const double2 ea = uni2(c0[pi(k)]);
        double2 e11, e12, e22, eb = make_double2(0, 0), ec = make_double2(0, 0);
        if (!two) {
            e11 = uni2(crecip(ea));
            e12 = e22 = make_double2(0, 0);
        } else {
            eb = uni2(colk[p]);
            ec = uni2(rp[p]);
            const double2 idet = crecip(csub(cmul(ea, ec), cmul(eb, eb)));
            e11 = uni2(cmul(ec, idet));
            e22 = uni2(cmul(ea, idet));
            e12 = uni2(make_double2(-(eb.x * idet.x - eb.y * idet.y), -(eb.x * idet.y + eb.y * idet.x)));
        }
        // column values of the owned columns and rows of Z'(k,.), Z'(k+1,.)
        const double2 *z0row = (!two && swap) ? zp : zk;
        double2 xc0[RB], xc1[RB], zr0[RB], zr1[RB];
#pragma unroll
        for (int bb = 0; bb < RB; ++bb) {
            const int j = qc + TC * bb;
            const bool trail = j > kk && j < n;
            xc0[bb] = trail ? c0[pi(j)] : make_double2(0, 0);
            xc1[bb] = (trail && two) ? rp[pi(j)] : make_double2(0, 0);
            zr0[bb] = (j == k) ? make_double2(1.0, 0.0) : (j < k ? z0row[j] : make_double2(0, 0));
            zr1[bb] = two ? ((j == k + 1) ? make_double2(1.0, 0.0) : (j < k ? zp[j] : make_double2(0, 0)))
                          : make_double2(0, 0);
        }
        // ---- rank-1 / rank-2 update.  For a column j only one of A (trailing,
        // j > kk) and Z (eliminated, j <= kk) changes; column groups bb are
        // uniform except the one holding the pivot columns.
#pragma unroll
        for (int aa = 0; aa < RA; ++aa) {
            const int i = pr + TR * aa;
            if (i > kk && i < n) {
                const double2 x0 = c0[pi(i)];
                if (!two) {
                    const double2 l0 = cmul(x0, e11);
#pragma unroll
                    for (int bb = 0; bb < RB; ++bb) {
                        const int j = qc + TC * bb;
                        if (TC * bb > k) {
                            a[aa][bb] = cfma_neg(a[aa][bb], l0, xc0[bb]);
                        } else if (TC * bb + TC - 1 < k) {
                            z[aa][bb] = cfma_neg(z[aa][bb], l0, zr0[bb]);
                        } else {
                            if (j > k) a[aa][bb] = cfma_neg(a[aa][bb], l0, xc0[bb]);
                            else z[aa][bb] = cfma_neg(z[aa][bb], l0, zr0[bb]);
                            if (j == k) a[aa][bb] = l0;
                        }
                    }
                } else {
                    const double2 x1 = rp[pi(i)];
                    const double2 l0 = cadd(cmul(x0, e11), cmul(x1, e12));
                    const double2 l1 = cadd(cmul(x0, e12), cmul(x1, e22));
#pragma unroll
                    for (int bb = 0; bb < RB; ++bb) {
                        const int j = qc + TC * bb;
                        if (TC * bb > kk) {
                            a[aa][bb] = cfma_neg(cfma_neg(a[aa][bb], l0, xc0[bb]), l1, xc1[bb]);
                        } else if (TC * bb + TC - 1 < k) {
                            z[aa][bb] = cfma_neg(cfma_neg(z[aa][bb], l0, zr0[bb]), l1, zr1[bb]);
                        } else {
                            if (j > kk) a[aa][bb] = cfma_neg(cfma_neg(a[aa][bb], l0, xc0[bb]), l1, xc1[bb]);
                            else z[aa][bb] = cfma_neg(cfma_neg(z[aa][bb], l0, zr0[bb]), l1, zr1[bb]);
                            if (j == k) a[aa][bb] = l0;
                            if (j == k + 1) a[aa][bb] = l1;
                        }
                    }
                }
            }
            if (two && i == k + 1) {
#pragma unroll
                for (int bb = 0; bb < RB; ++bb)
                    if (qc + TC * bb == k) a[aa][bb] = make_double2(0, 0);
            }
        }
        if (t == 0) {
            sd[k] = ea; sdoff[k] = eb; sdinv[k] = e11; sdinvoff[k] = e12; spiv[k] = two ? 1 : 0;
            if (two) { sd[k + 1] = ec; sdoff[k + 1] = eb; sdinv[k + 1] = e22; sdinvoff[k + 1] = e12; spiv[k + 1] = -1; }
        }
        __syncthreads();
        k += size;
    }
    if (singular) {
        if (t == 0) status[tk.status] = k + 1;
        return;
    }
    const int64_t dr = tk.drow;
    if (t < n) {
        D.d[dr + t] = sd[t]; D.doff[dr + t] = sdoff[t];
        D.dinv[dr + t] = sdinv[t]; D.dinvoff[dr + t] = sdinvoff[t];
        D.piv[dr + t] = spiv[t];
        D.perm[dr + t] = sperm[t];
    }
    // ---- outputs: unit lower L and TT = Z P^T (zero elsewhere in the tile)
    T2 *lout = enc_ptr<T2>(bases, tk.l);
    T2 *tt = enc_ptr<T2>(bases, tk.tt);
#pragma unroll
    for (int aa = 0; aa < RA; ++aa)
#pragma unroll
        for (int bb = 0; bb < RB; ++bb) {
            const int i = pr + TR * aa, j = qc + TC * bb;
            if (i < n && j < n && i >= j)
                lout[tile_elem(i, j, tk.ldt)] = from_d2<T2>(i == j ? make_double2(1.0, 0.0) : a[aa][bb]);
            // TT[i][perm[j]] = Z[i][j]; columns perm[j] for j >= n are padding
            const int col = j < n ? sperm[j] : j;
            const double2 zv = (i < n && j < n && i >= j) ? z[aa][bb] : make_double2(0, 0);
            tt[col * 64 + i] = from_d2<T2>(zv);
        }
}

// ------------------------------------------------- complex GEMM (MFMA) --
// C (=|-=) sum_p A_p B_p^T for 64x64 complex tiles, 4M (four real MFMAs per
// complex product), 256 threads: wave w owns the 32x32 quadrant
// (rows 32*(w>>1), cols 32*(w&1)).  The MFMA's first operand is taken from B
// and its second from A so that the accumulator holds C^T, whose per-lane
// layout maps to contiguous runs of column-major C.
typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Accumulator layout of the 16x16x4 products (lane l, register r holds
// D[row][l % 16]): f64 row = l/16 + 4r, f32 row = 4(l/16) + r.
template <> struct Mfma<double> {
    using acc = d4_t;
    __device__ __forceinline__ static int out_row(int lk, int r) { return lk + 4 * r; }
    __device__ __forceinline__ static acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<float> {
    using acc = f4_t;
    __device__ __forceinline__ static int out_row(int lk, int r) { return 4 * lk + r; }
    __device__ __forceinline__ static acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <typename T, int MODE>
__global__ __launch_bounds__(256) void gemm_nt_kernel(const GemmTask *tasks, const GemmPair *pairs, Bases bases) {
    using T2 = typename C2T<T>::type;
    using M = Mfma<T>;
    using acc_t = typename M::acc;
    const GemmTask tk = tasks[blockIdx.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    acc_t re[2][2], im[2][2];
    for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 2; ++q) { re[m][q] = acc_t{0, 0, 0, 0}; im[m][q] = acc_t{0, 0, 0, 0}; }
    for (int p = 0; p < tk.np; ++p) {
        const GemmPair pr = pairs[tk.p0 + p];
        const T2 *A = enc_ptr<T2>(bases, pr.a);
        const T2 *B = enc_ptr<T2>(bases, pr.b);
#pragma unroll 4
        for (int k0 = 0; k0 < 64; k0 += 4) {
            const int kcol = (k0 + lk) * 64;
            T2 w[2], x[2];
            w[0] = B[kcol + wc + li];
            w[1] = B[kcol + wc + 16 + li];
            x[0] = A[kcol + wr + li];
            x[1] = A[kcol + wr + 16 + li];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    re[m][q] = M::mma(w[q].x, x[m].x, re[m][q]);
                    re[m][q] = M::mma(-w[q].y, x[m].y, re[m][q]);
                    im[m][q] = M::mma(w[q].x, x[m].y, im[m][q]);
                    im[m][q] = M::mma(w[q].y, x[m].x, im[m][q]);
                }
        }
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
                T2 *c = C + col * 64 + row;
                if (MODE == 0) {
                    *c = T2{re[m][q][r], im[m][q][r]};
                } else {
                    T2 o = *c;
                    *c = T2{o.x - re[m][q][r], o.y - im[m][q][r]};
                }
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

// ------------------------------------------------------------ launchers --
namespace {
inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g < 65535 * 64 ? (g > 0 ? g : 1) : 65535 * 64);
}
}  // namespace

template <typename T>
hipError_t launch_fill_zero(void *p, int64_t n, hipStream_t s) {
    using T2 = typename C2T<T>::type;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero_kernel<T2>, dim3(grid_for(n, 256)), dim3(256), 0, s, (T2 *)p, n);
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

#ifndef BK64_TR
#define BK64_TR 32  // 32 x 16 threads: 8 elements of A and of Z per thread
#define BK64_TC 16
#endif
template <typename T>
hipError_t launch_bk(const BkTask *tasks, int64_t ntask, int maxn, const Bases &b, const DArrays &D, int *status,
                     double2 *scratch, hipStream_t s) {
    using T2 = typename C2T<T>::type;
    if (ntask <= 0) return hipSuccess;
    if (maxn <= 64) {
        hipLaunchKernelGGL((bk64_kernel<T2, BK64_TR, BK64_TC>), dim3((unsigned)ntask), dim3(BK64_TR * BK64_TC), 0, s,
                           tasks, b, D, status);
        return hipGetLastError();
    }
    int nthr = ((maxn + 63) / 64) * 64;
    if (nthr > 1024) return hipErrorInvalidValue;
    bool lds = bk_lds_bytes(maxn, nthr, true) <= 160 * 1024 - 256;
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
    if (mode == 0)
        hipLaunchKernelGGL((gemm_nt_kernel<T, 0>), dim3((unsigned)ntask), dim3(256), 0, s, tasks, pairs, b);
    else
        hipLaunchKernelGGL((gemm_nt_kernel<T, 1>), dim3((unsigned)ntask), dim3(256), 0, s, tasks, pairs, b);
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
hipError_t launch_asm(const AsmTask *tasks, int64_t ntask, const Bases &b, hipStream_t s) {
    using T2 = typename C2T<T>::type;
    if (ntask <= 0) return hipSuccess;
    hipLaunchKernelGGL(asm_kernel<T2>, dim3((unsigned)ntask), dim3(256), 0, s, tasks, b);
    return hipGetLastError();
}

#define D3M_INST(T)                                                                                          \
    template hipError_t launch_fill_zero<T>(void *, int64_t, hipStream_t);                                     \
    template hipError_t launch_coo_scatter<T>(void *, const int64_t *, const double2 *, int64_t, hipStream_t); \
    template hipError_t launch_bk<T>(const BkTask *, int64_t, int, const Bases &, const DArrays &, int *,      \
                                     double2 *, hipStream_t);                                                 \
    template hipError_t launch_gemm<T>(const GemmTask *, int64_t, const GemmPair *, const Bases &, int,        \
                                       hipStream_t);                                                          \
    template hipError_t launch_scale<T>(const ScaleTask *, int64_t, const Bases &, const DArrays &,            \
                                        hipStream_t);                                                         \
    template hipError_t launch_asm<T>(const AsmTask *, int64_t, const Bases &, hipStream_t);
D3M_INST(double)
D3M_INST(float)
#undef D3M_INST

}  // namespace d3m
