// Solve-phase kernels (recipe steps 6-7 of Section II) and the FP64
// refinement / adjoint helpers.  Vector tiles hold 64 rows x nrhs columns,
// column-major (one right-hand side after another), so one 64 x 64 factor
// tile is applied to many right-hand sides per read.
#include <algorithm>
#include <climits>
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace d3m {

template <typename T2>
__device__ __forceinline__ T2 *vptr(const VBases &vb, int64_t e, int nrhs) {
    return reinterpret_cast<T2 *>(vb.p[e >> ENC_SHIFT]) + (e & ENC_MASK) * 64 * (int64_t)nrhs;
}
// element of vector row R (tile R/64, row R%64), column c
__device__ __forceinline__ int64_t vrow_elem(int64_t R, int c, int nrhs) {
    return (R >> 6) * 64 * (int64_t)nrhs + (int64_t)c * 64 + (R & 63);
}

// X[row] = f[c][e] for rows whose edge is owned by this subdomain, else 0
template <typename T2>
__global__ void vsplit_kernel(T2 *X, const double2 *f, const int64_t *map, int64_t nrows, int nrhs, int64_t ne) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nrows * nrhs) return;
    int64_t tile = idx / (64 * nrhs);
    int rem = (int)(idx - tile * 64 * nrhs);
    int c = rem >> 6, r = rem & 63;
    int64_t e = map[tile * 64 + r];
    X[idx] = e >= 0 ? from_d2<T2>(f[(int64_t)c * ne + e]) : T2{0, 0};
}

// Tile products of the solve sweeps on MFMA: out (64 rows x nc <= 16 NCB
// right-hand sides) gets op(L) X for 64 x 64 factor tiles L, op = identity or
// transpose, so that one read of a factor tile serves every right-hand side
// of the work-group.  The product is formed transposed, out^T = X^T op(L)^T,
// with 16x16x4 MFMAs (first operand X^T, second op(L)^T; accumulator rows are
// right-hand sides, columns are output rows).  Wave w owns the output rows
// m = 16 w + (l % 16) for every column, so no partial sums cross waves.  Lane
// l holds op(L)(m, q) for the 16 inner indices q = 16 kg + 4 (l / 16) + s
// (kg, s = 0..3), read straight from memory: for op = identity 16 lanes read
// one 256-byte run of a column of L, for the transpose each lane reads four
// consecutive entries of column m.  The X block (inner index x right-hand
// side) is staged through LDS, column stride SV_PQ (odd, so the 16 columns
// one read touches fall in distinct banks), double-buffered across the
// products of one task.
constexpr int SV_PQ = 65;

template <typename T2, int NCB> struct SvSmem {
    T2 xs[2][16 * NCB * SV_PQ];  // X(q, c) at c * SV_PQ + q
};

// lf[4 kg + s] = op(L)(16 w + l % 16, 16 kg + 4 (l / 16) + s)
template <typename T2, bool TR>
__device__ __forceinline__ void sv_load_l(T2 (&lf)[16], const T2 *tile) {
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int m = 16 * (threadIdx.x >> 6) + li;
#pragma unroll
    for (int kg = 0; kg < 4; ++kg)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int q = 16 * kg + 4 * lk + s;
            lf[4 * kg + s] = TR ? tile[m * 64 + q] : tile[q * 64 + m];
        }
}

// this thread's share of the X block: columns c0 .. c0 + ncol - 1 of a vector
// tile, minus the same columns of sub (if given); zero beyond ncol
template <typename T2, int NCB>
__device__ __forceinline__ void sv_fetch_x(T2 (&xr)[4 * NCB], const T2 *src, const T2 *sub, int c0, int ncol) {
#pragma unroll
    for (int i = 0; i < 4 * NCB; ++i) {
        const int e = threadIdx.x + 256 * i;
        T2 v{0, 0};
        if ((e >> 6) < ncol) {
            v = src[(int64_t)c0 * 64 + e];
            if (sub) {
                const T2 u = sub[(int64_t)c0 * 64 + e];
                v = T2{v.x - u.x, v.y - u.y};
            }
        }
        xr[i] = v;
    }
}
template <typename T2, int NCB> __device__ __forceinline__ void sv_put_x(T2 *xs, const T2 (&xr)[4 * NCB]) {
#pragma unroll
    for (int i = 0; i < 4 * NCB; ++i) {
        const int e = threadIdx.x + 256 * i;
        xs[(e >> 6) * SV_PQ + (e & 63)] = xr[i];
    }
}

// Accumulators of a solve product (out^T layout of the MFMA).  FP64 factors
// accumulate in FP64 MFMA registers, with three real products per complex one
// (P1 = Re x Re l, P2 = Im x Im l, P3 = (Re x + Im x)(Re l + Im l);
// Re = P1 - P2, Im = P3 - P1 - P2: a quarter fewer MFMAs than four products).  FP32 factors use FP32 MFMAs over 16
// inner indices at a time and add each partial sum into FP64 registers, so
// the rounding of a long sum does not add to the refinement's work (the
// vectors are still stored in FP32).
template <typename T, int NCB> struct SvAcc;
template <int NCB> struct SvAcc<double, NCB> {
    d4_t re[NCB], im[NCB], p3[NCB];  // P1, P2, P3
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) re[cb] = im[cb] = p3[cb] = d4_t{0, 0, 0, 0};
    }
    __device__ __forceinline__ void flush() {}
    __device__ __forceinline__ void mma(double2 ax, double2 bl, double bsum, int cb) {
        re[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax.x, bl.x, re[cb], 0, 0, 0);
        im[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax.y, bl.y, im[cb], 0, 0, 0);
        p3[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax.x + ax.y, bsum, p3[cb], 0, 0, 0);
    }
    __device__ __forceinline__ double2 get(int cb, int r) const {
        return make_double2(re[cb][r] - im[cb][r], p3[cb][r] - re[cb][r] - im[cb][r]);
    }
};
template <int NCB> struct SvAcc<float, NCB> {
    f4_t re[NCB], im[NCB];
    d4_t dre[NCB], dim[NCB];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            re[cb] = im[cb] = f4_t{0, 0, 0, 0};
            dre[cb] = dim[cb] = d4_t{0, 0, 0, 0};
        }
    }
    __device__ __forceinline__ void flush() {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                dre[cb][r] += (double)re[cb][r];
                dim[cb][r] += (double)im[cb][r];
            }
            re[cb] = im[cb] = f4_t{0, 0, 0, 0};
        }
    }
    __device__ __forceinline__ void mma(float2 ax, float2 bl, float, int cb) {
        using M = Mfma<float>;
        re[cb] = M::mma(ax.x, bl.x, re[cb]);
        im[cb] = M::mma(ax.x, bl.y, im[cb]);
        re[cb] = M::mma(-ax.y, bl.y, re[cb]);
        im[cb] = M::mma(ax.y, bl.x, im[cb]);
    }
    __device__ __forceinline__ double2 get(int cb, int r) const { return make_double2(dre[cb][r], dim[cb][r]); }
};

// acc += (op(L) X)^T for the fragment lf and the staged block xs
template <typename T, int NCB>
__device__ __forceinline__ void sv_mma(SvAcc<T, NCB> &acc, const typename C2T<T>::type (&lf)[16],
                                       const typename C2T<T>::type *xs) {
    using T2 = typename C2T<T>::type;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int kg = 0; kg < 4; ++kg) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int q = 16 * kg + 4 * lk + s;
            const T2 bl = lf[4 * kg + s];
            const T bsum = bl.x + bl.y;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc.mma(xs[(16 * cb + li) * SV_PQ + q], bl, bsum, cb);
        }
        acc.flush();
    }
}

// Diagonal solve of a one-tile block from the input staged in xin.
// Forward: y = TT x (TT = L^{-1} P^T of the block), v = D^{-1} y (2x2 pivots
// never cross the tile).  Backward: x = TT^T (v - acc) (= P L^{-T} (v - acc)).
// xsp is a free LDS buffer.
// lf: this thread's fragment of TT (forward) or TT^T (backward), loaded by
// the caller.
template <typename T, bool BWD, int NCB>
__device__ __forceinline__ void sv_diag(const typename C2T<T>::type (&lf)[16], const VDiagTask &tk, int c0,
                                        int ncol, const VBases &vb, const DArrays &D, int nrhs,
                                        const typename C2T<T>::type *xin, typename C2T<T>::type *xsp) {
    using M = Mfma<T>;
    using T2 = typename C2T<T>::type;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int m = 16 * (threadIdx.x >> 6) + li;
    // pivot data of this row (forward), loaded ahead of the product
    const int64_t dr = tk.drow + m;
    const bool live = !BWD && m < tk.n;
    const double2 di = live ? D.dinv[dr] : make_double2(0, 0);
    const int pv = live ? D.piv[dr] : 0;
    const double2 dio = pv ? D.dinvoff[dr] : make_double2(0, 0);
    SvAcc<T, NCB> acc;
    acc.zero();
    sv_mma<T, NCB>(acc, lf, xin);
    T2 *out = vptr<T2>(vb, BWD ? tk.x : tk.y, nrhs) + (int64_t)c0 * 64;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = 16 * cb + M::out_row(lk, r);
            const T2 val = from_d2<T2>(acc.get(cb, r));
            if (c < ncol) out[c * 64 + m] = val;
            if (!BWD) xsp[c * SV_PQ + m] = val;
        }
    if (BWD) return;
    __syncthreads();
    T2 *v = vptr<T2>(vb, tk.v, nrhs) + (int64_t)c0 * 64;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = 16 * cb + M::out_row(lk, r);
            if (c < ncol) {
                double2 val = cmul(di, to_d2(xsp[c * SV_PQ + m]));
                if (pv != 0) val = cadd(val, cmul(dio, to_d2(xsp[c * SV_PQ + m + pv])));
                v[c * 64 + m] = from_d2<T2>(live ? val : make_double2(0, 0));
            }
        }
}

// One one-tile diagonal solve for the right-hand sides c0 .. c0 + ncol - 1,
// by the whole work-group.
template <typename T, bool BWD, int NCB>
__device__ __forceinline__ void vdiag_task(const VDiagTask &tk, const Bases &b, const VBases &vb, const DArrays &D,
                                           int nrhs, int c0, int ncol, SvSmem<typename C2T<T>::type, NCB> &sm) {
    using T2 = typename C2T<T>::type;
    T2 xr[4 * NCB], lf[16];
    if (BWD)
        sv_fetch_x<T2, NCB>(xr, vptr<T2>(vb, tk.v, nrhs), tk.acc >= 0 ? vptr<T2>(vb, tk.acc, nrhs) : nullptr, c0, ncol);
    else
        sv_fetch_x<T2, NCB>(xr, vptr<T2>(vb, tk.x, nrhs), nullptr, c0, ncol);
    sv_load_l<T2, BWD>(lf, enc_ptr<T2>(b, tk.tt));
    sv_put_x<T2, NCB>(sm.xs[0], xr);
    __syncthreads();
    sv_diag<T, BWD, NCB>(lf, tk, c0, ncol, vb, D, nrhs, sm.xs[0], sm.xs[1]);
}

template <typename T, bool BWD, int NCB>
__global__ __launch_bounds__(256) void vdiag_kernel(const VDiagTask *tasks, int64_t ntask, Bases b, VBases vb,
                                                    DArrays D, int nrhs) {
    using T2 = typename C2T<T>::type;
    __shared__ SvSmem<T2, NCB> sm;
    const int nyb = (nrhs + 16 * NCB - 1) / (16 * NCB);
    const int64_t item = xcd_task(ntask * nyb);
    if (item >= ntask * nyb) return;
    const int64_t task = item / nyb;
    const int c0 = (int)(item - task * nyb) * 16 * NCB;
    vdiag_task<T, BWD, NCB>(tasks[task], b, vb, D, nrhs, c0, min(16 * NCB, nrhs - c0), sm);
}

// Diagonal blocks of several tiles (blocks larger than 64 factored whole):
// one work-group per block, 32 right-hand sides per blockIdx.y, each thread
// one output at a time.
template <typename T2, bool BWD>
__global__ __launch_bounds__(256) void vdiag_multi_kernel(const VDiagTask *tasks, Bases b, VBases vb, DArrays D,
                                                          int nrhs) {
    __shared__ double2 Ls[64 * 65];
    const VDiagTask tk = tasks[blockIdx.x];
    const int t = tk.t;
    const T2 *TT = enc_ptr<T2>(b, tk.tt);
    const int64_t vt = 64 * (int64_t)nrhs;
    const int c0 = blockIdx.y * 32;
    const int ncol = min(32, nrhs - c0);
    const T2 *xin = BWD ? nullptr : vptr<T2>(vb, tk.x, nrhs);
    T2 *y = BWD ? vptr<T2>(vb, tk.x, nrhs) : vptr<T2>(vb, tk.y, nrhs);  // output
    const T2 *vv = vptr<T2>(vb, tk.v, nrhs);
    const T2 *accv = (BWD && tk.acc >= 0) ? vptr<T2>(vb, tk.acc, nrhs) : nullptr;
    for (int ot = 0; ot < t; ++ot) {
        double2 s[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) s[i] = make_double2(0, 0);
        for (int it = 0; it < t; ++it) {
            // forward: y[ot] += TT[ot, it] x[it];  backward: x[ot] += TT[it, ot]^T w[it]
            const T2 *tile = BWD ? TT + ((int64_t)ot * t + it) * TILE_ELEMS_D : TT + ((int64_t)it * t + ot) * TILE_ELEMS_D;
            T2 v[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = tile[threadIdx.x + 256 * i];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int e = threadIdx.x + 256 * i;
                Ls[(e >> 6) * 65 + (e & 63)] = to_d2(v[i]);
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int e = threadIdx.x + 256 * i;
                const int r = e & 63, c = e >> 6;
                if (c < ncol) {
                    double2 a = s[i];
                    if (!BWD) {
                        const T2 *xs = xin + it * vt + (int64_t)(c0 + c) * 64;
                        for (int q = 0; q < 64; ++q) a = cadd(a, cmul(Ls[q * 65 + r], to_d2(xs[q])));
                    } else {
                        const T2 *vs = vv + it * vt + (int64_t)(c0 + c) * 64;
                        const T2 *as = accv ? accv + it * vt + (int64_t)(c0 + c) * 64 : nullptr;
                        for (int q = 0; q < 64; ++q) {
                            double2 wv = to_d2(vs[q]);
                            if (as) wv = csub(wv, to_d2(as[q]));
                            a = cadd(a, cmul(Ls[r * 65 + q], wv));
                        }
                    }
                    s[i] = a;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = threadIdx.x + 256 * i;
            if ((e >> 6) < ncol) y[ot * vt + (int64_t)c0 * 64 + e] = from_d2<T2>(s[i]);
        }
    }
    if (!BWD) {
        __syncthreads();
        T2 *v = vptr<T2>(vb, tk.v, nrhs);
        for (int64_t e = threadIdx.x; e < (int64_t)t * 64 * ncol; e += blockDim.x) {
            const int ot = (int)(e / (64 * ncol));
            const int rem = (int)(e - (int64_t)ot * 64 * ncol);
            const int rr = rem & 63, c = c0 + (rem >> 6);
            const int row = ot * 64 + rr;
            const int64_t dr = tk.drow + row;
            double2 val = make_double2(0, 0);
            if (row < tk.n) {
                val = cmul(D.dinv[dr], to_d2(y[ot * vt + (int64_t)c * 64 + rr]));
                const int pv = D.piv[dr];
                if (pv != 0) {
                    const int pr = row + pv;
                    val = cadd(val, cmul(D.dinvoff[dr], to_d2(y[(pr >> 6) * vt + (int64_t)c * 64 + (pr & 63)])));
                }
            }
            v[ot * vt + (int64_t)c * 64 + rr] = from_d2<T2>(val);
        }
    }
}

// out (-=|=|+=) sum_p op(L_p) src_p with op = identity (mode 0) or
// transpose (modes 1, 2); each work-group takes 16 NCB right-hand sides of a
// task.  The column blocks of one task are consecutive items of one XCD's
// range (xcd_task), so the factor tile they share is read from HBM once and
// from that XCD's L2 after.  The
// factor tile and X block of product p + 1 are fetched while product p runs.
// When fuse[task] >= 0 this update is the last one its target receives before
// the diagonal solve fuse[task] (forward: the target is that block's x;
// backward: its accumulator), so the work-group goes on with that solve from
// the new values kept in LDS, saving a launch per sweep step.
// lane `l`'s value of a 64-bit register, wave-uniform
__device__ __forceinline__ int64_t rdlane64(int64_t v, int l) {
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
    return ((int64_t)hi << 32) | (uint32_t)lo;
}

// One update task (and its fused diagonal solve) for the right-hand sides
// c0 .. c0 + ncol - 1, by the whole work-group.
template <typename T, int MODE, int NCB>
__device__ __forceinline__ void vupd_task(const VUpdTask &tk, int64_t fz, const VUpdPair *pairs,
                                          const VDiagTask *vdiag, const Bases &b, const VBases &vb, const DArrays &D,
                                          int nrhs, int c0, int ncol, SvSmem<typename C2T<T>::type, NCB> &sm) {
    using M = Mfma<T>;
    using T2 = typename C2T<T>::type;
    constexpr bool TR = MODE != 0;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int m = 16 * (threadIdx.x >> 6) + li;
    SvAcc<T, NCB> acc;
    acc.zero();
    // lf holds the fragment of the next product; after the last one it takes
    // the fused diagonal solve's TT, whose loads then overlap the last product
    T2 lf[16], xr[4 * NCB];
    // the first product's operands come from the task itself: their loads go
    // out before anything that waits on another load
    if (tk.np > 0) {
        sv_load_l<T2, TR>(lf, enc_ptr<T2>(b, tk.l0));
        sv_fetch_x<T2, NCB>(xr, vptr<T2>(vb, tk.src0, nrhs), nullptr, c0, ncol);
    }
    // the task's pair list, 64 pairs at a time, one per lane: the addresses of
    // product p + 1 are read from a register (readlane), not loaded while
    // product p waits
    int64_t pl_l = 0, pl_s = 0;
    if (tk.np > 1 && lane < tk.np) {
        const VUpdPair pr = pairs[tk.p0 + lane];
        pl_l = pr.l;
        pl_s = pr.src;
    }
    VDiagTask dg{};
    if (fz >= 0) dg = vdiag[fz];
    T2 *out = vptr<T2>(vb, tk.out, nrhs) + (int64_t)c0 * 64;
    const T2 *vin = nullptr;
    if (fz >= 0 && TR) vin = vptr<T2>(vb, dg.v, nrhs) + (int64_t)c0 * 64;
    // the target block (and the fused backward solve's v) do not depend on the
    // products: their loads are issued first, so their latency overlaps them
    // (except for 32 FP64 columns, whose registers are taken by the products)
    constexpr bool kPre = !(std::is_same<T, double>::value && NCB == 2);
    T2 opre[NCB][4], vpre[NCB][4];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = 16 * cb + M::out_row(lk, r);
            opre[cb][r] = kPre && MODE != 1 && c < ncol ? out[c * 64 + m] : T2{0, 0};
            vpre[cb][r] = kPre && vin && c < ncol ? vin[c * 64 + m] : T2{0, 0};
        }
    if (tk.np == 0 && fz >= 0) sv_load_l<T2, TR>(lf, enc_ptr<T2>(b, dg.tt));
    for (int p = 0; p < tk.np; ++p) {
        T2 *xs = sm.xs[p & 1];
        sv_put_x<T2, NCB>(xs, xr);
        __syncthreads();
        T2 lc[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) lc[j] = lf[j];
        if (p + 1 < tk.np) {
            const int q = p + 1;
            if ((q & 63) == 0) {  // next 64 pairs of the list
                const int i = q + lane;
                if (i < tk.np) {
                    const VUpdPair pr = pairs[tk.p0 + i];
                    pl_l = pr.l;
                    pl_s = pr.src;
                }
            }
            const int64_t nl = rdlane64(pl_l, q & 63), ns = rdlane64(pl_s, q & 63);
            sv_load_l<T2, TR>(lf, enc_ptr<T2>(b, nl));
            sv_fetch_x<T2, NCB>(xr, vptr<T2>(vb, ns, nrhs), nullptr, c0, ncol);
        } else if (fz >= 0) {
            sv_load_l<T2, TR>(lf, enc_ptr<T2>(b, dg.tt));
        }
        sv_mma<T, NCB>(acc, lc, xs);
    }
    // the buffer not read by the last product (its previous readers passed the last barrier)
    T2 *xd = sm.xs[tk.np & 1];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = 16 * cb + M::out_row(lk, r);
            T2 nw{0, 0};
            if (c < ncol) {
                const double2 res = acc.get(cb, r);
                const T2 old = kPre ? opre[cb][r] : (MODE != 1 ? out[c * 64 + m] : T2{0, 0});
                if (MODE == 0) nw = from_d2<T2>(csub(to_d2(old), res));
                else if (MODE == 1) nw = from_d2<T2>(res);
                else nw = from_d2<T2>(cadd(to_d2(old), res));
                out[c * 64 + m] = nw;
                // input of the fused diagonal solve: x (forward) or v - acc (backward)
                if (TR && fz >= 0) nw = from_d2<T2>(csub(to_d2(kPre ? vpre[cb][r] : vin[c * 64 + m]), to_d2(nw)));
            }
            if (fz >= 0) xd[c * SV_PQ + m] = nw;
        }
    if (fz < 0) return;
    __syncthreads();
    sv_diag<T, TR, NCB>(lf, dg, c0, ncol, vb, D, nrhs, xd, sm.xs[(tk.np + 1) & 1]);
}

template <typename T, int MODE, int NCB>
__global__ __launch_bounds__(256, 2) void vupd_kernel(const VUpdTask *tasks, const int64_t *fuse, int64_t ntask,
                                                   const VUpdPair *pairs, const VDiagTask *vdiag, Bases b, VBases vb,
                                                   DArrays D, int nrhs) {
    using T2 = typename C2T<T>::type;
    __shared__ SvSmem<T2, NCB> sm;
    const int nyb = (nrhs + 16 * NCB - 1) / (16 * NCB);
    const int64_t item = xcd_task(ntask * nyb);
    if (item >= ntask * nyb) return;
    const int64_t task = item / nyb;
    const int c0 = (int)(item - task * nyb) * 16 * NCB;
    vupd_task<T, MODE, NCB>(tasks[task], fuse[task], pairs, vdiag, b, vb, D, nrhs, c0, min(16 * NCB, nrhs - c0), sm);
}

// A whole S1 sweep: work-group g runs the ordered task list of subdomain g
// ([off[g], off[g + 1]) of the task array; every target is written by one
// task, which reads only the inputs and the outputs of earlier tasks of the
// list), one task after another.  The barrier between tasks orders the
// global stores of one task before the loads of the next (one work-group,
// one compute unit).
template <typename T, int MODE, int NCB>
__global__ __launch_bounds__(256, 2) void vseq_kernel(const VUpdTask *tasks, const int64_t *fuse, const int64_t *off,
                                                   int nsub, const VUpdPair *pairs, const VDiagTask *vdiag, Bases b,
                                                   VBases vb, DArrays D, int nrhs) {
    using T2 = typename C2T<T>::type;
    __shared__ SvSmem<T2, NCB> sm;
    const int nyb = (nrhs + 16 * NCB - 1) / (16 * NCB);
    const int64_t item = xcd_task((int64_t)nsub * nyb);
    if (item >= (int64_t)nsub * nyb) return;
    const int64_t g = item / nyb;
    const int c0 = (int)(item - g * nyb) * 16 * NCB;
    const int ncol = min(16 * NCB, nrhs - c0);
    const int64_t t0 = off[g], t1 = off[g + 1];
    for (int64_t t = t0; t < t1; ++t) {
        __syncthreads();
        vupd_task<T, MODE, NCB>(tasks[t], fuse[t], pairs, vdiag, b, vb, D, nrhs, c0, ncol, sm);
    }
}

// A whole sweep over the factor of -K in one launch, from a work queue (the
// diagonal solves that no update precedes run as a launch of their own
// before it).  Items (update tasks, each with the diagonal solve of its
// target when it writes that tile last, times the column blocks of the
// right-hand sides) are
// taken in the sweep's sequential order from one global counter (head), so
// an item waits only for items taken before it by work-groups that are
// running: the first unfinished item always has its inputs, whatever the
// number of resident work-groups, and the queue drains.  cnt[t] counts the
// completed writes of vector tile t (one per item and column block); an item
// waits until every tile in its wait list has the writes that precede it in
// the sequential order, runs, and adds one to the count of the tile it
// wrote.  The counts are polled with relaxed loads; a satisfied wait ends
// with one agent-scope acquire (an invalidation of the L1 and L2 the
// work-group reads through), and the count goes up with an agent-scope
// release (an L2 write-back) once every wave's stores are complete: the
// XCDs have separate L2 caches.  Every wait is bounded by spin_ticks of the
// constant-rate wall clock: on expiry the work-group sets *err, and every
// work-group leaves at its next look at *err, so the launch always ends; the
// host reports the flag.
// s_waitcnt immediate of vmcnt(0) alone (GFX9 encoding: vmcnt in bits 3:0
// and 15:14, expcnt 6:4, lgkmcnt 11:8 left at their maxima)
constexpr int kWaitVm0 = 0x0F70;

template <typename T, int MODE, int NCB>
__global__ __launch_bounds__(256, 2) void vchain_kernel(const ChainItem *items, int64_t nitem, const ChainWait *waits,
                                                     const VUpdTask *tasks, const VUpdPair *pairs,
                                                     const VDiagTask *vdiag, Bases b,
                                                     VBases vb, DArrays D, int nrhs, unsigned *head, unsigned *err,
                                                     unsigned *cnt, uint64_t spin_ticks) {
    using T2 = typename C2T<T>::type;
    __shared__ SvSmem<T2, NCB> sm;
    __shared__ int64_t s_item;
    __shared__ int s_ok;
    const int nyb = (nrhs + 16 * NCB - 1) / (16 * NCB);
    const int64_t total = nitem * nyb;
    for (;;) {
        __syncthreads();  // the previous item is done with LDS and s_item
        if (threadIdx.x == 0) {
            const unsigned e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_item = e ? total
                       : (int64_t)__hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        // wave-uniform (scalar registers): the item's task data then comes
        // through scalar loads, as in the one-launch-per-step kernels
        const int64_t it = rdlane64(s_item, 0);
        if (it >= total) return;
        const int64_t k = it / nyb;
        const int c0 = (int)(it - k * nyb) * 16 * NCB;
        const ChainItem ci = items[k];
        if (threadIdx.x < 64) {
            bool ok = true;
            for (int w = threadIdx.x; ok && w < ci.nw; w += 64) {
                const ChainWait cw = waits[ci.w0 + w];
                const unsigned need = (unsigned)cw.writes * (unsigned)nyb;
                const uint64_t t0 = wall_clock64();
                while (__hip_atomic_load(cnt + cw.tile, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                        wall_clock64() - t0 > spin_ticks) {
                        __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = false;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            const bool all = __all(ok ? 1 : 0) != 0;
            if (threadIdx.x == 0) s_ok = all ? 1 : 0;
            // acquire once for the work-group: its waves share this compute
            // unit's L1 and this XCD's L2, and the invalidation completes
            // before the barrier lets the other waves load
            if (all) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __builtin_amdgcn_s_waitcnt(kWaitVm0);
            }
        }
        __syncthreads();
        if (!__builtin_amdgcn_readfirstlane(s_ok)) return;
        const int ncol = min(16 * NCB, nrhs - c0);
        vupd_task<T, MODE, NCB>(tasks[ci.idx], ci.fz, pairs, vdiag, b, vb, D, nrhs, c0, ncol, sm);
        // every wave's stores complete in L2 before the barrier; then one L2
        // write-back for the work-group, complete before the count goes up
        // (an explicit wait: the release sequence's own wait is dropped by
        // the compiler when no store of this wave is outstanding)
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
        __syncthreads();
        if (threadIdx.x == 0 && ci.sig >= 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_s_waitcnt(kWaitVm0);
            __hip_atomic_fetch_add(cnt + ci.sig, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// zeroes the write counts of both K sweeps and their queue heads (not the
// error flag, which stays set until the host has read it)
__global__ void vchain_reset_kernel(unsigned *head, unsigned *cnt, int64_t n) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) cnt[idx] = 0;
    if (idx < 2) head[idx] = 0;
}

// XK[R] = X[h0(R)] + X[h1(R)]  (the two subdomain copies of each multiplier row)
template <typename T2>
__global__ void vgather_h_kernel(T2 *XK, const T2 *X, const int64_t *hmap, int64_t nrows, int nrhs) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nrows * nrhs) return;
    int64_t tile = idx / (64 * nrhs);
    int rem = (int)(idx - tile * 64 * nrhs);
    int c = rem >> 6, r = rem & 63;
    int64_t R = tile * 64 + r;
    double2 s = make_double2(0, 0);
    int64_t a = hmap[2 * R], bb = hmap[2 * R + 1];
    if (a >= 0) s = cadd(s, to_d2(X[vrow_elem(a, c, nrhs)]));
    if (bb >= 0) s = cadd(s, to_d2(X[vrow_elem(bb, c, nrhs)]));
    XK[idx] = from_d2<T2>(s);
}

// X[R] = XK[lmap(R)] on the multiplier rows of every subdomain
template <typename T2>
__global__ void vscatter_lam_kernel(T2 *X, const T2 *XK, const int64_t *lmap, int64_t nrows, int nrhs) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nrows * nrhs) return;
    int64_t tile = idx / (64 * nrhs);
    int rem = (int)(idx - tile * 64 * nrhs);
    int c = rem >> 6, r = rem & 63;
    int64_t src = lmap[tile * 64 + r];
    if (src >= 0) X[idx] = XK[vrow_elem(src, c, nrhs)];
}

// E[c][e] (=|+=) X[owner row of e]
template <typename T2, bool ACC>
__global__ void vcollect_kernel(double2 *E, const T2 *X, const int64_t *cmap, int64_t ne, int nrhs) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ne * nrhs) return;
    int c = (int)(idx / ne);
    int64_t e = idx - (int64_t)c * ne;
    double2 v = to_d2(X[vrow_elem(cmap[e], c, nrhs)]);
    E[idx] = ACC ? cadd(E[idx], v) : v;
}

// Norm reductions.  nmax[p * nrhs + c] holds the bit pattern of a
// non-negative double (monotone under unsigned comparison) or of a NaN, which
// compares above every number, so a NaN anywhere in the data reaches the host.
// A block covers consecutive rows (kRowsPer * 256 in the load-norm kernel);
// each thread keeps running maxima for its rows and the block combines them
// in LDS, so a block that lies inside one problem issues one atomic per
// right-hand side.
constexpr int kRowsPer = 8;

__device__ __forceinline__ double nanmax(double m, double v) { return (v > m || v != v) ? v : m; }

__device__ __forceinline__ void atomic_max_bits(unsigned long long *a, double v) {
    atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

// Combines the running maxima m[c] (c < nc) of every thread of the block, for
// problem pcur (-1: the thread saw no row), into nmax[pcur * nrhs + c0 + c].
// Called by every thread of the block.
template <int NC>
__device__ __forceinline__ void block_fold_max(unsigned long long *nmax, int pcur, const double (&m)[NC], int nrhs,
                                               int c0, int nc) {
    __shared__ int s_pmin, s_pmax;
    __shared__ double s_red[NC][4];
    if (threadIdx.x == 0) {
        s_pmin = INT_MAX;
        s_pmax = -1;
    }
    __syncthreads();
    if (pcur >= 0) {
        atomicMin(&s_pmin, pcur);
        atomicMax(&s_pmax, pcur);
    }
    __syncthreads();
    const int pmin = s_pmin, pmax = s_pmax;
    if (pmax < 0) return;  // the whole block is past the last row
    if (pmin == pmax) {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double v = m[c];
            for (int off = 32; off >= 1; off >>= 1) v = nanmax(v, __shfl_xor(v, off));
            if (lane == 0) s_red[c][wv] = v;
        }
        __syncthreads();
        if ((int)threadIdx.x < nc) {
            const int c = threadIdx.x;
            const double v = nanmax(nanmax(s_red[c][0], s_red[c][1]), nanmax(s_red[c][2], s_red[c][3]));
            atomic_max_bits(&nmax[(int64_t)pmin * nrhs + c0 + c], v);
        }
    } else if (pcur >= 0) {  // a block across a problem boundary (batches)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < nc) atomic_max_bits(&nmax[(int64_t)pcur * nrhs + c0 + c], m[c]);
    }
}

// Et[e][c] = E[c][e]: the field with the right-hand sides of one edge
// contiguous, so that the residual's gathers of a matrix entry's column read
// 16 right-hand sides as one 256-byte run.  Tiles of 64 edges x 16 columns
// through LDS; reads and writes coalesced.
__global__ __launch_bounds__(256) void vtranspose_kernel(double2 *Et, const double2 *E, int64_t ne, int nrhs) {
    __shared__ double2 tile[16][65];
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int c0 = blockIdx.y * 16;
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = (t >> 6) + 4 * i, r = t & 63;
        if (r0 + r < ne && c0 + c < nrhs) tile[c][r] = E[(int64_t)(c0 + c) * ne + r0 + r];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int idx = t + 256 * i, r = idx >> 4, c = idx & 15;
        if (r0 + r < ne && c0 + c < nrhs) Et[(r0 + r) * nrhs + c0 + c] = tile[c][r];
    }
}

// r = f - S E (CSR of the global FEM matrix, FP64) from Et.  A block takes
// RES_ROWS rows and 16 right-hand sides (blockIdx.y); lane l of a wave works
// on right-hand side l % 16 of row l / 16 of the wave's four current rows, so
// the gather of Et for one matrix entry is a contiguous 256-byte run shared
// by 16 lanes.  nmax[p * nrhs + c] (zeroed by the caller) gets the largest
// |r[c][e]| (modulus) over the rows e of problem p = eprob[e]; rows with
// eprob[e] < 0 (PEC edges) get r = 0 and no norm contribution.
constexpr int RES_ROWS = 256;

__global__ __launch_bounds__(256) void residual_kernel(double2 *r, const double2 *f, const double2 *Et,
                                                       const int64_t *rowptr, const int32_t *col, const double2 *val,
                                                       const int32_t *eprob, int64_t ne, int nrhs,
                                                       unsigned long long *nmax) {
    __shared__ int s_pmin, s_pmax;
    __shared__ double s_red[16][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cl = lane & 15, rs = lane >> 4;
    const int c0 = blockIdx.y * 16, c = c0 + cl;
    const int nc = min(16, nrhs - c0);
    const bool cok = cl < nc;
    const int64_t base = (int64_t)blockIdx.x * RES_ROWS;
    int pcur = -1;
    double m = 0.0;
    for (int it = 0; it < RES_ROWS / 16; ++it) {
        const int64_t row = base + 16 * it + 4 * wave + rs;
        if (row >= ne) break;
        const int p = eprob[row];
        if (p < 0) {  // a PEC edge: no unknown, no residual
            if (cok) r[(int64_t)c * ne + row] = make_double2(0, 0);
            continue;
        }
        if (p != pcur) {  // a new problem (batches): fold this thread's maximum so far
            if (pcur >= 0 && cok) atomic_max_bits(&nmax[(int64_t)pcur * nrhs + c], m);
            pcur = p;
            m = 0.0;
        }
        double2 s = cok ? f[(int64_t)c * ne + row] : make_double2(0, 0);
        const int64_t k1 = rowptr[row + 1];
        for (int64_t k = rowptr[row]; k < k1; ++k) {
            const double2 v = val[k];
            const int64_t j = col[k];
            if (cok) s = cfms(s, v, Et[j * nrhs + c]);
        }
        if (cok) {
            r[(int64_t)c * ne + row] = s;
            m = nanmax(m, sqrt(s.x * s.x + s.y * s.y));
        }
    }
    // one atomic per block and right-hand side when the block lies in one problem
    if (threadIdx.x == 0) {
        s_pmin = INT_MAX;
        s_pmax = -1;
    }
    __syncthreads();
    if (pcur >= 0) {
        atomicMin(&s_pmin, pcur);
        atomicMax(&s_pmax, pcur);
    }
    __syncthreads();
    const int pmin = s_pmin, pmax = s_pmax;
    if (pmax < 0) return;
    if (pmin == pmax) {
        double v = cok ? m : 0.0;
        v = nanmax(v, __shfl_xor(v, 16));
        v = nanmax(v, __shfl_xor(v, 32));
        if (lane < 16) s_red[lane][wave] = v;
        __syncthreads();
        if ((int)threadIdx.x < nc) {
            const int cc = threadIdx.x;
            const double w = nanmax(nanmax(s_red[cc][0], s_red[cc][1]), nanmax(s_red[cc][2], s_red[cc][3]));
            atomic_max_bits(&nmax[(int64_t)pmin * nrhs + c0 + cc], w);
        }
    } else if (pcur >= 0 && cok) {
        atomic_max_bits(&nmax[(int64_t)pcur * nrhs + c], m);
    }
}

// nmax[p * nrhs + c] = max |v[c][e]| over the rows e of problem p (|z| =
// modulus); blockIdx.y = right-hand side, kRowsPer elements per thread
__global__ __launch_bounds__(256) void rownorm_max_kernel(unsigned long long *nmax, const double2 *v,
                                                          const int32_t *eprob, int64_t ne, int nrhs) {
    const int c = blockIdx.y;
    const int64_t base = (int64_t)blockIdx.x * 256 * kRowsPer;
    int pcur = -1;
    double m[1] = {0.0};
    for (int i = 0; i < kRowsPer; ++i) {
        const int64_t e = base + threadIdx.x + 256 * i;
        if (e >= ne) break;
        const int p = eprob[e];
        if (p < 0) continue;  // a PEC edge: not part of the norm
        if (p != pcur) {
            if (pcur >= 0) atomic_max_bits(&nmax[(int64_t)pcur * nrhs + c], m[0]);
            pcur = p;
            m[0] = 0.0;
        }
        const double2 z = v[(int64_t)c * ne + e];
        m[0] = nanmax(m[0], sqrt(z.x * z.x + z.y * z.y));
    }
    block_fold_max<1>(nmax, pcur, m, nrhs, c, 1);
}

// Largest |X(r, c) - X(owner(r), c)| over the subdomain copies r of shared
// edges that are not the owner copy (copy map: owner row, or -1) and every
// right-hand side, folded into *dmax (bit pattern of a non-negative double,
// NaN kept).  One atomic per block.
template <typename T2>
__global__ __launch_bounds__(256) void copy_disc_kernel(unsigned long long *dmax, const T2 *X, const int64_t *cmap,
                                                        int64_t nrows, int nrhs) {
    __shared__ double red[4];
    double m = 0.0;
    const int64_t total = nrows * nrhs;
    for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
        const int c = (int)(idx / nrows);
        const int64_t r = idx - (int64_t)c * nrows;
        const int64_t o = cmap[r];
        if (o < 0) continue;
        const double2 a = to_d2(X[vrow_elem(r, c, nrhs)]), b = to_d2(X[vrow_elem(o, c, nrhs)]);
        const double dx = a.x - b.x, dy = a.y - b.y;
        m = nanmax(m, sqrt(dx * dx + dy * dy));
    }
    for (int off = 32; off >= 1; off >>= 1) m = nanmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) m = nanmax(m, red[w]);
        atomic_max_bits(dmax, m);
    }
}

__global__ void conj_kernel(double2 *out, const double2 *in, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = make_double2(in[i].x, -in[i].y);
}

// grad[t] = k^2 Re sum_c w_t^T M_t E_t (M_t: unit-eps_r element mass, 6x6)
__global__ void adjoint_grad_kernel(double *grad, const double2 *w, const double2 *E, const int64_t *tet_edges,
                                    const double *mass, double k2, int64_t nt, int64_t ne, int nrhs) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    int64_t ed[6];
    for (int a = 0; a < 6; ++a) ed[a] = tet_edges[6 * t + a];
    const double *M = mass + 36 * t;
    double s = 0.0;
    for (int c = 0; c < nrhs; ++c) {
        double2 wl[6], el[6];
        for (int a = 0; a < 6; ++a) { wl[a] = w[(int64_t)c * ne + ed[a]]; el[a] = E[(int64_t)c * ne + ed[a]]; }
        for (int a = 0; a < 6; ++a) {
            double2 me = make_double2(0, 0);
            for (int bb = 0; bb < 6; ++bb) me = make_double2(me.x + M[6 * a + bb] * el[bb].x, me.y + M[6 * a + bb] * el[bb].y);
            s += wl[a].x * me.x - wl[a].y * me.y;
        }
    }
    grad[t] = k2 * s;
}

// ------------------------------------------------------------ launchers --
namespace {
inline dim3 g1(int64_t n, int b = 256) { return dim3((unsigned)((n + b - 1) / b > 0 ? (n + b - 1) / b : 1)); }
}  // namespace

template <typename T>
hipError_t launch_vsplit(void *X, const double2 *f, const int64_t *map, int64_t nrows, int nrhs, int64_t ne,
                         hipStream_t s) {
    using T2 = typename C2T<T>::type;
    hipLaunchKernelGGL(vsplit_kernel<T2>, g1(nrows * nrhs), dim3(256), 0, s, (T2 *)X, f, map, nrows, nrhs, ne);
    return hipGetLastError();
}
// right-hand sides per work-group: 16 (one MFMA column block) or 32; cols
// (16 or 32, 0 = 32) caps it
inline int sv_ncb(int nrhs, int cols) { return nrhs <= 16 || cols == 16 ? 1 : 2; }
inline unsigned sv_groups(int64_t ntask) { return (unsigned)(((ntask + kXcds - 1) / kXcds) * kXcds); }

template <typename T>
hipError_t launch_vdiag(const VDiagTask *tasks, int64_t ntask, int maxt, bool bwd, const Bases &b, const VBases &vb,
                        const DArrays &D, int nrhs, int cols, hipStream_t s) {
    using T2 = typename C2T<T>::type;
    if (ntask <= 0) return hipSuccess;
    if (maxt <= 1) {
        const int ncb = sv_ncb(nrhs, cols);
        dim3 grid(sv_groups(ntask * ((nrhs + 16 * ncb - 1) / (16 * ncb))));
        if (ncb == 1) {
            if (bwd) hipLaunchKernelGGL((vdiag_kernel<T, true, 1>), grid, dim3(256), 0, s, tasks, ntask, b, vb, D, nrhs);
            else hipLaunchKernelGGL((vdiag_kernel<T, false, 1>), grid, dim3(256), 0, s, tasks, ntask, b, vb, D, nrhs);
        } else {
            if (bwd) hipLaunchKernelGGL((vdiag_kernel<T, true, 2>), grid, dim3(256), 0, s, tasks, ntask, b, vb, D, nrhs);
            else hipLaunchKernelGGL((vdiag_kernel<T, false, 2>), grid, dim3(256), 0, s, tasks, ntask, b, vb, D, nrhs);
        }
    } else {
        dim3 grid((unsigned)ntask, (unsigned)((nrhs + 31) / 32));
        if (bwd) hipLaunchKernelGGL((vdiag_multi_kernel<T2, true>), grid, dim3(256), 0, s, tasks, b, vb, D, nrhs);
        else hipLaunchKernelGGL((vdiag_multi_kernel<T2, false>), grid, dim3(256), 0, s, tasks, b, vb, D, nrhs);
    }
    return hipGetLastError();
}

template <typename T, int NCB>
void launch_vupd_ncb(const VUpdTask *tasks, const int64_t *fuse, int64_t ntask, const VUpdPair *pairs,
                     const VDiagTask *vdiag, int mode, const Bases &b, const VBases &vb, const DArrays &D, int nrhs,
                     hipStream_t s) {
    dim3 grid(sv_groups(ntask * ((nrhs + 16 * NCB - 1) / (16 * NCB))));
    if (mode == 0)
        hipLaunchKernelGGL((vupd_kernel<T, 0, NCB>), grid, dim3(256), 0, s, tasks, fuse, ntask, pairs, vdiag, b, vb, D,
                           nrhs);
    else if (mode == 1)
        hipLaunchKernelGGL((vupd_kernel<T, 1, NCB>), grid, dim3(256), 0, s, tasks, fuse, ntask, pairs, vdiag, b, vb, D,
                           nrhs);
    else
        hipLaunchKernelGGL((vupd_kernel<T, 2, NCB>), grid, dim3(256), 0, s, tasks, fuse, ntask, pairs, vdiag, b, vb, D,
                           nrhs);
}
template <typename T>
hipError_t launch_vseq(const VUpdTask *tasks, const int64_t *fuse, const int64_t *off, int nsub,
                       const VUpdPair *pairs, const VDiagTask *vdiag, bool bwd, const Bases &b, const VBases &vb,
                       const DArrays &D, int nrhs, int cols, hipStream_t s) {
    if (nsub <= 0) return hipSuccess;
    const int ncb = sv_ncb(nrhs, cols);
    dim3 grid(sv_groups((int64_t)nsub * ((nrhs + 16 * ncb - 1) / (16 * ncb))));
    if (ncb == 1) {
        if (bwd) hipLaunchKernelGGL((vseq_kernel<T, 1, 1>), grid, dim3(256), 0, s, tasks, fuse, off, nsub, pairs, vdiag,
                                    b, vb, D, nrhs);
        else hipLaunchKernelGGL((vseq_kernel<T, 0, 1>), grid, dim3(256), 0, s, tasks, fuse, off, nsub, pairs, vdiag, b,
                                vb, D, nrhs);
    } else {
        if (bwd) hipLaunchKernelGGL((vseq_kernel<T, 1, 2>), grid, dim3(256), 0, s, tasks, fuse, off, nsub, pairs, vdiag,
                                    b, vb, D, nrhs);
        else hipLaunchKernelGGL((vseq_kernel<T, 0, 2>), grid, dim3(256), 0, s, tasks, fuse, off, nsub, pairs, vdiag, b,
                                vb, D, nrhs);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_vupd(const VUpdTask *tasks, const int64_t *fuse, int64_t ntask, const VUpdPair *pairs,
                       const VDiagTask *vdiag, int mode, const Bases &b, const VBases &vb, const DArrays &D, int nrhs,
                       int cols, hipStream_t s) {
    if (ntask <= 0) return hipSuccess;
    if (sv_ncb(nrhs, cols) == 1) launch_vupd_ncb<T, 1>(tasks, fuse, ntask, pairs, vdiag, mode, b, vb, D, nrhs, s);
    else launch_vupd_ncb<T, 2>(tasks, fuse, ntask, pairs, vdiag, mode, b, vb, D, nrhs, s);
    return hipGetLastError();
}
hipError_t launch_vchain_reset(unsigned *head, unsigned *cnt, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(vchain_reset_kernel, g1(std::max<int64_t>(n, 2)), dim3(256), 0, s, head, cnt, n);
    return hipGetLastError();
}

// work-groups of a work-queue sweep: as many as can be resident at once (the
// queue does not need them all resident; more would only wait for a slot),
// at most one per item
template <typename K>
unsigned chain_grid(K kernel, int64_t items) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0) != hipSuccess) return 0;
    const int64_t g = std::min<int64_t>((int64_t)std::max(per, 1) * std::max(cus, 1), items);
    return (unsigned)std::max<int64_t>(g, 1);
}

template <typename T, int MODE, int NCB>
hipError_t launch_vchain_ncb(const ChainItem *items, int64_t nitem, const ChainWait *waits, const VUpdTask *tasks,
                             const VUpdPair *pairs, const VDiagTask *vdiag, const Bases &b,
                             const VBases &vb, const DArrays &D, int nrhs, unsigned *head, unsigned *err,
                             unsigned *cnt, uint64_t spin_ticks, hipStream_t s) {
    auto kern = vchain_kernel<T, MODE, NCB>;
    const int64_t total = nitem * ((nrhs + 16 * NCB - 1) / (16 * NCB));
    const unsigned grid = chain_grid(kern, total);
    if (grid == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, items, nitem, waits, tasks, pairs, vdiag, b, vb, D, nrhs,
                       head, err, cnt, spin_ticks);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_vchain(const ChainItem *items, int64_t nitem, const ChainWait *waits, const VUpdTask *tasks,
                         const VUpdPair *pairs, const VDiagTask *vdiag, bool bwd, const Bases &b,
                         const VBases &vb, const DArrays &D, int nrhs, int cols, unsigned *head, unsigned *err,
                         unsigned *cnt, uint64_t spin_ticks, hipStream_t s) {
    if (nitem <= 0) return hipSuccess;
    const bool one = sv_ncb(nrhs, cols) == 1;
    if (bwd)
        return one ? launch_vchain_ncb<T, 2, 1>(items, nitem, waits, tasks, pairs, vdiag, b, vb, D, nrhs, head,
                                                err, cnt, spin_ticks, s)
                   : launch_vchain_ncb<T, 2, 2>(items, nitem, waits, tasks, pairs, vdiag, b, vb, D, nrhs, head,
                                                err, cnt, spin_ticks, s);
    return one ? launch_vchain_ncb<T, 0, 1>(items, nitem, waits, tasks, pairs, vdiag, b, vb, D, nrhs, head, err,
                                            cnt, spin_ticks, s)
               : launch_vchain_ncb<T, 0, 2>(items, nitem, waits, tasks, pairs, vdiag, b, vb, D, nrhs, head, err,
                                            cnt, spin_ticks, s);
}

template <typename T>
hipError_t launch_vgather_h(void *XK, const void *X, const int64_t *hmap, int64_t nrows_k, int nrhs, hipStream_t s) {
    using T2 = typename C2T<T>::type;
    if (nrows_k <= 0) return hipSuccess;
    hipLaunchKernelGGL(vgather_h_kernel<T2>, g1(nrows_k * nrhs), dim3(256), 0, s, (T2 *)XK, (const T2 *)X, hmap,
                       nrows_k, nrhs);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_vscatter_lam(void *X, const void *XK, const int64_t *lmap, int64_t nrows_s1, int nrhs,
                               hipStream_t s) {
    using T2 = typename C2T<T>::type;
    hipLaunchKernelGGL(vscatter_lam_kernel<T2>, g1(nrows_s1 * nrhs), dim3(256), 0, s, (T2 *)X, (const T2 *)XK, lmap,
                       nrows_s1, nrhs);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_vcollect(double2 *E, const void *X, const int64_t *cmap, int64_t ne, int nrhs, bool accumulate,
                           hipStream_t s) {
    using T2 = typename C2T<T>::type;
    if (accumulate)
        hipLaunchKernelGGL((vcollect_kernel<T2, true>), g1(ne * nrhs), dim3(256), 0, s, E, (const T2 *)X, cmap, ne, nrhs);
    else
        hipLaunchKernelGGL((vcollect_kernel<T2, false>), g1(ne * nrhs), dim3(256), 0, s, E, (const T2 *)X, cmap, ne, nrhs);
    return hipGetLastError();
}

hipError_t launch_residual(double2 *r, const double2 *f, const double2 *E, double2 *Et, const int64_t *rowptr,
                           const int32_t *col, const double2 *val, const int32_t *eprob, int64_t ne, int nrhs,
                           unsigned long long *nmax, hipStream_t s) {
    const unsigned cb = (unsigned)((nrhs + 15) / 16);
    hipLaunchKernelGGL(vtranspose_kernel, dim3(g1(ne, 64).x, cb), dim3(256), 0, s, Et, E, ne, nrhs);
    hipLaunchKernelGGL(residual_kernel, dim3(g1(ne, RES_ROWS).x, cb), dim3(256), 0, s, r, f, Et, rowptr, col, val,
                       eprob, ne, nrhs, nmax);
    return hipGetLastError();
}
hipError_t launch_rownorm_max(unsigned long long *nmax, const double2 *v, const int32_t *eprob, int64_t ne, int nrhs,
                              hipStream_t s) {
    hipLaunchKernelGGL(rownorm_max_kernel, dim3(g1(ne, 256 * kRowsPer).x, (unsigned)nrhs), dim3(256), 0, s, nmax, v,
                       eprob, ne, nrhs);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_copy_disc(unsigned long long *dmax, const void *X, const int64_t *cmap, int64_t nrows, int nrhs,
                            hipStream_t s) {
    using T2 = typename C2T<T>::type;
    const int64_t total = nrows * nrhs;
    const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL((copy_disc_kernel<T2>), dim3(grid), dim3(256), 0, s, dmax, (const T2 *)X, cmap, nrows, nrhs);
    return hipGetLastError();
}
hipError_t launch_conj(double2 *out, const double2 *in, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(conj_kernel, g1(n), dim3(256), 0, s, out, in, n);
    return hipGetLastError();
}
hipError_t launch_adjoint_grad(double *grad, const double2 *w, const double2 *E, const int64_t *tet_edges,
                               const double *mass, double k2, int64_t nt, int64_t ne, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(adjoint_grad_kernel, g1(nt), dim3(256), 0, s, grad, w, E, tet_edges, mass, k2, nt, ne, nrhs);
    return hipGetLastError();
}

#define D3M_INST(T)                                                                                               \
    template hipError_t launch_copy_disc<T>(unsigned long long *, const void *, const int64_t *, int64_t, int,      \
                                            hipStream_t);                                                         \
    template hipError_t launch_vsplit<T>(void *, const double2 *, const int64_t *, int64_t, int, int64_t,          \
                                         hipStream_t);                                                            \
    template hipError_t launch_vdiag<T>(const VDiagTask *, int64_t, int, bool, const Bases &, const VBases &,           \
                                        const DArrays &, int, int, hipStream_t);                                  \
    template hipError_t launch_vupd<T>(const VUpdTask *, const int64_t *, int64_t, const VUpdPair *,            \
                                       const VDiagTask *, int, const Bases &, const VBases &, const DArrays &, int, \
                                       int, hipStream_t);                                                         \
    template hipError_t launch_vseq<T>(const VUpdTask *, const int64_t *, const int64_t *, int, const VUpdPair *,  \
                                       const VDiagTask *, bool, const Bases &, const VBases &, const DArrays &, int, \
                                       int, hipStream_t);                                                         \
    template hipError_t launch_vchain<T>(const ChainItem *, int64_t, const ChainWait *, const VUpdTask *,         \
                                         const VUpdPair *, const VDiagTask *, bool, const Bases &,                  \
                                         const VBases &, const DArrays &, int, int, unsigned *, unsigned *,       \
                                         unsigned *, uint64_t, hipStream_t);                                      \
    template hipError_t launch_vgather_h<T>(void *, const void *, const int64_t *, int64_t, int, hipStream_t);     \
    template hipError_t launch_vscatter_lam<T>(void *, const void *, const int64_t *, int64_t, int, hipStream_t);  \
    template hipError_t launch_vcollect<T>(double2 *, const void *, const int64_t *, int64_t, int, bool,           \
                                           hipStream_t);
D3M_INST(double)
D3M_INST(float)
#undef D3M_INST

}  // namespace d3m
