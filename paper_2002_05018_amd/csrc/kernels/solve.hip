// Solve-phase kernels (recipe steps 6-7 of Section II) and the FP64
// refinement / adjoint helpers.  Vector tiles hold 64 rows x nrhs columns,
// column-major (one right-hand side after another), so one 64 x 64 factor
// tile is applied to every right-hand side while it sits in LDS.
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

// Tile products of the solve sweeps: out (64 x ncol, ncol <= 8 right-hand
// sides per block) gets op(L) X for 64 x 64 factor tiles L, op = identity
// or transpose.  Lane r of wave w (4 waves) accumulates row r over the
// inner indices q in [16 w, 16 w + 16); the four partial sums are added in
// a fixed order through LDS (results do not depend on timing).  For op =
// identity each lane reads its 16 entries of L straight from memory (one
// 1 KB row of lanes per load); for the transpose the tile is staged through
// LDS (row stride 65) first.  The X block is staged through LDS and read
// as a broadcast.
constexpr int SV_COLS = 8;

template <typename T2, bool TR> struct SolveSmem {
    double2 ls[TR ? 64 * 65 : 4 * SV_COLS * 64];  // staged tile; reused for the partial sums
    double2 xs[SV_COLS * 64];                     // X(q, c) at c * 64 + q
};

// this thread's 16 entries op(L)(r, q), q = 16 w + j
template <typename T2, bool TR>
__device__ __forceinline__ void load_ltile(double (&lx)[16], double (&ly)[16], const T2 *tile, double2 *ls) {
    const int r = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (!TR) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const T2 v = tile[(16 * w + j) * 64 + r];
            lx[j] = v.x;
            ly[j] = v.y;
        }
    } else {
        // stage: element e of the column-major tile is L(e & 63, e >> 6)
        T2 v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = tile[threadIdx.x + 256 * i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = threadIdx.x + 256 * i;
            ls[(e >> 6) * 65 + (e & 63)] = to_d2(v[i]);
        }
        __syncthreads();
        // L^T(r, q) = L(q, r) at ls[r * 65 + q]
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const double2 u = ls[r * 65 + 16 * w + j];
            lx[j] = u.x;
            ly[j] = u.y;
        }
    }
}

// X block (columns c0 .. c0 + ncol - 1 of a vector tile, minus sub) into xs
template <typename T2>
__device__ __forceinline__ void stage_x(double2 *xs, const T2 *src, const T2 *sub, int c0, int ncol) {
    double2 v[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int e = threadIdx.x + 256 * i;
        v[i] = make_double2(0, 0);
        if (e < 64 * ncol) {
            v[i] = to_d2(src[(int64_t)c0 * 64 + e]);
            if (sub) v[i] = csub(v[i], to_d2(sub[(int64_t)c0 * 64 + e]));
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int e = threadIdx.x + 256 * i;
        if (e < 64 * ncol) xs[e] = v[i];
    }
    __syncthreads();
}

__device__ __forceinline__ void tile_fma(double (&ax)[SV_COLS], double (&ay)[SV_COLS], const double (&lx)[16],
                                         const double (&ly)[16], const double2 *xs, int ncol) {
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int q = 16 * w + j;
#pragma unroll
        for (int c = 0; c < SV_COLS; ++c) {
            if (c < ncol) {
                const double2 x = xs[c * 64 + q];
                ax[c] = fma(lx[j], x.x, fma(-ly[j], x.y, ax[c]));
                ay[c] = fma(lx[j], x.y, fma(ly[j], x.x, ay[c]));
            }
        }
    }
}

// sum of the four waves' partials for (row r, column c) in a fixed order;
// thread (r, w) finishes columns w and w + 4
__device__ __forceinline__ void reduce_partials(double2 *red, const double (&ax)[SV_COLS], const double (&ay)[SV_COLS],
                                                double2 (&res)[2]) {
    const int r = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < SV_COLS; ++c) red[(w * SV_COLS + c) * 64 + r] = make_double2(ax[c], ay[c]);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = w + 4 * h;
        double2 s = red[(0 * SV_COLS + c) * 64 + r];
        s = cadd(s, red[(1 * SV_COLS + c) * 64 + r]);
        s = cadd(s, red[(2 * SV_COLS + c) * 64 + r]);
        s = cadd(s, red[(3 * SV_COLS + c) * 64 + r]);
        res[h] = s;
    }
}

// Forward: y = TT x (TT = L^{-1} P^T of the block), v = D^{-1} y.
// Backward: x = TT^T (v - acc) (= P L^{-T} (v - acc)).
// Blocks of one tile (n <= 64); chunk selects 8 right-hand sides.
// vdiag_finish applies TT (or TT^T) to the block already staged in sm.xs and
// writes the outputs.
template <typename T2, bool BWD, typename Smem>
__device__ __forceinline__ void vdiag_finish(const VDiagTask &tk, int chunk, const Bases &b, const VBases &vb,
                                             const DArrays &D, int nrhs, Smem &sm) {
    const int c0 = chunk * SV_COLS;
    const int ncol = min(SV_COLS, nrhs - c0);
    const int r = threadIdx.x & 63, w = threadIdx.x >> 6;
    double lx[16], ly[16], ax[SV_COLS], ay[SV_COLS];
#pragma unroll
    for (int c = 0; c < SV_COLS; ++c) ax[c] = ay[c] = 0.0;
    load_ltile<T2, BWD>(lx, ly, enc_ptr<T2>(b, tk.tt), sm.ls);
    tile_fma(ax, ay, lx, ly, sm.xs, ncol);
    double2 res[2];
    reduce_partials(sm.ls, ax, ay, res);
    if (BWD) {
        T2 *x = vptr<T2>(vb, tk.x, nrhs);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = w + 4 * h;
            if (c < ncol) x[(int64_t)(c0 + c) * 64 + r] = from_d2<T2>(res[h]);
        }
        return;
    }
    // v = D^{-1} y within the tile (2x2 pivots never cross it); y goes through xs
    T2 *y = vptr<T2>(vb, tk.y, nrhs);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = w + 4 * h;
        if (c < ncol) {
            sm.xs[c * 64 + r] = res[h];
            y[(int64_t)(c0 + c) * 64 + r] = from_d2<T2>(res[h]);
        }
    }
    __syncthreads();
    T2 *v = vptr<T2>(vb, tk.v, nrhs);
    const int64_t dr = tk.drow + r;
    const bool live = r < tk.n;
    const double2 di = live ? D.dinv[dr] : make_double2(0, 0);
    const int pv = live ? D.piv[dr] : 0;
    const double2 dio = pv ? D.dinvoff[dr] : make_double2(0, 0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = w + 4 * h;
        if (c < ncol) {
            double2 val = cmul(di, sm.xs[c * 64 + r]);
            if (pv != 0) val = cadd(val, cmul(dio, sm.xs[c * 64 + r + pv]));
            v[(int64_t)(c0 + c) * 64 + r] = from_d2<T2>(live ? val : make_double2(0, 0));
        }
    }
}

template <typename T2, bool BWD>
__global__ __launch_bounds__(256) void vdiag_kernel(const VDiagTask *tasks, Bases b, VBases vb, DArrays D, int nrhs) {
    __shared__ SolveSmem<T2, BWD> sm;
    const VDiagTask tk = tasks[blockIdx.x];
    const int c0 = blockIdx.y * SV_COLS;
    const int ncol = min(SV_COLS, nrhs - c0);
    if (BWD) {
        const T2 *accv = tk.acc >= 0 ? vptr<T2>(vb, tk.acc, nrhs) : nullptr;
        stage_x<T2>(sm.xs, vptr<T2>(vb, tk.v, nrhs), accv, c0, ncol);
    } else {
        stage_x<T2>(sm.xs, vptr<T2>(vb, tk.x, nrhs), nullptr, c0, ncol);
    }
    vdiag_finish<T2, BWD>(tk, blockIdx.y, b, vb, D, nrhs, sm);
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
// transpose (modes 1, 2); blockIdx.y selects 8 right-hand sides.  When
// fuse[task] >= 0 this update is the last one its target receives before the
// diagonal solve fuse[task] (forward: the target is that block's x; backward:
// its accumulator), so the work-group goes on with that solve from the new
// values kept in LDS, saving a launch per sweep step.
template <typename T2, int MODE>
__global__ __launch_bounds__(256) void vupd_kernel(const VUpdTask *tasks, const int64_t *fuse, const VUpdPair *pairs,
                                                   const VDiagTask *vdiag, Bases b, VBases vb, DArrays D, int nrhs) {
    constexpr bool TR = MODE != 0;
    __shared__ SolveSmem<T2, TR> sm;
    const VUpdTask tk = tasks[blockIdx.x];
    const int64_t fz = fuse[blockIdx.x];
    const int c0 = blockIdx.y * SV_COLS;
    const int ncol = min(SV_COLS, nrhs - c0);
    const int r = threadIdx.x & 63, w = threadIdx.x >> 6;
    double ax[SV_COLS], ay[SV_COLS];
#pragma unroll
    for (int c = 0; c < SV_COLS; ++c) ax[c] = ay[c] = 0.0;
    for (int p = 0; p < tk.np; ++p) {
        const VUpdPair pr = pairs[tk.p0 + p];
        double lx[16], ly[16];
        load_ltile<T2, TR>(lx, ly, enc_ptr<T2>(b, pr.l), sm.ls);
        stage_x<T2>(sm.xs, vptr<T2>(vb, pr.src, nrhs), nullptr, c0, ncol);
        tile_fma(ax, ay, lx, ly, sm.xs, ncol);
    }
    double2 res[2];
    reduce_partials(sm.ls, ax, ay, res);
    T2 *out = vptr<T2>(vb, tk.out, nrhs);
    VDiagTask dg{};
    const T2 *vin = nullptr;
    if (fz >= 0) {
        dg = vdiag[fz];
        if (TR) vin = vptr<T2>(vb, dg.v, nrhs);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = w + 4 * h;
        if (c < ncol) {
            T2 *o = out + (int64_t)(c0 + c) * 64 + r;
            double2 nw;
            if (MODE == 0) nw = csub(to_d2(*o), res[h]);
            else if (MODE == 1) nw = res[h];
            else nw = cadd(to_d2(*o), res[h]);
            *o = from_d2<T2>(nw);
            // input of the fused diagonal solve: x (forward) or v - acc (backward)
            if (fz >= 0) sm.xs[c * 64 + r] = TR ? csub(to_d2(vin[(int64_t)(c0 + c) * 64 + r]), nw) : nw;
        }
    }
    if (fz < 0) return;
    __syncthreads();
    vdiag_finish<T2, TR>(dg, blockIdx.y, b, vb, D, nrhs, sm);
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

// r = f - S E (CSR of the global FEM matrix, FP64)
__global__ void residual_kernel(double2 *r, const double2 *f, const double2 *E, const int64_t *rowptr,
                                const int32_t *col, const double2 *val, int64_t ne, int nrhs) {
    int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= ne) return;
    for (int c = 0; c < nrhs; ++c) {
        double2 s = f[(int64_t)c * ne + row];
        const double2 *Ec = E + (int64_t)c * ne;
        for (int64_t k = rowptr[row]; k < rowptr[row + 1]; ++k) s = cfms(s, val[k], Ec[col[k]]);
        r[(int64_t)c * ne + row] = s;
    }
}

// out[c] = max_e |v[c][e]| (infinity norm with |z| = modulus), as the bit
// pattern of a non-negative double (monotone under unsigned comparison)
__global__ void rownorm_max_kernel(unsigned long long *out, const double2 *v, int64_t ne, int nrhs) {
    int c = blockIdx.y;
    double m = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        double2 z = v[(int64_t)c * ne + e];
        m = fmax(m, sqrt(z.x * z.x + z.y * z.y));
    }
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(&out[c], (unsigned long long)__double_as_longlong(m));
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
template <typename T>
hipError_t launch_vdiag(const VDiagTask *tasks, int64_t ntask, int maxt, bool bwd, const Bases &b, const VBases &vb,
                        const DArrays &D, int nrhs, hipStream_t s) {
    using T2 = typename C2T<T>::type;
    if (ntask <= 0) return hipSuccess;
    if (maxt <= 1) {
        dim3 grid((unsigned)ntask, (unsigned)((nrhs + SV_COLS - 1) / SV_COLS));
        if (bwd) hipLaunchKernelGGL((vdiag_kernel<T2, true>), grid, dim3(256), 0, s, tasks, b, vb, D, nrhs);
        else hipLaunchKernelGGL((vdiag_kernel<T2, false>), grid, dim3(256), 0, s, tasks, b, vb, D, nrhs);
    } else {
        dim3 grid((unsigned)ntask, (unsigned)((nrhs + 31) / 32));
        if (bwd) hipLaunchKernelGGL((vdiag_multi_kernel<T2, true>), grid, dim3(256), 0, s, tasks, b, vb, D, nrhs);
        else hipLaunchKernelGGL((vdiag_multi_kernel<T2, false>), grid, dim3(256), 0, s, tasks, b, vb, D, nrhs);
    }
    return hipGetLastError();
}
template <typename T>
hipError_t launch_vupd(const VUpdTask *tasks, const int64_t *fuse, int64_t ntask, const VUpdPair *pairs,
                       const VDiagTask *vdiag, int mode, const Bases &b, const VBases &vb, const DArrays &D, int nrhs,
                       hipStream_t s) {
    using T2 = typename C2T<T>::type;
    if (ntask <= 0) return hipSuccess;
    dim3 grid((unsigned)ntask, (unsigned)((nrhs + SV_COLS - 1) / SV_COLS));
    if (mode == 0)
        hipLaunchKernelGGL((vupd_kernel<T2, 0>), grid, dim3(256), 0, s, tasks, fuse, pairs, vdiag, b, vb, D, nrhs);
    else if (mode == 1)
        hipLaunchKernelGGL((vupd_kernel<T2, 1>), grid, dim3(256), 0, s, tasks, fuse, pairs, vdiag, b, vb, D, nrhs);
    else
        hipLaunchKernelGGL((vupd_kernel<T2, 2>), grid, dim3(256), 0, s, tasks, fuse, pairs, vdiag, b, vb, D, nrhs);
    return hipGetLastError();
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

hipError_t launch_residual(double2 *r, const double2 *f, const double2 *E, const int64_t *rowptr, const int32_t *col,
                           const double2 *val, int64_t ne, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(residual_kernel, g1(ne), dim3(256), 0, s, r, f, E, rowptr, col, val, ne, nrhs);
    return hipGetLastError();
}
hipError_t launch_rownorm_max(unsigned long long *out, const double2 *v, int64_t ne, int nrhs, hipStream_t s) {
    int64_t blocks = (ne + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(rownorm_max_kernel, dim3((unsigned)blocks, (unsigned)nrhs), dim3(256), 0, s, out, v, ne, nrhs);
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
    template hipError_t launch_vsplit<T>(void *, const double2 *, const int64_t *, int64_t, int, int64_t,          \
                                         hipStream_t);                                                            \
    template hipError_t launch_vdiag<T>(const VDiagTask *, int64_t, int, bool, const Bases &, const VBases &,           \
                                        const DArrays &, int, hipStream_t);                                       \
    template hipError_t launch_vupd<T>(const VUpdTask *, const int64_t *, int64_t, const VUpdPair *,            \
                                       const VDiagTask *, int, const Bases &, const VBases &, const DArrays &, int, \
                                       hipStream_t);                                         \
    template hipError_t launch_vgather_h<T>(void *, const void *, const int64_t *, int64_t, int, hipStream_t);     \
    template hipError_t launch_vscatter_lam<T>(void *, const void *, const int64_t *, int64_t, int, hipStream_t);  \
    template hipError_t launch_vcollect<T>(double2 *, const void *, const int64_t *, int64_t, int, bool,           \
                                           hipStream_t);
D3M_INST(double)
D3M_INST(float)
#undef D3M_INST

}  // namespace d3m
