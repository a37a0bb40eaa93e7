// Task descriptors shared by the host planner and the HIP kernels.
//
// Every dense object is stored as 64 x 64 complex tiles (column-major inside
// a tile, interleaved re/im).  A tile is addressed by an "encoded offset":
// the array id in the top 8 bits and the element offset inside that array in
// the low 56 bits, so one task list serves the FP64 and the FP32 buffers.
#pragma once
#include <cstdint>

namespace d3m {

enum Arr : int {
    ARR_M = 0,   // subdomain augmented matrices [A_d D_d; D_d^T 0] (factored in place)
    ARR_MX = 1,  // panel products X = M P L^-T of the subdomain steps
    ARR_K = 2,   // LM Schur complement (-K) working tiles
    ARR_KX = 3,  // panel products of the K blocks
    ARR_KL = 4,  // factor tiles of -K (unit lower L_jj and L_ij)
    ARR_TT = 5,  // L_jj^{-1} P_j^T of every diagonal block
    ARR_KU = 6,  // update matrices of the multifrontal form of step 5
    ARR_COUNT = 7
};

constexpr int64_t TILE_ELEMS_D = 4096;  // complex elements of a 64 x 64 tile
constexpr int ENC_SHIFT = 56;
constexpr int64_t ENC_MASK = (int64_t(1) << ENC_SHIFT) - 1;
inline constexpr int64_t enc(int arr, int64_t off) { return (int64_t(arr) << ENC_SHIFT) | off; }

struct Bases {
    void *p[ARR_COUNT];
};

// C (=|-=) sum_p A_p B_p^T over 64 x 64 tiles
struct GemmTask {
    int64_t c;
    int32_t p0, np;
};
struct GemmPair {
    int64_t a, b;
};

// Bunch-Kaufman factorisation of one diagonal block (pivoting restricted to
// the block), its L, D, D^{-1}, perm and TT = L^{-1} P^T
struct BkTask {
    int64_t a;     // tile (0,0) of the block in the working array
    int64_t l;     // tile (0,0) of the L output (same tile layout)
    int64_t tt;    // TT tiles, tile (b,c) at tt + (c*t + b) * 4096
    int64_t drow;  // first row in the D arrays
    int32_t n;     // block order
    int32_t ldt;   // element stride between column tiles of the block
    int32_t status;
    int32_t np;    // pending updates A -= X W^T applied to the block first:
    int32_t p0;    //   pairs (X, W) p0 .. p0 + np - 1 of the pair list (one-tile blocks)
    int32_t pad;
};

// W = X D^{-1} for one tile (2x2 pivots may pair the first/last column with
// the neighbouring column tile)
struct ScaleTask {
    int64_t x, w;          // X tile, output tile
    int64_t xprev, xnext;  // neighbouring X tiles in the same tile row (-1: none)
    int64_t drow;          // D-array row of column 0 of this tile
    int32_t ncols;
    int32_t nq;            // pending updates of the panel's input tile (fused panel only):
    int32_t q0, pad;       //   pairs (X, W) q0 .. q0 + nq - 1, applied before the product
};

// Extend-add of the multifrontal form: dst (= or +=) the sum of source
// tiles srcs[s0 .. s0 + ns - 1] (encoded tile offsets).  A child's update
// matrix tile and its place in the parent's front cover the same rows and
// columns, so whole tiles are added.
struct AddTask {
    int64_t dst;
    int32_t s0, ns;
    int32_t accumulate;  // 1: dst += sum, 0: dst = sum (zero when ns == 0)
    int32_t pad;
};

// Assembly of one tile of the LM Schur complement from <= 2 subdomains
struct AsmTask {
    int64_t dst;
    int32_t nrow, ncol, ncontrib, pad;
    int64_t mbase[2];  // tile slot (ARR_M) of the subdomain's trailing multiplier triangle
    int32_t row0[2], col0[2];  // first row / column inside that triangle
};

// One tile of a factor's off-diagonal block L-hat_ij = X_ij D_jj^{-1}: its
// valid rows and columns (the growth monitor reads these entries only)
struct FactorTile {
    int64_t tile;
    int32_t rows, cols;
};

// element offset of tile (a, b), a >= b, inside a packed lower tile triangle
inline int64_t tri_slot(int64_t a, int64_t b) { return a * (a + 1) / 2 + b; }

// ---- solve sweeps ---------------------------------------------------------
// Vector tiles hold 64 rows x nrhs columns (column = right-hand side); a
// vector tile index v addresses element v*64*nrhs.  Encoded like matrix
// tiles, with vector array ids:
enum VArr : int { V_X = 0, V_Y = 1, V_V = 2, V_ACC = 3, V_KX = 4, V_KY = 5, V_KV = 6, V_KACC = 7, VARR_COUNT = 8 };

struct VDiagTask {   // y = TT x and v = D^{-1} y   (forward)  or
    int64_t tt;      // x = TT^T (v - acc)           (backward)
    int64_t x, y, v, acc;  // encoded first vector tile of the block (acc -1: zero)
    int64_t drow;
    int32_t t, n;
};
struct VUpdTask {    // out (=|-=|+=) sum_p op(L_p) src_p
    int64_t out;
    int32_t p0, np;
    int64_t l0, src0;  // pair p0 again, so the first tile loads need no pair-list read
};
struct VUpdPair {
    int64_t l, src;
};

// One item of a sweep over the factor of -K run as a single launch: update
// task vupd[idx], then diagonal solve vdiag[fz] if fz >= 0 (the solve of the
// item's target tile, which this item writes last).  Before it runs, vector
// tile waits[i].tile must have received waits[i].writes completed writes (per
// column block), for i in [w0, w0 + nw); afterwards the write count of tile
// sig goes up by one.
struct ChainItem {
    int32_t idx;
    int32_t w0, nw;
    int32_t sig;
    int32_t fz, pad;
};
struct ChainWait {
    int32_t tile, writes;
};

}  // namespace d3m
