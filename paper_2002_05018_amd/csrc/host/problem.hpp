// Host-side data of one D3M problem: mesh topology, FEM element data, the
// decomposition (subdomains, Lagrange multipliers, blocks of K), the block
// ordering and symbolic structure, and the tile plans that drive the GPU
// kernels.  Everything here is plain C++ and runs without a GPU.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace d3m {

using i64 = int64_t;
using i32 = int32_t;
using cplx = std::complex<double>;

constexpr int TILE = 64;                 // tile edge (rows = columns)
constexpr i64 TILE_ELEMS = TILE * TILE;  // complex elements per tile

struct Error {
    int code;
    std::string msg;
};

// ---------------------------------------------------------------- topology --
struct Mesh {
    i64 nv = 0, nt = 0, ne = 0, nf = 0;
    std::vector<double> xyz;        // [nv][3]
    std::vector<i64> tets;          // [nt][4], vertex ids increasing
    std::vector<i64> edges;         // [ne][2] (lo, hi), lexicographic
    std::vector<i64> tet_edges;     // [nt][6] local edge order (01,02,03,12,13,23)
    std::vector<i64> faces;         // [nf][3] increasing vertex ids
    std::vector<i64> face_tet;      // [nf][2] tetrahedra (-1 = none)
    std::vector<int8_t> face_loc;   // [nf][2] local face (opposite vertex 3-f)
    std::vector<i64> face_edges;    // [nf][3] edges (01, 02, 12)
    std::vector<double> volume;     // [nt]
    std::vector<double> grads;      // [nt][4][3] barycentric gradients
    std::vector<char> pec;          // [ne] 1: edge of a PEC triangle (tangential field zero, no unknown)
    i64 n_pec = 0;
};

// Builds topology and per-tetrahedron geometry; throws Error on a degenerate
// tetrahedron or a non-manifold face.
void build_mesh(Mesh &m, i64 nv, const double *xyz, i64 nt, const i64 *tets);
// Marks the edges of the given triangles (vertex-id triples, any order) as
// PEC; throws Error when a triple is not a face of the mesh.
void mark_pec(Mesh &m, i64 nfaces, const i64 *faces);

// Element matrices (Whitney 1-forms).  Kc and M are 6x6 row-major; T is 3x3.
void tet_curl_mass(const Mesh &m, i64 t, double Kc[36], double M[36]);
void tri_tangential_mass(const Mesh &m, i64 f, double T[9]);
// Unit normal of face f pointing away from tetrahedron face_tet[f][0].
void face_outward_normal(const Mesh &m, i64 f, double n[3]);
// Plane-wave load contributions of boundary face f for the three face edges.
void face_planewave_load(const Mesh &m, i64 f, double k, const double d[3],
                         const double p[3], const std::vector<double> &qs,
                         const std::vector<double> &qt,
                         const std::vector<double> &qw, cplx out[3]);
// Collapsed Gauss-Legendre rule on the reference triangle (q^2 points).
void triangle_rule(int q, std::vector<double> &s, std::vector<double> &t,
                   std::vector<double> &w);

// ----------------------------------------------------------- decomposition --
struct Subdomain {
    i64 n = 0;       // rows of the E part (edges of the subdomain)
    i64 nI = 0;      // interior edges (in one subdomain only)
    i64 m = 0;       // LM rows (multipliers touching the subdomain)
    std::vector<i64> edges;        // [n] global edge of each row, [I | B] (s1_order 0) or
                                   // nested dissection with -1 padding rows (1)
    std::vector<i64> sorted;       // global edges sorted (lookup)
    std::vector<i32> sorted_pos;   // row of sorted[i]
    std::vector<i32> blocks;       // canonical blocks touching d, sorted
    std::vector<i64> block_off;    // LM-region row offset of each block
    // lower-triangle COO of A_d in row order (row >= col), summed
    std::vector<i64> a_row, a_col;
    std::vector<cplx> a_val;
    // pattern of the COO as contributions (for re-assembly on eps update):
    // every contribution is (coo slot, tetrahedron, local a, local b); the
    // static part (ABC and Robin terms) is kept separately.
    std::vector<i64> contrib_slot, contrib_tet;
    std::vector<int8_t> contrib_a, contrib_b;
    std::vector<cplx> a_static;    // [nnz] ABC + Robin part of each entry
    i64 row_of(i64 e) const;       // -1 if e is not in the subdomain
};

struct Decomp {
    int N = 0;
    std::vector<i32> part;               // [nt]
    std::vector<i64> sub_ptr, sub_list;  // CSR of Sub(e)
    std::vector<i32> owner;              // [ne] min Sub(e)
    std::vector<Subdomain> sub;
    std::vector<i64> iface;              // interface faces
    std::vector<i32> iface_p, iface_q;   // p < q
    std::vector<i64> bface;              // boundary faces
    // Lagrange multipliers (p, q, e), sorted; blocks = distinct (p, q)
    std::vector<i64> lm_p, lm_q, lm_e;
    std::vector<i32> blk_p, blk_q;
    std::vector<i64> blk_start;          // [nblk + 1]
    i64 n_lm = 0;
    int nblk = 0;
    int s1_order = 0;                    // row order the subdomain matrices got (0 banded, 1 dissection)
};

// s1_order: 0 rows of each subdomain [interior | interface] by global id
// (A_d banded), 1 all edge rows in nested-dissection order, 2 the
// dissection when the median subdomain has at least kNdAutoRows edge rows
// (the banded order otherwise); the order taken is kept in dc.s1_order
void build_decomposition(Decomp &dc, const Mesh &m, const i32 *part, double k,
                         cplx alpha, const double *eps, int s1_order = 0);
constexpr int kNdLeaf = 1024;  // largest region of the dissection left uncut (edges)
// subdomains of 8^3 hexes (4,184 edges) and more factor faster in the
// dissection order, those of 6^3 (1,854) in the banded one
constexpr int kNdAutoRows = 4000;
// Recompute the A_d values for new eps (same pattern).
void reassemble_values(Decomp &dc, const Mesh &m, double k, const double *eps);

// ------------------------------------------------ ordering and symbolic --
struct BlockOrder {
    std::vector<i32> order;              // canonical block at each position
    std::vector<i32> pos;                // position of each canonical block
    std::vector<std::vector<i32>> strct; // struct(j), positions, increasing
    std::vector<i32> level;              // elimination-tree level by position
    int n_levels = 0;
};

void order_blocks(BlockOrder &bo, const Decomp &dc, const Mesh &m, const std::vector<int> &sub_group);

}  // namespace d3m
