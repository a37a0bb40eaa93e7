// Mesh topology and Whitney element matrices of the BVP in Section II
// (curl-curl operator, eps_r mass, first-order absorbing boundary and its
// plane-wave load).  Time convention e^{+j omega t}.
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

#include "problem.hpp"

namespace d3m {

namespace {

const int kTetEdge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
const int kTetFace[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
const int kTriEdge[3][2] = {{0, 1}, {0, 2}, {1, 2}};

inline void sub3(const double *a, const double *b, double *c) {
    c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2];
}
inline double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
inline void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

i64 edge_index(const Mesh &m, i64 a, i64 b) {
    // edges are sorted lexicographically by (lo, hi)
    i64 lo = 0, hi = m.ne;
    while (lo < hi) {
        i64 mid = (lo + hi) / 2;
        i64 x = m.edges[2 * mid], y = m.edges[2 * mid + 1];
        if (x < a || (x == a && y < b)) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// In-plane barycentric gradients and area of a triangle.
void tri_grads(const double *y0, const double *y1, const double *y2,
               double g[3][3], double &area, double nrm[3]) {
    double e1[3], e2[3];
    sub3(y1, y0, e1);
    sub3(y2, y0, e2);
    double a11 = dot3(e1, e1), a12 = dot3(e1, e2), a22 = dot3(e2, e2);
    double det = a11 * a22 - a12 * a12;
    for (int x = 0; x < 3; ++x) {
        g[1][x] = (a22 * e1[x] - a12 * e2[x]) / det;
        g[2][x] = (a11 * e2[x] - a12 * e1[x]) / det;
        g[0][x] = -(g[1][x] + g[2][x]);
    }
    cross3(e1, e2, nrm);
    double len = std::sqrt(dot3(nrm, nrm));
    area = 0.5 * len;
    for (int x = 0; x < 3; ++x) nrm[x] /= len;
}

// int_T N_a . N_b for N_ij = l_i g_j - l_j g_i, moments int l_p l_q = meas(1+d)/den
template <int NV, int NE>
void whitney_mass(const double g[NV][3], double meas, double den,
                  const int (*edges)[2], double *out) {
    double dots[NV][NV];
    for (int p = 0; p < NV; ++p)
        for (int q = 0; q < NV; ++q) dots[p][q] = dot3(g[p], g[q]);
    auto I = [&](int p, int q) { return meas * (p == q ? 2.0 : 1.0) / den; };
    for (int a = 0; a < NE; ++a) {
        int i = edges[a][0], j = edges[a][1];
        for (int b = 0; b < NE; ++b) {
            int k = edges[b][0], l = edges[b][1];
            out[a * NE + b] = dots[j][l] * I(i, k) - dots[j][k] * I(i, l) -
                              dots[i][l] * I(j, k) + dots[i][k] * I(j, l);
        }
    }
}

}  // namespace

void build_mesh(Mesh &m, i64 nv, const double *xyz, i64 nt, const i64 *tets) {
    if (nv <= 0 || nt <= 0) throw Error{-1, "empty mesh"};
    m.nv = nv;
    m.nt = nt;
    m.xyz.assign(xyz, xyz + 3 * nv);
    m.tets.resize(4 * nt);
    for (i64 t = 0; t < nt; ++t) {
        std::array<i64, 4> v{tets[4 * t], tets[4 * t + 1], tets[4 * t + 2], tets[4 * t + 3]};
        for (i64 x : v)
            if (x < 0 || x >= nv) throw Error{-1, "tetrahedron vertex id out of range"};
        std::sort(v.begin(), v.end());
        if (v[0] == v[1] || v[1] == v[2] || v[2] == v[3])
            throw Error{-1, "tetrahedron with repeated vertex"};
        for (int a = 0; a < 4; ++a) m.tets[4 * t + a] = v[a];
    }
    // edges
    std::vector<std::array<i64, 3>> ek(6 * nt);
    for (i64 t = 0; t < nt; ++t)
        for (int a = 0; a < 6; ++a)
            ek[6 * t + a] = {m.tets[4 * t + kTetEdge[a][0]], m.tets[4 * t + kTetEdge[a][1]], 6 * t + a};
    std::sort(ek.begin(), ek.end());
    m.tet_edges.assign(6 * nt, -1);
    m.edges.clear();
    for (size_t i = 0; i < ek.size(); ++i) {
        if (i == 0 || ek[i][0] != ek[i - 1][0] || ek[i][1] != ek[i - 1][1]) {
            m.edges.push_back(ek[i][0]);
            m.edges.push_back(ek[i][1]);
        }
        m.tet_edges[ek[i][2]] = (i64)m.edges.size() / 2 - 1;
    }
    m.ne = (i64)m.edges.size() / 2;
    // faces
    std::vector<std::array<i64, 4>> fk(4 * nt);
    for (i64 t = 0; t < nt; ++t)
        for (int f = 0; f < 4; ++f)
            fk[4 * t + f] = {m.tets[4 * t + kTetFace[f][0]], m.tets[4 * t + kTetFace[f][1]],
                             m.tets[4 * t + kTetFace[f][2]], 4 * t + f};
    std::sort(fk.begin(), fk.end());
    m.faces.clear();
    m.face_tet.clear();
    m.face_loc.clear();
    for (size_t i = 0; i < fk.size();) {
        size_t j = i;
        while (j < fk.size() && fk[j][0] == fk[i][0] && fk[j][1] == fk[i][1] && fk[j][2] == fk[i][2]) ++j;
        if (j - i > 2) throw Error{-1, "non-manifold mesh: a face shared by more than two tetrahedra"};
        m.faces.insert(m.faces.end(), {fk[i][0], fk[i][1], fk[i][2]});
        m.face_tet.push_back(fk[i][3] / 4);
        m.face_loc.push_back((int8_t)(fk[i][3] % 4));
        if (j - i == 2) {
            m.face_tet.push_back(fk[i + 1][3] / 4);
            m.face_loc.push_back((int8_t)(fk[i + 1][3] % 4));
        } else {
            m.face_tet.push_back(-1);
            m.face_loc.push_back(-1);
        }
        i = j;
    }
    m.nf = (i64)m.faces.size() / 3;
    m.face_edges.resize(3 * m.nf);
    for (i64 f = 0; f < m.nf; ++f)
        for (int a = 0; a < 3; ++a)
            m.face_edges[3 * f + a] = edge_index(m, m.faces[3 * f + kTriEdge[a][0]], m.faces[3 * f + kTriEdge[a][1]]);
    // geometry: gradients of the barycentrics and volumes
    m.volume.resize(nt);
    m.grads.resize(12 * nt);
    for (i64 t = 0; t < nt; ++t) {
        const double *x0 = &m.xyz[3 * m.tets[4 * t]];
        double r[3][3];
        for (int a = 0; a < 3; ++a) sub3(&m.xyz[3 * m.tets[4 * t + a + 1]], x0, r[a]);
        // rows r_a = x_{a+1} - x_0; grad l_{a+1} = (r_b x r_c) / det (cyclic)
        double c[3][3];
        cross3(r[1], r[2], c[0]);
        cross3(r[2], r[0], c[1]);
        cross3(r[0], r[1], c[2]);
        double det = dot3(r[0], c[0]);
        if (!(std::fabs(det) > 0.0)) throw Error{-1, "degenerate tetrahedron"};
        m.volume[t] = std::fabs(det) / 6.0;
        double *g = &m.grads[12 * t];
        for (int a = 0; a < 3; ++a)
            for (int x = 0; x < 3; ++x) g[3 * (a + 1) + x] = c[a][x] / det;
        for (int x = 0; x < 3; ++x) g[x] = -(g[3 + x] + g[6 + x] + g[9 + x]);
    }
}

void tet_curl_mass(const Mesh &m, i64 t, double Kc[36], double M[36]) {
    double g[4][3];
    for (int a = 0; a < 4; ++a)
        for (int x = 0; x < 3; ++x) g[a][x] = m.grads[12 * t + 3 * a + x];
    double V = m.volume[t];
    double curl[6][3];
    for (int a = 0; a < 6; ++a) {
        cross3(g[kTetEdge[a][0]], g[kTetEdge[a][1]], curl[a]);
        for (int x = 0; x < 3; ++x) curl[a][x] *= 2.0;
    }
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) Kc[6 * a + b] = V * dot3(curl[a], curl[b]);
    whitney_mass<4, 6>(g, V, 20.0, kTetEdge, M);
}

void tri_tangential_mass(const Mesh &m, i64 f, double T[9]) {
    double g[3][3], area, nrm[3];
    tri_grads(&m.xyz[3 * m.faces[3 * f]], &m.xyz[3 * m.faces[3 * f + 1]],
              &m.xyz[3 * m.faces[3 * f + 2]], g, area, nrm);
    whitney_mass<3, 3>(g, area, 12.0, kTriEdge, T);
}

void face_outward_normal(const Mesh &m, i64 f, double n[3]) {
    double g[3][3], area;
    const double *y0 = &m.xyz[3 * m.faces[3 * f]];
    tri_grads(y0, &m.xyz[3 * m.faces[3 * f + 1]], &m.xyz[3 * m.faces[3 * f + 2]], g, area, n);
    i64 t = m.face_tet[2 * f];
    int lf = m.face_loc[2 * f];
    i64 opp = m.tets[4 * t + (3 - lf)];
    double in[3];
    sub3(&m.xyz[3 * opp], y0, in);
    if (dot3(n, in) > 0)
        for (int x = 0; x < 3; ++x) n[x] = -n[x];
}

// Gauss-Legendre nodes on [-1, 1] by Newton's method on P_q (three-term
// recurrence), mapped to [0, 1]; collapsed onto the triangle by
// s = u, t = (1 - u) v with Jacobian (1 - u).
void triangle_rule(int q, std::vector<double> &s, std::vector<double> &t, std::vector<double> &w) {
    std::vector<double> x(q), wx(q);
    for (int i = 0; i < q; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_q(z), p0 = P_{q-1}(z); P_q' = q (z P_q - P_{q-1}) / (z^2 - 1)
            double dp = q * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                p0 = 1.0; p1 = z;
                for (int k = 2; k <= q; ++k) {
                    double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1; p1 = p2;
                }
                dp = q * (z * p1 - p0) / (z * z - 1.0);
                break;
            }
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= q; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1; p1 = p2;
        }
        double dp = q * (z * p1 - p0) / (z * z - 1.0);
        x[i] = 0.5 * (z + 1.0);
        wx[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // (2/((1-z^2)P'^2)) * 1/2
    }
    s.clear(); t.clear(); w.clear();
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
            s.push_back(x[i]);
            t.push_back((1.0 - x[i]) * x[j]);
            w.push_back(wx[i] * wx[j] * (1.0 - x[i]));
        }
}

// f contribution -int_t (l_i g_j - l_j g_i) . g_inc dS with
// g_inc = n x curl E_inc - jk E_inc,t = c exp(-jk d.r),
// c = -jk [n x (d x p) + p - n (n.p)].
void face_planewave_load(const Mesh &m, i64 f, double k, const double d[3],
                         const double p[3], const std::vector<double> &qs,
                         const std::vector<double> &qt,
                         const std::vector<double> &qw, cplx out[3]) {
    const double *y[3] = {&m.xyz[3 * m.faces[3 * f]], &m.xyz[3 * m.faces[3 * f + 1]],
                          &m.xyz[3 * m.faces[3 * f + 2]]};
    double g[3][3], area, nrm[3];
    tri_grads(y[0], y[1], y[2], g, area, nrm);
    double n[3];
    face_outward_normal(m, f, n);
    double dxp[3], nx[3];
    cross3(d, p, dxp);
    cross3(n, dxp, nx);
    double np = dot3(n, p);
    const cplx jk(0.0, k);
    cplx c[3];
    for (int x = 0; x < 3; ++x) c[x] = -jk * (nx[x] + p[x] - n[x] * np);
    cplx J[3] = {0.0, 0.0, 0.0};  // int l_i exp(-jk d.r)
    for (size_t q = 0; q < qw.size(); ++q) {
        double l[3] = {1.0 - qs[q] - qt[q], qs[q], qt[q]};
        double r[3];
        for (int x = 0; x < 3; ++x) r[x] = l[0] * y[0][x] + l[1] * y[1][x] + l[2] * y[2][x];
        cplx ph = std::exp(cplx(0.0, -k * dot3(d, r)));
        for (int i = 0; i < 3; ++i) J[i] += qw[q] * l[i] * ph;
    }
    for (int i = 0; i < 3; ++i) J[i] *= 2.0 * area;
    cplx gc[3];
    for (int i = 0; i < 3; ++i) gc[i] = g[i][0] * c[0] + g[i][1] * c[1] + g[i][2] * c[2];
    for (int a = 0; a < 3; ++a) {
        int i = kTriEdge[a][0], j = kTriEdge[a][1];
        out[a] = -(gc[j] * J[i] - gc[i] * J[j]);
    }
}

void mark_pec(Mesh &m, i64 nfaces, const i64 *faces) {
    m.pec.assign(m.ne, 0);
    m.n_pec = 0;
    for (i64 f = 0; f < nfaces; ++f) {
        std::array<i64, 3> v{faces[3 * f], faces[3 * f + 1], faces[3 * f + 2]};
        std::sort(v.begin(), v.end());
        // faces are stored in increasing (v0, v1, v2) order
        i64 lo = 0, hi = m.nf;
        while (lo < hi) {
            const i64 mid = (lo + hi) / 2;
            const std::array<i64, 3> w{m.faces[3 * mid], m.faces[3 * mid + 1], m.faces[3 * mid + 2]};
            if (w < v) lo = mid + 1; else hi = mid;
        }
        if (lo >= m.nf || m.faces[3 * lo] != v[0] || m.faces[3 * lo + 1] != v[1] || m.faces[3 * lo + 2] != v[2])
            throw Error{-1, "PEC triangle " + std::to_string(f) + " is not a face of the mesh"};
        for (int a = 0; a < 3; ++a) m.pec[m.face_edges[3 * lo + a]] = 1;
    }
    for (i64 e = 0; e < m.ne; ++e) m.n_pec += m.pec[e];
}

}  // namespace d3m
