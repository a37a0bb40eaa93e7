"""Lowest-order Nedelec (Whitney) FEM of the BVP in Section II -- oracle.

BVP (Section II, first two lines of the decomposed problem, mu_r = 1):

    curl curl E - k^2 eps_r E = -jk eta J_imp           in the cube
    n x curl E - jk E_t = n x curl E_inc - jk E_inc,t   on its boundary
    n x E = 0                                           on PEC surfaces

PEC surfaces are given as mesh triangles; every edge of such a triangle has
a zero tangential field and is eliminated (its row and column leave the
system, E = 0 there).  The impressed current is a point dipole J_imp =
m delta(r - r0) (current moment m = I l, in A m), whose load on edge e is
-jk eta m . N_e(r0), with eta the free-space impedance.

Time convention e^{+j omega t}; the incident plane wave is
E_inc = p exp(-jk d.r).  Multiplying by a test function v, integrating by
parts (int v . curl curl E = int curl v . curl E + oint v . (n x curl E)) and
inserting the boundary condition gives S u = f with

    S = Kc - k^2 M(eps_r) + jk T_abc,
    f = - oint N . g_inc dS,   g_inc = n x curl E_inc - jk E_inc,t .

Whitney basis of the edge (i, j) (local vertices i < j in global-id order,
so the edge points from the lower to the higher global vertex id):
N_ij = l_i G_j - l_j G_i with l the barycentrics and G = grad l;
curl N_ij = 2 G_i x G_j.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .quad import triangle_rule

ETA0 = 376.730313668  # free-space wave impedance, ohm (CODATA 2018)

TET_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
TET_FACES = [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)]
TET_FACE_OPP = [3, 2, 1, 0]
TRI_EDGES = [(0, 1), (0, 2), (1, 2)]


class Topology:
    """Edges, faces and their incidences of a tetrahedral mesh.

    Global edges are the sorted unique vertex pairs (lo, hi); ``tet_edges``
    [n_t, 6] gives the global edge of each local edge in TET_EDGES order.
    Faces are sorted unique vertex triples; ``face_tets`` lists the one or two
    tetrahedra of each face.
    """

    def __init__(self, xyz, tets):
        # local vertices in increasing global id: every local edge then points
        # from the lower to the higher global vertex, as the global edge does
        tets = np.sort(np.asarray(tets, dtype=np.int64), axis=1)
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.tets = tets
        nv = self.xyz.shape[0]
        self.n_vertices = nv
        a = np.stack([tets[:, i] for i, _ in TET_EDGES], axis=1)
        b = np.stack([tets[:, j] for _, j in TET_EDGES], axis=1)
        key = a * nv + b
        ukey, inv = np.unique(key.ravel(), return_inverse=True)
        self.edges = np.stack([ukey // nv, ukey % nv], axis=1)
        self.tet_edges = inv.reshape(-1, 6)
        self.n_edges = self.edges.shape[0]

        fk = []
        for f in TET_FACES:
            fk.append((tets[:, f[0]] * nv + tets[:, f[1]]) * nv + tets[:, f[2]])
        fk = np.stack(fk, axis=1).ravel()
        ufk, finv, cnt = np.unique(fk, return_inverse=True, return_counts=True)
        self.faces = np.stack([ufk // (nv * nv), (ufk // nv) % nv, ufk % nv], axis=1)
        self.n_faces = self.faces.shape[0]
        if np.any(cnt > 2):
            raise ValueError("non-manifold mesh")
        order = np.argsort(finv, kind="stable")
        ft = np.full((self.n_faces, 2), -1, dtype=np.int64)
        fl = np.full((self.n_faces, 2), -1, dtype=np.int64)
        starts = np.concatenate([[0], np.cumsum(cnt)[:-1]])
        for slot in range(2):
            has = cnt > slot
            idx = order[starts[has] + slot]
            ft[has, slot] = idx // 4
            fl[has, slot] = idx % 4
        self.face_tets = ft
        self.face_local = fl
        self.face_count = cnt
        # global edges of each face in TRI_EDGES order
        e = self.edges
        lookup = e[:, 0] * nv + e[:, 1]
        fa, fb, fc = self.faces[:, 0], self.faces[:, 1], self.faces[:, 2]
        fe = np.stack([np.searchsorted(lookup, fa * nv + fb),
                       np.searchsorted(lookup, fa * nv + fc),
                       np.searchsorted(lookup, fb * nv + fc)], axis=1)
        self.face_edges = fe

    def boundary_faces(self):
        return np.nonzero(self.face_count == 1)[0]


def tet_geometry(xyz, tets):
    """Barycentric gradients G [n_t, 4, 3] and volumes V [n_t]."""
    x = xyz[tets]  # [n_t, 4, 3]
    mx = x[:, 1:, :] - x[:, :1, :]  # rows x_i - x_0
    det = np.linalg.det(mx)
    inv = np.linalg.inv(mx)  # columns are grad of l_1..l_3
    g = np.empty((tets.shape[0], 4, 3))
    g[:, 1:, :] = np.transpose(inv, (0, 2, 1))
    g[:, 0, :] = -g[:, 1:, :].sum(axis=1)
    return g, np.abs(det) / 6.0


def curl_matrices(G, V):
    """Kc[a, b] = V (curl N_a) . (curl N_b), curl N_ij = 2 G_i x G_j."""
    c = np.stack([2.0 * np.cross(G[:, i], G[:, j]) for i, j in TET_EDGES], axis=1)
    return V[:, None, None] * np.einsum("tax,tbx->tab", c, c)


def _whitney_mass(G, meas, denom):
    """int N_a . N_b for N_ij = l_i g_j - l_j g_i on simplices whose moments
    are int l_p l_q = meas (1 + delta_pq) / denom."""
    nt = G.shape[0]
    nl = G.shape[1]
    edges = TET_EDGES if nl == 4 else TRI_EDGES
    dots = np.einsum("tpx,tqx->tpq", G, G)
    eye = np.eye(nl)
    I = meas[:, None, None] * (1.0 + eye)[None] / denom
    m = len(edges)
    M = np.empty((nt, m, m))
    for a, (i, j) in enumerate(edges):
        for b, (k, l) in enumerate(edges):
            M[:, a, b] = (dots[:, j, l] * I[:, i, k] - dots[:, j, k] * I[:, i, l]
                          - dots[:, i, l] * I[:, j, k] + dots[:, i, k] * I[:, j, l])
    return M


def mass_matrices(G, V):
    """Unit-eps_r element mass M[a,b] = int N_a . N_b (int l_p l_q = V(1+d_pq)/20)."""
    return _whitney_mass(G, V, 20.0)


def triangle_geometry(xyz, tri):
    """In-plane barycentric gradients g [n_f, 3, 3], areas A [n_f], unit normals."""
    y = xyz[tri]
    e1 = y[:, 1] - y[:, 0]
    e2 = y[:, 2] - y[:, 0]
    a11 = np.einsum("fx,fx->f", e1, e1)
    a12 = np.einsum("fx,fx->f", e1, e2)
    a22 = np.einsum("fx,fx->f", e2, e2)
    det = a11 * a22 - a12 * a12
    g1 = (a22[:, None] * e1 - a12[:, None] * e2) / det[:, None]
    g2 = (a11[:, None] * e2 - a12[:, None] * e1) / det[:, None]
    g = np.stack([-(g1 + g2), g1, g2], axis=1)
    nrm = np.cross(e1, e2)
    area = 0.5 * np.linalg.norm(nrm, axis=1)
    return g, area, nrm / (2.0 * area[:, None])


def tangential_mass(g, area):
    """T[a, b] = int_t N_a . N_b dS (int l_p l_q = A(1+d_pq)/12)."""
    return _whitney_mass(g, area, 12.0)


def outward_normals(topo: Topology, faces_idx):
    """Unit normals of boundary faces pointing away from their tetrahedron."""
    tri = topo.faces[faces_idx]
    _, _, nrm = triangle_geometry(topo.xyz, tri)
    t = topo.face_tets[faces_idx, 0]
    opp = topo.tets[t, np.asarray(TET_FACE_OPP)[topo.face_local[faces_idx, 0]]]
    inward = topo.xyz[opp] - topo.xyz[tri[:, 0]]
    flip = np.einsum("fx,fx->f", nrm, inward) > 0
    nrm[flip] *= -1.0
    return nrm


def planewave_face_load(xyz, tri, normals, k, d, p, q=12):
    """f_(i,j) contribution - int_t (l_i g_j - l_j g_i) . g_inc dS for each
    boundary face, g_inc = n x curl E_inc - jk E_inc,t,
    curl E_inc = -jk (d x p) exp(-jk d.r).  Returns [n_f, 3] (TRI_EDGES order).
    """
    g, area, _ = triangle_geometry(xyz, tri)
    n = normals
    dxp = np.cross(d, p)
    cvec = -1j * k * (np.cross(n, np.broadcast_to(dxp, n.shape))
                      + p[None, :] - n * (n @ p)[:, None])  # [n_f, 3]
    s, t, w = triangle_rule(q)
    y = xyz[tri]
    pts = (y[:, None, 0, :] * (1.0 - s - t)[None, :, None]
           + y[:, None, 1, :] * s[None, :, None]
           + y[:, None, 2, :] * t[None, :, None])  # [n_f, nq, 3]
    phase = np.exp(-1j * k * (pts @ d))  # [n_f, nq]
    lam = np.stack([1.0 - s - t, s, t], axis=0)  # [3, nq]
    J = 2.0 * area[:, None] * np.einsum("q,lq,fq->fl", w, lam, phase)  # int l_i phi
    gc = np.einsum("flx,fx->fl", g, cvec)  # g_l . cvec
    out = np.empty((tri.shape[0], 3), dtype=np.complex128)
    for a, (i, j) in enumerate(TRI_EDGES):
        out[:, a] = -(gc[:, j] * J[:, i] - gc[:, i] * J[:, j])
    return out


def edge_interpolant(xyz, edges, k, d, p):
    """DOFs int_edge E_inc . dl of the plane wave (lower -> higher vertex id)."""
    va = xyz[edges[:, 0]]
    vb = xyz[edges[:, 1]]
    dl = vb - va
    z = -1j * k * (dl @ d)
    small = np.abs(z) < 1e-8
    phi = np.where(small, 1.0 + z / 2.0, (np.exp(z) - 1.0) / np.where(small, 1.0, z))
    return (dl @ p) * np.exp(-1j * k * (va @ d)) * phi


class GlobalFEM:
    """Undecomposed FEM system S (CSR, complex symmetric), plane-wave and
    dipole loads.  ``S`` holds every edge; the unknowns are the edges not on
    a PEC triangle (``free``), and the system is S[free, free]."""

    def __init__(self, xyz, tets, eps_r, k, pec_faces=None):
        self.topo = Topology(xyz, tets)
        t = self.topo
        self.pec = np.zeros(t.n_edges, dtype=bool)
        if pec_faces is not None and len(pec_faces):
            nv = t.n_vertices
            fk = np.sort(np.asarray(pec_faces, dtype=np.int64), axis=1)
            keys = (fk[:, 0] * nv + fk[:, 1]) * nv + fk[:, 2]
            have = (t.faces[:, 0] * nv + t.faces[:, 1]) * nv + t.faces[:, 2]
            order = np.argsort(have)
            pos = np.searchsorted(have[order], keys)
            pos = np.minimum(pos, have.size - 1)
            if np.any(have[order][pos] != keys):
                raise ValueError("a PEC triangle is not a face of the mesh")
            self.pec[t.face_edges[order[pos]].ravel()] = True
        self.free = np.nonzero(~self.pec)[0]
        self.k = float(k)
        self.eps_r = np.asarray(eps_r, dtype=np.float64)
        self.G, self.V = tet_geometry(t.xyz, t.tets)
        if np.any(self.V <= 0):
            raise ValueError("degenerate tetrahedron")
        self.Kc = curl_matrices(self.G, self.V)
        self.M = mass_matrices(self.G, self.V)
        self.Se = self.Kc - (self.k ** 2) * self.eps_r[:, None, None] * self.M
        self.bfaces = t.boundary_faces()
        g, area, _ = triangle_geometry(t.xyz, t.faces[self.bfaces])
        self.Tb = tangential_mass(g, area)
        self.bnormals = outward_normals(t, self.bfaces)
        self.S = self._assemble()

    def _assemble(self):
        t = self.topo
        te = t.tet_edges
        rows = np.repeat(te, 6, axis=1).ravel()
        cols = np.tile(te, (1, 6)).ravel()
        vals = self.Se.astype(np.complex128).ravel()
        fe = t.face_edges[self.bfaces]
        r2 = np.repeat(fe, 3, axis=1).ravel()
        c2 = np.tile(fe, (1, 3)).ravel()
        v2 = (1j * self.k * self.Tb).ravel()
        n = t.n_edges
        S = sp.coo_matrix((np.concatenate([vals, v2]),
                           (np.concatenate([rows, r2]), np.concatenate([cols, c2]))),
                          shape=(n, n)).tocsr()
        S.sum_duplicates()
        return S

    def planewave_rhs(self, dirs, pols, q=12):
        """f [nrhs, n_edges] for plane waves (rows = right-hand sides)."""
        t = self.topo
        dirs = np.atleast_2d(dirs)
        pols = np.atleast_2d(pols)
        f = np.zeros((dirs.shape[0], t.n_edges), dtype=np.complex128)
        fe = t.face_edges[self.bfaces]
        for r in range(dirs.shape[0]):
            loc = planewave_face_load(t.xyz, t.faces[self.bfaces], self.bnormals,
                                      self.k, dirs[r], pols[r], q)
            np.add.at(f[r], fe.ravel(), loc.ravel())
        f[:, self.pec] = 0.0
        return f

    def dipole_rhs(self, pos, moment):
        """f [nrhs, n_edges] for point dipoles J_imp = m delta(r - r0), one per
        right-hand side: f_e = -jk eta m . N_e(r0) (zero on PEC edges)."""
        pos = np.atleast_2d(pos)
        moment = np.atleast_2d(np.asarray(moment, dtype=np.complex128))
        P = probe_matrix(self.topo, pos)  # [nrhs, 3, n_edges]
        f = -1j * self.k * ETA0 * np.einsum("rx,rxe->re", moment, P)
        f[:, self.pec] = 0.0
        return f

    def system(self):
        """S restricted to the unknowns (rows and columns of non-PEC edges)."""
        return self.S[self.free][:, self.free]

    def relative_residual(self, E, f):
        """max over right-hand sides of ||(S E - f)[free]||_inf / ||f[free]||_inf."""
        E = np.atleast_2d(E)
        f = np.atleast_2d(f)
        r = (self.system() @ E[:, self.free].T).T - f[:, self.free]
        return float(np.max(np.abs(r).max(axis=1) / np.abs(f[:, self.free]).max(axis=1)))

    def unit_mass(self):
        """Per-tetrahedron unit-eps_r mass matrices (for dS/d eps_r = -k^2 M)."""
        return self.M


def probe_matrix(topo: Topology, points):
    """Field evaluation E(r_m) = sum_a u_a N_a(r_m) as a dense real matrix
    P [n_points, 3, n_edges] (point location by barycentric coordinates)."""
    G, V = tet_geometry(topo.xyz, topo.tets)
    x0 = topo.xyz[topo.tets[:, 0]]
    P = np.zeros((len(points), 3, topo.n_edges))
    for m, r in enumerate(np.atleast_2d(points)):
        lam = np.empty((topo.tets.shape[0], 4))
        lam[:, 1:] = np.einsum("tix,tx->ti", G[:, 1:], r[None, :] - x0)
        lam[:, 0] = 1.0 - lam[:, 1:].sum(axis=1)
        t = int(np.argmax(lam.min(axis=1)))
        if lam[t].min() < -1e-12:
            raise ValueError(f"point {r} outside the mesh")
        for a, (i, j) in enumerate(TET_EDGES):
            P[m, :, topo.tet_edges[t, a]] += lam[t, i] * G[t, j] - lam[t, j] * G[t, i]
    return P
