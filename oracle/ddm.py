"""The decomposed system of Section II, eq. (1) -- oracle.

Readings of the paper used here (each is listed in the design notes):

* Robin transmission (third line of the decomposed BVP) with one LM set
  (the text after eq. (1)): on an interface triangle shared by subdomains
  p < q the LM is lambda = j_p - alpha e; the neighbour sees -lambda.  Hence
  A_p gets +alpha T_t and A_q gets -alpha T_t ("loss or gain at the
  interfaces"), and the constraint columns are D_p = +1, D_q = -1 on the
  shared edge.  With these opposite signs the Robin terms cancel when the
  subdomain systems are summed, which is what makes the method exact.
* Continuity (fourth line of the BVP) on edges shared by m >= 2 subdomains:
  one LM per edge of a spanning tree of its subdomains, whose candidate
  pairs are the subdomain pairs sharing an interface triangle that contains
  the edge; Kruskal over the candidates in lexicographic order.
* LMs are the triples (p, q, e); blocks of K are the subdomain pairs (p, q)
  ("super-nodes"); LMs are numbered by (p, q, e) lexicographically, so each
  block is a contiguous range sorted by global edge id.
* The sum in eq. (1) runs over subdomains: K = sum_d D_d^T A_d^{-1} D_d and
  g = sum_d D_d^T A_d^{-1} f_d (from A E + D lambda = f, D^T E = 0).
* A global load f is split with f_d[e] = f[e] for d = min Sub(e), else 0.
* Edges on PEC triangles are not unknowns: they belong to no subdomain
  system and carry no multipliers (the continuity of a field fixed to zero
  needs no constraint).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla

from .fem import GlobalFEM, TRI_EDGES, tangential_mass, triangle_geometry


class _DSU:
    def __init__(self, items):
        self.p = {x: x for x in items}

    def find(self, x):
        while self.p[x] != x:
            self.p[x] = self.p[self.p[x]]
            x = self.p[x]
        return x

    def union(self, a, b):
        ra, rb = self.find(a), self.find(b)
        if ra == rb:
            return False
        self.p[max(ra, rb)] = min(ra, rb)
        return True


class Decomposition:
    """Subdomain systems, LM numbering and signed maps of a partitioned mesh."""

    def __init__(self, fem: GlobalFEM, part, alpha):
        self.fem = fem
        topo = fem.topo
        self.part = np.asarray(part, dtype=np.int64)
        self.alpha = complex(alpha)
        N = int(self.part.max()) + 1
        self.N = N
        if np.any(np.bincount(self.part, minlength=N) == 0):
            raise ValueError("empty subdomain")

        # Sub(e): subdomains containing each unknown (non-PEC) edge
        pe = np.unique(np.stack([np.repeat(self.part, 6), topo.tet_edges.ravel()], 1), axis=0)
        self.sub_of_edge = [[] for _ in range(topo.n_edges)]
        for d, e in pe:
            if not fem.pec[e]:
                self.sub_of_edge[e].append(int(d))
        self.owner = np.array([s[0] if s else -1 for s in self.sub_of_edge], dtype=np.int64)
        # local numbering: sorted global ids of each subdomain's unknown edges
        self.sub_edges = []
        for d in range(N):
            ge = np.unique(topo.tet_edges[self.part == d].ravel())
            self.sub_edges.append(ge[~fem.pec[ge]])

        # interface triangles: faces whose two tetrahedra lie in different parts
        two = np.nonzero(topo.face_count == 2)[0]
        pa = self.part[topo.face_tets[two, 0]]
        pb = self.part[topo.face_tets[two, 1]]
        cut = pa != pb
        self.iface = two[cut]
        self.iface_pq = np.stack([np.minimum(pa[cut], pb[cut]), np.maximum(pa[cut], pb[cut])], 1)
        g, area, _ = triangle_geometry(topo.xyz, topo.faces[self.iface])
        self.Ti = tangential_mass(g, area)

        self._build_lms()
        self._build_subdomain_matrices()

    # --- LM trees (continuity on every shared edge) -------------------------
    def _build_lms(self):
        topo = self.fem.topo
        cand = {}
        for t, (p, q) in zip(self.iface, self.iface_pq):
            for e in topo.face_edges[t]:
                cand.setdefault(int(e), set()).add((int(p), int(q)))
        lms = []
        for e, subs in enumerate(self.sub_of_edge):
            if len(subs) < 2:  # interior, or a PEC edge (no subdomain holds it)
                continue
            dsu = _DSU(subs)
            chosen = []
            for (p, q) in sorted(cand.get(e, ())):
                if dsu.union(p, q):
                    chosen.append((p, q))
            if len(chosen) != len(subs) - 1:
                raise ValueError(f"edge {e}: subdomains {subs} not connected through interface triangles")
            for (p, q) in chosen:
                lms.append((p, q, e))
        lms.sort()
        self.lms = np.array(lms, dtype=np.int64).reshape(-1, 3)
        self.n_lm = self.lms.shape[0]
        pairs, starts = np.unique(self.lms[:, :2], axis=0, return_index=True)
        self.blocks = pairs  # block b = subdomain pair (p, q)
        self.block_start = np.concatenate([starts, [self.n_lm]]).astype(np.int64)
        self.n_blocks = pairs.shape[0]
        self.lm_block = np.searchsorted(starts, np.arange(self.n_lm), side="right") - 1

    # --- A_d: FEM-ABC matrix of subdomain d with Robin loss/gain ------------
    def _build_subdomain_matrices(self):
        fem, topo = self.fem, self.fem.topo
        self.A = []
        self.lm_of_sub = []
        self.D = []
        bf_tet = topo.face_tets[fem.bfaces, 0]
        for d in range(self.N):
            ge = self.sub_edges[d]
            nd = ge.size
            locmap = np.full(topo.n_edges, -1, dtype=np.int64)  # -1: not an unknown of d
            locmap[ge] = np.arange(nd)
            loc = {int(e): i for i, e in enumerate(ge)}
            rows, cols, vals = [], [], []
            tl = np.nonzero(self.part == d)[0]
            te = locmap[topo.tet_edges[tl]]
            rows.append(np.repeat(te, 6, 1).ravel()); cols.append(np.tile(te, (1, 6)).ravel())
            vals.append(fem.Se[tl].astype(np.complex128).ravel())
            bsel = np.nonzero(self.part[bf_tet] == d)[0]
            if bsel.size:
                fe = locmap[topo.face_edges[fem.bfaces[bsel]]]
                rows.append(np.repeat(fe, 3, 1).ravel()); cols.append(np.tile(fe, (1, 3)).ravel())
                vals.append((1j * fem.k * fem.Tb[bsel]).ravel())
            for sign, col in ((+1.0, 0), (-1.0, 1)):
                isel = np.nonzero(self.iface_pq[:, col] == d)[0]
                if isel.size:
                    fe = locmap[topo.face_edges[self.iface[isel]]]
                    rows.append(np.repeat(fe, 3, 1).ravel()); cols.append(np.tile(fe, (1, 3)).ravel())
                    vals.append((sign * self.alpha * self.Ti[isel]).ravel())
            r_, c_, v_ = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
            keep = (r_ >= 0) & (c_ >= 0)  # entries of PEC rows or columns leave the system
            A = sp.coo_matrix((v_[keep], (r_[keep], c_[keep])), shape=(nd, nd)).tocsc()
            A.sum_duplicates()
            self.A.append(A)
            # D_d restricted to the LMs touching d (sorted by global LM index)
            lmd = np.nonzero((self.lms[:, 0] == d) | (self.lms[:, 1] == d))[0]
            self.lm_of_sub.append(lmd)
            Dd = np.zeros((nd, lmd.size))
            for c, l in enumerate(lmd):
                p, q, e = self.lms[l]
                Dd[loc[int(e)], c] = 1.0 if p == d else -1.0
            self.D.append(Dd)

    # --- loads ---------------------------------------------------------------
    def split_load(self, f):
        """f_d[e] = f[e] if d = min Sub(e) else 0; f is [nrhs, n_edges]."""
        f = np.atleast_2d(f)
        out = []
        for d in range(self.N):
            ge = self.sub_edges[d]
            fd = np.where((self.owner[ge] == d)[None, :], f[:, ge], 0.0)
            out.append(fd.astype(np.complex128))
        return out

    def sum_subdomain_matrices(self):
        """sum_d R_d^T A_d R_d (equals S on the unknowns: the Robin terms cancel)."""
        n = self.fem.topo.n_edges
        tot = sp.csr_matrix((n, n), dtype=np.complex128)
        for d in range(self.N):
            ge = self.sub_edges[d]
            R = sp.csr_matrix((np.ones(ge.size), (np.arange(ge.size), ge)), shape=(ge.size, n))
            tot = tot + R.T @ self.A[d] @ R
        return tot

    def D_global(self):
        """Global D as a dense [sum n_d, n_lm] matrix (tiny meshes only)."""
        nd = [e.size for e in self.sub_edges]
        off = np.concatenate([[0], np.cumsum(nd)])
        D = np.zeros((off[-1], self.n_lm))
        for d in range(self.N):
            D[off[d]:off[d + 1], self.lm_of_sub[d]] = self.D[d]
        return D, off


class DomainMatrices:
    """Step 1 and step 2 of the recipe in Section II: dense domain matrices
    K_D^(d) = D_d^T A_d^{-1} D_d (sparse LU of A_d, an exact method), their
    assembly into the block-wise sparse K, and g = sum_d D_d^T A_d^{-1} f_d.
    """

    def __init__(self, dec: Decomposition):
        self.dec = dec
        self.lu = [sla.splu(A) for A in dec.A]
        self.KD = []
        for d in range(dec.N):
            if dec.D[d].shape[1]:
                Y = self.lu[d].solve(dec.D[d].astype(np.complex128))
                self.KD.append(dec.D[d].T @ Y)
            else:
                self.KD.append(np.zeros((0, 0), np.complex128))

    def assemble_blocks(self):
        """K as a dict {(P, Q): dense block} over block indices (both triangles)."""
        dec = self.dec
        K = {}
        for d in range(dec.N):
            lmd = dec.lm_of_sub[d]
            blk = dec.lm_block[lmd]
            for P in np.unique(blk):
                rp = np.nonzero(blk == P)[0]
                for Q in np.unique(blk):
                    rq = np.nonzero(blk == Q)[0]
                    key = (int(P), int(Q))
                    piece = self.KD[d][np.ix_(rp, rq)]
                    if key in K:
                        K[key] = K[key] + piece
                    else:
                        K[key] = piece.copy()
        return K

    def assemble_dense(self):
        """Dense K (small meshes only)."""
        dec = self.dec
        K = np.zeros((dec.n_lm, dec.n_lm), dtype=np.complex128)
        for d in range(dec.N):
            lmd = dec.lm_of_sub[d]
            K[np.ix_(lmd, lmd)] += self.KD[d]
        return K

    def subdomain_solves(self, fd_list):
        """y_d = A_d^{-1} f_d for every subdomain (f_d is [nrhs, n_d])."""
        return [self.lu[d].solve(fd_list[d].T.copy()).T for d in range(self.dec.N)]

    def reduced_rhs(self, fd_list):
        """g = sum_d D_d^T A_d^{-1} f_d, [nrhs, n_lm]."""
        dec = self.dec
        nrhs = fd_list[0].shape[0]
        g = np.zeros((nrhs, dec.n_lm), dtype=np.complex128)
        ys = self.subdomain_solves(fd_list)
        for d in range(dec.N):
            g[:, dec.lm_of_sub[d]] += ys[d] @ dec.D[d]
        return g

    def recover(self, fd_list, lam):
        """Step 7: E_d = A_d^{-1}(f_d - D_d lambda); E[e] taken from d = min Sub(e).

        Returns (E [nrhs, n_edges], max copy discrepancy over shared edges).
        """
        dec = self.dec
        n = dec.fem.topo.n_edges
        nrhs = lam.shape[0]
        E = np.zeros((nrhs, n), dtype=np.complex128)
        copies = np.full((nrhs, n), np.nan + 0j)
        disc = 0.0
        for d in range(dec.N):
            r = fd_list[d] - lam[:, dec.lm_of_sub[d]] @ dec.D[d].T
            Ed = self.lu[d].solve(r.T.copy()).T
            ge = dec.sub_edges[d]
            own = dec.owner[ge] == d
            E[:, ge[own]] = Ed[:, own]
            prev = copies[:, ge]
            seen = ~np.isnan(prev.real)
            if np.any(seen):
                disc = max(disc, float(np.max(np.abs(prev[seen] - Ed[seen]))))
            copies[:, ge] = np.where(seen, prev, Ed)
        return E, disc
