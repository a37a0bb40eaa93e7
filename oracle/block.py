"""Steps 3-6 of the recipe in Section II and Algorithm 1 -- oracle.

* Step 3 (reorder the clique graph of K): blocks P, Q of K are adjacent when
  they share a subdomain.  The paper uses METIS; it is not available, so the
  oracle orders blocks by geometric nested dissection of the box layout
  (split the longest box range in two, order left, right, then the blocks
  between the halves).  Any order gives the same lambda and E.
* Step 4 (symbolic factorisation): struct(j) = the later blocks i with
  L_ij != 0, by block elimination on the clique graph.
* Step 5, Algorithm 1 as corrected (the printed listing swaps the block
  indices of the permutation and of D, and updates from A instead of K):
  for each block j in order,
      P_j^T K_jj P_j = L_jj D_jj L_jj^T          (pivoting restricted to j)
      X_ij = K_ij P_j L_jj^{-T},  W_ij = X_ij D_jj^{-1}   (i in struct(j))
      K_ik <- K_ik - X_ij W_kj^T                (i >= k in struct(j))
  The global factor is P L D L^T P^T with L_jj as computed,
  L_ij = P_i^T W_ij and P = blkdiag(P_j).
* Step 6: forward, diagonal and backward substitution in the same block
  order.
* The multifrontal form of step 5 (named after the seven steps of Section
  II as a way to speed the block LDL^T up): the same factors, with the
  Schur updates gathered in the elimination tree instead of applied in
  place.  The parent of j is the first block of struct(j); the front of j
  is block column j of K plus the update matrices of j's children added in
  at their rows and columns (extend-add), and after j's pivot block and
  panels are formed its own update matrix
      U_j[i, k] = F_j[i, k] - X_ij W_kj^T      (i >= k in struct(j))
  goes to the parent.  F_j[i, k] for i, k in struct(j) holds only the
  children's contributions: the entries of K there belong to the front of
  block k.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .bk import bk_ldlt


def nested_dissection_boxes(blocks, parts):
    """Order of the blocks (subdomain pairs) by geometric nested dissection of
    the px x py x pz box layout, box id (bx*py + by)*pz + bz."""
    px, py, pz = parts
    coords = {}
    for b in range(px * py * pz):
        coords[b] = (b // (py * pz), (b // pz) % py, b % pz)
    blocks = [tuple(map(int, b)) for b in blocks]
    index = {b: i for i, b in enumerate(blocks)}
    order = []

    def inside(c, lo, hi):
        return all(lo[a] <= c[a] < hi[a] for a in range(3))

    def rec(lo, hi):
        ext = [hi[a] - lo[a] for a in range(3)]
        if max(ext) <= 1:
            return
        ax = int(np.argmax(ext))
        mid = lo[ax] + ext[ax] // 2
        lhi = list(hi); lhi[ax] = mid
        rlo = list(lo); rlo[ax] = mid
        rec(lo, lhi)
        rec(rlo, hi)
        sep = []
        for b in blocks:
            cp, cq = coords[b[0]], coords[b[1]]
            if not (inside(cp, lo, hi) and inside(cq, lo, hi)):
                continue
            lp, lq = cp[ax] < mid, cq[ax] < mid
            if lp != lq:
                sep.append(b)
        order.extend(index[b] for b in sorted(sep))

    rec([0, 0, 0], [px, py, pz])
    if sorted(order) != list(range(len(blocks))):
        raise ValueError("nested dissection did not order every block once")
    return np.array(order, dtype=np.int64)


def clique_adjacency(blocks):
    """Blocks are adjacent when they share a subdomain (the clique graph)."""
    nb = len(blocks)
    by_sub = {}
    for i, (p, q) in enumerate(blocks):
        by_sub.setdefault(int(p), []).append(i)
        by_sub.setdefault(int(q), []).append(i)
    adj = [set() for _ in range(nb)]
    for lst in by_sub.values():
        for a in lst:
            adj[a].update(lst)
    for a in range(nb):
        adj[a].discard(a)
    return adj


def symbolic(adj, order):
    """struct(j) in elimination positions (sorted), by block elimination:
    eliminating j connects all of its later neighbours."""
    nb = len(order)
    pos = np.empty(nb, dtype=np.int64)
    pos[order] = np.arange(nb)
    nbrs = [set(int(pos[x]) for x in adj[order[j]]) for j in range(nb)]
    struct = []
    for j in range(nb):
        s = sorted(x for x in nbrs[j] if x > j)
        struct.append(s)
        for a in s:
            nbrs[a].update(s)
            nbrs[a].discard(a)
    return struct


class BlockLDLT:
    """Algorithm 1 on a block dict (positions are elimination positions)."""

    def __init__(self, Kb, sizes, struct, pivoting=True):
        self.sizes = list(sizes)
        self.struct = struct
        l = len(sizes)
        K = {key: val.copy() for key, val in Kb.items()}
        for j in range(l):
            for i in struct[j]:
                if (i, j) not in K:
                    K[(i, j)] = np.zeros((sizes[i], sizes[j]), np.complex128)
        self.diag = []
        self.Lhat = {}
        for j in range(l):
            f = bk_ldlt(K[(j, j)], pivoting=pivoting)
            self.diag.append(f)
            Dinv = f.dinv()
            X, W = {}, {}
            for i in struct[j]:
                Kp = K[(i, j)][:, f.perm]                          # K_ij P_j
                Xt = sla.solve_triangular(f.L, Kp.T, lower=True, unit_diagonal=True)
                X[i] = Xt.T                                        # K_ij P_j L^-T
                W[i] = X[i] @ Dinv
            for a, i in enumerate(struct[j]):
                for k in struct[j][:a + 1]:
                    K[(i, k)] = K[(i, k)] - X[i] @ W[k].T
                self.Lhat[(i, j)] = W[i]

    def solve(self, g):
        """lambda for right-hand sides g given as a list of per-block arrays
        [n_j, nrhs] (positions in elimination order)."""
        l = len(self.sizes)
        gt = [x.astype(np.complex128).copy() for x in g]
        y = [None] * l
        for j in range(l):
            f = self.diag[j]
            y[j] = sla.solve_triangular(f.L, gt[j][f.perm], lower=True, unit_diagonal=True)
            for i in self.struct[j]:
                gt[i] -= self.Lhat[(i, j)] @ y[j]
        v = [np.linalg.solve(self.diag[j].D, y[j]) if self.sizes[j] else y[j] for j in range(l)]
        lam = [None] * l
        for j in reversed(range(l)):
            f = self.diag[j]
            r = v[j].copy()
            for i in self.struct[j]:
                r -= self.Lhat[(i, j)].T @ lam[i]
            mu = sla.solve_triangular(f.L.T, r, lower=False, unit_diagonal=True)
            lam[j] = np.empty_like(mu)
            lam[j][f.perm] = mu
        return lam

    def reconstruct_dense(self):
        """P L D L^T P^T as a dense matrix in elimination-position block order."""
        off = np.concatenate([[0], np.cumsum(self.sizes)]).astype(int)
        n = off[-1]
        L = np.zeros((n, n), np.complex128)
        D = np.zeros((n, n), np.complex128)
        P = np.zeros((n, n))
        for j, f in enumerate(self.diag):
            sj = slice(off[j], off[j + 1])
            L[sj, sj] = f.L
            D[sj, sj] = f.D
            P[off[j] + f.perm, off[j] + np.arange(self.sizes[j])] = 1.0
        for (i, j), W in self.Lhat.items():
            Pi = np.eye(self.sizes[i])[:, self.diag[i].perm]
            L[off[i]:off[i + 1], off[j]:off[j + 1]] = Pi.T @ W
        return P @ L @ D @ L.T @ P.T


def tree_parent(struct):
    """Parent of every block in the elimination tree: the first block of
    struct(j), -1 for a root."""
    return [s[0] if s else -1 for s in struct]


class MultifrontalLDLT(BlockLDLT):
    """Step 5 in multifrontal form: same factors as ``BlockLDLT`` (up to the
    order of rounding), the updates carried by update matrices.  ``update``
    keeps every block's update matrix U_j as a dict over (i, k), i >= k in
    struct(j)."""

    def __init__(self, Kb, sizes, struct, pivoting=True):
        self.sizes = list(sizes)
        self.struct = struct
        l = len(sizes)
        parent = tree_parent(struct)
        children = [[] for _ in range(l)]
        for c, p in enumerate(parent):
            if p >= 0:
                children[p].append(c)
        self.diag = []
        self.Lhat = {}
        self.update = []
        for j in range(l):
            rows = [j] + list(struct[j])
            # front of j: block column j of K, then every child's update
            # matrix added at its own rows and columns
            F = {}
            for a, i in enumerate(rows):
                for k in rows[:a + 1]:
                    F[(i, k)] = np.zeros((sizes[i], sizes[k]), np.complex128)
            for i in rows:
                if (i, j) in Kb:
                    F[(i, j)] += Kb[(i, j)]
            for c in children[j]:
                for (i, k), U in self.update[c].items():
                    if (i, k) not in F:
                        raise ValueError(f"update matrix of {c} reaches ({i}, {k}) outside the front of {j}")
                    F[(i, k)] += U
            f = bk_ldlt(F[(j, j)], pivoting=pivoting)
            self.diag.append(f)
            Dinv = f.dinv()
            X, W = {}, {}
            for i in struct[j]:
                Kp = F[(i, j)][:, f.perm]                          # F_ij P_j
                X[i] = sla.solve_triangular(f.L, Kp.T, lower=True, unit_diagonal=True).T
                W[i] = X[i] @ Dinv
                self.Lhat[(i, j)] = W[i]
            U = {}
            for a, i in enumerate(struct[j]):
                for k in struct[j][:a + 1]:
                    U[(i, k)] = F[(i, k)] - X[i] @ W[k].T
            self.update.append(U)
