"""Dense complex-symmetric Bunch-Kaufman LDL^T -- oracle.

The paper factors each diagonal block of K with Bunch-Kaufman symmetric
partial pivoting (Section II, reference [bunch1977]) restricted to that block:
pivot rows are searched only inside the block and no pivot is delayed to a
later block (Section I: the formulation has no delayed pivots).

Reading (the paper gives no constants): alpha_BK = (1 + sqrt 17)/8, the
magnitude |z| = |Re z| + |Im z| (the usual convention for complex symmetric
matrices), ties go to the lowest row index, and the transpose is a plain
transpose (K is complex symmetric, not Hermitian).  At step k, with
lam1 = max_{i>k} |a_ik| attained at row r:

  * lam1 = 0 and a_kk = 0  -> the block is singular (no delayed pivots);
  * |a_kk| >= alpha lam1   -> 1x1 pivot at k;
  * else sigma = max_{i >= k, i != r} |a_ir| and
      |a_kk| sigma >= alpha lam1^2  -> 1x1 pivot at k,
      |a_rr| >= alpha sigma          -> swap k<->r, 1x1 pivot,
      otherwise                      -> swap k+1<->r, 2x2 pivot
        E = [[a, b], [b, c]],  E^{-1} = [[c, -b], [-b, a]] / (ac - b^2).

The result is P^T A P = L D L^T with L unit lower triangular (row swaps are
applied to the already computed columns of L, so L is in one consistent row
order) and (P^T A P)[i, j] = A[perm[i], perm[j]].
"""
from __future__ import annotations

import math

import numpy as np

ALPHA_BK = (1.0 + math.sqrt(17.0)) / 8.0


class SingularBlock(Exception):
    def __init__(self, column):
        super().__init__(f"zero pivot column {column}")
        self.column = column


def cabs1(z):
    return np.abs(np.real(z)) + np.abs(np.imag(z))


class BKFactor:
    """perm, L, and the block diagonal D (as dense plus the pivot list)."""

    def __init__(self, perm, L, D, pivots):
        self.perm = perm
        self.L = L
        self.D = D
        self.pivots = pivots  # list of (k, size, partner_row)

    @property
    def n(self):
        return self.L.shape[0]

    def lapack_ipiv(self):
        """The same decisions in LAPACK ?sytrf(lower) ipiv form (1-based)."""
        ipiv = np.zeros(self.n, dtype=np.int64)
        for k, size, r in self.pivots:
            if size == 1:
                ipiv[k] = r + 1
            else:
                ipiv[k] = ipiv[k + 1] = -(r + 1)
        return ipiv

    def dinv(self):
        """D^{-1} from the 1x1 reciprocals and the 2x2 closed-form inverses."""
        Di = np.zeros_like(self.D)
        for k, size, _ in self.pivots:
            if size == 1:
                Di[k, k] = 1.0 / self.D[k, k]
            else:
                a, b, c = self.D[k, k], self.D[k + 1, k], self.D[k + 1, k + 1]
                det = a * c - b * b
                Di[k:k + 2, k:k + 2] = np.array([[c, -b], [-b, a]]) / det
        return Di

    def reconstruct(self):
        P = np.eye(self.n)[:, self.perm]
        return P @ self.L @ self.D @ self.L.T @ P.T


def bk_ldlt(A, alpha=ALPHA_BK, pivoting=True):
    """Factor a dense complex-symmetric matrix (full storage is read).

    ``pivoting=False`` gives the unpivoted LDL^T (1x1 pivots, no swaps).
    """
    A = np.array(A, dtype=np.complex128, copy=True)
    n = A.shape[0]
    perm = np.arange(n)
    L = np.eye(n, dtype=np.complex128)
    D = np.zeros((n, n), dtype=np.complex128)
    pivots = []
    k = 0
    while k < n:
        akk = cabs1(A[k, k])
        if k + 1 < n:
            col = cabs1(A[k + 1:, k])
            r = k + 1 + int(np.argmax(col))
            lam1 = float(col[r - k - 1])
        else:
            r, lam1 = k, 0.0
        if not pivoting:
            if A[k, k] == 0:
                raise SingularBlock(k)
            size, partner = 1, k
        elif max(akk, lam1) == 0.0:
            raise SingularBlock(k)
        elif akk >= alpha * lam1:
            size, partner = 1, k
        else:
            others = np.concatenate([cabs1(A[k:r, r]), cabs1(A[r + 1:, r])])
            sigma = float(others.max()) if others.size else 0.0
            if akk * sigma >= alpha * lam1 * lam1:
                size, partner = 1, k
            elif cabs1(A[r, r]) >= alpha * sigma:
                size, partner = 1, r
            else:
                size, partner = 2, r
        kk = k + size - 1
        if partner != kk:
            A[[kk, partner], :] = A[[partner, kk], :]
            A[:, [kk, partner]] = A[:, [partner, kk]]
            L[[kk, partner], :k] = L[[partner, kk], :k]
            perm[[kk, partner]] = perm[[partner, kk]]
        if size == 1:
            d = A[k, k]
            D[k, k] = d
            x = A[k + 1:, k].copy()
            l = x / d
            A[k + 1:, k + 1:] -= np.outer(l, x)
            L[k + 1:, k] = l
        else:
            a, b, c = A[k, k], A[k + 1, k], A[k + 1, k + 1]
            D[k:k + 2, k:k + 2] = np.array([[a, b], [b, c]])
            Einv = np.array([[c, -b], [-b, a]]) / (a * c - b * b)
            X = A[k + 2:, k:k + 2].copy()
            Lc = X @ Einv
            A[k + 2:, k + 2:] -= Lc @ X.T
            L[k + 2:, k:k + 2] = Lc
        pivots.append((k, size, partner))
        k += size
    return BKFactor(perm, L, D, pivots)
