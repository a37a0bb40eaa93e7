"""The seven steps of D3M (Section II) end to end, plus the adjoint -- oracle.

Step 1-2 (``ddm.DomainMatrices``), steps 3-4 (``block.nested_dissection_boxes``
and ``block.symbolic``), step 5 (``block.BlockLDLT``, or its multifrontal form
``block.MultifrontalLDLT``), step 6
(``BlockLDLT.solve``) and step 7 (``DomainMatrices.recover``).

Adjoint (a reading: the paper does not differentiate).  S is complex
symmetric (S^T = S), so for a real objective L(E) with PyTorch's gradient
G = dL/dRe E + j dL/dIm E,

    dL/d theta = Re(G^H dE/d theta) = -Re(w^T (dS/d theta) E),  w = S^{-1} conj(G),

and with dS/d eps_r,t = -k^2 M_t (the unit-eps_r element mass of tetrahedron
t) the gradient is dL/d eps_r,t = k^2 Re sum_rhs w_t^T M_t E_t.
"""
from __future__ import annotations

import time

import numpy as np
import scipy.sparse.linalg as sla

from .block import BlockLDLT, MultifrontalLDLT, clique_adjacency, nested_dissection_boxes, symbolic
from .ddm import Decomposition, DomainMatrices
from .fem import GlobalFEM


class D3MOracle:
    """Reference D3M solver for a ``workloads.Problem``-like set of arrays."""

    def __init__(self, xyz, tets, part, eps_r, k, alpha, parts=None, order=None,
                 pivoting=True, multifrontal=False, pec_faces=None):
        t0 = time.perf_counter()
        self.fem = GlobalFEM(xyz, tets, eps_r, k, pec_faces=pec_faces)
        self.dec = Decomposition(self.fem, part, alpha)
        self.parts = parts
        self.pivoting = pivoting
        self.multifrontal = multifrontal
        self.timings = {"setup": time.perf_counter() - t0}
        self._order = order

    @classmethod
    def from_problem(cls, prob, **kw):
        pec = getattr(prob, "pec_faces", None)
        return cls(prob.xyz, prob.tets, prob.part, prob.eps_r, prob.k, prob.alpha,
                   parts=prob.parts, pec_faces=pec, **kw)

    # steps 1-5
    def factor(self):
        dec = self.dec
        t0 = time.perf_counter()
        self.dm = DomainMatrices(dec)
        t1 = time.perf_counter()
        Kb = self.dm.assemble_blocks()
        t2 = time.perf_counter()
        if self._order is not None:
            order = np.asarray(self._order)
        elif self.parts is not None and dec.n_blocks:
            order = nested_dissection_boxes(dec.blocks, self.parts)
        else:
            order = np.arange(dec.n_blocks)
        self.order = order
        pos = np.empty(dec.n_blocks, dtype=np.int64)
        pos[order] = np.arange(dec.n_blocks)
        self.pos = pos
        self.struct = symbolic(clique_adjacency(dec.blocks), order)
        sizes = [int(dec.block_start[b + 1] - dec.block_start[b]) for b in order]
        Kpos = {(int(pos[P]), int(pos[Q])): v for (P, Q), v in Kb.items() if pos[P] >= pos[Q]}
        t3 = time.perf_counter()
        method = MultifrontalLDLT if self.multifrontal else BlockLDLT
        self.ldlt = method(Kpos, sizes, self.struct, pivoting=self.pivoting)
        t4 = time.perf_counter()
        self.timings.update(domain_matrices=t1 - t0, assemble=t2 - t1,
                            order_symbolic=t3 - t2, block_ldlt=t4 - t3)
        return self

    def _to_blocks(self, vec):
        dec = self.dec
        return [vec[:, dec.block_start[b]:dec.block_start[b + 1]].T for b in self.order]

    def _from_blocks(self, parts, nrhs):
        dec = self.dec
        out = np.zeros((nrhs, dec.n_lm), np.complex128)
        for j, b in enumerate(self.order):
            out[:, dec.block_start[b]:dec.block_start[b + 1]] = parts[j].T
        return out

    # steps 6-7
    def solve(self, f):
        """E [nrhs, n_edges] for global loads f [nrhs, n_edges]."""
        f = np.atleast_2d(np.asarray(f, dtype=np.complex128))
        t0 = time.perf_counter()
        fd = self.dec.split_load(f)
        g = self.dm.reduced_rhs(fd)
        t1 = time.perf_counter()
        lam = self._from_blocks(self.ldlt.solve(self._to_blocks(g)), f.shape[0])
        t2 = time.perf_counter()
        E, disc = self.dm.recover(fd, lam)
        t3 = time.perf_counter()
        self.g, self.lam, self.copy_discrepancy = g, lam, disc
        self.timings.update(reduce=t1 - t0, lm_solve=t2 - t1, recover=t3 - t2)
        return E

    def adjoint(self, G, E):
        """w = S^{-1} conj(G) through the same factors and the eps_r gradient."""
        w = self.solve(np.conj(np.atleast_2d(G)))
        return adjoint_gradient(self.fem, w, np.atleast_2d(E)), w


def adjoint_gradient(fem: GlobalFEM, w, E):
    """dL/d eps_r,t = k^2 Re sum_rhs w_t^T M_t E_t."""
    te = fem.topo.tet_edges
    M = fem.unit_mass()
    wt = w[:, te]  # [nrhs, n_t, 6]
    Et = E[:, te]
    return fem.k ** 2 * np.real(np.einsum("rta,tab,rtb->t", wt, M, Et))


def global_solve(fem: GlobalFEM, f):
    """The plain definition E = S^{-1} f by sparse LU of the undecomposed S
    (on the unknowns; zero on PEC edges)."""
    f = np.atleast_2d(f)
    E = np.zeros(f.shape, dtype=np.complex128)
    lu = sla.splu(fem.system().tocsc())
    E[:, fem.free] = lu.solve(f[:, fem.free].T.copy()).T
    return E


def relative_residual(S, E, f):
    """max over right-hand sides of ||S E - f||_inf / ||f||_inf."""
    E = np.atleast_2d(E)
    f = np.atleast_2d(f)
    r = (S @ E.T).T - f
    return float(np.max(np.abs(r).max(axis=1) / np.abs(f).max(axis=1)))
