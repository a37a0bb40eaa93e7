"""Pins of the oracle's multifrontal block LDL^T (the multifrontal form of
step 5 named after the seven steps of Section II).

The update matrix of block j is fixed by the matrix alone: with T the
subtree of j in the elimination tree (j and its descendants) and S =
struct(j), the updates that the columns of T send to the rows and columns of
S sum to K[S,T] K[T,T]^{-1} K[T,S] (eliminating T first is a partial
factorisation whose Schur complement on S is K[S,S] minus that product, and
the columns of T touch no row outside T and S).  So U_j = -K[S,T] K[T,T]^{-1}
K[T,S], checked with a dense inverse; a wrong extend-add row, a dropped
child or a transposed operand breaks it.  The factors then reconstruct K,
and the solution equals the plain sparse LU of S.
"""
import math

import numpy as np

import workloads as W
from oracle.block import BlockLDLT, MultifrontalLDLT, tree_parent
from oracle.d3m import D3MOracle, global_solve


def _setup(n=4, parts=(2, 2, 2), seed=21):
    prob = W.make_problem(n, parts, eps=("uniform", 1, 4), k=2 * math.pi, nrhs=2, seed=seed)
    o = D3MOracle.from_problem(prob, multifrontal=True).factor()
    return prob, o


def _dense_positions(o):
    K = o.dm.assemble_dense()
    idx = np.concatenate([np.arange(o.dec.block_start[b], o.dec.block_start[b + 1]) for b in o.order])
    return K[np.ix_(idx, idx)]


def test_update_matrices_are_subtree_schur_complements():
    prob, o = _setup()
    K = _dense_positions(o)
    sizes = o.ldlt.sizes
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    parent = tree_parent(o.struct)
    l = len(sizes)
    checked = 0
    for j in range(l):
        sub = {j}
        for c in range(j - 1, -1, -1):  # descendants come before j
            p = parent[c]
            while p != -1 and p < j:
                p = parent[p]
            if p == j:
                sub.add(c)
        T = np.concatenate([np.arange(off[b], off[b + 1]) for b in sorted(sub)])
        S = o.struct[j]
        if not S:
            continue
        Sx = np.concatenate([np.arange(off[b], off[b + 1]) for b in S])
        want = -K[np.ix_(Sx, T)] @ np.linalg.solve(K[np.ix_(T, T)], K[np.ix_(T, Sx)])
        scale = np.abs(want).max()
        for (i, k), U in o.ldlt.update[j].items():
            ri = np.searchsorted(Sx, np.arange(off[i], off[i + 1]))
            ck = np.searchsorted(Sx, np.arange(off[k], off[k + 1]))
            assert np.abs(U - want[np.ix_(ri, ck)]).max() <= 1e-10 * scale, (j, i, k)
        checked += 1
    assert checked >= l // 2


def test_multifrontal_reconstructs_K_and_solves_exactly():
    prob, o = _setup(seed=22)
    K = _dense_positions(o)
    rec = o.ldlt.reconstruct_dense()
    assert np.linalg.norm(rec - K) <= 1e-12 * np.linalg.norm(K)
    f = o.fem.planewave_rhs(prob.dirs, prob.pols)
    E = o.solve(f)
    E0 = global_solve(o.fem, f)
    assert np.abs(E - E0).max() <= 1e-10 * np.abs(E0).max()


def test_same_pivots_as_right_looking_form():
    """Both forms factor the same updated diagonal blocks (up to rounding),
    so on continuous random data they take the same pivots."""
    prob, o = _setup(seed=23)
    Kpos = {}
    K = _dense_positions(o)
    sizes = o.ldlt.sizes
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    for j in range(len(sizes)):
        for i in [j] + list(o.struct[j]):
            blk = K[off[i]:off[i + 1], off[j]:off[j + 1]]
            if np.any(blk):
                Kpos[(i, j)] = blk
    rl = BlockLDLT(Kpos, sizes, o.struct)
    mf = MultifrontalLDLT(Kpos, sizes, o.struct)
    for a, b in zip(rl.diag, mf.diag):
        assert list(a.perm) == list(b.perm)
        assert [p[1] for p in a.pivots] == [p[1] for p in b.pivots]
    for key, W_ in rl.Lhat.items():
        assert np.abs(mf.Lhat[key] - W_).max() <= 1e-10 * max(np.abs(W_).max(), 1e-300)
