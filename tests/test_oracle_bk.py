"""Pins of the oracle's dense Bunch-Kaufman LDL^T and of Algorithm 1.

* BK decisions are compared with LAPACK's own complex-symmetric
  factorisation (scipy.linalg.lapack.zsytrf, lower): the same 1x1/2x2
  choices and interchanges, and the same D entries.
* Block LDL^T is pinned by reconstruction P L D L^T P^T = K, by the
  unpivoted variant giving the same solution, and by a one-block K reducing
  to the dense factorisation.
"""
import numpy as np
import pytest
from scipy.linalg import lapack

from oracle.bk import SingularBlock, bk_ldlt
from oracle.block import BlockLDLT, clique_adjacency, symbolic


def _rand_sym(rng, n, diag_scale=1.0, spread=True):
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    if spread:
        A *= 10.0 ** rng.uniform(-2, 2, (n, n))
    A = A + A.T
    A[np.diag_indices(n)] *= diag_scale
    return A


def test_bk_matches_lapack_pivot_sequence():
    rng = np.random.default_rng(7)
    n_two = 0
    for trial in range(100):
        n = int(rng.integers(8, 97))
        A = _rand_sym(rng, n, diag_scale=[1.0, 0.05, 1e-3][trial % 3])
        f = bk_ldlt(A)
        ldu, ipiv, info = lapack.zsytrf(A, lower=1)
        assert info == 0
        assert np.array_equal(f.lapack_ipiv(), ipiv), trial
        n_two += sum(1 for p in f.pivots if p[1] == 2)
        # D blocks equal LAPACK's (diagonal and 2x2 off-diagonal entries)
        dl = np.diag(ldu)
        assert np.allclose(np.diag(f.D), dl, rtol=1e-10, atol=1e-12 * np.abs(dl).max())
        rec = f.reconstruct()
        assert np.linalg.norm(rec - A) <= 1e-13 * np.linalg.norm(A) * n
    assert n_two > 50  # the suite really exercises 2x2 pivots


def test_bk_forced_two_by_two():
    # zero diagonal with [[0,1],[1,0]] blocks: every pivot must be 2x2
    n = 8
    A = np.zeros((n, n), complex)
    for k in range(0, n, 2):
        A[k, k + 1] = A[k + 1, k] = 1.0 + 0.5j
    f = bk_ldlt(A)
    assert all(p[1] == 2 for p in f.pivots)
    assert np.allclose(f.reconstruct(), A, atol=1e-15)
    Dinv = f.dinv()
    assert np.allclose(Dinv @ f.D, np.eye(n), atol=1e-14)


def test_bk_is_not_hermitian():
    # a complex-symmetric matrix: the factorisation uses plain transposes
    rng = np.random.default_rng(3)
    A = _rand_sym(rng, 20)
    f = bk_ldlt(A)
    P = np.eye(20)[:, f.perm]
    assert np.allclose(P @ f.L @ f.D @ f.L.T @ P.T, A, rtol=1e-12, atol=1e-12 * np.abs(A).max())
    assert not np.allclose(P @ f.L @ f.D @ f.L.conj().T @ P.T, A)


def test_bk_singular_block_detected():
    A = np.zeros((4, 4), complex)
    A[0, 0] = 1.0
    with pytest.raises(SingularBlock) as ei:
        bk_ldlt(A)
    assert ei.value.column == 1


def _block_problem(rng, sizes, density=0.5):
    nb = len(sizes)
    off = np.concatenate([[0], np.cumsum(sizes)])
    n = off[-1]
    mask = rng.random((nb, nb)) < density
    mask = mask | mask.T
    np.fill_diagonal(mask, True)
    A = np.zeros((n, n), complex)
    for i in range(nb):
        for j in range(i + 1):
            if mask[i, j]:
                B = rng.standard_normal((sizes[i], sizes[j])) + 1j * rng.standard_normal((sizes[i], sizes[j]))
                A[off[i]:off[i + 1], off[j]:off[j + 1]] = B
                A[off[j]:off[j + 1], off[i]:off[i + 1]] = B.T
    for i in range(nb):
        s = slice(off[i], off[i + 1])
        A[s, s] = 0.5 * (A[s, s] + A[s, s].T)
    adj = [set(np.nonzero(mask[i])[0]) - {i} for i in range(nb)]
    return A, off, adj


def _blocks_of(A, off, struct):
    nb = len(off) - 1
    Kb = {}
    for j in range(nb):
        Kb[(j, j)] = A[off[j]:off[j + 1], off[j]:off[j + 1]]
        for i in struct[j]:
            Kb[(i, j)] = A[off[i]:off[i + 1], off[j]:off[j + 1]]
    return Kb


def test_block_ldlt_reconstructs_and_solves():
    rng = np.random.default_rng(11)
    sizes = [int(s) for s in rng.integers(3, 12, 9)]
    A, off, adj = _block_problem(rng, sizes)
    struct = symbolic(adj, np.arange(len(sizes)))
    F = BlockLDLT(_blocks_of(A, off, struct), sizes, struct)
    rec = F.reconstruct_dense()
    assert np.linalg.norm(rec - A) <= 1e-12 * np.linalg.norm(A)
    g = rng.standard_normal((off[-1], 3)) + 1j * rng.standard_normal((off[-1], 3))
    lam = np.concatenate(F.solve([g[off[j]:off[j + 1]] for j in range(len(sizes))]))
    assert np.linalg.norm(A @ lam - g) <= 1e-12 * np.linalg.norm(g) * 10
    # unpivoted variant gives the same solution
    F0 = BlockLDLT(_blocks_of(A, off, struct), sizes, struct, pivoting=False)
    lam0 = np.concatenate(F0.solve([g[off[j]:off[j + 1]] for j in range(len(sizes))]))
    assert np.linalg.norm(lam0 - lam) <= 1e-9 * np.linalg.norm(lam)


def test_one_block_is_dense_bk():
    rng = np.random.default_rng(5)
    A = _rand_sym(rng, 30)
    F = BlockLDLT({(0, 0): A}, [30], [[]])
    f = bk_ldlt(A)
    assert np.array_equal(F.diag[0].perm, f.perm)
    assert np.allclose(F.diag[0].L, f.L)


def test_symbolic_matches_dense_fill():
    # struct(j) equals the nonzero block pattern of L from boolean elimination
    rng = np.random.default_rng(2)
    for trial in range(10):
        nb = 15
        M = rng.random((nb, nb)) < 0.2
        M = M | M.T
        np.fill_diagonal(M, False)
        adj = [set(np.nonzero(M[i])[0]) for i in range(nb)]
        order = rng.permutation(nb)
        struct = symbolic(adj, order)
        B = M[np.ix_(order, order)].copy()
        for j in range(nb):
            below = np.nonzero(B[j + 1:, j])[0] + j + 1
            assert list(below) == struct[j]
            B[np.ix_(below, below)] = True
            np.fill_diagonal(B, False)


def test_clique_adjacency():
    blocks = [(0, 1), (0, 2), (1, 3), (2, 3)]
    adj = clique_adjacency(blocks)
    assert adj[0] == {1, 2} and adj[3] == {1, 2}
