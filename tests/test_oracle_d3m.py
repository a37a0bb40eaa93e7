"""Pins of the oracle's D3M pipeline (Section II, eq. (1), steps 1-7).

D3M is exact: with S and every A_d nonsingular its result is the plain
solution S^{-1} f of the undecomposed FEM system, for any Robin coefficient,
partition, LM tree and load split.  These tests pin the decomposed pipeline
to that definition (sparse LU of S, dense brute force on tiny meshes) and to
invariants that a wrong sign, index or transpose would break.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as sla

import workloads as W
from oracle.d3m import D3MOracle, adjoint_gradient, global_solve, relative_residual
from oracle.fem import GlobalFEM, probe_matrix


def _solve(prob, **kw):
    o = D3MOracle.from_problem(prob, **kw).factor()
    f = o.fem.planewave_rhs(prob.dirs, prob.pols)
    return o, f, o.solve(f)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_config1_exact_vs_global_sparse_lu():
    prob = W.make_config(1)
    o, f, E = _solve(prob)
    assert o.fem.topo.n_edges == 1854 and o.dec.n_lm == 246 and o.dec.n_blocks == 4
    Eg = global_solve(o.fem, f)
    assert _rel(E, Eg) <= 1e-10
    assert relative_residual(o.fem.S, E, f) <= 1e-12
    assert o.copy_discrepancy <= 1e-12 * np.abs(E).max()


@pytest.mark.parametrize("parts", [(2, 1, 1), (2, 2, 1), (2, 2, 2), (1, 3, 2)])
def test_exact_on_small_partitions(parts):
    prob = W.make_problem(4, parts, eps=("uniform", 1, 4), k=3 * math.pi, nrhs=2, seed=1)
    o, f, E = _solve(prob)
    Eg = global_solve(o.fem, f)
    assert _rel(E, Eg) <= 1e-10


@pytest.mark.parametrize("n,parts", [(2, (2, 1, 1)), (2, (2, 2, 1)), (2, (2, 2, 2)), (3, (2, 2, 2))])
def test_dense_saddle_brute_force(n, parts):
    # [A D; D^T 0][E; lam] = [f; 0] by dense LU; E copies must equal S^{-1} f
    prob = W.make_problem(n, parts, eps=("uniform", 1, 3), k=2 * math.pi, nrhs=1, seed=4)
    o, f, E = _solve(prob)
    dec = o.dec
    import scipy.linalg as la
    A = la.block_diag(*[a.toarray() for a in dec.A])
    D, off = dec.D_global()
    nA = A.shape[0]
    M = np.zeros((nA + dec.n_lm,) * 2, complex)
    M[:nA, :nA] = A
    M[:nA, nA:] = D
    M[nA:, :nA] = D.T
    fd = dec.split_load(f)
    rhs = np.concatenate([np.concatenate([x[0] for x in fd]), np.zeros(dec.n_lm)])
    sol = np.linalg.solve(M, rhs)
    Ed = sol[:nA]
    Edense = np.linalg.solve(o.fem.S.toarray(), f[0])
    for d in range(dec.N):
        assert _rel(Ed[off[d]:off[d + 1]], Edense[dec.sub_edges[d]]) <= 1e-12
    assert _rel(E[0], Edense) <= 1e-12
    assert _rel(o.lam[0], sol[nA:]) <= 1e-11


def test_domain_matrices_vs_dense_inverse():
    prob = W.make_problem(3, (2, 2, 1), eps=("uniform", 1, 4), k=2 * math.pi, seed=2)
    o = D3MOracle.from_problem(prob).factor()
    for d in range(o.dec.N):
        A = o.dec.A[d].toarray()
        Dd = o.dec.D[d]
        KD = Dd.T @ np.linalg.inv(A) @ Dd
        assert _rel(o.dm.KD[d], KD) <= 1e-12
        assert np.linalg.norm(o.dm.KD[d] - o.dm.KD[d].T) <= 1e-13 * np.linalg.norm(KD)


def test_robin_terms_cancel_in_assembly():
    prob = W.make_problem(4, (2, 2, 2), eps=("uniform", 1, 4), k=3.0, seed=3)
    o = D3MOracle.from_problem(prob)
    tot = o.dec.sum_subdomain_matrices()
    assert abs(tot - o.fem.S).max() <= 1e-14 * abs(o.fem.S).max()


@pytest.mark.parametrize("alpha_scale", [1j, -2j, 0.5j])
def test_alpha_invariance(alpha_scale):
    base = W.make_problem(4, (2, 2, 1), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=1, seed=5)
    _, _, E0 = _solve(base)
    other = W.make_problem(4, (2, 2, 1), eps=base.eps_r, k=2 * math.pi, nrhs=1, seed=5,
                           alpha=(0.5 if alpha_scale == 0.5j else 0.0) + alpha_scale * base.k,
                           dirs=base.dirs, pols=base.pols)
    _, _, E1 = _solve(other)
    assert _rel(E1, E0) <= 1e-10


def test_partition_invariance_and_single_domain():
    eps = np.random.default_rng(9).uniform(1, 4, 6 * 4 ** 3)
    sols = []
    for parts in [(1, 1, 1), (2, 2, 1), (1, 2, 2), (2, 2, 2)]:
        p = W.make_problem(4, parts, eps=eps, k=2 * math.pi, nrhs=1, seed=6)
        o, f, E = _solve(p)
        if parts == (1, 1, 1):
            assert o.dec.n_lm == 0
        sols.append(E)
    for E in sols[1:]:
        assert _rel(E, sols[0]) <= 1e-10


def test_order_invariance():
    prob = W.make_problem(4, (2, 2, 2), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=1, seed=8)
    o1, f, E1 = _solve(prob)
    rev = np.arange(o1.dec.n_blocks)[::-1]
    o2 = D3MOracle.from_problem(prob, order=rev).factor()
    E2 = o2.solve(f)
    assert _rel(E2, E1) <= 1e-10
    assert _rel(o2.lam, o1.lam) <= 1e-10


def test_k_solve_residual_and_reconstruction():
    prob = W.make_problem(4, (2, 2, 2), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=2, seed=10)
    o, f, E = _solve(prob)
    K = o.dm.assemble_dense()
    assert np.linalg.norm(K - K.T) <= 1e-14 * np.linalg.norm(K) * 10
    r = K @ o.lam.T - o.g.T
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(o.g)
    idx = np.concatenate([np.arange(o.dec.block_start[b], o.dec.block_start[b + 1]) for b in o.order])
    rec = o.ldlt.reconstruct_dense()
    assert np.linalg.norm(rec - K[np.ix_(idx, idx)]) <= 1e-12 * np.linalg.norm(K)


def test_reciprocity():
    prob = W.make_problem(4, (2, 2, 1), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=2, seed=12)
    o, f, E = _solve(prob)
    a, b = f[0] @ E[1], f[1] @ E[0]
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def _objective(E, P):
    # L = sum_rhs sum_m |E(r_m)|^2 with E(r_m) = P_m E
    v = np.einsum("mxe,re->rmx", P, E)
    return float(np.sum(np.abs(v) ** 2))


def test_adjoint_gradient_vs_central_differences():
    prob = W.make_problem(3, (2, 1, 1), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=2, seed=13)
    rng = np.random.default_rng(13)
    receivers = 0.5 + 0.3 * (rng.random((6, 3)) - 0.5)
    o, f, E = _solve(prob)
    P = probe_matrix(o.fem.topo, receivers)
    G = 2.0 * np.einsum("mxe,mxf,rf->re", P, P, E)  # dL/dRe E + j dL/dIm E
    grad, _ = o.adjoint(G, E)
    tets = rng.choice(len(prob.eps_r), 8, replace=False)
    h = 1e-6
    for t in tets:
        vals = []
        for s in (+1, -1):
            eps = prob.eps_r.copy()
            eps[t] += s * h
            F = GlobalFEM(prob.xyz, prob.tets, eps, prob.k)
            vals.append(_objective(global_solve(F, f), P))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - grad[t]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(grad).max())


def test_adjoint_matches_global_adjoint():
    prob = W.make_problem(3, (2, 2, 1), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=1, seed=14)
    o, f, E = _solve(prob)
    rng = np.random.default_rng(0)
    G = rng.standard_normal(E.shape) + 1j * rng.standard_normal(E.shape)
    grad, w = o.adjoint(G, E)
    wg = global_solve(o.fem, np.conj(G))
    assert _rel(w, wg) <= 1e-10
    assert _rel(grad, adjoint_gradient(o.fem, wg, E)) <= 1e-10
