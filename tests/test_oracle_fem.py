"""Pins of the oracle's FEM layer against closed forms and invariants.

Nothing here re-types an oracle formula: each check is a property the exact
Whitney / Nedelec discretisation of the BVP in Section II must have.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as sla

import workloads as W
from oracle import fem
from oracle.quad import triangle_rule


def _mesh(n):
    xyz, tets = W.kuhn_cube_mesh(n)
    return xyz, tets


@pytest.mark.parametrize("q", [4, 8])
def test_triangle_rule_monomials(q):
    s, t, w = triangle_rule(q)
    for a in range(2 * q - 1):
        for b in range(2 * q - 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            got = np.sum(w * s ** a * t ** b)
            assert abs(got - exact) <= 1e-14 * max(1.0, exact) + 1e-16


@pytest.mark.parametrize("n", [1, 2, 3, 6])
def test_edge_count_closed_form(n):
    xyz, tets = _mesh(n)
    topo = fem.Topology(xyz, tets)
    assert topo.n_edges == 7 * n ** 3 + 9 * n ** 2 + 3 * n
    assert len(topo.boundary_faces()) == 12 * n * n


def _global(n, eps=None, k=2 * math.pi):
    xyz, tets = _mesh(n)
    eps = np.ones(len(tets)) if eps is None else eps
    return fem.GlobalFEM(xyz, tets, eps, k)


def _assemble_elem(topo, Mt, weights=None):
    import scipy.sparse as sp
    te = topo.tet_edges
    w = np.ones(len(te)) if weights is None else weights
    r = np.repeat(te, 6, 1).ravel()
    c = np.tile(te, (1, 6)).ravel()
    v = (w[:, None, None] * Mt).ravel()
    return sp.coo_matrix((v, (r, c)), shape=(topo.n_edges,) * 2).tocsr()


def test_curl_kills_gradients():
    F = _global(3)
    topo = F.topo
    Kc = _assemble_elem(topo, F.Kc)
    rng = np.random.default_rng(0)
    phi = rng.standard_normal(topo.n_vertices)
    u = phi[topo.edges[:, 1]] - phi[topo.edges[:, 0]]  # DOFs of grad phi
    assert np.abs(Kc @ u).max() <= 1e-12 * np.abs(Kc).max() * np.abs(u).max() * 10


def test_curl_energy_of_rotation_field():
    # E = b x r has curl 2b: u^T Kc u = |2b|^2 Vol(cube) = 4|b|^2
    F = _global(3)
    topo = F.topo
    Kc = _assemble_elem(topo, F.Kc)
    b = np.array([0.3, -1.2, 0.7])
    va = topo.xyz[topo.edges[:, 0]]
    vb = topo.xyz[topo.edges[:, 1]]
    u = np.einsum("ex,ex->e", np.cross(b, va), vb - va)
    assert abs(u @ (Kc @ u) - 4 * b @ b) <= 1e-12 * 4 * b @ b


def test_mass_of_constant_field():
    F = _global(3)
    topo = F.topo
    rng = np.random.default_rng(1)
    eps = rng.uniform(1, 4, len(topo.tets))
    M = _assemble_elem(topo, F.M, eps)
    c = np.array([1.0, -2.0, 0.5])
    u = (topo.xyz[topo.edges[:, 1]] - topo.xyz[topo.edges[:, 0]]) @ c
    exact = np.sum(eps * F.V) * (c @ c)
    assert abs(u @ (M @ u) - exact) <= 1e-12 * exact


def test_abc_of_constant_field():
    # sum over the 6 faces of |c_t|^2 * area = 4|c|^2 on the unit cube
    F = _global(3)
    topo = F.topo
    S0 = F.S - _assemble_elem(topo, F.Se)  # jk T_abc
    T = S0 / (1j * F.k)
    c = np.array([0.4, 1.1, -0.9])
    u = (topo.xyz[topo.edges[:, 1]] - topo.xyz[topo.edges[:, 0]]) @ c
    val = u @ (T @ u)
    assert abs(val.imag) < 1e-14
    assert abs(val.real - 4 * c @ c) <= 1e-12 * 4 * c @ c


def test_global_matrix_is_complex_symmetric():
    rng = np.random.default_rng(2)
    F = _global(3, eps=rng.uniform(1, 4, 162))
    assert abs(F.S - F.S.T).max() <= 1e-14 * abs(F.S).max()
    assert abs(F.S - F.S.conj().T).max() > 0.0  # not Hermitian


def test_free_space_converges_to_plane_wave():
    # eps_r = 1 makes E_inc the exact solution of the BVP: the FEM DOFs
    # must approach the edge integrals of E_inc, error falling >= 1.8x per halving
    d = np.array([0.3, 0.5, 0.8]); d /= np.linalg.norm(d)
    h = np.array([1.0, 0, 0]); p = h - (h @ d) * d; p /= np.linalg.norm(p)
    errs = []
    for n in (3, 6, 12):
        F = _global(n)
        f = F.planewave_rhs(d[None], p[None])[0]
        u = sla.spsolve(F.S.tocsc(), f)
        ui = fem.edge_interpolant(F.topo.xyz, F.topo.edges, F.k, d, p)
        errs.append(np.linalg.norm(u - ui) / np.linalg.norm(ui))
    assert errs[0] / errs[1] >= 1.8 and errs[1] / errs[2] >= 1.8, errs
    assert errs[-1] < 0.05


def test_planewave_load_quadrature_converged():
    # k h = 1.05 is the coarsest resolution of the standard workloads
    F = _global(6, k=2 * math.pi)
    d = np.array([0.0, 0.6, 0.8]); p = np.array([1.0, 0.0, 0.0])
    f12 = F.planewave_rhs(d[None], p[None])
    f24 = F.planewave_rhs(d[None], p[None], q=24)
    assert np.abs(f12 - f24).max() <= 1e-13 * np.abs(f24).max()


def test_whitney_interpolation_of_constants():
    # for a constant field c the Whitney interpolant is exact: sum_a u_a N_a = c
    xyz, tets = _mesh(1)
    G, V = fem.tet_geometry(xyz, np.sort(tets, 1))
    c = np.array([0.2, -0.7, 1.3])
    lam = np.array([0.1, 0.2, 0.3, 0.4])
    for t in range(len(tets)):
        x = xyz[np.sort(tets[t])]
        val = np.zeros(3)
        for (i, j) in fem.TET_EDGES:
            u = c @ (x[j] - x[i])
            val += u * (lam[i] * G[t, j] - lam[j] * G[t, i])
        assert np.allclose(val, c, atol=1e-13)


@pytest.mark.parametrize("n", [2, 5])
def test_probe_matrix_reproduces_rotational_linear_fields(n):
    """The lowest-order edge-element space holds every field a + b x r exactly
    (its curl 2b is constant and its divergence zero), so the edge degrees of
    freedom u_e = int_e F . dl (for a linear F, the midpoint value dotted with
    the edge vector) probed anywhere in the mesh give F itself.  Pins the
    point location, the barycentrics and the basis of probe_matrix: a wrong
    tetrahedron, sign or gradient changes the value."""
    xyz, tets = W.kuhn_cube_mesh(n)
    topo = fem.Topology(xyz, tets)
    rng = np.random.default_rng(n)
    a = rng.standard_normal(3)
    b = rng.standard_normal(3)
    lo, hi = topo.xyz[topo.edges[:, 0]], topo.xyz[topo.edges[:, 1]]
    mid = 0.5 * (lo + hi)
    u = np.einsum("ex,ex->e", a + np.cross(b, mid), hi - lo)
    pts = np.concatenate([rng.random((40, 3)),
                          xyz[rng.choice(len(xyz), 4, replace=False)],       # vertices
                          0.5 * (lo[:3] + hi[:3])])                             # edge midpoints
    P = fem.probe_matrix(topo, pts)
    got = P @ u
    want = a[None, :] + np.cross(b[None, :], pts)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
