"""Pins of the oracle's PEC surfaces and impressed-current (point dipole)
source (the n x E = 0 condition and the -jk eta J_imp term of the BVP in
Section II).

* The PEC edge set: a plate of a x b hexes holds (a+1) b + a (b+1) + a b
  edges; a closed triangulated box surface with F triangles holds 3F/2.
* D3M with PEC surfaces (on a subdomain interface and inside a subdomain)
  equals the plain sparse solve of S on the unknowns.
* Shielding: a closed PEC box with the sources outside leaves exactly zero
  field on every edge strictly inside (those edges couple only to each
  other and to the box's PEC edges, and carry no load).
* Reciprocity of two dipoles, f_1^T E_2 = f_2^T E_1 (S symmetric), with PEC
  surfaces present.
* The dipole load in closed form: Whitney DOFs u_e = (a + b x r_e) . t_e of a
  linear field a + b x r (r_e the edge midpoint, t_e the edge vector) are
  exact, so u^T f = -jk eta m . (a + b x r0).
* The adjoint gradient with PEC surfaces equals central differences.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle.d3m import D3MOracle, global_solve
from oracle.fem import ETA0, GlobalFEM


def _problem(n, parts, pec, seed, ndip=2, eps=("uniform", 1, 3)):
    p = W.make_problem(n, parts, eps=eps, k=2 * math.pi, nrhs=2, seed=seed)
    p.pec_faces = pec
    rng = np.random.default_rng(seed + 100)
    p.dip_pos = rng.uniform(0.05, 0.95, (ndip, 3))
    u = rng.standard_normal((ndip, 3))
    p.dip_moment = u * np.exp(1j * rng.uniform(0, 2 * math.pi, ndip))[:, None]
    return p


def _loads(o, p):
    return np.concatenate([o.fem.planewave_rhs(p.dirs, p.pols), o.fem.dipole_rhs(p.dip_pos, p.dip_moment)])


def test_pec_edge_counts():
    xyz, tets = W.kuhn_cube_mesh(6)
    for a, b in [(2, 2), (3, 1), (4, 5)]:
        faces = W.plate_faces(6, tets, 2, 3, [0, 1], [a, 1 + b])
        assert faces.shape[0] == 2 * a * b
        fem = GlobalFEM(xyz, tets, np.ones(tets.shape[0]), 2 * math.pi, pec_faces=faces)
        assert fem.pec.sum() == (a + 1) * b + a * (b + 1) + a * b
    shell = W.box_shell_faces(6, tets, [1, 2, 1], [4, 4, 5])
    fem = GlobalFEM(xyz, tets, np.ones(tets.shape[0]), 2 * math.pi, pec_faces=shell)
    assert fem.pec.sum() * 2 == 3 * shell.shape[0]
    with pytest.raises(ValueError):
        GlobalFEM(xyz, tets, np.ones(tets.shape[0]), 1.0, pec_faces=np.array([[0, 1, 2]]))  # collinear: no face


def test_d3m_with_plates_equals_global_solve():
    xyz, tets = W.kuhn_cube_mesh(8)
    pec = np.concatenate([W.plate_faces(8, tets, 2, 4, [2, 1], [6, 5]),   # on the z interface
                          W.plate_faces(8, tets, 0, 2, [1, 5], [3, 7])])  # inside the x < 4 boxes
    p = _problem(8, (2, 2, 2), pec, seed=41)
    o = D3MOracle.from_problem(p).factor()
    f = _loads(o, p)
    assert np.all(f[:, o.fem.pec] == 0)
    E = o.solve(f)
    E0 = global_solve(o.fem, f)
    assert np.all(E[:, o.fem.pec] == 0)
    assert np.abs(E - E0).max() <= 1e-10 * np.abs(E0).max()
    assert o.fem.relative_residual(E, f) <= 1e-11
    assert o.copy_discrepancy <= 1e-12 * np.abs(E).max()
    # no multiplier sits on a PEC edge
    assert not np.any(o.fem.pec[o.dec.lms[:, 2]])


def test_closed_pec_box_shields_its_inside():
    n = 8
    xyz, tets = W.kuhn_cube_mesh(n)
    lo, hi = [2, 2, 3], [6, 5, 6]
    shell = W.box_shell_faces(n, tets, lo, hi)
    p = _problem(n, (2, 2, 2), shell, seed=42, ndip=2)
    p.dip_pos = np.array([[0.1, 0.1, 0.15], [0.9, 0.85, 0.1]])  # outside the box
    o = D3MOracle.from_problem(p).factor()
    f = _loads(o, p)
    E = o.solve(f)
    vi = np.stack([xyz[:, a] * n for a in range(3)], 1).round().astype(int)
    ev = vi[o.fem.topo.edges]  # [ne, 2 vertices, 3]
    inside = np.all((ev > np.array(lo)) & (ev < np.array(hi)), axis=(1, 2))
    assert inside.sum() > 20
    scale = np.abs(E).max(axis=1)  # per right-hand side
    assert np.all(scale > 0)
    assert np.all(np.abs(E[:, inside]).max(axis=1) <= 1e-12 * scale)
    outside = ~inside & ~o.fem.pec
    assert np.all(np.abs(E[:, outside]).max(axis=1) == scale)


def test_dipole_reciprocity_with_plates():
    xyz, tets = W.kuhn_cube_mesh(6)
    pec = W.plate_faces(6, tets, 1, 3, [1, 1], [5, 4])
    p = _problem(6, (2, 1, 2), pec, seed=43)
    o = D3MOracle.from_problem(p).factor()
    f = o.fem.dipole_rhs(p.dip_pos, p.dip_moment)
    E = o.solve(f)
    a, b = f[0] @ E[1], f[1] @ E[0]
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_dipole_load_closed_form():
    xyz, tets = W.kuhn_cube_mesh(4)
    fem = GlobalFEM(xyz, tets, np.ones(tets.shape[0]), 3.0)
    rng = np.random.default_rng(44)
    a, b = rng.standard_normal(3), rng.standard_normal(3)
    ed = fem.topo.edges
    mid = 0.5 * (xyz[ed[:, 0]] + xyz[ed[:, 1]])
    u = np.einsum("ex,ex->e", a + np.cross(b, mid), xyz[ed[:, 1]] - xyz[ed[:, 0]])
    pos = rng.uniform(0.05, 0.95, (3, 3))
    mom = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    f = fem.dipole_rhs(pos, mom)
    want = -1j * 3.0 * ETA0 * np.einsum("rx,rx->r", mom, a + np.cross(b, pos))
    assert np.allclose(f @ u, want, rtol=1e-12, atol=0)


def test_adjoint_gradient_with_plates_vs_central_differences():
    xyz, tets = W.kuhn_cube_mesh(4)
    pec = W.plate_faces(4, tets, 2, 2, [1, 1], [3, 3])
    p = _problem(4, (2, 2, 1), pec, seed=45, ndip=1)
    p.dip_moment = p.dip_moment / ETA0  # loads of the plane waves' size (keeps the differences' rounding small)
    o = D3MOracle.from_problem(p).factor()
    f = _loads(o, p)
    E = o.solve(f)
    w0 = np.random.default_rng(46).standard_normal(E.shape[1])

    def L(E):
        return float(np.sum(np.abs(E) ** 2 * w0))

    G = 2 * w0 * E  # dL/dRe E + j dL/dIm E
    g, _ = o.adjoint(G, E)
    for t in (3, 50, 200):
        h = 1e-4  # O(h^2) ~ 1e-8 relative; at 1e-6 rounding of L (~1e-13 relative) over 2h reaches 1e-5
        vals = []
        for s in (+1, -1):
            eps = p.eps_r.copy()
            eps[t] += s * h
            q = D3MOracle(p.xyz, p.tets, p.part, eps, p.k, p.alpha, parts=p.parts, pec_faces=pec).factor()
            vals.append(L(q.solve(f)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[t]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (t, fd, g[t])
