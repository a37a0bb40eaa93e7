"""PEC surfaces and impressed currents on the GPU (the n x E = 0 condition
and the -jk eta J_imp term of the BVP in Section II), through the C ABI,
against the oracle with the same PEC triangles and point dipoles.

Bars as for the other workloads, per right-hand side and element-wise: E
and lambda equal the oracle's to 1e-10 (FP64), E is exactly zero on PEC
edges, the library's residual (its global S without the PEC rows and
columns) is at most 1e-10 and equals the host residual with the oracle's
S on the unknowns; FP32 factors with FP64 refinement reach 1e-10 and the
oracle's field to 1e-9; a closed PEC box keeps its inside at zero; the
adjoint gradient equals the oracle's to 1e-10; the multifrontal form agrees;
and at full size (24^3 hexes, two plates, plane waves and dipoles) the field
at sampled edges equals the oracle fixture to 1e-10 with the oracle's
residual bar.
"""
import math

import numpy as np
import pytest

import workloads as W
from parity import assert_rhs_close, factor_as_benchmarked, host_residual, load_fixture

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(name):
    if name == "plates_2x2x2":
        xyz, tets = W.kuhn_cube_mesh(8)
        pec = np.concatenate([W.plate_faces(8, tets, 2, 4, [2, 1], [6, 5]),
                              W.plate_faces(8, tets, 0, 2, [1, 5], [3, 7])])
        p = W.make_problem(8, (2, 2, 2), eps=("uniform", 1, 3), k=2 * math.pi, nrhs=2, seed=61)
    elif name == "shell_2x2x2":
        xyz, tets = W.kuhn_cube_mesh(8)
        pec = W.box_shell_faces(8, tets, [2, 2, 3], [6, 5, 6])
        p = W.make_problem(8, (2, 2, 2), eps=("uniform", 1, 3), k=2 * math.pi, nrhs=1, seed=62)
    else:  # a plate through a whole-block-sized interface and a 208-row block
        xyz, tets = W.kuhn_cube_mesh(8)
        pec = W.plate_faces(8, tets, 1, 5, [1, 2], [7, 6])
        p = W.make_problem(8, (2, 1, 1), eps=("uniform", 1, 3), k=2 * math.pi, nrhs=2, seed=63)
    p.pec_faces = pec
    rng = np.random.default_rng(64)
    p.dip_pos = np.array([[0.1, 0.12, 0.15], [0.88, 0.85, 0.11]])
    p.dip_moment = rng.standard_normal((2, 3)) + 1j * rng.standard_normal((2, 3))
    return p


_cache = {}


def _oracle(name):
    if name not in _cache:
        from oracle.d3m import D3MOracle
        p = _case(name)
        print(f"[gpu pec] case {name}: {p.pec_faces.shape[0]} PEC triangles", flush=True)
        o = D3MOracle.from_problem(p).factor()
        f = np.concatenate([o.fem.planewave_rhs(p.dirs, p.pols), o.fem.dipole_rhs(p.dip_pos, p.dip_moment)])
        Eo = o.solve(f)
        _cache[name] = (p, o, f, Eo, o.lam.copy())
    return _cache[name]


@pytest.mark.parametrize("name", ["plates_2x2x2", "shell_2x2x2", "plate_2x1x1"])
def test_pec_fp64_matches_oracle(name):
    from paper_2002_05018_amd import Solver
    p, o, f, Eo, lamo = _oracle(name)
    s = Solver.from_problem(p)
    fl = np.concatenate([s.rhs_planewave(p.dirs, p.pols), s.rhs_dipole(p.dip_pos, p.dip_moment)])
    assert_rhs_close(fl, f, 1e-13, f"{name} loads")
    s.factor("fp64")
    E, info = s.solve(torch.from_numpy(f).cuda(), with_info=True)
    E = E.cpu().numpy()
    assert not np.any(E[:, o.fem.pec])
    assert_rhs_close(E, Eo, 1e-10, f"{name} E")
    lam = s.export("lambda", E.shape[0])
    assert_rhs_close(lam, lamo, 1e-10, f"{name} lambda")
    r = host_residual(o.fem.system(), E[:, o.fem.free], f[:, o.fem.free])
    assert np.all(r <= 1e-10), r
    assert info["residual"] <= 1e-10 and abs(info["residual"] - r.max()) <= 1e-3 * r.max() + 1e-15
    assert info["copy_discrepancy"] <= 1e-12 * np.abs(E).max()


def test_pec_shell_shields_on_gpu():
    from paper_2002_05018_amd import Solver
    p, o, f, Eo, lamo = _oracle("shell_2x2x2")
    s = Solver.from_problem(p)
    s.factor("fp64")
    E = s.solve(torch.from_numpy(f).cuda()).cpu().numpy()
    n = p.n
    vi = np.rint(p.xyz * n).astype(int)
    ev = vi[o.fem.topo.edges]
    inside = np.all((ev > np.array([2, 2, 3])) & (ev < np.array([6, 5, 6])), axis=(1, 2))
    assert inside.sum() > 20
    assert np.all(np.abs(E[:, inside]).max(axis=1) <= 1e-12 * np.abs(E).max(axis=1))


@pytest.mark.parametrize("name", ["plates_2x2x2", "plate_2x1x1"])
def test_pec_fp32_with_refinement(name):
    from paper_2002_05018_amd import Solver
    p, o, f, Eo, lamo = _oracle(name)
    s = Solver.from_problem(p)
    s.factor("fp32_ir")
    E, info = s.solve(torch.from_numpy(f).cuda(), with_info=True)
    assert info["converged"] and info["residual"] <= 1e-10, info
    assert_rhs_close(E.cpu().numpy(), Eo, 1e-9, f"{name} FP32+IR E")


def test_pec_adjoint_and_multifrontal():
    from oracle.d3m import adjoint_gradient
    from paper_2002_05018_amd import Solver
    p, o, f, Eo, lamo = _oracle("plates_2x2x2")
    fd = torch.from_numpy(f).cuda()
    s = Solver.from_problem(p, multifrontal=True)
    s.factor("fp64")
    E = s.solve(fd)
    assert_rhs_close(E.cpu().numpy(), Eo, 1e-10, "multifrontal E")
    rng = np.random.default_rng(65)
    G = rng.standard_normal(Eo.shape) + 1j * rng.standard_normal(Eo.shape)
    G[:, o.fem.pec] = 0.0
    g, w = s.adjoint(torch.from_numpy(G).cuda(), E, want_w=True)
    go, wo = o.adjoint(G, Eo)
    assert_rhs_close(w.cpu().numpy(), wo, 1e-10, "adjoint w")
    assert np.abs(g.cpu().numpy() - go).max() <= 1e-10 * np.abs(go).max()


def test_pec_plates_full_size_against_oracle():
    """The PEC-plate workload (24^3 hexes, 4x4x4 boxes, one plate on a
    subdomain interface and one inside a subdomain, 4 plane waves and 4
    dipoles), in the launch shapes the tuning table gives it (none: the
    defaults)."""
    from oracle.fem import GlobalFEM
    from paper_2002_05018_amd import Solver
    fx = load_fixture("pec")
    p = W.make_pec_config()
    print(f"[gpu pec] full size: {p.pec_faces.shape[0]} PEC triangles", flush=True)
    s = Solver.from_problem(p)
    f = np.concatenate([s.rhs_planewave(p.dirs, p.pols), s.rhs_dipole(p.dip_pos, p.dip_moment)])
    assert_rhs_close(f[:, fx["edges"]], fx["f"], 1e-13, "PEC plates loads")
    g = GlobalFEM(p.xyz, p.tets, p.eps_r, p.k, pec_faces=p.pec_faces)
    fo = np.concatenate([g.planewave_rhs(p.dirs, p.pols), g.dipole_rhs(p.dip_pos, p.dip_moment)])
    for prec, tol in (("fp64", 1e-10), ("fp32_ir", 1e-9)):
        factor_as_benchmarked(s, 8, prec)
        E, info = s.solve(torch.from_numpy(fo).cuda(), with_info=True)
        E = E.cpu().numpy()
        assert not np.any(E[:, g.pec])
        err = assert_rhs_close(E[:, fx["edges"]], fx["E"], tol, f"PEC plates {prec} E", scale=fx["E_inf"])
        r = host_residual(g.system(), E[:, g.free], fo[:, g.free])
        print(f"[gpu pec] full size {prec}: E vs oracle {err.max():.2e}, residual {r.max():.2e} "
              f"(oracle's own {fx['residual'].max():.2e})", flush=True)
        assert np.all(r <= 1e-10), r


@pytest.mark.parametrize("name", ["plates_2x2x2", "plate_2x1x1"])
def test_pec_with_nested_dissection_rows(name):
    """PEC identity rows and the dissection's padding rows together."""
    from paper_2002_05018_amd import Solver
    p, o, f, Eo, lamo = _oracle(name)
    s = Solver.from_problem(p, s1_order=1)
    assert s.info["s1_order"] == 1
    s.factor("fp64")
    E, info = s.solve(torch.from_numpy(f).cuda(), with_info=True)
    E = E.cpu().numpy()
    assert not np.any(E[:, o.fem.pec])
    assert_rhs_close(E, Eo, 1e-10, f"{name} E (nested dissection)")
    assert info["residual"] <= 1e-10
