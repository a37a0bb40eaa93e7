"""Host-side products of the library (d3m_setup with host_only = 1) against
the oracle: topology, subdomain matrices A_d, multipliers, plane-wave load,
ordering/symbolic consistency and field probes.  Independent code paths
(C++ vs NumPy) must agree to rounding."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.block import clique_adjacency, symbolic
from oracle.d3m import D3MOracle
from oracle.fem import probe_matrix

CASES = [W.make_config(1),
         W.make_problem(4, (2, 2, 2), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=2, seed=1),
         W.make_problem(5, (1, 3, 2), eps=("uniform", 1, 4), k=3.0, nrhs=2, seed=2)]


@pytest.fixture(scope="module", params=range(len(CASES)))
def pair(request):
    from paper_2002_05018_amd import Solver
    prob = CASES[request.param]
    return prob, Solver.from_problem(prob, host_only=True), D3MOracle.from_problem(prob)


def test_topology_and_multipliers(pair):
    prob, s, o = pair
    assert np.array_equal(s.export("edges"), o.fem.topo.edges)
    assert np.array_equal(s.export("lms"), o.dec.lms.reshape(-1, 3))
    assert s.info["n_blocks"] == o.dec.n_blocks


def test_subdomain_matrices(pair):
    prob, s, o = pair
    for d in range(o.dec.N):
        ge = s.export("sub_edges", d)
        ni = int(s.export("sub_ni", d)[0])
        assert np.array_equal(np.sort(ge), o.dec.sub_edges[d])
        mult = np.array([len(o.dec.sub_of_edge[e]) for e in ge])
        assert np.all(mult[:ni] == 1) and np.all(mult[ni:] >= 2)
        r, c, v = s.export("a_coo", d)
        assert np.all(r >= c)
        A = np.zeros((ge.size,) * 2, complex)
        A[r, c] = v
        A[c, r] = v
        Ao = o.dec.A[d].toarray()
        idx = np.searchsorted(o.dec.sub_edges[d], ge)
        assert np.abs(A - Ao[np.ix_(idx, idx)]).max() <= 1e-13 * np.abs(Ao).max()


def test_planewave_load(pair):
    prob, s, o = pair
    f = s.rhs_planewave(prob.dirs, prob.pols)
    fo = o.fem.planewave_rhs(prob.dirs, prob.pols)
    assert np.abs(f - fo).max() <= 1e-13 * np.abs(fo).max()


def test_order_and_struct(pair):
    prob, s, o = pair
    order = s.export("order")
    assert sorted(order) == list(range(o.dec.n_blocks))
    st = s.export("struct")
    ref = symbolic(clique_adjacency(o.dec.blocks), order)
    assert [list(map(int, x)) for x in st] == ref


def test_probe(pair):
    prob, s, o = pair
    rng = np.random.default_rng(0)
    pts = 0.05 + 0.9 * rng.random((5, 3))
    edges, coef = s.probe(pts)
    P = probe_matrix(o.fem.topo, pts)
    for m in range(len(pts)):
        Pm = np.zeros((3, o.fem.topo.n_edges))
        for a in range(6):
            Pm[:, edges[m, a]] += coef[m, a]
        assert np.abs(Pm - P[m]).max() <= 1e-12 * np.abs(P[m]).max()


def test_pivot_units_and_levels():
    """Pivot units: whole blocks (scope 1) or pieces of at most 64 rows
    (scope 0); the unit elimination tree must have at least as many levels
    as the block tree and cover every multiplier once."""
    from paper_2002_05018_amd import Solver
    prob = W.make_problem(8, (2, 2, 1), eps=("uniform", 1, 4), k=2 * math.pi, seed=3)
    whole = Solver.from_problem(prob, host_only=True, pivot_scope=1).info
    piece = Solver.from_problem(prob, host_only=True, pivot_scope=0).info
    assert whole["n_units"] == whole["n_blocks"]
    assert piece["n_units"] > piece["n_blocks"]  # blocks of 208 rows split into 4 pieces
    assert piece["n_unit_levels"] >= whole["n_unit_levels"] >= 2
    c1 = Solver.from_problem(W.make_config(1), host_only=True).info
    assert c1["n_units"] == 4 and c1["n_unit_levels"] == 3
