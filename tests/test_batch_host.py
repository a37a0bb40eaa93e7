"""Host-side checks of the batched form (no GPU): a batch handle holds the
disjoint union of its problems, each in its own numbering.

The subdomain matrices, edges and plane-wave loads of every problem inside a
batch must equal, bit for bit, those of the same problem set up alone (the
union only shifts ids), and the tuning calls must validate their arguments
and re-plan without touching the storage layout.
"""
import numpy as np
import pytest

import workloads as W
from paper_2002_05018_amd import D3MError, Solver


@pytest.fixture(scope="module")
def batch():
    probs = W.make_batch_config(seed=11, count=3, n_range=(4, 7), nrhs=2)
    s = Solver.batch(probs, probs[0].k, probs[0].alpha, host_only=True)
    singles = [Solver.from_problem(p, host_only=True) for p in probs]
    return probs, s, singles


def test_layout_is_problem_by_problem(batch):
    probs, s, singles = batch
    count, eo, to = s.layout()
    assert count == len(probs) == s.info["n_problems"]
    assert list(np.diff(eo)) == [t.n_edges for t in singles]
    assert list(np.diff(to)) == [p.tets.shape[0] for p in probs]
    edges = s.export("edges")
    v0 = 0
    for p, t in enumerate(singles):
        np.testing.assert_array_equal(edges[eo[p]:eo[p + 1]] - v0, t.export("edges"))
        v0 += probs[p].xyz.shape[0]


def test_subdomain_matrices_match_single_problems(batch):
    probs, s, singles = batch
    d0 = 0
    for p, t in enumerate(singles):
        for d in range(t.info["n_subdomains"]):
            rb, cb, vb = s.export("a_coo", d0 + d)
            rs, cs, vs = t.export("a_coo", d)
            np.testing.assert_array_equal(rb, rs)
            np.testing.assert_array_equal(cb, cs)
            np.testing.assert_array_equal(vb, vs)
        d0 += t.info["n_subdomains"]
    assert s.info["n_blocks"] == sum(t.info["n_blocks"] for t in singles)
    assert s.info["n_lm"] == sum(t.info["n_lm"] for t in singles)


def test_planewave_loads_per_problem(batch):
    probs, s, singles = batch
    _, eo, _ = s.layout()
    dirs = np.stack([p.dirs for p in probs])
    pols = np.stack([p.pols for p in probs])
    f = s.rhs_planewave_batch(dirs, pols)
    for p, t in enumerate(singles):
        np.testing.assert_array_equal(f[:, eo[p]:eo[p + 1]], t.rhs_planewave(probs[p].dirs, probs[p].pols))


def test_tuning_validates_and_replans(batch):
    probs, s, singles = batch
    s.set_tuning(s1_block=4, lookahead_tasks=100, solve_cols=16, k_block=3, panel_rows=16,
                 solve_seq=1, solve_narrow=512, k_overlap=1, solve_chain=1)
    assert s.tuning() == {"s1_block": 4, "solve_cols": 16, "lookahead_tasks": 100, "k_block": 3,
                          "side_early": 0, "k_fuse": 0, "panel_rows": 16,
                          "solve_seq": 1, "solve_narrow": 512, "k_overlap": 1, "solve_chain": 1}
    assert s.query()["array_bytes"] == s.info["array_bytes"]  # layout unchanged
    for bad in ({"s1_block": 17}, {"solve_cols": 8}, {"lookahead_tasks": -1}, {"k_block": 17},
                {"side_early": 2}, {"k_fuse": 2}, {"panel_rows": 32}, {"solve_seq": 2},
                {"solve_narrow": -1}, {"k_overlap": 2}, {"solve_chain": 2}):
        with pytest.raises(D3MError):
            s.set_tuning(**bad)
    s.set_tuning(s1_block=0, lookahead_tasks=0, solve_cols=0, k_block=0, panel_rows=0,
                 solve_seq=0, solve_narrow=0, k_overlap=0, solve_chain=0)


def test_empty_batch_rejected():
    from paper_2002_05018_amd import _lib
    import ctypes as C
    h = C.c_void_p()
    opt = _lib._options(host_only=True)
    rc = _lib._lib.d3m_setup_batch(None, 0, 1.0, _lib.d3m_c128(0, -1), C.byref(opt), C.byref(h))
    assert rc == -1
