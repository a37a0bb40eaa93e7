"""Nested-dissection row order of the subdomain matrices (d3m_options.s1_order = 1), host side.

The edge rows of each M_d follow a geometric nested dissection (interior and
interface edges alike; multipliers last), every leaf and separator starting
a new tile, with padding rows in between.  Checks:
  * the real rows are a permutation of the default order's rows, and A_d in
    the new order is A_d of the default order permuted, entry for entry;
    padding rows carry only a unit diagonal;
  * every row group starts at a tile boundary (the rows of a tile belong to
    one group), so tile-level fill stays inside the dissection's fronts;
  * the planned step-1 work falls against the banded default order as the
    subdomains grow: at most 0.6 of it at 12^3-hex subdomains and 0.4 at
    16^3 (the dissection's fronts against the band);
  * the factor schedule stays race-free.
"""
import numpy as np
import pytest

import workloads as W
from paper_2002_05018_amd import Solver


def _pair(n, parts, **kw):
    prob = W.make_problem(n, parts, eps=("uniform", 1, 4), k=2 * np.pi, nrhs=1, seed=3, **kw)
    return prob, Solver.from_problem(prob, host_only=True), Solver.from_problem(prob, host_only=True, s1_order=1)


@pytest.mark.parametrize("n,parts", [(6, (2, 2, 1)), (8, (2, 1, 1)), (7, (1, 3, 2))])
def test_rows_are_a_padded_permutation_with_the_same_matrix(n, parts):
    prob, s0, s1 = _pair(n, parts)
    for d in range(s0.info["n_subdomains"]):
        e0 = s0.export("sub_edges", d)
        e1 = s1.export("sub_edges", d)
        assert len(e1) % 64 == 0
        real = e1[e1 >= 0]
        assert np.array_equal(np.sort(real), np.sort(e0))
        # A_d: map both to global edge pairs
        r0, c0, v0 = s0.export("a_coo", d)
        r1, c1, v1 = s1.export("a_coo", d)
        pad = e1 < 0
        on_pad = pad[r1] | pad[c1]
        assert np.all(r1[on_pad] == c1[on_pad]) and np.all(v1[on_pad] == 1.0)
        assert np.count_nonzero(on_pad) == np.count_nonzero(pad)
        key0 = {}
        for r, c, v in zip(e0[r0], e0[c0], v0):
            key0[(min(r, c), max(r, c))] = v
        keep = ~on_pad
        assert np.count_nonzero(keep) == len(v0)
        for r, c, v in zip(e1[r1[keep]], e1[c1[keep]], v1[keep]):
            assert key0[(min(r, c), max(r, c))] == v


def test_groups_start_at_tile_boundaries():
    prob, s0, s1 = _pair(12, (2, 2, 2))
    e1 = s1.export("sub_edges", 0)
    # a padding run always ends at a tile boundary, and a tile holding a
    # padding row ends with it
    for t in range(len(e1) // 64):
        tile = e1[64 * t:64 * (t + 1)]
        pads = np.nonzero(tile < 0)[0]
        if pads.size:
            assert np.all(tile[pads[0]:] < 0), t


def test_planned_step1_work_against_the_band():
    for n, limit in ((24, 0.6), (32, 0.4)):
        _, s0, s1 = _pair(n, (2, 2, 2))
        f0, f1 = s0.info["flops_domain"], s1.info["flops_domain"]
        assert f1 <= limit * f0, (n, f1 / f0)
        assert s1.info["factor_bytes"] < s0.info["factor_bytes"]


def test_factor_schedule_race_free():
    _, s0, s1 = _pair(12, (2, 2, 2))
    n, rep = s1.check_schedule()
    assert n == 0, rep


def test_automatic_order_follows_subdomain_size():
    # s1_order 2: the dissection for subdomains of about 8^3 hexes and more
    # (median of at least 4,000 edge rows), the banded order below
    small = Solver.from_problem(W.make_problem(12, (2, 2, 2), eps=("uniform", 1, 4), k=2 * np.pi, nrhs=1, seed=3),
                                host_only=True, s1_order=2)
    large = Solver.from_problem(W.make_problem(16, (2, 2, 2), eps=("uniform", 1, 4), k=2 * np.pi, nrhs=1, seed=3),
                                host_only=True, s1_order=2)
    assert small.info["s1_order"] == 0 and large.info["s1_order"] == 1
    assert Solver.from_problem(W.make_config(1), host_only=True).info["s1_order"] == 0
