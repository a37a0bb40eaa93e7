"""Work-queue form of the two K solve sweeps (d3m_tuning.solve_chain), host side.

The item lists are checked by d3m_debug_check_schedule's queue simulation:
every item's accesses are read again from the task data, the sequential
order from the level-by-level schedule, and workers take items from one
counter and wait on write counts as the kernel does, under pseudo-random
interleavings (1, 7, 64 and 512 workers; one and two column blocks).  It
must find no violation on the parity and full-size workloads, and it must
report a planted missing wait.
"""
import math

import pytest

import workloads as W
from paper_2002_05018_amd import D3MError, Solver

CASES = {
    "cfg1": lambda: W.make_config(1),
    "cross_lines_2x2x2": lambda: W.make_problem(4, (2, 2, 2), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=3, seed=1),
    "uneven_1x3x2": lambda: W.make_problem(7, (1, 3, 2), eps=("uniform", 1, 4), k=5.0, nrhs=1, seed=4,
                                           cuts=[[0, 7], [0, 2, 3, 7], [0, 5, 7]]),
    "cfg2": lambda: W.make_config(2),
    "cfg5_sphere": lambda: W.make_config(5),
    "pec": lambda: W.make_pec_config(),
}


@pytest.mark.parametrize("name", list(CASES))
def test_queue_simulation_finds_no_violation(name):
    s = Solver.from_problem(CASES[name](), host_only=True)
    n, rep = s.check_solve_chain()
    assert n == 0, rep


def test_queue_simulation_multifrontal_and_batch():
    s = Solver.from_problem(W.make_config(2), host_only=True, multifrontal=True)
    n, rep = s.check_solve_chain()
    assert n == 0, rep
    # a batch holds several elimination forests of different heights: roots
    # below the top level go before the backward queue
    probs = W.make_batch_config(seed=11, count=4, n_range=(4, 9), nrhs=2)
    b = Solver.batch(probs, probs[0].k, probs[0].alpha, host_only=True)
    n, rep = b.check_solve_chain()
    assert n == 0, rep


def test_planted_missing_wait_is_reported():
    s = Solver.from_problem(W.make_config(2), host_only=True)
    n, rep = s.check_solve_chain(drop_wait=True)
    assert n > 0
    assert "writes, expected" in rep


def test_whole_block_units_have_no_queue_form():
    # pivot units of several tiles keep the level-by-level sweeps
    s = Solver.from_problem(W.make_problem(8, (2, 1, 1), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=2, seed=2),
                            host_only=True, pivot_scope=1)
    with pytest.raises(D3MError, match="several tiles"):
        s.check_solve_chain()
