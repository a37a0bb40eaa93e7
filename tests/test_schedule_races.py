"""Static race check of the factorisation schedule (d3m_debug_check_schedule,
no GPU): the launches of one factorisation are replayed with their streams,
event records and waits, and every tile a work-group reads or writes is
checked against the accesses of other work-groups and launches that are not
ordered with it.  Every schedule variant the tuning can select (look-ahead
thresholds forcing the side streams, early or late side launches, chain
blocking, fused next-level updates, the block-column tracked schedule),
both pivot scopes and the multifrontal form must be race-free; leaving out
the stream waits (a planted mistake) must be reported."""
import math

import pytest

import workloads as W

VARIANTS = [dict(), dict(lookahead_tasks=1), dict(lookahead_tasks=1, side_early=1),
            dict(lookahead_tasks=1, s1_block=1, k_block=1), dict(lookahead_tasks=1, s1_block=4, k_block=4, k_fuse=1),
            dict(lookahead_tasks=1, k_overlap=1), dict(lookahead_tasks=1, k_overlap=1, side_early=1, k_fuse=1)]


@pytest.fixture(scope="module")
def problems():
    return [W.make_problem(8, (2, 2, 2), eps=("uniform", 1, 4), k=2 * math.pi, nrhs=1, seed=71),
            W.make_problem(7, (1, 3, 2), eps=("uniform", 1, 4), k=5.0, nrhs=1, seed=72,
                           cuts=[[0, 7], [0, 2, 3, 7], [0, 5, 7]])]


@pytest.mark.parametrize("scope", [0, 1])
@pytest.mark.parametrize("v", range(len(VARIANTS)))
def test_factor_schedules_are_race_free(problems, v, scope):
    from paper_2002_05018_amd import Solver
    for p in problems:
        s = Solver.from_problem(p, host_only=True, pivot_scope=scope)
        s.set_tuning(**VARIANTS[v])
        for force_side in (False, True):
            n, rep = s.check_schedule(force_side=force_side)
            assert n == 0, (VARIANTS[v], scope, force_side, rep)


def test_multifrontal_and_batch_schedules_are_race_free(problems):
    from paper_2002_05018_amd import Solver
    for p in problems:
        s = Solver.from_problem(p, host_only=True, multifrontal=True)
        for kb in (1, 2, 4):
            s.set_tuning(k_block=kb, lookahead_tasks=1)
            assert s.check_schedule() == (0, "")
    batch = W.make_batch_config(seed=11, count=3, n_range=(4, 7), nrhs=1)
    b = Solver.batch(batch, batch[0].k, batch[0].alpha, host_only=True)
    b.set_tuning(lookahead_tasks=1, k_overlap=1)
    assert b.check_schedule()[0] == 0


def test_planted_missing_waits_are_reported(problems):
    from paper_2002_05018_amd import Solver
    s = Solver.from_problem(problems[0], host_only=True)
    for tune in (dict(lookahead_tasks=1), dict(lookahead_tasks=1, k_overlap=1)):
        s.set_tuning(**tune)
        n, rep = s.check_schedule(drop_waits=True)
        assert n > 0 and "unordered" in rep, tune


def test_benchmark_schedule_at_48_cubed_is_race_free():
    """The launch shapes of the 48^3 benchmark entry (both forms), and the
    side-stream schedule for whole-block units that the library does not
    launch: no unordered conflicting tile access."""
    from paper_2002_05018_amd import Solver
    p = W.make_config(4)
    tune = dict(k_block=4, k_fuse=1, lookahead_tasks=512, panel_rows=64, s1_block=4, side_early=0)
    for scope in (0, 1):
        s = Solver.from_problem(p, host_only=True, pivot_scope=scope)
        for ko in (0, 1):
            s.set_tuning(**dict(tune, k_overlap=ko))
            n, rep = s.check_schedule(force_side=True)
            assert n == 0, (scope, ko, rep)
